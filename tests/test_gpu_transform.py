"""GPU parity of the grouped transform and its adjoint against the FP64 oracle.

Element-by-element relative l2 error on seeded inputs; the FP32 path is compared with
the oracle evaluated on the FP32-rounded inputs.  Bars: 1e-5 (FP32) and 1e-12 (FP64 at
the library's default window); cases with an explicitly small window use the larger of
that bar and 20x the window's model error."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import index_set as oidx
from oracle import transform as otr
from paper_2010_10199_amd import lib
from tests.gpu_util import (TOL, check, dtype_code, gpu_adjoint, gpu_trafo, max_err, max_tol, nfft_model_error, rel,
                            say, to_dev)

pytestmark = pytest.mark.gpu

# (name, d, ds, N, M or ragged sizes, R, m, sigma)
CASES = [
    ("1d-ragged-tail", 3, 1, (16,), 700, 1, 0, 0.0),
    ("2d-two-rhs", 4, 2, (12, 6), 1000, 2, 0, 0.0),
    ("3d", 4, 3, (8, 6, 4), 600, 1, 0, 0.0),
    ("3d-m3-sigma2.5-R3", 5, 3, (6, 4, 4), 257, 3, 3, 2.5),
    ("ragged-with-empty", 3, 2, (10, 6), [300, 0, 957], 3, 0, 0.0),
    ("single-node", 2, 2, (4, 4), 1, 1, 0, 0.0),
    ("only-empty-set", 3, 0, (), 300, 2, 0, 0.0),
    ("bandwidth-2", 3, 3, (2, 2, 2), 513, 1, 0, 0.0),
    ("wide-window-small-grid", 2, 2, (4, 4), 400, 1, 8, 2.0),
    # enough nodes per grid cell for the cell gather (and the polynomial gather in FP32)
    ("cells-2d-R2", 3, 2, (8, 6), 20000, 2, 0, 0.0),
    ("cells-ragged-2d", 3, 2, (6, 4), [10000, 12000], 2, 0, 0.0),
    ("cells-3d", 3, 3, (4, 4, 4), 30000, 1, 0, 0.0),
    # an order-2 grid with more than 32 tiles per row (the flattened column fold): m = 8,
    # tiles of one cell
    ("wide-grid-m8", 2, 2, (4, 24), 600, 1, 8, 2.0),
    # column sums of an order-2 term too large for the adjoint DFT's LDS (n = 64, 13 tiles per
    # row): the separate tile-sum fold kernel
    ("unstaged-fold-2d", 2, 2, (4, 32), 800, 1, 6, 2.0),
    # every window width of the order-2 tile spread (tile sides 13, 9, 7, 3 here; 11, 5 and 1
    # in the m = 3, 6 and 8 cases), several tiles per row of the 28-point grid
    ("2d-m2", 3, 2, (16, 14), 3000, 1, 2, 2.0),
    ("2d-m4", 3, 2, (16, 14), 3000, 2, 4, 2.0),
    ("2d-m5", 3, 2, (16, 14), 3000, 1, 5, 2.0),
    ("2d-m7", 3, 2, (16, 14), 3000, 1, 7, 2.0),
]

# forward gather path per order of the cell cases: FP32 takes the polynomial gather for
# order 2, FP64 the cell gather
PATHS = {
    "cells-2d-R2": {1: "cell", 2: "poly"},
    "cells-ragged-2d": {1: "cell", 2: "poly"},
    "cells-3d": {1: "cell", 2: "poly", 3: "cell"},
}


def _inputs(case_id, d, ds, N, Msz, R, prec):
    iset = oidx.grouped_index_set(d, ds, N)
    ragged = isinstance(Msz, list)
    Mx = sum(Msz) if ragged else Msz
    x = W.uniform_nodes(W.rng(100 + case_id, W.P_NODES), Mx, d, prec)
    fhat = W.complex_normal(W.rng(100 + case_id, W.P_COEFFS), (R, iset.n_coeffs), prec)
    y = W.complex_normal(W.rng(100 + case_id, W.P_SAMPLES), (R * Mx if not ragged else Mx,), prec)
    offsets = list(np.concatenate([[0], np.cumsum(Msz)])) if ragged else None
    return iset, x, fhat, y, offsets


def _tol(prec, m, sigma, ds):
    if m == 0:
        return TOL[prec]
    return max(TOL[prec], 20 * max(1, ds) * nfft_model_error(m, sigma or 2.0))


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_forward_and_adjoint_parity(case, prec):
    name, d, ds, N, Msz, R, m, sigma = case
    cid = CASES.index(case)
    say(f"[parity] {name} {prec} d={d} ds={ds} N={N} M={Msz} R={R} m={m} sigma={sigma}")
    iset, x, fhat, y, offsets = _inputs(cid, d, ds, N, Msz, R, prec)
    Mx = x.shape[0]
    tol = _tol(prec, m, sigma, ds)
    # forward
    f = gpu_trafo(d, ds, N, x, fhat, prec, R=R, offsets=offsets, m=m, sigma=sigma)
    mtol = max_tol(prec, ds, m, sigma)
    if offsets is None:
        ref = otr.forward(iset, x, fhat)
        check("forward", f, ref, fhat, tol, mtol)
    else:
        ref = np.concatenate([otr.forward(iset, x[offsets[b]:offsets[b + 1]], fhat[b]) if offsets[b + 1] > offsets[b]
                              else np.zeros(0, complex) for b in range(R)])
        err = rel(f, ref)
        em = max(max_err(f[offsets[b]:offsets[b + 1]], ref[offsets[b]:offsets[b + 1]], fhat[b]) for b in range(R))
        say(f"  forward rel l2 {err:.3e} (tol {tol:.1e}), max/l1 {em:.3e} (tol {mtol:.1e})")
        assert err <= tol and em <= mtol
    # adjoint
    yy = y.reshape(R, Mx) if offsets is None else y
    a = gpu_adjoint(d, ds, N, x, yy, prec, iset.n_coeffs, R=R, offsets=offsets, m=m, sigma=sigma)
    if offsets is None:
        refa = otr.adjoint(iset, x, yy)
    else:
        refa = np.stack([otr.adjoint(iset, x[offsets[b]:offsets[b + 1]], y[offsets[b]:offsets[b + 1]])
                         for b in range(R)])
    if offsets is None:
        check("adjoint", a, refa, yy, tol, mtol)
    else:
        erra = rel(a, refa)
        em = max(max_err(a[b], refa[b], y[offsets[b]:offsets[b + 1]]) for b in range(R) if offsets[b + 1] > offsets[b])
        say(f"  adjoint rel l2 {erra:.3e} (tol {tol:.1e}), max/l1 {em:.3e} (tol {mtol:.1e})")
        assert erra <= tol and em <= mtol
        for b in range(R):          # an empty dataset's coefficients are exactly zero
            if offsets[b + 1] == offsets[b]:
                assert not np.any(a[b])


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", sorted(PATHS))
def test_cell_cases_take_the_intended_gather(name, prec):
    """The cell cases above run through the gather paths they are meant to cover (their
    parity is checked by test_forward_and_adjoint_parity)."""
    import torch
    case = next(c for c in CASES if c[0] == name)
    _, d, ds, N, Msz, R, m, sigma = case
    iset, x, fhat, y, offsets = _inputs(CASES.index(case), d, ds, N, Msz, R, prec)
    p, keep = lib.make_problem(d, ds, N, M=x.shape[0] if offsets is None else 0, R=R, dtype=dtype_code(prec),
                               offsets=offsets)
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    want = {"sorted": lib.GT_GATHER_SORTED, "cell": lib.GT_GATHER_CELL, "poly": lib.GT_GATHER_POLY}
    for t, kind in PATHS[name].items():
        if prec == "f64" and kind == "poly":
            kind = "cell"
        got = plan.gather_path(t)
        say(f"[path] {name} {prec} order {t}: {got} (want {kind})")
        assert got == want[kind]
    plan.close()
    torch.cuda.synchronize()


def test_config1_fp64_full():
    """d=6, d_s=2, N=(16, 8), M=2000, FP64: full forward and adjoint."""
    d, ds, N, M = 6, 2, (16, 8), 2000
    iset = oidx.grouped_index_set(d, ds, N)
    x, fhat, y = W.trafo_inputs(1, d, ds, M, iset.n_coeffs, 1, "f64")
    say("[config1] full fp64")
    f = gpu_trafo(d, ds, N, x, fhat, "f64")
    check("forward", f, otr.forward(iset, x, fhat), fhat, TOL["f64"], max_tol("f64", ds))
    a = gpu_adjoint(d, ds, N, x, y.reshape(1, M), "f64", iset.n_coeffs)
    check("adjoint", a, otr.adjoint(iset, x, y.reshape(1, M)), y.reshape(1, M), TOL["f64"], max_tol("f64", ds))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_config2_full_size_sampled(prec):
    """d=10, d_s=2, N=(64, 16), M=50,000, KB m=6, sigma=2: the launch the benchmark times.

    Forward checked on 3,000 sampled nodes, adjoint on 400 sampled coefficients (each an
    exact sum over all 50,000 nodes).  FP64 at the fixed m=6 is held to 20x the window's
    error model instead of 1e-12 (m=6 cannot reach 1e-12 at sigma=2)."""
    d, ds, N, M = 10, 2, (64, 16), 50000
    iset = oidx.grouped_index_set(d, ds, N)
    x, fhat, y = W.trafo_inputs(2, d, ds, M, iset.n_coeffs, 1, prec)
    say(f"[config2] {prec}")
    f = gpu_trafo(d, ds, N, x, fhat, prec, m=6, sigma=2.0)[0]
    g = np.random.default_rng(0)
    S = np.sort(g.choice(M, 3000, replace=False))
    tol = TOL[prec] if prec == "f32" else 20 * ds * nfft_model_error(6, 2.0)
    mtol = max_tol(prec, ds, 6, 2.0)
    check("forward (3,000 nodes)", f[S], otr.forward(iset, x[S], fhat[0]), fhat, tol, mtol)
    a = gpu_adjoint(d, ds, N, x, y.reshape(1, M), prec, iset.n_coeffs, m=6, sigma=2.0)[0]
    K = np.sort(g.choice(iset.n_coeffs, 400, replace=False))
    check("adjoint (400 coefficients)", a[K], otr.adjoint_at(iset, x, y.reshape(-1), K), y, tol, mtol)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_adjoint_identity_large(prec):
    """<F fhat, y> = <fhat, F^H y> on the GPU results at a size the oracle does not run."""
    d, ds, N, M, R = 12, 3, (24, 10, 6), 120000, 2
    iset = oidx.grouped_index_set(d, ds, N)
    x, fhat, y = W.trafo_inputs(6, d, ds, M, iset.n_coeffs, R, prec)
    say(f"[adjoint-identity] {prec} M={M}")
    f = gpu_trafo(d, ds, N, x, fhat, prec, R=R)
    a = gpu_adjoint(d, ds, N, x, y.reshape(R, M), prec, iset.n_coeffs, R=R)
    for r in range(R):
        lhs = np.vdot(y.reshape(R, M)[r].astype(complex), f[r])
        rhs = np.vdot(a[r], fhat[r].astype(complex))
        err = abs(lhs - rhs) / (np.linalg.norm(f[r]) * np.linalg.norm(y.reshape(R, M)[r]))
        say(f"  r={r} identity err {err:.3e}")
        assert err <= (1e-6 if prec == "f32" else 1e-13)


def test_node_wrapping_and_edges():
    """Nodes at -1/2, just below 1/2, and outside [-1/2, 1/2) (reduced mod 1) give the
    oracle's values at the wrapped nodes."""
    d, ds, N = 2, 2, (8, 6)
    iset = oidx.grouped_index_set(d, ds, N)
    base = np.array([[-0.5, -0.5], [0.5 - 1e-12, 0.25], [0.0, 0.5 - 2 ** -40], [0.1, -0.3]])
    shifted = base + np.array([[3.0, -2.0], [-1.0, 5.0], [7.0, 1.0], [-4.0, 2.0]])
    fhat = W.complex_normal(W.rng(150, W.P_COEFFS), (1, iset.n_coeffs), "f64")
    f = gpu_trafo(d, ds, N, shifted, fhat, "f64")
    ref = otr.forward(iset, base, fhat[0])
    err = rel(f[0], ref)
    say(f"[wrap] rel err {err:.3e}")
    assert err <= 1e-11


def test_invalid_arguments_are_rejected():
    import torch
    from paper_2010_10199_amd import lib
    x = torch.zeros(10, 3, dtype=torch.float64, device="cuda")
    x[3, 1] = float("nan")
    fh = torch.zeros(lib.gt_num_coeffs(3, 2, [4, 4]), dtype=torch.complex128, device="cuda")
    f = torch.zeros(10, dtype=torch.complex128, device="cuda")
    p, _ = lib.make_problem(3, 2, [4, 4], M=10, dtype=lib.GT_C128)
    with pytest.raises(lib.GroupedError) as e:
        lib.grouped_trafo(p, x, fh, f)
    assert e.value.code == lib.GT_EINVAL and "NaN" in str(e.value)
    x[3, 1] = 0.0
    for bad in [dict(N=[5, 4]), dict(ds=4, N=[4, 4, 4]), dict(m=9), dict(sigma=1.2)]:
        kw = dict(d=3, ds=2, N=[4, 4], M=10, dtype=lib.GT_C128)
        kw.update(bad)
        p, _ = lib.make_problem(kw.pop("d"), kw.pop("ds"), kw.pop("N"), **kw)
        with pytest.raises(lib.GroupedError) as e:
            lib.grouped_trafo(p, x, fh, f)
        assert e.value.code in (lib.GT_EINVAL, lib.GT_EUNSUPPORTED)
    # no nodes at all: shared (M = 0) or ragged with every dataset empty
    for kw in [dict(M=0), dict(M=0, R=2, offsets=[0, 0, 0])]:
        p, keep = lib.make_problem(3, 2, [4, 4], dtype=lib.GT_C128, **kw)
        with pytest.raises(lib.GroupedError) as e:
            lib.grouped_trafo(p, x, fh, f)
        assert e.value.code == lib.GT_EINVAL and keep is not None


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_caller_graph_capture_matches_oracle(prec):
    """Plan calls allocate nothing and synchronise nothing, so a caller can capture them in a
    graph: here torch.cuda.CUDAGraph drives HIP stream capture, and the library's side
    stream joins the capture through its fork/join events.  The graph is replayed several
    times with ordinary torch work on the inputs between replays, and every replay is
    checked against the oracle."""
    import torch
    from paper_2010_10199_amd import lib
    from tests.gpu_util import cdtype, dtype_code, to_dev
    d, ds, N, M = 5, 2, (16, 8), 3000
    iset = oidx.grouped_index_set(d, ds, N)
    x, fhat, y = W.trafo_inputs(160, d, ds, M, iset.n_coeffs, 1, prec)
    tol = TOL[prec]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=dtype_code(prec))
        plan = lib.Plan(p, to_dev(x))
        f0 = to_dev(fhat.reshape(-1))
        y0 = to_dev(y.reshape(-1))
        fd = f0.clone()
        yd = y0.clone()
        fo = torch.empty(M, dtype=cdtype(prec), device="cuda")
        ao = torch.empty(iset.n_coeffs, dtype=cdtype(prec), device="cuda")
        plan.trafo(fd, fo)              # eager call first (sets kernel attributes)
        plan.adjoint(yd, ao)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.trafo(fd, fo)
        plan.adjoint(yd, ao)
    for call in range(5):
        scale, ys = 1.0 + 0.5 * call, 2.0 - 0.25 * call
        with torch.cuda.stream(s):
            fd.copy_(f0 * scale)        # eager work on the stream between replays
            yd.copy_(y0 * ys)
            g.replay()
        torch.cuda.synchronize()
        e1 = rel(fo.cpu().numpy(), otr.forward(iset, x, fhat[0] * scale))
        e2 = rel(ao.cpu().numpy(), otr.adjoint(iset, x, y.reshape(-1) * ys))
        say(f"[graph] {prec} replay {call}: forward {e1:.2e} adjoint {e2:.2e}")
        assert e1 <= tol and e2 <= tol
    del g
    plan.close()
