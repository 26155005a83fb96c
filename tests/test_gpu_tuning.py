"""Launch choices and graph replay against the FP64 oracle.

Every forward gather a plan can be switched to, the configuration gt_plan_tune picks, and the
plan's own graph replays compute the transform to the same bars as the default launches
(relative l2 and max|err|/||input||_1, as in test_gpu_transform.py).  A second plan of the
same signature takes the cached choice without timing."""
import numpy as np
import pytest

import workloads as W
from oracle import index_set as oidx
from oracle import transform as otr
from paper_2010_10199_amd import lib
from tests.gpu_util import TOL, check, dtype_code, max_tol, say, to_dev

pytestmark = pytest.mark.gpu

# (name, d, ds, N, M, R): enough nodes per grid cell that every order can take the cell
# gather (and order 2 the polynomial gather in FP32)
CASES = [
    ("cells-3d-R2", 3, 3, (4, 4, 4), 30000, 2),
    ("order2-d5", 5, 2, (16, 8), 20000, 1),
]
NAMES = {lib.GT_GATHER_SORTED: "sorted", lib.GT_GATHER_CELL: "cell", lib.GT_GATHER_POLY: "poly",
         lib.GT_GATHER_DIRECT: "direct"}


def _setup(case, prec):
    import torch
    name, d, ds, N, M, R = case
    cid = 40 + CASES.index(case)
    iset = oidx.grouped_index_set(d, ds, N)
    x = W.uniform_nodes(W.rng(cid, W.P_NODES), M, d, prec)
    fhat = W.complex_normal(W.rng(cid, W.P_COEFFS), (R, iset.n_coeffs), prec)
    y = W.complex_normal(W.rng(cid, W.P_SAMPLES), (R, M), prec)
    p, keep = lib.make_problem(d, ds, N, M=M, R=R, dtype=dtype_code(prec))
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    ct = torch.complex64 if prec == "f32" else torch.complex128
    bufs = dict(fhat=to_dev(fhat.reshape(-1)), y=to_dev(y.reshape(-1)),
                f=torch.empty(R * M, dtype=ct, device="cuda"), a=torch.empty(R * iset.n_coeffs, dtype=ct, device="cuda"))
    torch.cuda.synchronize()
    ref_f = otr.forward(iset, x, fhat)
    ref_a = otr.adjoint(iset, x, y)
    return iset, x, fhat, y, plan, bufs, ref_f, ref_a


def _run(plan, bufs, stream, R, M, n):
    import torch
    plan.trafo(bufs["fhat"], bufs["f"], stream)
    plan.adjoint(bufs["y"], bufs["a"], stream)
    torch.cuda.synchronize()
    return (bufs["f"].cpu().numpy().astype(np.complex128).reshape(R, M),
            bufs["a"].cpu().numpy().astype(np.complex128).reshape(R, n))


def _check_both(label, got_f, got_a, fhat, y, ref_f, ref_a, prec, ds):
    check(f"{label} forward", got_f, ref_f, fhat, TOL[prec], max_tol(prec, ds))
    check(f"{label} adjoint", got_a, ref_a, y, TOL[prec], max_tol(prec, ds))


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_every_gather_form(case, prec):
    import torch
    name, d, ds, N, M, R = case
    say(f"[forms] {name} {prec}")
    iset, x, fhat, y, plan, bufs, ref_f, ref_a = _setup(case, prec)
    s = torch.cuda.Stream()
    for t in range(1, ds + 1):
        for path in (lib.GT_GATHER_SORTED, lib.GT_GATHER_CELL, lib.GT_GATHER_POLY, lib.GT_GATHER_DIRECT):
            if path == lib.GT_GATHER_POLY and (t != 2 or prec == "f64"):
                with pytest.raises(lib.GroupedError) as e:
                    plan.set_gather_path(t, path)
                assert e.value.code == lib.GT_EUNSUPPORTED
                continue
            plan.set_gather_path(t, path)
            assert plan.gather_path(t) == path
            f, a = _run(plan, bufs, s.cuda_stream, R, M, iset.n_coeffs)
            _check_both(f"order {t} {NAMES[path]}", f, a, fhat, y, ref_f, ref_a, prec, ds)
    for t in range(1, ds + 1):
        for form in (lib.GT_ADJ_DIRECT, lib.GT_ADJ_WINDOW):
            plan.set_adjoint_form(t, form)
            assert plan.adjoint_form(t) == form
            f, a = _run(plan, bufs, s.cuda_stream, R, M, iset.n_coeffs)
            _check_both(f"order {t} adjoint form {form}", f, a, fhat, y, ref_f, ref_a, prec, ds)
    plan.close()


# (name, d, ds, N, M, R): every order direct in both directions.  Right-hand sides 1, 9
# (two column blocks, padded) and 16; groups from 3 to 225 frequencies (the adjoint's row
# tiles per wavefront 1 to 8); node counts with a ragged last chunk.
DIRECT_CASES = [
    ("d5-N12-6-4-R1", 5, 3, (12, 6, 4), 1500, 1),
    ("d4-N32-16-R9", 4, 2, (32, 16), 2100, 9),
    ("d6-N8-8-6-R16", 6, 3, (8, 8, 6), 1300, 16),
    ("d3-N2-2-2-R3", 3, 3, (2, 2, 2), 700, 3),
]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", DIRECT_CASES, ids=[c[0] for c in DIRECT_CASES])
def test_direct_forms_match_oracle(case, prec):
    import torch
    name, d, ds, N, M, R = case
    say(f"[direct] {name} {prec}")
    cid = 60 + DIRECT_CASES.index(case)
    iset = oidx.grouped_index_set(d, ds, N)
    x = W.uniform_nodes(W.rng(cid, W.P_NODES), M, d, prec)
    fhat = W.complex_normal(W.rng(cid, W.P_COEFFS), (R, iset.n_coeffs), prec)
    y = W.complex_normal(W.rng(cid, W.P_SAMPLES), (R, M), prec)
    p, keep = lib.make_problem(d, ds, N, M=M, R=R, dtype=dtype_code(prec))
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    for t in range(1, ds + 1):
        plan.set_gather_path(t, lib.GT_GATHER_DIRECT)
        plan.set_adjoint_form(t, lib.GT_ADJ_DIRECT)
    ct = torch.complex64 if prec == "f32" else torch.complex128
    bufs = dict(fhat=to_dev(fhat.reshape(-1)), y=to_dev(y.reshape(-1)),
                f=torch.empty(R * M, dtype=ct, device="cuda"), a=torch.empty(R * iset.n_coeffs, dtype=ct, device="cuda"))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    f, a = _run(plan, bufs, s.cuda_stream, R, M, iset.n_coeffs)
    _check_both("direct", f, a, fhat, y, otr.forward(iset, x, fhat), otr.adjoint(iset, x, y), prec, ds)
    plan.close()


def test_direct_forms_availability():
    """Ragged datasets, more than 16 right-hand sides and (adjoint) groups of more than 256
    frequencies keep the window forms."""
    import torch
    d, ds, M = 3, 2, 400
    x = W.uniform_nodes(W.rng(70, W.P_NODES), M, d, "f32")
    for kw, fwd_ok, adj_ok in (
            (dict(N=(8, 18), M=M, R=1), True, False),            # order 2: 17^2 = 289 frequencies
            (dict(N=(8, 8), M=M, R=17), False, False),
            (dict(N=(8, 8), M=0, R=2, offsets=[0, 150, M]), False, False)):
        p, keep = lib.make_problem(d, ds, kw["N"], M=kw["M"], R=kw["R"], dtype=lib.GT_C64, offsets=kw.get("offsets"))
        plan = lib.Plan(p, to_dev(x), keepalive=keep)
        for want, call in ((fwd_ok, lambda: plan.set_gather_path(2, lib.GT_GATHER_DIRECT)),
                           (adj_ok, lambda: plan.set_adjoint_form(2, lib.GT_ADJ_DIRECT))):
            if want:
                call()
            else:
                with pytest.raises(lib.GroupedError) as e:
                    call()
                assert e.value.code == lib.GT_EUNSUPPORTED
        plan.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_weighted_lsqr_on_direct_forms(prec):
    """LSQR with Sobolev weights (the column scale enters both direct kernels) on a plan whose
    orders all use the direct sums, against the oracle's twelfth iterate: 1e-10 in FP64 (as
    the window forms' iterate test), 1e-3 in FP32 (the iteration carries the transforms'
    rounding along; a sanity bar, the kernels are the same templates as in FP64)."""
    import torch
    from oracle import lsqr as olsqr
    d, ds, N, M, R = 4, 3, (10, 6, 4), 2500, 2
    iset = oidx.grouped_index_set(d, ds, N)
    x = W.uniform_nodes(W.rng(71, W.P_NODES), M, d, prec)
    y1 = W.complex_normal(W.rng(71, W.P_SAMPLES), (M,), prec)
    K = iset.full_frequencies()
    omega = np.prod((1.0 + np.abs(K)) ** 0.5, axis=1)
    lambdas = [0.5, 20.0]
    p, keep = lib.make_problem(d, ds, N, M=M, R=R, dtype=dtype_code(prec))
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    for t in range(1, ds + 1):
        plan.set_gather_path(t, lib.GT_GATHER_DIRECT)
        plan.set_adjoint_form(t, lib.GT_ADJ_DIRECT)
    ct = torch.complex64 if prec == "f32" else torch.complex128
    out = torch.empty(R * iset.n_coeffs, dtype=ct, device="cuda")
    iters = 12
    plan.lsqr(to_dev(np.tile(y1, R)), lambdas, to_dev(omega), iters, 0.0, out)
    torch.cuda.synchronize()
    fg = out.cpu().numpy().astype(np.complex128).reshape(R, -1)
    bar = 1e-10 if prec == "f64" else 1e-3
    for r, lam in enumerate(lambdas):
        ref = olsqr.lsqr(lambda v: otr.forward(iset, x, v), lambda q: otr.adjoint(iset, x, q), y1, iset.n_coeffs,
                         lam, omega, iters)
        e = float(np.linalg.norm(fg[r] - ref.fhat) / np.linalg.norm(ref.fhat))
        say(f"  lsqr direct {prec} lambda={lam}: rel {e:.3e} (bar {bar:.0e})")
        assert e <= bar
    plan.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_tuned_plan_and_cached_choice(case, prec):
    import torch
    name, d, ds, N, M, R = case
    say(f"[tune] {name} {prec}")
    lib.release_all()   # no cached choice from earlier tests
    iset, x, fhat, y, plan, bufs, ref_f, ref_a = _setup(case, prec)
    assert plan.tuning() == {}
    s = torch.cuda.Stream()
    rep = plan.tune(s.cuda_stream)
    say(f"  report: {rep}")
    assert rep["cached"] is False and rep["forward_ms"] > 0 and rep["adjoint_ms"] > 0
    for t in range(1, ds + 1):
        chosen = rep["gather"][str(t)]["chosen"]
        assert NAMES[plan.gather_path(t)] == chosen
        assert rep["gather"][str(t)][chosen] == min(v for k, v in rep["gather"][str(t)].items() if k != "chosen")
    if ds >= 2:
        assert str(rep["tile_waves_cu"]["chosen"]) in rep["tile_waves_cu"]
    f, a = _run(plan, bufs, s.cuda_stream, R, M, iset.n_coeffs)
    _check_both("tuned", f, a, fhat, y, ref_f, ref_a, prec, ds)
    # a second plan of the same signature (other nodes) takes the cached choice
    x2 = W.uniform_nodes(W.rng(77, W.P_NODES), M, d, prec)
    p2, keep2 = lib.make_problem(d, ds, N, M=M, R=R, dtype=dtype_code(prec))
    plan2 = lib.Plan(p2, to_dev(x2), keepalive=keep2)
    rep2 = plan2.tuning()
    assert rep2["cached"] is True
    for t in range(1, ds + 1):
        assert plan2.gather_path(t) == plan.gather_path(t)
    f2, a2 = _run(plan2, bufs, s.cuda_stream, R, M, iset.n_coeffs)
    _check_both("cached", f2, a2, fhat, y, otr.forward(iset, x2, fhat), otr.adjoint(iset, x2, y), prec, ds)
    plan2.close()
    plan.close()
    lib.release_all()
    p3, keep3 = lib.make_problem(d, ds, N, M=M, R=R, dtype=dtype_code(prec))
    plan3 = lib.Plan(p3, to_dev(x2), keepalive=keep3)
    assert plan3.tuning() == {}   # the release cleared the cache
    plan3.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_graph_replays(case, prec):
    """Replays of the plan's captured graphs, with the program's own eager work and
    synchronisations between them and new input values in the same buffers, each checked
    against the oracle; a new output buffer gets a graph of its own."""
    import torch
    name, d, ds, N, M, R = case
    say(f"[graph] {name} {prec}")
    iset, x, fhat, y, plan, bufs, ref_f, ref_a = _setup(case, prec)
    s = torch.cuda.Stream()
    plan.set_graph(True)
    for rep in range(4):
        fh = W.complex_normal(W.rng(500 + rep, W.P_COEFFS), (R, iset.n_coeffs), prec)
        yy = W.complex_normal(W.rng(500 + rep, W.P_SAMPLES), (R, M), prec)
        bufs["fhat"].copy_(to_dev(fh.reshape(-1)))
        bufs["y"].copy_(to_dev(yy.reshape(-1)))
        junk = torch.randn(1 << 16, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        f, a = _run(plan, bufs, s.cuda_stream, R, M, iset.n_coeffs)
        assert torch.isfinite(junk)
        _check_both(f"replay {rep}", f, a, fh, yy, otr.forward(iset, x, fh), otr.adjoint(iset, x, yy), prec, ds)
    ct = bufs["f"].dtype
    other = dict(bufs, f=torch.empty(R * M, dtype=ct, device="cuda"),
                 a=torch.empty(R * iset.n_coeffs, dtype=ct, device="cuda"))
    fh = W.complex_normal(W.rng(500 + 3, W.P_COEFFS), (R, iset.n_coeffs), prec)
    yy = W.complex_normal(W.rng(500 + 3, W.P_SAMPLES), (R, M), prec)
    f, a = _run(plan, other, s.cuda_stream, R, M, iset.n_coeffs)
    _check_both("new buffers", f, a, fh, yy, otr.forward(iset, x, fh), otr.adjoint(iset, x, yy), prec, ds)
    plan.set_graph(False)
    f, a = _run(plan, other, s.cuda_stream, R, M, iset.n_coeffs)
    _check_both("eager again", f, a, fh, yy, otr.forward(iset, x, fh), otr.adjoint(iset, x, yy), prec, ds)
    plan.close()


# (name, d, ds, N, M or ragged sizes, R, prec)
UPDATE_CASES = [
    ("shared-R2-f32", 4, 2, (16, 8), 20000, 2, "f32"),
    ("shared-3d-f64", 4, 3, (8, 6, 4), 6000, 1, "f64"),
    ("ragged-f32", 3, 2, (12, 8), [4000, 0, 9000, 2500], 4, "f32"),
    # the update's per-(term, dataset) sort: empty datasets first, last and in a row, one-node
    # datasets
    ("ragged-many-f64", 3, 2, (12, 8), [0, 1, 0, 0, 37, 5, 1, 2600, 0, 300, 0], 11, "f64"),
]


@pytest.mark.parametrize("case", UPDATE_CASES, ids=[c[0] for c in UPDATE_CASES])
def test_update_nodes_matches_oracle(case):
    """gt_plan_update_nodes: after moving the nodes (twice, the second time back to a copy of
    the first set) the plan's transforms match the oracle for the new nodes; the order-2 tile
    list rebuilt on the device gives the same order-2 adjoint coefficients as a fresh plan's
    host-built one (same kernels, same segment order: bit for bit); a retune afterwards rebuilds the cell items
    from the new positions; NaN nodes are rejected and a later update recovers."""
    import torch
    name, d, ds, N, Msz, R, prec = case
    say(f"[update] {name}")
    cid = 80 + UPDATE_CASES.index(case)
    iset = oidx.grouped_index_set(d, ds, N)
    ragged = isinstance(Msz, list)
    Mx = sum(Msz) if ragged else Msz
    offsets = list(np.concatenate([[0], np.cumsum(Msz)])) if ragged else None
    x0 = W.uniform_nodes(W.rng(cid, W.P_NODES), Mx, d, prec)
    x1 = W.uniform_nodes(W.rng(cid + 100, W.P_NODES), Mx, d, prec)
    fhat = W.complex_normal(W.rng(cid, W.P_COEFFS), (R, iset.n_coeffs), prec)
    ny = R * Mx if not ragged else Mx
    y = W.complex_normal(W.rng(cid, W.P_SAMPLES), (ny,), prec)
    p, keep = lib.make_problem(d, ds, N, M=0 if ragged else Mx, R=R, dtype=dtype_code(prec), offsets=offsets)
    plan = lib.Plan(p, to_dev(x0), keepalive=keep)
    ct = torch.complex64 if prec == "f32" else torch.complex128
    fd, yd = to_dev(fhat.reshape(-1)), to_dev(y)
    f = torch.empty(ny, dtype=ct, device="cuda")
    a = torch.empty(R * iset.n_coeffs, dtype=ct, device="cuda")

    def run(pl):
        pl.trafo(fd, f)
        pl.adjoint(yd, a)
        torch.cuda.synchronize()
        return f.cpu().numpy().astype(np.complex128), a.cpu().numpy().astype(np.complex128).reshape(R, -1)

    def oracle(xx):
        if not ragged:
            return otr.forward(iset, xx, fhat).reshape(-1), otr.adjoint(iset, xx, y.reshape(R, Mx))
        fo = np.zeros(Mx, complex)
        ao = np.zeros((R, iset.n_coeffs), complex)
        for b in range(R):
            lo, hi = offsets[b], offsets[b + 1]
            if hi > lo:
                fo[lo:hi] = otr.forward(iset, xx[lo:hi], fhat[b])
                ao[b] = otr.adjoint(iset, xx[lo:hi], y[lo:hi])
        return fo, ao

    for step, xx in enumerate((x1, x0.copy())):
        plan.update_nodes(to_dev(xx))
        for t in range(1, ds + 1):
            assert plan.gather_path(t) == lib.GT_GATHER_SORTED
        got_f, got_a = run(plan)
        ref_f, ref_a = oracle(xx)
        check(f"update {step} forward", got_f, ref_f, fhat, TOL[prec], max_tol(prec, ds))
        check(f"update {step} adjoint", got_a, ref_a, y.reshape(R, -1) if not ragged else y, TOL[prec],
              max_tol(prec, ds))
        fresh_p, fresh_k = lib.make_problem(d, ds, N, M=0 if ragged else Mx, R=R, dtype=dtype_code(prec),
                                            offsets=offsets)
        fresh = lib.Plan(fresh_p, to_dev(xx), keepalive=fresh_k)
        _, fresh_a = run(fresh)
        fresh.close()
        # the coefficients of orders 1 and 2 (the order-1 spread sums its grid copies in a fixed
        # order, the tile spread its patches; order 3 adds into one grid with LDS atomics)
        for order in (1, 2):
            sel = np.concatenate([np.arange(iset.offsets[i], iset.offsets[i + 1])
                                  for i, u in enumerate(iset.terms) if len(u) == order] or [np.zeros(0, int)])
            assert np.array_equal(got_a[:, sel], fresh_a[:, sel]), \
                f"order {order}: the moved plan differs from a fresh plan for the same nodes"
    s = torch.cuda.Stream()
    plan.tune(s.cuda_stream)
    torch.cuda.synchronize()
    got_f, got_a = run(plan)
    ref_f, ref_a = oracle(x0)
    check("retuned forward", got_f, ref_f, fhat, TOL[prec], max_tol(prec, ds))
    bad = x1.copy()
    bad[Mx // 2, 0] = np.nan
    with pytest.raises(lib.GroupedError) as e:
        plan.update_nodes(to_dev(bad))
    assert e.value.code == lib.GT_EINVAL
    plan.update_nodes(to_dev(x1))
    got_f, got_a = run(plan)
    ref_f, ref_a = oracle(x1)
    check("after a rejected update forward", got_f, ref_f, fhat, TOL[prec], max_tol(prec, ds))
    plan.close()


def test_side_streams_are_reused_across_plans():
    """A destroyed plan's second stream goes to the next plan on the device: plans created one
    after another, two plans alive at once, and a plan created after gt_release_all (which
    destroys the kept streams) all match the oracle, with order 1 on the second stream."""
    import torch
    d, ds, N, M = 4, 2, (12, 6), 2000
    iset = oidx.grouped_index_set(d, ds, N)
    x = W.uniform_nodes(W.rng(77, W.P_NODES), M, d, "f64")
    fhat = W.complex_normal(W.rng(77, W.P_COEFFS), (1, iset.n_coeffs), "f64")
    y = W.complex_normal(W.rng(77, W.P_SAMPLES), (M,), "f64")
    ref_f = otr.forward(iset, x, fhat).reshape(-1)
    ref_a = otr.adjoint(iset, x, y.reshape(1, M)).reshape(-1)
    xd, fd, yd = to_dev(x), to_dev(fhat.reshape(-1)), to_dev(y)

    def new_plan():
        p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C128)
        return lib.Plan(p, xd, keepalive=keep)

    def check_plan(pl, label):
        f = torch.empty(M, dtype=torch.complex128, device="cuda")
        a = torch.empty(iset.n_coeffs, dtype=torch.complex128, device="cuda")
        pl.trafo(fd, f)
        pl.adjoint(yd, a)
        torch.cuda.synchronize()
        check(f"{label} forward", f.cpu().numpy(), ref_f, fhat, TOL["f64"], max_tol("f64", ds))
        check(f"{label} adjoint", a.cpu().numpy(), ref_a, y, TOL["f64"], max_tol("f64", ds))

    for k in range(3):                      # one after another: each takes the last one's stream
        pl = new_plan()
        check_plan(pl, f"sequential {k}")
        pl.close()
    p1, p2 = new_plan(), new_plan()         # alive together: two different streams
    check_plan(p1, "pair 1")
    check_plan(p2, "pair 2")
    p1.close()
    p2.close()
    lib.release_all()                       # the kept streams destroyed
    pl = new_plan()
    check_plan(pl, "after release")
    pl.close()
