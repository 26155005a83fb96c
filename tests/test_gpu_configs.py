"""GPU parity at the shapes of the remaining workloads, at full size where the oracle can
check sampled outputs one by one:

* d=20, d_s=3, N=(32, 12, 6), 1,351 terms, 166,111 coefficients, M=500,000 (batched LSQR
  workload): FP32 forward on sampled nodes and adjoint on sampled coefficients (each an
  exact sum over all 500,000 nodes), 16 right-hand sides on a reduced node set;
* d=12, d_s=2, N=(48, 16), 79 terms, 15,415 coefficients, M=200,000 (group-lasso
  workload): FP32 and FP64 sampled transforms, and FISTA on a reduced node set against the
  oracle's iterations with the same step constant.

Bars as in test_gpu_transform.py: 1e-5 (FP32) and 1e-12 (FP64 at its default window)
relative l2 error over the sampled outputs, and the per-element bar max|error| / ||input||_1."""
import numpy as np
import pytest

import workloads as W
from oracle import fista as ofista
from oracle import index_set as oidx
from oracle import transform as otr
from paper_2010_10199_amd import lib
from tests.gpu_util import (TOL, gpu_adjoint, gpu_trafo, max_err, max_tol, oracle_adjoint_at, oracle_forward_at, rel,
                            say)
from tests.test_gpu_solvers import _fista_gpu

pytestmark = pytest.mark.gpu

C3 = (20, 3, (32, 12, 6))
C4 = (12, 2, (48, 16))


def _sampled(iset, x, fhat, y, f, a, nodes, per_order, seed=0):
    """Forward on `nodes` sampled nodes and adjoint on the empty set plus per_order[t]
    coefficients drawn uniformly from the coefficients of order t; returns the relative l2
    errors, the per-element errors relative to ||fhat||_1 and ||y||_1 (the form of the fast
    transform's error bound) and the sample sizes."""
    g = np.random.default_rng(seed)
    M = x.shape[0]
    S = np.sort(g.choice(M, nodes, replace=False))
    order = np.concatenate([np.full(iset.term_slice(i).stop - iset.term_slice(i).start, len(iset.terms[i]))
                            for i in range(iset.n_terms)])
    K = [0]
    for t, cnt in per_order.items():
        pool = np.flatnonzero(order == t)
        K += list(g.choice(pool, min(cnt, len(pool)), replace=False))
    K = np.array(sorted(set(int(k) for k in K)))
    rf = oracle_forward_at(iset, x, fhat, S)
    ra = oracle_adjoint_at(iset, x, y, K)
    return (rel(f[S], rf), rel(a[K], ra), max_err(f[S], rf, fhat), max_err(a[K], ra, y), len(S), len(K),
            {t: int((order[K] == t).sum()) for t in per_order})


def test_config3_full_size_sampled_fp32():
    """Full size in FP32: forward on 5,000 sampled nodes, adjoint on 1,101 sampled
    coefficients (the empty set, 200 of order 1, 500 of order 2, 400 of order 3), each an
    exact sum over all 500,000 nodes."""
    d, ds, N = C3
    M = 500000
    iset = oidx.grouped_index_set(d, ds, N)
    x, fhat, y = W.trafo_inputs(3, d, ds, M, iset.n_coeffs, 1, "f32")
    say(f"[config3] fp32 M={M} terms={iset.n_terms} coeffs={iset.n_coeffs}")
    f = gpu_trafo(d, ds, N, x, fhat, "f32")[0]
    a = gpu_adjoint(d, ds, N, x, y.reshape(1, M), "f32", iset.n_coeffs)[0]
    e1, e2, m1, m2, ns, nk, by = _sampled(iset, x, fhat[0], y.reshape(-1), f, a, 5000, {1: 200, 2: 500, 3: 400})
    mt = max_tol("f32", ds)
    say(f"  forward {e1:.3e} max/l1 {m1:.3e} ({ns} nodes) adjoint {e2:.3e} max/l1 {m2:.3e} ({nk} coefficients, "
        f"per order {by}); max tol {mt:.1e}")
    assert by[3] >= 300 and nk >= 1000
    assert e1 <= TOL["f32"] and e2 <= TOL["f32"] and m1 <= mt and m2 <= mt


def test_config3_sixteen_rhs_reduced():
    """16 right-hand sides in one launch (as the batched LSQR runs them) on 20,000 nodes:
    every right-hand side checked on sampled outputs."""
    d, ds, N = C3
    M, R = 20000, 16
    iset = oidx.grouped_index_set(d, ds, N)
    x, fhat, y = W.trafo_inputs(3, d, ds, M, iset.n_coeffs, R, "f32")
    f = gpu_trafo(d, ds, N, x, fhat, "f32", R=R)
    a = gpu_adjoint(d, ds, N, x, y.reshape(R, M), "f32", iset.n_coeffs, R=R)
    mt = max_tol("f32", ds)
    for r in range(R):
        e1, e2, m1, m2, _, _, _ = _sampled(iset, x, fhat[r], y.reshape(R, M)[r], f[r], a[r], 100,
                                           {1: 10, 2: 10, 3: 10}, seed=r)
        say(f"[config3 R=16] r={r} forward {e1:.3e} ({m1:.1e}) adjoint {e2:.3e} ({m2:.1e})")
        assert e1 <= TOL["f32"] and e2 <= TOL["f32"] and m1 <= mt and m2 <= mt


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_config4_full_size_sampled(prec):
    d, ds, N = C4
    M = 200000
    iset = oidx.grouped_index_set(d, ds, N)
    x, fhat, y = W.trafo_inputs(4, d, ds, M, iset.n_coeffs, 1, prec)
    say(f"[config4] {prec} M={M}")
    f = gpu_trafo(d, ds, N, x, fhat, prec)[0]
    a = gpu_adjoint(d, ds, N, x, y.reshape(1, M), prec, iset.n_coeffs)[0]
    e1, e2, m1, m2, ns, nk, by = _sampled(iset, x, fhat[0], y.reshape(-1), f, a, 3000, {1: 150, 2: 350})
    mt = max_tol(prec, ds)
    say(f"  forward {e1:.3e} max/l1 {m1:.3e} ({ns} nodes) adjoint {e2:.3e} max/l1 {m2:.3e} ({nk} coefficients, "
        f"per order {by}); max tol {mt:.1e}")
    assert e1 <= TOL[prec] and e2 <= TOL[prec] and m1 <= mt and m2 <= mt


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_config4_fista_reduced_vs_oracle(prec):
    """Group lasso on the d=12 shape with the B-spline target (3 one- and 2 two-dimensional
    terms) + 1% noise on 600 nodes; two lambda values of the lambda_max grid, 10 constant
    steps with the same L (1.5 x a 10-step oracle power iteration) on both sides."""
    d, ds, N = C4
    M = 600
    iset = oidx.grouped_index_set(d, ds, N)
    x = W.uniform_nodes(W.rng(4, W.P_NODES, 1), M, d, prec)
    y = W.add_noise(W.rng(4, W.P_NOISE, 1), W.bspline_target(x).astype(np.complex128), 0.01)
    y = y.astype(np.complex64 if prec == "f32" else np.complex128)
    A = lambda v: otr.forward(iset, x, v)
    AH = lambda r: otr.adjoint(iset, x, r)
    g = AH(y.astype(np.complex128))
    lam_max = max(np.linalg.norm(g[iset.term_slice(i)]) for i in range(iset.n_terms))
    lams = [lam_max * 10 ** (-3 * j / 7) for j in (2, 5)]
    L = 1.5 * ofista.power_iteration(A, AH, iset.n_coeffs, 10)
    K = 10
    fg, _ = _fista_gpu(d, ds, N, x, np.tile(y, 2).reshape(2, M), lams, prec, K, L)
    for r, lam in enumerate(lams):
        ref = ofista.fista(A, AH, y.astype(np.complex128), iset.offsets, lam, L, K)
        e = rel(fg[r], ref.fhat)
        act = sum(np.linalg.norm(ref.fhat[iset.term_slice(i)]) > 0 for i in range(iset.n_terms))
        say(f"[config4 fista] {prec} lambda={lam:.4g} rel {e:.3e} active groups {act}")
        assert e <= (1e-5 if prec == "f32" else 1e-10)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_config4_fista_eight_lambdas_dense_oracle(prec):
    """The group-lasso shape (d=12, d_s=2, N=48/16: 79 groups, 15,415 coefficients) on 3,000
    nodes with the B-spline target + 1 % noise and all eight lambda values of the benchmark's
    grid (lambda_max 10^(-3j/7)) in one batched call, 15 constant steps, against the oracle's
    iterates with the dense matrix of eq. FM as its operator (L = 1.05 x a 20-step oracle
    power iteration on the same matrix)."""
    d, ds, N = C4
    M, K = 3000, 15
    iset = oidx.grouped_index_set(d, ds, N)
    x = W.uniform_nodes(W.rng(4, W.P_NODES, 2), M, d, prec)
    y = W.add_noise(W.rng(4, W.P_NOISE, 2), W.bspline_target(x).astype(np.complex128), 0.01)
    y = y.astype(np.complex64 if prec == "f32" else np.complex128)
    A = otr.dense_matrix(iset, x)
    mv = lambda v: A @ v
    rmv = lambda u: (u.conj() @ A).conj()
    g = rmv(y.astype(np.complex128))
    lam_max = max(np.linalg.norm(g[iset.term_slice(i)]) for i in range(iset.n_terms))
    lams = [lam_max * 10 ** (-3 * j / 7) for j in range(8)]
    L = 1.05 * ofista.power_iteration(mv, rmv, iset.n_coeffs, 20)
    say(f"[config4 fista dense] {prec} M={M} lambda_max={lam_max:.4g} L={L:.4g}")
    fg, _ = _fista_gpu(d, ds, N, x, np.tile(y, 8).reshape(8, M), lams, prec, K, L)
    refs = [ofista.fista(mv, rmv, y.astype(np.complex128), iset.offsets, lam, L, K).fhat for lam in lams]
    big = max(np.linalg.norm(f) for f in refs)
    worst = 0.0
    for r, lam in enumerate(lams):
        # (the zero solution at lambda_max is compared relative to the largest solution)
        nrm = np.linalg.norm(refs[r])
        e = float(np.linalg.norm(fg[r] - refs[r]) / (nrm if nrm > 1e-12 * big else big))
        worst = max(worst, e)
        say(f"  lambda={lam:.4g}: rel {e:.3e}")
    assert worst <= (1e-5 if prec == "f32" else 1e-10)
    del A


@pytest.fixture(scope="module")
def config3_lsqr_slice():
    """The batched-LSQR workload's index set (d=20, d_s=3, N=32/12/6: 1,351 groups, 166,111
    coefficients) on an 800-node slice: the sparse trigonometric target (8 monomials) + 1 %
    noise, 16 lambda = logspace(-4, 1), and the oracle's 5-iterate LSQR for every lambda
    (dense matrix of eq. FM as its operator)."""
    from oracle import lsqr as olsqr
    d, ds, N = C3
    M, K = 800, 5
    iset = oidx.grouped_index_set(d, ds, N)
    x = W.uniform_nodes(W.rng(3, W.P_NODES, 1), M, d, "f32")
    target, _ = W.sparse_trig_target(3, x, N)
    y = W.add_noise(W.rng(3, W.P_NOISE, 1), target, 0.01).astype(np.complex64)
    lams = np.logspace(-4, 1, 16)
    A = otr.dense_matrix(iset, x)
    mv = lambda v: A @ v
    rmv = lambda u: (u.conj() @ A).conj()
    ref = np.stack([olsqr.lsqr(mv, rmv, y.astype(np.complex128), iset.n_coeffs, lam, None, K).fhat for lam in lams])
    del A
    return d, ds, N, M, K, iset, x, y, lams, ref


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_config3_lsqr_sixteen_lambdas_vs_oracle(config3_lsqr_slice, prec):
    """All 16 lambda values in one call (lsqr_solve_path: one shared bidiagonalisation) and
    as 16 right-hand sides with their own lambda (lsqr_solve), against the oracle's iterates
    for every lambda; the two GPU forms agree with each other."""
    import torch
    from tests.gpu_util import cdtype, dtype_code, to_dev
    d, ds, N, M, K, iset, x, y, lams, ref = config3_lsqr_slice
    L = len(lams)
    xd = to_dev(x.astype(np.float32 if prec == "f32" else np.float64))
    yd = to_dev(y if prec == "f32" else y.astype(np.complex128))
    p1, k1 = lib.make_problem(d, ds, N, M=M, R=1, dtype=dtype_code(prec))
    path = torch.empty(L * iset.n_coeffs, dtype=cdtype(prec), device="cuda")
    info = lib.lsqr_solve_path(p1, xd, yd, lams, None, K, 0.0, path)
    got_path = path.cpu().numpy().astype(np.complex128).reshape(L, -1)
    pR, kR = lib.make_problem(d, ds, N, M=M, R=L, dtype=dtype_code(prec))
    outR = torch.empty(L * iset.n_coeffs, dtype=cdtype(prec), device="cuda")
    lib.lsqr_solve(pR, xd, yd.repeat(L), lams, None, K, 0.0, outR)
    got_rhs = outR.cpu().numpy().astype(np.complex128).reshape(L, -1)
    tol = 1e-5 if prec == "f32" else 1e-10
    worst = 0.0
    for j, lam in enumerate(lams):
        e1, e2 = rel(got_path[j], ref[j]), rel(got_rhs[j], ref[j])
        worst = max(worst, e1, e2)
        assert info[j][0].iters == K
        say(f"[config3 lsqr] {prec} lambda={lam:.3e}: path {e1:.2e} per-rhs {e2:.2e}")
        assert e1 <= tol and e2 <= tol
    agree = rel(got_path, got_rhs)
    say(f"[config3 lsqr] {prec} worst {worst:.2e}; path vs per-rhs {agree:.2e}")
    assert agree <= (1e-5 if prec == "f32" else 1e-12)
