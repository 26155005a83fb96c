"""GPU parity at the shapes of the remaining workloads, at full size where the oracle can
check sampled outputs one by one:

* d=20, d_s=3, N=(32, 12, 6), 1,351 terms, 166,111 coefficients, M=500,000 (batched LSQR
  workload): FP32 forward on sampled nodes and adjoint on sampled coefficients (each an
  exact sum over all 500,000 nodes), 16 right-hand sides on a reduced node set;
* d=12, d_s=2, N=(48, 16), 79 terms, 15,415 coefficients, M=200,000 (group-lasso
  workload): FP32 and FP64 sampled transforms, and FISTA on a reduced node set against the
  oracle's iterations with the same step constant.

Bars as in test_gpu_transform.py: 1e-5 (FP32) and 1e-12 (FP64 at its default window)
relative l2 error over the sampled outputs."""
import numpy as np
import pytest

import workloads as W
from oracle import fista as ofista
from oracle import index_set as oidx
from oracle import transform as otr
from tests.gpu_util import TOL, gpu_adjoint, gpu_trafo, rel, say
from tests.test_gpu_solvers import _fista_gpu

pytestmark = pytest.mark.gpu

C3 = (20, 3, (32, 12, 6))
C4 = (12, 2, (48, 16))


def _sampled(iset, x, fhat, y, f, a, nodes, coeffs, seed=0):
    g = np.random.default_rng(seed)
    M = x.shape[0]
    S = np.sort(g.choice(M, nodes, replace=False))
    # coefficients: the empty set, some of every order
    K = [0]
    for t in range(1, 4):
        terms = [i for i in range(iset.n_terms) if len(iset.terms[i]) == t]
        if not terms:
            continue
        for i in g.choice(terms, min(len(terms), coeffs // 3), replace=False):
            sl = iset.term_slice(int(i))
            K.append(int(g.integers(sl.start, sl.stop)))
    K = np.array(sorted(set(K)))
    e1 = rel(f[S], otr.forward(iset, x[S], fhat))
    e2 = rel(a[K], otr.adjoint_at(iset, x, y, K))
    return e1, e2, len(S), len(K)


def test_config3_full_size_sampled_fp32():
    d, ds, N = C3
    M = 500000
    iset = oidx.grouped_index_set(d, ds, N)
    x, fhat, y = W.trafo_inputs(3, d, ds, M, iset.n_coeffs, 1, "f32")
    say(f"[config3] fp32 M={M} terms={iset.n_terms} coeffs={iset.n_coeffs}")
    f = gpu_trafo(d, ds, N, x, fhat, "f32")[0]
    a = gpu_adjoint(d, ds, N, x, y.reshape(1, M), "f32", iset.n_coeffs)[0]
    e1, e2, ns, nk = _sampled(iset, x, fhat[0], y.reshape(-1), f, a, 300, 45)
    say(f"  forward {e1:.3e} ({ns} nodes) adjoint {e2:.3e} ({nk} coefficients)")
    assert e1 <= TOL["f32"] and e2 <= TOL["f32"]


def test_config3_sixteen_rhs_reduced():
    """16 right-hand sides in one launch (as the batched LSQR runs them) on 20,000 nodes:
    every right-hand side checked on sampled outputs."""
    d, ds, N = C3
    M, R = 20000, 16
    iset = oidx.grouped_index_set(d, ds, N)
    x, fhat, y = W.trafo_inputs(3, d, ds, M, iset.n_coeffs, R, "f32")
    f = gpu_trafo(d, ds, N, x, fhat, "f32", R=R)
    a = gpu_adjoint(d, ds, N, x, y.reshape(R, M), "f32", iset.n_coeffs, R=R)
    worst = 0.0
    for r in (0, 7, 15):
        e1, e2, _, _ = _sampled(iset, x, fhat[r], y.reshape(R, M)[r], f[r], a[r], 100, 30, seed=r)
        say(f"[config3 R=16] r={r} forward {e1:.3e} adjoint {e2:.3e}")
        worst = max(worst, e1, e2)
    assert worst <= TOL["f32"]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_config4_full_size_sampled(prec):
    d, ds, N = C4
    M = 200000
    iset = oidx.grouped_index_set(d, ds, N)
    x, fhat, y = W.trafo_inputs(4, d, ds, M, iset.n_coeffs, 1, prec)
    say(f"[config4] {prec} M={M}")
    f = gpu_trafo(d, ds, N, x, fhat, prec)[0]
    a = gpu_adjoint(d, ds, N, x, y.reshape(1, M), prec, iset.n_coeffs)[0]
    e1, e2, ns, nk = _sampled(iset, x, fhat[0], y.reshape(-1), f, a, 1500, 90)
    say(f"  forward {e1:.3e} ({ns} nodes) adjoint {e2:.3e} ({nk} coefficients)")
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


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
