"""GPU parity of the grouped transform in the half-period cosine basis (Sec. 5) against the
FP64 cosine oracle: forward and adjoint element by element (relative l2 error and the
per-element bar max|error| / ||input||_1), the adult-data shape at the paper's training size
on sampled outputs, LSQR and FISTA iterates, and the node gradient.  Bars as for the
exponential basis: 1e-5 (FP32) and 1e-12 (FP64); the FP32 path is compared with the oracle
on the FP32-rounded inputs."""
import numpy as np
import pytest

import workloads as W
from oracle import cosine as ocos
from oracle import fista as ofista
from oracle import lsqr as olsqr
from paper_2010_10199_amd import lib
from tests.gpu_util import TOL, cdtype, check, dtype_code, max_err, max_tol, rel, say, to_dev

pytestmark = pytest.mark.gpu

# (name, d, ds, N, M or ragged sizes, R)
CASES = [
    ("1d", 3, 1, (16,), 700, 1),
    ("2d-two-rhs", 4, 2, (12, 6), 1500, 2),
    ("3d", 4, 3, (8, 6, 4), 900, 1),
    ("ragged-with-empty", 3, 2, (10, 6), [400, 0, 1100], 3),
    ("only-empty-set", 3, 0, (), 300, 1),
    ("bandwidth-2", 3, 3, (2, 2, 2), 500, 1),
    ("cells-2d", 3, 2, (8, 6), 20000, 1),
]


def _run(d, ds, N, x, fhat, y, prec, R=1, offsets=None):
    import torch
    Mx = x.shape[0]
    p, keep = lib.make_problem(d, ds, N, M=Mx if offsets is None else 0, R=R, dtype=dtype_code(prec),
                               offsets=offsets, basis=lib.GT_BASIS_COS)
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    nout = R * Mx if offsets is None else Mx
    f = torch.empty(nout, dtype=cdtype(prec), device="cuda")
    a = torch.empty(fhat.size, dtype=cdtype(prec), device="cuda")
    plan.trafo(to_dev(fhat.reshape(-1)), f)
    plan.adjoint(to_dev(y.reshape(-1)), a)
    torch.cuda.synchronize()
    plan.close()
    return f.cpu().numpy().astype(np.complex128), a.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_cosine_forward_and_adjoint_parity(case, prec):
    name, d, ds, N, Msz, R = case
    cid = CASES.index(case)
    ragged = isinstance(Msz, list)
    Mx = sum(Msz) if ragged else Msz
    iset = ocos.cosine_index_set(d, ds, N)
    x = W.unit_cube_nodes(W.rng(300 + cid, W.P_NODES), Mx, d, prec)
    fhat = W.complex_normal(W.rng(300 + cid, W.P_COEFFS), (R, iset.n_coeffs), prec)
    y = W.complex_normal(W.rng(300 + cid, W.P_SAMPLES), (Mx if ragged else R * Mx,), prec)
    offsets = list(np.concatenate([[0], np.cumsum(Msz)])) if ragged else None
    say(f"[cosine] {name} {prec} d={d} ds={ds} N={N} M={Msz} R={R}")
    f, a = _run(d, ds, N, x, fhat, y, prec, R, offsets)
    tol, mtol = TOL[prec], max_tol(prec, ds)
    if not ragged:
        check("forward", f.reshape(R, Mx), ocos.forward(iset, x, fhat), fhat, tol, mtol)
        check("adjoint", a.reshape(R, -1), ocos.adjoint(iset, x, y.reshape(R, Mx)), y.reshape(R, Mx), tol, mtol)
    else:
        for b in range(R):
            sl = slice(offsets[b], offsets[b + 1])
            if offsets[b + 1] > offsets[b]:
                check(f"forward dataset {b}", f[sl], ocos.forward(iset, x[sl], fhat[b]), fhat[b], tol, mtol)
                check(f"adjoint dataset {b}", a.reshape(R, -1)[b], ocos.adjoint(iset, x[sl], y[sl]), y[sl], tol, mtol)
            else:
                assert not np.any(a.reshape(R, -1)[b])


def test_cosine_nodes_on_and_outside_the_cube():
    """Nodes at 0 and 1 and outside [0, 1] (the basis' even, 2-periodic extension) give the
    oracle's values at the same points."""
    d, ds, N = 2, 2, (8, 6)
    iset = ocos.cosine_index_set(d, ds, N)
    x = np.array([[0.0, 1.0], [1.0, 0.0], [0.5, 0.25], [-0.3, 1.7], [2.25, -1.0], [0.999999, 1e-9]])
    fhat = W.complex_normal(W.rng(310, W.P_COEFFS), (1, iset.n_coeffs), "f64")
    y = W.complex_normal(W.rng(310, W.P_SAMPLES), (x.shape[0],), "f64")
    f, a = _run(d, ds, N, x, fhat, y, "f64")
    e1, e2 = rel(f, ocos.forward(iset, x, fhat[0])), rel(a, ocos.adjoint(iset, x, y))
    say(f"[cosine edges] forward {e1:.2e} adjoint {e2:.2e}")
    assert e1 <= 1e-12 and e2 <= 1e-12


def test_cosine_adult_shape_full_size_fp32():
    """The adult-data model of Sec. 5 (d = 12, d_s = 2, N = 82 / 10: 79 terms, 6,319
    coefficients) at the paper's training size M = 36,160 with synthetic nodes on [0, 1]^12:
    forward on 2,000 sampled nodes, adjoint on 300 sampled coefficients (exact sums over all
    nodes)."""
    d, ds, N, M = 12, 2, (82, 10), 36160
    iset = ocos.cosine_index_set(d, ds, N)
    assert iset.n_coeffs == 6319 and iset.n_terms == 79
    x = W.unit_cube_nodes(W.rng(311, W.P_NODES), M, d, "f32")
    fhat = W.complex_normal(W.rng(311, W.P_COEFFS), (1, iset.n_coeffs), "f32")
    y = W.complex_normal(W.rng(311, W.P_SAMPLES), (M,), "f32")
    f, a = _run(d, ds, N, x, fhat, y, "f32")
    g = np.random.default_rng(5)
    S = np.sort(g.choice(M, 2000, replace=False))
    K = np.sort(g.choice(iset.n_coeffs, 300, replace=False))
    mtol = max_tol("f32", ds)
    check("forward (2,000 nodes)", f[S], ocos.forward(iset, x[S], fhat[0]), fhat, TOL["f32"], mtol)
    sub = ocos.adjoint(iset, x, y)[K]
    check("adjoint (300 coefficients)", a[K], sub, y, TOL["f32"], mtol)


def _cos_problem(seed, prec="f64"):
    d, ds, N, M = 4, 2, (10, 6), 2500
    iset = ocos.cosine_index_set(d, ds, N)
    x = W.unit_cube_nodes(W.rng(seed, W.P_NODES), M, d, prec)
    ft = W.complex_normal(W.rng(seed, W.P_COEFFS), (iset.n_coeffs,), "f64")
    f = np.zeros(iset.n_coeffs, dtype=complex)
    for ti in (1, 3, 6):
        f[iset.term_slice(ti)] = ft[iset.term_slice(ti)]
    y = ocos.forward(iset, x, f) + 0.05 * W.complex_normal(W.rng(seed, W.P_NOISE), (M,), "f64")
    return d, ds, N, M, iset, x, y.astype(np.complex64 if prec == "f32" else np.complex128)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cosine_lsqr_and_fista_iterates_match_oracle(prec):
    """LSQR and FISTA (constant step, two lambda values) on the cosine basis against the
    oracle with the cosine matrix as operator.  LSQR: FP64 iterates of the weighted problem
    (12 steps) against the oracle's; FP32 converged solutions against the dense normal
    equations (LSQR iterates amplify the FP32 rounding of the transforms through the loss of
    orthogonality of the bidiagonalisation, so they are compared only in FP64).  FISTA:
    iterates in both precisions."""
    import torch
    d, ds, N, M, iset, x, y = _cos_problem(312, prec)
    A = lambda v: ocos.forward(iset, x, v)
    AH = lambda r: ocos.adjoint(iset, x, r)
    omega = np.prod((1.0 + np.abs(iset.full_frequencies())) ** 1.0, axis=1)
    lams = [0.3, 30.0]
    p, keep = lib.make_problem(d, ds, N, M=M, R=2, dtype=dtype_code(prec), basis=lib.GT_BASIS_COS)
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    yy = to_dev(np.tile(y, 2))
    out = torch.empty(2 * iset.n_coeffs, dtype=cdtype(prec), device="cuda")
    tol = 1e-10 if prec == "f64" else 1e-5
    if prec == "f64":
        plan.lsqr(yy, lams, to_dev(omega), 12, 0.0, out)
        got = out.cpu().numpy().reshape(2, -1)
        for r, lam in enumerate(lams):
            ref = olsqr.lsqr(A, AH, y.astype(np.complex128), iset.n_coeffs, lam, omega, 12).fhat
            e = rel(got[r], ref)
            say(f"[cosine lsqr] {prec} lambda={lam} iterate rel {e:.2e}")
            assert e <= tol
    else:
        info = plan.lsqr(yy, lams, None, 400, 1e-8, out)
        got = out.cpu().numpy().reshape(2, -1)
        D = ocos.dense_matrix(iset, x)
        for r, lam in enumerate(lams):
            ref = np.linalg.solve(D.T @ D + 2 * lam * np.eye(iset.n_coeffs), D.T @ y.astype(np.complex128))
            e = rel(got[r], ref)
            say(f"[cosine lsqr] {prec} lambda={lam} converged rel {e:.2e} iters {info[r].iters}")
            assert e <= tol
    L = 1.05 * ofista.power_iteration(A, AH, iset.n_coeffs, 50)
    flams = [20.0, 200.0]
    outf = torch.zeros(2 * iset.n_coeffs, dtype=cdtype(prec), device="cuda")
    plan.fista(yy, flams, None, 30, L, 1.0, 0.0, outf)
    gotf = outf.cpu().numpy().reshape(2, -1)
    for r, lam in enumerate(flams):
        ref = ofista.fista(A, AH, y.astype(np.complex128), iset.offsets, lam, L, 30).fhat
        e = rel(gotf[r], ref)
        nz = sum(np.linalg.norm(ref[iset.term_slice(i)]) > 0 for i in range(iset.n_terms))
        say(f"[cosine fista] {prec} lambda={lam} rel {e:.2e} active groups {nz}")
        assert e <= tol
    plan.close()


def test_cosine_node_gradient_matches_central_differences():
    """d f / d x on the cosine basis: the GPU node gradient against central differences of the
    oracle's forward transform (h = 1e-6, FP64)."""
    import torch
    d, ds, N, M = 3, 2, (8, 6), 40
    iset = ocos.cosine_index_set(d, ds, N)
    x = W.unit_cube_nodes(W.rng(313, W.P_NODES), M, d, "f64")
    fhat = W.complex_normal(W.rng(313, W.P_COEFFS), (iset.n_coeffs,), "f64")
    gup = W.complex_normal(W.rng(313, W.P_GRAD), (M,), "f64")
    p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C128, basis=lib.GT_BASIS_COS)
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    gx = torch.empty((M, d), dtype=torch.float64, device="cuda")
    plan.node_grad(to_dev(fhat), to_dev(gup), gx)
    torch.cuda.synchronize()
    plan.close()
    h = 1e-6
    D = np.zeros((M, d), dtype=complex)
    for j in range(d):
        xp, xm = x.copy(), x.copy()
        xp[:, j] += h
        xm[:, j] -= h
        D[:, j] = (ocos.forward(iset, xp, fhat) - ocos.forward(iset, xm, fhat)) / (2 * h)
    want = (np.conj(D) * gup[:, None]).real
    e = rel(gx.cpu().numpy(), want)
    say(f"[cosine node gradient] rel {e:.2e}")
    assert e <= 1e-7
