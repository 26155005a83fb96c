"""GPU parity of the sensitivity analysis and the active-set refit (Sec. 2 eq. gsi,
Sec. 4.1 eq. activeset) against the oracle:

* gt_sensitivity: the global sensitivity indices of random coefficient vectors (R = 3),
  with and without a term mask, against the oracle's Parseval sums (both sum in FP64 from
  the same coefficients: 1e-12 relative);
* transforms on masked index sets I_N(U) (a random subset; a subset without order-2 terms)
  against the oracle's transform on the same subset (bars of test_gpu_transform.py);
* the pipeline of Sec. 4.1 on the B-spline target (3 one- and 2 two-dimensional terms,
  1 % noise): LSQR fit on U_2, indices on the GPU, the active set taken by gt_active_set
  and by the oracle's rule from the same coefficients (identical), the five true terms in
  it, then the LSQR refit on I_N(U*) with new bandwidths against the oracle's LSQR
  iterates on the same index set (FP64, 1e-9)."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import index_set as oidx
from oracle import lsqr as olsqr
from oracle import sensitivity as osens
from oracle import transform as otr
from paper_2010_10199_amd import lib
from tests.gpu_util import TOL, cdtype, dtype_code, rel, say, to_dev

pytestmark = pytest.mark.gpu


def _rho_gpu(p, fhat_dev, R, nterms):
    import torch
    rho = torch.empty(R * nterms, dtype=torch.float64, device="cuda")
    lib.sensitivity(p, fhat_dev, rho)
    return rho.cpu().numpy().reshape(R, nterms)


@pytest.mark.parametrize("masked", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sensitivity_matches_oracle(prec, masked):
    d, ds, N, R = 6, 3, (12, 8, 4), 3
    nt = lib.gt_num_terms(d, ds)
    mask = (np.random.default_rng(5).random(nt) < 0.5).astype(np.uint8) if masked else None
    iset = oidx.grouped_index_set(d, ds, N, keep=mask)
    p, keep = lib.make_problem(d, ds, N, M=1, R=R, dtype=dtype_code(prec), term_mask=mask)
    assert lib.problem_size(p) == (iset.n_terms, iset.n_coeffs)
    fh = W.complex_normal(W.rng(60, W.P_COEFFS), (R, iset.n_coeffs), prec)
    fh[1] *= 0.0                                         # a zero variance: every index 0
    say(f"[sensitivity] {prec} masked={masked} terms={iset.n_terms} coeffs={iset.n_coeffs}")
    got = _rho_gpu(p, to_dev(fh.reshape(-1)), R, iset.n_terms)
    want = osens.sensitivity_indices(iset, fh.astype(np.complex128))
    e = max(rel(got[r], want[r]) for r in (0, 2))
    say(f"  rel err {e:.3e}; sum {got[0, 1:].sum():.15f}")
    assert e <= 1e-12
    assert np.all(got[1] == 0.0) and np.all(got[:, 0] == 0.0)


@pytest.mark.parametrize("which", ["random", "no-order-2"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_masked_transform_parity(prec, which):
    import torch
    d, ds, N, M = 5, 3, (12, 8, 4), 1500
    full = oidx.anova_terms(d, ds)
    if which == "random":
        mask = (np.random.default_rng(6).random(len(full)) < 0.5).astype(np.uint8)
    else:
        mask = np.array([0 if len(u) == 2 else 1 for u in full], dtype=np.uint8)
    iset = oidx.grouped_index_set(d, ds, N, keep=mask)
    x, fh, y = W.trafo_inputs(61, d, ds, M, iset.n_coeffs, 1, prec)
    y = y.reshape(-1)
    p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=dtype_code(prec), term_mask=mask)
    say(f"[masked transform] {prec} {which} terms={iset.n_terms} coeffs={iset.n_coeffs}")
    f = torch.empty(M, dtype=cdtype(prec), device="cuda")
    a = torch.empty(iset.n_coeffs, dtype=cdtype(prec), device="cuda")
    lib.grouped_trafo(p, to_dev(x), to_dev(fh[0]), f)
    lib.grouped_adjoint(p, to_dev(x), to_dev(y), a)
    torch.cuda.synchronize()
    e1 = rel(f.cpu().numpy(), otr.forward(iset, x, fh[0]))
    e2 = rel(a.cpu().numpy(), otr.adjoint(iset, x, y))
    say(f"  forward {e1:.3e} adjoint {e2:.3e}")
    assert e1 <= TOL[prec] and e2 <= TOL[prec]


def test_active_set_and_refit_fp64():
    import torch
    d, ds, N, M = 7, 2, (16, 8), 5000
    x = W.uniform_nodes(W.rng(62, W.P_NODES), M, d, "f64")
    y = W.add_noise(W.rng(62, W.P_NOISE), W.bspline_target(x).astype(np.complex128), 0.01)
    # fit on all terms of order <= 2
    full = oidx.grouped_index_set(d, ds, N)
    p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C128)
    fh = torch.empty(full.n_coeffs, dtype=torch.complex128, device="cuda")
    info = lib.lsqr_solve(p, to_dev(x), to_dev(y), [1e-3], None, 40, 0.0, fh)
    say(f"[active set] fit on U_2: {full.n_terms} terms, {info[0].iters} LSQR iterations")
    rho = _rho_gpu(p, fh, 1, full.n_terms)[0]
    eps = (0.01, 0.01)
    mask, na = lib.active_set(p, rho, eps)
    want = osens.active_set(full, osens.sensitivity_indices(full, fh.cpu().numpy()), eps)
    terms = [u for u, k in zip(oidx.anova_terms(d, ds), mask) if k]
    say(f"  U* = {terms}")
    assert np.array_equal(mask, want)
    for u in [(), (0,), (1,), (2,), (3, 4), (5, 6)]:
        assert u in terms
    assert na == len(terms)
    # refit on I_N(U*) with new bandwidths
    N2 = (24, 12)
    sub = oidx.grouped_index_set(d, ds, N2, keep=mask)
    p2, keep2 = lib.make_problem(d, ds, N2, M=M, R=1, dtype=lib.GT_C128, term_mask=mask)
    assert lib.problem_size(p2) == (sub.n_terms, sub.n_coeffs)
    f2 = torch.empty(sub.n_coeffs, dtype=torch.complex128, device="cuda")
    K = 20
    lib.lsqr_solve(p2, to_dev(x), to_dev(y), [0.0], None, K, 0.0, f2)
    ref = olsqr.lsqr(lambda v: otr.forward(sub, x, v), lambda r: otr.adjoint(sub, x, r), y, sub.n_coeffs, 0.0,
                     None, K)
    e = rel(f2.cpu().numpy(), ref.fhat)
    r_full = np.linalg.norm(otr.forward(full, x, fh.cpu().numpy()) - y) / np.linalg.norm(y)
    r_sub = np.linalg.norm(otr.forward(sub, x, ref.fhat) - y) / np.linalg.norm(y)
    say(f"  refit: {sub.n_terms} terms, {sub.n_coeffs} coefficients; vs oracle iterates {e:.3e}; "
        f"relative residual {r_full:.4f} (fit on U_2) -> {r_sub:.4f} (refit)")
    assert e <= 1e-9


def test_testfun_error_and_active_set_fp64():
    """The paper's test function (Sec. 4, eq. testfun; d = 9, d_s = 3) at reduced size
    (N = 10/4/4, 2,674 coefficients, M = 4,000, exact samples): 12 LSQR iterations at
    lambda = 1 on the GPU against the oracle's iterates; the L2 error of eq. L2error of both
    (Parseval, exact coefficients) agrees to 1e-9; the indices of the GPU solution give, with
    thresholds 0.005, exactly the printed U* (9 one-, 9 two-, 3 three-dimensional terms)."""
    import torch
    d, ds, N, M, K = 9, 3, (10, 4, 4), 4000, 12
    iset = oidx.grouped_index_set(d, ds, N)
    x = W.uniform_nodes(W.rng(63, W.P_NODES), M, d, "f64")
    y = W.testfun(x).astype(np.complex128)
    exact, n2 = W.testfun_coeffs(iset.terms, iset.freqs), W.testfun_norm2()
    p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C128)
    fh = torch.empty(iset.n_coeffs, dtype=torch.complex128, device="cuda")
    lib.lsqr_solve(p, to_dev(x), to_dev(y), [1.0], None, K, 0.0, fh)
    fg = fh.cpu().numpy()
    ref = olsqr.lsqr(lambda v: otr.forward(iset, x, v), lambda r: otr.adjoint(iset, x, r), y, iset.n_coeffs, 1.0,
                     None, K)
    e_gpu = float(osens.l2_error(iset, fg, exact, n2))
    e_ref = float(osens.l2_error(iset, ref.fhat, exact, n2))
    say(f"[testfun] L2 error GPU {e_gpu:.6f} oracle {e_ref:.6f}; iterates {rel(fg, ref.fhat):.3e}")
    assert abs(e_gpu - e_ref) <= 1e-9 * e_ref
    rho = _rho_gpu(p, fh, 1, iset.n_terms)[0]
    mask, na = lib.active_set(p, rho, (0.005, 0.005, 0.005))
    got = {u for u, k in zip(oidx.anova_terms(d, ds), mask) if k and u}
    want = set()
    for g in ((0, 2, 7), (1, 4, 5), (3, 6, 8)):
        for t in (1, 2, 3):
            want.update(itertools.combinations(g, t))
    say(f"  U*: {len(got)} terms; printed U*: {len(want)}")
    assert got == want and na == 22


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mask_keeping_only_the_empty_set(prec):
    """Degenerate index set: a mask dropping every term leaves the empty set alone, on
    ragged datasets (one of them empty): the forward gives each dataset its constant, the
    adjoint each dataset's sum of samples, the indices are all zero."""
    import torch
    d, ds, N = 4, 2, (8, 6)
    sizes = [300, 0, 512]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    mask = np.zeros(oidx.anova_terms(d, ds).__len__(), dtype=np.uint8)
    iset = oidx.grouped_index_set(d, ds, N, keep=mask)
    assert iset.terms == [()]
    R, Mt = len(sizes), int(offs[-1])
    x = W.uniform_nodes(W.rng(64, W.P_NODES), Mt, d, prec)
    fh = W.complex_normal(W.rng(64, W.P_COEFFS), (R, 1), prec)
    y = W.complex_normal(W.rng(64, W.P_SAMPLES), (Mt,), prec)
    p, keep = lib.make_problem(d, ds, N, M=0, R=R, dtype=dtype_code(prec), offsets=offs, term_mask=mask)
    assert lib.problem_size(p) == (1, 1)
    f = torch.empty(Mt, dtype=cdtype(prec), device="cuda")
    a = torch.empty(R, dtype=cdtype(prec), device="cuda")
    lib.grouped_trafo(p, to_dev(x), to_dev(fh.reshape(-1)), f)
    lib.grouped_adjoint(p, to_dev(x), to_dev(y), a)
    rho = _rho_gpu(p, a, R, 1)
    torch.cuda.synchronize()
    want_f = np.concatenate([np.full(sizes[b], fh[b, 0]) for b in range(R)])
    want_a = np.array([y[offs[b]:offs[b + 1]].astype(np.complex128).sum() for b in range(R)])
    e1, e2 = rel(f.cpu().numpy(), want_f), rel(a.cpu().numpy(), want_a)
    say(f"[empty set only] {prec} forward {e1:.3e} adjoint {e2:.3e}")
    assert e1 <= TOL[prec] and e2 <= TOL[prec] and np.all(rho == 0.0)
