"""GPU LSQR / FISTA / power iteration against the oracle's iterations (same algorithm,
same iteration counts, same step constants), plus converged solutions against dense
solves.  FP64 path: iterates agree to 1e-9 relative; FP32 bulk path (FP64 scalars):
converged solutions agree with the FP64 solution to 1e-5."""
import numpy as np
import pytest

import workloads as W
from oracle import fista as ofista
from oracle import index_set as oidx
from oracle import lsqr as olsqr
from oracle import transform as otr
from paper_2010_10199_amd import lib
from tests.gpu_util import cdtype, dtype_code, rel, say, to_dev

pytestmark = pytest.mark.gpu


def _lsqr_gpu(d, ds, N, x, y, lambdas, prec, iters, omega=None, tol=0.0):
    import torch
    R = len(lambdas)
    iset = oidx.grouped_index_set(d, ds, N)
    p, keep = lib.make_problem(d, ds, N, M=x.shape[0], R=R, dtype=dtype_code(prec))
    out = torch.empty(R * iset.n_coeffs, dtype=cdtype(prec), device="cuda")
    om = None if omega is None else to_dev(omega.astype(np.float64))
    info = lib.lsqr_solve(p, to_dev(x), to_dev(y), lambdas, om, iters, tol, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(complex).reshape(R, -1), info


def _fista_gpu(d, ds, N, x, y, lambdas, prec, iters, L, eta=0.0, omega=None, f0=None, tol=0.0):
    import torch
    R = len(lambdas)
    iset = oidx.grouped_index_set(d, ds, N)
    p, keep = lib.make_problem(d, ds, N, M=x.shape[0], R=R, dtype=dtype_code(prec))
    if f0 is None:
        out = torch.zeros(R * iset.n_coeffs, dtype=cdtype(prec), device="cuda")
    else:
        out = to_dev(f0.astype(np.complex64 if prec == "f32" else np.complex128).reshape(-1))
    om = None if omega is None else to_dev(omega.astype(np.float64))
    info = lib.fista_group_lasso(p, to_dev(x), to_dev(y), lambdas, om, iters, L, eta, tol, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(complex).reshape(R, -1), info


def _sobolev(iset, s):
    K = iset.full_frequencies()
    return np.prod((1.0 + np.abs(K)) ** s, axis=1)


def test_lsqr_config1_fp64():
    """d=6, d_s=2, N=(16,8), M=2000, exact data y = F fhat_true, lambda=0, 30 iterations."""
    d, ds, N, M = 6, 2, (16, 8), 2000
    iset = oidx.grouped_index_set(d, ds, N)
    x, ftrue, _ = W.trafo_inputs(1, d, ds, M, iset.n_coeffs, 1, "f64")
    y = otr.forward(iset, x, ftrue[0])
    say("[lsqr config1] fp64 30 iterations")
    fg, info = _lsqr_gpu(d, ds, N, x, y.reshape(1, M), [0.0], "f64", 30)
    ref = olsqr.lsqr(lambda v: otr.forward(iset, x, v), lambda r: otr.adjoint(iset, x, r), y, iset.n_coeffs, 0.0,
                     None, 30)
    e_iter = rel(fg[0], ref.fhat)
    e_true = rel(fg[0], ftrue[0])
    say(f"  vs oracle 30-iterate {e_iter:.3e}; vs fhat_true {e_true:.3e}; iters {info[0].iters}")
    assert info[0].iters == 30
    assert e_iter <= 1e-9
    assert e_true <= 1e-3


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lsqr_batched_lambdas_converged(prec):
    """Several lambda in one launch (weighted and unweighted) against dense normal equations."""
    d, ds, N, M = 5, 3, (10, 6, 4), 4000
    iset = oidx.grouped_index_set(d, ds, N)
    x, _, yy = W.trafo_inputs(31, d, ds, M, iset.n_coeffs, 1, prec)
    y = yy[0]
    lambdas = [1e-3, 0.1, 10.0, 300.0]
    R = len(lambdas)
    A = otr.dense_matrix(iset, x)
    for weighted in (False, True):
        omega = _sobolev(iset, 1.0) if weighted else None
        say(f"[lsqr batched] {prec} weighted={weighted}")
        stop = 1e-13 if prec == "f64" else 1e-8    # normal-equation residual, relative to its start
        fg, info = _lsqr_gpu(d, ds, N, x, np.tile(y, R).reshape(R, M), lambdas, prec, 300, omega=omega, tol=stop)
        Wd = np.diag(omega if weighted else np.ones(iset.n_coeffs))
        for r, lam in enumerate(lambdas):
            ref = np.linalg.solve(A.conj().T @ A + 2 * lam * Wd, A.conj().T @ y.astype(complex))
            e = rel(fg[r], ref)
            say(f"  lambda={lam} rel {e:.3e} iters {info[r].iters} flags {info[r].flags}")
            assert e <= (1e-5 if prec == "f32" else 1e-10)


def test_lsqr_iterates_match_oracle_fp64():
    d, ds, N, M = 4, 2, (12, 8), 3000
    iset = oidx.grouped_index_set(d, ds, N)
    x, _, yy = W.trafo_inputs(32, d, ds, M, iset.n_coeffs, 1, "f64")
    omega = _sobolev(iset, 0.5)
    lambdas = [0.5, 20.0]
    fg, _ = _lsqr_gpu(d, ds, N, x, np.tile(yy[0], 2).reshape(2, M), lambdas, "f64", 12, omega=omega)
    for r, lam in enumerate(lambdas):
        ref = olsqr.lsqr(lambda v: otr.forward(iset, x, v), lambda q: otr.adjoint(iset, x, q), yy[0], iset.n_coeffs,
                         lam, omega, 12)
        e = rel(fg[r], ref.fhat)
        say(f"[lsqr iterate] lambda={lam} rel {e:.3e}")
        assert e <= 1e-10


def test_power_iteration_matches_oracle():
    import torch
    d, ds, N, M = 4, 2, (12, 8), 3000
    iset = oidx.grouped_index_set(d, ds, N)
    x, _, _ = W.trafo_inputs(33, d, ds, M, iset.n_coeffs, 1, "f64")
    p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C128)
    plan = lib.Plan(p, to_dev(x))
    est = plan.norm_estimate(50)
    ref = ofista.power_iteration(lambda v: otr.forward(iset, x, v), lambda r: otr.adjoint(iset, x, r),
                                 iset.n_coeffs, 50)
    say(f"[power] gpu {est:.10e} oracle {ref:.10e}")
    assert abs(est - ref) / ref <= 1e-10
    plan.close()


def _fista_case(prec, seed=34):
    d, ds, N, M = 4, 2, (10, 6), 3000
    iset = oidx.grouped_index_set(d, ds, N)
    x, ftrue, yy = W.trafo_inputs(seed, d, ds, M, iset.n_coeffs, 1, prec)
    # a target with only a few active groups plus noise
    f = np.zeros(iset.n_coeffs, dtype=complex)
    for ti in (1, 3, 6):
        f[iset.term_slice(ti)] = ftrue[0][iset.term_slice(ti)]
    y = otr.forward(iset, x, f) + 0.05 * yy[0]
    y = y.astype(np.complex64 if prec == "f32" else np.complex128)
    return d, ds, N, M, iset, x, y


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fista_constant_step_matches_oracle(prec):
    d, ds, N, M, iset, x, y = _fista_case(prec)
    lambdas = [30.0, 300.0, 3000.0]
    L = 1.05 * ofista.power_iteration(lambda v: otr.forward(iset, x, v), lambda r: otr.adjoint(iset, x, r),
                                      iset.n_coeffs, 50)
    K = 60
    fg, info = _fista_gpu(d, ds, N, x, np.tile(y, 3).reshape(3, M), lambdas, prec, K, L)
    for r, lam in enumerate(lambdas):
        ref = ofista.fista(lambda v: otr.forward(iset, x, v), lambda q: otr.adjoint(iset, x, q), y, iset.offsets,
                           lam, L, K)
        e = rel(fg[r], ref.fhat)
        nz = sum(np.linalg.norm(ref.fhat[iset.term_slice(i)]) > 0 for i in range(iset.n_terms))
        say(f"[fista] {prec} lambda={lam} rel {e:.3e} active groups {nz}")
        assert e <= (1e-5 if prec == "f32" else 1e-10)


def test_fista_weighted_prox_fp64():
    """Sobolev weights (s = 1.5): the prox needs the bisection + Newton root for xi."""
    d, ds, N, M, iset, x, y = _fista_case("f64", seed=35)
    omega = _sobolev(iset, 1.5)
    L = 1.05 * ofista.power_iteration(lambda v: otr.forward(iset, x, v), lambda r: otr.adjoint(iset, x, r),
                                      iset.n_coeffs, 50)
    lambdas = [10.0, 200.0]
    fg, _ = _fista_gpu(d, ds, N, x, np.tile(y, 2).reshape(2, M), lambdas, "f64", 40, L, omega=omega)
    for r, lam in enumerate(lambdas):
        ref = ofista.fista(lambda v: otr.forward(iset, x, v), lambda q: otr.adjoint(iset, x, q), y, iset.offsets,
                           lam, L, 40, omega=omega)
        e = rel(fg[r], ref.fhat)
        say(f"[fista weighted] lambda={lam} rel {e:.3e}")
        assert e <= 1e-10


def test_fista_backtracking_fp64():
    """Algorithm with backtracking from a small L0 (eta = 2): same L sequence and iterates."""
    d, ds, N, M, iset, x, y = _fista_case("f64", seed=36)
    L0 = 50.0
    fg, info = _fista_gpu(d, ds, N, x, y.reshape(1, M), [100.0], "f64", 30, L0, eta=2.0)
    ref = ofista.fista(lambda v: otr.forward(iset, x, v), lambda q: otr.adjoint(iset, x, q), y, iset.offsets,
                       100.0, L0, 30, eta=2.0)
    e = rel(fg[0], ref.fhat)
    say(f"[fista backtracking] rel {e:.3e} L gpu {info[0].L} oracle {ref.L} backtracks {ref.backtracks}")
    assert ref.backtracks > 0
    assert abs(info[0].L - ref.L) <= 1e-12 * ref.L
    assert e <= 1e-10


def test_fista_zero_above_lambda_max():
    d, ds, N, M, iset, x, y = _fista_case("f64", seed=37)
    g = otr.adjoint(iset, x, y)
    lmax = max(np.linalg.norm(g[iset.term_slice(i)]) for i in range(iset.n_terms))
    L = 1.05 * ofista.power_iteration(lambda v: otr.forward(iset, x, v), lambda r: otr.adjoint(iset, x, r),
                                      iset.n_coeffs, 50)
    fg, _ = _fista_gpu(d, ds, N, x, y.reshape(1, M), [lmax * 1.001], "f64", 20, L)
    say(f"[fista zero] max |f| = {np.abs(fg).max():.3e}")
    assert np.abs(fg).max() == 0.0


def test_solver_argument_errors():
    import torch
    d, ds, N, M = 3, 2, (6, 4), 100
    x = torch.zeros(M, d, dtype=torch.float64, device="cuda")
    y = torch.zeros(M, dtype=torch.complex128, device="cuda")
    n = lib.gt_num_coeffs(d, ds, N)
    out = torch.zeros(n, dtype=torch.complex128, device="cuda")
    p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C128)
    with pytest.raises(lib.GroupedError) as e:
        lib.lsqr_solve(p, x, y, [-1.0], None, 5, 0.0, out)
    assert e.value.code == lib.GT_EINVAL
    with pytest.raises(lib.GroupedError) as e:
        lib.fista_group_lasso(p, x, y, [0.0], None, 5, 1.0, 0.0, 0.0, out)
    assert e.value.code == lib.GT_EINVAL
    bad = torch.ones(n, dtype=torch.float64, device="cuda")
    bad[3] = -1.0
    with pytest.raises(lib.GroupedError) as e:
        lib.lsqr_solve(p, x, y, [1.0], bad, 5, 0.0, out)
    assert e.value.code == lib.GT_EINVAL


def test_fp32_solvers_on_cell_and_polynomial_gathers():
    """Batched FP32 LSQR and FISTA on a node set whose cells are filled enough for the cell
    gather (order 1) and the polynomial gather (order 2): LSQR against the dense normal
    equations, FISTA against the oracle's iterates with the same step constant."""
    d, ds, N, M = 3, 2, (8, 6), 20000
    iset = oidx.grouped_index_set(d, ds, N)
    x, ftrue, yy = W.trafo_inputs(35, d, ds, M, iset.n_coeffs, 1, "f32")
    p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C64)
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    paths = (plan.gather_path(1), plan.gather_path(2))
    plan.close()
    say(f"[solvers on cells] gather paths {paths}")
    assert paths == (lib.GT_GATHER_CELL, lib.GT_GATHER_POLY)
    y = yy[0]
    A = otr.dense_matrix(iset, x)
    lambdas = [1e-2, 10.0, 1000.0]
    R = len(lambdas)
    fg, info = _lsqr_gpu(d, ds, N, x, np.tile(y, R).reshape(R, M), lambdas, "f32", 200, tol=1e-8)
    for r, lam in enumerate(lambdas):
        ref = np.linalg.solve(A.conj().T @ A + 2 * lam * np.eye(iset.n_coeffs), A.conj().T @ y.astype(complex))
        e = rel(fg[r], ref)
        say(f"  lsqr lambda={lam} rel {e:.3e} iters {info[r].iters}")
        assert e <= 1e-5
    f = np.zeros(iset.n_coeffs, dtype=complex)
    for ti in (1, 5):
        f[iset.term_slice(ti)] = ftrue[0][iset.term_slice(ti)]
    yf = (otr.forward(iset, x, f) + 0.05 * y).astype(np.complex64)
    L = 1.05 * ofista.power_iteration(lambda v: otr.forward(iset, x, v), lambda q: otr.adjoint(iset, x, q),
                                      iset.n_coeffs, 30)
    K = 30
    flam = [100.0, 2000.0]
    fgf, _ = _fista_gpu(d, ds, N, x, np.tile(yf, 2).reshape(2, M), flam, "f32", K, L)
    for r, lam in enumerate(flam):
        ref = ofista.fista(lambda v: otr.forward(iset, x, v), lambda q: otr.adjoint(iset, x, q),
                           yf.astype(np.complex128), iset.offsets, lam, L, K)
        e = rel(fgf[r], ref.fhat)
        say(f"  fista lambda={lam} rel {e:.3e}")
        assert e <= 1e-5


def test_fista_path_with_backtracking_matches_oracle_fp64():
    """The warm-started path in one call (one plan), Algorithm algo:fista with backtracking
    from a small L_0 (eta = 2) and Sobolev weights (s = 1.5, the prox's bisection + Newton
    root for xi): every stage against the oracle's path, each stage from the previous
    solution with t_1 = 1 and L_0 restarted."""
    import torch
    d, ds, N, M, iset, x, y = _fista_case("f64", seed=38)
    omega = _sobolev(iset, 1.5)
    lams = [400.0, 120.0, 40.0]
    L0, K = 50.0, 25
    p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C128)
    path = torch.zeros(len(lams) * iset.n_coeffs, dtype=torch.complex128, device="cuda")
    infos = lib.fista_group_lasso_path(p, to_dev(x), to_dev(y), lams, to_dev(omega), K, L0, 2.0, 0.0, None, path)
    got = path.cpu().numpy().reshape(len(lams), -1)
    prev = None
    for j, lam in enumerate(lams):
        ref = ofista.fista(lambda v: otr.forward(iset, x, v), lambda q: otr.adjoint(iset, x, q), y, iset.offsets,
                           lam, L0, K, f0=prev, omega=omega, eta=2.0)
        e = rel(got[j], ref.fhat)
        say(f"[fista path] stage {j} lambda={lam} rel {e:.3e} L gpu {infos[j][0].L} oracle {ref.L} "
            f"backtracks {ref.backtracks} iters {infos[j][0].iters}")
        assert ref.backtracks > 0
        assert abs(infos[j][0].L - ref.L) <= 1e-12 * ref.L
        assert infos[j][0].iters == K and not infos[j][0].flags & lib.GT_SOLVE_BACKTRACK_CAP
        assert e <= 1e-10
        prev = ref.fhat


def test_fista_backtrack_cap_flags_only_the_capped_side():
    """Two right-hand sides in one call: lambda above lambda_max keeps f = 0, so its test
    ||F(f - h)||^2 <= L ||f - h||^2 holds at once (0 <= 0); the other starts from a tiny L_0
    with eta = 1.01, so 30 increases per iteration cannot reach a passing L.  Only the
    second reports the cap."""
    d, ds, N, M, iset, x, y = _fista_case("f64", seed=39)
    g = otr.adjoint(iset, x, y)
    lmax = max(np.linalg.norm(g[iset.term_slice(i)]) for i in range(iset.n_terms))
    fg, info = _fista_gpu(d, ds, N, x, np.tile(y, 2).reshape(2, M), [2.0 * lmax, 0.01 * lmax], "f64", 3, 1e-6,
                          eta=1.01)
    say(f"[fista cap] flags {info[0].flags} {info[1].flags} L {info[0].L} {info[1].L}")
    assert not info[0].flags & lib.GT_SOLVE_BACKTRACK_CAP
    assert info[0].L == 1e-6 and np.abs(fg[0]).max() == 0.0
    assert info[1].flags & lib.GT_SOLVE_BACKTRACK_CAP
    # 30 increases in each of the 3 iterations; L persists across iterations (the algorithm
    # carries L_k into the next iteration)
    assert abs(info[1].L - 1e-6 * 1.01 ** 90) <= 1e-12 * info[1].L
    assert info[0].iters == info[1].iters == 3


def test_lsqr_breakdown_is_flagged_not_an_error():
    """Only the empty-set term (d_s = 0), M = 4, values exact in binary: samples in the range
    of F (all ones: beta_1 = 2, u_1 = 1/2, alpha_1 = 2, v_1 = 1) make u_2 = F v_1 - alpha_1 u_1
    exactly zero (beta_2 = 0) after one step, and the solution is their mean 1; samples
    orthogonal to the range (alternating signs) make alpha_1 = 0 at once, and the solution
    stays zero.  Both report GT_SOLVE_BREAKDOWN."""
    import torch
    x = np.zeros((4, 2))
    for y, want in ((np.ones(4, complex), 1.0), (np.array([1.0, -1.0, 1.0, -1.0], complex), 0.0)):
        p, keep = lib.make_problem(2, 0, [], M=4, R=1, dtype=lib.GT_C128)
        out = torch.empty(1, dtype=torch.complex128, device="cuda")
        info = lib.lsqr_solve(p, to_dev(x), to_dev(y), [0.0], None, 10, 0.0, out)
        got = out.cpu().numpy()[0]
        say(f"[lsqr breakdown] fhat {got} iters {info[0].iters} flags {info[0].flags}")
        assert info[0].flags & lib.GT_SOLVE_BREAKDOWN
        assert abs(got - want) <= 1e-15 * max(1.0, abs(want))
        assert info[0].iters <= 1


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_plan_solvers_match_one_shot_calls(prec):
    """gt_plan_lsqr / gt_plan_fista on one plan give the one-shot calls' results, twice in a
    row on the same plan (the plan's buffers carry no state between calls)."""
    import torch
    d, ds, N, M, iset, x, y = _fista_case(prec, seed=40)
    lams = [0.5, 50.0]
    R = len(lams)
    yy = np.tile(y, R).reshape(R, M)
    ref_l, _ = _lsqr_gpu(d, ds, N, x, yy, lams, prec, 15)
    ref_f, _ = _fista_gpu(d, ds, N, x, yy, [300.0, 3000.0], prec, 20, 0.0)
    p, keep = lib.make_problem(d, ds, N, M=M, R=R, dtype=dtype_code(prec))
    plan = lib.Plan(p, to_dev(x), keepalive=keep)
    tol = 1e-12 if prec == "f64" else 1e-5
    for call in range(2):
        out = torch.empty(R * iset.n_coeffs, dtype=cdtype(prec), device="cuda")
        plan.lsqr(to_dev(yy), lams, None, 15, 0.0, out)
        e1 = rel(out.cpu().numpy().reshape(R, -1), ref_l)
        outf = torch.zeros(R * iset.n_coeffs, dtype=cdtype(prec), device="cuda")
        plan.fista(to_dev(yy), [300.0, 3000.0], None, 20, 0.0, 1.0, 0.0, outf)
        e2 = rel(outf.cpu().numpy().reshape(R, -1), ref_f)
        say(f"[plan solvers] {prec} call {call}: lsqr {e1:.2e} fista {e2:.2e}")
        assert e1 <= tol and e2 <= tol
    plan.close()


def test_released_and_destroyed_plans_are_rejected():
    import torch
    d, ds, N, M = 3, 2, (6, 4), 200
    x = W.uniform_nodes(W.rng(41, W.P_NODES), M, d, "f64")
    p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C128)
    n = lib.gt_num_coeffs(d, ds, N)
    fh = torch.zeros(n, dtype=torch.complex128, device="cuda")
    f = torch.zeros(M, dtype=torch.complex128, device="cuda")
    a = lib.Plan(p, to_dev(x), keepalive=keep)
    b = lib.Plan(p, to_dev(x), keepalive=keep)
    a.trafo(fh, f)
    lib.release_all()
    for pl in (a, b):
        with pytest.raises(lib.GroupedError) as e:
            pl.trafo(fh, f)
        assert e.value.code == lib.GT_EINVAL
        assert lib.load().gt_plan_destroy(pl.handle) == lib.GT_EINVAL
        pl.handle = None
    c = lib.Plan(p, to_dev(x), keepalive=keep)     # the library still works afterwards
    c.trafo(fh, f)
    c.close()
    torch.cuda.synchronize()


def test_allocation_failures_are_reported_and_leave_the_library_usable():
    """Every device allocation of a plan creation and of an LSQR call, failed in turn through
    the allocation-failure hook, gives GT_ENOMEM; afterwards the same calls succeed and
    match the result obtained before."""
    import torch
    d, ds, N, M = 3, 2, (6, 4), 500
    iset = oidx.grouped_index_set(d, ds, N)
    x, _, yy = W.trafo_inputs(42, d, ds, M, iset.n_coeffs, 1, "f64")
    xd, yd = to_dev(x), to_dev(yy[0])
    p, keep = lib.make_problem(d, ds, N, M=M, R=1, dtype=lib.GT_C128)
    out = torch.empty(iset.n_coeffs, dtype=torch.complex128, device="cuda")
    lib.debug_fail_alloc(0)
    lib.lsqr_solve(p, xd, yd, [0.1], None, 5, 0.0, out)
    ref = out.cpu().numpy()
    nalloc = lib.debug_alloc_count()
    say(f"[alloc hook] an LSQR call makes {nalloc} device allocations")
    assert nalloc >= 10
    try:
        for k in range(1, nalloc + 1):
            lib.debug_fail_alloc(k)
            with pytest.raises(lib.GroupedError) as e:
                lib.lsqr_solve(p, xd, yd, [0.1], None, 5, 0.0, out)
            assert e.value.code == lib.GT_ENOMEM, (k, e.value)
    finally:
        lib.debug_fail_alloc(0)
    torch.cuda.synchronize()
    lib.lsqr_solve(p, xd, yd, [0.1], None, 5, 0.0, out)
    assert rel(out.cpu().numpy(), ref) <= 1e-13
