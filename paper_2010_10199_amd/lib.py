"""ctypes binding of libgrouped.so (the C ABI declared in include/grouped.h).

Argument marshalling only: every step of the transforms and solvers runs in the HIP
library.  Torch tensors supply device memory (``data_ptr``) and the stream
(``torch.cuda.current_stream().cuda_stream``).  There is no CPU fallback: loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgrouped.so")

GT_OK, GT_EINVAL, GT_ENOMEM, GT_EHIP, GT_EUNSUPPORTED = 0, -1, -2, -3, -4
GT_C64, GT_C128 = 1, 2
GT_MAX_ORDER = 3
GT_SOLVE_CONVERGED, GT_SOLVE_MAX_ITER, GT_SOLVE_BREAKDOWN, GT_SOLVE_BACKTRACK_CAP = 1, 2, 4, 8
GT_GATHER_SORTED, GT_GATHER_CELL, GT_GATHER_POLY, GT_GATHER_DIRECT = 0, 1, 2, 3
GT_ADJ_WINDOW, GT_ADJ_DIRECT = 0, 1
GT_BASIS_EXP, GT_BASIS_COS = 0, 1

# every symbol include/grouped.h declares
EXPORTS = [
    "gt_num_terms", "gt_num_coeffs", "gt_term_table", "gt_problem_size", "grouped_trafo", "grouped_adjoint",
    "gt_plan_create", "gt_plan_destroy", "gt_plan_trafo", "gt_plan_adjoint", "gt_plan_node_grad",
    "gt_plan_order_info", "gt_plan_gather_path", "lsqr_solve", "fista_group_lasso", "gt_plan_norm_estimate",
    "gt_sensitivity", "gt_active_set", "gt_last_error", "gt_prof_enable", "gt_prof_report", "gt_version",
    "gt_plan_lsqr", "gt_plan_fista", "fista_group_lasso_path", "gt_release_all", "gt_debug_fail_alloc",
    "gt_debug_alloc_count", "gt_plan_norm_estimate_noalloc", "lsqr_solve_path", "gt_plan_lsqr_path",
    "gt_plan_set_gather_path", "gt_plan_tune", "gt_plan_tuning", "gt_plan_set_graph", "gt_plan_adjoint_form",
    "gt_plan_set_adjoint_form", "gt_plan_update_nodes", "gt_plan_set_fused",
]


class GtProblem(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("ds", C.c_int32), ("N", C.c_int32 * GT_MAX_ORDER), ("M", C.c_int64),
        ("R", C.c_int32), ("offsets", C.POINTER(C.c_int64)), ("dtype", C.c_int32), ("m", C.c_int32),
        ("sigma", C.c_double), ("term_mask", C.POINTER(C.c_uint8)), ("basis", C.c_int32),
    ]


class GtSolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("flags", C.c_int32), ("resid", C.c_double), ("t_k", C.c_double),
                ("L", C.c_double)]


class GroupedError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not built: run python -m paper_2010_10199_amd.build")
    # torch carries its own HIP runtime; loading it first makes the library bind to that same
    # runtime (the shared-object name is the same), so device memory and streams are shared.
    # Loaded the other way round, the process holds two runtimes and the library's finds no
    # device once torch has initialised its own.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER(GtProblem)
    sig = {
        "gt_num_terms": (i64, [i32, i32]),
        "gt_num_coeffs": (i64, [i32, i32, C.POINTER(i32)]),
        "gt_term_table": (C.c_int, [P, C.POINTER(i32), C.POINTER(i64)]),
        "gt_problem_size": (C.c_int, [P, C.POINTER(i64), C.POINTER(i64)]),
        "gt_sensitivity": (C.c_int, [P, vp, vp, vp]),
        "gt_active_set": (C.c_int, [P, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(C.c_uint8), C.POINTER(i64)]),
        "grouped_trafo": (C.c_int, [P, vp, vp, vp, vp]),
        "grouped_adjoint": (C.c_int, [P, vp, vp, vp, vp]),
        "gt_plan_create": (C.c_int, [P, vp, vp, C.POINTER(vp)]),
        "gt_plan_destroy": (C.c_int, [vp]),
        "gt_plan_trafo": (C.c_int, [vp, vp, vp, vp]),
        "gt_plan_adjoint": (C.c_int, [vp, vp, vp, vp]),
        "gt_plan_node_grad": (C.c_int, [vp, vp, vp, vp, vp]),
        "gt_plan_order_info": (C.c_int, [vp, i32, C.POINTER(i32), C.POINTER(i32)]),
        "gt_plan_gather_path": (C.c_int, [vp, i32, C.POINTER(i32)]),
        "gt_plan_set_gather_path": (C.c_int, [vp, i32, i32]),
        "gt_plan_adjoint_form": (C.c_int, [vp, i32, C.POINTER(i32)]),
        "gt_plan_set_adjoint_form": (C.c_int, [vp, i32, i32]),
        "gt_plan_update_nodes": (C.c_int, [vp, vp, vp]),
        "gt_plan_tune": (C.c_int, [vp, vp]),
        "gt_plan_tuning": (i64, [vp, C.c_char_p, i64]),
        "gt_plan_set_graph": (C.c_int, [vp, i32]),
        "gt_plan_set_fused": (C.c_int, [vp, i32]),
        "gt_plan_norm_estimate": (C.c_int, [vp, i32, C.POINTER(dbl), vp]),
        "gt_plan_norm_estimate_noalloc": (C.c_int, [vp, i32, C.POINTER(dbl), vp]),
        "lsqr_solve": (C.c_int, [P, vp, vp, C.POINTER(dbl), vp, i32, dbl, vp, C.POINTER(GtSolveInfo), vp]),
        "fista_group_lasso": (C.c_int, [P, vp, vp, C.POINTER(dbl), vp, i32, dbl, dbl, dbl, vp,
                                        C.POINTER(GtSolveInfo), vp]),
        "fista_group_lasso_path": (C.c_int, [P, vp, vp, i32, C.POINTER(dbl), vp, i32, dbl, dbl, dbl, vp, vp,
                                             C.POINTER(GtSolveInfo), vp]),
        "gt_plan_lsqr": (C.c_int, [vp, vp, C.POINTER(dbl), vp, i32, dbl, vp, C.POINTER(GtSolveInfo), vp]),
        "gt_plan_fista": (C.c_int, [vp, vp, C.POINTER(dbl), vp, i32, dbl, dbl, dbl, vp, C.POINTER(GtSolveInfo), vp]),
        "lsqr_solve_path": (C.c_int, [P, vp, vp, i32, C.POINTER(dbl), vp, i32, dbl, vp, C.POINTER(GtSolveInfo), vp]),
        "gt_plan_lsqr_path": (C.c_int, [vp, vp, i32, C.POINTER(dbl), vp, i32, dbl, vp, C.POINTER(GtSolveInfo), vp]),
        "gt_release_all": (C.c_int, []),
        "gt_debug_fail_alloc": (C.c_int, [i64]),
        "gt_debug_alloc_count": (i64, []),
        "gt_last_error": (C.c_char_p, []),
        "gt_prof_enable": (C.c_int, [i32]),
        "gt_prof_report": (i64, [C.c_char_p, i64]),
        "gt_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != GT_OK:
        raise GroupedError(rc, load().gt_last_error().decode())


def make_problem(d: int, ds: int, N: Sequence[int], M: int = 0, R: int = 1, dtype: int = GT_C64,
                 m: int = 0, sigma: float = 0.0, offsets: Optional[Sequence[int]] = None,
                 term_mask: Optional[Sequence[int]] = None, basis: int = GT_BASIS_EXP):
    """Build a GtProblem; returns (problem, keepalive) - keep the second alive while in use.
    term_mask: None, or gt_num_terms(d, ds) flags (0 drops the term; see gt_problem);
    basis: GT_BASIS_EXP or GT_BASIS_COS."""
    p = GtProblem()
    p.basis = int(basis)
    p.d, p.ds = int(d), int(ds)
    for i in range(GT_MAX_ORDER):
        p.N[i] = int(N[i]) if i < len(N) else 0
    p.M, p.R, p.dtype, p.m, p.sigma = int(M), int(R), int(dtype), int(m), float(sigma)
    keep = []
    if offsets is not None:
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        keep.append(offs)
        p.offsets = offs.ctypes.data_as(C.POINTER(C.c_int64))
    else:
        p.offsets = None
    if term_mask is not None:
        mk = np.ascontiguousarray(np.asarray(term_mask, dtype=np.uint8))
        if mk.shape != (gt_num_terms(d, ds),):
            raise ValueError("term_mask needs gt_num_terms(d, ds) entries")
        keep.append(mk)
        p.term_mask = mk.ctypes.data_as(C.POINTER(C.c_uint8))
    else:
        p.term_mask = None
    return p, keep


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream=None):
    if stream is not None:
        return int(stream)
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------- index set
def gt_num_terms(d: int, ds: int) -> int:
    return int(load().gt_num_terms(d, ds))


def gt_num_coeffs(d: int, ds: int, N: Sequence[int]) -> int:
    arr = (C.c_int32 * max(1, len(N)))(*[int(v) for v in N])
    return int(load().gt_num_coeffs(d, ds, arr))


def gt_term_table(d: int, ds: int, N: Sequence[int], term_mask: Optional[Sequence[int]] = None):
    """(coords |U| x 3 int32 with -1 padding, offsets |U|+1 int64); with a term mask, the
    kept terms only."""
    p, _keep = make_problem(d, ds, N, M=1, term_mask=term_mask)
    nt = problem_size(p)[0]
    coords = np.zeros((nt, 3), dtype=np.int32)
    offs = np.zeros(nt + 1, dtype=np.int64)
    _check(load().gt_term_table(C.byref(p), coords.ctypes.data_as(C.POINTER(C.c_int32)),
                                offs.ctypes.data_as(C.POINTER(C.c_int64))))
    return coords, offs


def problem_size(problem):
    """(terms, coefficients) of the problem's index set (term mask applied)."""
    nt, nc = C.c_int64(), C.c_int64()
    _check(load().gt_problem_size(C.byref(problem), C.byref(nt), C.byref(nc)))
    return int(nt.value), int(nc.value)


# ---------------------------------------------------------------- sensitivity analysis
def sensitivity(problem, fhat, rho, stream=None):
    """Global sensitivity indices into rho (device float64, R x |U|); synchronises."""
    _check(load().gt_sensitivity(C.byref(problem), _ptr(fhat), _ptr(rho), _stream(stream)))


def active_set(problem, rho, eps):
    """Active-set mask (gt_num_terms(d, ds) uint8) from one right-hand side's indices
    (host array of the problem's |U| values) and ds thresholds; returns (mask, count)."""
    r = np.ascontiguousarray(np.asarray(rho, dtype=np.float64))
    e = np.ascontiguousarray(np.asarray(eps, dtype=np.float64).reshape(-1))
    mask = np.zeros(gt_num_terms(problem.d, problem.ds), dtype=np.uint8)
    na = C.c_int64()
    _check(load().gt_active_set(C.byref(problem), r.ctypes.data_as(C.POINTER(C.c_double)),
                                e.ctypes.data_as(C.POINTER(C.c_double)),
                                mask.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(na)))
    return mask, int(na.value)


# ---------------------------------------------------------------- one-shot transforms
def grouped_trafo(problem, x, fhat, f, stream=None):
    _check(load().grouped_trafo(C.byref(problem), _ptr(x), _ptr(fhat), _ptr(f), _stream(stream)))


def grouped_adjoint(problem, x, y, fhat, stream=None):
    _check(load().grouped_adjoint(C.byref(problem), _ptr(x), _ptr(y), _ptr(fhat), _stream(stream)))


def _omega(omega):
    """Device pointer of the FP64 weights (None: omega = 1)."""
    if omega is None:
        return None
    import torch
    if omega.dtype != torch.float64:
        raise TypeError("omega must be a float64 device tensor (the weights are FP64 on both paths)")
    return _ptr(omega)


def _lam(lambdas):
    return np.ascontiguousarray(np.asarray(lambdas, dtype=np.float64))


def lsqr_solve(problem, x, y, lambdas, omega, max_iter, tol, fhat, stream=None):
    lam = _lam(lambdas)
    info = (GtSolveInfo * problem.R)()
    _check(load().lsqr_solve(C.byref(problem), _ptr(x), _ptr(y), lam.ctypes.data_as(C.POINTER(C.c_double)),
                             _omega(omega), int(max_iter), float(tol), _ptr(fhat), info, _stream(stream)))
    return list(info)


def fista_group_lasso(problem, x, y, lambdas, omega, max_iter, L, eta, tol, fhat, stream=None):
    lam = _lam(lambdas)
    info = (GtSolveInfo * problem.R)()
    _check(load().fista_group_lasso(C.byref(problem), _ptr(x), _ptr(y), lam.ctypes.data_as(C.POINTER(C.c_double)),
                                    _omega(omega), int(max_iter), float(L), float(eta), float(tol), _ptr(fhat),
                                    info, _stream(stream)))
    return list(info)


def lsqr_solve_path(problem, x, y, lambdas, omega, max_iter, tol, fhat_path, stream=None):
    """All lambda values on each right-hand side with one shared bidiagonalisation; returns
    info as a list of len(lambdas) lists of R entries."""
    lam = _lam(lambdas)
    K, R = len(lam), problem.R
    info = (GtSolveInfo * (K * R))()
    _check(load().lsqr_solve_path(C.byref(problem), _ptr(x), _ptr(y), int(K),
                                  lam.ctypes.data_as(C.POINTER(C.c_double)), _omega(omega), int(max_iter), float(tol),
                                  _ptr(fhat_path), info, _stream(stream)))
    return [list(info[j * R:(j + 1) * R]) for j in range(K)]


def fista_group_lasso_path(problem, x, y, lambdas, omega, max_iter, L, eta, tol, fhat0, fhat_path, stream=None):
    """Warm-started path: returns info as a list of len(lambdas) lists of R entries."""
    lam = _lam(lambdas)
    K, R = len(lam), problem.R
    info = (GtSolveInfo * (K * R))()
    _check(load().fista_group_lasso_path(C.byref(problem), _ptr(x), _ptr(y), int(K),
                                         lam.ctypes.data_as(C.POINTER(C.c_double)), _omega(omega), int(max_iter),
                                         float(L), float(eta), float(tol), _ptr(fhat0), _ptr(fhat_path), info,
                                         _stream(stream)))
    return [list(info[j * R:(j + 1) * R]) for j in range(K)]


def release_all():
    _check(load().gt_release_all())


def debug_fail_alloc(k: int):
    """Arm the allocation-failure hook: the k-th device allocation from now fails (0: off)."""
    _check(load().gt_debug_fail_alloc(int(k)))


def debug_alloc_count() -> int:
    return int(load().gt_debug_alloc_count())


# ---------------------------------------------------------------- plans
class Plan:
    """Owns a gt_plan for (problem, nodes); the nodes are copied into the plan."""

    def __init__(self, problem, x, stream=None, keepalive=None):
        self._lib = load()
        self.problem = problem
        self._keep = keepalive
        h = C.c_void_p()
        _check(self._lib.gt_plan_create(C.byref(problem), _ptr(x), _stream(stream), C.byref(h)))
        self.handle = h

    def trafo(self, fhat, f, stream=None):
        _check(self._lib.gt_plan_trafo(self.handle, _ptr(fhat), _ptr(f), _stream(stream)))

    def adjoint(self, y, fhat, stream=None):
        _check(self._lib.gt_plan_adjoint(self.handle, _ptr(y), _ptr(fhat), _stream(stream)))

    def node_grad(self, fhat, g, gx, stream=None):
        _check(self._lib.gt_plan_node_grad(self.handle, _ptr(fhat), _ptr(g), _ptr(gx), _stream(stream)))

    def order_info(self, t: int):
        m, n = C.c_int32(), C.c_int32()
        _check(self._lib.gt_plan_order_info(self.handle, int(t), C.byref(m), C.byref(n)))
        return int(m.value), int(n.value)

    def lsqr(self, y, lambdas, omega, max_iter, tol, fhat, stream=None):
        lam = _lam(lambdas)
        info = (GtSolveInfo * self.problem.R)()
        _check(self._lib.gt_plan_lsqr(self.handle, _ptr(y), lam.ctypes.data_as(C.POINTER(C.c_double)),
                                      _omega(omega), int(max_iter), float(tol), _ptr(fhat), info, _stream(stream)))
        return list(info)

    def lsqr_path(self, y, lambdas, omega, max_iter, tol, fhat_path, stream=None):
        lam = _lam(lambdas)
        K, R = len(lam), self.problem.R
        info = (GtSolveInfo * (K * R))()
        _check(self._lib.gt_plan_lsqr_path(self.handle, _ptr(y), int(K), lam.ctypes.data_as(C.POINTER(C.c_double)),
                                           _omega(omega), int(max_iter), float(tol), _ptr(fhat_path), info,
                                           _stream(stream)))
        return [list(info[j * R:(j + 1) * R]) for j in range(K)]

    def fista(self, y, lambdas, omega, max_iter, L, eta, tol, fhat, stream=None):
        lam = _lam(lambdas)
        info = (GtSolveInfo * self.problem.R)()
        _check(self._lib.gt_plan_fista(self.handle, _ptr(y), lam.ctypes.data_as(C.POINTER(C.c_double)),
                                       _omega(omega), int(max_iter), float(L), float(eta), float(tol), _ptr(fhat),
                                       info, _stream(stream)))
        return list(info)

    def norm_estimate(self, iters=50, stream=None) -> float:
        out = C.c_double()
        _check(self._lib.gt_plan_norm_estimate(self.handle, int(iters), C.byref(out), _stream(stream)))
        return float(out.value)

    def norm_estimate_noalloc(self, iters=50, stream=None) -> float:
        """gt_plan_norm_estimate with its work buffers in the library's fixed device array."""
        out = C.c_double()
        _check(self._lib.gt_plan_norm_estimate_noalloc(self.handle, int(iters), C.byref(out), _stream(stream)))
        return float(out.value)

    def gather_path(self, t: int) -> int:
        """GT_GATHER_SORTED / GT_GATHER_CELL / GT_GATHER_POLY for order t."""
        path = C.c_int32()
        _check(self._lib.gt_plan_gather_path(self.handle, int(t), C.byref(path)))
        return int(path.value)

    def update_nodes(self, x, stream=None):
        """gt_plan_update_nodes: new positions for the plan's nodes (same count and layout)."""
        _check(self._lib.gt_plan_update_nodes(self.handle, _ptr(x), _stream(stream)))

    def set_gather_path(self, t: int, path: int):
        _check(self._lib.gt_plan_set_gather_path(self.handle, int(t), int(path)))

    def adjoint_form(self, t: int) -> int:
        """GT_ADJ_WINDOW / GT_ADJ_DIRECT for order t."""
        form = C.c_int32()
        _check(self._lib.gt_plan_adjoint_form(self.handle, int(t), C.byref(form)))
        return int(form.value)

    def set_adjoint_form(self, t: int, form: int):
        _check(self._lib.gt_plan_set_adjoint_form(self.handle, int(t), int(form)))

    def tune(self, stream=None) -> dict:
        """gt_plan_tune on `stream` (a created stream); returns the tuning report."""
        _check(self._lib.gt_plan_tune(self.handle, _stream(stream)))
        return self.tuning()

    def tuning(self) -> dict:
        import json
        n = self._lib.gt_plan_tuning(self.handle, None, 0)
        if n < 0:
            _check(int(n))
        buf = C.create_string_buffer(int(n))
        self._lib.gt_plan_tuning(self.handle, buf, len(buf))
        return json.loads(buf.value.decode() or "{}")

    def set_graph(self, on: bool = True):
        _check(self._lib.gt_plan_set_graph(self.handle, 1 if on else 0))

    def set_fused(self, on: bool = True):
        """Orders 1 and 2 in shared launches (three per direction) or in separate ones."""
        _check(self._lib.gt_plan_set_fused(self.handle, 1 if on else 0))

    def close(self):
        if getattr(self, "handle", None):
            self._lib.gt_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prof_enable(on: bool = True):
    _check(load().gt_prof_enable(1 if on else 0))


def prof_report() -> dict:
    import json
    lib = load()
    # gt_prof_report clears the records, so it is called once with a large buffer
    buf = C.create_string_buffer(1 << 16)
    lib.gt_prof_report(buf, len(buf))
    return json.loads(buf.value.decode() or "{}")
