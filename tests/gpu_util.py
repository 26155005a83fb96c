"""Helpers for GPU tests: move seeded numpy inputs to the device, run the C-ABI entry points,
and measure relative errors against the oracle."""
from __future__ import annotations

import math
import sys

import numpy as np

from paper_2010_10199_amd import lib

TOL = {"f32": 1e-5, "f64": 1e-12}   # relative l2 error of the transforms vs the FP64 oracle
# Per-element bar in the form of the fast transform's error bound (Sec. 3, the bound after
# eq. somafm): max_x |f(x) - f~(x)| <= E ||fhat||_1 (adjoint: max_k |..| <= E ||y||_1), with
# E the window's error per axis times the term order, here 4 d_s times the Kaiser-Bessel
# error model, plus an allowance for rounding and the window tables: about 17 units of
# roundoff in FP32 (2e-6) and 450 in FP64 (5e-14; there the degree-14 window polynomial and
# the deconvolution table dominate), where the deconvolution factors 1 / Phi_hat reach about
# 10 at the band edge.  Measured worst cases: 3.8e-7 (FP32) and 7.2e-15 (FP64).
ROUND = {"f32": 2e-6, "f64": 5e-14}
DEFAULT_M = {"f32": 4, "f64": 8}    # the library's window at sigma = 2 when the problem leaves m = 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def nfft_model_error(m: int, sigma: float) -> float:
    """Kaiser-Bessel error model of the library's window choice (per axis)."""
    return 2.3 * math.exp(-2 * math.pi * m * math.sqrt(1 - 1 / sigma))


def rel(a, b) -> float:
    a = np.asarray(a).astype(np.complex128)
    b = np.asarray(b).astype(np.complex128)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def dtype_code(prec):
    return lib.GT_C64 if prec == "f32" else lib.GT_C128


def cdtype(prec):
    import torch
    return torch.complex64 if prec == "f32" else torch.complex128


def gpu_trafo(d, ds, N, x, fhat, prec, M=None, R=1, offsets=None, m=0, sigma=0.0):
    """f = F fhat through grouped_trafo; returns numpy complex128 (R x M or ragged)."""
    import torch
    Mx = x.shape[0]
    p, keep = lib.make_problem(d, ds, N, M=Mx if offsets is None else 0, R=R, dtype=dtype_code(prec), m=m,
                               sigma=sigma, offsets=offsets)
    xd = to_dev(x)
    fd = to_dev(fhat)
    nout = R * Mx if offsets is None else Mx
    out = torch.empty(nout, dtype=cdtype(prec), device="cuda")
    lib.grouped_trafo(p, xd, fd, out)
    torch.cuda.synchronize()
    res = out.cpu().numpy().astype(np.complex128)
    return res.reshape(R, Mx) if offsets is None else res


def gpu_adjoint(d, ds, N, x, y, prec, n_coeffs, R=1, offsets=None, m=0, sigma=0.0):
    import torch
    Mx = x.shape[0]
    p, keep = lib.make_problem(d, ds, N, M=Mx if offsets is None else 0, R=R, dtype=dtype_code(prec), m=m,
                               sigma=sigma, offsets=offsets)
    xd = to_dev(x)
    yd = to_dev(y)
    out = torch.empty(R * n_coeffs, dtype=cdtype(prec), device="cuda")
    lib.grouped_adjoint(p, xd, yd, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128).reshape(R, n_coeffs)


def max_tol(prec: str, ds: int, m: int = 0, sigma: float = 0.0) -> float:
    """Bar of max|got - ref| / ||input||_1 for a transform with window m (0: the default)."""
    mm = m or DEFAULT_M[prec]
    return ROUND[prec] + 4 * max(1, ds) * nfft_model_error(mm, sigma or 2.0)


def max_err(got, ref, src) -> float:
    """max |got - ref| / ||src||_1 per right-hand side (rows of 2-D arrays), the largest."""
    got = np.atleast_2d(np.asarray(got).astype(np.complex128))
    ref = np.atleast_2d(np.asarray(ref).astype(np.complex128))
    src = np.atleast_2d(np.asarray(src).astype(np.complex128))
    out = 0.0
    for r in range(got.shape[0]):
        l1 = float(np.abs(src[r % src.shape[0]]).sum())
        if got.shape[1]:
            out = max(out, float(np.abs(got[r] - ref[r]).max()) / max(l1, 1e-300))
    return out


def check(label, got, ref, src, tol_l2, tol_max):
    """Assert the relative l2 error and the per-element bound; print both."""
    e2 = rel(got, ref)
    em = max_err(got, ref, src)
    say(f"  {label}: rel l2 {e2:.3e} (tol {tol_l2:.1e}), max/l1 {em:.3e} (tol {tol_max:.1e})")
    assert e2 <= tol_l2, f"{label}: relative l2 error {e2:.3e} > {tol_l2:.1e}"
    assert em <= tol_max, f"{label}: max error / l1 norm {em:.3e} > {tol_max:.1e}"
    return e2, em


def _workers() -> int:
    import os
    return max(1, min(16, os.cpu_count() or 1))


def oracle_forward_at(iset, x, fhat, S):
    """Oracle forward values at the nodes S, evaluated on node chunks in a thread pool (the
    oracle's exponentials release the interpreter lock); the same sums as one call."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import transform as otr
    chunks = [c for c in np.array_split(np.asarray(S), _workers()) if len(c)]
    with ThreadPoolExecutor(len(chunks)) as ex:
        parts = list(ex.map(lambda c: otr.forward(iset, x[c], fhat), chunks))
    return np.concatenate(parts)


def oracle_adjoint_at(iset, x, y, K):
    """Oracle adjoint entries K (each an exact sum over all nodes), on coefficient chunks in
    a thread pool."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import transform as otr
    chunks = [c for c in np.array_split(np.asarray(K), _workers()) if len(c)]
    with ThreadPoolExecutor(len(chunks)) as ex:
        parts = list(ex.map(lambda c: otr.adjoint_at(iset, x, y, c), chunks))
    return np.concatenate(parts)
