"""Helpers for GPU tests: move seeded numpy inputs to the device, run the C-ABI entry points,
and measure relative errors against the oracle."""
from __future__ import annotations

import math
import sys

import numpy as np

from paper_2010_10199_amd import lib

TOL = {"f32": 1e-5, "f64": 1e-12}   # relative l2 error of the transforms vs the FP64 oracle


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
