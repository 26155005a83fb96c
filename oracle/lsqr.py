"""LSQR for the weighted Tikhonov problem of Sec. 4.1 (oracle; test infrastructure only).

Problem (eq. new_min_prob):   min_fhat  1/2 ||y - F fhat||_2^2 + lambda ||fhat||_W^2,
W = diag(omega), ||fhat||_W^2 = fhat^H W fhat.  With x = W^{1/2} fhat and A = F W^{-1/2}
this is  1/2 ( ||y - A x||^2 + 2 lambda ||x||^2 ),  i.e. damped least squares with
damping parameter sqrt(2 lambda); the paper solves it with LSQR [Paige & Saunders 1982],
which it cites but does not print.  The iteration below is the Golub-Kahan
bidiagonalisation of A started from b = y with the damping removed by one extra plane
rotation per step, written out from that method; all rotations are real because the
bidiagonal entries alpha, beta are norms.  The result is fhat = W^{-1/2} x_K.

The oracle runs one right-hand side at a time in float64.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np


@dataclass
class LsqrResult:
    fhat: np.ndarray
    iters: int
    phibar: float         # last phibar of the recurrences (residual estimate of the damped system)
    normal_est: float     # |phibar| * alpha * |c|: estimate of the normal-equation residual in x
    breakdown: bool


def lsqr(matvec: Callable[[np.ndarray], np.ndarray],
         rmatvec: Callable[[np.ndarray], np.ndarray],
         y: np.ndarray, n: int, lam: float = 0.0,
         omega: Optional[np.ndarray] = None, iters: int = 30) -> LsqrResult:
    """K = `iters` LSQR steps for eq. new_min_prob with operator F given by matvec/rmatvec."""
    if lam < 0:
        raise ValueError("lambda must be >= 0")
    y = np.asarray(y, dtype=np.complex128)
    if omega is None:
        s = np.ones(n)
    else:
        omega = np.asarray(omega, dtype=np.float64)
        if np.any(omega <= 0):
            raise ValueError("weights must be > 0")
        s = 1.0 / np.sqrt(omega)                     # W^{-1/2}
    damp = np.sqrt(2.0 * lam)

    def A(v):
        return matvec(s * v)

    def AH(u):
        return s * rmatvec(u)

    x = np.zeros(n, dtype=np.complex128)
    beta = np.linalg.norm(y)
    if beta == 0.0:
        return LsqrResult(x, 0, 0.0, 0.0, True)
    u = y / beta
    v = AH(u)
    alpha = np.linalg.norm(v)
    if alpha == 0.0:
        return LsqrResult(x, 0, beta, 0.0, True)
    v = v / alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    normal = alpha * beta
    breakdown = False
    k = 0
    for k in range(1, iters + 1):
        # continue the bidiagonalisation
        u = A(v) - alpha * u
        beta = np.linalg.norm(u)
        if beta > 0:
            u = u / beta
        v = AH(u) - beta * v
        alpha = np.linalg.norm(v)
        if alpha > 0:
            v = v / alpha
        # rotation eliminating the damping row
        rhobar1 = np.hypot(rhobar, damp)
        c1, s1 = rhobar / rhobar1, damp / rhobar1
        phibar = c1 * phibar
        # rotation eliminating the subdiagonal beta
        rho = np.hypot(rhobar1, beta)
        c, sn = rhobar1 / rho, beta / rho
        theta = sn * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = sn * phibar
        # update solution and search direction
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        normal = abs(phibar) * alpha * abs(c)      # phibar carries a sign
        if beta == 0.0 or alpha == 0.0:
            breakdown = True
            break
    return LsqrResult(s * x, k, float(phibar), float(normal), breakdown)
