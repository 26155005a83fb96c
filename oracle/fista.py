"""Group-lasso proximal map and FISTA (oracle; test infrastructure only).

Problem (eq. alligatoah):  min_fhat 1/2 ||y - F fhat||^2 + lambda sum_u ||fhat(u)||_{W(u)}
with W(u) = diag(omega_k), ||z||_W^2 = sum_k omega_k |z_k|^2.  Every ANOVA term u is a
group, the empty set included (the sum in eq. alligatoah runs over all of U).

* prox (Theorem theorem:projection, built on Lemma lemma:lennykrawitz): for the map
  argmin_x 1/2 ||x - z||^2 + tau sum_u ||x_u||_{W(u)}, group u becomes 0 when
  tau >= ||(z_k / omega_k)||_W = (sum_k |z_k|^2 / omega_k)^{1/2}; otherwise
  x_k = z_k / (1 + xi omega_k) with xi the root of
  t(xi) = sum_k omega_k |z_k|^2 / (1/xi + omega_k)^2 = tau^2.
* root finding (the remark after the Theorem): decide whether t(1) >= tau^2; if so
  bisect xi on [0, 1], else bisect zeta = 1/xi on [0, 1]; then refine with Newton
  steps.  This oracle takes 60 bisection halvings and at most 20 Newton steps that stop
  once |t - tau^2| <= 1e-15 tau^2 (the paper fixes neither count; t is strictly
  increasing, so the root is unique and any converged finder agrees).
* fista: Algorithm algo:fista.  With eta > 1 the backtracking loop runs; its test on
  squared residuals (complex inner product read as Re(a^H b)) is evaluated in the
  algebraically identical form ||F(f - h)||^2 > L ||f - h||^2, see the comment there.
  Without eta (or eta <= 1) the constant step size variant named in the remark after
  the algorithm runs, with the step constant L held fixed.
* power_iteration: estimate of ||F||_2^2 used to choose a constant L.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional, Sequence

import numpy as np

BISECT_STEPS = 60
NEWTON_STEPS = 20
BACKTRACK_CAP = 30


def _t(xi: float, a: np.ndarray, w: np.ndarray) -> float:
    """t(xi) with a = |z_k|^2 and w = omega_k (Theorem's equation for xi, squared)."""
    return float(np.sum(w * a / (1.0 / xi + w) ** 2))


def _t_of_zeta(zeta: float, a: np.ndarray, w: np.ndarray) -> float:
    """t(1/zeta) = sum omega |z|^2 / (zeta + omega)^2."""
    return float(np.sum(w * a / (zeta + w) ** 2))


def solve_xi(z: np.ndarray, w: np.ndarray, tau: float) -> float:
    """Root xi > 0 of t(xi) = tau^2 for one group (caller ensures tau < ||z / omega||_W)."""
    a = np.abs(z) ** 2
    target = tau * tau
    if _t(1.0, a, w) >= target:
        lo, hi = 0.0, 1.0                      # xi in (0, 1]; t increasing in xi
        for _ in range(BISECT_STEPS):
            mid = 0.5 * (lo + hi)
            if mid > 0 and _t(mid, a, w) < target:
                lo = mid
            else:
                hi = mid
        xi = 0.5 * (lo + hi)
    else:
        lo, hi = 0.0, 1.0                      # zeta = 1/xi in (0, 1); t(1/zeta) decreasing
        for _ in range(BISECT_STEPS):
            mid = 0.5 * (lo + hi)
            if _t_of_zeta(mid, a, w) > target:
                lo = mid
            else:
                hi = mid
        xi = 1.0 / (0.5 * (lo + hi))
    for _ in range(NEWTON_STEPS):              # Newton on t(xi) - tau^2
        den = 1.0 + xi * w
        val = float(np.sum(w * a * xi * xi / den ** 2)) - target
        if abs(val) <= 1e-15 * target:
            break
        der = float(np.sum(w * a * 2.0 * xi / den ** 3))
        if der <= 0:
            break
        step = xi - val / der
        xi = step if step > 0 else 0.5 * xi
    return xi


def prox(z: np.ndarray, offsets: Sequence[int], tau: float,
         omega: Optional[np.ndarray] = None) -> np.ndarray:
    """argmin_x 1/2||x - z||^2 + tau sum_u ||x_u||_{W(u)} (Theorem theorem:projection)."""
    z = np.asarray(z, dtype=np.complex128)
    w_all = np.ones(z.shape[0]) if omega is None else np.asarray(omega, dtype=np.float64)
    x = np.zeros_like(z)
    for g in range(len(offsets) - 1):
        sl = slice(int(offsets[g]), int(offsets[g + 1]))
        zu, wu = z[sl], w_all[sl]
        zero_level = np.sqrt(np.sum(np.abs(zu) ** 2 / wu))     # ||(z_k/omega_k)||_W
        if tau >= zero_level:
            continue                                           # Lemma (iii): group is zero
        xi = solve_xi(zu, wu, tau)
        x[sl] = zu / (1.0 + xi * wu)
    return x


def objective(matvec, y, fhat, offsets, lam, omega=None) -> float:
    """1/2 ||y - F fhat||^2 + lambda sum_u ||fhat_u||_{W(u)} (eq. alligatoah)."""
    r = y - matvec(fhat)
    w_all = np.ones(fhat.shape[0]) if omega is None else np.asarray(omega)
    pen = 0.0
    for g in range(len(offsets) - 1):
        sl = slice(int(offsets[g]), int(offsets[g + 1]))
        pen += np.sqrt(np.sum(w_all[sl] * np.abs(fhat[sl]) ** 2))
    return 0.5 * float(np.vdot(r, r).real) + lam * pen


def power_iteration(matvec, rmatvec, n: int, iters: int = 50) -> float:
    """Rayleigh-quotient estimate of ||F||_2^2 = lambda_max(F^H F), start vector all ones."""
    v = np.ones(n, dtype=np.complex128) / np.sqrt(n)
    est = 0.0
    for _ in range(iters):
        w = rmatvec(matvec(v))
        est = float(np.vdot(v, w).real)
        nrm = np.linalg.norm(w)
        if nrm == 0:
            break
        v = w / nrm
    return est


@dataclass
class FistaResult:
    fhat: np.ndarray
    iters: int
    L: float
    t: float
    backtracks: int


def fista(matvec: Callable[[np.ndarray], np.ndarray],
          rmatvec: Callable[[np.ndarray], np.ndarray],
          y: np.ndarray, offsets: Sequence[int], lam: float, L: float, iters: int,
          f0: Optional[np.ndarray] = None, omega: Optional[np.ndarray] = None,
          eta: Optional[float] = None) -> FistaResult:
    """Algorithm algo:fista for eq. alligatoah (one right-hand side, float64)."""
    if lam <= 0:
        raise ValueError("lambda must be > 0")
    if L <= 0:
        raise ValueError("L must be > 0")
    y = np.asarray(y, dtype=np.complex128)
    n = int(offsets[-1])
    f_prev = np.zeros(n, dtype=np.complex128) if f0 is None else np.asarray(f0, np.complex128).copy()
    h = f_prev.copy()
    t = 1.0
    backtracks = 0
    f = f_prev
    for _ in range(iters):
        Fh = matvec(h)
        grad = rmatvec(Fh - y)                      # gradient of 1/2||y - F h||^2 at h

        def p(Lk):
            return prox(h - grad / Lk, offsets, lam / Lk, omega)

        f = p(L)
        if eta is not None and eta > 1.0:
            # The algorithm's while-test
            #   ||y - F f||^2 - ||y - F h||^2 > 2 Re<f - h, grad> + L ||f - h||^2
            # equals ||F (f - h)||^2 > L ||f - h||^2 exactly (expand the first difference
            # around h).  The literal difference of two squared residuals cancels
            # catastrophically near convergence and then triggers spurious backtracks, so
            # the equivalent form is evaluated.
            for _b in range(BACKTRACK_CAP):
                dlt = f - h
                Fd = matvec(dlt)
                if float(np.vdot(Fd, Fd).real) <= L * float(np.vdot(dlt, dlt).real):
                    break
                L = eta * L
                backtracks += 1
                f = p(L)
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        h = f + ((t - 1.0) / t_next) * (f - f_prev)
        f_prev = f
        t = t_next
    return FistaResult(f, iters, L, t, backtracks)
