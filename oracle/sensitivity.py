"""Global sensitivity indices and the active set (oracle; test infrastructure only).

Paper passages:
* rho(u, f) = sigma^2(f_u) / sigma^2(f),  sigma^2(f) = ||f||^2 - |fhat_0|^2   (Sec. 2, eq. gsi)
* for a trigonometric polynomial with coefficients on a grouped index set, the ANOVA term
  f_u collects exactly the group of u (its frequencies have support u, eq. metallica), so
  by Parseval's identity ||f_u||^2 = sum of |fhat_k|^2 over the group, and sigma^2(f) is the
  sum over every group but the empty set's
* U* = {empty set} union {u : rho(u, S f) > eps_{|u|}}                          (eq. activeset)
* eps(X, I_N(U)) = ||f - S f|| / ||f||, by Parseval
  ||f - S f||^2 = ||f||^2 + sum_{k in I} |fhat_k - c_k(f)|^2 - sum_{k in I} |c_k(f)|^2  (Sec. 4, eq. L2error)
"""
from __future__ import annotations

import numpy as np

from .index_set import GroupedIndexSet, anova_terms


def term_energies(iset: GroupedIndexSet, fhat: np.ndarray) -> np.ndarray:
    """||f_u||^2 for every term of the index set (Parseval): shape (..., |U|)."""
    fhat = np.asarray(fhat, dtype=np.complex128)
    out = np.zeros(fhat.shape[:-1] + (iset.n_terms,))
    for i in range(iset.n_terms):
        g = fhat[..., iset.term_slice(i)]
        out[..., i] = np.sum(g.real ** 2 + g.imag ** 2, axis=-1)
    return out


def sensitivity_indices(iset: GroupedIndexSet, fhat: np.ndarray) -> np.ndarray:
    """rho(u, f) of eq. gsi for every term (0 for the empty set and for a zero variance)."""
    e = term_energies(iset, fhat)
    var = np.sum(e[..., 1:], axis=-1, keepdims=True)
    rho = np.where(var > 0, e / np.where(var > 0, var, 1.0), 0.0)
    rho[..., 0] = 0.0
    return rho


def active_set(iset: GroupedIndexSet, rho: np.ndarray, eps) -> np.ndarray:
    """Flags over anova_terms(d, ds) of U* (eq. activeset) from the indices rho of the index
    set's terms and one threshold per order."""
    full = anova_terms(iset.d, iset.ds)
    where = {u: i for i, u in enumerate(iset.terms)}
    mask = np.zeros(len(full), dtype=np.uint8)
    for c, u in enumerate(full):
        if not u:
            mask[c] = 1
        elif u in where:
            mask[c] = 1 if rho[where[u]] > eps[len(u) - 1] else 0
    return mask


def l2_error(iset: GroupedIndexSet, fhat: np.ndarray, exact: np.ndarray, norm2: float) -> float:
    """eps(X, I_N(U)) of eq. L2error from the approximation's coefficients fhat, the
    target's exact coefficients on the same index set and its squared L2 norm."""
    fhat = np.asarray(fhat, dtype=np.complex128)
    exact = np.asarray(exact, dtype=np.complex128)
    if fhat.shape[-1] != iset.n_coeffs or exact.shape[-1] != iset.n_coeffs:
        raise ValueError("coefficient vectors must match the index set")
    e2 = norm2 + np.sum(np.abs(fhat - exact) ** 2, axis=-1) - np.sum(np.abs(exact) ** 2, axis=-1)
    return np.sqrt(np.maximum(e2, 0.0) / norm2)
