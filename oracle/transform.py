"""Direct (non-fast) grouped Fourier transform, adjoint and node gradient (oracle).

Test infrastructure only.  float64 / complex128 throughout.

* forward:  f_x = sum_u sum_{k in I^{u,d}} fhat_k e^{2 pi i <k, x>}
  (Definition def:skatoons), evaluated per term through the reduced form of eq. somafm:
  the block F(X, I^{u,d}) equals the |u|-dimensional matrix
  (e^{2 pi i <l, x_u>})_{x, l in (I_N minus {0})^{|u|}} acting on the group's coefficients.
* adjoint:  (F^H y)_u = F(X_u, ...)^H y, stacked over u (Sec. 3, the adjoint display).
* dense_matrix: the full d-dimensional Fourier matrix of eq. FM over the grouped set,
  built from the zero-padded frequencies k in Z^d (used only as a brute-force check).
* node_gradient: d f_x / d x_j = sum_{u containing j} sum_l 2 pi i l_j fhat_{u,l}
  e^{2 pi i <l, x_u>}, the analytic derivative of the definition (not in the paper).

The phase <l, x_u> is reduced modulo 1 before the exponential; e^{2 pi i theta} is
1-periodic in theta, so this changes nothing but the rounding of large arguments.
"""
from __future__ import annotations

import numpy as np

from .index_set import GroupedIndexSet

_CHUNK = 1 << 14   # nodes per block of the explicit per-term matrix (memory bound only)


def _phase_matrix(xu: np.ndarray, ell: np.ndarray) -> np.ndarray:
    """e^{2 pi i <l, x_u>} for every node (rows) and reduced frequency (columns)."""
    theta = xu @ ell.T.astype(np.float64)
    theta = theta - np.round(theta)
    return np.exp(2j * np.pi * theta)


def _as_batch(a: np.ndarray):
    a = np.asarray(a)
    return (a[None, :], True) if a.ndim == 1 else (a, False)


def forward(iset: GroupedIndexSet, x: np.ndarray, fhat: np.ndarray) -> np.ndarray:
    """f = F(X, I(U)) fhat for fhat of shape (|I|,) or (R, |I|); returns (M,) or (R, M)."""
    x = np.asarray(x, dtype=np.float64)
    F, single = _as_batch(np.asarray(fhat, dtype=np.complex128))
    M = x.shape[0]
    out = np.zeros((F.shape[0], M), dtype=np.complex128)
    for i, u in enumerate(iset.terms):
        c = F[:, iset.term_slice(i)]                     # (R, G)
        if not u:
            out += c[:, :1]                               # empty set: the k = 0 coefficient
            continue
        ell = iset.freqs[i]
        for a in range(0, M, _CHUNK):
            b = min(M, a + _CHUNK)
            E = _phase_matrix(x[a:b][:, list(u)], ell)    # (chunk, G)
            out[:, a:b] += (E @ c.T).T
    return out[0] if single else out


def adjoint(iset: GroupedIndexSet, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """fhat = F(X, I(U))^H y for y of shape (M,) or (R, M); returns (|I|,) or (R, |I|)."""
    x = np.asarray(x, dtype=np.float64)
    Y, single = _as_batch(np.asarray(y, dtype=np.complex128))
    M = x.shape[0]
    out = np.zeros((Y.shape[0], iset.n_coeffs), dtype=np.complex128)
    for i, u in enumerate(iset.terms):
        sl = iset.term_slice(i)
        if not u:
            out[:, sl] = Y.sum(axis=1, keepdims=True)
            continue
        ell = iset.freqs[i]
        acc = np.zeros((Y.shape[0], ell.shape[0]), dtype=np.complex128)
        for a in range(0, M, _CHUNK):
            b = min(M, a + _CHUNK)
            E = _phase_matrix(x[a:b][:, list(u)], ell)
            acc += Y[:, a:b] @ E.conj()
        out[:, sl] = acc
    return out[0] if single else out


def dense_matrix(iset: GroupedIndexSet, x: np.ndarray) -> np.ndarray:
    """Explicit M x |I| matrix (e^{2 pi i <k, x>}) of eq. FM with k in Z^d (tiny cases only)."""
    K = iset.full_frequencies().astype(np.float64)
    theta = np.asarray(x, dtype=np.float64) @ K.T
    theta = theta - np.round(theta)
    return np.exp(2j * np.pi * theta)


def node_gradient(iset: GroupedIndexSet, x: np.ndarray, fhat: np.ndarray) -> np.ndarray:
    """D[m, j] = d f_m / d x_{m,j} for one coefficient vector; returns (M, d) complex."""
    x = np.asarray(x, dtype=np.float64)
    c_all = np.asarray(fhat, dtype=np.complex128)
    M = x.shape[0]
    D = np.zeros((M, iset.d), dtype=np.complex128)
    for i, u in enumerate(iset.terms):
        if not u:
            continue
        ell = iset.freqs[i]
        c = c_all[iset.term_slice(i)]
        for a in range(0, M, _CHUNK):
            b = min(M, a + _CHUNK)
            E = _phase_matrix(x[a:b][:, list(u)], ell)
            for pos, j in enumerate(u):
                D[a:b, j] += E @ (2j * np.pi * ell[:, pos] * c)
    return D


def adjoint_at(iset: GroupedIndexSet, x: np.ndarray, y: np.ndarray, idx) -> np.ndarray:
    """Selected entries of F^H y: fhat_k = sum_x y_x e^{-2 pi i <k, x>} for k = K[idx] (eq. FM).

    Used to check full-size adjoints on a sample of coefficients; y of shape (M,)."""
    K = iset.full_frequencies()[np.asarray(idx)].astype(np.float64)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.complex128)
    out = np.zeros(K.shape[0], dtype=np.complex128)
    for a in range(0, x.shape[0], _CHUNK):
        b = min(x.shape[0], a + _CHUNK)
        theta = x[a:b] @ K.T
        theta = theta - np.round(theta)
        out += y[a:b] @ np.exp(-2j * np.pi * theta)
    return out
