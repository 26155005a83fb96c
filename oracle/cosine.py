"""Grouped cosine transform (oracle; test infrastructure only).  float64 / complex128.

The non-periodic variant of the grouped transform (Sec. 5, the half-period cosine basis, as
the extension remark after the adjoint display in Sec. 3 allows for any complete
orthonormal system of product form):

* basis on [0, 1]^d:  phi_k(x) = sqrt(2)^{|supp k|} prod_j cos(pi k_j x_j),  k in N_0^d;
* groups (Sec. 5, after eq. appl:bandwidths):  I^{u,d}_N = {k : supp k = u, 1 <= k_j <= N - 1
  for j in u}, so (N - 1)^{|u|} members as for the exponential groups; the empty set holds
  k = 0 (phi_0 = 1);
* forward:  f(x) = sum_u sum_{k in I^{u,d}_{N_u}} fhat_k phi_k(x);
* adjoint:  fhat_k = sum_x phi_k(x) y_x (the basis is real, so F^H y = F^T y).

Ordering (the paper leaves it open; the same rule as the exponential groups): terms by
order, then lexicographically; inside a group the reduced frequency l = k_u runs row-major
over {1, ..., N-1}^{|u|}, last coordinate fastest, each ascending.

Evaluated directly: per term the matrix prod_{j in u} sqrt(2) cos(pi l_j x_j) over the
group's frequencies, chunked over the nodes.
"""
from __future__ import annotations

import itertools
from typing import List

import numpy as np

from .index_set import GroupedIndexSet, anova_terms

_CHUNK = 1 << 14   # nodes per block of the explicit per-term matrix (memory bound only)


def cosine_band(N: int) -> List[int]:
    """{1, ..., N - 1}: the frequencies of one active coordinate of a cosine group."""
    if N < 2 or N % 2:
        raise ValueError("bandwidth N must be even and >= 2")
    return list(range(1, N))


def cosine_index_set(d: int, ds: int, N, keep=None) -> GroupedIndexSet:
    """The grouped cosine index set: U_{d_s} (or the kept subset, the empty set always kept)
    with groups {1..N_{|u|}-1}^{|u|}, in the order stated above."""
    N = tuple(int(n) for n in N)
    if len(N) < ds:
        raise ValueError("need one bandwidth per order 1..ds")
    terms = anova_terms(d, ds)
    if keep is not None:
        if len(keep) != len(terms):
            raise ValueError("keep needs one flag per term of U_{d_s}")
        terms = [u for u, k in zip(terms, keep) if k or not u]
    freqs = []
    for u in terms:
        t = len(u)
        if t == 0:
            freqs.append(np.zeros((1, 0), dtype=np.int64))
        else:
            freqs.append(np.array(list(itertools.product(cosine_band(N[t - 1]), repeat=t)), dtype=np.int64))
    offsets = np.zeros(len(terms) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([f.shape[0] for f in freqs])
    return GroupedIndexSet(d, ds, N[:ds], terms, offsets, freqs)


def _basis_matrix(xu: np.ndarray, ell: np.ndarray) -> np.ndarray:
    """prod_j sqrt(2) cos(pi l_j x_j) for every node (rows) and frequency (columns)."""
    out = np.ones((xu.shape[0], ell.shape[0]))
    for j in range(ell.shape[1]):
        out *= np.sqrt(2.0) * np.cos(np.pi * np.outer(xu[:, j], ell[:, j].astype(np.float64)))
    return out


def _as_batch(a):
    a = np.asarray(a)
    return (a[None, :], True) if a.ndim == 1 else (a, False)


def forward(iset: GroupedIndexSet, x: np.ndarray, fhat: np.ndarray) -> np.ndarray:
    """f = C fhat for fhat (|I|,) or (R, |I|); returns (M,) or (R, M)."""
    x = np.asarray(x, dtype=np.float64)
    F, single = _as_batch(np.asarray(fhat, dtype=np.complex128))
    M = x.shape[0]
    out = np.zeros((F.shape[0], M), dtype=np.complex128)
    for i, u in enumerate(iset.terms):
        c = F[:, iset.term_slice(i)]
        if not u:
            out += c[:, :1]
            continue
        for a in range(0, M, _CHUNK):
            b = min(M, a + _CHUNK)
            B = _basis_matrix(x[a:b][:, list(u)], iset.freqs[i])
            out[:, a:b] += (B @ c.T).T
    return out[0] if single else out


def adjoint(iset: GroupedIndexSet, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """fhat = C^T y for y (M,) or (R, M); returns (|I|,) or (R, |I|)."""
    x = np.asarray(x, dtype=np.float64)
    Y, single = _as_batch(np.asarray(y, dtype=np.complex128))
    M = x.shape[0]
    out = np.zeros((Y.shape[0], iset.n_coeffs), dtype=np.complex128)
    for i, u in enumerate(iset.terms):
        sl = iset.term_slice(i)
        if not u:
            out[:, sl] = Y.sum(axis=1, keepdims=True)
            continue
        acc = np.zeros((Y.shape[0], iset.freqs[i].shape[0]), dtype=np.complex128)
        for a in range(0, M, _CHUNK):
            b = min(M, a + _CHUNK)
            acc += Y[:, a:b] @ _basis_matrix(x[a:b][:, list(u)], iset.freqs[i])
        out[:, sl] = acc
    return out[0] if single else out


def dense_matrix(iset: GroupedIndexSet, x: np.ndarray) -> np.ndarray:
    """Explicit M x |I| matrix (phi_k(x)) with k in N_0^d: the product over all d coordinates
    of sqrt(2) cos(pi k_j x_j) for k_j > 0 and 1 for k_j = 0 (tiny cases only)."""
    K = iset.full_frequencies()
    x = np.asarray(x, dtype=np.float64)
    A = np.ones((x.shape[0], K.shape[0]))
    for j in range(iset.d):
        kj = K[:, j].astype(np.float64)
        A *= np.where(kj > 0, np.sqrt(2.0) * np.cos(np.pi * np.outer(x[:, j], kj)), 1.0)
    return A
