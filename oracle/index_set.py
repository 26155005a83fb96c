"""ANOVA term sets and grouped frequency index sets (oracle; test infrastructure only).

Paper passages:
* U_{d_s} = {u subset of D : |u| <= d_s}            (Sec. 2, eq. pizmosch)
* I_N = Z intersect [-N/2, N/2), N even             (Sec. 2, before eq. metallica)
* I_N^{u,d} = {k : supp k = u, k_j in I_N}          (eq. metallica)
* |I_N^{u,d}| = (N - 1)^{|u|}                       (Remark rem:cardinality)
* I_N(U) = disjoint union over u of I_{N_u}^{u,d}   (eq. groupedset)

Ordering (the paper leaves it open, Sec. 3 before eq. bananarama): terms by order
|u|, then lexicographically by the sorted coordinate tuple (the empty set first);
inside a group the reduced frequency l = k_u runs row-major over (I_N minus {0})^{|u|}
with the last coordinate fastest and each coordinate ascending
-N/2, ..., -1, 1, ..., N/2 - 1.  Coordinates are 0-based here (the paper's D = {1..d}).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np


def anova_terms(d: int, ds: int) -> List[Tuple[int, ...]]:
    """U_{d_s} in this project's order (eq. pizmosch)."""
    if d < 1 or ds < 0 or ds > d:
        raise ValueError("need d >= 1 and 0 <= ds <= d")
    out: List[Tuple[int, ...]] = []
    for t in range(ds + 1):
        out.extend(itertools.combinations(range(d), t))
    return out


def nonzero_band(N: int) -> List[int]:
    """I_N minus {0}, ascending (eq. metallica restricted to one coordinate)."""
    if N < 2 or N % 2:
        raise ValueError("bandwidth N must be even and >= 2")
    return [k for k in range(-N // 2, N // 2) if k != 0]


def group_frequencies(t: int, N: int) -> np.ndarray:
    """Reduced frequencies l in (I_N minus {0})^t, row-major, shape ((N-1)^t, t)."""
    if t == 0:
        return np.zeros((1, 0), dtype=np.int64)
    band = nonzero_band(N)
    return np.array(list(itertools.product(band, repeat=t)), dtype=np.int64)


@dataclass
class GroupedIndexSet:
    d: int
    ds: int
    N: Tuple[int, ...]                 # N[t-1] = bandwidth of every term of order t
    terms: List[Tuple[int, ...]]
    offsets: np.ndarray                # len(terms)+1 coefficient offsets
    freqs: List[np.ndarray]            # per term: reduced frequencies ((N-1)^t, t)

    @property
    def n_terms(self) -> int:
        return len(self.terms)

    @property
    def n_coeffs(self) -> int:
        return int(self.offsets[-1])

    def term_slice(self, i: int) -> slice:
        return slice(int(self.offsets[i]), int(self.offsets[i + 1]))

    def full_frequencies(self) -> np.ndarray:
        """All k in Z^d of the grouped set, in coefficient order (k_u = l, k elsewhere 0)."""
        K = np.zeros((self.n_coeffs, self.d), dtype=np.int64)
        for i, u in enumerate(self.terms):
            if u:
                K[self.term_slice(i)][:, list(u)] = self.freqs[i]
        return K

    def term_of_coeff(self) -> np.ndarray:
        out = np.empty(self.n_coeffs, dtype=np.int64)
        for i in range(self.n_terms):
            out[self.term_slice(i)] = i
        return out


def grouped_index_set(d: int, ds: int, N: Sequence[int], keep=None) -> GroupedIndexSet:
    """I_N(U) with N_u = N[|u|-1] (eq. groupedset with order-dependent bandwidths), for
    U = U_{d_s}, or for the subset of U_{d_s} whose flags in `keep` (one per term of
    anova_terms(d, ds), in that order) are nonzero; the empty set is always kept."""
    N = tuple(int(n) for n in N)
    if len(N) < ds:
        raise ValueError("need one bandwidth per order 1..ds")
    terms = anova_terms(d, ds)
    if keep is not None:
        if len(keep) != len(terms):
            raise ValueError("keep needs one flag per term of U_{d_s}")
        terms = [u for u, k in zip(terms, keep) if k or not u]
    freqs = []
    sizes = []
    for u in terms:
        t = len(u)
        f = group_frequencies(t, N[t - 1] if t else 2)
        freqs.append(f)
        sizes.append(f.shape[0])
    offsets = np.zeros(len(terms) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    return GroupedIndexSet(d, ds, N[:ds], terms, offsets, freqs)


def count_coeffs(d: int, ds: int, N: Sequence[int]) -> int:
    """|I_N(U_{d_s})| = sum over u of (N_{|u|} - 1)^{|u|} (Remark rem:cardinality)."""
    from math import comb
    return 1 + sum(comb(d, t) * (int(N[t - 1]) - 1) ** t for t in range(1, ds + 1))
