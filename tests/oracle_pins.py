"""Pins of the oracle against what the paper and the mathematics fix.

Each function returns a non-negative error; the pin holds when it is below the stated
tolerance.  ``test_oracle_*.py`` asserts the tolerances, and ``test_oracle_mutations.py``
plants plausible mistakes in the oracle and checks that some pin then fails.
None of these re-types the oracle's formula: they compare with numpy.fft, with exact
orthogonality of rank-1 lattices, with independent enumeration rules, with the dense
d-dimensional matrix built from full frequency vectors, with scipy's LSQR, with dense
linear algebra, with finite differences and with exact grid quadrature.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np

from oracle import cosine as ocos
from oracle import fista as ofista
from oracle import index_set as oidx
from oracle import lsqr as olsqr
from oracle import sensitivity as osens
from oracle import transform as otr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


# ---------------------------------------------------------------- index set
def pin_printed_counts() -> float:
    """|I_N(U)| and |U| printed in the paper (tests/golden/cardinalities.json)."""
    with open(os.path.join(GOLDEN, "cardinalities.json")) as fh:
        cases = json.load(fh)["cases"]
    err = 0
    for c in cases:
        if "coeffs" in c:
            iset = oidx.grouped_index_set(c["d"], c["ds"], c["N"])
            err += abs(iset.n_coeffs - c["coeffs"])
            err += abs(oidx.count_coeffs(c["d"], c["ds"], c["N"]) - c["coeffs"])
        if "terms" in c:
            err += abs(len(oidx.anova_terms(c["d"], c["ds"])) - c["terms"])
    return float(err)


def pin_ordering(d=4, ds=3, N=(6, 4, 4)) -> float:
    """Coefficient order equals the rule stated in the oracle header, enumerated independently."""
    iset = oidx.grouped_index_set(d, ds, N)
    expect = []
    for t in range(ds + 1):
        for u in itertools.combinations(range(d), t):
            band = [k for k in range(-N[t - 1] // 2, N[t - 1] // 2) if k != 0] if t else []
            for ell in itertools.product(band, repeat=t):
                k = [0] * d
                for c, v in zip(u, ell):
                    k[c] = v
                expect.append(k)
    got = iset.full_frequencies()
    if got.shape != (len(expect), d):
        return 1.0
    return float(np.abs(got - np.array(expect)).sum())


# ---------------------------------------------------------------- transform
def pin_dense_matrix(seed=1, d=4, ds=3, N=(6, 4, 4), M=37) -> float:
    """Forward and adjoint equal products with the d-dimensional matrix of eq. FM (k in Z^d)."""
    g = np.random.default_rng(seed)
    iset = oidx.grouped_index_set(d, ds, N)
    x = g.random((M, d)) - 0.5
    fh = g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)
    y = g.standard_normal(M) + 1j * g.standard_normal(M)
    # independent construction: full frequency vectors from the ordering rule
    K = []
    for t in range(ds + 1):
        for u in itertools.combinations(range(d), t):
            band = [k for k in range(-N[t - 1] // 2, N[t - 1] // 2) if k != 0] if t else []
            for ell in itertools.product(band, repeat=t):
                k = np.zeros(d)
                k[list(u)] = ell
                K.append(k)
    K = np.array(K)
    A = np.cos(2 * np.pi * x @ K.T) + 1j * np.sin(2 * np.pi * x @ K.T)
    return max(rel(otr.forward(iset, x, fh), A @ fh), rel(otr.adjoint(iset, x, y), A.conj().T @ y))


def pin_adjoint_at(seed=5, d=5, ds=3, N=(6, 4, 4), M=43, picks=60) -> float:
    """Selected adjoint entries equal rows of the conjugate transpose of the d-dimensional
    matrix of eq. FM (k in Z^d), built independently from the ordering rule: (A^H y)[idx]
    for a sample of coefficients that includes the empty set and terms of orders 1, 2, 3,
    taken out of order and with a repeated index."""
    g = np.random.default_rng(seed)
    iset = oidx.grouped_index_set(d, ds, N)
    x = g.random((M, d)) - 0.5
    y = g.standard_normal(M) + 1j * g.standard_normal(M)
    K = []
    for t in range(ds + 1):
        for u in itertools.combinations(range(d), t):
            band = [k for k in range(-N[t - 1] // 2, N[t - 1] // 2) if k != 0] if t else []
            for ell in itertools.product(band, repeat=t):
                k = np.zeros(d)
                k[list(u)] = ell
                K.append(k)
    K = np.array(K)
    order = (K != 0).sum(axis=1)
    idx = [0] + [int(g.choice(np.flatnonzero(order == t))) for t in range(1, ds + 1)]
    idx += list(g.choice(len(K), picks, replace=False)) + [idx[2]]
    idx = np.array(idx)[g.permutation(len(idx))]
    A = np.cos(2 * np.pi * x @ K.T) + 1j * np.sin(2 * np.pi * x @ K.T)
    return rel(otr.adjoint_at(iset, x, y, idx), (A.conj().T @ y)[idx])


def pin_hypercube_fft(d=3, N=6) -> float:
    """U = P(D), N_u = N, nodes on the grid l/N: the grouped transform is a d-dim inverse FFT.

    The groups of P(D) partition I_N^d (eq. hypercube), so F fhat on the grid equals
    N^d * numpy.fft.ifftn of the coefficients placed at k mod N, and F^H y equals
    numpy.fft.fftn of the samples read at k mod N.
    """
    iset = oidx.grouped_index_set(d, d, [N] * d)
    grid = np.array(list(itertools.product(range(N), repeat=d)))       # l in {0..N-1}^d
    x = grid / N
    x = np.where(x >= 0.5, x - 1.0, x)                                   # same torus points
    g = np.random.default_rng(7)
    fh = g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)
    K = iset.full_frequencies()
    if len(K) != N ** d:
        return 1.0
    C = np.zeros((N,) * d, dtype=complex)
    for val, k in zip(fh, K):
        C[tuple(np.mod(k, N))] += val
    ref = (N ** d) * np.fft.ifftn(C)
    got = otr.forward(iset, x, fh)
    e1 = rel(got, np.array([ref[tuple(l)] for l in grid]))
    y = g.standard_normal(len(grid)) + 1j * g.standard_normal(len(grid))
    Y = np.zeros((N,) * d, dtype=complex)
    for val, l in zip(y, grid):
        Y[tuple(l)] = val
    F = np.fft.fftn(Y)
    e2 = rel(otr.adjoint(iset, x, y), np.array([F[tuple(np.mod(k, N))] for k in K]))
    return max(e1, e2)


def lattice(iset, M, seed=3, tries=20000):
    """Rank-1 lattice x_j = (j z / M) mod 1 whose Fourier matrix has orthogonal columns.

    F^H F = M I holds exactly when the values <k, z> mod M are distinct over the index set
    (character orthogonality on Z_M); z is searched at random and checked by brute force.
    """
    K = iset.full_frequencies()
    g = np.random.default_rng(seed)
    for _ in range(tries):
        z = g.integers(1, M, size=iset.d)
        r = np.mod(K @ z, M)
        if len(np.unique(r)) == len(r):
            j = np.arange(M)[:, None]
            x = np.mod(j * z[None, :], M) / M
            return np.where(x >= 0.5, x - 1.0, x), z
    raise RuntimeError("no lattice generator found")


def pin_lattice_orthogonality(d=3, ds=2, N=(8, 4), M=211) -> float:
    """F^H F fhat = M fhat on a reconstructing rank-1 lattice (pins forward and adjoint together)."""
    iset = oidx.grouped_index_set(d, ds, N)
    x, _ = lattice(iset, M)
    g = np.random.default_rng(5)
    fh = g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)
    return rel(otr.adjoint(iset, x, otr.forward(iset, x, fh)), M * fh)


def pin_adjoint_identity(seed=2, d=5, ds=3, N=(10, 6, 4), M=50) -> float:
    """<F fhat, y> = <fhat, F^H y>."""
    g = np.random.default_rng(seed)
    iset = oidx.grouped_index_set(d, ds, N)
    x = g.random((M, d)) - 0.5
    fh = g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)
    y = g.standard_normal(M) + 1j * g.standard_normal(M)
    a = np.vdot(y, otr.forward(iset, x, fh))
    b = np.vdot(otr.adjoint(iset, x, y), fh)
    return abs(a - b) / abs(a)


def pin_modulation(seed=4, d=4, ds=2, N=(8, 6), M=30, j=2, shift=0.137) -> float:
    """Shifting x_j by s multiplies every coefficient with u containing j by e^{2 pi i l_j s}."""
    g = np.random.default_rng(seed)
    iset = oidx.grouped_index_set(d, ds, N)
    x = g.random((M, d)) - 0.5
    fh = g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)
    K = iset.full_frequencies()
    mod = fh * np.exp(2j * np.pi * K[:, j] * shift)
    xs = x.copy()
    xs[:, j] += shift
    return rel(otr.forward(iset, xs, fh), otr.forward(iset, x, mod))


def pin_group_isolation(seed=6, d=5, ds=2, N=(8, 6), M=25) -> float:
    """A coefficient vector supported on one group u depends only on x_u; the empty set is constant."""
    g = np.random.default_rng(seed)
    iset = oidx.grouped_index_set(d, ds, N)
    x = g.random((M, d)) - 0.5
    err = 0.0
    for ti in (0, 3, iset.n_terms - 1):
        u = iset.terms[ti]
        fh = np.zeros(iset.n_coeffs, dtype=complex)
        sl = iset.term_slice(ti)
        fh[sl] = g.standard_normal(sl.stop - sl.start)
        x2 = x.copy()
        others = [c for c in range(d) if c not in u]
        x2[:, others] = g.random((M, len(others))) - 0.5
        err = max(err, rel(otr.forward(iset, x2, fh), otr.forward(iset, x, fh)))
        if not u:
            err = max(err, float(np.abs(otr.forward(iset, x, fh) - fh[0]).max()))
    return err


def pin_single_frequency(seed=8, d=4, ds=3, N=(6, 4, 4), M=20) -> float:
    """fhat = unit vector at (u, l) gives exactly e^{2 pi i <l, x_u>} (closed form by cos/sin)."""
    g = np.random.default_rng(seed)
    iset = oidx.grouped_index_set(d, ds, N)
    x = g.random((M, d)) - 0.5
    K = iset.full_frequencies()
    err = 0.0
    for p in g.choice(iset.n_coeffs, size=6, replace=False):
        e = np.zeros(iset.n_coeffs)
        e[p] = 1.0
        ang = 2 * math.pi * (x @ K[p])
        err = max(err, float(np.abs(otr.forward(iset, x, e) - (np.cos(ang) + 1j * np.sin(ang))).max()))
    return err


def pin_gradient_fd(seed=9, d=4, ds=2, N=(8, 6), M=12, h=1e-5) -> float:
    """Node gradient against central finite differences of the forward transform."""
    g = np.random.default_rng(seed)
    iset = oidx.grouped_index_set(d, ds, N)
    x = g.random((M, d)) * 0.8 - 0.4
    fh = g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)
    D = otr.node_gradient(iset, x, fh)
    FD = np.zeros_like(D)
    for j in range(d):
        xp, xm = x.copy(), x.copy()
        xp[:, j] += h
        xm[:, j] -= h
        FD[:, j] = (otr.forward(iset, xp, fh) - otr.forward(iset, xm, fh)) / (2 * h)
    return rel(D, FD)


# ---------------------------------------------------------------- LSQR
def _small_problem(seed, d=3, ds=2, N=(8, 4), M=120):
    g = np.random.default_rng(seed)
    iset = oidx.grouped_index_set(d, ds, N)
    x = g.random((M, d)) - 0.5
    y = g.standard_normal(M) + 1j * g.standard_normal(M)
    return iset, x, y, g


def pin_lsqr_dense(seed=11, lam=0.3, weighted=True) -> float:
    """Converged LSQR equals the dense solve of (F^H F + 2 lambda W) fhat = F^H y."""
    iset, x, y, g = _small_problem(seed)
    A = otr.dense_matrix(iset, x)
    omega = (1.0 + g.random(iset.n_coeffs) * 3.0) if weighted else None
    W = np.diag(omega if omega is not None else np.ones(iset.n_coeffs))
    ref = np.linalg.solve(A.conj().T @ A + 2 * lam * W, A.conj().T @ y)
    res = olsqr.lsqr(lambda v: otr.forward(iset, x, v), lambda r: otr.adjoint(iset, x, r),
                     y, iset.n_coeffs, lam, omega, iters=4 * iset.n_coeffs)
    return rel(res.fhat, ref)


def pin_lsqr_scipy(seed=12, lam=0.05, iters=7) -> float:
    """The K-th iterate equals scipy.sparse.linalg.lsqr's K-th iterate (same damping sqrt(2 lambda))."""
    from scipy.sparse.linalg import lsqr as sp_lsqr
    iset, x, y, _ = _small_problem(seed)
    A = otr.dense_matrix(iset, x)
    ref = sp_lsqr(A, y, damp=math.sqrt(2 * lam), iter_lim=iters, atol=0, btol=0, conlim=0)[0]
    res = olsqr.lsqr(lambda v: otr.forward(iset, x, v), lambda r: otr.adjoint(iset, x, r),
                     y, iset.n_coeffs, lam, None, iters=iters)
    return rel(res.fhat, ref)


def pin_lsqr_lattice(lam=0.7) -> float:
    """Orthogonal F (F^H F = M I): fhat = F^H y / (M + 2 lambda), reached in one step."""
    iset = oidx.grouped_index_set(3, 2, (8, 4))
    M = 211
    x, _ = lattice(iset, M)
    g = np.random.default_rng(13)
    y = g.standard_normal(M) + 1j * g.standard_normal(M)
    ref = otr.adjoint(iset, x, y) / (M + 2 * lam)
    res = olsqr.lsqr(lambda v: otr.forward(iset, x, v), lambda r: otr.adjoint(iset, x, r),
                     y, iset.n_coeffs, lam, None, iters=3)
    return rel(res.fhat, ref)


# ---------------------------------------------------------------- prox / FISTA
def pin_prox_soft_threshold(seed=21) -> float:
    """omega = 1: the prox is block soft-thresholding x_u = (1 - tau/||z_u||)_+ z_u."""
    g = np.random.default_rng(seed)
    offsets = [0, 1, 8, 15, 64]
    z = g.standard_normal(64) + 1j * g.standard_normal(64)
    tau = 2.5
    ref = np.zeros_like(z)
    for a, b in zip(offsets[:-1], offsets[1:]):
        nrm = np.linalg.norm(z[a:b])
        ref[a:b] = max(0.0, 1.0 - tau / nrm) * z[a:b]
    return rel(ofista.prox(z, offsets, tau), ref)


def pin_prox_minimises(seed=22) -> float:
    """Weighted prox output minimises its objective: compare with scipy.optimize on tiny groups."""
    from scipy.optimize import minimize
    g = np.random.default_rng(seed)
    offsets = [0, 3, 7]
    n = 7
    z = g.standard_normal(n) + 1j * g.standard_normal(n)
    omega = 1.0 + 4.0 * g.random(n)
    err = 0.0
    for tau in (0.3, 1.1, 2.0):
        x = ofista.prox(z, offsets, tau, omega)

        def obj(v):
            c = v[:n] + 1j * v[n:]
            val = 0.5 * np.sum(np.abs(c - z) ** 2)
            for a, b in zip(offsets[:-1], offsets[1:]):
                val += tau * np.sqrt(np.sum(omega[a:b] * np.abs(c[a:b]) ** 2) + 1e-300)
            return val
        v0 = np.concatenate([x.real, x.imag])
        best = minimize(obj, np.concatenate([z.real, z.imag]), method="Nelder-Mead",
                        options=dict(maxiter=40000, xatol=1e-12, fatol=1e-14))
        # the oracle's value must not exceed the numerical optimum
        err = max(err, max(0.0, obj(v0) - best.fun))
        # and random perturbations must not improve it (convexity)
        for _ in range(50):
            dv = g.standard_normal(2 * n) * 1e-3
            err = max(err, max(0.0, obj(v0) - obj(v0 + dv)))
    return err


def pin_prox_zero_threshold(seed=23) -> float:
    """Lemma (iii): a group is zero exactly when tau >= (sum |z_k|^2 / omega_k)^{1/2}."""
    g = np.random.default_rng(seed)
    z = g.standard_normal(9) + 1j * g.standard_normal(9)
    omega = 1.0 + g.random(9)
    lvl = math.sqrt(float(np.sum(np.abs(z) ** 2 / omega)))
    above = ofista.prox(z, [0, 9], lvl * 1.0001, omega)
    below = ofista.prox(z, [0, 9], lvl * 0.999, omega)
    return float(np.abs(above).max()) + (1.0 if np.abs(below).max() == 0 else 0.0)


def pin_prox_ridge_link(seed=24) -> float:
    """Lemma (i)/(ii): the prox equals the ridge minimiser y/(1 + 2 xi' omega) at the matching xi'.

    Pick xi' > 0, set lambda = ||(y_k / (1/(2 xi') + omega_k))||_W (Lemma (ii)); then the
    group prox at tau = lambda must return diag(1/(1 + 2 xi' omega)) y (Lemma (i)).
    """
    g = np.random.default_rng(seed)
    y = g.standard_normal(11) + 1j * g.standard_normal(11)
    omega = 1.0 + 3.0 * g.random(11)
    err = 0.0
    for xi2 in (0.05, 0.7, 4.0, 40.0):
        lam = math.sqrt(float(np.sum(omega * np.abs(y / (1.0 / (2 * xi2) + omega)) ** 2)))
        ridge = y / (1.0 + 2 * xi2 * omega)
        err = max(err, rel(ofista.prox(y, [0, 11], lam, omega), ridge))
    return err


def _fista_problem(seed=31, d=3, ds=2, N=(8, 4), M=150):
    g = np.random.default_rng(seed)
    iset = oidx.grouped_index_set(d, ds, N)
    x = g.random((M, d)) - 0.5
    y = g.standard_normal(M) + 1j * g.standard_normal(M)
    A = otr.dense_matrix(iset, x)
    return iset, x, y, A


def _kkt(iset, A, y, f, lam) -> float:
    """Group-lasso optimality: (F^H(y - F f))_u = lam f_u/||f_u|| if f_u != 0, else its norm <= lam."""
    gr = A.conj().T @ (y - A @ f)
    err = 0.0
    for i in range(iset.n_terms):
        sl = iset.term_slice(i)
        nf = np.linalg.norm(f[sl])
        if nf > 1e-12:
            err = max(err, np.linalg.norm(gr[sl] - lam * f[sl] / nf) / lam)
        else:
            err = max(err, max(0.0, np.linalg.norm(gr[sl]) - lam) / lam)
    return float(err)


def pin_fista_kkt(lam=6.0, iters=600) -> float:
    """KKT certificate at the FISTA output (constant step L = ||F||^2)."""
    iset, x, y, A = _fista_problem()
    L = np.linalg.norm(A, 2) ** 2
    res = ofista.fista(lambda v: A @ v, lambda r: A.conj().T @ r, y, iset.offsets, lam, L, iters)
    return _kkt(iset, A, y, res.fhat, lam)


def pin_fista_zero_above_lambda_max() -> float:
    """lambda >= max_u ||(F^H y)_u|| gives the zero solution from a zero start."""
    iset, x, y, A = _fista_problem()
    gy = A.conj().T @ y
    lmax = max(np.linalg.norm(gy[iset.term_slice(i)]) for i in range(iset.n_terms))
    L = np.linalg.norm(A, 2) ** 2
    res = ofista.fista(lambda v: A @ v, lambda r: A.conj().T @ r, y, iset.offsets, lmax * 1.001, L, 50)
    return float(np.abs(res.fhat).max())


def pin_fista_lattice(lam=9.0) -> float:
    """Orthogonal F: the group-lasso solution is (1 - lam/||(F^H y)_u||)_+ (F^H y)_u / M."""
    iset = oidx.grouped_index_set(3, 2, (8, 4))
    M = 211
    x, _ = lattice(iset, M)
    A = otr.dense_matrix(iset, x)
    g = np.random.default_rng(33)
    y = g.standard_normal(M) + 1j * g.standard_normal(M)
    gy = A.conj().T @ y
    ref = np.zeros_like(gy)
    for i in range(iset.n_terms):
        sl = iset.term_slice(i)
        nrm = np.linalg.norm(gy[sl])
        ref[sl] = max(0.0, 1.0 - lam / nrm) * gy[sl] / M
    res = ofista.fista(lambda v: A @ v, lambda r: A.conj().T @ r, y, iset.offsets, lam, float(M), 40)
    return rel(res.fhat, ref)


def pin_fista_backtracking(lam=6.0) -> float:
    """Backtracking from a too-small L0 (it must backtrack) reaches a KKT point as well."""
    iset, x, y, A = _fista_problem()
    L = np.linalg.norm(A, 2) ** 2
    b = ofista.fista(lambda v: A @ v, lambda r: A.conj().T @ r, y, iset.offsets, lam, L / 50, 600, eta=2.0)
    return _kkt(iset, A, y, b.fhat, lam) + (0.0 if b.backtracks > 0 else 1.0)


def pin_power_iteration() -> float:
    """Power-iteration estimate against the dense spectral norm ||F||_2^2."""
    iset, x, y, A = _fista_problem()
    est = ofista.power_iteration(lambda v: A @ v, lambda r: A.conj().T @ r, iset.n_coeffs, 300)
    ref = np.linalg.norm(A, 2) ** 2
    return abs(est - ref) / ref


def pin_fista_first_steps() -> float:
    """t_1 = 1 makes the first momentum coefficient zero: with a negligible lambda the
    first two FISTA iterates are two plain gradient steps f <- f - F^H(F f - y)/L."""
    iset, x, y, A = _fista_problem()
    L = np.linalg.norm(A, 2) ** 2
    f1 = np.zeros(iset.n_coeffs, dtype=complex)
    f1 = f1 - A.conj().T @ (A @ f1 - y) / L
    f2 = f1 - A.conj().T @ (A @ f1 - y) / L
    r1 = ofista.fista(lambda v: A @ v, lambda r: A.conj().T @ r, y, iset.offsets, 1e-300, L, 1)
    r2 = ofista.fista(lambda v: A @ v, lambda r: A.conj().T @ r, y, iset.offsets, 1e-300, L, 2)
    return max(rel(r1.fhat, f1), rel(r2.fhat, f2))


def pin_fista_rate(lam=3.0, K=60) -> float:
    """Beck-Teboulle bound F(f_k) - F* <= 2 L ||f_0 - f*||^2 / (k+1)^2 for every k <= K.

    Returns the largest ratio (gap / bound) minus 1, clipped at 0."""
    iset, x, y, A = _fista_problem()
    L = np.linalg.norm(A, 2) ** 2
    mv, rmv = (lambda v: A @ v), (lambda r: A.conj().T @ r)
    star = ofista.fista(mv, rmv, y, iset.offsets, lam, L, 1500).fhat
    Fs = ofista.objective(mv, y, star, iset.offsets, lam)
    worst = 0.0
    for k in range(1, K + 1):
        fk = ofista.fista(mv, rmv, y, iset.offsets, lam, L, k).fhat
        gap = ofista.objective(mv, y, fk, iset.offsets, lam) - Fs
        bound = 2 * L * np.linalg.norm(star) ** 2 / (k + 1) ** 2
        worst = max(worst, gap / bound)
    return max(0.0, worst - 1.0)


# ---------------------------------------------------------------- pin table
# (name, function, keyword arguments, tolerance): the pin holds when error <= tolerance.
# ---------------------------------------------------------------- sensitivity analysis
def _random_fhat(iset, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)


def pin_gsi_quadrature(seed=41, d=3, ds=2, N=(6, 4), K=8) -> float:
    """rho(u) of eq. gsi against the variances of the evaluated term functions: on the
    tensor grid {j/K}^d with K >= N, the grid mean of |g|^2 is exactly the squared L2 norm of
    a trigonometric polynomial g with frequencies in [-N/2, N/2), so ||f_u||^2 and sigma^2(f)
    come from the transform evaluated on the grid, not from the coefficients."""
    iset = oidx.grouped_index_set(d, ds, N)
    fh = _random_fhat(iset, seed)
    fh[0] = 3.0 - 2.0j                                   # the empty set's value must not count
    axis = np.arange(K) / K - 0.5
    x = np.array(list(itertools.product(axis, repeat=d)))
    f = otr.forward(iset, x, fh)
    var = np.mean(np.abs(f - np.mean(f)) ** 2)
    want = np.zeros(iset.n_terms)
    for i in range(1, iset.n_terms):
        fu = np.zeros_like(fh)
        fu[iset.term_slice(i)] = fh[iset.term_slice(i)]
        want[i] = np.mean(np.abs(otr.forward(iset, x, fu)) ** 2) / var
    return rel(osens.sensitivity_indices(iset, fh), want)


def pin_gsi_invariants(seed=42, d=5, ds=3, N=(8, 6, 4)) -> float:
    """The indices of the non-empty terms add up to 1; they do not change when the
    coefficients are scaled or the empty set's coefficient changes; rho(empty set) = 0."""
    iset = oidx.grouped_index_set(d, ds, N)
    fh = _random_fhat(iset, seed)
    rho = osens.sensitivity_indices(iset, fh)
    g = fh * (0.3 - 1.7j)
    g[0] = 11.0
    rho2 = osens.sensitivity_indices(iset, g)
    return max(abs(np.sum(rho[1:]) - 1.0), float(np.max(np.abs(rho2 - rho))), abs(rho[0]))


def pin_active_set_rule() -> float:
    """eq. activeset on a worked example (d = 3, d_s = 2): terms empty, {0}, {1}, {2},
    {0,1}, {0,2}, {1,2}; thresholds 0.1 (order 1) and 0.05 (order 2); an index equal to its
    threshold is not above it."""
    iset = oidx.grouped_index_set(3, 2, (4, 4))
    rho = np.array([0.0, 0.5, 0.09, 0.1, 0.2, 0.05, 0.06])
    got = osens.active_set(iset, rho, (0.1, 0.05))
    return float(np.sum(got != np.array([1, 1, 0, 0, 1, 0, 1])))


def pin_subset_transform(seed=43, d=4, ds=3, N=(8, 6, 4), M=40) -> float:
    """The transform on I_N(U) for a subset U equals the full transform with the dropped
    groups' coefficients zero, and its adjoint is the full adjoint restricted to U.  The
    empty set's flag is 0 here: the empty set stays in every index set whatever its flag."""
    full = oidx.grouped_index_set(d, ds, N)
    keep = [0, 1, 0, 1, 1, 0, 0, 1, 1, 1, 0, 1, 0, 1, 0]
    sub = oidx.grouped_index_set(d, ds, N, keep=keep)
    g = np.random.default_rng(seed)
    x = g.random((M, d)) - 0.5
    y = g.standard_normal(M) + 1j * g.standard_normal(M)
    fs = _random_fhat(sub, seed + 1)
    ff = np.zeros(full.n_coeffs, complex)
    rows = []
    for i, u in enumerate(sub.terms):
        j = full.terms.index(u)
        ff[full.term_slice(j)] = fs[sub.term_slice(i)]
        rows.append(np.arange(full.offsets[j], full.offsets[j + 1]))
    rows = np.concatenate(rows)
    has_empty = 0.0 if sub.terms and sub.terms[0] == () else 1.0   # U* contains the empty set (eq. activeset)
    return max(rel(otr.forward(sub, x, fs), otr.forward(full, x, ff)),
               rel(otr.adjoint(sub, x, y), otr.adjoint(full, x, y)[rows]), has_empty)


# ---------------------------------------------------------------- the paper's test function
def pin_bspline_closed_form(j=4, K=4000, pts=57) -> float:
    """The closed-form B-spline pieces of the test function (workloads) against their Fourier
    series as printed (Sec. 4, after eq. testfun), truncated at |k| < K; B2 against 2 sqrt(3)|x|."""
    import workloads as W
    x = np.linspace(-0.5, 0.5, pts, endpoint=False) + 0.0041
    if j == 2:
        return float(np.max(np.abs(W.bspline(x, 2) - 2.0 * math.sqrt(3.0) * np.abs(x))))
    k = np.arange(-K, K)
    ser = np.exp(2j * np.pi * np.outer(x, k)) @ W.bspline_coeff(k, j)
    return float(np.max(np.abs(ser.real - W.bspline(x, j))))


def pin_bspline_unit_norm(K=200000) -> float:
    """The printed normalisation constants give ||B_j|| = 1 (Parseval, |k| <= K)."""
    import workloads as W
    k = np.arange(-K, K + 1)
    return max(abs(float(np.sum(W.bspline_coeff(k, j) ** 2)) - 1.0) for j in (2, 4, 6))


def pin_testfun_anova() -> float:
    """The exact coefficients of the test function: f_empty = 3 c2 c4 c6 (printed), and the
    terms with non-zero coefficients are exactly U* = P({1,3,8}) u P({2,5,6}) u P({4,7,9})
    (1-based, printed): 9 one-, 9 two- and 3 three-dimensional terms."""
    import workloads as W
    iset = oidx.grouped_index_set(9, 3, (6, 4, 4))
    c = W.testfun_coeffs(iset.terms, iset.freqs)
    prod = W.BSPLINE_NORM[2] * W.BSPLINE_NORM[4] * W.BSPLINE_NORM[6]
    err = abs(c[0] - 3.0 * prod)
    groups = [(1, 3, 8), (2, 5, 6), (4, 7, 9)]
    want = set()
    for g in groups:
        for t in range(1, 4):
            want.update(tuple(i - 1 for i in s) for s in itertools.combinations(g, t))
    got = {u for i, u in enumerate(iset.terms) if u and np.any(np.abs(c[iset.term_slice(i)]) > 0)}
    counts = [sum(1 for u in got if len(u) == t) for t in (1, 2, 3)]
    return float(err + len(got ^ want) + (counts != [9, 9, 3]))


def pin_l2_error_quadrature(seed=44, N=8, K=20000) -> float:
    """eq. L2error by Parseval against direct quadrature of |B4 - S B4|^2 on a fine grid
    (d = 1, a random trigonometric polynomial S on I_N)."""
    import workloads as W
    iset = oidx.grouped_index_set(1, 1, (N,))
    g = np.random.default_rng(seed)
    fh = (g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)) * 0.1
    exact = np.concatenate([[W.BSPLINE_NORM[4]], W.bspline_coeff(iset.freqs[1][:, 0], 4)])
    fh += exact
    e = osens.l2_error(iset, fh, exact, 1.0)
    x = (np.arange(K) / K - 0.5)[:, None]
    diff = W.bspline(x[:, 0], 4) - otr.forward(iset, x, fh)
    want = math.sqrt(float(np.mean(np.abs(diff) ** 2)))
    return abs(e - want) / want


def pin_testfun_gsi_closed_form() -> float:
    """Sensitivity indices of the test function's exact coefficients (on a wide index set,
    N = 512/64/24) against the variances of its ANOVA terms in closed form (printed terms
    eq. onedimterm, eq. twodimterm, eq. threedimterm): with P = c2 c4 c6 and c_k the
    constant of the B-spline on coordinate k, term u inside a product has variance
    (P / prod_{k in u} c_k)^2 prod_{k in u} (1 - c_k^2), and the function 3 (1 - P^2)."""
    import workloads as W
    iset = oidx.grouped_index_set(9, 3, (512, 64, 24))
    rho = osens.sensitivity_indices(iset, W.testfun_coeffs(iset.terms, iset.freqs))
    P = W.BSPLINE_NORM[2] * W.BSPLINE_NORM[4] * W.BSPLINE_NORM[6]
    ck = {k: W.BSPLINE_NORM[j] for g in W.TESTFUN_GROUPS for k, j in zip(g, W.TESTFUN_ORDERS)}
    want = np.zeros(iset.n_terms)
    for i, u in enumerate(iset.terms):
        if u and any(set(u) <= set(g) for g in W.TESTFUN_GROUPS):
            want[i] = (P / np.prod([ck[k] for k in u])) ** 2 * np.prod([1.0 - ck[k] ** 2 for k in u])
    return float(np.max(np.abs(rho - want / (3.0 * (1.0 - P * P)))))


# ---------------------------------------------------------------- cosine basis (Sec. 5)
def _cos_full_frequencies(d, ds, N):
    """k in N_0^d of the cosine groups, from the ordering rule (independent enumeration)."""
    K = []
    for t in range(ds + 1):
        for u in itertools.combinations(range(d), t):
            band = list(range(1, N[t - 1])) if t else []
            for ell in itertools.product(band, repeat=t):
                k = [0] * d
                for c, v in zip(u, ell):
                    k[c] = v
                K.append(k)
    return np.array(K, dtype=np.int64)


def pin_cos_dense_matrix(seed=51, d=4, ds=3, N=(6, 4, 4), M=31) -> float:
    """Cosine forward, adjoint and dense matrix against the basis of Sec. 5 evaluated node by
    node and frequency by frequency with math.cos (k in N_0^d from the ordering rule)."""
    g = np.random.default_rng(seed)
    iset = ocos.cosine_index_set(d, ds, N)
    x = g.random((M, d))
    K = _cos_full_frequencies(d, ds, N)
    if not np.array_equal(K, iset.full_frequencies()):
        return 1.0
    A = np.array([[math.prod(math.sqrt(2.0) * math.cos(math.pi * kj * xj) if kj else 1.0
                             for kj, xj in zip(k, xm)) for k in K] for xm in x])
    fh = g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)
    y = g.standard_normal(M) + 1j * g.standard_normal(M)
    return max(rel(ocos.forward(iset, x, fh), A @ fh), rel(ocos.adjoint(iset, x, y), A.T @ y),
               rel(ocos.dense_matrix(iset, x), A))


def pin_cos_dct(d=3, N=6) -> float:
    """U = P(D), nodes on the tensor grid x_m = (m + 1/2) / N: the groups {1..N-1}^{|u|} over
    all u partition {0..N-1}^d, and the grouped cosine transform is a d-dimensional DCT:
    forward = scipy.fft.dctn(type 3) of fhat_k prod_{k_j > 0} 2^{-1/2}; adjoint = dctn(type 2)
    of the samples times prod_j (1/2 if k_j = 0 else 2^{-1/2})."""
    import scipy.fft
    iset = ocos.cosine_index_set(d, d, [N] * d)
    grid = np.array(list(itertools.product(range(N), repeat=d)))
    x = (grid + 0.5) / N
    K = iset.full_frequencies()
    if len(K) != N ** d:
        return 1.0
    g = np.random.default_rng(52)
    fh = g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)
    Cc = np.zeros((N,) * d, dtype=complex)
    for val, k in zip(fh, K):
        Cc[tuple(k)] = val * 2.0 ** (-0.5 * np.count_nonzero(k))
    ref = scipy.fft.dctn(Cc.real, type=3) + 1j * scipy.fft.dctn(Cc.imag, type=3)
    e1 = rel(ocos.forward(iset, x, fh), np.array([ref[tuple(m)] for m in grid]))
    y = g.standard_normal(len(grid)) + 1j * g.standard_normal(len(grid))
    Y = np.zeros((N,) * d, dtype=complex)
    for val, m in zip(y, grid):
        Y[tuple(m)] = val
    D = scipy.fft.dctn(Y.real, type=2) + 1j * scipy.fft.dctn(Y.imag, type=2)
    want = np.array([D[tuple(k)] * np.prod([0.5 if kj == 0 else 2.0 ** -0.5 for kj in k]) for k in K])
    return max(e1, rel(ocos.adjoint(iset, x, y), want))


def pin_cos_orthogonality(d=3, ds=2, N=(8, 4), M=9) -> float:
    """On the full tensor grid of M > N - 1 half-period points per axis the grouped cosine
    matrix has orthogonal columns of squared norm M^d (discrete cosine orthogonality,
    sum_m cos(pi j (2m + 1) / (2M)) = 0 for 0 < j < 2M)."""
    iset = ocos.cosine_index_set(d, ds, N)
    x = (np.array(list(itertools.product(range(M), repeat=d))) + 0.5) / M
    A = ocos.dense_matrix(iset, x)
    G = A.T @ A
    return float(np.abs(G - M ** d * np.eye(iset.n_coeffs)).max() / M ** d)


def pin_cos_adjoint_identity(seed=53, d=5, ds=3, N=(10, 6, 4), M=40) -> float:
    g = np.random.default_rng(seed)
    iset = ocos.cosine_index_set(d, ds, N)
    x = g.random((M, d))
    fh = g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)
    y = g.standard_normal(M) + 1j * g.standard_normal(M)
    lhs = np.vdot(y, ocos.forward(iset, x, fh))
    rhs = np.vdot(ocos.adjoint(iset, x, y), fh)
    return float(abs(lhs - rhs) / (np.linalg.norm(y) * np.linalg.norm(ocos.forward(iset, x, fh))))


def pin_cos_even_periodic(seed=54, d=3, ds=3, N=(6, 4, 4), M=25) -> float:
    """Each basis function is even and 2-periodic in every coordinate: reflecting a node's
    coordinate (x -> -x) or shifting it by 2 leaves the forward transform unchanged."""
    g = np.random.default_rng(seed)
    iset = ocos.cosine_index_set(d, ds, N)
    x = g.random((M, d))
    fh = g.standard_normal(iset.n_coeffs) + 1j * g.standard_normal(iset.n_coeffs)
    f = ocos.forward(iset, x, fh)
    x2 = x.copy()
    x2[:, 0] = -x2[:, 0]
    x2[:, 1] = x2[:, 1] + 2.0
    x2[:, 2] = 2.0 - x2[:, 2]
    return rel(ocos.forward(iset, x2, fh), f)


PINS = [
    ("printed_counts", pin_printed_counts, {}, 0.0),
    ("ordering", pin_ordering, {}, 0.0),
    ("dense_matrix", pin_dense_matrix, {}, 1e-12),
    ("adjoint_at", pin_adjoint_at, {}, 1e-12),
    ("hypercube_fft_1d", pin_hypercube_fft, dict(d=1, N=8), 1e-12),
    ("hypercube_fft_2d", pin_hypercube_fft, dict(d=2, N=6), 1e-12),
    ("hypercube_fft_3d", pin_hypercube_fft, dict(d=3, N=4), 1e-12),
    ("lattice_orthogonality", pin_lattice_orthogonality, {}, 1e-12),
    ("adjoint_identity", pin_adjoint_identity, {}, 1e-12),
    ("modulation", pin_modulation, {}, 1e-12),
    ("group_isolation", pin_group_isolation, {}, 1e-12),
    ("single_frequency", pin_single_frequency, {}, 1e-12),
    # central differences, h = 1e-5: truncation ~ (2 pi 8 h)^2/6, rounding ~ 1e-16/h
    ("gradient_fd", pin_gradient_fd, {}, 1e-8),
    ("lsqr_dense", pin_lsqr_dense, dict(weighted=False), 1e-9),
    ("lsqr_dense_weighted", pin_lsqr_dense, dict(weighted=True), 1e-9),
    ("lsqr_scipy_1", pin_lsqr_scipy, dict(iters=1), 1e-10),
    ("lsqr_scipy_3", pin_lsqr_scipy, dict(iters=3), 1e-10),
    ("lsqr_scipy_7", pin_lsqr_scipy, dict(iters=7), 1e-10),
    ("lsqr_scipy_15", pin_lsqr_scipy, dict(iters=15), 1e-10),
    ("lsqr_lattice", pin_lsqr_lattice, {}, 1e-12),
    ("prox_soft_threshold", pin_prox_soft_threshold, {}, 1e-13),
    ("prox_minimises", pin_prox_minimises, {}, 1e-9),
    ("prox_zero_threshold", pin_prox_zero_threshold, {}, 0.0),
    ("prox_ridge_link", pin_prox_ridge_link, {}, 1e-12),
    ("fista_kkt", pin_fista_kkt, {}, 1e-12),
    ("fista_zero_above_lambda_max", pin_fista_zero_above_lambda_max, {}, 0.0),
    ("fista_lattice", pin_fista_lattice, {}, 1e-12),
    ("fista_backtracking", pin_fista_backtracking, {}, 1e-12),
    ("fista_first_steps", pin_fista_first_steps, {}, 1e-13),
    ("fista_rate", pin_fista_rate, {}, 0.0),
    ("power_iteration", pin_power_iteration, {}, 1e-6),
    ("gsi_quadrature", pin_gsi_quadrature, {}, 1e-12),
    ("gsi_invariants", pin_gsi_invariants, {}, 1e-13),
    ("active_set_rule", pin_active_set_rule, {}, 0.0),
    ("subset_transform", pin_subset_transform, {}, 1e-12),
    ("bspline_closed_form_2", pin_bspline_closed_form, dict(j=2), 1e-12),
    ("bspline_closed_form_4", pin_bspline_closed_form, dict(j=4), 1e-10),
    ("bspline_closed_form_6", pin_bspline_closed_form, dict(j=6), 1e-12),
    ("bspline_unit_norm", pin_bspline_unit_norm, {}, 1e-12),
    ("testfun_anova", pin_testfun_anova, {}, 1e-15),
    ("l2_error_quadrature", pin_l2_error_quadrature, {}, 1e-10),
    ("testfun_gsi_closed_form", pin_testfun_gsi_closed_form, {}, 1e-5),
    ("cos_dense_matrix", pin_cos_dense_matrix, {}, 1e-12),
    ("cos_dct_1d", pin_cos_dct, dict(d=1, N=8), 1e-12),
    ("cos_dct_2d", pin_cos_dct, dict(d=2, N=6), 1e-12),
    ("cos_dct_3d", pin_cos_dct, dict(d=3, N=4), 1e-12),
    ("cos_orthogonality", pin_cos_orthogonality, {}, 1e-12),
    ("cos_adjoint_identity", pin_cos_adjoint_identity, {}, 1e-12),
    ("cos_even_periodic", pin_cos_even_periodic, {}, 1e-12),
]
