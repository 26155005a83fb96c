"""Seeded synthetic inputs shared by the oracle's tests, the GPU tests and the benchmark.

This module holds no arithmetic of the grouped transform or of the solvers: it only
draws nodes, coefficients, samples and noise, and describes the five workload shapes
(dimension, superposition threshold, bandwidths, node counts, batch sizes).  Every
array is generated in float64 and, for single-precision runs, rounded to float32 so
that both sides of a parity test receive exactly the same bits.

Seeding: ``numpy.random.SeedSequence(201010199)`` with a spawn key
``(workload, purpose)``; generator PCG64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

ROOT_SEED = 201010199

# purposes (second component of the spawn key)
P_NODES, P_COEFFS, P_SAMPLES, P_NOISE, P_SIZES, P_TERMS, P_GRAD = range(7)


def rng(workload: int, purpose: int, extra: int = 0) -> np.random.Generator:
    """Independent PCG64 stream for (workload, purpose, extra)."""
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(int(workload), int(purpose), int(extra)))
    return np.random.Generator(np.random.PCG64(ss))


def real_dtype(precision: str):
    return {"f32": np.float32, "f64": np.float64}[precision]


def complex_dtype(precision: str):
    return {"f32": np.complex64, "f64": np.complex128}[precision]


def uniform_nodes(g: np.random.Generator, M: int, d: int, precision: str = "f64") -> np.ndarray:
    """M x d nodes iid uniform on [-1/2, 1/2)^d (torus representatives), row-major.

    Drawn in float64, then rounded to the run's precision.  Rounding to float32 can
    produce exactly +1/2 from a value just below it; such entries are mapped to -1/2,
    the same point of the torus.
    """
    x = g.random((M, d)) - 0.5
    x = x.astype(real_dtype(precision))
    x[x >= 0.5] = -0.5
    return np.ascontiguousarray(x)


def unit_cube_nodes(g: np.random.Generator, M: int, d: int, precision: str = "f64") -> np.ndarray:
    """M x d nodes iid uniform on [0, 1)^d (the domain of the cosine basis), row-major; drawn
    in float64 and rounded to the run's precision (a value that rounds up to 1 stays 1,
    which is inside the closed cube)."""
    x = g.random((M, d)).astype(real_dtype(precision))
    return np.ascontiguousarray(x)


def complex_normal(g: np.random.Generator, shape, precision: str = "f64") -> np.ndarray:
    """Circularly symmetric complex normal: real and imaginary parts iid N(0, 1/2)."""
    z = (g.standard_normal(shape) + 1j * g.standard_normal(shape)) * math.sqrt(0.5)
    return z.astype(complex_dtype(precision))


def bspline2(x: np.ndarray) -> np.ndarray:
    """Periodised order-2 B-spline piece of the paper's test function (Sec. 4, eq. testfun).

    Its Fourier series c2 * sum_k sinc^2(pi k / 2) cos(pi k) e^{2 pi i k x} sums to
    2*sqrt(3)*|x| on [-1/2, 1/2): mean c2 = sqrt(3)/2 and unit L2 norm.
    """
    return 2.0 * math.sqrt(3.0) * np.abs(x)


# ---------------------------------------------------------------- the paper's test function
# f(x) = B2(x_1) B4(x_3) B6(x_8) + B2(x_2) B4(x_5) B6(x_6) + B2(x_4) B4(x_7) B6(x_9) on T^9
# (Sec. 4, eq. testfun; 0-based coordinates below), with B_j the periodised B-spline pieces
# whose Fourier coefficients are c_j sinc^j(pi k / j) cos(pi k) and unit L2 norm.  This is
# the target's definition (samples and exact coefficients for error reports), not a step of
# the method.
TESTFUN_GROUPS = ((0, 2, 7), (1, 4, 5), (3, 6, 8))     # coordinates of B2, B4, B6 in each product
TESTFUN_ORDERS = (2, 4, 6)
BSPLINE_NORM = {2: math.sqrt(3.0 / 4.0), 4: math.sqrt(315.0 / 604.0), 6: math.sqrt(277200.0 / 655177.0)}


def bspline(x: np.ndarray, j: int) -> np.ndarray:
    """B_j(x) in closed form: c_j times the cardinal B-spline of order j with knot spacing 1/j
    and unit integral, centred at 1/2 and taken 1-periodic (x in [-1/2, 1/2))."""
    x = np.asarray(x, dtype=np.float64)
    t = np.where(x < 0.0, x + 0.5, x - 0.5)              # distance from the centre 1/2, periodised
    s = j * t + j / 2.0                                  # argument of the order-j spline on [0, j]
    acc = np.zeros_like(s)
    for i in range(j + 1):
        acc += (-1) ** i * math.comb(j, i) * np.maximum(s - i, 0.0) ** (j - 1)
    return BSPLINE_NORM[j] * j * acc / math.factorial(j - 1)


def bspline_coeff(k: np.ndarray, j: int) -> np.ndarray:
    """Fourier coefficient c_j sinc^j(pi k / j) cos(pi k) of B_j (k integer)."""
    k = np.asarray(k, dtype=np.float64)
    a = np.pi * k / j
    sinc = np.where(k == 0, 1.0, np.sin(a) / np.where(k == 0, 1.0, a))
    return BSPLINE_NORM[j] * sinc ** j * np.cos(np.pi * k)


def testfun(x: np.ndarray) -> np.ndarray:
    """The test function at nodes x (M x 9)."""
    x = np.asarray(x, dtype=np.float64)
    f = np.zeros(x.shape[0])
    for g in TESTFUN_GROUPS:
        p = np.ones(x.shape[0])
        for c, j in zip(g, TESTFUN_ORDERS):
            p *= bspline(x[:, c], j)
        f += p
    return f


def testfun_coeffs(terms, freqs) -> np.ndarray:
    """Exact Fourier coefficients of the test function on a grouped index set given as its
    terms (coordinate tuples) and each term's frequencies (rows of k restricted to u): a
    product touches term u when u lies in its coordinates, with the other factors at k = 0."""
    out = []
    for u, ell in zip(terms, freqs):
        ell = np.asarray(ell).reshape(-1, len(u)) if u else np.zeros((1, 0))
        v = np.zeros(ell.shape[0])
        for g in TESTFUN_GROUPS:
            if not set(u) <= set(g):
                continue
            p = np.ones(ell.shape[0])
            for c, j in zip(g, TESTFUN_ORDERS):
                p = p * (bspline_coeff(ell[:, u.index(c)], j) if c in u else BSPLINE_NORM[j])
            v += p
        out.append(v)
    return np.concatenate(out).astype(np.complex128)


def testfun_norm2() -> float:
    """||f||^2: three products of unit norm, and six cross products of disjoint coordinates
    equal to the product of their means (c2 c4 c6)^2."""
    m = BSPLINE_NORM[2] * BSPLINE_NORM[4] * BSPLINE_NORM[6]
    return 3.0 + 6.0 * m * m


@dataclass
class Workload:
    """One synthetic workload: sizes plus its generated inputs."""
    name: str
    d: int
    ds: int
    N: Tuple[int, ...]           # bandwidth per order |u| = 1..ds
    M: int                       # nodes (total over datasets when ragged)
    R: int = 1                   # batch: lambda values / right-hand sides / datasets
    m: int = 0                   # window half-width (0 = library default)
    sigma: float = 2.0
    precision: str = "f64"
    sizes: Optional[List[int]] = None   # ragged dataset sizes
    lambdas: Optional[np.ndarray] = None
    iters: int = 0
    extra: Dict = field(default_factory=dict)


# The five workloads (sizes from the task's configuration list).
def config_shapes() -> Dict[int, dict]:
    return {
        1: dict(name="fp64-lsqr-d6", d=6, ds=2, N=(16, 8), M=2000, R=1, precision="f64", iters=30),
        2: dict(name="trafo-d10", d=10, ds=2, N=(64, 16), M=50000, R=1, m=6, sigma=2.0),
        3: dict(name="batched-lsqr-d20", d=20, ds=3, N=(32, 12, 6), M=500000, R=16, precision="f32"),
        4: dict(name="batched-fista-d12", d=12, ds=2, N=(48, 16), M=200000, R=8, precision="f32", iters=200),
        5: dict(name="autograd-ragged-d8", d=8, ds=2, N=(32, 10), M=0, R=64, precision="f32"),
    }


def trafo_inputs(workload: int, d: int, ds: int, M: int, n_coeffs: int, R: int = 1,
                 precision: str = "f64"):
    """Nodes, coefficients (R x |I|) and samples (R x M) for a transform-only run."""
    x = uniform_nodes(rng(workload, P_NODES), M, d, precision)
    fhat = complex_normal(rng(workload, P_COEFFS), (R, n_coeffs), precision)
    y = complex_normal(rng(workload, P_SAMPLES), (R, M), precision)
    return x, fhat, y


def ragged_sizes(workload: int, B: int, lo: int, hi: int) -> List[int]:
    """Dataset sizes uniform in [lo, hi] (inclusive), seeded."""
    g = rng(workload, P_SIZES)
    return [int(v) for v in g.integers(lo, hi + 1, size=B)]


def add_noise(g: np.random.Generator, f: np.ndarray, rel: float) -> np.ndarray:
    """f + eta with eta complex normal of standard deviation rel * RMS(f) (real noise for real f)."""
    rms = float(np.sqrt(np.mean(np.abs(f) ** 2)))
    if np.iscomplexobj(f):
        eta = (g.standard_normal(f.shape) + 1j * g.standard_normal(f.shape)) * math.sqrt(0.5)
    else:
        eta = g.standard_normal(f.shape)
    return f + rel * rms * eta


def sparse_trig_target(workload: int, x: np.ndarray, N: Sequence[int], n_terms: int = 8):
    """Target made of `n_terms` random low-order trigonometric monomials.

    Each monomial picks an order |u| uniform in {1..len(N)}, a coordinate set u of that
    size, a frequency vector l with entries in I_N minus {0} (N = N[|u|-1]) and a CN(0,1)
    amplitude a; the target is sum_p a_p exp(2 pi i <l_p, x_{u_p}>).  Returns the samples
    and the list of (u, l, a) so that callers can state the exact coefficients.
    """
    g = rng(workload, P_TERMS)
    M, d = x.shape
    xs = x.astype(np.float64)
    out = np.zeros(M, dtype=np.complex128)
    picks = []
    for _ in range(n_terms):
        t = int(g.integers(1, len(N) + 1))
        u = tuple(sorted(int(c) for c in g.choice(d, size=t, replace=False)))
        Nt = N[t - 1]
        nz = [k for k in range(-Nt // 2, Nt // 2) if k != 0]
        ell = tuple(int(nz[int(g.integers(0, len(nz)))]) for _ in range(t))
        a = complex(g.standard_normal() + 1j * g.standard_normal()) * math.sqrt(0.5)
        ph = np.zeros(M)
        for c, l in zip(u, ell):
            ph += l * xs[:, c]
        out += a * np.exp(2j * np.pi * ph)
        picks.append((u, ell, a))
    return out, picks


def bspline_target(x: np.ndarray, singles=(0, 1, 2), pairs=((3, 4), (5, 6))) -> np.ndarray:
    """Sum of centred B2 pieces: 3 one-dimensional and 2 two-dimensional ANOVA terms.

    f(x) = sum_{i in singles} (B2(x_i) - c2) + sum_{(i,j) in pairs} (B2(x_i) - c2)(B2(x_j) - c2),
    c2 = sqrt(3)/2, so exactly five ANOVA terms are non-zero.
    """
    c2 = math.sqrt(3.0) / 2.0
    xs = x.astype(np.float64)
    f = np.zeros(x.shape[0])
    for i in singles:
        f += bspline2(xs[:, i]) - c2
    for i, j in pairs:
        f += (bspline2(xs[:, i]) - c2) * (bspline2(xs[:, j]) - c2)
    return f
