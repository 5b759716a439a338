"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module draws node sets and coefficient vectors and nothing else: it holds none of the
method's arithmetic (no window, no transform, no least squares).  Both the CPU oracle side
and the GPU side receive exactly the arrays produced here.

Draw order for one problem: nodes first, then the real parts of the coefficients, then the
imaginary parts, right-hand sides slowest.  The generator is numpy's PCG64
(``numpy.random.default_rng(seed)``).

Node families follow the paper: jittered equispaced nodes (eq. 3.8 and the variant centred on
zero), Chebyshev nodes (eq. 3.10), logarithmically spaced nodes (Remark 3.6), equispaced
nodes (Section 3.2), uniform random nodes; plus the 2-D polar and spiral trajectories used as
MRI-like test workloads.
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int = 0) -> np.random.Generator:
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- node families (N x d, float64)

def uniform_nodes(g: np.random.Generator, N: int, d: int = 1) -> np.ndarray:
    """x ~ U[-1/2, 1/2)^d, shape (N, d)."""
    return g.uniform(-0.5, 0.5, size=(N, d))


def clustered_nodes(g: np.random.Generator, N: int, d: int, ncluster: int, radius: float,
                    centre: float = 0.1) -> np.ndarray:
    """N - ncluster uniform nodes plus ncluster nodes uniform in the box of half-width `radius`
    (x units) around (centre, ..., centre): a dense spot like the centre of a polar or spiral
    trajectory, which makes some |I(l)| far larger than the mean."""
    x = g.uniform(-0.5, 0.5, size=(N, d))
    x[:ncluster] = centre + g.uniform(-radius, radius, size=(ncluster, d))
    return x


def jittered_nodes(g: np.random.Generator, N: int) -> np.ndarray:
    """x_j = (j - N/2)/N + U(-1/(4N), 1/(4N)), j = 0..N-1 (may leave [-1/2,1/2) at j = 0)."""
    j = np.arange(N, dtype=np.float64)
    return ((j - N / 2) / N + g.uniform(-1.0 / (4 * N), 1.0 / (4 * N), size=N))[:, None]


def jittered_nodes_paper(g: np.random.Generator, N: int) -> np.ndarray:
    """Eq. (3.8): y_j = -1/2 + (j-1)/N + theta/(4N), theta ~ U(0,1), j = 1..N."""
    j = np.arange(1, N + 1, dtype=np.float64)
    return (-0.5 + (j - 1) / N + g.uniform(0.0, 1.0, size=N) / (4 * N))[:, None]


def equispaced_nodes(N: int) -> np.ndarray:
    """x_j = j/N, j = -N/2..N/2-1 (Section 3.2)."""
    j = np.arange(-N // 2, N // 2, dtype=np.float64)
    return (j / N)[:, None]


def chebyshev_nodes(N: int) -> np.ndarray:
    """Eq. (3.10): y_j = cos((2(N-j)+1) pi / (2N)) / 2, j = 1..N."""
    j = np.arange(1, N + 1, dtype=np.float64)
    return (0.5 * np.cos((2 * (N - j) + 1) * np.pi / (2 * N)))[:, None]


def log_nodes(N: int) -> np.ndarray:
    """Remark 3.6: y_j = (6/5)^(j-N), j = 1..N (they lie in (0, 1]; wrapped by the method)."""
    j = np.arange(1, N + 1, dtype=np.float64)
    return ((6.0 / 5.0) ** (j - N))[:, None]


def polar_nodes(nrays: int = 1024, nrad: int = 512) -> np.ndarray:
    """Polar (radial MRI) trajectory: spokes at theta_s = pi s / nrays, radii
    rho_t = (t - (nrad-1)/2) / nrad; the half-sample offset keeps the origin unsampled."""
    s = np.arange(nrays, dtype=np.float64)
    t = np.arange(nrad, dtype=np.float64)
    th = np.pi * s / nrays
    rho = (t - (nrad - 1) / 2.0) / nrad
    x0 = np.outer(np.cos(th), rho).ravel()
    x1 = np.outer(np.sin(th), rho).ravel()
    return np.stack([x0, x1], axis=1)


def spiral_nodes(ninter: int = 32, nsamp: int = 2048, turns: int = 4) -> np.ndarray:
    """Archimedean spiral with `ninter` interleaves: r_p = (p+1/2)/(2 nsamp),
    phi_p = 2 pi turns (p+1/2)/nsamp + 2 pi i/ninter."""
    p = np.arange(nsamp, dtype=np.float64)
    i = np.arange(ninter, dtype=np.float64)
    r = 0.5 * (p + 0.5) / nsamp
    phi = 2 * np.pi * turns * (p + 0.5) / nsamp
    ang = phi[None, :] + 2 * np.pi * i[:, None] / ninter
    x0 = (r[None, :] * np.cos(ang)).ravel()
    x1 = (r[None, :] * np.sin(ang)).ravel()
    return np.stack([x0, x1], axis=1)


# ---------------------------------------------------------------- coefficients

def complex_normal(g: np.random.Generator, shape) -> np.ndarray:
    """Complex array with i.i.d. N(0,1) real and imaginary parts (real parts drawn first)."""
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return re + 1j * im


def round_to(a: np.ndarray, precision: str) -> np.ndarray:
    """Round a complex128 array once to the given storage precision and return it as
    complex128 again, so both sides consume identical values."""
    if precision == "f32":
        return a.astype(np.complex64).astype(np.complex128)
    return np.asarray(a, dtype=np.complex128)


# ---------------------------------------------------------------- named workloads

def _smooth7(n: int) -> bool:
    for p in (2, 3, 5, 7):
        while n % p == 0:
            n //= p
    return n == 1


def batched_sizes(g: np.random.Generator, nprob: int = 256, lo: int = 1024, hi: int = 16384):
    """Uneven batch: M_i log-uniform in [lo, hi] rounded to the nearest even M_i whose
    oversampled length 2 M_i is 7-smooth; N_i = round(r_i M_i), r_i ~ U[1.5, 4]."""
    raw = np.exp(g.uniform(math.log(lo), math.log(hi), size=nprob))
    r = g.uniform(1.5, 4.0, size=nprob)
    Ms = []
    for v in raw:
        best = None
        for delta in range(0, 4096, 2):
            for cand in (int(round(v / 2)) * 2 + delta, int(round(v / 2)) * 2 - delta):
                if cand >= 2 and _smooth7(2 * cand):
                    best = cand
                    break
            if best is not None:
                break
        Ms.append(best)
    Ms = np.array(Ms, dtype=np.int64)
    Ns = np.maximum(1, np.round(r * Ms)).astype(np.int64)
    return Ms, Ns


CONFIGS = {
    # 1-D overdetermined iNFFT, uniform random nodes
    "c1": dict(d=1, M=(256,), N=512, sigma=2.0, m=4, nodes="uniform", rho=1e-8, rhs=1),
    # 1-D jittered nodes, the large single-GPU workload
    "c2": dict(d=1, M=(65536,), N=131072, sigma=2.0, m=6, nodes="jittered", rho=1e-12, rhs=1),
    # 2-D polar trajectory
    "c3": dict(d=2, M=(512, 512), N=524288, sigma=2.0, m=4, nodes="polar", rho=1e-8, rhs=1),
    # 2-D spiral trajectory, 16 right-hand sides
    # batched uneven 1-D problems (M_i, N_i from batched_sizes), 8 right-hand sides each
    "c4": dict(d=1, nprob=256, lo=1024, hi=16384, sigma=2.0, m=4, nodes="uniform", rho=1e-8, rhs=8),
    "c5": dict(d=2, M=(256, 256), N=65536, sigma=2.0, m=4, nodes="spiral", rho=1e-8, rhs=16),
    # ansatz 1 (underdetermined, M = 4N): Example 3.14's largest first-experiment case, Dirichlet
    # kernel, sigma 2, jittered nodes (3.8); then the same shape at GPU scale
    "a1": dict(d=1, M=(16384,), N=4096, sigma=2.0, m=4, nodes="jittered_paper", rho=0.0, rhs=1,
               kernel="dirichlet"),
    "a1_large": dict(d=1, M=(1048576,), N=262144, sigma=2.0, m=4, nodes="jittered_paper", rho=0.0, rhs=1,
                     kernel="dirichlet"),
}


def make_nodes(cfg: dict, g: np.random.Generator) -> np.ndarray:
    kind, N, d = cfg["nodes"], cfg["N"], cfg["d"]
    if kind == "uniform":
        return uniform_nodes(g, N, d)
    if kind == "jittered":
        return jittered_nodes(g, N)
    if kind == "jittered_paper":
        return jittered_nodes_paper(g, N)
    if kind == "equispaced":
        return equispaced_nodes(N)
    if kind == "chebyshev":
        return chebyshev_nodes(N)
    if kind == "polar":
        nrad = 512 if N == 524288 else int(round(math.sqrt(N / 2)))
        return polar_nodes(N // nrad, nrad)
    if kind == "spiral":
        return spiral_nodes(32, N // 32, 4)
    raise ValueError(kind)


def make_problem(cfg: dict, seed: int = 0, rhs: int | None = None):
    """Nodes (N, d) then coefficients (R, *M) complex128, drawn in that order."""
    g = rng(seed)
    x = make_nodes(cfg, g)
    R = cfg.get("rhs", 1) if rhs is None else rhs
    fhat = complex_normal(g, (R,) + tuple(cfg["M"]))
    return x, fhat


def make_batch(cfg: dict, seed: int = 0, rhs: int | None = None):
    """Uneven batch: sizes first (M_i, then r_i), then per problem its nodes and its R
    right-hand sides of coefficients.  Returns Ms, Ns, list of x_i (N_i, 1), list of fhat_i (R, M_i)."""
    g = rng(seed)
    Ms, Ns = batched_sizes(g, cfg["nprob"], cfg["lo"], cfg["hi"])
    R = cfg.get("rhs", 1) if rhs is None else rhs
    xs, fhs = [], []
    for M, N in zip(Ms, Ns):
        xs.append(uniform_nodes(g, int(N), 1))
        fhs.append(complex_normal(g, (R, int(M))))
    return Ms, Ns, xs, fhs
