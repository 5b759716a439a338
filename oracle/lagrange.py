"""Lagrange-interpolation inverse for M = N (Section 3.1), evaluated directly in O(N^2)
(oracle; test infrastructure only -- used to pin the direct sums).

For nonequispaced nodes y_j and auxiliary nodes x_l (disjoint from the y_j),
    a_l = prod_n sin(pi (x_l - y_n)),   b_j = prod_{n != j} 1 / sin(pi (y_j - y_n))      (3.4)
    g_l = f(x_l) = a_l sum_j f_j b_j (cot(pi (x_l - y_j)) - i)                            (3.5)
and with equispaced x_l the coefficients follow from one inverse DFT (Algorithm 3.3, step 6):
    f_check_k = (1/N) sum_l g_l e^{-2 pi i k x_l}.
Products of many sines over- or underflow, so |a_l| |b_j| is formed as exp(ln|a_l| + ln|b_j|)
with the signs taken from the sines themselves (the logarithmic form of Algorithm 3.3, steps
1-3, without the fast summation; the stabilising shift s of Remark 3.2 is not needed because
the sum of the two logarithms is formed before exponentiating).
"""
from __future__ import annotations

import numpy as np

from .direct import centred


def aux_nodes(N: int) -> np.ndarray:
    """Equispaced x_l = -1/2 + (l-1)/N + 1/(2N), l = 1..N (half-way between grid points, so
    they avoid jittered nodes of the form (3.8))."""
    l = np.arange(1, N + 1, dtype=np.float64)
    return -0.5 + (l - 1) / N + 1.0 / (2 * N)


def lagrange_values(y, f, x) -> np.ndarray:
    """g_l of (3.5) for all auxiliary nodes x_l."""
    y = np.asarray(y, dtype=np.float64).ravel()
    x = np.asarray(x, dtype=np.float64).ravel()
    f = np.asarray(f, dtype=np.complex128).ravel()
    Sxy = np.sin(np.pi * (x[:, None] - y[None, :]))          # (N_x, N)
    Syy = np.sin(np.pi * (y[:, None] - y[None, :]))
    np.fill_diagonal(Syy, 1.0)
    if np.any(Sxy == 0) or np.any(Syy == 0):
        raise ZeroDivisionError("node sets must be disjoint and nodes distinct (Remark 3.1)")
    ln_a = np.sum(np.log(np.abs(Sxy)), axis=1)
    sg_a = np.prod(np.sign(Sxy), axis=1)
    ln_b = -np.sum(np.log(np.abs(Syy)), axis=1)
    sg_b = np.prod(np.sign(Syy), axis=1)
    ab = (sg_a[:, None] * sg_b[None, :]) * np.exp(ln_a[:, None] + ln_b[None, :])
    cot = np.cos(np.pi * (x[:, None] - y[None, :])) / Sxy
    return np.sum(ab * f[None, :] * (cot - 1j), axis=1)


def inverse(y, f) -> np.ndarray:
    """f_check (centred, length N) from samples f at nodes y, Algorithm 3.3 with direct sums."""
    N = len(np.ravel(y))
    x = aux_nodes(N)
    g = lagrange_values(y, f, x)
    k = centred(N)
    E = np.exp(-2j * np.pi * np.outer(k, x))
    return (E @ g) / N
