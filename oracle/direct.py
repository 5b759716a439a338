"""Exact trigonometric sums (oracle; test infrastructure only).

  f_j = sum_k fhat_k e^{+2 pi i k.x_j}      (1.1), (2.1)
  h_k = sum_j f_j    e^{-2 pi i k.x_j}      (1.2)
  A   = (e^{2 pi i k.x_j})_{j,k}            (1.3)

k runs over the centred range -M_t/2 .. M_t/2-1 in each dimension, stored ascending
(coefficient index i <-> k = i - M/2), multi-dimensional arrays row-major.

The phase k x is reduced modulo 1 without rounding the product: x is split into a high part
with 26 significant bits and a low remainder, so k * x_hi is exact for |k| < 2^26 and the
fractional part is taken exactly before the small low-order product is added.
"""
from __future__ import annotations

import numpy as np


def centred(M: int) -> np.ndarray:
    return np.arange(-(M // 2), M // 2, dtype=np.int64)


def _split(x):
    x = np.asarray(x, dtype=np.float64)
    c = 134217729.0  # 2^27 + 1 (Veltkamp split)
    t = c * x
    hi = t - (t - x)
    lo = x - hi
    return hi, lo


def phase_matrix(x1: np.ndarray, k: np.ndarray, sign: int = +1) -> np.ndarray:
    """E[j, i] = exp(sign * 2 pi i k_i x_j) for a single coordinate vector x1 (N,)."""
    hi, lo = _split(x1)
    kf = k.astype(np.float64)
    p_hi = np.outer(hi, kf)              # exact products
    p_hi = p_hi - np.floor(p_hi)         # exact fractional part
    ph = p_hi + np.outer(lo, kf)         # small remainder added once
    return np.exp(sign * 2j * np.pi * ph)


def ndft(x: np.ndarray, fhat: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """f = A fhat for x (N, d) and fhat (..., M_0, ..., M_{d-1}); returns (..., N)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    if x.shape[0] == 1 and x.shape[1] != 1 and fhat.ndim == 1:
        x = x.T
    N, d = x.shape
    M = fhat.shape[fhat.ndim - d:]
    lead = fhat.shape[: fhat.ndim - d]
    F = fhat.reshape((-1,) + tuple(M))
    out = np.empty((F.shape[0], N), dtype=np.complex128)
    for s in range(0, N, chunk):
        e = slice(s, min(N, s + chunk))
        if d == 1:
            E0 = phase_matrix(x[e, 0], centred(M[0]), +1)
            out[:, e] = F @ E0.T
        elif d == 2:
            E0 = phase_matrix(x[e, 0], centred(M[0]), +1)   # (n, M0)
            E1 = phase_matrix(x[e, 1], centred(M[1]), +1)   # (n, M1)
            for r in range(F.shape[0]):
                T = E0 @ F[r]                                # (n, M1)
                out[r, e] = np.sum(T * E1, axis=1)
        else:
            raise NotImplementedError("d > 2")
    return out.reshape(lead + (N,))


def ndft_adjoint(x: np.ndarray, f: np.ndarray, M, chunk: int = 2048) -> np.ndarray:
    """h = A^* f for x (N, d), f (..., N); returns (..., M_0, ..., M_{d-1})."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    M = tuple(int(v) for v in np.atleast_1d(M))
    lead = f.shape[:-1]
    Fv = f.reshape(-1, N)
    out = np.zeros((Fv.shape[0],) + M, dtype=np.complex128)
    for s in range(0, N, chunk):
        e = slice(s, min(N, s + chunk))
        if d == 1:
            E0 = phase_matrix(x[e, 0], centred(M[0]), -1)
            out += Fv[:, e] @ E0
        elif d == 2:
            E0 = phase_matrix(x[e, 0], centred(M[0]), -1)
            E1 = phase_matrix(x[e, 1], centred(M[1]), -1)
            for r in range(Fv.shape[0]):
                out[r] += (E0 * Fv[r, e][:, None]).T @ E1
        else:
            raise NotImplementedError("d > 2")
    return out.reshape(lead + M)


def ndft_matrix(x: np.ndarray, M) -> np.ndarray:
    """Dense A in C^{N x prod(M)}, columns ordered like a row-major coefficient array."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    M = tuple(int(v) for v in np.atleast_1d(M))
    if x.shape[1] == 1:
        return phase_matrix(x[:, 0], centred(M[0]), +1)
    E0 = phase_matrix(x[:, 0], centred(M[0]), +1)
    E1 = phase_matrix(x[:, 1], centred(M[1]), +1)
    return (E0[:, :, None] * E1[:, None, :]).reshape(x.shape[0], -1)


def ndft_grad_x(x: np.ndarray, fhat: np.ndarray) -> np.ndarray:
    """Exact d f_j / d x_{j,t} = sum_k 2 pi i k_t fhat_k e^{2 pi i k.x_j}; returns (..., N, d)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    M = fhat.shape[fhat.ndim - d:]
    outs = []
    for t in range(d):
        shape = [1] * d
        shape[t] = M[t]
        kt = centred(M[t]).reshape(shape).astype(np.float64)
        outs.append(ndft(x, fhat * (2j * np.pi * kt)))
    return np.stack(outs, axis=-1)
