"""Ansatz 1 of Section 3.2.1 (inverse NFFT, underdetermined case): per-node optimisation of the
columns of B^* (Algorithm 3.10) and the two estimates it feeds (oracle; test infrastructure only).

The Frobenius problem (3.13), min ||A D^* F^* B^* - M I_N||_F over B with the sparsity of the
window matrix, splits by columns (3.18)-(3.19): column j of B^* meets only column j of M I_N, so
each node has its own small least-squares problem

    K = A D^* F^*,  K[h, l] = K(x_h - l/M_sigma)                                   (3.14)-(3.15)
    K_j = the columns l of K with l in I(x_j)                                      (3.16), (3.21)
    b~_j = argmin_b ||K_j b - M e_j||_2 = M (K_j^* K_j)^{-1} K_j^* e_j             (3.22)

and f_check = (1/M) D^* F^* B_opt^* f estimates fhat (approximation (3.12)); the inverse adjoint of
Remark 3.15 uses the same matrix, f_tilde = (1/M) B_opt F D h.

Readings where the paper is silent:
  * unknowns: the members of I(x_j) under the stencil of `nfft` (|u - tau| <= m: 2m taps, 2m+1
    when the node's offset u equals m exactly);
  * b~_j is complex: K is complex for the window kernel, whose k range -M/2..M/2-1 is not
    symmetric (with the Dirichlet kernel of Remark 3.11 K is real and so is b~_j);
  * ridge: argmin ||K_j b - M e_j||^2 + lambda_j ||b||^2 with
    lambda_j = rho trace(K_j^* K_j) / |I(x_j)|  (rho = 0 is (3.22); a rank-deficient K_j then
    gets the minimum-norm solution);
  * the D inside K is the inverse's D of the plan (the window's, or the Dirichlet kernel's);
  * d = 1 only: the section works on the 1-D torus.

Storage: rows[j, tau] = conj(b~_j[tau]) / M on the stencil of node j (zero off I(x_j)), so that
`bopt.apply(x, f, rows, p)` = D^* F^* rows^* f is f_check and `bopt.apply_adjoint(x, h, rows, p)`
is f_tilde.

Two routes to b~_j:
  E  the definition: K assembled entry by entry from (3.15), then the ridge problem by lstsq on
     the stacked matrix [K_j; sqrt(lambda_j) I];
  T  Toeplitz: K^* K = F D (A^* A) D^* F^*, and A^* A is the Toeplitz matrix with symbol
     P(q) = sum_h e^{2 pi i q x_h}, so the band (K^* K)[l, l+d] =: S(l, d) is
         S(l, d) = sum_{|q| < M} P(q) R_d(q) e^{-2 pi i q l / M_sigma},
         R_d(q)  = sum_k D_k D_{k+q} e^{-2 pi i (k+q) d / M_sigma}   (D real),
     each sum taken directly; then the normal equations (S-band Gram + lambda_j I) y = K_j^* e_j.
"""
from __future__ import annotations

import numpy as np

from .bopt import kernel_K_1d
from .direct import centred, phase_matrix
from .nfft import Params, prepare_nodes, tap_offsets


def _check(p: Params):
    if p.d != 1:
        raise ValueError("ansatz 1 is defined for d = 1")


def stencil(x, p: Params):
    """Per node: grid index of each tap (FFT order, (N, 2m+1)) and the membership mask of
    I(x_j) (3.16) under the closed-interval test |u - tau| <= m."""
    _check(p)
    _, l0, u = prepare_nodes(x, p)
    taus = tap_offsets(p)[:, 0]
    idx = np.mod(l0[:, 0][:, None] + taus[None, :], p.Ms[0])
    mem = np.abs(u[:, 0][:, None] - taus[None, :]) <= p.m
    return idx, mem


def K_matrix(x, p: Params) -> np.ndarray:
    """(3.14): K[h, l] = K(x_h - l/M_sigma), l over the grid in FFT order (l mod M_sigma)."""
    _check(p)
    xw, _, _ = prepare_nodes(x, p)
    Ms = p.Ms[0]
    lpos = np.arange(Ms)
    lval = np.where(lpos < Ms // 2, lpos, lpos - Ms)
    K = np.empty((xw.shape[0], Ms), dtype=np.complex128)
    for h in range(xw.shape[0]):
        K[h] = kernel_K_1d(xw[h, 0] - lval / Ms, p, 0)
    return K


def K_columns(x, cols, p: Params) -> np.ndarray:
    """The columns `cols` (grid indices in FFT order) of K, through the factor
    K[:, l] = E diag(D) e^{-2 pi i k l / M_sigma} with E[h, k] = e^{2 pi i k x_h}."""
    _check(p)
    xw, _, _ = prepare_nodes(x, p)
    Ms = p.Ms[0]
    k = centred(p.M[0])
    cols = np.asarray(cols, dtype=np.int64)
    lval = np.where(cols < Ms // 2, cols, cols - Ms)
    W = p.deconv_inv(0)[:, None] * np.exp(-2j * np.pi * np.outer(k, lval) / Ms)
    out = np.empty((xw.shape[0], len(cols)), dtype=np.complex128)
    for s in range(0, xw.shape[0], 1024):
        E = phase_matrix(xw[s:s + 1024, 0], k, +1)
        out[s:s + 1024] = E @ W
    return out


def _ridge(Kj, rhs_col, rho):
    n = Kj.shape[1]
    lam = rho * float(np.real(np.sum(np.abs(Kj) ** 2))) / n
    if lam > 0:
        A = np.vstack([Kj, np.sqrt(lam) * np.eye(n)])
        b = np.concatenate([rhs_col, np.zeros(n)])
    else:
        A, b = Kj, rhs_col
    return np.linalg.lstsq(A, b, rcond=None)[0]


def rows_E(x, p: Params, rho: float, nodes=None, K=None) -> np.ndarray:
    """Route E: y_j = argmin ||K_j y - e_j||^2 + lambda_j ||y||^2, rows[j] = conj(y_j) on I(x_j).
    `nodes` restricts the solve to those nodes (other rows stay zero); `K` may pass the dense K."""
    idx, mem = stencil(x, p)
    N = idx.shape[0]
    rows = np.zeros(idx.shape, dtype=np.complex128)
    js = range(N) if nodes is None else nodes
    for j in js:
        t = np.nonzero(mem[j])[0]
        Kj = K[:, idx[j, t]] if K is not None else K_columns(x, idx[j, t], p)
        e = np.zeros(N, dtype=np.complex128)
        e[j] = 1.0
        rows[j, t] = np.conj(_ridge(Kj, e, rho))
    return rows


def toeplitz_symbol(x, p: Params) -> np.ndarray:
    """P(q) = sum_h e^{2 pi i q x_h} for q = -(M-1) .. M-1 (index q + M - 1): the entries
    (A^* A)[k, k'] = P(k' - k)."""
    _check(p)
    xw, _, _ = prepare_nodes(x, p)
    q = np.arange(-(p.M[0] - 1), p.M[0], dtype=np.int64)
    P = np.zeros(q.shape[0], dtype=np.complex128)
    for s in range(0, xw.shape[0], 1024):
        P += phase_matrix(xw[s:s + 1024, 0], q, +1).sum(axis=0)
    return P


def correlation_R(p: Params) -> np.ndarray:
    """R_d(q) = sum_k D_k D_{k+q} e^{-2 pi i (k+q) d / M_sigma} for d = 0..2m and
    q = -(M-1) .. M-1; shape (2m+1, 2M-1).  Depends only on (M, sigma, m, kernel)."""
    _check(p)
    M, Ms = p.M[0], p.Ms[0]
    D = p.deconv_inv(0)
    k = centred(M)
    R = np.zeros((2 * p.m + 1, 2 * M - 1), dtype=np.complex128)
    for qi, q in enumerate(range(-(M - 1), M)):
        lo = max(-(M // 2), -(M // 2) - q)
        hi = min(M // 2 - 1, M // 2 - 1 - q)
        if lo > hi:
            continue
        kk = np.arange(lo, hi + 1)
        w = D[kk + M // 2] * D[kk + q + M // 2]
        for d in range(2 * p.m + 1):
            R[d, qi] = np.sum(w * np.exp(-2j * np.pi * (kk + q) * d / Ms))
    return R


def gram_band(x, p: Params) -> np.ndarray:
    """S(l, d) = (K^* K)[l, l+d] (indices mod M_sigma) for l in FFT order and d = 0..2m, from
    the Toeplitz factorisation, every sum direct; shape (2m+1, M_sigma)."""
    Ms = p.Ms[0]
    P = toeplitz_symbol(x, p)
    R = correlation_R(p)
    q = np.arange(-(p.M[0] - 1), p.M[0])
    l = np.arange(Ms)
    Ph = np.exp(-2j * np.pi * np.outer(q, l) / Ms)       # (2M-1, M_sigma)
    return (P[None, :] * R) @ Ph


def gram_band_direct(K: np.ndarray, p: Params) -> np.ndarray:
    """The same band read off the dense K^* K (route E)."""
    G = K.conj().T @ K
    Ms = p.Ms[0]
    l = np.arange(Ms)
    return np.stack([G[l, (l + d) % Ms] for d in range(2 * p.m + 1)])


def rows_T(x, p: Params, rho: float, nodes=None, S=None) -> np.ndarray:
    """Route T: normal equations with the Gram read from the band S and the right-hand side
    K_j^* e_j = conj K(x_j - l/M_sigma) from (3.15)."""
    idx, mem = stencil(x, p)
    xw, _, _ = prepare_nodes(x, p)
    Ms = p.Ms[0]
    if S is None:
        S = gram_band(x, p)
    rows = np.zeros(idx.shape, dtype=np.complex128)
    js = range(idx.shape[0]) if nodes is None else nodes
    for j in js:
        t = np.nonzero(mem[j])[0]
        ls = idx[j, t]
        n = len(t)
        G = np.empty((n, n), dtype=np.complex128)
        for a in range(n):
            for b in range(n):
                d = t[b] - t[a]
                G[a, b] = S[d, ls[a]] if d >= 0 else np.conj(S[-d, ls[b]])
        lval = np.where(ls < Ms // 2, ls, ls - Ms)
        r = np.conj(kernel_K_1d(xw[j, 0] - lval / Ms, p, 0))
        lam = rho * float(np.real(np.trace(G))) / n
        rows[j, t] = np.conj(np.linalg.solve(G + lam * np.eye(n), r))
    return rows


def plain_rows(x, p: Params) -> np.ndarray:
    """The window matrix B in the same storage (rows = w~_m(x_j - l/M_sigma) / M), i.e. the
    unoptimised B^* of (3.13) for comparison."""
    from . import kb
    _, _, u = prepare_nodes(x, p)
    taus = tap_offsets(p)[:, 0]
    return kb.window(u[:, 0][:, None] - taus[None, :], p.m, p.b).astype(np.complex128) / p.M[0]


def objective(x, rows, p: Params, K=None) -> float:
    """(3.24): ||A D^* F^* B^* - M I_N||_F for B^* = M rows^* placed on the stencils (dense)."""
    idx, _ = stencil(x, p)
    if K is None:
        K = K_matrix(x, p)
    N = idx.shape[0]
    Bs = np.zeros((p.Ms[0], N), dtype=np.complex128)
    for j in range(N):
        np.add.at(Bs[:, j], idx[j], p.M[0] * np.conj(rows[j]))
    return float(np.linalg.norm(K @ Bs - p.M[0] * np.eye(N)))
