"""Gradient of the NFFT f = B(x) F D fhat with respect to the node positions (oracle; test
infrastructure only).

    d f_j / d x_{j,t} = sum_tau g[l0_j + tau] * M_sigma_t w'(u_{j,t} - tau_t) prod_{s != t} w(u_{j,s} - tau_s)

with g = F D fhat and w' the derivative of the window inside its support.  For a real loss L
and the upstream gradient gf = dL/d conj(f) (PyTorch's convention for complex tensors),
    dL/d x_{j,t} = sum_r Re( conj(gf_{r,j}) d f_{r,j} / d x_{j,t} ).
B_opt is held fixed: it is a constant computed once for a node set.
"""
from __future__ import annotations

import numpy as np

from . import kb
from .nfft import Params, prepare_nodes, tap_offsets, trafo_grid


def nfft_dfdx(x, fhat, p: Params) -> np.ndarray:
    """d f / d x, shape (R, N, d) complex."""
    _, l0, u = prepare_nodes(x, p)
    taus = tap_offsets(p)
    N, T = l0.shape[0], taus.shape[0]
    g = trafo_grid(fhat, p).reshape(-1, int(np.prod(p.Ms)))
    idx = np.zeros((N, T), dtype=np.int64)
    W = []
    dW = []
    for t in range(p.d):
        idx = idx * p.Ms[t] + np.mod(l0[:, t][:, None] + taus[None, :, t], p.Ms[t])
        v = u[:, t][:, None] - taus[None, :, t]
        W.append(kb.window(v, p.m, p.b))
        dW.append(p.Ms[t] * kb.window_deriv(v, p.m, p.b))
    out = np.empty((g.shape[0], N, p.d), dtype=np.complex128)
    for t in range(p.d):
        wt = dW[t].copy()
        for s in range(p.d):
            if s != t:
                wt = wt * W[s]
        out[:, :, t] = np.einsum("rnt,nt->rn", g[:, idx], wt)
    return out


def nfft_grad_x(x, fhat, gradf, p: Params) -> np.ndarray:
    """dL/dx (N, d) float64 for upstream gradf (R, N) or (N,)."""
    dfdx = nfft_dfdx(x, fhat, p)
    gf = np.atleast_2d(np.asarray(gradf, dtype=np.complex128))
    return np.sum(np.real(np.conj(gf)[:, :, None] * dfdx), axis=0)


# ------------------------------------------------------------------ gradient through B_opt(x)

def _deriv_pair_matrices(X, p: Params, t: int, power: int):
    """F_t(x_i - x_j) and F_t'(x_i - x_j) for all pairs of coordinate t, where
    F_t(y) = sum_k c_k e^{2 pi i k y} with c = D (power 1) or D^2 (power 2) of the inverse:
    e^{2 pi i k (x_i - x_j)} = e^{2 pi i k x_i} conj(e^{2 pi i k x_j}) gives E diag(c) E^*."""
    from .direct import centred, phase_matrix
    k = centred(p.M[t]).astype(np.float64)
    c = p.deconv_inv(t) ** power
    E = phase_matrix(np.asarray(X[:, t], dtype=np.float64).ravel(), centred(p.M[t]), +1)
    F = (E * c[None, :]) @ E.conj().T
    dF = (E * (2j * np.pi * k * c)[None, :]) @ E.conj().T
    return F, dF


def _kernel_and_deriv(Y, p: Params):
    """K(y) and its partial derivatives dK/dy_t for rows of Y (x units), K of the inverse."""
    from .direct import centred, phase_matrix
    n = Y.shape[0]
    parts, dparts = [], []
    for t in range(p.d):
        k = centred(p.M[t]).astype(np.float64)
        c = p.deconv_inv(t)
        y = Y[:, t] - np.floor(Y[:, t] + 0.5)
        E = phase_matrix(y, centred(p.M[t]), +1)
        parts.append(E @ c)
        dparts.append(E @ (2j * np.pi * k * c))
    K = np.ones(n, dtype=np.complex128)
    for t in range(p.d):
        K = K * parts[t]
    dK = []
    for t in range(p.d):
        v = dparts[t].copy()
        for s in range(p.d):
            if s != t:
                v = v * parts[s]
        dK.append(v)
    return K, dK


def bopt_grad_x(x, f, gfc, p: Params, rho: float) -> np.ndarray:
    """dL/dx (N, d) through B_opt(x) for fcheck = D^* F^* B_opt(x)^* f (3.32) and a real loss L with
    upstream gradient gfc (R, *M) (PyTorch's convention), f held fixed.  Per grid index l,
    (G + lambda I) b = r (Algorithm 3.17 with the ridge; membership I(l) is piecewise constant in x
    and has no derivative), so with bdot = dL/d conj(b) and a = (G + lambda I)^{-1} bdot,
        dL = Re a^* (dr - dG b),
    where only row and column k of G and entry k of r move with x_k.  With the upstream grid
    gradient gdot = F D gfc, bdot_j = sum_r conj(gdot_{r,l}) f_{r,j}."""
    from .bopt import Members, gram_system, grid_multi_index
    from .nfft import trafo_grid
    xw, _, _ = prepare_nodes(x, p)
    f = np.atleast_2d(np.asarray(f, dtype=np.complex128))
    gd = trafo_grid(gfc, p, inverse=True).reshape(f.shape[0], -1)
    mem = Members(x, p)
    scale = float(np.prod(p.Ms))
    out = np.zeros((xw.shape[0], p.d))
    for l in range(mem.G):
        js, _, _ = mem.of(l)
        n = len(js)
        if n == 0:
            continue
        G, r = gram_system(x, l, js, p)
        lam = rho * np.real(np.trace(G)) / n
        A = G + lam * np.eye(n)
        b = np.linalg.solve(A, r)
        bdot = np.sum(np.conj(gd[:, l])[:, None] * f[:, js], axis=0)
        a = np.linalg.solve(A, bdot)
        X = xw[js]
        lv = grid_multi_index(l, p) / np.array(p.Ms, dtype=np.float64)
        _, dK = _kernel_and_deriv(lv[None, :] - X, p)
        Fq = [_deriv_pair_matrices(X, p, t, 2) for t in range(p.d)]
        for t in range(p.d):
            dQ = scale * Fq[t][1]
            for s in range(p.d):
                if s != t:
                    dQ = dQ * Fq[s][0]
            # dQ[i, j] = scale * d/dy_t Q(y) at y = x_i - x_j
            dr = -np.conj(dK[t])                       # d r_k / d x_{k,t}
            term_r = np.conj(a) * dr
            term_row = -np.conj(a) * (dQ @ b)           # row k of dG: d/dx_k Q(x_k - x_j)
            term_col = b * (np.conj(a) @ dQ)            # column k: -d/dx_k Q(x_i - x_k), with the sign of -dG b
            out[js, t] += np.real(term_r + term_row + term_col)
    return out
