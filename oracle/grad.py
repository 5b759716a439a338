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
