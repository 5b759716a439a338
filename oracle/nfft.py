"""FP64 NFFT and adjoint NFFT, exactly as the three factors of Section 2 (oracle; test
infrastructure only).

  D = diag(1/(M_sigma w_hat(k)))                          (2.4)
  F = (e^{2 pi i k l / M_sigma})_{l,k}                    (2.5)  (unnormalised, +i)
  B = (w~_m(x_j - l/M_sigma))_{j,l}                       (2.6)
  NFFT       f   = B F D fhat                              (Section 2.1)
  adjoint    h~  = D^* F^* B^* f                           (2.8)

d-dimensional inputs use the tensor product of the 1-D factors.  The grid index l (centred,
-M_sigma/2 .. M_sigma/2-1) is stored at position l mod M_sigma (FFT order).

Stencil.  Per node and dimension: wrap x to [-1/2, 1/2) by x - floor(x + 1/2), t = x M_sigma,
l0 = ceil(t - m), u = t - l0; taps l = l0 + tau, tau = 0..2m, with grid-unit window argument
u - tau; a tap is in the support when |u - tau| <= m (closed interval, (3.16)/(3.29)).  The
same float64 operation order defines the sparsity pattern of B and B_opt everywhere.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import kb
from .direct import centred


class Params:
    """kernel: what the inverse (Algorithm 3.17 and the modified adjoint (3.32)) uses as D:
    "window" the NFFT's D, or "dirichlet" (Remark 3.19): w_hat(k) = 1 for |k| < M/2 and the entry
    of k = -M/2 set to zero, i.e. D_k = 1/M_sigma, D_{-M/2} = 0, so that K = D_{M/2-1}/M_sigma (3.23).
    The NFFT and its adjoint always use the window."""

    def __init__(self, M, sigma: float = 2.0, m: int = 4, kernel: str = "window"):
        self.M = tuple(int(v) for v in np.atleast_1d(M))
        self.d = len(self.M)
        self.sigma = float(sigma)
        self.m = int(m)
        Ms = []
        for Mt in self.M:
            if Mt <= 0 or Mt % 2:
                raise ValueError("M must be a positive even integer")
            v = self.sigma * Mt
            if abs(v - round(v)) > 1e-9 or int(round(v)) % 2:
                raise ValueError("sigma*M must be an even integer")
            Ms.append(int(round(v)))
        self.Ms = tuple(Ms)
        if self.sigma < 1.0:
            raise ValueError("sigma >= 1 required")
        if any(2 * self.m + 2 > v for v in self.Ms) or self.m < 1:
            raise ValueError("need 1 <= m and 2m+2 <= M_sigma")
        self.b = kb.shape_b(self.sigma)
        if kernel not in ("window", "dirichlet"):
            raise ValueError("kernel must be 'window' or 'dirichlet'")
        self.kernel = kernel

    @property
    def taps(self) -> int:
        return (2 * self.m + 1) ** self.d

    def deconv(self, t: int) -> np.ndarray:
        """D entries for dimension t, indexed by k + M/2."""
        return kb.deconv(centred(self.M[t]), self.Ms[t], self.m, self.b)

    def deconv_full(self) -> np.ndarray:
        D = self.deconv(0)
        for t in range(1, self.d):
            D = np.multiply.outer(D, self.deconv(t))
        return D

    def deconv_inv(self, t: int) -> np.ndarray:
        """D of the inverse for dimension t (the window's, or the Dirichlet kernel's)."""
        if self.kernel == "window":
            return self.deconv(t)
        D = np.full(self.M[t], 1.0 / self.Ms[t])
        D[0] = 0.0   # k = -M/2
        return D

    def deconv_inv_full(self) -> np.ndarray:
        D = self.deconv_inv(0)
        for t in range(1, self.d):
            D = np.multiply.outer(D, self.deconv_inv(t))
        return D


def prepare_nodes(x, p: Params):
    """Wrapped nodes, stencil base l0 (int64) and offsets u = x M_sigma - l0, all (N, d)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    if x.shape[1] != p.d:
        x = x.reshape(-1, p.d)
    if not np.all(np.isfinite(x)):
        raise ValueError("non-finite node")
    xw = x - np.floor(x + 0.5)
    Ms = np.array(p.Ms, dtype=np.float64)
    t = xw * Ms
    l0 = np.ceil(t - p.m)
    u = t - l0
    return xw, l0.astype(np.int64), u


def tap_offsets(p: Params) -> np.ndarray:
    """All tap multi-indices tau in {0..2m}^d, first dimension slowest; shape (T, d)."""
    r = range(2 * p.m + 1)
    return np.array(list(itertools.product(*([r] * p.d))), dtype=np.int64)


def tap_weights(x, p: Params):
    """Per node and tap: flattened grid index (row-major, FFT order) and the entry of B,
    w~_m(x_j - l/M_sigma) = prod_t w(u_t - tau_t); shapes (N, T)."""
    _, l0, u = prepare_nodes(x, p)
    taus = tap_offsets(p)
    N = l0.shape[0]
    idx = np.zeros((N, taus.shape[0]), dtype=np.int64)
    wts = np.ones((N, taus.shape[0]), dtype=np.float64)
    for t in range(p.d):
        lt = np.mod(l0[:, t][:, None] + taus[None, :, t], p.Ms[t])
        idx = idx * p.Ms[t] + lt
        wts = wts * kb.window(u[:, t][:, None] - taus[None, :, t], p.m, p.b)
    return idx, wts


def _place(fhat_scaled, p: Params):
    """Zero-pad centred coefficients onto the M_sigma grid at k mod M_sigma."""
    R = fhat_scaled.shape[0]
    g = np.zeros((R,) + p.Ms, dtype=np.complex128)
    sl = [slice(None)]
    pos = [np.mod(centred(p.M[t]), p.Ms[t]) for t in range(p.d)]
    g[(slice(None),) + np.ix_(*pos)] = fhat_scaled
    return g


def _extract(G, p: Params):
    pos = [np.mod(centred(p.M[t]), p.Ms[t]) for t in range(p.d)]
    return G[(slice(None),) + np.ix_(*pos)]


def _axes(p):
    return tuple(range(1, p.d + 1))


def trafo_grid(fhat, p: Params, inverse: bool = False) -> np.ndarray:
    """g = F D fhat on the oversampled grid, (R, *M_sigma); D of the inverse when `inverse`."""
    fh = np.asarray(fhat, dtype=np.complex128).reshape((-1,) + p.M)
    ghat = _place(fh * (p.deconv_inv_full() if inverse else p.deconv_full()), p)
    # sum_k ghat_k e^{+2 pi i k l / M_sigma}: numpy's ifftn carries 1/prod(M_sigma)
    return np.fft.ifftn(ghat, axes=_axes(p)) * float(np.prod(p.Ms))


def trafo(x, fhat, p: Params) -> np.ndarray:
    """NFFT f = B F D fhat; fhat (R, *M) or (*M); returns (R, N) or (N,)."""
    single = np.asarray(fhat).ndim == p.d
    g = trafo_grid(fhat, p).reshape(-1, int(np.prod(p.Ms)))
    idx, wts = tap_weights(x, p)
    f = np.einsum("rnt,nt->rn", g[:, idx], wts)
    return f[0] if single else f


def adjoint_grid(x, f, p: Params) -> np.ndarray:
    """g~ = B^* f on the oversampled grid, (R, *M_sigma)."""
    f = np.atleast_2d(np.asarray(f, dtype=np.complex128))
    idx, wts = tap_weights(x, p)
    G = int(np.prod(p.Ms))
    out = np.zeros((f.shape[0], G), dtype=np.complex128)
    for r in range(f.shape[0]):
        np.add.at(out[r], idx.ravel(), (f[r][:, None] * wts).ravel())
    return out.reshape((f.shape[0],) + p.Ms)


def grid_to_coeffs(gt, p: Params, inverse: bool = False) -> np.ndarray:
    """h~ = D^* F^* g~ restricted to the centred M range, (R, *M); D of the inverse when `inverse`."""
    H = np.fft.fftn(gt, axes=_axes(p))     # sum_l g~_l e^{-2 pi i k l / M_sigma}
    return _extract(H, p) * (p.deconv_inv_full() if inverse else p.deconv_full())


def adjoint(x, f, p: Params) -> np.ndarray:
    """Adjoint NFFT h~ = D^* F^* B^* f; f (R, N) or (N,); returns (R, *M) or (*M)."""
    single = np.asarray(f).ndim == 1
    h = grid_to_coeffs(adjoint_grid(x, f, p), p)
    return h[0] if single else h


# ------------------------------------------------------------ dense factors (tiny sizes only)

def _grid_centred(Ms_t):
    return centred(Ms_t)


def dense_D(p: Params) -> np.ndarray:
    return np.diag(p.deconv_full().ravel()).astype(np.complex128)


def dense_F(p: Params) -> np.ndarray:
    """F in C^{prod M_sigma x prod M}; rows in FFT order (l mod M_sigma), columns centred k."""
    F = None
    for t in range(p.d):
        lpos = np.arange(p.Ms[t])
        lval = np.where(lpos < p.Ms[t] // 2, lpos, lpos - p.Ms[t])
        k = centred(p.M[t])
        Ft = np.exp(2j * np.pi * np.outer(lval, k) / p.Ms[t])
        F = Ft if F is None else np.kron(F, Ft)
    return F


def dense_B(x, p: Params) -> np.ndarray:
    """B in R^{N x prod M_sigma} (2.6)."""
    idx, wts = tap_weights(x, p)
    N = idx.shape[0]
    B = np.zeros((N, int(np.prod(p.Ms))), dtype=np.float64)
    for j in range(N):
        np.add.at(B[j], idx[j], wts[j])
    return B
