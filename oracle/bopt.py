"""Optimisation of the sparse matrix B, Algorithm 3.17, and the modified adjoint NFFT
(oracle; test infrastructure only).

For each oversampled grid index l the paper solves (3.29)-(3.31)

    b~_l = argmin_b || L_l b - e_l ||_2,   L_l = F D H_l,
    L_l[s, j] = K(s/M_sigma - x_j),  s over the grid, j in I(l)                     (3.30)
    K(y) = (1/M_sigma) sum_k e^{2 pi i k y} / w_hat(-k)                              (3.15)

and composes B_opt column by column (Algorithm 3.17, step 3).  I(l) is the set of nodes whose
truncated window reaches l (3.29); the membership test is |u_j - tau| <= m per dimension with
tau = (l - l0_j) mod M_sigma (see `nfft`).

Readings taken where the paper is silent or assumes full rank:
  * unknowns: one per member of I(l) (the paper's "2m+1" is the 1-D bound);
  * B_opt is complex: (3.31) is the complex least-squares solution (K is complex over the
    asymmetric range -M/2..M/2-1);
  * ridge: b~_l = argmin ||L_l b - e_l||^2 + lambda ||b||^2 with
    lambda = rho * trace(L_l^* L_l) / |I(l)|  (rho = 0 gives the paper's (3.31); with rho = 0
    and a rank-deficient L_l the minimum-norm solution is returned);
  * empty I(l): the column of B_opt is zero.

Three independent routes to b~_l (each exact in exact arithmetic):
  E  the definition: L_l assembled entry by entry from (3.15), stacked least squares;
  R  reduced: F has orthogonal columns (F^* F = M_sigma^d I), so the same minimiser solves
     min ||D H_l b - q_l||^2 + (lambda/M_sigma^d) ||b||^2, q_l = M_sigma^-d e^{-2 pi i k.l/M_sigma};
  G  normal equations in closed form: (L_l^* L_l)[i,j] = M_sigma^d Q(x_i - x_j) with
     Q(y) = sum_k e^{2 pi i k.y} / (M_sigma w_hat(k))^2, and (L_l^* e_l)[j] = conj K(l/M_sigma - x_j),
     both as direct O(M) sums, then a dense solve of (G + lambda I) b = r.
"""
from __future__ import annotations

import numpy as np

from . import kb
from .direct import centred, phase_matrix
from .nfft import Params, prepare_nodes, tap_offsets, grid_to_coeffs, trafo_grid


# ---------------------------------------------------------------- membership I(l)

class Members:
    """CSR over flattened grid indices l: members (node j, tap row index t) sorted by (l, j)."""

    def __init__(self, x, p: Params):
        _, l0, u = prepare_nodes(x, p)
        taus = tap_offsets(p)
        N, T = l0.shape[0], taus.shape[0]
        v = u[:, None, :] - taus[None, :, :]
        mem = np.all(np.abs(v) <= p.m, axis=2)
        lflat = np.zeros((N, T), dtype=np.int64)
        for t in range(p.d):
            lflat = lflat * p.Ms[t] + np.mod(l0[:, t][:, None] + taus[None, :, t], p.Ms[t])
        jj, tt = np.nonzero(mem)
        ll = lflat[jj, tt]
        order = np.lexsort((jj, ll))
        self.l = ll[order]
        self.j = jj[order]
        self.t = tt[order]
        self.z = -v[jj, tt][order]          # tau - u, the argument of K in grid units
        G = int(np.prod(p.Ms))
        self.ptr = np.searchsorted(self.l, np.arange(G + 1))
        self.N, self.T, self.G = N, T, G
        self.l0, self.u = l0, u

    def of(self, l: int):
        s, e = self.ptr[l], self.ptr[l + 1]
        return self.j[s:e], self.t[s:e], self.z[s:e]

    def sizes(self) -> np.ndarray:
        return np.diff(self.ptr)


def grid_multi_index(l: int, p: Params):
    idx = []
    for t in reversed(range(p.d)):
        idx.append(l % p.Ms[t])
        l //= p.Ms[t]
    lm = np.array(idx[::-1], dtype=np.int64)
    # centred value of the grid index
    Ms = np.array(p.Ms)
    return np.where(lm < Ms // 2, lm, lm - Ms)


# ---------------------------------------------------------------- kernels K, Q (direct sums)

def kernel_K_1d(y, p: Params, t: int) -> np.ndarray:
    """(3.15) K(y) = (1/M_sigma) sum_{k=-M/2}^{M/2-1} e^{2 pi i k y} / w_hat(-k) in dimension t,
    i.e. sum_k D_k e^{2 pi i k y} with the inverse's D (w_hat is even)."""
    k = centred(p.M[t])
    coef = p.deconv_inv(t)
    y = np.asarray(y, dtype=np.float64).ravel()
    y = y - np.floor(y + 0.5)
    return phase_matrix(y, k, +1) @ coef


def kernel_Q_1d(y, p: Params, t: int) -> np.ndarray:
    """Q(y) = sum_k D_k^2 e^{2 pi i k y} in dimension t."""
    k = centred(p.M[t])
    coef = p.deconv_inv(t) ** 2
    y = np.asarray(y, dtype=np.float64).ravel()
    y = y - np.floor(y + 0.5)
    return phase_matrix(y, k, +1) @ coef


def gram_Q_1d(xt, p: Params, t: int) -> np.ndarray:
    """Q(x_i - x_j) for all pairs of one coordinate: e^{2 pi i k (x_i - x_j)} factors into
    e^{2 pi i k x_i} conj(e^{2 pi i k x_j}), so the matrix is E diag(c) E^* with
    E[i, k] = e^{2 pi i k x_i} and c_k = D_k^2 (the same sum as kernel_Q_1d)."""
    k = centred(p.M[t])
    coef = p.deconv_inv(t) ** 2
    E = phase_matrix(np.asarray(xt, dtype=np.float64).ravel(), k, +1)
    return (E * coef[None, :]) @ E.conj().T


def kernel_K(Y, p: Params) -> np.ndarray:
    """Tensor-product K for arguments Y (n, d) in x units."""
    Y = np.atleast_2d(Y)
    out = np.ones(Y.shape[0], dtype=np.complex128)
    for t in range(p.d):
        out = out * kernel_K_1d(Y[:, t], p, t)
    return out


def kernel_Q(Y, p: Params) -> np.ndarray:
    Y = np.atleast_2d(Y)
    out = np.ones(Y.shape[0], dtype=np.complex128)
    for t in range(p.d):
        out = out * kernel_Q_1d(Y[:, t], p, t)
    return out


def _grid_points(p: Params) -> np.ndarray:
    """All grid points s/M_sigma in FFT storage order, shape (G, d)."""
    axes = []
    for t in range(p.d):
        s = np.arange(p.Ms[t])
        s = np.where(s < p.Ms[t] // 2, s, s - p.Ms[t])
        axes.append(s / p.Ms[t])
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([a.ravel() for a in mesh], axis=1)


# ---------------------------------------------------------------- the three routes

def L_matrix(x, js, p: Params) -> np.ndarray:
    """(3.30) L_l: rows s over the whole grid (FFT order), columns j in js."""
    xw, _, _ = prepare_nodes(x, p)
    S = _grid_points(p)
    L = np.empty((S.shape[0], len(js)), dtype=np.complex128)
    for c, j in enumerate(js):
        L[:, c] = kernel_K(S - xw[j][None, :], p)
    return L


def solve_E(x, l: int, js, p: Params, rho: float) -> np.ndarray:
    n = len(js)
    if n == 0:
        return np.zeros(0, dtype=np.complex128)
    L = L_matrix(x, js, p)
    e = np.zeros(L.shape[0], dtype=np.complex128)
    e[l] = 1.0
    lam = rho * np.real(np.trace(L.conj().T @ L)) / n
    if lam > 0:
        A = np.vstack([L, np.sqrt(lam) * np.eye(n)])
        rhs = np.concatenate([e, np.zeros(n)])
    else:
        A, rhs = L, e
    return np.linalg.lstsq(A, rhs, rcond=None)[0]


def _H(xw_sel, p: Params) -> np.ndarray:
    """H_l = (e^{-2 pi i k.x_j})_{k,j}, k flattened row-major."""
    H = None
    for t in range(p.d):
        Ht = phase_matrix(xw_sel[:, t], centred(p.M[t]), -1).T   # (M_t, n)
        H = Ht if H is None else (H[:, None, :] * Ht[None, :, :]).reshape(-1, Ht.shape[1])
    return H


def solve_R(x, l: int, js, p: Params, rho: float) -> np.ndarray:
    n = len(js)
    if n == 0:
        return np.zeros(0, dtype=np.complex128)
    xw, _, _ = prepare_nodes(x, p)
    DH = p.deconv_inv_full().ravel()[:, None] * _H(xw[np.asarray(js)], p)
    lv = grid_multi_index(l, p)
    q = np.ones(1, dtype=np.complex128)
    for t in range(p.d):
        k = centred(p.M[t])
        qt = np.exp(-2j * np.pi * k * lv[t] / p.Ms[t]) / p.Ms[t]
        q = np.multiply.outer(q, qt).ravel()
    lam = rho * np.real(np.sum(np.abs(DH) ** 2)) / n
    if lam > 0:
        A = np.vstack([DH, np.sqrt(lam) * np.eye(n)])
        rhs = np.concatenate([q, np.zeros(n)])
    else:
        A, rhs = DH, q
    return np.linalg.lstsq(A, rhs, rcond=None)[0]


def gram_system(x, l: int, js, p: Params):
    """G = L_l^* L_l and r = L_l^* e_l in closed form (direct sums)."""
    xw, _, _ = prepare_nodes(x, p)
    X = xw[np.asarray(js)]
    n = len(js)
    G = np.full((n, n), float(np.prod(p.Ms)), dtype=np.complex128)
    for t in range(p.d):
        G *= gram_Q_1d(X[:, t], p, t)
    lv = grid_multi_index(l, p) / np.array(p.Ms, dtype=np.float64)
    r = np.conj(kernel_K(lv[None, :] - X, p))
    return G, r


def solve_G(x, l: int, js, p: Params, rho: float) -> np.ndarray:
    n = len(js)
    if n == 0:
        return np.zeros(0, dtype=np.complex128)
    G, r = gram_system(x, l, js, p)
    lam = rho * np.real(np.trace(G)) / n
    return np.linalg.solve(G + lam * np.eye(n), r)


ROUTES = {"E": solve_E, "R": solve_R, "G": solve_G}


def bopt_rows(x, p: Params, rho: float, route: str = "R", ls=None, members: Members | None = None):
    """B_opt in row layout: rows[j, tau] (tau flattened over {0..2m}^d, first dim slowest),
    zero where the tap is outside the support.  With `ls` given, only those columns l are
    solved (the other entries stay zero) and the solved entries are returned in a mask."""
    mem = members or Members(x, p)
    rows = np.zeros((mem.N, mem.T), dtype=np.complex128)
    solved = np.zeros((mem.N, mem.T), dtype=bool)
    solve = ROUTES[route]
    it = range(mem.G) if ls is None else ls
    for l in it:
        js, ts, _ = mem.of(int(l))
        if len(js) == 0:
            continue
        b = solve(x, int(l), js, p, rho)
        rows[js, ts] = b
        solved[js, ts] = True
    return rows, solved


# ---------------------------------------------------------------- modified adjoint and its adjoint

def _tap_grid_index(x, p: Params):
    _, l0, _ = prepare_nodes(x, p)
    taus = tap_offsets(p)
    idx = np.zeros((l0.shape[0], taus.shape[0]), dtype=np.int64)
    for t in range(p.d):
        idx = idx * p.Ms[t] + np.mod(l0[:, t][:, None] + taus[None, :, t], p.Ms[t])
    return idx


def apply(x, f, rows, p: Params) -> np.ndarray:
    """(3.32) f_check = D^* F^* B_opt^* f; f (R, N) or (N,) -> (R, *M) or (*M)."""
    single = np.asarray(f).ndim == 1
    f = np.atleast_2d(np.asarray(f, dtype=np.complex128))
    idx = _tap_grid_index(x, p)
    G = int(np.prod(p.Ms))
    gt = np.zeros((f.shape[0], G), dtype=np.complex128)
    for r in range(f.shape[0]):
        np.add.at(gt[r], idx.ravel(), (np.conj(rows) * f[r][:, None]).ravel())
    h = grid_to_coeffs(gt.reshape((f.shape[0],) + p.Ms), p, inverse=True)
    return h[0] if single else h


def apply_adjoint(x, h, rows, p: Params) -> np.ndarray:
    """Remark 3.24: f = B_opt F D h; h (R, *M) or (*M) -> (R, N) or (N,)."""
    single = np.asarray(h).ndim == p.d
    g = trafo_grid(h, p, inverse=True).reshape(-1, int(np.prod(p.Ms)))
    idx = _tap_grid_index(x, p)
    f = np.einsum("rnt,nt->rn", g[:, idx], rows)
    return f[0] if single else f


def dense_from_rows(x, rows, p: Params) -> np.ndarray:
    """B_opt as a dense N x prod(M_sigma) matrix (tiny sizes)."""
    idx = _tap_grid_index(x, p)
    B = np.zeros((rows.shape[0], int(np.prod(p.Ms))), dtype=np.complex128)
    for j in range(rows.shape[0]):
        np.add.at(B[j], idx[j], rows[j])
    return B


def frobenius_objective(x, B, p: Params) -> float:
    """|| K^* B - I ||_F with K^* = F D A^*, dense (tiny sizes), (3.34)."""
    from .direct import ndft_matrix
    from .nfft import dense_D, dense_F
    A = ndft_matrix(x, p.M)
    Kstar = dense_F(p) @ dense_D(p) @ A.conj().T
    return float(np.linalg.norm(Kstar @ B - np.eye(Kstar.shape[0])))
