"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np
import torch

import workloads as W
from oracle import bopt as obopt
from oracle import nfft as onfft

CT = {"f32": torch.complex64, "f64": torch.complex128}


def dev(a, precision):
    return torch.from_numpy(np.ascontiguousarray(a)).to(CT[precision]).cuda()


def nodes_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def problem(M, N, d=1, nodes="uniform", seed=0, rhs=1, sigma=2.0, m=4):
    g = W.rng(seed)
    if nodes == "uniform":
        x = W.uniform_nodes(g, N, d)
    elif nodes == "jittered":
        x = W.jittered_nodes(g, N)
    elif nodes == "equispaced":
        x = W.equispaced_nodes(N)
    else:
        raise ValueError(nodes)
    fh = W.complex_normal(g, (rhs,) + tuple(M))
    f = W.complex_normal(g, (rhs, N))
    p = onfft.Params(M, sigma, m)
    return x, fh, f, p


def check_columns(x, p, rho, mem, ls, rows_gpu):
    """Per grid index: the column itself where cond(G + lambda I) <= 1e6, else the excess of
    the least-squares objective, (b - b*)^* (G + lambda I) (b - b*), against the optimum
    J* = 1 - r^* b*: the error measure that conditioning does not inflate."""
    nobj = 0
    for l in ls:
        js, ts, _ = mem.of(int(l))
        G, r = obopt.gram_system(x, int(l), js, p)
        n = len(js)
        A = G + rho * np.real(np.trace(G)) / n * np.eye(n)
        b_o = obopt.solve_G(x, int(l), js, p, rho)
        b_g = rows_gpu[js, ts]
        ev = np.linalg.eigvalsh(A)
        if ev[-1] / ev[0] <= 1e6:
            assert rel(b_g, b_o) <= 1e-9, int(l)
        else:
            d = b_g - b_o
            excess = float(np.real(np.vdot(d, A @ d)))
            J = 1.0 - float(np.real(np.vdot(r, b_o)))
            assert excess <= 1e-10 * J, (int(l), n, excess, J)
            nobj += 1
    return nobj


def check_all_columns(x, p, rho, rows_gpu):
    """check_columns over every grid index with members; grid indices with no member must leave
    no entry (the rows of B_opt hold entries only for members)."""
    mem = obopt.Members(x, p)
    ls = np.nonzero(mem.sizes())[0]
    return check_columns(x, p, rho, mem, ls, rows_gpu)


def apply_own_vs_oracle(x, p, rho, rows_gpu, fs, out_gpu, tol=1e-8):
    """The modified adjoint computed with the GPU's own B_opt against the oracle's modified adjoint
    with the oracle's B_opt (Gram route), on samples fs of a trigonometric polynomial (the paper's
    setting f = A fhat): <= 1e-8 relative."""
    rows_o, _ = obopt.bopt_rows(x, p, rho, route="G")
    ref = obopt.apply(x, fs, rows_o, p)
    err = rel(out_gpu, ref)
    assert err <= tol, ("apply with own B_opt vs oracle", err)
    return err
