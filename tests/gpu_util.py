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
