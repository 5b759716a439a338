"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np
import torch

import workloads as W
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
