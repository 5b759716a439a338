"""The whole path captured in a HIP graph (through torch.cuda.graph) and replayed several times,
with eager work and synchronisations between the replays: every replay must match the eager
result (sums in LDS may associate differently, so the comparison is to rounding)."""
import numpy as np
import pytest
import torch

import workloads as W

from gpu_util import dev, host, nodes_dev, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("d", [1, 2])
def test_graph_replays_match_eager(precision, tol, d):
    from paper_1811_05335_amd import NfftPlan
    M = (300,) if d == 1 else (24, 20)
    N = 700
    g = W.rng(20 + d)
    x = W.uniform_nodes(g, N, d)
    fh = dev(W.complex_normal(g, (2,) + M), precision)
    gf = dev(W.complex_normal(g, (2, N)), precision)
    xd = nodes_dev(x)
    P = NfftPlan(M, xd, sigma=2.0, m=3, precision=precision, rho=1e-8, max_rhs=2)

    def step():
        P.set_nodes(xd)
        f = P.trafo(fh)
        h = P.adjoint(f)
        P.precompute_B()
        fc = P.apply(f)
        fa = P.apply_adjoint(fc)
        gx = P.grad_x(fh, gf)
        return f, h, fc, fa, gx

    eager = [host(o) if o.is_complex() else o.cpu().numpy() for o in step()]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = step()
    for rep in range(4):
        graph.replay()
        torch.cuda.synchronize()
        got = [host(o) if o.is_complex() else o.cpu().numpy() for o in outs]
        for a, b in zip(got, eager):
            assert rel(a, b) <= tol, rep
        # eager work between replays reuses the plan's buffers
        _ = P.trafo(fh)
        torch.cuda.synchronize()
    P.close()
