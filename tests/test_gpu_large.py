"""Local problems of Algorithm 3.17 with more members than the register tiers hold (|I(l)| > 32):
the blocked Cholesky pass, against the oracle's Gram route on every such grid index, with
sizes spanning one block, several blocks and a ragged last block; in one and two dimensions."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import bopt as obopt
from oracle import nfft as onfft

from gpu_util import check_columns, host, nodes_dev, rel

pytestmark = pytest.mark.gpu

# M, N, d, m, nodes in the dense spot, half-width of the spot in grid cells, rho
CASES = [
    ((32, 32), 700, 2, 3, 300, 2.5, 1e-8),
    ((24, 20), 400, 2, 2, 150, 1.5, 1e-8),
    ((64,), 600, 1, 4, 200, 2.0, 1e-8),
    ((48,), 300, 1, 3, 80, 1.0, 1e-10),
]


def clustered(M, N, d, m, ncl, half_cells, seed):
    g = W.rng(seed)
    x = W.clustered_nodes(g, N, d, ncl, half_cells / (2 * M[0]))
    p = onfft.Params(M, 2.0, m)
    return x, p


@pytest.mark.parametrize("M,N,d,m,ncl,half,rho", CASES)
def test_large_problems_match_oracle(M, N, d, m, ncl, half, rho):
    from paper_1811_05335_amd import NfftPlan
    x, p = clustered(M, N, d, m, ncl, half, seed=11)
    mem = obopt.Members(x, p)
    sizes = mem.sizes()
    assert sizes.max() > 64          # the multi-block path runs
    P = NfftPlan(M, nodes_dev(x), sigma=2.0, m=m, precision="f64", rho=rho)
    P.precompute_B()
    st = P.status()
    assert st["failed_solves"] == 0 and st["oversized"] == 0
    assert st["max_members"] == sizes.max()
    assert st["min_members"] == sizes[sizes > 0].min()
    assert st["empty_columns"] == int(np.sum(sizes == 0))
    rows_gpu = host(P.get_B())
    big = np.nonzero(sizes > 32)[0]
    g = W.rng(3)
    small = g.choice(np.nonzero((sizes > 0) & (sizes <= 32))[0], size=32, replace=False)
    # 1-D: every problem of 17..32 members (16-lane groups with two rows per lane solve them)
    mid = np.nonzero((sizes > 16) & (sizes <= 32))[0] if d == 1 else np.zeros(0, dtype=np.int64)
    ls = np.unique(np.concatenate([big, small, mid]))
    check_columns(x, p, rho, mem, ls, rows_gpu)
    P.close()


@pytest.mark.parametrize("M,N,d,m,ncl,half,thr", [((32, 32), 700, 2, 3, 300, 2.5, 32),
                                                   ((64,), 600, 1, 4, 200, 2.0, 64)])
def test_large_problems_under_graph_capture_replay_the_recorded_pass(M, N, d, m, ncl, half, thr):
    """Under graph capture the large-problem pass (beyond 32 members in 2-D, beyond 64 in 1-D, where
    a wavefront per problem takes 33..64) replays the one the eager call recorded: every column,
    large problems included, equals the eager B_opt and nothing is oversized."""
    from paper_1811_05335_amd import NfftPlan
    x, p = clustered(M, N, d, m, ncl, half, seed=12)
    sizes = obopt.Members(x, p).sizes()
    assert np.any(sizes > thr) and (d == 2 or np.any((sizes > 32) & (sizes <= thr)))
    xd = nodes_dev(x)
    P = NfftPlan(M, xd, sigma=2.0, m=m, precision="f64", rho=1e-8)
    P.precompute_B()
    eager = host(P.get_B())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        P.precompute_B()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        st = P.status()
        assert st["oversized"] == 0 and st["failed_solves"] == 0
        assert st["max_members"] == sizes.max()
        assert np.array_equal(host(P.get_B()), eager), rep
    P.close()
