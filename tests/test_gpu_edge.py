"""Nodes on or within rounding of grid lines: the tap 2m belongs to the window exactly when
|u - 2m| <= m in FP64, the oracle's membership test; NFFT, adjoint and B_opt must take the same
decision (the polar trajectory has such nodes on its axis spokes)."""
import numpy as np
import pytest

import workloads as W
from oracle import bopt as obopt
from oracle import nfft as onfft

from gpu_util import check_columns, dev, host, nodes_dev, rel

pytestmark = pytest.mark.gpu


def grid_line_nodes(M, N, d, seed):
    """Uniform nodes, a third moved onto grid lines of one coordinate (u = m), a third just below
    the grid line through 0, with x M_sigma in (-9e-16, -3e-16): there u rounds to just below m
    while u - 2m rounds to -m, so tap 2m is still a member in FP64."""
    g = W.rng(seed)
    x = W.uniform_nodes(g, N, d)
    Ms = 2 * M[0]
    k = g.integers(-Ms // 2, Ms // 2, size=N)
    third = N // 3
    x[:third, 0] = k[:third] / Ms
    x[third:2 * third, 0] = -g.uniform(3e-16, 9e-16, third) / Ms
    if d == 2:
        x[:third:2, 1] = -0.0
    return x


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("M,d,m", [((64,), 1, 4), ((32, 24), 2, 4)])
def test_grid_line_nodes_match_oracle(precision, tol, M, d, m):
    from paper_1811_05335_amd import NfftPlan
    N = 600
    x = grid_line_nodes(M, N, d, seed=21)
    p = onfft.Params(M, 2.0, m)
    # the case is present: some nodes have u < m but tap 2m inside the support in FP64
    t = (x - np.floor(x + 0.5)) * np.array(p.Ms)
    u = t - np.ceil(t - m)
    assert np.any((u[:, 0] < m) & (np.abs(u[:, 0] - 2 * m) <= m))
    g = W.rng(22)
    fh = W.complex_normal(g, (1,) + M)
    if precision == "f32":
        fh = W.round_to(fh, "f32")
    P = NfftPlan(M, nodes_dev(x), sigma=2.0, m=m, precision=precision, rho=1e-8)
    fd = P.trafo(dev(fh, precision))
    f = host(fd)
    assert rel(f, onfft.trafo(x, fh, p)) <= tol
    assert rel(host(P.adjoint(fd)), onfft.adjoint(x, f, p)) <= tol
    if precision == "f64":
        P.precompute_B()
        st = P.status()
        mem = obopt.Members(x, p)
        sizes = mem.sizes()
        assert st["failed_solves"] == 0 and st["oversized"] == 0
        assert st["max_members"] == sizes.max() and st["empty_columns"] == int(np.sum(sizes == 0))
        rows = host(P.get_B())
        _, solved = obopt.bopt_rows(x, p, 1e-8, route="G", ls=np.nonzero(sizes)[0][:1], members=mem)
        # sparsity pattern of B_opt equals the oracle's membership
        pattern = np.zeros(rows.shape, dtype=bool)
        pattern[mem.j, mem.t] = True
        assert np.array_equal(rows != 0, pattern)
        ls = W.rng(23).choice(np.nonzero(sizes)[0], size=48, replace=False)
        check_columns(x, p, 1e-8, mem, ls, rows)
    P.close()
