"""Parity at the full benchmark workload (1-D jittered, M = 2^16, N = 2^17, sigma = 2, m = 6, ridge
1e-12) in the plan configuration the benchmark times, and at the small uniform workload
(M = 256, N = 512, m = 4, ridge 1e-8) in full.

Full-vector comparisons where the FP64 oracle is fast (NFFT, adjoint, modified adjoint with the
exported B_opt, its adjoint, node gradient); B_opt itself on sampled grid indices against the
oracle's reduced route; exact sums on sampled nodes.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import bopt as obopt
from oracle import direct as odirect
from oracle import grad as ograd
from oracle import nfft as onfft

from gpu_util import apply_own_vs_oracle, check_all_columns, check_columns, dev, host, nodes_dev, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    cfg = W.CONFIGS["c2"]
    x, fh = W.make_problem(cfg, seed=0, rhs=1)
    gf = W.complex_normal(W.rng(1), (1, cfg["N"]))
    p = onfft.Params(cfg["M"], cfg["sigma"], cfg["m"])
    return cfg, x, fh, gf, p


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_full_c2_path_matches_oracle(c2, precision):
    from paper_1811_05335_amd import NfftPlan
    cfg, x, fh, gf, p = c2
    tol = 1e-12 if precision == "f64" else 1e-5
    if precision == "f32":
        fh = W.round_to(fh, "f32")
        gf = W.round_to(gf, "f32")
    P = NfftPlan(cfg["M"], nodes_dev(x), sigma=cfg["sigma"], m=cfg["m"], precision=precision,
                 rho=cfg["rho"], max_rhs=1)
    fd = P.trafo(dev(fh, precision))
    f = host(fd)
    assert rel(f, onfft.trafo(x, fh, p)) <= tol
    # exact sums on sampled nodes: within the window error of m = 6 (FP64), or within the FP32
    # rounding of the transform (FP32)
    idx = W.rng(2).choice(cfg["N"], size=512, replace=False)
    exact = odirect.ndft(x[idx], fh[0])
    if precision == "f64":
        env = 4 * np.pi * (np.sqrt(6) + 6) * 0.5 ** 0.25 * np.exp(-2 * np.pi * 6 * np.sqrt(0.5))
        assert np.max(np.abs(f[0, idx] - exact)) <= env * np.sum(np.abs(fh))
    else:
        assert rel(f[0, idx], exact) <= 1e-5
    h = host(P.adjoint(fd))
    assert rel(h, onfft.adjoint(x, f, p)) <= tol
    P.precompute_B()
    st = P.status()
    assert st["failed_solves"] == 0 and st["oversized"] == 0 and st["empty_columns"] == 0
    assert (st["min_members"], st["max_members"]) == (11, 13)
    rows = host(P.get_B())
    # sampled columns of B_opt: each against the oracle's Gram route, <= 1e-9 where
    # cond(G + lambda I) <= 1e6, else by the excess of the least-squares objective
    mem = obopt.Members(x, p)
    ls = np.sort(W.rng(3).choice(mem.G, size=64, replace=False))
    check_columns(x, p, cfg["rho"], mem, ls, rows)
    # and against the reduced route (rows of the same columns)
    ref, solved = obopt.bopt_rows(x, p, cfg["rho"], route="R", ls=ls[:16], members=mem)
    assert solved.sum() >= 16 * 11
    assert rel(rows[solved], ref[solved]) <= 1e-7
    rows_used = rows.astype(np.complex64).astype(np.complex128) if precision == "f32" else rows
    fc = host(P.apply(fd))
    assert rel(fc, obopt.apply(x, f, rows_used, p)) <= tol
    # the modified adjoint inverts the NFFT on the paper's jittered nodes (reported accuracy)
    assert rel(fc, fh) <= 1e-4
    fa = host(P.apply_adjoint(dev(fc, precision)))
    assert rel(fa, obopt.apply_adjoint(x, fc, rows_used, p)) <= tol
    gx = P.grad_x(dev(fh, precision), dev(gf, precision)).cpu().numpy()
    assert rel(gx, ograd.nfft_grad_x(x, fh, gf, p)) <= (1e-10 if precision == "f64" else 1e-4)
    P.close()


def test_full_c1_pipeline_matches_oracle():
    """M = 256, N = 512 uniform nodes, m = 4, ridge 1e-8: NFFT, every column of B_opt, modified
    adjoint; complex128."""
    from paper_1811_05335_amd import NfftPlan
    cfg = W.CONFIGS["c1"]
    x, fh = W.make_problem(cfg, seed=0)
    p = onfft.Params(cfg["M"], cfg["sigma"], cfg["m"])
    P = NfftPlan(cfg["M"], nodes_dev(x), sigma=2.0, m=cfg["m"], precision="f64", rho=cfg["rho"])
    fd = P.trafo(dev(fh, "f64"))
    f = host(fd)
    assert rel(f, onfft.trafo(x, fh, p)) <= 1e-12
    P.precompute_B()
    rows = host(P.get_B())
    check_all_columns(x, p, cfg["rho"], rows)
    fc = host(P.apply(fd))
    # with the GPU's own B_opt against the oracle's apply with the oracle's B_opt, and with the same
    apply_own_vs_oracle(x, p, cfg["rho"], rows, f, fc, tol=1e-8)
    assert rel(fc, obopt.apply(x, f, rows, p)) <= 1e-12
    fs = odirect.ndft(x, fh)
    apply_own_vs_oracle(x, p, cfg["rho"], rows, fs, host(P.apply(dev(fs, "f64"))), tol=1e-8)
