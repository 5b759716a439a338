"""Parity at the two-dimensional workloads in full: the polar trajectory (M = 512 x 512, 1024
spokes x 512 samples, N = 524288, m = 4, ridge 1e-8; |I(l)| from 0 to about 5000 at the centre)
and the 32-interleave spiral (M = 256 x 256, N = 65536, 16 right-hand sides, m = 4, ridge 1e-8).

NFFT and adjoint against the FP64 oracle on every output; B_opt on sampled grid indices (the
largest problems, size quantiles and random ones) against the oracle's Gram route, with the
conditioning-aware column check; the modified adjoint with the exported B_opt in full.
"""
import time

import numpy as np
import pytest
import torch

import workloads as W
from oracle import bopt as obopt
from oracle import nfft as onfft

from gpu_util import check_columns, dev, host, nodes_dev, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["c5", "c3"])
def wl(request):
    cfg = W.CONFIGS[request.param]
    rhs = 4 if request.param == "c5" else 1
    x, fh = W.make_problem(cfg, seed=0, rhs=rhs)
    p = onfft.Params(cfg["M"], cfg["sigma"], cfg["m"])
    mem = obopt.Members(x, p)
    return request.param, cfg, x, fh, p, mem


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_full_2d_trafo_and_adjoint(wl, precision):
    from paper_1811_05335_amd import NfftPlan
    name, cfg, x, fh, p, _ = wl
    tol = 1e-12 if precision == "f64" else 1e-5
    if precision == "f32":
        fh = W.round_to(fh, "f32")
    R = fh.shape[0]
    P = NfftPlan(cfg["M"], nodes_dev(x), sigma=cfg["sigma"], m=cfg["m"], precision=precision,
                 rho=cfg["rho"], max_rhs=R)
    fd = P.trafo(dev(fh, precision))
    f = host(fd)
    assert rel(f, onfft.trafo(x, fh, p)) <= tol, name
    h = host(P.adjoint(fd))
    assert rel(h, onfft.adjoint(x, f, p)) <= tol, name
    P.close()


def sample_grid_indices(sizes, seed):
    nz = np.nonzero(sizes > 0)[0]
    order = nz[np.argsort(sizes[nz], kind="stable")]
    pick = list(order[-3:])                                  # the largest problems
    for q in (0.5, 0.9, 0.99, 0.999, 0.9999):              # size quantiles
        pick.append(order[min(len(order) - 1, int(q * len(order)))])
    pick += list(W.rng(seed).choice(nz, size=24, replace=False))
    return np.unique(np.asarray(pick))


def test_full_2d_precompute_and_apply(wl):
    from paper_1811_05335_amd import NfftPlan
    name, cfg, x, fh, p, mem = wl
    sizes = mem.sizes()
    P = NfftPlan(cfg["M"], nodes_dev(x), sigma=cfg["sigma"], m=cfg["m"], precision="f64",
                 rho=cfg["rho"], max_rhs=fh.shape[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.precompute_B()
    st = P.status()
    print(f"[{name}] precompute_B {time.perf_counter() - t0:.3f} s, |I(l)| up to {sizes.max()}", flush=True)
    assert st["failed_solves"] == 0 and st["oversized"] == 0
    assert st["max_members"] == sizes.max()
    assert st["min_members"] == sizes[sizes > 0].min()
    assert st["empty_columns"] == int(np.sum(sizes == 0))
    rows = host(P.get_B())
    ls = sample_grid_indices(sizes, seed=5)
    check_columns(x, p, cfg["rho"], mem, ls, rows)
    # the modified adjoint with this B_opt is an exact linear map: FP64 to rounding
    f = onfft.trafo(x, fh, p)
    fc = host(P.apply(dev(f, "f64")))
    assert rel(fc, obopt.apply(x, f, rows, p)) <= 1e-12, name
    P.close()
