"""The Dirichlet kernel of Remark 3.19 for the inverse (w_hat = 1 for |k| < M/2, the entry of
k = -M/2 zeroed): B_opt, the modified adjoint and its adjoint against the oracle with the same
kernel, in one and two dimensions, with problems beyond the register tiers, and in a batch."""
import numpy as np
import pytest

import workloads as W
from oracle import bopt as obopt
from oracle import direct as odirect
from oracle import nfft as onfft

from gpu_util import check_columns, dev, host, nodes_dev, rel

pytestmark = pytest.mark.gpu

CASES = [
    ((64,), 256, 1, "jittered", 4, 1e-10),
    ((40,), 150, 1, "uniform", 3, 1e-8),
    ((12, 16), 300, 2, "uniform", 3, 1e-8),
    ((32, 32), 700, 2, "clustered", 3, 1e-8),
]


def nodes(kind, N, d, M, seed):
    g = W.rng(seed)
    if kind == "jittered":
        return W.jittered_nodes(g, N)
    if kind == "clustered":
        return W.clustered_nodes(g, N, d, 300, 2.5 / (2 * M[0]))
    return W.uniform_nodes(g, N, d)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("M,N,d,kind,m,rho", CASES)
def test_dirichlet_inverse_matches_oracle(precision, M, N, d, kind, m, rho):
    from paper_1811_05335_amd import NfftPlan
    x = nodes(kind, N, d, M, seed=70)
    p = onfft.Params(M, 2.0, m, kernel="dirichlet")
    g = W.rng(71)
    fh = W.complex_normal(g, (2,) + M)
    f = W.complex_normal(g, (2, N))
    if precision == "f32":
        fh, f = W.round_to(fh, "f32"), W.round_to(f, "f32")
    P = NfftPlan(M, nodes_dev(x), sigma=2.0, m=m, precision=precision, rho=rho, max_rhs=2, kernel="dirichlet")
    # the NFFT itself keeps the window
    tol = 1e-12 if precision == "f64" else 1e-5
    assert rel(host(P.trafo(dev(fh, precision))), onfft.trafo(x, fh, onfft.Params(M, 2.0, m))) <= tol
    P.precompute_B()
    st = P.status()
    assert st["failed_solves"] == 0 and st["oversized"] == 0
    rows = host(P.get_B())
    assert np.max(np.abs(rows.imag)) <= 1e-6 * np.max(np.abs(rows))   # real B_opt, up to ridge-conditioned rounding
    if precision == "f64":
        mem = obopt.Members(x, p)
        sizes = mem.sizes()
        ls = np.nonzero(sizes)[0]
        if len(ls) > 200:
            ls = np.concatenate([np.nonzero(sizes > 32)[0], W.rng(72).choice(ls, 100, replace=False)])
        check_columns(x, p, rho, mem, np.unique(ls), rows)
    r = rows if precision == "f64" else rows.astype(np.complex64).astype(np.complex128)
    fc = host(P.apply(dev(f, precision)))
    assert np.all(fc[..., 0] == 0) if d == 1 else np.all(fc[:, 0, :] == 0) and np.all(fc[:, :, 0] == 0)
    assert rel(fc, obopt.apply(x, f, r, p)) <= tol
    assert rel(host(P.apply_adjoint(dev(fh, precision))), obopt.apply_adjoint(x, fh, r, p)) <= tol
    P.close()


def test_dirichlet_reconstruction_jittered():
    """Example 3.23's setting (Dirichlet, sigma = 2, jittered nodes, N = 4M, m = 4): the estimate
    from samples of a trigonometric polynomial against its coefficients, GPU and oracle alike."""
    from paper_1811_05335_amd import NfftPlan
    M = 512
    g = W.rng(73)
    x = W.jittered_nodes(g, 4 * M)
    fh = W.complex_normal(g, (M,))
    f = odirect.ndft(x, fh)
    p = onfft.Params((M,), 2.0, 4, kernel="dirichlet")
    P = NfftPlan((M,), nodes_dev(x), sigma=2.0, m=4, precision="f64", rho=1e-12, kernel="dirichlet")
    P.precompute_B()
    fc = host(P.apply(dev(f[None], "f64")))[0]
    e_gpu = rel(fc[1:], fh[1:])
    rows, _ = obopt.bopt_rows(x, p, 1e-12, "G")
    e_ora = rel(obopt.apply(x, f, rows, p)[1:], fh[1:])
    assert e_gpu < 1e-5 and abs(e_gpu - e_ora) <= 1e-3 * e_ora + 1e-12
    P.close()


def test_dirichlet_batch_matches_single_plans():
    from paper_1811_05335_amd import NfftBatchPlan, NfftPlan
    g = W.rng(74)
    Ms = [40, 128, 1152]
    Ns = [100, 300, 2600]
    xs = [W.uniform_nodes(g, N, 1) for N in Ns]
    fs = [W.complex_normal(g, (1, N)) for N in Ns]
    B = NfftBatchPlan(Ms, Ns, nodes_dev(np.concatenate(xs)), precision="f64", kernel="dirichlet")
    B.precompute_B()
    cb = host(B.apply(dev(np.concatenate([a.ravel() for a in fs]), "f64")))
    o = 0
    for M, N, x, f in zip(Ms, Ns, xs, fs):
        P = NfftPlan((M,), nodes_dev(x), precision="f64", kernel="dirichlet")
        P.precompute_B()
        assert rel(cb[o:o + M], host(P.apply(dev(f, "f64")))[0]) <= 1e-15
        o += M
        P.close()
    B.close()
