"""The rest of the C ABI boundary on the GPU: plans in a caller-owned workspace (no device
allocation after creation, results equal to an ordinary plan's), B_opt exported and imported,
and the B optimisation with local problems beyond the register tiers under HIP graph capture
(the recorded pass replayed, and a stale record detected on the device)."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from oracle import bopt as obopt
from oracle import nfft as onfft

from gpu_util import check_columns, dev, host, nodes_dev, rel

pytestmark = pytest.mark.gpu


def clustered(d, seed):
    """Uniform nodes plus a dense spot: local problems of up to a few hundred members."""
    g = W.rng(seed)
    if d == 2:
        M, N, m, ncl, half = (32, 32), 900, 3, 400, 2.5
    else:
        M, N, m, ncl, half = (64,), 500, 4, 250, 2.0
    x = W.clustered_nodes(g, N, d, ncl, half / (2 * M[0]))
    fh = W.complex_normal(g, (2,) + M)
    f = W.complex_normal(g, (2, N))
    return M, N, m, x, fh, f


def run_path(P, fh, f, precision):
    out = {}
    out["trafo"] = host(P.trafo(dev(fh, precision)))
    out["adjoint"] = host(P.adjoint(dev(f, precision)))
    P.precompute_B()
    out["B"] = host(P.get_B())
    out["apply"] = host(P.apply(dev(f, precision)))
    out["apply_adjoint"] = host(P.apply_adjoint(dev(fh, precision)))
    out["grad_x"] = P.grad_x(dev(fh, precision), dev(f, precision)).cpu().numpy()
    out["grad_x_bopt"] = P.grad_x_bopt(dev(f, precision), dev(fh, precision)).cpu().numpy()
    return out


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("d", [1, 2])
def test_workspace_plan_matches_ordinary_plan_and_allocates_nothing(d, precision):
    from paper_1811_05335_amd import NfftPlan
    M, N, m, x, fh, f = clustered(d, 40 + d)
    p = onfft.Params(M, 2.0, m)
    assert obopt.Members(x, p).sizes().max() > (64 if d == 1 else 32)
    if precision == "f32":
        fh, f = W.round_to(fh, "f32"), W.round_to(f, "f32")
    ref = run_path(NfftPlan(M, nodes_dev(x), m=m, precision=precision, rho=1e-6, max_rhs=2), fh, f, precision)
    P = NfftPlan(M, nodes_dev(x), m=m, precision=precision, rho=1e-6, max_rhs=2, workspace=True, large_mib=128)
    nbytes = P.device_bytes()
    # inputs and outputs of the raw calls allocated first; then nothing on the device may change
    fh_d, f_d = dev(fh, precision), dev(f, precision)
    ct = fh_d.dtype
    outs = [torch.empty((2, N), dtype=ct, device="cuda"), torch.empty((2,) + M, dtype=ct, device="cuda"),
            torch.empty((2,) + M, dtype=ct, device="cuda"), torch.empty((2, N), dtype=ct, device="cuda"),
            torch.empty((N, d), dtype=torch.float64, device="cuda"),
            torch.empty((N, d), dtype=torch.float64, device="cuda")]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    from paper_1811_05335_amd import _lib
    lib = _lib.load()
    P._sync_stream()
    h = P._h
    vp = C.c_void_p
    for rep in range(2):
        _lib.check(lib.nfft_trafo(h, vp(fh_d.data_ptr()), vp(outs[0].data_ptr()), 2))
        _lib.check(lib.nfft_adjoint(h, vp(f_d.data_ptr()), vp(outs[1].data_ptr()), 2))
        _lib.check(lib.infft_precompute_B(h))
        _lib.check(lib.infft_apply(h, vp(f_d.data_ptr()), vp(outs[2].data_ptr()), 2))
        _lib.check(lib.infft_apply_adjoint(h, vp(fh_d.data_ptr()), vp(outs[3].data_ptr()), 2))
        _lib.check(lib.nfft_grad_x(h, vp(fh_d.data_ptr()), vp(f_d.data_ptr()), vp(outs[4].data_ptr()), 2))
        _lib.check(lib.infft_grad_x_bopt(h, vp(f_d.data_ptr()), vp(fh_d.data_ptr()), vp(outs[5].data_ptr()), 2))
    _lib.check(lib.infft_autotune(h, 2))
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert P.device_bytes() == nbytes
    st = P.status()
    assert st["failed_solves"] == 0 and st["oversized"] == 0
    P.bopt_version = P.nodes_version
    got = {"trafo": host(outs[0]), "adjoint": host(outs[1]), "B": host(P.get_B()), "apply": host(outs[2]),
           "apply_adjoint": host(outs[3]), "grad_x": outs[4].cpu().numpy(), "grad_x_bopt": outs[5].cpu().numpy()}
    # equal up to the order of the 2-D spreading's atomic sums
    tol = 1e-13 if precision == "f64" else 1e-6
    for k in got:
        assert rel(got[k], ref[k]) <= tol, k
    P.close()


def test_workspace_plan_reports_a_large_problem_that_does_not_fit():
    from paper_1811_05335_amd import InfftError, NfftPlan
    M, N, m, x, fh, f = clustered(2, 44)
    P = NfftPlan(M, nodes_dev(x), m=m, precision="f64", rho=1e-6, workspace=True, large_mib=1)
    with pytest.raises(InfftError, match="ENOMEM"):
        P.precompute_B()
    P.close()


def test_workspace_plan_ansatz1():
    from paper_1811_05335_amd import InfftError, NfftPlan
    g = W.rng(45)
    M, N = (256,), 64
    x = W.jittered_nodes_paper(g, N)
    f = W.complex_normal(g, (N,))
    P = NfftPlan(M, nodes_dev(x), m=3, precision="f32", rho=1e-10, kernel="dirichlet")
    P.precompute_Bstar()
    Q = NfftPlan(M, nodes_dev(x), m=3, precision="f32", rho=1e-10, kernel="dirichlet", workspace=True, ansatz1=True)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    Q.precompute_Bstar()
    Q.precompute_Bstar()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert rel(host(Q.get_B()), host(P.get_B())) <= 1e-13
    assert rel(host(Q.apply(dev(f, "f32"))), host(P.apply(dev(f, "f32")))) <= 1e-6
    R = NfftPlan(M, nodes_dev(x), m=3, precision="f32", rho=1e-10, kernel="dirichlet", workspace=True)
    with pytest.raises(InfftError, match="ESTATE"):
        R.precompute_Bstar()
    for pl in (P, Q, R):
        pl.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("d", [1, 2])
def test_export_import_round_trip(d, precision):
    from paper_1811_05335_amd import InfftError, NfftPlan
    M, N, m, x, fh, f = clustered(d, 46 + d)
    if precision == "f32":
        f = W.round_to(f, "f32")
    P = NfftPlan(M, nodes_dev(x), m=m, precision=precision, rho=1e-6, max_rhs=2)
    with pytest.raises(InfftError, match="ESTATE"):
        P.export_B()
    P.precompute_B()
    blob = P.export_B()
    # a plan made on other nodes takes the exported nodes and B_opt
    y = W.uniform_nodes(W.rng(3), N, d)
    Q = NfftPlan(M, nodes_dev(y), m=m, precision=precision, rho=1e-6, max_rhs=2)
    Q.import_B(blob)
    assert torch.equal(Q.get_B(), P.get_B())
    # the same up to the order of the 2-D spreading's atomic sums
    assert rel(host(Q.apply(dev(f, precision))), host(P.apply(dev(f, precision)))) <= (
        1e-13 if precision == "f64" else 1e-6)
    assert torch.equal(Q.trafo(dev(fh, precision) if precision == "f64" else dev(W.round_to(fh, "f32"), "f32")),
                       P.trafo(dev(fh, precision) if precision == "f64" else dev(W.round_to(fh, "f32"), "f32")))
    from paper_1811_05335_amd import infft
    infft(dev(f, precision), Q, Q._x)          # the imported nodes are the plan's
    # the blob is bound to its parameters
    R = NfftPlan(M, nodes_dev(x), m=m, precision=precision, rho=1e-8, max_rhs=2)
    with pytest.raises(InfftError, match="EINVAL"):
        R.import_B(blob)
    with pytest.raises(InfftError, match="EINVAL"):
        Q.import_B(blob[:-8])
    for pl in (P, Q, R):
        pl.close()


@pytest.mark.parametrize("d", [1, 2])
def test_captured_precompute_with_large_problems(d):
    """Recorded outside capture, the pass for problems beyond the register tiers replays under
    capture: every replay equals the eager B_opt with nothing oversized.  A replay whose record is
    no longer the plan's (an eager precompute has recorded since) is found stale on the device: the
    large problems get zero columns and are counted as oversized, the other columns are as before.
    A graph captured on the new record replays correctly; after other nodes are loaded, its replay
    finds the listed problems differ from its record and counts them as oversized."""
    from paper_1811_05335_amd import InfftError, NfftPlan
    M, N, m, x, fh, f = clustered(d, 50 + d)
    p = onfft.Params(M, 2.0, m)
    lim = 64 if d == 1 else 32
    mem = obopt.Members(x, p)
    sizes = mem.sizes()
    big = np.nonzero(sizes > lim)[0]
    assert len(big) > 0
    P = NfftPlan(M, nodes_dev(x), m=m, precision="f64", rho=1e-6)
    # no record yet: refused under capture, before anything is enqueued
    g0 = torch.cuda.CUDAGraph()
    with pytest.raises(InfftError, match="ESTATE"):
        with torch.cuda.graph(g0):
            P.precompute_B()
    del g0
    P.close()

    def capture():
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            P2.precompute_B()
        return gr

    P2 = NfftPlan(M, nodes_dev(x), m=m, precision="f64", rho=1e-6)
    P2.precompute_B()
    eager = P2.get_B().clone()
    graph = capture()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(P2.get_B(), eager), rep
        assert P2.status()["oversized"] == 0
        P2.trafo(dev(fh, "f64"))
    check_columns(x, p, 1e-6, mem, big[:6], host(eager))
    # an eager precompute records anew: the old graph's record is stale
    P2.precompute_B()
    graph.replay()
    assert P2.status()["oversized"] == len(big)
    rows, ref = host(P2.get_B()), host(eager)
    zero = np.zeros(rows.shape, dtype=bool)
    for l in big:
        js, ts, _ = mem.of(int(l))
        zero[js, ts] = True
    assert np.all(rows[zero] == 0) and np.array_equal(rows[~zero], ref[~zero])
    # a graph captured on the current record replays it
    P2.precompute_B()
    graph2 = capture()
    for rep in range(2):
        graph2.replay()
        torch.cuda.synchronize()
        assert torch.equal(P2.get_B(), eager), rep
        assert P2.status()["oversized"] == 0
    # other nodes: the listed problems differ from the record
    y = clustered(d, 60 + d)[3]
    nbig_y = int(np.sum(obopt.Members(y, p).sizes() > lim))
    P2.set_nodes(nodes_dev(y))
    graph2.replay()
    assert P2.status()["oversized"] == nbig_y > 0
    P2.close()


@pytest.mark.parametrize("d", [1, 2])
def test_fp32_plan_recomputes_its_fp64_bopt_and_keeps_the_record(d):
    """An FP32 plan's B optimisation keeps only the FP32 copy of B_opt; infft_get_B recomputes the
    FP64 values, which equal an FP64 plan's bit for bit (the same FP64 solver), without touching
    the FP32 copy (the apply is unchanged) and without replacing the record of the large-problem
    pass: a graph captured on that record still replays with nothing oversized."""
    from paper_1811_05335_amd import NfftPlan
    M, N, m, x, fh, f = clustered(d, 70 + d)
    p = onfft.Params(M, 2.0, m)
    assert obopt.Members(x, p).sizes().max() > (64 if d == 1 else 32)
    f32 = dev(W.round_to(f, "f32"), "f32")
    P64 = NfftPlan(M, nodes_dev(x), m=m, precision="f64", rho=1e-6)
    P32 = NfftPlan(M, nodes_dev(x), m=m, precision="f32", rho=1e-6)
    P64.precompute_B()
    P32.precompute_B()
    a0 = host(P32.apply(f32))
    B = P32.get_B()
    assert torch.equal(B, P64.get_B())
    # the 1-D spreading is a gather (bitwise repeatable); 2-D sums with atomics
    tol = 0.0 if d == 1 else 1e-6
    assert rel(host(P32.apply(f32)), a0) <= tol
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        P32.precompute_B()
    for rep in range(2):
        gr.replay()
        torch.cuda.synchronize()
        assert P32.status()["oversized"] == 0 and P32.status()["failed_solves"] == 0, rep
        assert rel(host(P32.apply(f32)), a0) <= tol, rep
        assert torch.equal(P32.get_B(), B), rep
    for pl in (P64, P32):
        pl.close()


@pytest.mark.parametrize("d", [1, 2])
def test_captured_precompute_on_an_empty_record(d):
    """Recorded on nodes without problems beyond the register tiers, a captured B optimisation has
    no large-problem pass to replay: its last tier counts such a problem as oversized and zeroes its
    column.  Nodes with large problems copied into the graph's node buffer give, on replay, zero
    columns for exactly those problems, counted as oversized, and elsewhere the B_opt of an eager
    precompute on the same nodes."""
    from paper_1811_05335_amd import NfftPlan
    M, N, m, x, fh, f = clustered(d, 80 + d)
    p = onfft.Params(M, 2.0, m)
    lim = 64 if d == 1 else 32
    y = W.uniform_nodes(W.rng(90 + d), N, d)
    assert obopt.Members(y, p).sizes().max() <= lim
    mem = obopt.Members(x, p)
    big = np.nonzero(mem.sizes() > lim)[0]
    assert len(big) > 0
    xbuf = nodes_dev(y)
    P = NfftPlan(M, xbuf, m=m, precision="f64", rho=1e-6)
    P.precompute_B()
    eager_y = P.get_B().clone()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        P.set_nodes(xbuf)
        P.precompute_B()
    for rep in range(2):
        gr.replay()
        torch.cuda.synchronize()
        assert torch.equal(P.get_B(), eager_y), rep
        assert P.status()["oversized"] == 0, rep
    Q = NfftPlan(M, nodes_dev(x), m=m, precision="f64", rho=1e-6)
    Q.precompute_B()
    ref = host(Q.get_B())
    xbuf.copy_(nodes_dev(x))
    gr.replay()
    torch.cuda.synchronize()
    assert P.status()["oversized"] == len(big)
    rows = host(P.get_B())
    zero = np.zeros(rows.shape, dtype=bool)
    for l in big:
        js, ts, _ = mem.of(int(l))
        zero[js, ts] = True
    assert np.all(rows[zero] == 0) and np.array_equal(rows[~zero], ref[~zero])
    for pl in (P, Q):
        pl.close()
