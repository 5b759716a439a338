"""Many 1-D problems of uneven sizes in one batch plan (every stage one launch for all problems):
each problem's results equal those of its own single-problem plan and match the FP64 oracle;
the batch step captured in a HIP graph replays like the eager step; and the full batched
workload (256 problems, M_i log-uniform in [1024, 16384], N_i = r_i M_i, 8 right-hand sides)
on sampled problems."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import bopt as obopt
from oracle import grad as ograd
from oracle import nfft as onfft

from gpu_util import check_columns, dev, host, nodes_dev, rel

pytestmark = pytest.mark.gpu

# sizes span one-pass FFTs and the two-pass split (2 M_i above 4096 for FP32, 2048 for FP64),
# mixed radices, and a tiny problem
SMALL_BATCH_M = [16, 40, 100, 256, 1152, 2304, 70, 500]
SMALL_BATCH_R = [2.0, 3.5, 1.5, 2.5, 1.7, 2.2, 4.0, 3.0]


def small_batch(seed, R):
    g = W.rng(seed)
    Ms = np.array(SMALL_BATCH_M, dtype=np.int64)
    Ns = np.round(np.array(SMALL_BATCH_R) * Ms).astype(np.int64)
    xs = [W.uniform_nodes(g, int(N), 1) for N in Ns]
    fhs = [W.complex_normal(g, (R, int(M))) for M in Ms]
    fs = [W.complex_normal(g, (R, int(N))) for N in Ns]
    return Ms, Ns, xs, fhs, fs


def flat(arrs):
    return np.concatenate([a.reshape(-1) for a in arrs])


def split(v, sizes, R):
    out, o = [], 0
    for n in sizes:
        out.append(v[o:o + R * n].reshape(R, n))
        o += R * n
    return out


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_matches_single_plans_and_oracle(precision):
    from paper_1811_05335_amd import NfftBatchPlan, NfftPlan
    R = 3
    Ms, Ns, xs, fhs, fs = small_batch(31, R)
    if precision == "f32":
        fhs = [W.round_to(a, "f32") for a in fhs]
        fs = [W.round_to(a, "f32") for a in fs]
    tol = 1e-12 if precision == "f64" else 1e-5
    xall = np.concatenate(xs)
    B = NfftBatchPlan(Ms, Ns, nodes_dev(xall), sigma=2.0, m=4, precision=precision, rho=1e-8, max_rhs=R)
    fb = host(B.trafo(dev(flat(fhs), precision)))
    hb = host(B.adjoint(dev(flat(fs), precision)))
    B.precompute_B()
    st = B.status()
    assert st["failed_solves"] == 0 and st["oversized"] == 0
    rows_b = host(B.get_B())
    cb = host(B.apply(dev(flat(fs), precision)))
    ab = host(B.apply_adjoint(dev(flat(fhs), precision)))
    gb = B.grad_x(dev(flat(fhs), precision), dev(flat(fs), precision)).cpu().numpy()[:, 0]
    f_s, h_s, c_s, a_s = split(fb, Ns, R), split(hb, Ms, R), split(cb, Ms, R), split(ab, Ns, R)
    no = np.concatenate([[0], np.cumsum(Ns)])
    for i, (M, N) in enumerate(zip(Ms, Ns)):
        M, N = int(M), int(N)
        P = NfftPlan((M,), nodes_dev(xs[i]), sigma=2.0, m=4, precision=precision, rho=1e-8, max_rhs=R)
        fh_d, f_d = dev(fhs[i], precision), dev(fs[i], precision)
        # the same kernels with the same per-problem parameters: identical results
        assert rel(f_s[i], host(P.trafo(fh_d))) <= 1e-15, i
        assert rel(h_s[i], host(P.adjoint(f_d))) <= 1e-15, i
        P.precompute_B()
        assert rel(rows_b[no[i]:no[i + 1]], host(P.get_B())) <= 1e-15, i
        assert rel(c_s[i], host(P.apply(f_d))) <= 1e-15, i
        assert rel(a_s[i], host(P.apply_adjoint(fh_d))) <= 1e-15, i
        assert rel(gb[no[i]:no[i + 1]], P.grad_x(fh_d, f_d).cpu().numpy()[:, 0]) <= 1e-15, i
        P.close()
        # and the oracle
        p = onfft.Params((M,), 2.0, 4)
        assert rel(f_s[i], onfft.trafo(xs[i], fhs[i], p)) <= tol, i
        assert rel(h_s[i], onfft.adjoint(xs[i], fs[i], p)) <= tol, i
        rows = rows_b[no[i]:no[i + 1]]
        if precision == "f32":
            rows = rows.astype(np.complex64).astype(np.complex128)
        assert rel(c_s[i], obopt.apply(xs[i], fs[i], rows, p)) <= tol, i
        assert rel(a_s[i], obopt.apply_adjoint(xs[i], fhs[i], rows, p)) <= tol, i
        gtol = 1e-10 if precision == "f64" else 1e-4
        assert rel(gb[no[i]:no[i + 1]], ograd.nfft_grad_x(xs[i], fhs[i], fs[i], p)[:, 0]) <= gtol, i
        if precision == "f64" and M <= 256:
            mem = obopt.Members(xs[i], p)
            check_columns(xs[i], p, 1e-8, mem, np.nonzero(mem.sizes())[0], rows_b[no[i]:no[i + 1]])
    B.close()


def test_batch_step_in_graph_matches_eager():
    from paper_1811_05335_amd import NfftBatchPlan
    R = 2
    Ms, Ns, xs, fhs, fs = small_batch(32, R)
    xd = nodes_dev(np.concatenate(xs))
    B = NfftBatchPlan(Ms, Ns, xd, sigma=2.0, m=4, precision="f32", rho=1e-8, max_rhs=R)
    fh = dev(flat(fhs), "f32")

    def step():
        f = B.trafo(fh)
        h = B.adjoint(f)
        B.precompute_B()
        fc = B.apply(f)
        fa = B.apply_adjoint(fc)
        gx = B.grad_x(fh, f)
        return f, h, fc, fa, gx

    eager = [o.cpu().numpy() for o in step()]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = step()
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip([o.cpu().numpy() for o in outs], eager):
            assert rel(a, b) <= 1e-6, rep
        _ = B.trafo(fh)
        torch.cuda.synchronize()
    B.close()


def test_batch_rejects_more_rhs_than_planned():
    from paper_1811_05335_amd import InfftError, NfftBatchPlan
    Ms, Ns, xs, fhs, fs = small_batch(33, 1)
    B = NfftBatchPlan(Ms[:3], Ns[:3], nodes_dev(np.concatenate(xs[:3])), precision="f64", max_rhs=1)
    two = dev(np.concatenate([np.tile(a, (2, 1)).reshape(-1) for a in fhs[:3]]), "f64")
    with pytest.raises((InfftError, ValueError)):
        B.trafo(two)
    B.close()


def test_full_batched_workload_every_problem():
    """256 problems, 8 right-hand sides, FP32 transforms and FP64 B optimisation: on every problem
    the NFFT, the adjoint, the modified adjoint (with the plan's B_opt), its adjoint and the node
    gradient against the FP64 oracle (FP32 transforms <= 1e-5, node gradient <= 1e-4), and four
    sampled columns of B_opt per problem (the largest local problem among them) against the
    oracle's Gram route with the conditioning-aware check."""
    from paper_1811_05335_amd import NfftBatchPlan
    cfg = W.CONFIGS["c4"]
    R = cfg["rhs"]
    Ms, Ns, xs, fhs = W.make_batch(cfg, seed=0)
    fhs32 = [W.round_to(a, "f32") for a in fhs]
    g = W.rng(21)
    gfs32 = [W.round_to(W.complex_normal(g, (R, int(N))), "f32") for N in Ns]
    B = NfftBatchPlan(Ms, Ns, nodes_dev(np.concatenate(xs)), sigma=cfg["sigma"], m=cfg["m"], precision="f32",
                      rho=cfg["rho"], max_rhs=R)
    fh_d = dev(flat(fhs32), "f32")
    gf_d = dev(flat(gfs32), "f32")
    f = B.trafo(fh_d)
    h = host(B.adjoint(gf_d))
    B.precompute_B()
    st = B.status()
    assert st["failed_solves"] == 0 and st["oversized"] == 0
    fc = host(B.apply(gf_d))
    fa = host(B.apply_adjoint(fh_d))
    gx = B.grad_x(fh_d, gf_d).cpu().numpy()[:, 0]
    rows_b = host(B.get_B())
    f_s, h_s, c_s, a_s = split(host(f), Ns, R), split(h, Ms, R), split(fc, Ms, R), split(fa, Ns, R)
    no = np.concatenate([[0], np.cumsum(Ns)])
    worst = {}
    for i in range(len(Ms)):
        p = onfft.Params((int(Ms[i]),), cfg["sigma"], cfg["m"])
        rows = rows_b[no[i]:no[i + 1]]
        rows32 = rows.astype(np.complex64).astype(np.complex128)
        errs = {
            "trafo": rel(f_s[i], onfft.trafo(xs[i], fhs32[i], p)),
            "adjoint": rel(h_s[i], onfft.adjoint(xs[i], gfs32[i], p)),
            "apply": rel(c_s[i], obopt.apply(xs[i], gfs32[i], rows32, p)),
            "apply_adjoint": rel(a_s[i], obopt.apply_adjoint(xs[i], fhs32[i], rows32, p)),
        }
        for k, e in errs.items():
            assert e <= 1e-5, (i, k, e)
        eg = rel(gx[no[i]:no[i + 1]], ograd.nfft_grad_x(xs[i], fhs32[i], gfs32[i], p)[:, 0])
        assert eg <= 1e-4, (i, "grad_x", eg)
        errs["grad_x"] = eg
        for k, e in errs.items():
            worst[k] = max(worst.get(k, 0.0), e)
        mem = obopt.Members(xs[i], p)
        sizes = mem.sizes()
        nz = np.nonzero(sizes)[0]
        ls = list(W.rng(i).choice(nz, size=3, replace=False)) + [int(nz[np.argmax(sizes[nz])])]
        check_columns(xs[i], p, cfg["rho"], mem, ls, rows)
    print("worst relative errors over the 256 problems:", worst, flush=True)
    B.close()
