"""Throughput of the direct inverse NFFT hot path on one MI355X.

One step = one pass of the whole path over one node set and one coefficient batch:
  node preprocessing (wrap, stencil, sort into tiles, I(l) lists)
  NFFT                     f  = B F D fhat
  adjoint NFFT             h  = D^* F^* B^* f
  optimisation of B        Algorithm 3.17 (FP64 local least squares)
  modified adjoint NFFT    fc = D^* F^* B_opt^* f        (the inverse NFFT, (3.32))
  backward kernels         B_opt F D h (gradient of the modified adjoint) and the node gradient

value = nodes * right-hand sides / step time, inputs resident on the GPU.  The same step runs in
FP32 (complex64 spreading and FFT; the B solves stay FP64) and in FP64; the FP32 figure is the
headline `value`.  The CPU baseline times the FP64 oracle on this host (the B optimisation on a
sample of grid indices, scaled) and its outputs give the relative errors of the GPU results.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

WORKLOAD = dict(W.CONFIGS["c2"])
WORKLOAD_NAME = "1-D jittered nodes, M=2^16, N=2^17, sigma=2, Kaiser-Bessel m=6"

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rhs", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=48, help="grid indices of the sampled oracle B solve")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of a graph replay")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the plans' default FFT workgroup shapes and spreading chunk (profiling: the "
                         "autotuner's timings are perturbed under a profiler)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run every call on the main stream (same as --overlap none)")
    ap.add_argument("--overlap", choices=("none", "pre", "tail", "full"), default="none",
                    help="none: one stream (the fastest replay: the B optimisation's first solve fills "
                         "every CU, so branches gain little and cost cross-queue waits); pre: the B "
                         "optimisation on a second stream; tail: also the node gradient beside the "
                         "inverse adjoint (own stream and work slot); full: the adjoint and the node "
                         "gradient on their own streams and work slots from the start")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one device-to-device copy of this size first (counter calibration under a profiler)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the batched and polar workloads reported beside the headline")
    ap.add_argument("--leg", choices=("rhs8", "batched", "polar", "spiral", "small", "ansatz1", "variants"),
                    help="run only this workload beside the headline and print its figures as one JSON line "
                         "(for profiling one workload; not a bench line)")
    ap.add_argument("--fp64", dest="fp64", action="store_true", default=True)
    ap.add_argument("--no-fp64", dest="fp64", action="store_false")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


class Stage:
    """Elapsed time of one library call, from events on the plan's (torch's current) stream."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {}

    def run(self, name, fn):
        s = self.torch.cuda.Event(enable_timing=True)
        e = self.torch.cuda.Event(enable_timing=True)
        s.record()
        out = fn()
        e.record()
        self.pairs.setdefault(name, []).append((s, e))
        return out

    def mean_ms(self):
        return {k: float(np.mean([s.elapsed_time(e) for s, e in v])) for k, v in self.pairs.items()}


def gpu_run(precision, x, fh, gf, steps, warmup, rho, m, sigma, M, use_graph=True, overlap="full", autotune=True):
    import torch
    from paper_1811_05335_amd import NfftPlan

    ct = torch.complex64 if precision == "f32" else torch.complex128
    xd = torch.from_numpy(x).cuda()
    fhd = torch.from_numpy(fh).to(ct).cuda()
    gfd = torch.from_numpy(gf).to(ct).cuda()
    R = fh.shape[0]
    P = NfftPlan(M, xd, sigma=sigma, m=m, precision=precision, rho=rho, max_rhs=R, work_slots=3)
    tuned = P.autotune() if autotune else {}   # FFT workgroup shapes, measured once per plan like an FFT plan

    side, s_adj, s_grad = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()

    def step(stage=None):
        """One pass of the path.  overlap "none" (the default) runs every call on one stream, the
        NFFT's node gradient right after the NFFT from the grid it left.  The other modes overlap
        the calls that do not depend on each other: the B optimisation (nodes only, none of the
        transforms' buffers) on a second stream, joined before the modified adjoint; the adjoint
        of the NFFT's output on a third stream and work slot; the node gradient on a fourth."""
        run = (lambda n, f: stage.run(n, f)) if stage else (lambda n, f: f())
        cur = torch.cuda.current_stream()
        pre = stage is None and overlap in ("pre", "tail", "full")
        par = stage is None and overlap == "full"
        tail = stage is None and overlap == "tail"
        P.set_slot(0)
        run("a1_nodes", lambda: P.set_nodes(xd))
        if pre:
            side.wait_stream(cur)
            with torch.cuda.stream(side):
                P.precompute_B()
        if par:
            s_grad.wait_stream(cur)
            with torch.cuda.stream(s_grad):
                P.set_slot(2)
                gx = P.grad_x(fhd, gfd)
            P.set_slot(0)
        f = run("a2-a4_trafo", lambda: P.trafo(fhd))
        serial = not (pre or par or tail)
        if serial:
            # the NFFT's node gradient from the grid the NFFT just left (its backward, without a
            # second FFT of fhat)
            gx = run("a8_grad_x", lambda: P.grad_x_after_trafo(gfd))
        if par:
            s_adj.wait_stream(cur)
            with torch.cuda.stream(s_adj):
                P.set_slot(1)
                h = P.adjoint(f)
            P.set_slot(0)
        else:
            h = run("a5_adjoint", lambda: P.adjoint(f))
        if pre:
            cur.wait_stream(side)
        else:
            run("a6_precompute_B", lambda: P.precompute_B())
        fc = run("a7_apply", lambda: P.apply(f))
        if tail:
            s_grad.wait_stream(cur)
            with torch.cuda.stream(s_grad):
                P.set_slot(2)
                gx = P.grad_x(fhd, gfd)
            P.set_slot(0)
        fa = run("a8_apply_adjoint", lambda: P.apply_adjoint(fc))
        if par:
            cur.wait_stream(s_adj)
        if par or tail:
            cur.wait_stream(s_grad)
        elif not serial:
            gx = run("a8_grad_x", lambda: P.grad_x(fhd, gfd))
        return f, h, fc, fa, gx

    # eager launches
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        eager_outs = step()
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / steps
    # per-call breakdown, eager, in a separately timed loop
    st = Stage(torch)
    for _ in range(max(3, min(steps, 20))):
        step(st)
    torch.cuda.synchronize()
    eager_host = [o.cpu().numpy() for o in eager_outs]
    ms_graph, graph_dev = None, None
    if use_graph:
        warm = torch.cuda.Stream()
        warm.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(warm):
            for _ in range(2):
                step()
        torch.cuda.current_stream().wait_stream(warm)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            gouts = step()
        for _ in range(warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            graph.replay()
        torch.cuda.synchronize()
        ms_graph = (time.perf_counter() - t0) * 1e3 / steps
        graph_host = [o.cpu().numpy() for o in gouts]
        graph_dev = max(rel(a, b) for a, b in zip(graph_host, eager_host))
        # per replay with HIP events, warm (back to back) and with the last-level cache flushed
        # before each replay (a 512 MiB write between replays, outside the events)
        warm_ms, flushed_ms = replay_times(torch, graph, max(10, min(steps, 20)))
    # per kernel class: average launch duration from HIP events the library records around each
    # launch on the plan's stream (eager launches, one class at a time)
    kclass = {}
    for cls in ("solve", "fft", "spread", "interp", "nodes"):
        P.profile_begin(cls)
        nsteps = max(3, min(steps, 20))
        for _ in range(nsteps):
            step()
        tot_ms, nl = P.profile_end()
        kclass[cls] = dict(ms_per_step=tot_ms / nsteps, launches_per_step=nl / nsteps,
                           ms_per_launch=tot_ms / max(nl, 1))
    status = P.status()
    rows = P.get_B().cpu().numpy()
    torch.cuda.synchronize()
    P.close()
    return dict(ms_eager=ms_eager, ms_graph=ms_graph, breakdown=st.mean_ms(), status=status, outs=eager_host,
                rows=rows, graph_vs_eager=graph_dev, kclass=kclass, tuned=tuned,
                replay_warm_ms=warm_ms if use_graph else None, replay_flushed_ms=flushed_ms if use_graph else None)


FLUSH_BYTES = 512 << 20   # twice the 256 MB Infinity Cache (MALL)


def replay_times(torch, graph, reps):
    """Median milliseconds of one graph replay timed with events on the current stream: warm
    (replays back to back) and flushed (a 512 MiB buffer written between replays, so the step's
    inputs and tables come from HBM rather than the MALL)."""
    buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda")
    out = {}
    for mode in ("warm", "flushed"):
        ts = []
        for _ in range(reps):
            if mode == "flushed":
                buf.fill_(1.0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            graph.replay()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        out[mode] = float(np.median(ts))
    del buf
    return out["warm"], out["flushed"]


def algorithmic_bytes(N, M, G, T, R, csize, wsize):
    """Bytes each operation must move at least once (inputs, outputs, the oversampled grid written
    and read once, stored weights once)."""
    return {
        "a2-a4_trafo": R * (M * csize + 2 * G * csize + N * csize) + N * 8,
        "a5_adjoint": R * (N * csize + 2 * G * csize + M * csize) + N * 8,
        "a7_apply": R * (N * csize + 2 * G * csize + M * csize) + N * (T * wsize + 4),
        "a8_apply_adjoint": R * (M * csize + 2 * G * csize + N * csize) + N * (T * wsize + 4),
    }


def member_counts(x, Ms, m):
    """|I(l)| for every grid index l (1-D), from the stencil l0 = ceil(x M_sigma - m), u = x M_sigma - l0:
    the cells l-2m+1..l contribute all their nodes, the cell l-2m those with |u - 2m| <= m."""
    xw = x[:, 0] - np.floor(x[:, 0] + 0.5)
    t = xw * Ms
    l0 = np.ceil(t - m)
    u = t - l0
    c = np.mod(l0.astype(np.int64), Ms)
    cnt = np.bincount(c, minlength=Ms)
    edge = np.bincount(c[np.abs(u - 2 * m) <= m], minlength=Ms)
    n = np.zeros(Ms, dtype=np.int64)
    for tau in range(2 * m):
        n += np.roll(cnt, tau)
    n += np.roll(edge, 2 * m)
    return n


def solve_traffic(precision):
    """Measured HBM bytes per launch of the solve kernel, from the committed counter summary, or None
    once the kernel source differs from the one the counters were taken on."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "k_solve_t1_c2_hbm.md")
    src = os.path.join(ROOT, "paper_1811_05335_amd", "csrc", "solve.hip")
    try:
        text = open(path).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    mh = re.search(r"source_sha256: ([0-9a-f]{64})", text)
    mt = re.search(r"traffic_bytes_per_launch_%s: ([0-9]+)" % precision, text)
    if not mh or not mt or mh.group(1) != digest:
        return None
    return int(mt.group(1))


def solve_flops(n):
    """FP64 flops of one local problem as the 1-D kernel computes it (real Sherman-Morrison form):
    Gram entries n(n+1)/2 Taylor evaluations (10 fma), right-hand side n (10 fma), Cholesky n^3/3,
    three right-hand sides forward (3 n^2) and two back (2 n^2), combination 10 n."""
    n = np.asarray(n, dtype=np.float64)
    return n * (n + 1) / 2 * 20 + n * 20 + n ** 3 / 3 + 5 * n ** 2 + 10 * n


def timed_graph(torch, fn, steps, warmup):
    """Milliseconds per call of fn replayed from a HIP graph (fn captured once)."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fn()
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def class_ms(P, cls, fn, reps):
    """Average launch time of one kernel class inside fn (HIP events on the plan's stream)."""
    P.profile_begin(cls)
    for _ in range(reps):
        fn()
    tot, n = P.profile_end()
    return tot / max(n, 1), n / reps


def secondary_batched(steps, warmup):
    """The batched workload: 256 uneven 1-D problems, 8 right-hand sides, FP32 transforms."""
    import torch
    from paper_1811_05335_amd import NfftBatchPlan
    cfg = W.CONFIGS["c4"]
    R, m = cfg["rhs"], cfg["m"]
    Ms, Ns, xs, fhs = W.make_batch(cfg, seed=0)
    P_, N_ = int(Ms.sum()), int(Ns.sum())
    G_ = 2 * P_
    xd = torch.from_numpy(np.concatenate(xs)).cuda()
    fh = torch.from_numpy(np.concatenate([W.round_to(a, "f32").reshape(-1) for a in fhs])).to(torch.complex64).cuda()
    B = NfftBatchPlan(Ms, Ns, xd, sigma=cfg["sigma"], m=m, precision="f32", rho=cfg["rho"], max_rhs=R)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.precompute_B()
    torch.cuda.synchronize()
    t_pre = (time.perf_counter() - t0) * 1e3
    f = B.trafo(fh)
    out = {}
    out["ms_trafo"] = timed_graph(torch, lambda: B.trafo(fh), steps, warmup)
    out["ms_adjoint"] = timed_graph(torch, lambda: B.adjoint(f), steps, warmup)
    out["ms_apply"] = timed_graph(torch, lambda: B.apply(f), steps, warmup)
    out["ms_apply_adjoint"] = timed_graph(torch, lambda: B.apply_adjoint(fh), steps, warmup)
    out["ms_precompute_graph"] = timed_graph(torch, lambda: B.precompute_B(), max(3, steps // 4), 1)
    out["ms_precompute_eager_first"] = t_pre
    T, c, wB = 2 * m + 1, 8, 8
    # bytes each call must move at least once (the oversampled grid written and read once)
    alg = {
        "trafo": R * (P_ * c + 2 * G_ * c + N_ * c) + N_ * 12,
        "adjoint": R * (N_ * c + 2 * G_ * c + P_ * c) + N_ * 12,
        "apply": R * (N_ * c + 2 * G_ * c + P_ * c) + N_ * (T * wB + 4),
        "apply_adjoint": R * (P_ * c + 2 * G_ * c + N_ * c) + N_ * (T * wB + 4),
    }
    for k, b in alg.items():
        ms = out["ms_" + k]
        out["hbm_frac_" + k] = b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    # the spreading kernel of the modified adjoint: samples and B_opt read once, grid written once
    ms_sp, _ = class_ms(B, "spread", lambda: B.apply(f), 5)
    sp_bytes = R * N_ * c + N_ * (T * wB + 8) + R * G_ * c
    out["spread_apply_kernel"] = dict(ms=ms_sp, bytes=sp_bytes, GBps=sp_bytes / (ms_sp * 1e-3) / 1e9,
                                      frac=sp_bytes / (ms_sp * 1e-3) / 1e9 / HBM_PEAK_GBS)
    ms_ad, _ = class_ms(B, "spread", lambda: B.adjoint(f), 5)
    ad_bytes = R * N_ * c + N_ * 16 + R * G_ * c
    out["spread_adjoint_kernel"] = dict(ms=ms_ad, bytes=ad_bytes, GBps=ad_bytes / (ms_ad * 1e-3) / 1e9,
                                        frac=ad_bytes / (ms_ad * 1e-3) / 1e9 / HBM_PEAK_GBS)
    st = B.status()
    out["status"] = {k: st[k] for k in ("failed_solves", "oversized", "min_members", "max_members")}
    out["nodes_per_s_trafo_plus_apply"] = N_ * R / ((out["ms_trafo"] + out["ms_apply"]) * 1e-3)
    out["config"] = dict(problems=len(Ms), sum_M=P_, sum_N=N_, rhs=R, m=m, sigma=cfg["sigma"], dtype="f32")
    B.close()
    return out


def secondary_rhs8(steps, warmup):
    """The 1-D jittered workload with 8 right-hand sides (FP32): per-call graph replays and the
    spreading kernels against their algorithmic bytes, where R amortises the node data."""
    import torch
    from paper_1811_05335_amd import NfftPlan
    cfg = W.CONFIGS["c2"]
    R, m = 8, cfg["m"]
    x, fh = W.make_problem(cfg, seed=0, rhs=R)
    N, M = cfg["N"], cfg["M"][0]
    G = 2 * M
    xd = torch.from_numpy(x).cuda()
    fhd = torch.from_numpy(W.round_to(fh, "f32")).to(torch.complex64).cuda()
    P = NfftPlan(cfg["M"], xd, sigma=cfg["sigma"], m=m, precision="f32", rho=cfg["rho"], max_rhs=R)
    P.autotune()
    P.precompute_B()
    f = P.trafo(fhd)
    fc = P.apply(f)
    out = {"rhs": R}
    out["ms_trafo"] = timed_graph(torch, lambda: P.trafo(fhd), steps, warmup)
    out["ms_adjoint"] = timed_graph(torch, lambda: P.adjoint(f), steps, warmup)
    out["ms_apply"] = timed_graph(torch, lambda: P.apply(f), steps, warmup)
    out["ms_apply_adjoint"] = timed_graph(torch, lambda: P.apply_adjoint(fc), steps, warmup)
    T, c = 2 * m + 1, 8
    # spreading: samples, stencil base and offset (or the B_opt row) read once, the grid written once
    for name, fn, wbytes in (("spread_adjoint_kernel", lambda: P.adjoint(f), 12),
                             ("spread_apply_kernel", lambda: P.apply(f), T * 8 + 4)):
        ms_k, _ = class_ms(P, "spread", fn, 10)
        b = R * N * c + N * wbytes + R * G * c
        out[name] = dict(ms=ms_k, bytes=b, GBps=b / (ms_k * 1e-3) / 1e9, frac=b / (ms_k * 1e-3) / 1e9 / HBM_PEAK_GBS)
    out["nodes_rhs_per_s_trafo_plus_apply"] = N * R / ((out["ms_trafo"] + out["ms_apply"]) * 1e-3)
    P.close()
    return out


def secondary_polar(steps, warmup):
    """The polar trajectory: M = 512 x 512, N = 524288, FP32 transforms, FP64 B optimisation."""
    import torch
    from paper_1811_05335_amd import NfftPlan
    cfg = W.CONFIGS["c3"]
    x, fh = W.make_problem(cfg, seed=0, rhs=1)
    xd = torch.from_numpy(x).cuda()
    fhd = torch.from_numpy(W.round_to(fh, "f32")).to(torch.complex64).cuda()
    P = NfftPlan(cfg["M"], xd, sigma=cfg["sigma"], m=cfg["m"], precision="f32", rho=cfg["rho"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.precompute_B()
    torch.cuda.synchronize()
    out = {"ms_precompute": (time.perf_counter() - t0) * 1e3}
    f = P.trafo(fhd)
    out["ms_trafo"] = timed_graph(torch, lambda: P.trafo(fhd), steps, warmup)
    out["ms_adjoint"] = timed_graph(torch, lambda: P.adjoint(f), steps, warmup)
    out["ms_apply"] = timed_graph(torch, lambda: P.apply(f), steps, warmup)
    N, G, Pc, T = cfg["N"], 1024 * 1024, 512 * 512, 81
    ms_sp, _ = class_ms(P, "spread", lambda: P.apply(f), 5)
    sp_bytes = N * 8 + N * (T * 8 + 8) + G * 8
    out["spread_apply_kernel"] = dict(ms=ms_sp, bytes=sp_bytes, GBps=sp_bytes / (ms_sp * 1e-3) / 1e9,
                                      frac=sp_bytes / (ms_sp * 1e-3) / 1e9 / HBM_PEAK_GBS)
    st = P.status()
    out["status"] = {k: st[k] for k in ("failed_solves", "oversized", "min_members", "max_members")}
    out["nodes_per_s_trafo_plus_apply"] = N / ((out["ms_trafo"] + out["ms_apply"]) * 1e-3)
    P.close()
    return out


def secondary_spiral(steps, warmup):
    """The differentiable spiral: M = 256 x 256, N = 65536 on a 32-interleave spiral, 16 right-hand
    sides (FP32), loss ||infft(nfft(fhat, x)) - fhat||^2 with gradients for fhat and x."""
    import torch
    from paper_1811_05335_amd import NfftPlan, infft, nfft
    cfg = W.CONFIGS["c5"]
    R = cfg["rhs"]
    x, fh = W.make_problem(cfg, seed=0, rhs=R)
    xd = torch.from_numpy(x).cuda()
    fhd = torch.from_numpy(W.round_to(fh, "f32")).to(torch.complex64).cuda()
    P = NfftPlan(cfg["M"], xd, sigma=cfg["sigma"], m=cfg["m"], precision="f32", rho=cfg["rho"], max_rhs=R)
    Pi = NfftPlan(cfg["M"], xd, sigma=cfg["sigma"], m=cfg["m"], precision="f32", rho=cfg["rho"], max_rhs=R)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Pi.precompute_B()
    torch.cuda.synchronize()
    out = {"ms_precompute": (time.perf_counter() - t0) * 1e3}

    def it():
        a = fhd.clone().requires_grad_(True)
        xx = xd.clone().requires_grad_(True)
        loss = (infft(nfft(a, xx, P), Pi) - a).abs().pow(2).sum()
        loss.backward()
        return loss, a.grad, xx.grad

    for _ in range(warmup):
        it()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        loss, ga, gx = it()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    st = Pi.status()
    out.update(ms_loss_and_gradients=ms, node_rhs_per_s=cfg["N"] * R / (ms * 1e-3),
               relative_residual=float(loss.item()) ** 0.5 / float(fhd.abs().pow(2).sum().item()) ** 0.5,
               timing="eager autograd (forward NFFT and modified adjoint, backward adjoint NFFT, node "
                      "gradient and inverse adjoint)",
               status={k: st[k] for k in ("failed_solves", "oversized", "min_members", "max_members")})
    P.close()
    Pi.close()
    return out


def secondary_variants(steps, warmup):
    """Rows beside the headline path, at its workload (1-D jittered, M = 2^16, N = 2^17, FP32
    transforms, FP64 solves): the Dirichlet-kernel variant of Algorithm 3.17 (B optimisation and
    modified adjoint, graph replays) next to the window kernel, and the node gradient through
    B_opt(x) (eager: the call reads the sizes of problems above 32 members back)."""
    import torch
    from paper_1811_05335_amd import NfftPlan
    cfg = W.CONFIGS["c2"]
    x, _ = W.make_problem(cfg, seed=0, rhs=1)
    g = W.rng(7)
    xd = torch.from_numpy(x).cuda()
    fd = torch.from_numpy(W.round_to(W.complex_normal(g, (1, cfg["N"])), "f32")).to(torch.complex64).cuda()
    gcd = torch.from_numpy(W.round_to(W.complex_normal(g, (1,) + tuple(cfg["M"])), "f32")).to(torch.complex64).cuda()
    out = {}
    for kernel in ("window", "dirichlet"):
        P = NfftPlan(cfg["M"], xd, sigma=cfg["sigma"], m=cfg["m"], precision="f32", rho=cfg["rho"], max_rhs=1,
                     kernel=kernel)
        P.autotune()
        ms_pre = timed_graph(torch, P.precompute_B, steps, warmup)
        ms_apply = timed_graph(torch, lambda: P.apply(fd), steps, warmup)
        ms_apply_adj = timed_graph(torch, lambda: P.apply_adjoint(gcd), steps, warmup)
        st = P.status()
        r = dict(ms_precompute_B=ms_pre, ms_apply=ms_apply, ms_apply_adjoint=ms_apply_adj,
                 failed_solves=st["failed_solves"])
        if kernel == "window":
            for _ in range(warmup):
                P.grad_x_bopt(fd, gcd)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                P.grad_x_bopt(fd, gcd)
            torch.cuda.synchronize()
            r["ms_grad_x_bopt"] = (time.perf_counter() - t0) * 1e3 / steps
        out[kernel] = r
        P.close()
    out["timing"] = "graph replays per call; the node gradient through B_opt(x) eager"
    return out


def secondary_small(steps, warmup):
    """The small 1-D uniform workload (M = 256, N = 512, m = 4, FP64): the whole path per step."""
    import torch
    from paper_1811_05335_amd import NfftPlan
    cfg = W.CONFIGS["c1"]
    x, fh = W.make_problem(cfg, seed=0, rhs=1)
    xd = torch.from_numpy(x).cuda()
    fhd = torch.from_numpy(fh).cuda()
    P = NfftPlan(cfg["M"], xd, sigma=cfg["sigma"], m=cfg["m"], precision="f64", rho=cfg["rho"])

    def step():
        P.set_nodes(xd)
        f = P.trafo(fhd)
        P.adjoint(f)
        P.precompute_B()
        fc = P.apply(f)
        P.apply_adjoint(fc)
        P.grad_x(fhd, f)

    ms = timed_graph(torch, step, steps, warmup)
    P.close()
    return {"ms_per_step": ms, "nodes_per_s": cfg["N"] / (ms * 1e-3), "dtype": "f64",
            "timing": "hipGraph replay of the whole path (launch-latency bound at this size)"}


def secondary_ansatz1(steps, warmup):
    """Algorithm 3.10 (ansatz 1) at Example 3.14's largest case and at GPU scale (Dirichlet kernel,
    sigma 2, m 4, M = 4N, FP64): the precompute of B_opt^* (eager: it creates inner plans on first
    use and is not capturable), then the estimate f_check and the inverse adjoint (graph replays),
    and the relative residual ||A f_check - f|| / ||f|| with A applied by the plan's NFFT."""
    import torch
    from paper_1811_05335_amd import NfftPlan
    out = {}
    for name in ("a1", "a1_large"):
        cfg = W.CONFIGS[name]
        x, fh = W.make_problem(cfg, seed=0, rhs=1)
        xd = torch.from_numpy(x).cuda()
        P = NfftPlan(cfg["M"], xd, sigma=cfg["sigma"], m=cfg["m"], precision="f64", rho=cfg["rho"],
                     kernel=cfg["kernel"])
        f = P.trafo(torch.from_numpy(fh).cuda())
        P.precompute_Bstar()            # first call: inner plans
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        reps = max(3, steps // 4)
        ev[0].record()
        for _ in range(reps):
            P.precompute_Bstar()
        ev[1].record()
        torch.cuda.synchronize()
        pre_ms = ev[0].elapsed_time(ev[1]) / reps
        st = P.status()
        fc = P.apply(f)
        ap_ms = timed_graph(torch, lambda: P.apply(f), steps, warmup)
        ad_ms = timed_graph(torch, lambda: P.apply_adjoint(fc), steps, warmup)
        res = float(torch.linalg.vector_norm(P.trafo(fc) - f) / torch.linalg.vector_norm(f))
        out[name] = {"N": cfg["N"], "M": cfg["M"][0], "m": cfg["m"], "kernel": cfg["kernel"],
                     "precompute_ms": pre_ms, "apply_ms": ap_ms, "apply_adjoint_ms": ad_ms,
                     "nodes_per_s_precompute": cfg["N"] / (pre_ms * 1e-3),
                     "failed_solves": st["failed_solves"], "residual": res}
        P.close()
    return out


def cpu_description():
    """Host CPU: logical cores, model name and the thread settings the oracle runs under."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh_:
            for ln in fh_:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        pools = [{"api": d.get("internal_api"), "threads": d.get("num_threads")} for d in threadpool_info()]
    except Exception:
        pools = []
    return {"os_cpu_count": os.cpu_count(), "model": model, "thread_pools": pools,
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"),
            "fft": "numpy.fft (pocketfft, one thread)"}


def cpu_baseline(x, fh, gf, rho, m, sigma, M, sample):
    """The FP64 oracle as it stands on this host's cores, twice: with every BLAS thread and with one.
    The NFFT, adjoint, modified adjoint, its adjoint and the node gradient run in full; the B
    optimisation runs the Gram route (closed-form normal equations by direct O(M) sums, then a
    dense solve) on `sample` grid indices and its time is scaled to all of them."""
    from contextlib import nullcontext
    from oracle import bopt, grad, nfft
    from threadpoolctl import threadpool_info, threadpool_limits

    p = nfft.Params(M, sigma, m)
    mem = bopt.Members(x, p)
    g = np.random.default_rng(1)
    ls = np.sort(g.choice(mem.G, size=min(sample, mem.G), replace=False))
    runs = {}
    for label, nthreads in (("all_cores", None), ("one_thread", 1)):
        with (threadpool_limits(limits=nthreads) if nthreads else nullcontext()):
            threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
            t = {}
            c0 = time.perf_counter()
            f = nfft.trafo(x, fh, p)
            t["trafo"] = time.perf_counter() - c0
            c0 = time.perf_counter()
            h = nfft.adjoint(x, f, p)
            t["adjoint"] = time.perf_counter() - c0
            c0 = time.perf_counter()
            rows, solved = bopt.bopt_rows(x, p, rho, route="G", ls=ls, members=mem)
            t_s = time.perf_counter() - c0
            t["precompute_B_sampled"] = t_s
            t["precompute_B_scaled"] = t_s * mem.G / len(ls)
            c0 = time.perf_counter()
            fc = bopt.apply(x, f, rows, p)
            t["apply"] = time.perf_counter() - c0
            c0 = time.perf_counter()
            bopt.apply_adjoint(x, fc, rows, p)
            t["apply_adjoint"] = time.perf_counter() - c0
            c0 = time.perf_counter()
            gx = grad.nfft_grad_x(x, fh, gf, p)
            t["grad_x"] = time.perf_counter() - c0
            total = (t["trafo"] + t["adjoint"] + t["precompute_B_scaled"] + t["apply"] + t["apply_adjoint"]
                     + t["grad_x"])
            runs[label] = dict(total_s=total, parts_s=t, threads=threads)
    return dict(runs=runs, sample=len(ls), f=f, h=h, ls=ls, solved=solved, rows=rows, gx=gx, p=p)


def main():
    a = parse()
    ovl = "none" if a.no_overlap else a.overlap
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (the path has no multi-GPU mode); --gpus must be 1"}))
        sys.exit(2)
    if a.copy_calibration_mb:
        import torch
        src = torch.ones(a.copy_calibration_mb * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.leg:
        legs = {"rhs8": lambda: secondary_rhs8(max(10, a.steps), 3),
                "batched": lambda: secondary_batched(max(5, a.steps // 2), 2),
                "polar": lambda: secondary_polar(max(5, a.steps // 2), 2),
                "spiral": lambda: secondary_spiral(5, 1),
                "small": lambda: secondary_small(max(20, a.steps), 3),
                "ansatz1": lambda: secondary_ansatz1(max(10, a.steps), 3),
                "variants": lambda: secondary_variants(max(10, a.steps // 2), 3)}
        print(json.dumps({"leg": a.leg, "figures": legs[a.leg]()}, default=str))
        return
    cfg = WORKLOAD
    M, N, sigma, m, rho = cfg["M"], cfg["N"], cfg["sigma"], cfg["m"], cfg["rho"]
    R = a.rhs
    x, fh = W.make_problem(cfg, seed=0, rhs=R)
    gf = W.complex_normal(W.rng(1), (R, N))
    fh32 = W.round_to(fh, "f32")
    gf32 = W.round_to(gf, "f32")
    log(f"[bench] workload: {WORKLOAD_NAME}, rhs={R}; FP32 run")
    r32 = gpu_run("f32", x, fh32, gf32, a.steps, a.warmup, rho, m, sigma, M, use_graph=not a.eager,
                  overlap=ovl, autotune=a.autotune)
    ms32 = r32["ms_graph"] if r32["ms_graph"] else r32["ms_eager"]
    br32, st32, out32, rows32 = r32["breakdown"], r32["status"], r32["outs"], r32["rows"]
    log(f"[bench] FP32 graph {r32['ms_graph']} ms/step, eager {r32['ms_eager']:.3f} ms/step {br32}")
    res64 = None
    if a.fp64:
        log("[bench] FP64 run")
        r64 = gpu_run("f64", x, fh, gf, a.steps, a.warmup, rho, m, sigma, M, use_graph=not a.eager,
                      overlap=ovl, autotune=a.autotune)
        ms64 = r64["ms_graph"] if r64["ms_graph"] else r64["ms_eager"]
        out64, rows64 = r64["outs"], r64["rows"]
        log(f"[bench] FP64 graph {r64['ms_graph']} ms/step, eager {r64['ms_eager']:.3f} ms/step {r64['breakdown']}")
        res64 = dict(value=N * R / (ms64 * 1e-3), ms_per_step=ms64, eager_ms_per_step=r64["ms_eager"],
                     replay_ms={"warm": r64["replay_warm_ms"], "mall_flushed": r64["replay_flushed_ms"]},
                     breakdown_ms=r64["breakdown"], graph_vs_eager_rel=r64["graph_vs_eager"])

    G = int(np.prod([int(round(sigma * v)) for v in M]))
    P_ = int(np.prod(M))
    T = 2 * m + 1
    algo = algorithmic_bytes(N, P_, G, T, R, 8, 8)
    stage_roof = {}
    for k, b in algo.items():
        if k in br32:
            gbs = b / (br32[k] * 1e-3) / 1e9
            stage_roof[k] = dict(bytes=b, ms=br32[k], GBps=gbs, frac=gbs / HBM_PEAK_GBS)

    dom = max(br32, key=br32.get)
    kc = r32["kclass"]
    dom_k = max(kc, key=lambda k: kc[k]["ms_per_step"])
    Ms = int(round(sigma * M[0]))
    nl = member_counts(x, Ms, m)
    flops = float(np.sum(solve_flops(nl[nl > 0])))
    ms_solve = kc["solve"]["ms_per_launch"]
    roof_solve = {"bound": "alu", "kernel": "k_solve_t1 (B optimisation, FP64, one thread per grid index)",
                  "achieved": flops / (ms_solve * 1e-3) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                  "frac": flops / (ms_solve * 1e-3) / 1e12 / 78.6, "traffic": solve_traffic("f32"),
                  "algorithmic_flops_per_launch": flops, "ms_per_launch": ms_solve,
                  "units_per_launch": int(np.sum(nl > 0))}
    # HBM view of the streaming kernels: bytes they must move at least once per launch
    G_ = Ms
    c8 = 8
    kbytes = {
        "fft": 2 * G_ * c8,                                   # one pass reads and writes the grid
        "spread": N * (c8 + 4 + 8) + G_ * c8,                 # samples, stencil base, offset; grid once
        "interp": G_ * c8 + N * (c8 + 4 + 8),
    }
    kroof = {}
    for k, b in kbytes.items():
        mpl = kc[k]["ms_per_launch"]
        kroof[k] = dict(bytes_per_launch=b, ms_per_launch=mpl, GBps=b / (mpl * 1e-3) / 1e9,
                        frac=b / (mpl * 1e-3) / 1e9 / HBM_PEAK_GBS)
    line = {
        "metric": "nodes/sec for NFFT + modified adjoint iNFFT, FP32 vs FP64, at rel. error",
        "value": N * R / (ms32 * 1e-3),
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD_NAME,
            "M": M[0], "N": N, "sigma": sigma, "m": m, "rhs": R, "rho": rho,
            "nodes": "x_j = (j - N/2)/N + U(-1/(4N), 1/(4N)), seed 0",
            "step": "nodes + trafo + adjoint + B optimisation (FP64) + modified adjoint + both backward kernels",
            "parallelism": "single GPU",
        },
        "precompute_dtype": "f64",
        "autotuned_fft_rows": {k: v for k, v in r32["tuned"].items() if k != "spread_rhs"},
        "autotuned_spread_rhs": r32["tuned"].get("spread_rhs"),
        "roofline": roof_solve,
        "kernel_classes": kc,
        "dominant_kernel_class": dom_k,
        "streaming_kernels_hbm": kroof,
        "timing": ("hipGraph replay of the whole step" if r32["ms_graph"] else "eager launches")
                  + {"none": "; every call on one stream, the NFFT's node gradient from the grid the NFFT left",
                     "pre": "; B optimisation on a second stream, overlapped with the NFFT and the adjoint",
                     "tail": "; B optimisation on a second stream, overlapped with the NFFT and the adjoint; "
                             "node gradient on a third stream and work slot, beside the inverse adjoint",
                     "full": "; independent calls overlapped on four streams and three work slots: the B "
                             "optimisation with the NFFT and the adjoint, the adjoint with the B optimisation, "
                             "the node gradient with the rest"}[ovl],
        "eager_ms_per_step": r32["ms_eager"],
        # one replay timed with HIP events: back to back, and after a 512 MiB write that evicts the
        # step's working set (about 90 MB) from the 256 MB Infinity Cache
        "replay_ms": {"warm": r32["replay_warm_ms"], "mall_flushed": r32["replay_flushed_ms"]},
        "graph_vs_eager_rel": r32["graph_vs_eager"],
        "breakdown_ms": br32,
        # the metric as defined for the paper's path, N R / (t_trafo + t_apply), from the eager
        # per-call breakdown (B optimisation excluded), beside the whole-step value
        "nodes_per_s_trafo_plus_apply": N * R / ((br32["a2-a4_trafo"] + br32["a7_apply"]) * 1e-3),
        "dominant_call": dom,
        "stage_hbm": stage_roof,
        "status": {k: st32[k] for k in ("failed_solves", "oversized", "min_members", "max_members", "empty_columns")},
        "fp64": res64,
        "fp32_over_fp64": (res64["ms_per_step"] / ms32) if res64 else None,
    }
    if not a.no_secondary:
        log("[bench] batched workload (256 uneven 1-D problems, 8 right-hand sides)")
        line["secondary"] = {"rhs8_1d": secondary_rhs8(max(10, a.steps), 3)}
        log(f"[bench] 8 right-hand sides: {line['secondary']['rhs8_1d']}")
        line["secondary"]["batched_1d"] = secondary_batched(max(5, a.steps // 2), 2)
        log(f"[bench] batched: {line['secondary']['batched_1d']}")
        log("[bench] polar workload (512 x 512, N = 524288)")
        line["secondary"]["polar_2d"] = secondary_polar(max(5, a.steps // 2), 2)
        log(f"[bench] polar: {line['secondary']['polar_2d']}")
        log("[bench] spiral workload (256 x 256, N = 65536, 16 RHS, loss and gradients)")
        line["secondary"]["spiral_2d_autograd"] = secondary_spiral(5, 1)
        log(f"[bench] spiral: {line['secondary']['spiral_2d_autograd']}")
        line["secondary"]["small_1d"] = secondary_small(max(20, a.steps), 3)
        log(f"[bench] small: {line['secondary']['small_1d']}")
        log("[bench] ansatz 1 (Algorithm 3.10): N = 4096, M = 16384 and N = 262144, M = 1048576")
        line["secondary"]["ansatz1_1d"] = secondary_ansatz1(max(10, a.steps), 3)
        log(f"[bench] ansatz 1: {line['secondary']['ansatz1_1d']}")
        log("[bench] Dirichlet-kernel B optimisation and the node gradient through B_opt(x), 1-D jittered")
        line["secondary"]["variants_1d"] = secondary_variants(max(10, a.steps // 2), 3)
        log(f"[bench] variants: {line['secondary']['variants_1d']}")
    if not a.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline (B optimisation sampled on {a.cpu_sample} grid indices)")
        cb = cpu_baseline(x, fh, gf, rho, m, sigma, M, a.cpu_sample)
        allc, one = cb["runs"]["all_cores"], cb["runs"]["one_thread"]
        f_o, h_o = cb["f"], cb["h"]
        err = {
            "f32_trafo": rel(out32[0], nfft_ref(cb, x, fh32)),
            "f32_adjoint": rel(out32[1], adj_ref(cb, x, out32[0])),
        }
        if res64:
            err["f64_trafo"] = rel(out64[0], f_o)
            err["f64_adjoint"] = rel(out64[1], adj_ref(cb, x, out64[0]))
            # B_opt on the sampled grid indices against the oracle's reduced route
            mask = cb["solved"]
            err["f64_bopt_sampled"] = rel(rows64[mask], cb["rows"][mask])
            err["f32_bopt_sampled"] = rel(rows32[mask], cb["rows"][mask])
        line["rel_err"] = err
        line["cpu_baseline"] = {
            "value": N * R / allc["total_s"],
            "unit": "nodes/s",
            "cores": allc["threads"],
            "kind": "oracle",
            "sample": (f"full NFFT, adjoint, modified adjoint, its adjoint and node gradient; B optimisation by the "
                       f"Gram route (direct O(M) kernel sums, dense solve) on {cb['sample']} of {G} grid indices, "
                       f"time scaled by {G / cb['sample']:.0f}"),
            "parts_s": allc["parts_s"],
            "one_thread": {"value": N * R / one["total_s"], "threads": one["threads"], "parts_s": one["parts_s"]},
            "host": cpu_description(),
        }
        log(f"[bench] CPU oracle {allc['total_s']:.2f} s/step on {allc['threads']} threads, "
            f"{one['total_s']:.2f} s on one; errors {err}")
    print(json.dumps(line))


def nfft_ref(cb, x, fh32):
    from oracle import nfft
    return nfft.trafo(x, fh32, cb["p"])


def adj_ref(cb, x, f):
    from oracle import nfft
    return nfft.adjoint(x, np.asarray(f, dtype=np.complex128), cb["p"])


if __name__ == "__main__":
    main()
