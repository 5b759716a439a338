"""Work slots: transforms on different slots and streams overlap on the device and give the same
results, bit for bit, as the same calls in sequence on one slot, eagerly and in replays of a
captured graph."""
import pytest
import torch

import workloads as W

from gpu_util import dev, nodes_dev

pytestmark = pytest.mark.gpu


def _path(P, fh, gf, xd, streams=None):
    """nodes, NFFT, adjoint, B optimisation, modified adjoint and its adjoint, node gradient;
    with `streams` (pre, adj, grad) the independent calls run on their own stream and slot."""
    cur = torch.cuda.current_stream()
    P.set_slot(0)
    P.set_nodes(xd)
    if streams is None:
        f = P.trafo(fh)
        h = P.adjoint(f)
        P.precompute_B()
        fc = P.apply(f)
        fa = P.apply_adjoint(fc)
        gx = P.grad_x(fh, gf)
        return f, h, fc, fa, gx
    s_pre, s_adj, s_grad = streams
    s_pre.wait_stream(cur)
    with torch.cuda.stream(s_pre):
        P.precompute_B()
    s_grad.wait_stream(cur)
    with torch.cuda.stream(s_grad):
        P.set_slot(2)
        gx = P.grad_x(fh, gf)
    P.set_slot(0)
    f = P.trafo(fh)
    s_adj.wait_stream(cur)
    with torch.cuda.stream(s_adj):
        P.set_slot(1)
        h = P.adjoint(f)
    P.set_slot(0)
    cur.wait_stream(s_pre)
    fc = P.apply(f)
    fa = P.apply_adjoint(fc)
    cur.wait_stream(s_adj)
    cur.wait_stream(s_grad)
    return f, h, fc, fa, gx


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_slots_overlap_matches_sequence(precision):
    from paper_1811_05335_amd import NfftPlan
    M, N = 4096, 8192
    g = W.rng(120)
    x = W.jittered_nodes(g, N)
    fh = dev(W.complex_normal(g, (1, M)), precision)
    gf = dev(W.complex_normal(g, (1, N)), precision)
    xd = nodes_dev(x)
    P = NfftPlan((M,), xd, sigma=2.0, m=6, precision=precision, rho=1e-12, work_slots=3)
    ref = [t.cpu() for t in _path(P, fh, gf, xd)]
    streams = (torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream())
    for _ in range(2):
        out = [t.cpu() for t in _path(P, fh, gf, xd, streams)]
        for a, b in zip(out, ref):
            assert torch.equal(a, b)
    # captured with the streams forked inside the graph, replayed with eager work in between
    warm = torch.cuda.Stream()
    warm.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(warm):
        _path(P, fh, gf, xd, streams)
    torch.cuda.current_stream().wait_stream(warm)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gouts = _path(P, fh, gf, xd, streams)
    for _ in range(3):
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(gouts, ref):
            assert torch.equal(a.cpu(), b)
        _path(P, fh, gf, xd)   # eager work on slot 0 between replays
        torch.cuda.synchronize()


def test_slot_errors():
    from paper_1811_05335_amd import NfftPlan, NfftBatchPlan
    from paper_1811_05335_amd._lib import InfftError, load
    x = nodes_dev(W.uniform_nodes(W.rng(121), 40, 1))
    P = NfftPlan((32,), x, sigma=2.0, m=3, work_slots=2)
    P.set_slot(1)
    with pytest.raises(InfftError):
        P.set_slot(2)
    with pytest.raises(InfftError):
        P.set_slot(-1)
    with pytest.raises(InfftError):
        NfftPlan((32,), x, sigma=2.0, m=3, work_slots=9)
    PB = NfftBatchPlan([16, 16], [10, 30], x, sigma=2.0, m=2)
    assert load().nfft_set_slot(PB._h, 0) == -1      # INFFT_EINVAL: batch plans have one slot
