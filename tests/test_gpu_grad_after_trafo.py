"""nfft_grad_x_after_trafo: the NFFT's node gradient from the grid the last nfft_trafo on the work
slot left.  It runs the same gradient kernel on the same grid as nfft_grad_x, so the two agree bit
for bit (and nfft_grad_x is checked against the oracle elsewhere); every call that writes the
slot's grid ends the grid's validity; slots are independent; captured graphs replay it."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import grad as ograd
from oracle import nfft as onfft

from gpu_util import dev, nodes_dev, rel

pytestmark = pytest.mark.gpu


CASES = [
    # M, d, N, m, precision, rhs
    ((4096,), 1, 8192, 6, "f32", 1),
    ((4096,), 1, 6000, 4, "f64", 3),
    ((256,), 1, 300, 5, "f64", 2),       # one FFT pass (M_sigma within one workgroup)
    ((32, 32), 2, 1500, 3, "f32", 2),
    ((32, 32), 2, 1500, 3, "f64", 1),
]


@pytest.mark.parametrize("M,d,N,m,precision,R", CASES)
def test_after_trafo_equals_grad_x(M, d, N, m, precision, R):
    from paper_1811_05335_amd import NfftPlan
    g = W.rng(140)
    x = W.uniform_nodes(g, N, d)
    fh = dev(W.complex_normal(g, (R,) + M), precision)
    gf = dev(W.complex_normal(g, (R, N)), precision)
    P = NfftPlan(M, nodes_dev(x), sigma=2.0, m=m, precision=precision, max_rhs=R)
    P.trafo(fh)
    g1 = P.grad_x_after_trafo(gf)
    g2 = P.grad_x(fh, gf)
    assert torch.equal(g1, g2)
    if precision == "f64" and N <= 2000:
        p = onfft.Params(M, 2.0, m)
        want = ograd.nfft_grad_x(x, fh.cpu().numpy(), gf.cpu().numpy(), p)
        assert rel(g1.cpu().numpy(), want) <= 1e-10


def test_validity_follows_the_slot_grid():
    from paper_1811_05335_amd import NfftPlan, NfftBatchPlan
    from paper_1811_05335_amd._lib import InfftError, load
    M, N = (512,), 700
    g = W.rng(141)
    x = W.uniform_nodes(g, N, 1)
    fh = dev(W.complex_normal(g, (2,) + M), "f64")
    gf = dev(W.complex_normal(g, (2, N)), "f64")
    P = NfftPlan(M, nodes_dev(x), sigma=2.0, m=4, precision="f64", rho=1e-10, max_rhs=2, work_slots=2)
    ref = P.grad_x(fh, gf)
    with pytest.raises(InfftError):           # nfft_grad_x wrote the grid
        P.grad_x_after_trafo(gf)
    f = P.trafo(fh)
    with pytest.raises(InfftError):           # nrhs differs from the trafo's
        P.grad_x_after_trafo(gf[:1])
    P.precompute_B()                          # uses none of the slot's buffers
    assert torch.equal(P.grad_x_after_trafo(gf), ref)
    P.set_slot(1)                             # another slot: its grid holds nothing yet
    with pytest.raises(InfftError):
        P.grad_x_after_trafo(gf)
    P.adjoint(f)
    P.set_slot(0)                             # slot 0 still holds the trafo
    assert torch.equal(P.grad_x_after_trafo(gf), ref)
    for call in (lambda: P.adjoint(f), lambda: P.apply(f), lambda: P.apply_adjoint(fh),
                 lambda: P.set_nodes(nodes_dev(x))):
        P.trafo(fh)
        call()
        with pytest.raises(InfftError):
            P.grad_x_after_trafo(gf)
    P.trafo(fh)
    assert torch.equal(P.grad_x_after_trafo(gf), ref)
    # more right-hand sides than one pass holds: the grid keeps only the last chunk
    P1 = NfftPlan(M, nodes_dev(x), sigma=2.0, m=4, precision="f64", max_rhs=1)
    P1.trafo(fh)
    with pytest.raises(InfftError):
        P1.grad_x_after_trafo(gf)
    PB = NfftBatchPlan([16, 16], [10, 20], nodes_dev(W.uniform_nodes(g, 30, 1)), sigma=2.0, m=2)
    out = torch.empty((30, 1), dtype=torch.float64, device="cuda")
    gfb = torch.zeros(30, dtype=torch.complex128, device="cuda")
    assert load().nfft_grad_x_after_trafo(PB._h, gfb.data_ptr(), out.data_ptr(), 1) == -1   # INFFT_EINVAL


def test_captured_trafo_and_gradient_replay():
    from paper_1811_05335_amd import NfftPlan
    M, N = (2048,), 4096
    g = W.rng(142)
    x = W.jittered_nodes(g, N)
    fh = dev(W.complex_normal(g, (1,) + M), "f32")
    gf = dev(W.complex_normal(g, (1, N)), "f32")
    P = NfftPlan(M, nodes_dev(x), sigma=2.0, m=6, precision="f32", max_rhs=1)
    P.trafo(fh)
    ref = P.grad_x_after_trafo(gf).clone()

    def seq():
        P.trafo(fh)
        return P.grad_x_after_trafo(gf)

    warm = torch.cuda.Stream()
    warm.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(warm):
        seq()
    torch.cuda.current_stream().wait_stream(warm)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out = seq()
    for _ in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        P.adjoint(P.trafo(fh))                # eager work between replays
        torch.cuda.synchronize()
    assert np.isfinite(ref.cpu().numpy()).all()


def test_autograd_backward_reuses_the_forward_grid_only_when_it_is_current():
    """autograd.nfft's backward takes the node gradient from the forward's grid when that trafo was
    the plan's last and nothing wrote the grid since, else recomputes it: the gradients are the
    same bit for bit either way, including after another trafo on the plan (a different grid)."""
    from paper_1811_05335_amd import NfftPlan, autograd
    M, N = (1024,), 1500
    g = W.rng(143)
    x = nodes_dev(W.uniform_nodes(g, N, 1))
    fh0 = dev(W.complex_normal(g, (2,) + M), "f64")
    other = dev(W.complex_normal(g, (2,) + M), "f64")
    w = dev(W.complex_normal(g, (2, N)), "f64")
    P = NfftPlan(M, x, sigma=2.0, m=4, precision="f64", max_rhs=2, work_slots=2)

    def grads(between):
        fh = fh0.clone().requires_grad_(True)
        xx = x.clone().requires_grad_(True)
        f = autograd.nfft(fh, xx, P)
        between()
        loss = torch.sum(torch.real(torch.conj(w) * f))
        loss.backward()
        return fh.grad.clone(), xx.grad.clone()

    ref = grads(lambda: None)                               # grid current: reused
    for between in (lambda: P.adjoint(w),                   # grid written: recomputed
                    lambda: P.trafo(other),                 # another trafo's grid: recomputed
                    lambda: (P.set_slot(1), P.trafo(other), P.set_slot(0))):
        got = grads(between)
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
