"""infft_apply_noalloc: the modified adjoint (3.32) with its work buffers in the library's static
device scratch instead of the plan's, for callers that cannot allocate device memory.  Called
through the C ABI and compared with infft_apply on the same plan, on two calls in a row, the second
with a smaller input; the first call's larger contents of the scratch must not leak into the
second.  Device memory stays unchanged across the calls, and a plan whose work buffers exceed the
scratch is refused with a clear error."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W

from gpu_util import dev, host, nodes_dev, rel

pytestmark = pytest.mark.gpu


def _noalloc(P, f, nrhs):
    from paper_1811_05335_amd import _lib
    lib = _lib.load()
    out = torch.empty((nrhs,) + P.M, dtype=P.ctype, device="cuda")
    P._sync_stream()
    _lib.check(lib.infft_apply_noalloc(P._h, C.c_void_p(f.data_ptr()), C.c_void_p(out.data_ptr()), nrhs))
    return out


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("d", [1, 2])
def test_apply_noalloc_matches_apply_on_two_calls(d, precision):
    from paper_1811_05335_amd import NfftPlan
    g = W.rng(70 + d)
    cases = [((4096,), 9000, 3) if d == 1 else ((96, 80), 20000, 3),    # first call: larger input
             ((64,), 150, 1) if d == 1 else ((16, 20), 300, 1)]        # second call: smaller
    tol = 0.0 if d == 1 else (1e-13 if precision == "f64" else 1e-6)    # 2-D: atomic sum order
    for M, N, R in cases:
        x = W.uniform_nodes(g, N, d)
        f = W.complex_normal(g, (R, N))
        if precision == "f32":
            f = W.round_to(f, "f32")
        P = NfftPlan(M, nodes_dev(x), m=4 if d == 1 else 3, precision=precision, rho=1e-8, max_rhs=2)
        P.precompute_B()
        fd = dev(f, precision)
        ref = host(P.apply(fd))
        torch.cuda.synchronize()
        out = torch.empty((R,) + M, dtype=P.ctype, device="cuda")
        free0 = torch.cuda.mem_get_info()[0]
        from paper_1811_05335_amd import _lib
        lib = _lib.load()
        P._sync_stream()
        _lib.check(lib.infft_apply_noalloc(P._h, C.c_void_p(fd.data_ptr()), C.c_void_p(out.data_ptr()), R))
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        got = host(out)
        if tol == 0.0:
            assert np.array_equal(got, ref), (M, N, R)
        else:
            assert rel(got, ref) <= tol, (M, N, R)
        # the plan's own buffers are untouched: the NFFT's grid stays valid for the node gradient
        fh = dev(W.complex_normal(g, (1,) + M), precision)
        P.trafo(fh)
        _noalloc(P, fd[:1], 1)
        P.grad_x_after_trafo(fd[:1])
        P.close()


def test_apply_noalloc_refuses_work_buffers_beyond_the_scratch():
    from paper_1811_05335_amd import InfftError, NfftPlan
    M = (1024, 1024)          # FP64 grid of 2048 x 2048 points: 64 MiB per grid, two grids needed
    x = W.uniform_nodes(W.rng(75), 1000, 2)
    P = NfftPlan(M, nodes_dev(x), m=2, precision="f64", rho=1e-8)
    P.precompute_B()
    f = dev(W.complex_normal(W.rng(76), (1, 1000)), "f64")
    with pytest.raises(InfftError, match="static scratch"):
        _noalloc(P, f, 1)
    Q = NfftPlan((64,), nodes_dev(W.uniform_nodes(W.rng(77), 100, 1)), m=3, precision="f64")
    with pytest.raises(InfftError, match="ESTATE"):
        _noalloc(Q, dev(W.complex_normal(W.rng(78), (1, 100)), "f64"), 1)
    P.close()
    Q.close()
