"""MI355X (gfx950) direct inverse NFFT: NFFT, adjoint NFFT, the optimisation of the sparse
matrix B (Algorithm 3.17) and the modified adjoint NFFT (3.32), as hand-written HIP kernels
behind a C ABI (include/infft.h).  This package is the thin Python binding plus the
torch.autograd wrappers."""
from .plan import (  # noqa: F401
    NfftBatchPlan,
    NfftPlan,
    infft_apply,
    infft_apply_adjoint,
    infft_get_B,
    infft_precompute_B,
    infft_precompute_Bstar,
    nfft_adjoint,
    nfft_grad_x,
    nfft_plan,
    nfft_plan_batched,
    nfft_plan_destroy,
    nfft_plan_status,
    nfft_set_nodes,
    nfft_trafo,
)
from ._lib import InfftError  # noqa: F401
from .autograd import NfftFunction, InfftApplyFunction, nfft, infft  # noqa: F401
