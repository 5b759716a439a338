"""ctypes loader for libinfft.so (built in-tree by paper_1811_05335_amd.build)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinfft.so")

INFFT_OK = 0
INFFT_EINVAL = -1
INFFT_ENOMEM = -2
INFFT_EDEVICE = -3
INFFT_ESINGULAR = -4
INFFT_ESTATE = -5
INFFT_F32 = 0
INFFT_F64 = 1
KERNEL_CLASSES = {"nodes": 1, "fft": 2, "spread": 3, "interp": 4, "solve": 5}

ERROR_NAMES = {
    INFFT_EINVAL: "INFFT_EINVAL",
    INFFT_ENOMEM: "INFFT_ENOMEM",
    INFFT_EDEVICE: "INFFT_EDEVICE",
    INFFT_ESINGULAR: "INFFT_ESINGULAR",
    INFFT_ESTATE: "INFFT_ESTATE",
}


INFFT_KERNEL_WINDOW = 0
INFFT_KERNEL_DIRICHLET = 1
KERNELS = {"window": INFFT_KERNEL_WINDOW, "dirichlet": INFFT_KERNEL_DIRICHLET}


class Options(C.Structure):
    _fields_ = [
        ("precision", C.c_int),
        ("max_rhs", C.c_int),
        ("rho", C.c_double),
        ("tile", C.c_int * 2),
        ("inverse_kernel", C.c_int),
        ("work_slots", C.c_int),
        ("large_mib", C.c_int),
        ("ansatz1", C.c_int),
        ("reserved", C.c_int * 2),
    ]


class Status(C.Structure):
    _fields_ = [
        ("nonfinite_nodes", C.c_int64),
        ("failed_solves", C.c_int64),
        ("empty_columns", C.c_int64),
        ("oversized", C.c_int64),
        ("min_members", C.c_int64),
        ("max_members", C.c_int64),
        ("bopt_ready", C.c_int32),
        ("max_supported", C.c_int32),
    ]


class InfftError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load() -> C.CDLL:
    """Loads the HIP library; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1811_05335_amd.build` "
            "(the library has no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "infft_default_options": (None, [C.POINTER(Options)]),
        "nfft_plan": (i32, [C.POINTER(vp), i32, C.POINTER(i64), i64, dbl, i32, vp, C.POINTER(Options), vp]),
        "nfft_plan_batched": (i32, [C.POINTER(vp), i32, C.POINTER(i64), C.POINTER(i64), dbl, i32, vp,
                                    C.POINTER(Options), vp]),
        "nfft_plan_workspace_bytes": (i32, [i32, C.POINTER(i64), i64, dbl, i32, C.POINTER(Options),
                                            C.POINTER(C.c_size_t)]),
        "nfft_plan_ws": (i32, [C.POINTER(vp), i32, C.POINTER(i64), i64, dbl, i32, vp, C.POINTER(Options), vp,
                               C.c_size_t, vp]),
        "infft_plan_export": (i32, [vp, vp, C.POINTER(C.c_size_t)]),
        "infft_plan_import": (i32, [vp, vp, C.c_size_t]),
        "nfft_set_nodes": (i32, [vp, vp]),
        "nfft_set_stream": (i32, [vp, vp]),
        "nfft_set_slot": (i32, [vp, C.c_int]),
        "nfft_trafo": (i32, [vp, vp, vp, i32]),
        "nfft_adjoint": (i32, [vp, vp, vp, i32]),
        "infft_precompute_B": (i32, [vp]),
        "infft_precompute_Bstar": (i32, [vp]),
        "infft_apply": (i32, [vp, vp, vp, i32]),
        "infft_apply_adjoint": (i32, [vp, vp, vp, i32]),
        "infft_apply_noalloc": (i32, [vp, vp, vp, i32]),
        "nfft_grad_x": (i32, [vp, vp, vp, vp, i32]),
        "nfft_grad_x_after_trafo": (i32, [vp, vp, vp, i32]),
        "infft_grad_x_bopt": (i32, [vp, vp, vp, vp, i32]),
        "infft_get_B": (i32, [vp, vp]),
        "nfft_plan_status": (i32, [vp, C.POINTER(Status)]),
        "nfft_plan_device_bytes": (i64, [vp]),
        "nfft_plan_destroy": (None, [vp]),
        "infft_last_error": (C.c_char_p, []),
        "infft_profile_begin": (i32, [vp, i32]),
        "infft_autotune": (i32, [vp, i32]),
        "infft_autotune_rows": (i32, [vp, i32, i32]),
        "infft_autotune_rhs_chunk": (i32, [vp]),
        "infft_profile_end": (i32, [vp, C.POINTER(dbl), C.POINTER(i64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int) -> None:
    if code != INFFT_OK:
        msg = load().infft_last_error().decode(errors="replace")
        raise InfftError(code, msg)
