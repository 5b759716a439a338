"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every function the
header declares, and rejects invalid arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "infft.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b([A-Za-z_0-9]+)\s*\(", src)
    return sorted({n for n in names if n.startswith(("nfft_", "infft_")) and n != "infft_plan_s"})


@pytest.fixture(scope="module")
def lib():
    from paper_1811_05335_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libinfft.so not built")
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["nfft_plan", "nfft_trafo", "nfft_adjoint", "infft_precompute_B", "infft_apply",
              "infft_apply_adjoint", "nfft_grad_x", "nfft_plan_destroy", "nfft_plan_status"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_default_options(lib):
    from paper_1811_05335_amd import _lib
    o = _lib.Options()
    lib.infft_default_options(C.byref(o))
    assert o.precision == _lib.INFFT_F64 and o.max_rhs == 1 and o.rho == 1e-8


@pytest.mark.parametrize("d,M,N,sigma,m,msg", [
    (3, (8,), 10, 2.0, 4, "d must be 1 or 2"),
    (1, (7,), 10, 2.0, 4, "even"),
    (1, (8,), 10, 2.0, 9, "m must be"),
    (1, (8,), 10, 2.0, 1, "m must be"),
    (1, (8,), 0, 2.0, 4, "N out of range"),
    (1, (8,), 10, 0.5, 4, "sigma"),
    (1, (10,), 10, 1.5, 4, "even integer"),
    (1, (8,), 10, 1.0, 4, "2m+2"),
    (1, (22,), 10, 2.0, 4, "product of 2, 3, 5, 7"),
])
def test_invalid_arguments_rejected_on_host(lib, d, M, N, sigma, m, msg):
    from paper_1811_05335_amd import _lib
    h = C.c_void_p()
    Ms = (C.c_int64 * max(1, len(M)))(*M)
    rc = lib.nfft_plan(C.byref(h), d, Ms, N, sigma, m, C.c_void_p(8), None, None)
    assert rc == _lib.INFFT_EINVAL
    assert msg in lib.infft_last_error().decode()
    assert not h.value


def test_null_plan_calls_fail_cleanly(lib):
    from paper_1811_05335_amd import _lib
    assert lib.nfft_trafo(None, None, None, 1) == _lib.INFFT_EINVAL
    assert lib.infft_precompute_B(None) == _lib.INFFT_EINVAL
    assert lib.nfft_plan_device_bytes(None) == 0
    lib.nfft_plan_destroy(None)


def test_product_path_has_no_oracle_import():
    pkg = os.path.join(ROOT, "paper_1811_05335_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".hpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, fn


def _ws_bytes(lib, M, N, m=4, sigma=2.0, **opt):
    from paper_1811_05335_amd import _lib
    o = _lib.Options()
    lib.infft_default_options(C.byref(o))
    for k, v in opt.items():
        setattr(o, k, v)
    Ms = (C.c_int64 * len(M))(*M)
    nb = C.c_size_t(123)
    rc = lib.nfft_plan_workspace_bytes(len(M), Ms, N, sigma, m, C.byref(o), C.byref(nb))
    return rc, nb.value


def test_workspace_size_query_is_host_only_and_consistent(lib):
    """The size query validates like nfft_plan and runs no device work, so it answers here.  The
    size grows with every buffer it must hold: right-hand sides per pass (grids), work slots, the
    memory kept for large local problems (exactly large_mib MiB more), the FP32 copy of B_opt, and
    the inner plans of Algorithm 3.10."""
    from paper_1811_05335_amd import _lib
    rc, base = _ws_bytes(lib, (65536,), 131072, m=6, precision=_lib.INFFT_F32)
    assert rc == 0 and base > 0
    G, cs = 131072, 8
    rc, r4 = _ws_bytes(lib, (65536,), 131072, m=6, precision=_lib.INFFT_F32, max_rhs=4)
    assert rc == 0 and r4 - base >= 3 * 2 * G * cs          # two grids per slot, 3 more RHS
    rc, s2 = _ws_bytes(lib, (65536,), 131072, m=6, precision=_lib.INFFT_F32, work_slots=2)
    assert rc == 0 and s2 - base >= 2 * G * cs
    rc, l8 = _ws_bytes(lib, (65536,), 131072, m=6, precision=_lib.INFFT_F32, large_mib=8)
    rc2, l9 = _ws_bytes(lib, (65536,), 131072, m=6, precision=_lib.INFFT_F32, large_mib=9)
    assert rc == rc2 == 0 and l9 - l8 == 1 << 20
    rc, f64 = _ws_bytes(lib, (65536,), 131072, m=6, precision=_lib.INFFT_F64)
    # FP32 plans hold an FP32 copy of B_opt (13 taps x N x 8 bytes); FP64 plans grids twice as large
    assert rc == 0 and base - f64 >= 13 * 131072 * 8 - 5 * 2 * G * 8
    rc, a1 = _ws_bytes(lib, (16384,), 4096, m=4, precision=_lib.INFFT_F32, ansatz1=1)
    rc2, na1 = _ws_bytes(lib, (16384,), 4096, m=4, precision=_lib.INFFT_F32)
    assert rc == rc2 == 0 and a1 > na1
    # invalid arguments: the same messages as nfft_plan, *bytes = 0
    rc, b = _ws_bytes(lib, (15,), 100)
    assert rc == _lib.INFFT_EINVAL and b == 0 and "even" in lib.infft_last_error().decode()
    rc, b = _ws_bytes(lib, (16, 16), 100, ansatz1=1)
    assert rc == _lib.INFFT_EINVAL and "d = 1" in lib.infft_last_error().decode()


def test_workspace_plan_rejects_bad_workspace_on_host(lib):
    from paper_1811_05335_amd import _lib
    h = C.c_void_p()
    Ms = (C.c_int64 * 1)(64)
    assert lib.nfft_plan_ws(C.byref(h), 1, Ms, 100, 2.0, 4, C.c_void_p(8), None, None, 0, None) == _lib.INFFT_EINVAL
    assert "workspace is null" in lib.infft_last_error().decode()
    assert lib.nfft_plan_ws(C.byref(h), 1, Ms, 100, 2.0, 4, C.c_void_p(8), None, C.c_void_p(4096 + 8), 1 << 30,
                            None) == _lib.INFFT_EINVAL
    assert "aligned" in lib.infft_last_error().decode()
    assert lib.nfft_plan_ws(C.byref(h), 1, Ms, 100, 2.0, 4, C.c_void_p(8), None, C.c_void_p(4096), 1024,
                            None) == _lib.INFFT_ENOMEM
    assert not h.value
    o = _lib.Options()
    lib.infft_default_options(C.byref(o))
    o.large_mib = 4
    assert lib.nfft_plan(C.byref(h), 1, Ms, 100, 2.0, 4, C.c_void_p(8), C.byref(o), None) == _lib.INFFT_EINVAL
    assert lib.infft_plan_export(None, None, None) == _lib.INFFT_EINVAL
    assert lib.infft_plan_import(None, None, 0) == _lib.INFFT_EINVAL
