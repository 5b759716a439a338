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
