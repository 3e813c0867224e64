"""The C ABI library loads and exports every symbol include/wpcd.h declares
(CPU only: no call here touches a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wpcd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wpcd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    import paper_1508_07441_amd as P
    assert names == sorted(P.ABI_FUNCTIONS)


def test_library_exports_every_declared_symbol():
    import paper_1508_07441_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libwpcd.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(P.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_null_arguments_rejected_without_device():
    import paper_1508_07441_amd as P
    L = P.lib()
    assert L.wpcd_create(0, None, None) == P.WPCD_E_INVALID
    assert L.wpcd_build_basis(None, None, None) == P.WPCD_E_INVALID
    assert L.wpcd_build_p(None, 0, None) == P.WPCD_E_INVALID
    assert L.wpcd_solve(None, None, 0, 0, None, None, None) == P.WPCD_E_INVALID
    assert L.wpcd_last_error(None) == b"null context"
    L.wpcd_destroy(None)


def test_struct_layouts_match_header():
    import paper_1508_07441_amd as P
    # sizes follow from the C declarations with natural alignment
    assert ctypes.sizeof(P.wpcd_basis_desc) == 4 * 2 + 8 * 2 + 8 + 8 * 2 + 4 * 4 + 8 * 2
    assert ctypes.sizeof(P.wpcd_potential_desc) == 8 + 8 * 2 + 8
    assert ctypes.sizeof(P.wpcd_solve_opts) == 4 * 2 + 8 + 8
    assert ctypes.sizeof(P.wpcd_energy_result) == 8 * 2 + 4 * 4 + 8 * 9
    assert ctypes.sizeof(P.wpcd_kernel_time) == 32 + 8 + 8


def test_create_without_gpu_reports_device_error():
    import paper_1508_07441_amd as P
    h = ctypes.c_void_p()
    st = P.lib().wpcd_create(0, None, ctypes.byref(h))
    if st == P.WPCD_OK:      # a GPU is visible: nothing to check here
        P.lib().wpcd_destroy(h)
    else:
        assert st in (P.WPCD_E_DEVICE, P.WPCD_E_INVALID)
