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
    assert L.wpcd_set_multipliers(None, None, 0) == P.WPCD_E_INVALID
    assert L.wpcd_solve_multi(None, 0, None, None, 0, None, None, None) == P.WPCD_E_INVALID
    assert L.wpcd_save_p(None, None) == P.WPCD_E_INVALID
    assert L.wpcd_bound_state(None, 0.0, 0.0, None) == P.WPCD_E_INVALID
    assert L.wpcd_load_p(None, None, None) == P.WPCD_E_INVALID
    assert L.wpcd_solve_dev(None, None, 0, 0, None, None) == P.WPCD_E_INVALID
    assert L.wpcd_learn_train(None, None, None) == P.WPCD_E_INVALID
    assert L.wpcd_mlp_eval(None, 1, 1, 1, None, 1, None, None, None, None, None) == P.WPCD_E_INVALID
    assert L.wpcd_set_autotune(None, 0) == P.WPCD_E_INVALID
    assert L.wpcd_set_graphs(None, 0) == P.WPCD_E_INVALID
    assert L.wpcd_get_autotune(None, None, 0, None) == P.WPCD_E_INVALID
    assert L.wpcd_last_error(None) == b"null context"
    L.wpcd_destroy(None)


STRUCTS = ("wpcd_basis_desc", "wpcd_potential_desc", "wpcd_solve_opts", "wpcd_energy_result",
           "wpcd_learn_desc", "wpcd_learn_report", "wpcd_tune_entry", "wpcd_kernel_time")


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the ctypes mirrors equal what the C
    compiler lays out from include/wpcd.h."""
    import shutil
    import subprocess
    import paper_1508_07441_amd as P
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for st in STRUCTS:
        lines.append(f'printf("{st} size %zu\\n", sizeof({st}));')
        for f, _ in getattr(P, st)._fields_:
            lines.append(f'printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for st in STRUCTS:
        T = getattr(P, st)
        assert got[(st, "size")] == ctypes.sizeof(T), st
        for f, _ in T._fields_:
            assert got[(st, f)] == getattr(T, f).offset, (st, f)


def test_create_without_gpu_reports_device_error():
    import paper_1508_07441_amd as P
    h = ctypes.c_void_p()
    st = P.lib().wpcd_create(0, None, ctypes.byref(h))
    if st == P.WPCD_OK:      # a GPU is visible: nothing to check here
        P.lib().wpcd_destroy(h)
    else:
        assert st in (P.WPCD_E_DEVICE, P.WPCD_E_INVALID)
