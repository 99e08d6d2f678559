"""The C-ABI library loads and exports every entry point the header declares;
argument validation happens on the host before any launch (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2207_08716_amd import abi, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ptporo.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(abi.LIB_PATH):
        pytest.skip("libptporo.so not built")
    return abi.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "pt_iteration" in names and "pt_create" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(abi.EXPORTS)


def test_create_validates_arguments(lib):
    p = abi.params_from(inputs.Physics(), False)
    h = C.c_void_p()
    assert lib.pt_create(1, 4, 4, 8, C.byref(p), C.byref(h)) == -1
    assert lib.pt_create(4, 4, 4, 4, C.byref(p), C.byref(h)) == -1   # pitch < nx + 1
    bad = abi.params_from(inputs.Physics(dt=0.0), False)
    assert lib.pt_create(4, 4, 4, 8, C.byref(bad), C.byref(h)) == -1
    bad = abi.params_from(inputs.Physics(), False)
    bad.version = 99
    assert lib.pt_create(4, 4, 4, 8, C.byref(bad), C.byref(h)) == -1
    assert lib.pt_create(4, 5, 6, 8, C.byref(p), C.byref(h)) == 0
    try:
        assert lib.pt_field_elems(h) == 7 * 6 * 8
        # unaligned, null, bad id, bad copy
        assert lib.pt_bind_field(h, 0, 0, C.c_void_p(0x1008)) == -1
        assert lib.pt_bind_field(h, 0, 0, None) == -1
        assert lib.pt_bind_field(h, 99, 0, C.c_void_p(0x1000)) == -1
        assert lib.pt_bind_field(h, abi.FIELD_ID["mus"], 1, C.c_void_p(0x1000)) == -1
        assert b"copy" in lib.pt_last_error(h)
        # nothing bound: every launching call refuses before touching the device
        assert lib.pt_iteration(h, 1, 0) == -1
        assert lib.pt_begin_step(h, 0) == -1
        assert lib.pt_refresh(h, 0.5, 0.5) == -1
        sz = C.c_size_t()
        assert lib.pt_workspace_size(h, C.byref(sz)) == 0 and sz.value > 0
        assert lib.pt_bind_workspace(h, C.c_void_p(0x1000), 8) == -1
    finally:
        lib.pt_destroy(h)
    assert lib.pt_status_str(-3) == b"diverged (non-finite norm)"
