"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/ovl.h declares, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import pytest

from paper_2204_01583_amd import ovl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "ovl.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ovl_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert header_functions() == sorted(ovl.EXPORTS)


def test_library_exports_every_symbol():
    lib = ovl.load()
    for name in header_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    assert ovl.status_string(0) == "OVL_OK"
    assert ovl.status_string(1) == "OVL_NOT_CONVERGED"
    assert ovl.status_string(-1) == "OVL_E_ARG"
    assert ovl.status_string(-6) == "OVL_E_BREAKDOWN"
    assert ovl.status_string(99) == "unknown status"


def test_null_arguments_rejected():
    lib = ovl.load()
    assert lib.ovl_create(None, None, None, 0, None) == ovl.E_ARG
    assert lib.ovl_set_masses(None, 1.0, 0.0) == ovl.E_ARG
    assert lib.ovl_set_contour(None, 8, 1.3, 1.2, 1.0) == ovl.E_ARG
    assert lib.ovl_apply_hw(None, None, None, 1) == ovl.E_ARG
    assert lib.ovl_destroy(None) == ovl.OK
    assert lib.ovl_last_error(None) == b"null context"


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="host without a GPU only")
def test_create_without_gpu_reports_hip_error():
    lib = ovl.load()
    h = ctypes.c_void_p()
    d = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    assert lib.ovl_create(ctypes.byref(h), d, None, 0, None) == ovl.E_HIP
    assert not h.value
