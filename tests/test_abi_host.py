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
    return sorted(set(re.findall(r"\b(ovl_[a-z0-9_]+)\s*\(", txt)))


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


def test_suggest_contour_meets_target():
    """The circle suggested for a gap and a spectral radius keeps the oracle's
    two-contour filter within the target on the whole |lambda| in [gap, lmax]
    (host-only call)."""
    import numpy as np
    from oracle.contour import nodes, scalar_filter
    from paper_2204_01583_amd import ovl
    for gap, lmax, target in ((0.126, 2.3, 1e-12), (0.05, 2.5, 1e-8), (0.3, 1.9, 1e-5)):
        nq, g, r = ovl.suggest_contour(gap, lmax, target)
        assert nq % 2 == 0 and 2 * nq <= 2048
        z, c = nodes(nq, g, r, 1.0)
        lam = np.concatenate([np.linspace(gap, lmax, 400), -np.linspace(gap, lmax, 400)])
        err = np.abs(scalar_filter(lam, z, c) - np.sign(lam)).max()
        assert err < target, (gap, lmax, target, nq, err)
        # two fewer nodes would not do (the choice is the smallest even count)
        z2, c2 = nodes(nq - 2, g, r, 1.0)
        assert np.abs(scalar_filter(lam, z2, c2) - np.sign(lam)).max() > 0.5 * target
    with pytest.raises(ovl.OvlError):
        ovl.suggest_contour(1e-4, 2.3, 1e-14)     # needs more than 2048 shifts
