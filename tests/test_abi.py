"""The C-ABI library loads, exports every symbol include/tgba.h declares, and
rejects invalid arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tgba.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tgba_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary_calls():
    names = _declared()
    for must in ("tgba_build_basis", "tgba_assemble_heff", "tgba_eig", "tgba_dsf", "tgba_quench"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2410_04204_amd import _lib
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(_lib.EXPORTS) == set(_declared())


@pytest.mark.parametrize("N,h", [(7, 1.0), (0, 1.0), (66, 1.0), (10, 0.0), (10, -1.0), (10, float("nan"))])
def test_invalid_models_are_rejected_before_device_use(N, h):
    from paper_2410_04204_amd import _lib
    L = _lib.load()
    m = _lib.Model(N, h, 0.1)
    t = _lib.Trunc(_lib.TGBA_TRUNC_ECUT, 5.0, 0, None, 0)
    out = ctypes.c_void_p()
    rc = L.tgba_build_basis(ctypes.byref(m), ctypes.byref(t), None, ctypes.byref(out))
    assert rc == -1 and out.value is None
    assert L.tgba_last_error().decode()


def test_invalid_truncations_are_rejected():
    from paper_2410_04204_amd import _lib
    L = _lib.load()
    m = _lib.Model(40, 1.0, 0.1)
    out = ctypes.c_void_p()
    for t in (_lib.Trunc(7, 5.0, 0, None, 0), _lib.Trunc(_lib.TGBA_TRUNC_ECUT, -1.0, 0, None, 0),
              _lib.Trunc(_lib.TGBA_TRUNC_CHI, -1.0, 0, None, 100), _lib.Trunc(_lib.TGBA_TRUNC_CHI, 5.0, 0, None, -3)):
        assert L.tgba_build_basis(ctypes.byref(m), ctypes.byref(t), None, ctypes.byref(out)) == -1


def test_null_arguments_are_rejected():
    from paper_2410_04204_amd import _lib
    L = _lib.load()
    assert L.tgba_assemble_heff(None, 0, None, 1, 0, None) == -1
    assert L.tgba_basis_sector_size(None, 0, None, None) == -1


def test_timing_hook_without_launches():
    """Enabling, reading and disabling the kernel timing needs no device."""
    import paper_2410_04204_amd as tg
    from paper_2410_04204_amd import _lib
    tg.timing_enable(True)
    assert tg.timing_read() == (0.0, 0, 0.0)
    tg.timing_enable(False)
    assert _lib.load().tgba_timing_read(None, None, None) == -1


def test_autotune_switches_and_empty_report():
    import paper_2410_04204_amd as tg
    tg.autotune_enable(-1)
    assert tg.autotune_report() == {}
    tg.autotune_enable(False)
    tg.autotune_enable(True)


def test_capture_api_rejects_misuse_before_device_use():
    from paper_2410_04204_amd import _lib
    L = _lib.load()
    assert L.tgba_capture_begin(None) == -1  # TGBA_EINVAL: the NULL stream cannot be captured
    out = ctypes.c_void_p()
    assert L.tgba_capture_end(None, ctypes.byref(out)) == -1  # no capture is active
    assert out.value is None
    assert L.tgba_plan_info(None, None, None) == -1
