"""The C ABI library loads, exports every declared symbol and validates its
arguments before touching a device (runs without a GPU)."""

import ctypes
import os

import pytest

from helpers import LIB, header_functions

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libclamp.so not built")


class Scene(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("looks", ctypes.c_int32), ("pupil_radius", ctypes.c_float),
                ("pupil_mask", ctypes.c_void_p), ("range_support", ctypes.c_int32)]


@pytest.fixture(scope="module")
def lib():
    lib = ctypes.CDLL(LIB)
    lib.clamp_last_error.restype = ctypes.c_char_p
    return lib


def test_header_declares_the_entry_points():
    names = header_functions()
    for want in ("clamp_plan_create", "clamp_plan_destroy", "clamp_plan_workspace_size",
                 "clamp_aperture_op", "clamp_fwd_init", "clamp_fwd_agent", "clamp_prior_gauss",
                 "clamp_mace_step", "clamp_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def _create(lib, scene):
    h = ctypes.c_void_p()
    st = lib.clamp_plan_create(ctypes.byref(scene), 1, ctypes.byref(h))
    return st, h


def test_plan_create_rejects_unsupported_lengths(lib):
    st, h = _create(lib, Scene(100, 64, 4, 2, 10.0, None))
    assert st == -3 and not h.value
    assert b"supported" in lib.clamp_last_error()
    st, _ = _create(lib, Scene(64, 1024, 4, 2, 10.0, None))
    assert st == -3


def test_plan_create_rejects_bad_scenes(lib):
    assert _create(lib, Scene(64, 64, 0, 2, 10.0, None))[0] == -1
    assert _create(lib, Scene(64, 64, 4, 0, 10.0, None))[0] == -1
    assert _create(lib, Scene(64, 64, 4, 2, 0.0, None))[0] == -1
    assert _create(lib, Scene(64, 64, 4, 2, float("nan"), None))[0] == -1
    h = ctypes.c_void_p()
    assert lib.clamp_plan_create(None, 1, ctypes.byref(h)) == -1
    assert lib.clamp_plan_create(ctypes.byref(Scene(64, 64, 4, 2, 8.0, None)), 0, ctypes.byref(h)) == -1
    assert lib.clamp_plan_create(ctypes.byref(Scene(64, 64, 4, 2, 8.0, None)), 1, None) == -1


def test_calls_reject_null_plan(lib):
    assert lib.clamp_aperture_op(None, 0, 0, None, None, 1, None, None) == -1
    assert lib.clamp_fwd_agent(None, 0, None, None, None, None, None, None, None) == -1
    assert lib.clamp_mace_step(None, 0, None, None, None, None, None, None, None) == -1
    assert lib.clamp_prior_gauss(None, 0, ctypes.c_float(1.0), None, None, None, None) == -1
    assert lib.clamp_plan_set_timing_stages(None, ctypes.c_uint32(1)) == -1
    assert lib.clamp_plan_destroy(None) == 0
    assert b"plan" in lib.clamp_last_error()


def test_valid_plan_without_gpu_reports_device_error(lib):
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    st, h = _create(lib, Scene(64, 64, 4, 2, 16.0, None))
    assert st == -4 and not h.value


def test_unet_workspace_size_checks_shapes(lib):
    b = ctypes.c_size_t()
    ok = lib.clamp_unet_workspace_size(1, 8, 16, 128, 0, ctypes.byref(b))
    assert ok == 0 and b.value > 0
    for dims in ((1, 12, 16, 128), (1, 8, 20, 128), (1, 8, 16, 96), (0, 8, 16, 128)):
        assert lib.clamp_unet_workspace_size(*dims, 0, ctypes.byref(b)) != 0
