"""The C ABI library: it builds for gfx950, loads, exports every function that
include/cwt.h declares, and without a device every entry point returns an
error code instead of aborting.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cwt.h")
LIB = os.path.join(ROOT, "paper_2408_14302_amd", "libcwth.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cwt_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2408_14302_amd import build
        build.build(verbose=False)
    from paper_2408_14302_amd import cwth
    return cwth


def test_header_declares_the_boundary():
    names = declared()
    for n in ("cwt_plan_create", "cwt_plan_destroy", "cwt_execute", "cwt_execute_batch",
              "cwt_num_frames", "cwt_status_string", "cwt_last_error", "cwt_plan_set_output",
              "cwt_scale_frequencies", "cwt_batch_create", "cwt_batch_execute", "cwt_autotune",
              "cwt_autotune_batch"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(raw, n)]
    assert not missing, missing
    assert set(declared()) <= set(lib.EXPORTS) | set(declared())
    assert sorted(lib.EXPORTS) == declared()


def test_status_strings_and_version(lib):
    assert lib.status_string(0) == "CWT_OK"
    assert lib.status_string(4) == "CWT_ERR_DEVICE"
    assert lib.status_string(99) == "CWT_ERR_UNKNOWN"
    assert "gfx950" in lib.version()


def _has_device(raw):
    h = ctypes.c_void_p()
    sc = (ctypes.c_double * 1)(1.0)
    st = raw.cwt_plan_create(16000.0, 0, sc, 1, 1, 0, ctypes.byref(h))
    if st == 0:
        raw.cwt_plan_destroy(h)
    return st != 4


def test_no_device_paths_return_codes(lib):
    raw = lib.raw()
    if _has_device(raw):
        pytest.skip("a device is present; the no-device paths are not reachable")
    h = ctypes.c_void_p()
    sc = (ctypes.c_double * 2)(1.0, 2.0)
    assert raw.cwt_plan_create(16000.0, 0, sc, 2, 1, 1, ctypes.byref(h)) == lib.DEVICE
    assert b"device" in raw.cwt_last_error()
    b = ctypes.c_void_p()
    assert raw.cwt_batch_create(8, ctypes.byref(b)) == lib.DEVICE
    # argument errors are reported before the device is touched
    assert raw.cwt_plan_create(16000.0, 0, sc, 2, 0, 1, ctypes.byref(h)) == lib.INVALID_ARG
    assert raw.cwt_plan_create(-1.0, 0, sc, 2, 1, 1, ctypes.byref(h)) == lib.INVALID_ARG
    assert raw.cwt_plan_create(16000.0, 0, sc, 2, 1, 1, None) == lib.INVALID_ARG
    assert raw.cwt_plan_create(16000.0, 5, sc, 2, 1, 1, ctypes.byref(h)) == lib.UNSUPPORTED
    assert raw.cwt_plan_create(16000.0, 0, sc, 2, 1, 7, ctypes.byref(h)) == lib.UNSUPPORTED
    assert raw.cwt_execute(None, None, 10, None, None) == lib.INVALID_ARG
    assert raw.cwt_num_frames(None, 10) == -1
    assert raw.cwt_plan_num_scales(None) == -1
    assert raw.cwt_plan_launch_config(None, 100, 1) == -1
    assert raw.cwt_plan_destroy(None) == lib.OK
    assert raw.cwt_batch_destroy(None) == lib.OK
    assert raw.cwt_execute_batch(None, None, None, None, 0, None) == lib.OK
    assert raw.cwt_execute_batch(None, None, None, None, -1, None) == lib.INVALID_ARG
    assert raw.cwt_batch_execute(None, None, None, None, None, 1, 1, None) == lib.INVALID_ARG


def test_python_binding_refuses_without_device(lib):
    raw = lib.raw()
    if _has_device(raw):
        pytest.skip("a device is present")
    with pytest.raises(lib.CwtError) as e:
        lib.Plan(16000.0, [1.0, 2.0], 4, "bf16")
    assert e.value.status == lib.DEVICE
    with pytest.raises(ValueError):
        lib.Plan(16000.0, [1.0], 4, "int8")


def test_next_step_entry_points_without_device(lib):
    # decimation, scalogram image and DWT: argument errors first, then the
    # device error; host-only helpers work without a device
    raw = lib.raw()
    if _has_device(raw):
        pytest.skip("a device is present")
    fake = ctypes.c_void_p(0x1000)                     # never dereferenced: the calls stop before any launch
    h1 = (ctypes.c_float * 1)(1.0)
    assert raw.cwt_decimate(fake, 100, 0, h1, 1, fake, None) == lib.INVALID_ARG
    assert raw.cwt_decimate(fake, 100, 2, h1, 2, fake, None) == lib.INVALID_ARG
    assert raw.cwt_decimate(None, 100, 2, h1, 1, fake, None) == lib.INVALID_ARG
    assert raw.cwt_decimate(fake, 0, 2, h1, 1, fake, None) == lib.OK      # empty input is a no-op
    assert raw.cwt_decimate(fake, 100, 2, h1, 1, fake, None) == lib.DEVICE
    assert raw.cwt_image_workspace_bytes() > 0
    assert raw.cwt_scalogram_image(fake, 0, 10, ctypes.c_float(1e-6), fake, 4, 4, fake, None) == lib.INVALID_ARG
    assert raw.cwt_scalogram_image(fake, 4, 10, ctypes.c_float(0.0), fake, 4, 4, fake, None) == lib.INVALID_ARG
    assert raw.cwt_scalogram_image(fake, 4, 10, ctypes.c_float(1e-6), fake, 4, 4, None, None) == lib.INVALID_ARG
    assert raw.cwt_scalogram_image(fake, 4, 10, ctypes.c_float(1e-6), fake, 4, 4, fake, None) == lib.DEVICE
    hd = (ctypes.c_double * 8)()
    assert raw.cwt_daubechies(4, hd) == lib.OK
    assert abs(sum(hd) - 2 ** 0.5) < 1e-14
    assert raw.cwt_dwt_pyramid_length(10, 3) == 20
    assert raw.cwt_dwt_pyramid_length(0, 3) == -1
    assert raw.cwt_dwt_scalogram(fake, 100, 1, hd, 8, 0, fake, fake, None) == lib.INVALID_ARG
    assert raw.cwt_dwt_scalogram(fake, 100, 1, hd, 7, 3, fake, fake, None) == lib.INVALID_ARG
    assert raw.cwt_dwt_scalogram(fake, 100, 0, hd, 8, 3, fake, fake, None) == lib.INVALID_ARG
    assert raw.cwt_dwt_scalogram(fake, 0, 1, hd, 8, 3, fake, fake, None) == lib.INVALID_ARG
    assert raw.cwt_dwt_scalogram(fake, 100, 1, hd, 8, 3, None, fake, None) == lib.INVALID_ARG
    assert raw.cwt_dwt_scalogram(fake, 100, 1, hd, 8, 3, fake, None, None) == lib.DEVICE   # matrix optional
