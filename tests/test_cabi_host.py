"""Host-side checks of libtb.so: it loads, exports every symbol include/tb.h
declares, and validates its arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_2411_03029_amd as tb
from paper_2411_03029_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    with open(os.path.join(ROOT, "include", "tb.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tb_[a-z_0-9]+)\s*\(", text)))


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_header_symbols_exported():
    lib = _lib.load()
    names = _header_functions()
    assert set(names) == set(_lib.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_library_is_gfx950():
    with open(_lib.LIB_PATH, "rb") as fh:
        blob = fh.read()
    assert b"gfx950" in blob


def test_status_strings():
    lib = _lib.load()
    for code, name in enumerate(["TB_OK", "TB_ERR_INVALID_ARG", "TB_ERR_UNSUPPORTED",
                                 "TB_ERR_OOM", "TB_ERR_HIP", "TB_ERR_NUMERIC", "TB_ERR_IO"]):
        assert lib.tb_status_string(code).decode() == name


@pytest.mark.parametrize("args,status", [
    ((_lib.TB_KERNEL_FOURIER, 2, 64, 0.0, 0.0), _lib.TB_ERR_INVALID_ARG),    # tol
    ((_lib.TB_KERNEL_FOURIER, 2, 64, 0.0, 1.5), _lib.TB_ERR_INVALID_ARG),    # tol
    ((_lib.TB_KERNEL_FOURIER, 2, 60, 0.0, 1e-3), _lib.TB_ERR_INVALID_ARG),   # n != 8*2^L
    ((_lib.TB_KERNEL_HELMHOLTZ, 3, 64, 0.0, 1e-3), _lib.TB_ERR_INVALID_ARG), # omega
    ((_lib.TB_KERNEL_HELMHOLTZ, 4, 64, 1.0, 1e-3), _lib.TB_ERR_UNSUPPORTED), # d
    ((_lib.TB_KERNEL_RADON, 1, 64, 0.0, 1e-3), _lib.TB_ERR_UNSUPPORTED),     # d
    ((7, 2, 64, 0.0, 1e-3), _lib.TB_ERR_INVALID_ARG),                        # kind
    ((_lib.TB_KERNEL_NUDFT, 2, 64, 0.0, 1e-3), _lib.TB_ERR_INVALID_ARG),     # no coordinates
])
def test_construct_rejects_bad_arguments(args, status):
    lib = _lib.load()
    h = ctypes.c_void_p(123)
    got = lib.tb_construct(*args, None, None, ctypes.byref(h))
    assert got == status
    assert h.value is None
    assert len(lib.tb_last_error()) > 0


def test_null_plan_and_pointers():
    lib = _lib.load()
    assert lib.tb_apply(None, None, None, 1, 1, None) == _lib.TB_ERR_INVALID_ARG
    assert lib.tb_apply_adjoint(None, None, None, 1, 1, None) == _lib.TB_ERR_INVALID_ARG
    assert lib.tb_apply_noalloc(None, None, None, 1, 1, 0, None) == _lib.TB_ERR_INVALID_ARG
    assert lib.tb_plan_info(None, None) == _lib.TB_ERR_INVALID_ARG
    assert lib.tb_plan_save(None, b"/tmp/x") == _lib.TB_ERR_INVALID_ARG
    assert lib.tb_plan_autotune(None, 1, 1, None, None, None) == _lib.TB_ERR_INVALID_ARG
    lib.tb_destroy(None)


def test_plan_load_errors(tmp_path):
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.tb_plan_load(str(tmp_path / "missing").encode(), None, 0, None,
                            ctypes.byref(h)) == _lib.TB_ERR_IO
    bad = tmp_path / "bad.tbplan"
    bad.write_bytes(b"TBPLAN01" + b"\0" * 100)
    assert lib.tb_plan_load(str(bad).encode(), None, 0, None, ctypes.byref(h)) == _lib.TB_ERR_IO
    assert b"checksum" in lib.tb_last_error()


def test_plan_load_rejects_corrupted_oracle_file(tmp_path):
    from oracle import butterfly as bf, kernels, planio
    plan = bf.construct(kernels.Operator(kernels.FOURIER, 2, 16), 1e-3)
    raw = bytearray(planio.plan_bytes(plan))
    raw[120] ^= 0x01
    path = tmp_path / "c.tbplan"
    path.write_bytes(bytes(raw))
    h = ctypes.c_void_p()
    assert _lib.load().tb_plan_load(str(path).encode(), None, 0, None,
                                    ctypes.byref(h)) == _lib.TB_ERR_IO


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device error path")
def test_construct_without_device_reports_hip_error():
    with pytest.raises(tb.TBError) as ei:
        tb.construct("fourier", 2, 64, 1e-3)
    assert ei.value.status == _lib.TB_ERR_HIP
