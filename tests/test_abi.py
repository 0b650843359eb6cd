"""The C-ABI library loads, exports every declared symbol and rejects bad
arguments on the host before touching the GPU (no GPU needed)."""
import ctypes

import pytest

import paper_2403_18619_amd as fw
from paper_2403_18619_amd import _binding as B


def test_exports_every_header_symbol():
    syms = fw.header_symbols()
    assert {"fw_solve_i32", "fw_solve_f32", "fw_solve_ex_i32", "fw_solve_ex_f32",
            "fw_check", "fw_status_string", "fw_last_error", "fw_version",
            "fw_phase_times", "fw_solve_batched_i32", "fw_solve_batched_f32",
            "fw_backward_f32", "fw_backward_batched_f32"} <= set(syms)
    raw = ctypes.CDLL(fw.LIB_PATH)
    for s in syms:
        assert hasattr(raw, s), f"{s} declared in fw.h but not exported"


def test_version_and_status_strings():
    assert fw.version() >> 16 == 1
    for code in (0, -1, -2, -3, -4, -5):
        assert fw.status_string(code).startswith("FW_")
    assert fw.status_string(42) == "unknown status"


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails its host check


@pytest.mark.parametrize("fn", ["fw_solve_i32", "fw_solve_f32"])
def test_invalid_arguments_rejected_on_host(fn):
    f = getattr(fw.lib, fn)
    assert f(FAKE, None, -1, 4, None) == fw.FW_ERR_INVALID_ARG
    assert "negative" in fw.last_error()
    assert f(None, None, 4, 4, None) == fw.FW_ERR_INVALID_ARG
    assert "NULL" in fw.last_error()
    assert f(FAKE, None, 8, 7, None) == fw.FW_ERR_INVALID_ARG
    assert "ld" in fw.last_error()
    assert f(FAKE, None, 1 << 31, 1 << 31, None) == fw.FW_ERR_INVALID_ARG
    assert f(FAKE, None, 1 << 30, 1 << 60, None) == fw.FW_ERR_INVALID_ARG
    assert f(None, None, 0, 0, None) == fw.FW_OK          # empty problem: a no-op


@pytest.mark.parametrize("fn", ["fw_solve_ex_i32", "fw_solve_ex_f32"])
def test_invalid_options_rejected_on_host(fn):
    f = getattr(fw.lib, fn)
    for opt in (B.fw_options(48, 0, 0, 0), B.fw_options(256, 0, 0, 0), B.fw_options(0, 7, 0, 0),
                B.fw_options(0, -1, 0, 0), B.fw_options(0, 0, 0, 32)):
        assert f(FAKE, None, 16, 16, ctypes.byref(opt), None) == fw.FW_ERR_INVALID_ARG
        assert fw.last_error()
    # a valid request the persistent schedule does not run: refused on the host
    opt = B.fw_options(64, fw.SCHED_PERSISTENT, 0, 0)
    assert f(FAKE, None, 16, 16, ctypes.byref(opt), None) == fw.FW_ERR_UNSUPPORTED
    assert "128" in fw.last_error()


def test_python_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError):
        fw.solve(torch.zeros(4, 4, dtype=torch.int32))


@pytest.mark.parametrize("fn", ["fw_solve_batched_i32", "fw_solve_batched_f32"])
def test_batched_invalid_arguments_rejected_on_host(fn):
    f = getattr(fw.lib, fn)
    assert f(FAKE, None, FAKE, FAKE, -1, 16, None, None) == fw.FW_ERR_INVALID_ARG
    assert f(None, None, FAKE, FAKE, 4, 16, None, None) == fw.FW_ERR_INVALID_ARG
    assert f(FAKE, None, None, FAKE, 4, 16, None, None) == fw.FW_ERR_INVALID_ARG
    assert f(FAKE, None, FAKE, FAKE, 4, 0, None, None) == fw.FW_ERR_INVALID_ARG
    assert f(FAKE, None, FAKE, FAKE, 4, 1 << 20, None, None) == fw.FW_ERR_INVALID_ARG
    opt = B.fw_options(64, 0, 0, 0)
    assert f(FAKE, None, FAKE, FAKE, 4, 16, ctypes.byref(opt), None) == fw.FW_ERR_UNSUPPORTED
    assert f(None, None, None, None, 0, 16, None, None) == fw.FW_OK


def test_backward_invalid_arguments_rejected_on_host():
    f = fw.lib.fw_backward_f32
    assert f(FAKE, FAKE, FAKE, -1, 4, None) == fw.FW_ERR_INVALID_ARG
    assert f(FAKE, FAKE, FAKE, 8, 7, None) == fw.FW_ERR_INVALID_ARG
    assert f(None, FAKE, FAKE, 4, 4, None) == fw.FW_ERR_INVALID_ARG
    assert f(FAKE, None, FAKE, 4, 4, None) == fw.FW_ERR_INVALID_ARG
    assert f(FAKE, FAKE, None, 4, 4, None) == fw.FW_ERR_INVALID_ARG
    assert f(None, None, None, 0, 0, None) == fw.FW_OK
    g = fw.lib.fw_backward_batched_f32
    assert g(FAKE, FAKE, FAKE, FAKE, FAKE, -1, 16, None) == fw.FW_ERR_INVALID_ARG
    assert g(FAKE, FAKE, FAKE, None, FAKE, 4, 16, None) == fw.FW_ERR_INVALID_ARG
    assert g(FAKE, None, FAKE, FAKE, FAKE, 4, 16, None) == fw.FW_ERR_INVALID_ARG
    assert g(FAKE, FAKE, FAKE, FAKE, FAKE, 4, 0, None) == fw.FW_ERR_INVALID_ARG
    assert g(FAKE, FAKE, FAKE, FAKE, FAKE, 4, 4097, None) == fw.FW_ERR_UNSUPPORTED
    assert "4096" in fw.last_error()
    assert g(FAKE, FAKE, FAKE, FAKE, FAKE, 70000, 16, None) == fw.FW_ERR_UNSUPPORTED
    assert g(None, None, None, None, None, 0, 16, None) == fw.FW_OK


def test_tuners_reject_bad_arguments_on_host():
    i32, dbl = ctypes.c_int32(), ctypes.c_double()
    for fn in (fw.lib.fw_tune_batched_i32, fw.lib.fw_tune_batched_f32):
        assert fn(FAKE, None, FAKE, FAKE, -1, 16, 10, 1, ctypes.byref(i32), ctypes.byref(dbl), None) == fw.FW_ERR_INVALID_ARG
        assert fn(None, None, FAKE, FAKE, 4, 16, 10, 1, ctypes.byref(i32), ctypes.byref(dbl), None) == fw.FW_ERR_INVALID_ARG
        assert fn(FAKE, None, FAKE, FAKE, 4, 0, 10, 1, ctypes.byref(i32), ctypes.byref(dbl), None) == fw.FW_ERR_INVALID_ARG
        assert fn(FAKE, None, FAKE, FAKE, 4, 16, -1, 1, ctypes.byref(i32), ctypes.byref(dbl), None) == fw.FW_ERR_INVALID_ARG
        assert fn(FAKE, None, FAKE, FAKE, 4, 16, 10, 0, ctypes.byref(i32), ctypes.byref(dbl), None) == fw.FW_ERR_INVALID_ARG
        assert fn(None, None, None, None, 0, 16, 0, 1, None, None, None) == fw.FW_OK
    for fn in (fw.lib.fw_tune_solve_i32, fw.lib.fw_tune_solve_f32):
        assert fn(FAKE, None, -1, 4, 1, None, None, None, None) == fw.FW_ERR_INVALID_ARG
        assert fn(FAKE, None, 8, 7, 1, None, None, None, None) == fw.FW_ERR_INVALID_ARG
        assert fn(FAKE, None, 8, 8, 0, None, None, None, None) == fw.FW_ERR_INVALID_ARG
        assert fn(None, None, 0, 0, 1, None, None, None, None) == fw.FW_OK


def test_batched_rejects_negative_team():
    opt = B.fw_options(0, 0, 0, 0, -2)
    assert fw.lib.fw_solve_batched_f32(FAKE, None, FAKE, FAKE, 4, 16, ctypes.byref(opt), None) == fw.FW_ERR_INVALID_ARG


def test_f64_entry_points_reject_bad_arguments_on_host():
    assert fw.lib.fw_solve_f64(FAKE, None, -1, 4, None) == fw.FW_ERR_INVALID_ARG
    assert fw.lib.fw_solve_f64(FAKE, None, 8, 7, None) == fw.FW_ERR_INVALID_ARG
    assert fw.lib.fw_solve_f64(FAKE, None, 1 << 30, 1 << 59, None) == fw.FW_ERR_INVALID_ARG   # 8-byte elements overflow
    assert fw.lib.fw_solve_f64(None, None, 0, 0, None) == fw.FW_OK
    opt = B.fw_options(48, 0, 0, 0, 0)
    assert fw.lib.fw_solve_ex_f64(FAKE, None, 16, 16, ctypes.byref(opt), None) == fw.FW_ERR_INVALID_ARG
    assert fw.lib.fw_solve_batched_f64(FAKE, None, FAKE, FAKE, -1, 16, None, None) == fw.FW_ERR_INVALID_ARG
