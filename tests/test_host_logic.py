"""Host-side logic without a GPU: the library's host-only entry points (the
training schedule, workspace sizing, argument checks that return before any
device call) and the benchmark's contract and accounting."""

import ctypes
import os
import subprocess
import sys

import pytest

from oracle import training as otr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2502_01157_amd", "librf.so")


class _AdamArgs(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 4), ("t", ctypes.c_int32 * 4), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("softplus_density", ctypes.c_int32)]


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librf.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    lib.rf_last_error.restype = ctypes.c_char_p
    lib.rf_train_schedule.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_AdamArgs)]
    lib.rf_sample_workspace.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
    lib.rf_adam_step.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p] + [ctypes.c_void_p] * 8
    return lib


def test_training_schedule_matches_the_oracle(lib):
    for total in (40, 1000, 20000):
        for it in sorted({0, 1, total // 4 - 1, total // 4, total // 3, total - total // 10 - 1,
                          total - total // 10, total - 1}):
            a = _AdamArgs()
            assert lib.rf_train_schedule(it, total, ctypes.byref(a)) == 0
            ref = otr.schedule(it, total)
            for g, name in enumerate(otr.GROUPS):
                assert a.lr[g] == pytest.approx(ref["lr"][name], rel=1e-6, abs=0.0), (it, name)
                assert a.t[g] == ref["t"][name], (it, name)
    a = _AdamArgs()
    assert lib.rf_train_schedule(5, 5, ctypes.byref(a)) == 1
    assert b"outside" in lib.rf_last_error()
    assert lib.rf_train_schedule(-1, 5, ctypes.byref(a)) == 1


def test_sample_workspace_and_argument_checks(lib):
    n = ctypes.c_size_t()
    assert lib.rf_sample_workspace(1_000_000, ctypes.byref(n)) == 0
    assert n.value == 8 * (1_000_000 + (1_000_000 + 1023) // 1024)
    assert lib.rf_sample_workspace(-1, ctypes.byref(n)) == 1
    # a NULL state or a moving group without a step count is refused before any launch
    # (the array arguments are placeholders: the library only checks them for NULL here)
    a = _AdamArgs()
    assert lib.rf_train_schedule(10, 40, ctypes.byref(a)) == 0
    assert lib.rf_adam_step(10, 3, ctypes.addressof(a), *([None] * 7), None) == 1
    state = (ctypes.c_void_p * 6)(*([16] * 6))
    a.t[1] = 0
    assert lib.rf_adam_step(10, 3, ctypes.addressof(a), *([16] * 6), ctypes.addressof(state), None) == 1
    assert b"step count" in lib.rf_last_error()
    a.t[1] = 11
    a.beta2 = 1.0
    assert lib.rf_adam_step(10, 3, ctypes.addressof(a), *([16] * 6), ctypes.addressof(state), None) == 1
    assert b"betas" in lib.rf_last_error()
    assert lib.rf_adam_step(10, 4, ctypes.addressof(a), *([16] * 6), ctypes.addressof(state), None) == 1


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_bench_accounting():
    sys.path.insert(0, ROOT)
    import bench

    # SH degree 3 (B = 16), mean degree 17: forward 13 per face + 6B + 12, logged backward 6B + 12 + 14 + 6B + 2 + 20
    assert bench.flops_per_visit(17.0, 16, "forward") == 13 * 17 + 96 + 12
    assert bench.flops_per_visit(17.0, 16, "backward") == 240
    assert bench.flops_per_visit(17.0, 16, "backward_recompute") == 13 * 17 + 240
    # bytes of a visited cell: row offsets, 4 + 12 bytes per face, 49 attributes
    assert bench.visit_bytes(17.0, 16, "f32") == 4 + 16 * 17 + 49 * 4
    assert bench.visit_bytes(17.0, 16, "bf16") == 4 + 16 * 17 + 49 * 2
    assert bench.visit_bytes(17.0, 16, "f32", "backward_recompute") == 4 + 16 * 17 + 49 * 4 + 52 * 4
    assert bench.visit_bytes(17.0, 16, "bf16", "backward") == 24 + 49 * 2 + 52 * 4
    assert bench.VALU_PEAK_TFLOPS == pytest.approx(78.64, rel=1e-3)
    assert bench.FP32_PEAK_TFLOPS == 157.3
