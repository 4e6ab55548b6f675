"""Host-only checks of the C-ABI library: it loads, exports every function that
include/mpg.h declares, and rejects bad arguments before touching the GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mpg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mp_[a-z_]+)\s*\(", src)))


def test_header_declares_boundary():
    names = _declared()
    for n in ["mp_plan_create", "mp_analyze", "mp_run", "mp_get_atoms", "mp_get_coefs",
              "mp_get_energy", "mp_resynth", "mp_plan_destroy", "mp_strerror"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2202_12380_amd import mpg
    L = mpg.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(mpg.EXPORTS) == set(_declared())


def test_strerror_and_argument_errors_without_gpu():
    from paper_2202_12380_amd import mpg
    L = mpg.lib()
    assert L.mp_strerror(0) == b"ok"
    assert b"unsupported Gabor system" in L.mp_strerror(mpg.MP_E_GRID)
    cases = [
        ([(0, 64, 16, 64), (0, 64, 24, 95)], [1024], 1e-4, 0, mpg.MP_E_GRID),   # M odd
        ([(0, 64, 16, 64), (0, 64, 24, 96)], [1024], 1e-4, 0x40, mpg.MP_E_GRID),  # split DFT, M = 96
        ([(0, 1024, 16, 64)], [4096], 1e-4, 0, mpg.MP_E_GRID),                  # gl > 8 M
        ([(3, 64, 16, 64)], [1024], 1e-4, 0, mpg.MP_E_ARG),                     # unknown window
        ([(0, 64, 16, 64)], [64], 1e-4, 0, mpg.MP_E_LEN),                       # too short
        ([(0, 64, 16, 64)], [0], 1e-4, 0, mpg.MP_E_ARG),
        ([(0, 64, 16, 64)], [1024], 1.5, 0, mpg.MP_E_ARG),                      # eps >= 1
        ([(5, 64, 16, 64)], [1024], 1e-4, 0, mpg.MP_E_ARG),                     # window
        ([(0, 64, 16, 64)], [1024], 1e-4, 0x400, mpg.MP_E_ARG),                 # flags
        ([(1, 2, 1, 4)], [64], 1e-4, 0, mpg.MP_E_ARG),                          # one-sample window: real atoms
        ([(0, 64, 16, 64)], [1024], 1e-4, 0x201, mpg.MP_E_ARG),                 # FP64 DFT flag on an FP64 plan
        ([(0, 64, 16, 64)], [1024], 1e-4, 0x240, mpg.MP_E_ARG),                 # two DFT choices
        ([(0, 32768, 8192, 32768)], [65536], 1e-4, 0x200, mpg.MP_E_LIMIT),      # FP64 DFT frame exceeds LDS
        ([(0, 32768, 8192, 32768)], [65536], 1e-4, 1, mpg.MP_E_LIMIT),          # FP64 frame FFT exceeds LDS
        ([(0, 32768, 8192, 32768)], [65536], 1e-4, 0x40, mpg.MP_E_LIMIT),       # split DFT frame exceeds LDS
        ([(0, 64, 16, 64)], [1024], 1e-4, 0x41, mpg.MP_E_ARG),                  # split DFT with FP64
        ([(0, 64, 16, 64)], [1024], 1e-4, 0xC0, mpg.MP_E_ARG),                  # two DFT formats
        ([(0, 64, 16, 64)], [1024], 1e-4, 0x1001, mpg.MP_E_ARG),                # FP32 schedule on an FP64 plan
        ([(0, 64, 16, 64)], [1024], 1e-4, 0x10000, mpg.MP_E_ARG),               # unknown flag bit
        ([(0, 64, 16, 64)], [1024], 1e-4, 0xC000, mpg.MP_E_ARG),                # two tile sizes
        ([(0, 64, 16, 64)], [1024], 1e-4, 0x8000, mpg.MP_E_ARG),                # 32-row tiles need 512 threads
        ([(0, 64, 16, 64)], [1024], 1e-4, 0x4001, mpg.MP_E_ARG),                # tile on an FP64 plan
    ]
    for dicts, lens, eps, flags, code in cases:
        with pytest.raises(mpg.MPError) as e:
            mpg.mp_plan_create(dicts, lens, eps, flags)
        assert e.value.code == code, (dicts, lens, e.value.code)
    # null handles
    assert L.mp_plan_destroy(None) == mpg.MP_E_ARG
    assert L.mp_run(None, 0, 0.0, None) == mpg.MP_E_ARG
    assert L.mp_run_resets(None, None, 0, 0, 0.0, 1, 0.0, None) == mpg.MP_E_ARG
    assert L.mp_resynth(None, 0, None, 0, None) == mpg.MP_E_ARG
    assert L.mp_resynth_static(None, 0, None, 0, None) == mpg.MP_E_ARG
    # autotuner: bad arguments are rejected before any plan is made
    import ctypes as C
    arr = (mpg.mp_dict * 1)(mpg.mp_dict(0, 64, 16, 64))
    Ls = (C.c_int64 * 1)(1024)
    out = C.c_void_p()
    fake_x = C.c_void_p(16)  # never dereferenced: every case fails validation first
    assert L.mp_autotune(arr, 1, Ls, 1, 1e-4, 0, fake_x, 0, 100, None, None, None) == mpg.MP_E_ARG
    assert L.mp_autotune(arr, 1, Ls, 1, 1e-4, 0, None, 0, 100, None, C.byref(out), None) == mpg.MP_E_ARG
    assert L.mp_autotune(arr, 1, Ls, 1, 1e-4, 0, fake_x, 0, 0, None, C.byref(out), None) == mpg.MP_E_ARG
    for f in (mpg.MP_SCHED_NT512, mpg.MP_SCHED_TILE8, mpg.MP_SCHED_TILE32):
        assert L.mp_autotune(arr, 1, Ls, 1, 1e-4, f, fake_x, 0, 100, None, C.byref(out), None) == mpg.MP_E_ARG
    assert out.value is None


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2202_12380_amd import mpg
    monkeypatch.setattr(mpg, "_lib", None)
    monkeypatch.setattr(mpg, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        mpg.lib()
