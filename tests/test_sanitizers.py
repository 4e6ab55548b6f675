"""Host-side sanitizer runs (CPU only).

* The FP64 oracle is rebuilt with gcc's AddressSanitizer and
  UndefinedBehaviorSanitizer (aborting on the first report) and driven
  through its whole API: analysis, kernel tables, MP in every mode (plain,
  pedantic, gamma-gated, relative threshold, eps = 0, common grids of
  non-nested hops and of channel counts that are not powers of two, folded
  windows), replay, resets, synthesis, argument errors.
* The host code of libmpg (plan validation, padding, layout arithmetic, the
  C-ABI's argument checks) is rebuilt with clang's sanitizers on the host
  side only and driven through every entry point that a CPU-only host
  reaches: invalid arguments of all kinds, valid plans (which then stop at
  the missing device), null handles.
Each run is a child process with the sanitizer runtime preloaded.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow


def _run(code, preload, env_extra=None):
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = ROOT
    if env_extra:
        env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=1500)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    return r.stdout


ORACLE_DRIVER = r'''
import sys
import numpy as np
import oracle.build as B
B.build = lambda *a, **k: sys.argv[1]
from oracle import core as O
rng = np.random.default_rng(5)
cfgs = [
    ([(0, 64, 16, 64), (0, 128, 32, 128)], 1024, 1e-4, 0),
    ([(1, 32, 8, 32), (2, 64, 16, 32)], 512, 1e-3, O.PEDANTIC),
    ([(0, 32, 8, 32), (0, 64, 16, 64)], 512, 1e-3, O.CONJ_GATE_GAMMA),
    ([(0, 64, 16, 64), (0, 256, 64, 256)], 1024, 1e-3, O.THR_REL),
    ([(0, 16, 4, 16), (0, 32, 8, 32)], 128, 0.0, 0),
    ([(0, 64, 24, 64), (1, 128, 40, 128)], 960, 1e-4, 0),
    ([(0, 24, 6, 24), (0, 32, 8, 32)], 192, 1e-4, 0),
    ([(1, 36, 9, 12), (0, 20, 5, 20)], 240, 1e-3, 0),
    ([(2, 128, 16, 64), (0, 96, 16, 64)], 1024, 1e-4, O.KEEP_BOX),
]
for dicts, L, eps, fl in cfgs:
    x = rng.standard_normal(L - 7)
    r = O.mp(dicts, x, eps, K=60, flags=fl)
    O.mp_replay(dicts, x, eps, r.w, r.m, r.n, flags=fl, return_planes=True)
    O.resynth(dicts, r.L_padded, r.w, r.m, r.n, r.c)
    for d in dicts:
        xp = np.zeros(O.padded_length(dicts, len(x)))
        xp[:len(x)] = x
        O.dgt(d, xp)
        O.dgt(d, xp, direct=True)
    for dw in dicts:
        for dv in dicts:
            O.kernel_table(dw, dv, eps)
    O.mp_resets(dicts, x, eps, K=80, reset_it=20)
    O.kernel_direct(dicts[0], dicts[-1], 3, dicts[0][2])
for n in (1, 2, 6, 8, 12, 64):
    a = rng.standard_normal(n)
    O.dft(a)
    if n & (n - 1) == 0:
        O.fft(a)
# argument errors
for bad in ([(0, 64, 16, 63)], [(0, 1024, 16, 64)], [(3, 64, 16, 64)], [(1, 2, 1, 4)]):
    O.check_dicts(bad)
print("oracle ok")
'''


def test_oracle_under_address_and_ub_sanitizers():
    with tempfile.TemporaryDirectory() as td:
        lib = os.path.join(td, "libmporacle_san.so")
        subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fPIC", "-shared",
                        "-o", lib, os.path.join(ROOT, "oracle", "mp_oracle.c"), "-lm"], check=True)
        pre = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
        pre2 = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
        out = _run(ORACLE_DRIVER.replace("sys.argv[1]", repr(lib)), pre + ":" + pre2)
        assert "oracle ok" in out


HOST_DRIVER = r'''
import ctypes as C
from paper_2202_12380_amd import mpg
mpg.LIB_PATH = LIBPATH
L = mpg.lib()
assert L.mp_strerror(0) == b"ok"
for code in range(-9, 1):
    L.mp_strerror(code)
cases = [
    ([(0, 64, 16, 64), (0, 64, 24, 95)], [1024], 1e-4, 0),
    ([(0, 64, 16, 64), (0, 64, 24, 96)], [1024], 1e-4, 0x40),
    ([(0, 1024, 16, 64)], [4096], 1e-4, 0),
    ([(3, 64, 16, 64)], [1024], 1e-4, 0),
    ([(0, 64, 16, 64)], [64], 1e-4, 0),
    ([(0, 64, 16, 64)], [0], 1e-4, 0),
    ([(0, 64, 16, 64)], [1024], 1.5, 0),
    ([(0, 64, 16, 64)], [1024], 1e-4, 0x400),
    ([(1, 2, 1, 4)], [64], 1e-4, 0),
    ([(0, 64, 16, 64)], [1024], 1e-4, 0x241),
    ([(0, 32768, 8192, 32768)], [65536], 1e-4, 0x200),
    ([(0, 32768, 8192, 32768)], [65536], 1e-4, 1),
    ([(0, 64, 16, 64)], [1024], 1e-4, 0x1001),
    # valid plans: validation and layout run, then the missing device stops them
    ([(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)], [16384, 30000, 999], 1e-4, 0),
    ([(0, 96, 24, 96), (0, 128, 32, 128)], [3000], 1e-4, 1),
    ([(2, 128, 16, 64), (0, 64, 24, 64)], [5000], 1e-3, 0x130),
]
for dicts, lens, eps, flags in cases:
    try:
        mpg.mp_plan_create(dicts, lens, eps, flags)
    except mpg.MPError as e:
        assert e.code < 0
arr = (mpg.mp_dict * 1)(mpg.mp_dict(0, 64, 16, 64))
Ls = (C.c_int64 * 1)(1024)
out = C.c_void_p()
assert L.mp_plan_create(None, 1, Ls, 1, 1e-4, 0, C.byref(out)) == mpg.MP_E_ARG
assert L.mp_plan_create(arr, 0, Ls, 1, 1e-4, 0, C.byref(out)) == mpg.MP_E_ARG
assert L.mp_plan_create(arr, 1, Ls, 1, 1e-4, 0, None) == mpg.MP_E_ARG
for f in (L.mp_run, L.mp_plan_destroy):
    pass
assert L.mp_plan_destroy(None) == mpg.MP_E_ARG
assert L.mp_run(None, 0, 0.0, None) == mpg.MP_E_ARG
assert L.mp_run_resets(None, None, 0, 0, 0.0, 1, 0.0, None) == mpg.MP_E_ARG
assert L.mp_resynth(None, 0, None, 0, None) == mpg.MP_E_ARG
assert L.mp_resynth_static(None, 0, None, 0, None) == mpg.MP_E_ARG
fake_x = C.c_void_p(16)
assert L.mp_autotune(arr, 1, Ls, 1, 1e-4, 0, fake_x, 0, 0, None, C.byref(out), None) == mpg.MP_E_ARG
print("host ok")
'''


def test_library_host_code_under_address_and_ub_sanitizers():
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    rt = None
    base = "/opt/rocm/llvm/lib/clang"
    if os.path.isdir(base):
        for v in sorted(os.listdir(base)):
            c = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
            if os.path.exists(c):
                rt = c
    if rt is None:
        pytest.skip("clang ASan runtime not available")
    csrc = os.path.join(ROOT, "paper_2202_12380_amd", "csrc")
    with tempfile.TemporaryDirectory() as td:
        objs = []
        for src in ("mpg_api.cpp", "mpg_kernels.hip"):
            o = os.path.join(td, src + ".o")
            # sanitizers on the host compilation only (device code is unchanged)
            cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                   "-Xarch_host", "-fsanitize=address,undefined",
                   "-Xarch_host", "-fno-sanitize-recover=all",
                   "-Xarch_host", "-fno-omit-frame-pointer",
                   "-I", os.path.join(ROOT, "include"), "-I", csrc, "-x", "hip", "-c", os.path.join(csrc, src),
                   "-o", o]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-3000:]
            objs.append(o)
        lib = os.path.join(td, "libmpg_san.so")
        r = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libasan",
                            "-Xarch_host", "-fsanitize=address,undefined", "-o", lib, *objs,
                            "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        out = _run(HOST_DRIVER.replace("LIBPATH", repr(lib)), rt)
        assert "host ok" in out
