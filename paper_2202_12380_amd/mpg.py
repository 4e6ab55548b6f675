"""Thin ctypes binding of libmpg.so (C-ABI in include/mpg.h).

Argument marshalling only: every step of the pursuit runs in the HIP library.
Device buffers and streams come from PyTorch (``tensor.data_ptr()``,
``torch.cuda.current_stream().cuda_stream``).  Loading fails loudly when the
library has not been built.
"""
import ctypes as C
import os
from typing import Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpg.so")

MP_OK = 0
MP_E_ARG, MP_E_GRID, MP_E_LEN, MP_E_NOMEM, MP_E_HIP, MP_E_STATE, MP_E_LIMIT = range(-1, -8, -1)
MP_WIN_BLACKMAN, MP_WIN_HANN, MP_WIN_GAUSS = 0, 1, 2
MP_PREC_F32, MP_PREC_F64 = 0x0, 0x1
MP_THR_REL, MP_CONJ_GATE_GAMMA = 0x10, 0x20
MP_DFT_F16SPLIT, MP_DFT_BF16SPLIT = 0x40, 0x80
MP_DFT_F32, MP_DFT_F64 = 0x0, 0x200
MP_PEDANTIC = 0x100
MP_SCHED_NT512, MP_SCHED_G128 = 0x1000, 0x2000
MP_SCHED_TILE8, MP_SCHED_TILE32 = 0x4000, 0x8000
MP_TUNE_MAX = 10
MP_DTYPE_F32, MP_DTYPE_F64 = 0, 1
MP_STATIC_RESYNTH_MAX = 1 << 22
MP_STOP_NONE, MP_STOP_K, MP_STOP_SNR, MP_STOP_ENEG, MP_STOP_ZERO = range(5)


class mp_dict(C.Structure):
    _fields_ = [("window", C.c_int32), ("gl", C.c_int32), ("a", C.c_int32), ("M", C.c_int32)]


class mp_atom(C.Structure):
    _fields_ = [("w", C.c_int32), ("m", C.c_int32), ("n", C.c_int32), ("pad", C.c_int32),
                ("re", C.c_double), ("im", C.c_double), ("E_after", C.c_double)]


ATOM_DTYPE = np.dtype([("w", np.int32), ("m", np.int32), ("n", np.int32), ("pad", np.int32),
                       ("re", np.float64), ("im", np.float64), ("E_after", np.float64)])


class mp_signal_info(C.Structure):
    _fields_ = [("L", C.c_int64), ("L_padded", C.c_int64), ("x_offset", C.c_int64),
                ("n_coefs", C.c_int64), ("n_atoms", C.c_int64), ("stop_reason", C.c_int32),
                ("pad", C.c_int32), ("E0", C.c_double), ("E", C.c_double)]


class mp_kernel_info(C.Structure):
    _fields_ = [("amin", C.c_int32), ("Mmax", C.c_int32), ("D", C.c_int32),
                ("delta_box", C.c_int32), ("mu_lo", C.c_int32), ("mu_hi", C.c_int32),
                ("n_nonzero", C.c_int64)]


class mp_tune_report(C.Structure):
    _fields_ = [("n_cand", C.c_int32), ("chosen", C.c_int32), ("flags", C.c_uint32 * MP_TUNE_MAX),
                ("threads", C.c_int32 * MP_TUNE_MAX), ("group_leaves", C.c_int32 * MP_TUNE_MAX),
                ("tile_rows", C.c_int32 * MP_TUNE_MAX), ("probe_ms", C.c_double * MP_TUNE_MAX),
                ("probe_bytes", C.c_double * MP_TUNE_MAX)]

    def as_dict(self):
        n = self.n_cand
        return {"chosen": self.chosen,
                "schedules": [{"flags": int(self.flags[i]), "threads": int(self.threads[i]),
                               "group_leaves": int(self.group_leaves[i]), "tile_rows": int(self.tile_rows[i]),
                               "probe_ms": float(self.probe_ms[i]), "probe_bytes": float(self.probe_bytes[i])}
                              for i in range(n)]}


class mp_stats(C.Structure):
    _fields_ = [("atoms", C.c_int64), ("updated", C.c_int64), ("blocks", C.c_int64),
                ("l1_groups", C.c_int64), ("loop_ms", C.c_double), ("analyze_ms", C.c_double),
                ("dgt_ms", C.c_double), ("group_leaves", C.c_int32), ("threads", C.c_int32),
                ("tile_rows", C.c_int32), ("early_groups", C.c_int32)]


EXPORTS = ["mp_plan_create", "mp_analyze", "mp_run", "mp_run_resets",
           "mp_get_atoms", "mp_get_energy",
           "mp_get_coefs", "mp_get_residual", "mp_resynth", "mp_resynth_static", "mp_signal_info_get",
           "mp_kernel_info_get", "mp_get_kernel", "mp_get_stats", "mp_plan_destroy",
           "mp_autotune", "mp_strerror"]

_lib = None


def lib():
    """Loads libmpg.so; raises if it is missing (no fallback of any kind)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmpg.so is not built: run `python -m paper_2202_12380_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.mp_plan_create.argtypes = [C.POINTER(mp_dict), i32, C.POINTER(C.c_int64), i32, dbl, C.c_uint32,
                                 C.POINTER(vp)]
    L.mp_analyze.argtypes = [vp, vp, i32, vp]
    L.mp_autotune.argtypes = [C.POINTER(mp_dict), i32, C.POINTER(C.c_int64), i32, dbl, C.c_uint32, vp, i32, i64,
                              vp, C.POINTER(vp), C.POINTER(mp_tune_report)]
    L.mp_run.argtypes = [vp, i64, dbl, vp]
    L.mp_run_resets.argtypes = [vp, vp, i32, i64, dbl, i64, dbl, vp]
    L.mp_get_atoms.argtypes = [vp, i32, vp, i64, C.POINTER(C.c_int64)]
    L.mp_get_energy.argtypes = [vp, i32, vp, i64, C.POINTER(C.c_int64)]
    L.mp_get_coefs.argtypes = [vp, i32, i32, vp, vp]
    L.mp_get_residual.argtypes = [vp, i32, i32, vp, vp]
    L.mp_resynth.argtypes = [vp, i32, vp, i32, vp]
    L.mp_resynth_static.argtypes = [vp, i32, vp, i32, vp]
    L.mp_signal_info_get.argtypes = [vp, i32, C.POINTER(mp_signal_info)]
    L.mp_kernel_info_get.argtypes = [vp, i32, i32, C.POINTER(mp_kernel_info)]
    L.mp_get_kernel.argtypes = [vp, i32, i32, vp, vp, i64]
    L.mp_get_stats.argtypes = [vp, C.POINTER(mp_stats)]
    L.mp_plan_destroy.argtypes = [vp]
    L.mp_strerror.argtypes = [C.c_int]
    L.mp_strerror.restype = C.c_char_p
    for name in EXPORTS:
        if name != "mp_strerror":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class MPError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s: %s (%d)" % (what, lib().mp_strerror(code).decode(), code))
        self.code = code


def _chk(rc, what):
    if rc != MP_OK:
        raise MPError(rc, what)


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return int(stream) if not hasattr(stream, "cuda_stream") else stream.cuda_stream


# ----------------------------------------------------------------------------
# functions with the C names (pointers as ints)

def mp_plan_create(dicts: Sequence[Sequence[int]], lengths: Sequence[int], kernel_tol: float,
                   flags: int = 0) -> int:
    W = len(dicts)
    arr = (mp_dict * W)(*[mp_dict(*map(int, d)) for d in dicts])
    Ls = (C.c_int64 * len(lengths))(*map(int, lengths))
    out = C.c_void_p()
    _chk(lib().mp_plan_create(arr, W, Ls, len(lengths), float(kernel_tol), int(flags), C.byref(out)),
         "mp_plan_create")
    return out.value


def mp_autotune(dicts: Sequence[Sequence[int]], lengths: Sequence[int], kernel_tol: float, flags: int,
                x_ptr: int, dtype: int, probe_atoms: int, stream=None):
    """Returns (plan handle, mp_tune_report)."""
    W = len(dicts)
    arr = (mp_dict * W)(*[mp_dict(*map(int, d)) for d in dicts])
    Ls = (C.c_int64 * len(lengths))(*map(int, lengths))
    out = C.c_void_p()
    rep = mp_tune_report()
    _chk(lib().mp_autotune(arr, W, Ls, len(lengths), float(kernel_tol), int(flags), x_ptr, int(dtype),
                           int(probe_atoms), _stream(stream), C.byref(out), C.byref(rep)), "mp_autotune")
    return out.value, rep


def mp_analyze(plan: int, x_ptr: int, dtype: int, stream=None):
    _chk(lib().mp_analyze(plan, x_ptr, dtype, _stream(stream)), "mp_analyze")


def mp_run(plan: int, max_atoms: int = 0, target_snr_db: float = 0.0, stream=None):
    _chk(lib().mp_run(plan, int(max_atoms), float(target_snr_db), _stream(stream)), "mp_run")


def mp_run_resets(plan: int, x_ptr: int, dtype: int, max_atoms: int = 0, target_snr_db: float = 0.0,
                  reset_it: int = 0, reset_db: float = 0.0, stream=None):
    _chk(lib().mp_run_resets(plan, x_ptr, dtype, int(max_atoms), float(target_snr_db), int(reset_it),
                             float(reset_db), _stream(stream)), "mp_run_resets")


def mp_signal_info_get(plan: int, sig: int) -> mp_signal_info:
    inf = mp_signal_info()
    _chk(lib().mp_signal_info_get(plan, sig, C.byref(inf)), "mp_signal_info_get")
    return inf


def mp_get_atoms(plan: int, sig: int) -> np.ndarray:
    n = C.c_int64()
    _chk(lib().mp_get_atoms(plan, sig, None, 0, C.byref(n)), "mp_get_atoms")
    out = np.zeros(n.value, ATOM_DTYPE)
    if n.value:
        _chk(lib().mp_get_atoms(plan, sig, out.ctypes.data, n.value, C.byref(n)), "mp_get_atoms")
    return out


def mp_get_energy(plan: int, sig: int) -> np.ndarray:
    n = C.c_int64()
    _chk(lib().mp_get_energy(plan, sig, None, 0, C.byref(n)), "mp_get_energy")
    out = np.zeros(n.value)
    _chk(lib().mp_get_energy(plan, sig, out.ctypes.data, n.value, C.byref(n)), "mp_get_energy")
    return out


def mp_get_coefs(plan: int, sig: int, w: int, c_ptr: int, stream=None):
    _chk(lib().mp_get_coefs(plan, sig, w, c_ptr, _stream(stream)), "mp_get_coefs")


def mp_get_residual(plan: int, sig: int, w: int, dst_ptr: int, stream=None):
    _chk(lib().mp_get_residual(plan, sig, w, dst_ptr, _stream(stream)), "mp_get_residual")


def mp_resynth(plan: int, sig: int, y_ptr: int, dtype: int, stream=None):
    _chk(lib().mp_resynth(plan, sig, y_ptr, dtype, _stream(stream)), "mp_resynth")


def mp_resynth_static(plan: int, sig: int, y_ptr: int, dtype: int, stream=None):
    _chk(lib().mp_resynth_static(plan, sig, y_ptr, dtype, _stream(stream)), "mp_resynth_static")


def mp_kernel_info_get(plan: int, w: int, v: int) -> mp_kernel_info:
    k = mp_kernel_info()
    _chk(lib().mp_kernel_info_get(plan, w, v, C.byref(k)), "mp_kernel_info_get")
    return k


def mp_get_kernel(plan: int, w: int, v: int) -> np.ndarray:
    k = mp_kernel_info_get(plan, w, v)
    if k.delta_box < 0:
        return np.zeros((0, 0), np.complex128)
    rows, cols = 2 * k.delta_box + 1, k.mu_hi - k.mu_lo + 1
    re = np.zeros(rows * cols)
    im = np.zeros(rows * cols)
    _chk(lib().mp_get_kernel(plan, w, v, re.ctypes.data, im.ctypes.data, rows * cols), "mp_get_kernel")
    return (re + 1j * im).reshape(rows, cols)


def mp_get_stats(plan: int) -> mp_stats:
    s = mp_stats()
    _chk(lib().mp_get_stats(plan, C.byref(s)), "mp_get_stats")
    return s


def mp_plan_destroy(plan: int):
    _chk(lib().mp_plan_destroy(plan), "mp_plan_destroy")


# ----------------------------------------------------------------------------
# convenience wrapper used by tests and the benchmark

class Plan:
    """Owns one mp_plan; torch supplies device memory and the stream."""

    def __init__(self, dicts, lengths, kernel_tol=1e-4, flags=0, _handle=None):
        self.dicts = [tuple(map(int, d)) for d in dicts]
        self.lengths = [int(L) for L in lengths]
        self.flags = flags
        self.f64 = bool(flags & MP_PREC_F64)
        self.h = _handle if _handle is not None else mp_plan_create(self.dicts, self.lengths, kernel_tol, flags)

    @classmethod
    def autotuned(cls, dicts, lengths, x, kernel_tol=1e-4, flags=0, probe_atoms=2000, stream=None):
        """The fastest schedule for this batch (mp_autotune); returns (plan, report dict).
        The plan must be analysed again before use."""
        import torch
        assert x.is_cuda and x.is_contiguous() and x.dim() == 1
        dt = MP_DTYPE_F32 if x.dtype == torch.float32 else MP_DTYPE_F64
        h, rep = mp_autotune(dicts, lengths, kernel_tol, flags, x.data_ptr(), dt, probe_atoms, stream)
        return cls(dicts, lengths, kernel_tol, flags, _handle=h), rep.as_dict()

    def close(self):
        if self.h:
            mp_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def analyze(self, x, stream=None):
        """x: 1-D torch tensor on the GPU (float32 or float64), the batch packed back to back."""
        import torch
        assert x.is_cuda and x.is_contiguous() and x.dim() == 1
        assert x.numel() == sum(self.lengths)
        dt = MP_DTYPE_F32 if x.dtype == torch.float32 else MP_DTYPE_F64
        assert x.dtype in (torch.float32, torch.float64)
        self._x = x  # keep alive until the stream has consumed it
        mp_analyze(self.h, x.data_ptr(), dt, stream)

    def run(self, max_atoms=0, target_snr_db=0.0, stream=None):
        mp_run(self.h, max_atoms, target_snr_db, stream)

    def run_resets(self, max_atoms=0, target_snr_db=0.0, reset_it=0, reset_db=0.0, stream=None):
        """Alg. 2 on the signal given to the last analyze(); reset_it <= 0: the
        default criterion derived from the kernel threshold."""
        import torch
        dt = MP_DTYPE_F32 if self._x.dtype == torch.float32 else MP_DTYPE_F64
        mp_run_resets(self.h, self._x.data_ptr(), dt, max_atoms, target_snr_db, reset_it, reset_db, stream)

    def info(self, sig=0):
        return mp_signal_info_get(self.h, sig)

    def atoms(self, sig=0):
        return mp_get_atoms(self.h, sig)

    def energy(self, sig=0):
        return mp_get_energy(self.h, sig)

    def residual(self, sig, w):
        import torch
        inf = self.info(sig)
        d = self.dicts[w]
        N, MR = inf.L_padded // d[2], d[3] // 2 + 1
        t = torch.empty((N, MR), dtype=torch.complex128 if self.f64 else torch.complex64, device="cuda")
        mp_get_residual(self.h, sig, w, t.data_ptr())
        return t

    def coefs(self, sig, w):
        import torch
        inf = self.info(sig)
        d = self.dicts[w]
        N, MR = inf.L_padded // d[2], d[3] // 2 + 1
        t = torch.empty((N, MR), dtype=torch.complex128, device="cuda")
        mp_get_coefs(self.h, sig, w, t.data_ptr())
        return t

    def resynth(self, sig=0, dtype=None):
        import torch
        inf = self.info(sig)
        dt = torch.float64 if dtype is None else dtype
        y = torch.empty(inf.L_padded, dtype=dt, device="cuda")
        mp_resynth(self.h, sig, y.data_ptr(), MP_DTYPE_F64 if dt == torch.float64 else MP_DTYPE_F32)
        return y

    def kernel(self, w, v):
        return mp_get_kernel(self.h, w, v)

    def kernel_info(self, w, v):
        return mp_kernel_info_get(self.h, w, v)

    def stats(self):
        return mp_get_stats(self.h)
