"""ctypes wrapper around the C oracle (``mp_oracle.c``).

TEST INFRASTRUCTURE ONLY: see the package docstring.  Every routine is FP64.
"""
import ctypes as C
import math
from dataclasses import dataclass
from typing import Sequence

import numpy as np

from . import build as _build

WIN_BLACKMAN = 0
WIN_HANN = 1
WIN_GAUSS = 2      # exp(-pi t^2 / (a M)): its width depends on the lattice
THR_REL = 1
CONJ_GATE_GAMMA = 2
PEDANTIC = 4
KEEP_BOX = 8       # keep the survivors' whole bounding box (a reading, see the header)

STOP_K, STOP_SNR, STOP_ENEG, STOP_ZERO = 1, 2, 3, 4


class _Dict(C.Structure):
    _fields_ = [("window", C.c_int32), ("gl", C.c_int32), ("a", C.c_int32),
                ("M", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("stop_reason", C.c_int32),
                ("pad_", C.c_int32), ("L_padded", C.c_int64), ("E0", C.c_double),
                ("E_final", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(_build.build())
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        _lib.orc_window.argtypes = [C.c_int32, C.c_int32, dp]
        _lib.orc_window_ga.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, dp]
        _lib.orc_check_dicts.argtypes = [C.POINTER(_Dict), C.c_int32]
        _lib.orc_padded_length.argtypes = [C.POINTER(_Dict), C.c_int32, C.c_int64]
        _lib.orc_padded_length.restype = C.c_int64
        _lib.orc_fft.argtypes = [C.c_int32, dp, dp, C.c_int32]
        _lib.orc_dft.argtypes = [C.c_int32, dp, dp, C.c_int32]
        _lib.orc_dgt.argtypes = [C.POINTER(_Dict), dp, C.c_int64, dp, dp]
        _lib.orc_dgt_direct.argtypes = [C.POINTER(_Dict), dp, C.c_int64, dp, dp]
        _lib.orc_kernel_direct.argtypes = [C.POINTER(_Dict), C.POINTER(_Dict),
                                           C.c_int64, C.c_int64,
                                           C.POINTER(C.c_double), C.POINTER(C.c_double)]
        _lib.orc_kernel_table.argtypes = [C.POINTER(_Dict), C.POINTER(_Dict), C.c_double,
                                          C.c_uint32, C.POINTER(C.c_int32), C.c_void_p,
                                          C.c_void_p, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32)]
        _lib.orc_mp.argtypes = [C.POINTER(_Dict), C.c_int32, dp, C.c_int64, C.c_double,
                                C.c_uint32, C.c_int64, C.c_double, C.c_int64, ip, ip, ip,
                                dp, dp, dp, dp, dp, C.c_void_p, C.c_void_p, C.POINTER(_Stats)]
        _lib.orc_mp_replay.argtypes = [C.POINTER(_Dict), C.c_int32, dp, C.c_int64, C.c_double,
                                       C.c_uint32, C.c_int64, ip, ip, ip, dp, dp, dp, dp, dp, dp,
                                       C.c_void_p, C.c_void_p, C.POINTER(_Stats)]
        _lib.orc_resynth.argtypes = [C.POINTER(_Dict), C.c_int32, C.c_int64, C.c_int64,
                                     ip, ip, ip, dp, dp, dp]
    return _lib


def _dicts(dicts: Sequence[Sequence[int]]):
    arr = (_Dict * len(dicts))()
    for i, d in enumerate(dicts):
        arr[i] = _Dict(*[int(v) for v in d])
    return arr


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle error %d" % rc)


def window(win: int, gl: int, a: int = 0, M: int = 0) -> np.ndarray:
    """Window of a dictionary (win, gl, a, M); a and M matter for the Gaussian."""
    g = np.zeros(gl)
    _check(lib().orc_window_ga(win, gl, a, M, g))
    return g


def check_dicts(dicts) -> int:
    return lib().orc_check_dicts(_dicts(dicts), len(dicts))


def padded_length(dicts, L: int) -> int:
    return lib().orc_padded_length(_dicts(dicts), len(dicts), L)


def fft(x: np.ndarray, sign: int = -1) -> np.ndarray:
    re = np.ascontiguousarray(x.real, dtype=np.float64).copy()
    im = np.ascontiguousarray(np.imag(x), dtype=np.float64).copy()
    _check(lib().orc_fft(len(re), re, im, sign))
    return re + 1j * im


def dft(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """DFT of any length (orc_dft)."""
    re = np.ascontiguousarray(x.real, dtype=np.float64).copy()
    im = np.ascontiguousarray(np.imag(x), dtype=np.float64).copy()
    _check(lib().orc_dft(len(re), re, im, sign))
    return re + 1j * im


def dgt(d, x: np.ndarray, direct: bool = False) -> np.ndarray:
    """Reduced DGT plane (N x M/2+1, complex128) of a real signal."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    L = len(x)
    N, MR = L // d[2], d[3] // 2 + 1
    re = np.zeros(N * MR)
    im = np.zeros(N * MR)
    f = lib().orc_dgt_direct if direct else lib().orc_dgt
    _check(f(_dicts([d]), x, L, re, im))
    return (re + 1j * im).reshape(N, MR)


def kernel_direct(dw, dv, mu: int, Delta: int) -> complex:
    re, im = C.c_double(), C.c_double()
    _check(lib().orc_kernel_direct(_dicts([dw]), _dicts([dv]), mu, Delta,
                                   C.byref(re), C.byref(im)))
    return complex(re.value, im.value)


@dataclass
class KernelTable:
    D: int
    Mmax: int
    amin: int
    h: np.ndarray  # (2D+1, Mmax) complex128, column index delta + D
    box_mu: int
    box_delta: int


def kernel_table(dw, dv, eps: float, flags: int = 0) -> KernelTable:
    D = C.c_int32()
    _check(lib().orc_kernel_table(_dicts([dw]), _dicts([dv]), eps, flags, C.byref(D),
                                  None, None, None, None))
    Mmax = dw[3] * dv[3] // math.gcd(dw[3], dv[3])   # lcm: the common grid's bins
    n = (2 * D.value + 1) * Mmax
    re = np.zeros(n)
    im = np.zeros(n)
    bm, bd = C.c_int32(), C.c_int32()
    _check(lib().orc_kernel_table(_dicts([dw]), _dicts([dv]), eps, flags, C.byref(D),
                                  re.ctypes.data, im.ctypes.data, C.byref(bm),
                                  C.byref(bd)))
    return KernelTable(D.value, Mmax, math.gcd(dw[2], dv[2]),
                       (re + 1j * im).reshape(2 * D.value + 1, Mmax), bm.value, bd.value)


@dataclass
class MPResult:
    w: np.ndarray
    m: np.ndarray
    n: np.ndarray
    c: np.ndarray
    E: np.ndarray      # error estimate after each selection
    gap: np.ndarray    # relative top-2 gap of the selection score at each selection
    E0: float
    L_padded: int
    stop_reason: int
    planes: list       # final residual planes per system (or None)
    best: np.ndarray = None   # the selected score (|rho|^2, or the pedantic score)

    @property
    def n_atoms(self):
        return len(self.w)


def mp(dicts, x: np.ndarray, eps: float, K: int = 0, target_db: float = 0.0,
       flags: int = 0, cap: int = None, return_planes: bool = False) -> MPResult:
    x = np.ascontiguousarray(x, dtype=np.float64)
    L = len(x)
    Lp = padded_length(dicts, L)
    if Lp < 0:
        raise RuntimeError("oracle error %d" % Lp)
    kmax = K if K > 0 else Lp // 5
    if cap is None:
        cap = kmax
    cap = max(int(cap), 1)
    aw = np.zeros(cap, np.int32)
    am = np.zeros(cap, np.int32)
    an = np.zeros(cap, np.int32)
    cre = np.zeros(cap)
    cim = np.zeros(cap)
    Ea = np.zeros(cap)
    gp = np.zeros(cap)
    bs = np.zeros(cap)
    sizes = [(Lp // d[2]) * (d[3] // 2 + 1) for d in dicts]
    fr = fi = None
    if return_planes:
        fr = np.zeros(sum(sizes))
        fi = np.zeros(sum(sizes))
    st = _Stats()
    _check(lib().orc_mp(_dicts(dicts), len(dicts), x, L, eps, flags, K, target_db, cap,
                        aw, am, an, cre, cim, Ea, gp, bs,
                        fr.ctypes.data if fr is not None else None,
                        fi.ctypes.data if fi is not None else None, C.byref(st)))
    k = st.n_atoms
    planes = None
    if return_planes:
        planes, o = [], 0
        for d, s in zip(dicts, sizes):
            planes.append((fr[o:o + s] + 1j * fi[o:o + s]).reshape(Lp // d[2], d[3] // 2 + 1))
            o += s
    return MPResult(aw[:k].copy(), am[:k].copy(), an[:k].copy(), cre[:k] + 1j * cim[:k],
                    Ea[:k].copy(), gp[:k].copy(), st.E0, st.L_padded, st.stop_reason,
                    planes, bs[:k].copy())


@dataclass
class ReplayResult:
    c: np.ndarray       # adjusted coefficient of each replayed atom (oracle arithmetic)
    E: np.ndarray       # error estimate after each step
    gap: np.ndarray     # top-2 gap of the oracle's scores before each step
    best: np.ndarray    # largest selection score before each step
    chosen: np.ndarray  # score of the replayed atom before each step
    E0: float
    L_padded: int
    planes: list        # residual planes after the last step (or None)


def mp_replay(dicts, x: np.ndarray, eps: float, w, m, n, flags: int = 0,
              return_planes: bool = False) -> ReplayResult:
    """Runs the oracle's loop on x with the selections (w, m, n) of another run
    instead of its own maxima (orc_mp_replay)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    L = len(x)
    Lp = padded_length(dicts, L)
    if Lp < 0:
        raise RuntimeError("oracle error %d" % Lp)
    w = np.ascontiguousarray(w, np.int32)
    m = np.ascontiguousarray(m, np.int32)
    n = np.ascontiguousarray(n, np.int32)
    k = len(w)
    sz = max(k, 1)
    cre, cim, Ea, gp, best, ch = (np.zeros(sz) for _ in range(6))
    if k == 0:
        w = m = n = np.zeros(1, np.int32)
    sizes = [(Lp // d[2]) * (d[3] // 2 + 1) for d in dicts]
    fr = fi = None
    if return_planes:
        fr = np.zeros(sum(sizes))
        fi = np.zeros(sum(sizes))
    st = _Stats()
    _check(lib().orc_mp_replay(_dicts(dicts), len(dicts), x, L, eps, flags, k, w, m, n,
                               cre, cim, Ea, gp, best, ch,
                               fr.ctypes.data if fr is not None else None,
                               fi.ctypes.data if fi is not None else None, C.byref(st)))
    planes = None
    if return_planes:
        planes, o = [], 0
        for d, s in zip(dicts, sizes):
            planes.append((fr[o:o + s] + 1j * fi[o:o + s]).reshape(Lp // d[2], d[3] // 2 + 1))
            o += s
    return ReplayResult(cre[:k] + 1j * cim[:k], Ea[:k].copy(), gp[:k].copy(), best[:k].copy(),
                        ch[:k].copy(), st.E0, st.L_padded, planes)


def resynth(dicts, Lp: int, w, m, n, c) -> np.ndarray:
    w = np.ascontiguousarray(w, np.int32)
    m = np.ascontiguousarray(m, np.int32)
    n = np.ascontiguousarray(n, np.int32)
    c = np.asarray(c, np.complex128)
    y = np.zeros(Lp)
    _check(lib().orc_resynth(_dicts(dicts), len(dicts), Lp, len(w), w, m, n,
                             np.ascontiguousarray(c.real), np.ascontiguousarray(c.imag), y))
    return y


@dataclass
class ResetResult:
    w: np.ndarray
    m: np.ndarray
    n: np.ndarray
    c: np.ndarray
    E: np.ndarray        # inner error estimate after each selection (restarts at the true error)
    gap: np.ndarray      # relative top-2 gap of |rho|^2 at each selection
    E0: float
    L_padded: int
    stop_reason: int
    E_true: np.ndarray   # true error ||x - D c||^2 after each reset round
    k_rounds: np.ndarray  # selections made when each round ended
    residual: np.ndarray  # final true residual over the padded length

    @property
    def n_atoms(self):
        return len(self.w)


def mp_resets(dicts, x: np.ndarray, eps: float, K: int = 0, target_db: float = 0.0,
              reset_it: int = 0, reset_db: float = 0.0, flags: int = 0) -> ResetResult:
    """Approximate coefficient-domain MP with resets (Alg. 2), composed of this
    oracle's own steps.  Each inner loop is mp() (Alg. 1) started from the
    coefficients of the current true residual, rho = D* r, with error E = ||r||^2;
    it runs until reset_it selections, or (reset_db < 0) until its estimate
    falls to 10^(reset_db/10) of the error at the last reset, or any stop rule
    of Alg. 1.  The outer update adds the selections to the solution and
    subtracts their synthesis (resynth()) from r; ||r||^2 becomes the error.
    The procedure ends when the true error reaches target_db below ||x||^2,
    after K selections (0: L_padded/5), when the coefficients vanish, or when
    an inner loop selects nothing.  reset_it <= 0 selects the default
    criterion derived from eps (see below)."""
    if reset_it <= 0:
        # the default criterion derived from the kernel threshold (Sec. 7,
        # 'reset'; a reading, the paper does not print it): ceil(32 / eps)
        # selections per round, and a reset once the estimate has fallen by
        # the factor eps below the error at the last reset
        reset_it = int(math.ceil(32.0 / eps)) if eps > 0 else (1 << 62)
        if reset_db == 0.0 and eps > 0:
            reset_db = 10.0 * math.log10(eps)
    x = np.ascontiguousarray(x, dtype=np.float64)
    L = len(x)
    Lp = padded_length(dicts, L)
    if Lp < 0:
        raise RuntimeError("oracle error %d" % Lp)
    r = np.zeros(Lp)
    r[:L] = x
    E0 = float(r @ r)
    kmax = K if K > 0 else Lp // 5
    Etg = E0 * 10.0 ** (-target_db / 10.0) if target_db > 0 else -np.inf
    ws, ms, ns, cs, Es, gs, Et, kr = [], [], [], [], [], [], [], []
    k, Eout, stop = 0, E0, 0
    while True:
        Ein = Etg
        if reset_db < 0:
            Ein = max(Ein, Eout * 10.0 ** (reset_db / 10.0))
        t_db = 10.0 * np.log10(Eout / Ein) if 0 < Ein < Eout else 0.0
        kin = min(reset_it, kmax - k)
        res = mp(dicts, r, eps, K=kin, target_db=t_db, flags=flags, cap=kin)
        ws.append(res.w)
        ms.append(res.m)
        ns.append(res.n)
        cs.append(res.c)
        Es.append(res.E)
        gs.append(res.gap)
        k += res.n_atoms
        if res.n_atoms:
            r = r - resynth(dicts, Lp, res.w, res.m, res.n, res.c)
        Eout = float(r @ r)
        Et.append(Eout)
        kr.append(k)
        if Eout <= Etg:
            stop = 2
        elif k >= kmax:
            stop = 1
        elif res.stop_reason == 4:
            stop = 4
        elif res.n_atoms == 0:
            stop = res.stop_reason or 1
        if stop:
            break
    cat = lambda v, t: np.concatenate(v).astype(t) if v else np.zeros(0, t)
    return ResetResult(cat(ws, np.int32), cat(ms, np.int32), cat(ns, np.int32), cat(cs, np.complex128),
                       cat(Es, np.float64), cat(gs, np.float64), E0, Lp, stop, np.array(Et),
                       np.array(kr, np.int64), r)
