"""Seeded synthetic inputs for the five workloads (numpy only).

This module is shared by the GPU tests, the oracle tests and the benchmark.  It
imports nothing from the library or from the oracle, and it holds none of the
pursuit's arithmetic: it only describes workloads and draws signals.  The
planted-atom recipe builds its atoms with its own window code.

Seeds: ``numpy.random.Generator(PCG64(SeedSequence([config_id, signal_idx])))``.

Workloads (stand-ins for the paper's piano recording and Matlab noise, which are
not available):

* C1 - one Blackman system (gl=512, a=128, M=512), L = 16384, FP64 signal:
  50 unit Gabor atoms on the grid with complex N(0,1) amplitudes plus white
  noise at 20 dB SNR; threshold 1e-4, K = 1000.
* C2 - three Blackman systems (256/1024/4096 taps, a = gl/4, M = gl), FP32
  signal of 441000 samples at 44.1 kHz: harmonic tones with vibrato, linear
  chirps, damped clicks and pink noise 30 dB below the rest; run to 40 dB or
  K = 1e5.
* C3 - 256 signals of C2's kind with lengths log-uniform in [2^14, 2^18].
* C4 - C3's batch with other DGT precisions and thresholds (same inputs).
* C5 - five Blackman systems (128 .. 32768 taps), L = 2^22, the C1 recipe with
  50 atoms per 2^14 samples spread over the five systems, batch of 16.
"""
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

BLACKMAN = 0
HANN = 1
FS = 44100.0
_TAB = 16384


def rng(config_id: int, signal_idx: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([config_id, signal_idx])))


@dataclass
class Workload:
    name: str
    config_id: int
    dicts: List[Tuple[int, int, int, int]]   # (window, gl, a, M)
    eps: float
    K: int                                   # 0: default (L/5)
    target_db: float                         # 0: none
    batch: int
    dtype: str                               # "f64" or "f32" input samples
    lengths: List[int] = field(default_factory=list)


def _audio_dicts():
    return [(BLACKMAN, g, g // 4, g) for g in (256, 1024, 4096)]


def workload(cid: int) -> Workload:
    if cid == 1:
        return Workload("C1 plain MP, one Blackman system 512/128/512, L=16384", 1,
                        [(BLACKMAN, 512, 128, 512)], 1e-4, 1000, 0.0, 1, "f64", [16384])
    if cid == 2:
        return Workload("C2 three Blackman systems 256/1024/4096 a=gl/4, L=441000", 2,
                        _audio_dicts(), 1e-4, 100000, 40.0, 1, "f32", [441000])
    if cid == 3:
        return Workload("C3 batch of 256 audio-like signals, L log-uniform in [2^14, 2^18]",
                        3, _audio_dicts(), 1e-4, 0, 40.0, 256, "f32", c3_lengths(256))
    if cid == 5:
        return Workload("C5 five Blackman systems 128..32768 a=gl/4, L=2^22, batch 16", 5,
                        [(BLACKMAN, g, g // 4, g) for g in (128, 512, 2048, 8192, 32768)],
                        1e-4, 500000, 50.0, 16, "f32", [1 << 22] * 16)
    raise ValueError(cid)


def noise_study():
    """The convergence experiment on noise (Sec. 6.1, Fig. 4): white Gaussian
    noise of 6.04e6 samples (seeded stand-in for the paper's randn signal), the
    three Blackman systems M = 512/1024/2048 with a = M/4, and the thresholds
    1e-4, 1e-3, 5e-3, 1e-2.  Returns (dicts, thresholds, x)."""
    dicts = [(BLACKMAN, g, g // 4, g) for g in (512, 1024, 2048)]
    x = rng(6, 0).standard_normal(6_040_000)
    return dicts, (1e-4, 1e-3, 5e-3, 1e-2), x


def c3_lengths(batch: int, lo: int = 1 << 14, hi: int = 1 << 18, config_id: int = 3):
    g = rng(config_id, 1_000_000)
    u = g.uniform(np.log(lo), np.log(hi), size=batch)
    return [int(np.floor(np.exp(v))) for v in u]


# --------------------------------------------------------------------------
# planted Gabor atoms (C1, C5)

def _blackman(gl: int) -> np.ndarray:
    t = np.arange(gl) - gl // 2
    g = 0.42 + 0.5 * np.cos(2 * np.pi * t / gl) + 0.08 * np.cos(4 * np.pi * t / gl)
    return g / np.sqrt(np.sum(g * g))


def add_atom(x: np.ndarray, gl: int, a: int, M: int, m: int, n: int, alpha: complex):
    """x += Re(alpha * g(l - n a) exp(2 pi i m (l - n a) / M)), circular in l."""
    L = len(x)
    t = np.arange(-gl // 2, gl // 2)
    val = (alpha * _blackman(gl) * np.exp(2j * np.pi * ((m * t) % M) / M)).real
    np.add.at(x, (n * a + t) % L, val)


def planted(L: int, systems, n_atoms: int, snr_db: float, g: np.random.Generator,
            m_range=None):
    """Sum of Re(alpha d_{m,n}) over random on-grid atoms plus white noise."""
    x0 = np.zeros(L)
    picks = []
    for _ in range(n_atoms):
        gl, a, M = systems[int(g.integers(len(systems)))]
        n = int(g.integers(0, L // a))
        lo, hi = (1, M // 2 - 1) if m_range is None else m_range
        m = int(g.integers(lo, hi + 1))
        alpha = complex(g.standard_normal(), g.standard_normal())
        add_atom(x0, gl, a, M, m, n, alpha)
        picks.append((gl, a, M, m, n, alpha))
    if snr_db is None:
        return x0, picks
    e = g.standard_normal(L)
    e *= np.sqrt(np.sum(x0 * x0) / np.sum(e * e) / 10 ** (snr_db / 10))
    return x0 + e, picks


# --------------------------------------------------------------------------
# audio-like recipe (C2, C3)

def _fade(n: int, nf: int) -> np.ndarray:
    env = np.ones(n)
    nf = min(nf, n // 2)
    if nf > 0:
        ramp = 0.5 - 0.5 * np.cos(np.pi * np.arange(nf) / nf)
        env[:nf] = ramp
        env[n - nf:] = ramp[::-1]
    return env


def audio_like(L: int, g: np.random.Generator, scale_events: bool = True) -> np.ndarray:
    T = L / FS
    s = L / 441000.0 if scale_events else 1.0
    n_tones = max(1, int(round(4 * s)))
    n_chirps = max(1, int(round(3 * s)))
    n_clicks = max(1, int(round(30 * s)))
    x = np.zeros(L)
    # harmonic tones with vibrato
    for _ in range(n_tones):
        f0 = float(np.exp(g.uniform(np.log(55.0), np.log(880.0))))
        dur = min(g.uniform(1.0, 4.0), T)
        on = g.uniform(0.0, max(T - dur, 0.0))
        amp = float(np.exp(g.uniform(np.log(0.1), np.log(1.0))))
        vr = g.uniform(4.0, 7.0)
        vd = g.uniform(0.005, 0.02)
        vph = g.uniform(0, 2 * np.pi)
        i0s = int(on * FS)
        n = min(int(dur * FS), L - i0s)
        if n <= 0:
            continue
        t = np.arange(n) / FS
        # instantaneous frequency f0 (1 + vd sin(2 pi vr t + vph)), integrated
        phase_base = 2 * np.pi * f0 * (t - vd / (2 * np.pi * vr) * (np.cos(2 * np.pi * vr * t + vph) - np.cos(vph)))
        env = _fade(n, int(0.02 * FS))
        # one period of sum_h sin(h phi + theta_h) / h (harmonics below 16 kHz),
        # tabulated by an inverse FFT and read by linear interpolation
        H = max(1, int(np.ceil(16000.0 / f0)) - 1)
        theta = g.uniform(0, 2 * np.pi, size=H)
        spec = np.zeros(_TAB // 2 + 1, np.complex128)
        h = np.arange(1, H + 1)
        spec[h] = (_TAB / 2) / h * np.exp(1j * (theta - np.pi / 2))
        table = np.fft.irfft(spec, n=_TAB)
        pos = np.mod(phase_base, 2 * np.pi) * (_TAB / (2 * np.pi))
        i0 = np.floor(pos).astype(np.int64) % _TAB
        fr = pos - np.floor(pos)
        sig = table[i0] * (1 - fr) + table[(i0 + 1) % _TAB] * fr
        x[i0s:i0s + n] += amp * env * sig
    # linear chirps
    for _ in range(n_chirps):
        fa, fb = g.uniform(100.0, 12000.0, size=2)
        dur = min(g.uniform(0.3, 2.0), T)
        on = g.uniform(0.0, max(T - dur, 0.0))
        amp = float(np.exp(g.uniform(np.log(0.05), np.log(0.5))))
        i0 = int(on * FS)
        n = min(int(dur * FS), L - i0)
        if n <= 0:
            continue
        t = np.arange(n) / FS
        ph = 2 * np.pi * (fa * t + 0.5 * (fb - fa) / dur * t * t)
        x[i0:i0 + n] += amp * _fade(n, int(0.02 * FS)) * np.sin(ph)
    # damped clicks
    for _ in range(n_clicks):
        f = g.uniform(500.0, 8000.0)
        tau = g.uniform(0.001, 0.010)
        amp = float(np.exp(g.uniform(np.log(0.05), np.log(0.5))))
        i0 = int(g.uniform(0.0, T) * FS)
        n = min(int(8 * tau * FS), L - i0)
        if n <= 0:
            continue
        t = np.arange(n) / FS
        x[i0:i0 + n] += amp * np.exp(-t / tau) * np.sin(2 * np.pi * f * t + g.uniform(0, 2 * np.pi))
    # pink noise, 30 dB below the deterministic part: white noise shaped by
    # 1/sqrt(f) on the next power-of-two length, truncated to L
    nf = 1 << int(np.ceil(np.log2(L)))
    X = np.fft.rfft(g.standard_normal(nf))
    f = np.arange(len(X), dtype=np.float64)
    f[0] = 1.0
    X /= np.sqrt(f)
    X[0] = 0.0
    pn = np.fft.irfft(X, n=nf)[:L]
    ed = float(np.sum(x * x))
    if ed <= 0.0:
        ed = float(L)
    pn *= np.sqrt(ed / np.sum(pn * pn) / 10 ** 3.0)
    return x + pn


# --------------------------------------------------------------------------

def signals(cid: int, batch: int = None, lengths=None):
    """Seeded input signals for workload ``cid`` (list of 1-D numpy arrays)."""
    wl = workload(cid)
    if cid in (1,):
        g = rng(1, 0)
        gl, a, M = 512, 128, 512
        x, _ = planted(16384, [(gl, a, M)], 50, 20.0, g)
        return [x.astype(np.float64)]
    if cid in (2, 3, 4):
        if cid == 2:
            return [audio_like(441000, rng(2, 0), scale_events=False).astype(np.float32)]
        lens = lengths if lengths is not None else wl.lengths
        if batch is not None:
            lens = lens[:batch]
        return [audio_like(L, rng(3, i)).astype(np.float32) for i, L in enumerate(lens)]
    if cid == 5:
        b = batch if batch is not None else wl.batch
        L = 1 << 22
        sys5 = [(gl, gl // 4, gl) for gl in (128, 512, 2048, 8192, 32768)]
        out = []
        for i in range(b):
            x, _ = planted(L, sys5, 50 * (L >> 14), 20.0, rng(5, i))
            out.append(x.astype(np.float32))
        return out
    raise ValueError(cid)
