"""GPU parity: the HIP path, called through the C-ABI, against the FP64 oracle on
the same seeded inputs."""
import numpy as np
import pytest

from oracle import core as O
from paper_2202_12380_amd import signals as S
from gpu_helpers import gpu_run, oracle_run, assert_identical, assert_tolerance, first_mismatch

pytestmark = pytest.mark.gpu

F64 = 0x1


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


# --------------------------------------------------------------------------
# kernel tables (FP64 precompute on the device) vs the oracle's tables

@pytest.mark.parametrize("dicts", [
    [(0, 512, 128, 512)],
    [(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)],
    [(1, 64, 16, 64), (0, 128, 64, 256)],
    [(2, 4096, 512, 2048)],                        # the Gaussian of the kernel figure
    [(2, 64, 8, 32), (0, 96, 16, 64)],             # windows longer than M
    [(0, 64, 24, 64), (0, 128, 16, 128)],          # hops not nested: grid step gcd = 8
])
@pytest.mark.parametrize("eps,rel", [(1e-4, False), (1e-3, True)])
def test_kernel_tables_match_oracle(dicts, eps, rel):
    _torch()
    from paper_2202_12380_amd import mpg
    L = max(d[3] for d in dicts) * 4
    plan = mpg.Plan(dicts, [L], eps, mpg.MP_THR_REL if rel else 0)
    for w, dw in enumerate(dicts):
        for v, dv in enumerate(dicts):
            t = O.kernel_table(dw, dv, eps, O.THR_REL if rel else 0)
            ki = plan.kernel_info(w, v)
            assert ki.D == t.D and ki.amin == t.amin and ki.Mmax == t.Mmax
            assert ki.delta_box == t.box_delta
            g = plan.kernel(w, v)
            # oracle entries on the same box
            mus = np.arange(ki.mu_lo, ki.mu_hi + 1) % t.Mmax
            rows = np.arange(-ki.delta_box, ki.delta_box + 1) + t.D
            ref = t.h[np.ix_(rows, mus)]
            full = O.kernel_table(dw, dv, 0.0).h[np.ix_(rows, mus)]
            thr = eps * (np.abs(O.kernel_table(dw, dv, 0.0).h).max() if rel else 1.0)
            near = np.abs(np.abs(full) - thr) < 1e-12
            assert np.array_equal((g != 0)[~near], (ref != 0)[~near])
            assert np.max(np.abs(g - ref)[~near]) < 1e-14
            # nothing survives outside the box
            assert np.count_nonzero(t.h) == np.count_nonzero(ref)


# --------------------------------------------------------------------------
# DGT planes

@pytest.mark.parametrize("prec", ["f64", "f32", "f32dft64"])
@pytest.mark.parametrize("dicts,L", [
    ([(0, 512, 128, 512)], 16384),
    ([(0, 64, 16, 64), (0, 256, 64, 256)], 3000),     # ragged: padded to 3072
    ([(1, 32, 8, 32), (0, 128, 32, 128), (0, 128, 128, 512)], 1024),
    ([(2, 256, 32, 128), (0, 96, 16, 64), (2, 64, 64, 64)], 2048),   # folded windows
    ([(0, 64, 24, 64), (1, 128, 40, 128)], 3000),    # hops dividing neither M: padded to 3840
    ([(0, 16384, 4096, 16384), (0, 4096, 1024, 4096)], 1 << 16),   # long frames: all FFT stage shapes
    ([(0, 4, 2, 4), (0, 8, 2, 8), (1, 2, 1, 2)], 64),   # frames of 2, 4 and 8 samples
])
def test_dgt_planes(prec, dicts, L):
    torch = _torch()
    from paper_2202_12380_amd import mpg
    x = np.random.default_rng(L).standard_normal(L)
    flags = {"f64": F64, "f32": 0, "f32dft64": mpg.MP_DFT_F64}[prec]
    dt = torch.float64 if prec == "f64" else torch.float32
    xs = x if prec == "f64" else x.astype(np.float32).astype(np.float64)
    plan = mpg.Plan(dicts, [L], 1e-4, flags)
    plan.analyze(torch.from_numpy(xs).to(dt).cuda())
    Lp = O.padded_length(dicts, L)
    xp = np.zeros(Lp)
    xp[:L] = xs
    for w, d in enumerate(dicts):
        ref = O.dgt(d, xp)
        got = plan.residual(0, w).cpu().numpy()
        scale = np.abs(ref).max()
        # FP64 FFT rounded to FP32: half an FP32 ulp of each coefficient
        tol = {"f64": 1e-13, "f32": 3e-6, "f32dft64": 1.2e-7}[prec]
        assert np.max(np.abs(got - ref)) <= tol * scale
    inf = plan.info(0)
    assert inf.L_padded == Lp
    assert abs(inf.E0 - float(xs @ xs)) <= 1e-12 * float(xs @ xs)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_dgt_planes_batch(prec):
    # several signals of different lengths in one launch per system: the
    # frame -> signal lookup, per-signal energies and padding
    torch = _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 64, 16, 64), (1, 256, 64, 256), (2, 128, 32, 64)]
    lens = [3000, 700, 5000, 1024, 2500, 513]
    rng = np.random.default_rng(77)
    xs = [rng.standard_normal(L) for L in lens]
    if prec == "f32":
        xs = [v.astype(np.float32).astype(np.float64) for v in xs]
    flags = F64 if prec == "f64" else 0
    dt = torch.float64 if prec == "f64" else torch.float32
    plan = mpg.Plan(dicts, lens, 1e-4, flags)
    plan.analyze(torch.from_numpy(np.concatenate(xs)).to(dt).cuda())
    tol = 1e-13 if prec == "f64" else 3e-6
    for s_, (L, v) in enumerate(zip(lens, xs)):
        Lp = O.padded_length(dicts, L)
        xp = np.zeros(Lp)
        xp[:L] = v
        inf = plan.info(s_)
        assert inf.L_padded == Lp
        assert abs(inf.E0 - float(v @ v)) <= 1e-12 * float(v @ v)
        for w, d in enumerate(dicts):
            ref = O.dgt(d, xp)
            got = plan.residual(s_, w).cpu().numpy()
            assert np.max(np.abs(got - ref)) <= tol * np.abs(ref).max()


@pytest.mark.parametrize("fmt,tol", [(0x40, 3e-6), (0x80, 5e-5)])
@pytest.mark.parametrize("dicts,L", [
    ([(0, 512, 128, 512)], 16384),
    ([(0, 64, 16, 64), (0, 256, 64, 256)], 3000),
    ([(1, 32, 8, 32), (0, 128, 32, 128), (0, 128, 128, 512)], 1024),
    ([(0, 16384, 4096, 16384), (0, 4096, 1024, 4096)], 1 << 16),
    ([(0, 4, 2, 4), (0, 8, 2, 8)], 64),
    ([(2, 256, 32, 128), (0, 96, 16, 64)], 2048),                    # folded windows
])
def test_dgt_planes_split_mfma(fmt, tol, dicts, L):
    # DFT on matrix cores with FP16 (0x40) or BF16 (0x80) hi/lo operand pairs;
    # tolerance relative to the plane maximum: the pair carries 22 (FP16) or
    # 16 (BF16) significant bits, two GEMM stages
    torch = _torch()
    from paper_2202_12380_amd import mpg
    x = np.random.default_rng(L + 1).standard_normal(L).astype(np.float32).astype(np.float64)
    plan = mpg.Plan(dicts, [L], 1e-4, fmt)
    plan.analyze(torch.from_numpy(x).to(torch.float32).cuda())
    Lp = O.padded_length(dicts, L)
    xp = np.zeros(Lp)
    xp[:L] = x
    for w, d in enumerate(dicts):
        ref = O.dgt(d, xp)
        got = plan.residual(0, w).cpu().numpy()
        assert np.max(np.abs(got - ref)) <= tol * np.abs(ref).max()


@pytest.mark.parametrize("fmt,tol", [(0x40, 3e-6), (0x80, 5e-5)])
@pytest.mark.parametrize("pedantic,x64", [(False, False), (True, False), (False, True)])
def test_dgt_planes_split_mfma_batch(fmt, tol, pedantic, x64):
    # every frame-group shape of the matrix-core DFT (M = 256 .. 4096, 8 .. 1
    # frames per wave) on a batch of uneven lengths, so that frame groups
    # straddle signals, with a folded Gaussian window (gl = 2 M); planes
    # element by element; without pedantic selection, the first selection has
    # the largest score of its planes (the leaves hold their 16-bin maxima)
    torch = _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 256, 64, 256), (0, 512, 128, 512), (2, 2048, 128, 1024), (0, 2048, 512, 2048),
             (0, 4096, 1024, 4096)]
    lens = [9000, 4100, 16384, 5000, 8192, 4097]
    rng = np.random.default_rng(fmt + 5)
    xs = [rng.standard_normal(L).astype(np.float32).astype(np.float64) for L in lens]
    flags = fmt | (mpg.MP_PEDANTIC if pedantic else 0)
    plan = mpg.Plan(dicts, lens, 1e-4, flags)
    # x64: FP64 samples (the path the reset procedure's residual takes)
    plan.analyze(torch.from_numpy(np.concatenate(xs)).to(torch.float64 if x64 else torch.float32).cuda())
    planes = []
    for s_, (L, v) in enumerate(zip(lens, xs)):
        Lp = O.padded_length(dicts, L)
        assert plan.info(s_).L_padded == Lp
        xp = np.zeros(Lp)
        xp[:L] = v
        planes.append([])
        for w, d in enumerate(dicts):
            ref = O.dgt(d, xp)
            got = plan.residual(s_, w).cpu().numpy()
            assert np.max(np.abs(got - ref)) <= tol * np.abs(ref).max(), (s_, w)
            planes[-1].append(np.abs(got.astype(np.complex128)) ** 2)
    if not pedantic:
        # the leaves: the first selection of each signal has the largest
        # |rho|^2 of its planes (to the rounding of the FP32 score)
        plan.run(1)
        for s_ in range(len(lens)):
            a = plan.atoms(s_)
            assert len(a) == 1
            top = max(float(p.max()) for p in planes[s_])
            sel = planes[s_][int(a["w"][0])][int(a["n"][0]), int(a["m"][0])]
            assert sel >= top * (1.0 - 1e-6), (s_, sel, top)


# --------------------------------------------------------------------------
# MP loop, FP64: identical atom sequence

def test_mp_fp64_c1_identical():
    _torch()
    wl = S.workload(1)
    x = S.signals(1)[0]
    plan, ga = gpu_run(wl.dicts, [x], wl.eps, K=wl.K, flags=F64)
    orc = oracle_run(wl.dicts, x, wl.eps, K=wl.K)
    assert_identical(ga[0], orc)
    assert plan.info(0).stop_reason == 1


@pytest.mark.parametrize("dicts,L,eps,K", [
    ([(0, 64, 16, 64), (0, 128, 32, 128)], 2048, 1e-4, 400),
    ([(0, 128, 32, 128), (0, 64, 16, 64)], 1999, 1e-3, 300),
    ([(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)], 16384, 1e-4, 600),
    ([(1, 32, 8, 32), (0, 128, 32, 128), (0, 128, 128, 512)], 1024, 1e-5, 300),
    ([(0, 64, 16, 64)], 128, 1e-4, 60),                 # shortest allowed length, wraps
    ([(0, 16, 4, 16), (0, 32, 8, 32)], 128, 0.0, 120),  # eps = 0: full kernels
    ([(2, 128, 16, 64), (0, 96, 16, 64), (2, 512, 64, 256)], 4096, 1e-4, 400),  # Gaussian, gl > M
    ([(0, 64, 24, 64), (0, 128, 16, 128), (2, 256, 40, 128)], 3840, 1e-4, 400),  # gcd grids
])
def test_mp_fp64_identical(dicts, L, eps, K):
    _torch()
    x = np.random.default_rng(L + K).standard_normal(L)
    _, ga = gpu_run(dicts, [x], eps, K=K, flags=F64)
    orc = oracle_run(dicts, x, eps, K=K)
    assert_identical(ga[0], orc)


def _planted_low_high(dicts, L, seed, noise=0.05):
    # real atoms near DC and near Nyquist, where the conjugate-partner
    # condition of Alg. 3 changes the update, plus noise
    from oracle import textbook as T
    rng = np.random.default_rng(seed)
    x = noise * rng.standard_normal(L)
    for d in dicts:
        M = d[3]
        for m in (3, 4, 5, M // 2 - 3, M // 2 - 4):
            n = int(rng.integers(0, L // d[2]))
            x += (complex(rng.standard_normal(), rng.standard_normal()) * T.atom(d, m, n, L)).real
    return x


@pytest.mark.parametrize("dicts,L,eps,K,planted", [
    ([(0, 32, 8, 32), (0, 64, 16, 64)], 2048, 1e-3, 300, True),
    ([(1, 64, 16, 64), (0, 128, 32, 128)], 4096, 1e-4, 400, True),
    ([(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)], 16384, 1e-4, 600, False),
    ([(1, 16, 4, 32), (2, 32, 8, 32)], 1024, 1e-4, 200, True),   # windows shorter than M
])
def test_mp_fp64_gamma_gate_identical(dicts, L, eps, K, planted):
    # literal Alg. 3: the partner term only when gamma != 0 (MP_CONJ_GATE_GAMMA)
    _torch()
    x = _planted_low_high(dicts, L, L + K) if planted else np.random.default_rng(L + K).standard_normal(L)
    _, ga = gpu_run(dicts, [x], eps, K=K, flags=F64 | 0x20)
    orc = oracle_run(dicts, x, eps, K=K, flags=0x20)
    assert_identical(ga[0], orc)
    # the condition matters on these inputs (the ungated oracle differs)
    if planted:
        og = oracle_run(dicts, x, eps, K=K)
        n = min(og.n_atoms, orc.n_atoms)
        same = (og.w[:n] == orc.w[:n]) & (og.m[:n] == orc.m[:n]) & (og.n[:n] == orc.n[:n])
        assert og.n_atoms != orc.n_atoms or not same.all() or np.max(np.abs(og.E - orc.E)) > 1e-9 * og.E0


def test_mp_fp32_gamma_gate_batch():
    _torch()
    dicts = [(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)]
    lens = [16384, 9000, 20000]
    xs = [S.audio_like(L, S.rng(84, i)).astype(np.float32) for i, L in enumerate(lens)]
    _, ga = gpu_run(dicts, xs, 1e-4, K=0, snr_db=25.0, flags=0x20)
    for i, x in enumerate(xs):
        orc = oracle_run(dicts, x, 1e-4, snr_db=25.0, x_dtype=np.float32, flags=0x20)
        assert_tolerance(ga[i], orc)


@pytest.mark.parametrize("dicts,L,eps,K", [
    ([(0, 64, 16, 64), (0, 256, 64, 256)], 4096, 1e-3, 400),
    ([(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)], 16384, 1e-4, 500),
])
def test_mp_fp64_relative_threshold_identical(dicts, L, eps, K):
    # MP_THR_REL: each cross-kernel thresholded relative to its own peak
    _torch()
    x = np.random.default_rng(L + 3).standard_normal(L)
    plan, ga = gpu_run(dicts, [x], eps, K=K, flags=F64 | 0x10)
    orc = oracle_run(dicts, x, eps, K=K, flags=0x10)
    assert_identical(ga[0], orc)
    # the cross-kernel boxes are larger than with the absolute threshold
    pa = __import__("paper_2202_12380_amd.mpg", fromlist=["mpg"]).Plan(dicts, [L], eps, F64)
    assert plan.kernel_info(0, 1).delta_box >= pa.kernel_info(0, 1).delta_box
    assert plan.kernel_info(0, 1).mu_hi - plan.kernel_info(0, 1).mu_lo > pa.kernel_info(0, 1).mu_hi - pa.kernel_info(0, 1).mu_lo


@pytest.mark.parametrize("dicts,L,eps,K,dc", [
    ([(0, 64, 16, 64), (0, 128, 32, 128)], 2048, 1e-4, 400, 0.0),
    ([(0, 64, 16, 64), (0, 128, 32, 128)], 2048, 1e-4, 400, 3.0),   # strong DC: scores differ most
    ([(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)], 16384, 1e-4, 600, 0.5),
])
def test_mp_pedantic_fp64_identical(dicts, L, eps, K, dc):
    _torch()
    x = np.random.default_rng(L + K + 1).standard_normal(L) + dc
    _, ga = gpu_run(dicts, [x], eps, K=K, flags=F64 | 0x100)
    orc = oracle_run(dicts, x, eps, K=K, flags=0x100)
    assert_identical(ga[0], orc)


def test_mp_pedantic_fp32_batch():
    _torch()
    dicts = [(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)]
    lens = [16384, 9000, 20000]
    xs = [(S.audio_like(L, S.rng(79, i)) + 0.05).astype(np.float32) for i, L in enumerate(lens)]
    _, ga = gpu_run(dicts, xs, 1e-4, K=0, snr_db=25.0, flags=0x100)
    for i, x in enumerate(xs):
        orc = oracle_run(dicts, x, 1e-4, snr_db=25.0, x_dtype=np.float32, flags=0x100)
        assert_tolerance(ga[i], orc)


# --------------------------------------------------------------------------
# MP loop, FP32: identical up to the first small top-2 gap, E within 1e-5 ||x||^2

def test_mp_fp32_c1():
    _torch()
    wl = S.workload(1)
    x = S.signals(1)[0]
    _, ga = gpu_run(wl.dicts, [x], wl.eps, K=wl.K, flags=0)
    orc = oracle_run(wl.dicts, x, wl.eps, K=wl.K, x_dtype=np.float32)
    fm, kg = assert_tolerance(ga[0], orc)
    assert fm >= 100


@pytest.mark.parametrize("eps", [1e-3, 1e-4, 1e-5])
@pytest.mark.parametrize("fmt", [0x0, 0x40, 0x80])
def test_mp_precision_study_batch(fmt, eps):
    # the precision study's grid on a small batch: FP32 FFT (0x0), FP16 pairs
    # (0x40) and BF16 pairs (0x80) on matrix cores, thresholds 1e-3 .. 1e-5.
    # Every run is checked over its whole length by replaying its selections
    # on the oracle (each selection a maximum within the measured coefficient
    # error, E within 1e-5 ||x||^2).  FP32 and FP16 pairs also keep the literal
    # sequence rule; BF16 pairs start from planes with ~1e-5 relative error, so
    # for them the agreement length is reported only.
    _torch()
    from gpu_helpers import gpu_run_staged, replay_check, agreement, C_BF16, C_FP32
    dicts = [(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)]
    lens = [16384, 9000, 20000]
    xs = [S.audio_like(L, S.rng(78, i)).astype(np.float32) for i, L in enumerate(lens)]
    _, ga, cps = gpu_run_staged(dicts, xs, eps, [500, 2000, 1 << 17], snr_db=25.0, flags=fmt,
                                keep=range(len(xs)))
    c = C_BF16 if fmt == 0x80 else C_FP32
    for i, x in enumerate(xs):
        orc = oracle_run(dicts, x, eps, snr_db=25.0, x_dtype=np.float32)
        if fmt == 0x80:
            print("bf16 pairs:", agreement(ga[i], orc, c=c))
        else:
            assert_tolerance(ga[i], orc, floor=(fmt, eps, i) in PRECISION_FLOOR_CASES)
        replay_check(dicts, x.astype(np.float64), eps, ga[i], cps[i], c_model=c)


# (analysis format, threshold, signal) of the precision-study batch whose FP32
# loop leaves the oracle's sequence at a top-2 gap above 1e-6 but within the
# floor of the measured coefficient error (gpu_helpers.fp32_gap_floor)
PRECISION_FLOOR_CASES = {(0x40, 1e-5, 2)}


def test_mp_fp32_gaussian_long_windows():
    # Gaussian and Blackman windows longer than M (folded analysis)
    _torch()
    dicts = [(2, 512, 64, 256), (0, 2048, 256, 1024), (2, 8192, 512, 4096)]
    lens = [16384, 17000, 20000]                   # at least 2 gl = 16384
    xs = [S.audio_like(L, S.rng(78, i)).astype(np.float32) for i, L in enumerate(lens)]
    _, ga = gpu_run(dicts, xs, 1e-4, K=0, snr_db=25.0, flags=0)
    for i, x in enumerate(xs):
        orc = oracle_run(dicts, x, 1e-4, snr_db=25.0, x_dtype=np.float32)
        assert_tolerance(ga[i], orc)


def test_mp_fp32_gcd_grids():
    # hops 96 and 160 nest neither each other nor their M: common grid step 32
    _torch()
    dicts = [(0, 256, 96, 256), (0, 1024, 160, 1024), (2, 512, 64, 256)]
    lens = [16000, 30000, 15360]
    xs = [S.audio_like(L, S.rng(79, i)).astype(np.float32) for i, L in enumerate(lens)]
    _, ga = gpu_run(dicts, xs, 1e-4, K=0, snr_db=25.0, flags=0)
    for i, x in enumerate(xs):
        orc = oracle_run(dicts, x, 1e-4, snr_db=25.0, x_dtype=np.float32)
        assert_tolerance(ga[i], orc)


@pytest.mark.parametrize("sched,threads,groups,tile", [
    (0x1000, 512, 256, 16),              # MP_SCHED_NT512: the LDS fallback launch shape
    (0x2000, 768, 128, 16),              # MP_SCHED_G128: 128-leaf groups
    (0x4000, 768, 256, 8),               # MP_SCHED_TILE8: 8-row tiles
    (0x9000, 512, 256, 32),              # MP_SCHED_NT512 | MP_SCHED_TILE32: 32-row tiles
])
def test_mp_fp32_launch_shapes(sched, threads, groups, tile):
    # the plan's other FP32 schedules give the same atoms within the FP32 rule
    _torch()
    dicts = [(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)]
    lens = [16384, 12345]
    xs = [S.audio_like(L, S.rng(80, i)).astype(np.float32) for i, L in enumerate(lens)]
    plan, ga = gpu_run(dicts, xs, 1e-4, K=0, snr_db=25.0, flags=sched)
    st = plan.stats()
    assert (st.threads, st.group_leaves, st.tile_rows) == (threads, groups, tile)
    for i, x in enumerate(xs):
        orc = oracle_run(dicts, x, 1e-4, snr_db=25.0, x_dtype=np.float32)
        assert_tolerance(ga[i], orc)


def test_mp_fp32_schedules_identical_and_autotune():
    # every FP32 schedule (threads per signal, leaves per tree group, rows per
    # neighbourhood tile) gives the same atoms bit for bit; the autotuner
    # returns one of them, usable after a fresh analysis
    torch = _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)]
    lens = [16384, 9000, 12345]
    xs = [S.audio_like(L, S.rng(81, i)).astype(np.float32) for i, L in enumerate(lens)]
    NT, G1, T8, T32 = mpg.MP_SCHED_NT512, mpg.MP_SCHED_G128, mpg.MP_SCHED_TILE8, mpg.MP_SCHED_TILE32
    runs = {}
    for f in (0, G1, NT, NT | G1, T8, G1 | T8, NT | T8, NT | G1 | T8, NT | T32, NT | G1 | T32):
        plan, ga = gpu_run(dicts, xs, 1e-4, K=0, snr_db=25.0, flags=f)
        st = plan.stats()
        # the 768-thread 128-leaf plans bound the groups a selection touches
        # above their 24 preloaded slots: they take the early-load kernel
        assert st.early_groups == (1 if (st.threads, st.group_leaves) == (768, 128) else 0)
        runs[(st.threads, st.group_leaves, st.tile_rows)] = ga
    assert set(runs) == {(768, 256, 16), (768, 128, 16), (512, 256, 16), (512, 128, 16), (768, 256, 8),
                         (768, 128, 8), (512, 256, 8), (512, 128, 8), (512, 256, 32), (512, 128, 32)}
    ref = runs[(768, 256, 16)]
    for shape, ga in runs.items():
        for a, b in zip(ga, ref):
            assert len(a) == len(b), shape
            assert np.array_equal(a, b), shape
    x = torch.from_numpy(np.concatenate(xs)).cuda()
    plan, rep = mpg.Plan.autotuned(dicts, lens, x, 1e-4, 0, probe_atoms=300)
    assert len(rep["schedules"]) == 10 and 0 <= rep["chosen"] < 10
    assert all(s["probe_ms"] > 0 for s in rep["schedules"])
    st = plan.stats()
    ch = rep["schedules"][rep["chosen"]]
    assert (st.threads, st.group_leaves, st.tile_rows) == (ch["threads"], ch["group_leaves"], ch["tile_rows"])
    assert all(len(plan.atoms(s)) == 300 for s in range(len(lens)))  # the probe's state
    plan.analyze(x)
    plan.run(0, 25.0)
    torch.cuda.synchronize()
    for s in range(len(lens)):
        assert np.array_equal(plan.atoms(s), ref[s])


def test_mp_fp32_early_group_loads():
    # windows eight hops long in four systems: a selection of the longest
    # system touches about 30 tree groups of 256 leaves, more than the 24 the
    # 768-thread loop preloads, so the plan takes the kernel that loads the
    # rest before merging; its atoms equal the 512-thread loop's bit for bit
    # (that kernel merges such groups after the preloaded ones) and the
    # oracle's within the FP32 rule
    _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 512, 64, 512), (0, 1024, 128, 1024), (0, 2048, 256, 2048), (0, 4096, 512, 4096)]
    lens = [16384, 14000]
    xs = [S.audio_like(L, S.rng(84, i)).astype(np.float32) for i, L in enumerate(lens)]
    plan, ga = gpu_run(dicts, xs, 1e-4, K=0, snr_db=25.0, flags=0)
    st = plan.stats()
    assert (st.threads, st.group_leaves, st.early_groups) == (768, 256, 1)
    assert st.l1_groups > 12 * st.atoms  # tree groups merged per selection, on average
    plan5, g5 = gpu_run(dicts, xs, 1e-4, K=0, snr_db=25.0, flags=mpg.MP_SCHED_NT512)
    st5 = plan5.stats()
    assert (st5.threads, st5.early_groups) == (512, 0)
    for a, b in zip(ga, g5):
        assert np.array_equal(a, b)
    for i, x in enumerate(xs):
        orc = oracle_run(dicts, x, 1e-4, snr_db=25.0, x_dtype=np.float32)
        assert_tolerance(ga[i], orc)


def test_resets_fp32_early_group_loads():
    # the reset procedure (Alg. 2) on a plan that takes the early-load loop
    # kernel: the same atoms as the 512-thread kernel bit for bit, the true
    # residual's energy reported, the oracle's composition within the FP32 rule
    torch = _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 512, 64, 512), (0, 1024, 128, 1024), (0, 2048, 256, 2048), (0, 4096, 512, 4096)]
    lens = [16384, 12000]
    xs = [S.audio_like(L, S.rng(85, i)).astype(np.float32) for i, L in enumerate(lens)]
    x = torch.from_numpy(np.concatenate(xs)).cuda()
    runs = []
    for flags in (0, mpg.MP_SCHED_NT512):
        plan = mpg.Plan(dicts, lens, 1e-3, flags)
        assert plan.stats().early_groups == (1 if flags == 0 else 0)
        plan.analyze(x)
        plan.run_resets(100000, 25.0, 300, -6.0)
        torch.cuda.synchronize()
        runs.append(plan)
    for s, xv in enumerate(xs):
        a, b = runs[0].atoms(s), runs[1].atoms(s)
        assert np.array_equal(a, b)
        inf = runs[0].info(s)
        assert inf.stop_reason == mpg.MP_STOP_SNR
        xp = np.zeros(inf.L_padded)
        xp[:len(xv)] = xv.astype(np.float64)
        yp = runs[0].resynth(s).cpu().numpy()
        assert abs(np.sum((xp - yp) ** 2) - inf.E) <= 1e-9 * inf.E0
        orc = O.mp_resets(dicts, xv.astype(np.float64), 1e-3, K=100000, target_db=25.0, reset_it=300, reset_db=-6.0)
        assert_tolerance(a, orc)


def test_mp_fp32_loop_with_fp64_dft():
    # FP32 plan whose analysis DFT runs in FP64 (MP_DFT_F64): the loop follows
    # the FP32 rule, and the initial coefficients are the FP64 ones rounded
    torch = _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 256, 64, 256), (0, 1024, 256, 1024)]
    lens = [16384, 9000]
    xs = [S.audio_like(L, S.rng(82, i)).astype(np.float32) for i, L in enumerate(lens)]
    _, ga = gpu_run(dicts, xs, 1e-4, K=0, snr_db=25.0, flags=mpg.MP_DFT_F64)
    for i, x in enumerate(xs):
        orc = oracle_run(dicts, x, 1e-4, snr_db=25.0, x_dtype=np.float32)
        assert_tolerance(ga[i], orc)


def test_autotune_fp64_plan_has_one_schedule():
    torch = _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 64, 16, 64), (0, 128, 32, 128)]
    x = np.random.default_rng(83).standard_normal(2048)
    xt = torch.from_numpy(x).cuda()
    plan, rep = mpg.Plan.autotuned(dicts, [len(x)], xt, 1e-4, F64, probe_atoms=50)
    assert len(rep["schedules"]) == 1 and rep["chosen"] == 0
    assert plan.stats().threads == rep["schedules"][0]["threads"]
    plan.analyze(xt)
    plan.run(300)
    torch.cuda.synchronize()
    assert_identical(plan.atoms(0), oracle_run(dicts, x, 1e-4, K=300))


def test_mp_fp32_batch_ragged():
    _torch()
    dicts = [(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)]
    lens = [16384, 9000, 20000, 8192, 12345]
    xs = [S.audio_like(L, S.rng(77, i)).astype(np.float32) for i, L in enumerate(lens)]
    _, ga = gpu_run(dicts, xs, 1e-4, K=0, snr_db=25.0, flags=0)
    for i, x in enumerate(xs):
        orc = oracle_run(dicts, x, 1e-4, snr_db=25.0, x_dtype=np.float32)
        assert_tolerance(ga[i], orc)


# --------------------------------------------------------------------------
# stop rules and degenerate inputs

def test_stop_rules():
    torch = _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 64, 16, 64), (0, 128, 32, 128)]
    x = np.random.default_rng(3).standard_normal(1024)
    # K
    plan, ga = gpu_run(dicts, [x], 1e-4, K=7, flags=F64)
    assert len(ga[0]) == 7 and plan.info(0).stop_reason == mpg.MP_STOP_K
    # SNR
    plan, ga = gpu_run(dicts, [x], 1e-4, K=100000, snr_db=10.0, flags=F64)
    E = plan.energy(0)
    assert plan.info(0).stop_reason == mpg.MP_STOP_SNR and E[-1] <= 0.1 * E[0] < E[-2]
    # E < 0 at a coarse threshold, compared with the oracle
    plan, ga = gpu_run(dicts, [x], 5e-2, K=100000, flags=F64)
    orc = oracle_run(dicts, x, 5e-2, K=100000, cap=100000)
    assert plan.info(0).stop_reason == mpg.MP_STOP_ENEG == orc.stop_reason
    assert_identical(ga[0], orc)
    # zero signal, batched with a nonzero one
    plan, ga = gpu_run(dicts, [np.zeros(1024), x], 1e-4, K=50, flags=0)
    assert len(ga[0]) == 0 and plan.info(0).stop_reason == mpg.MP_STOP_ZERO
    assert len(ga[1]) == 50
    # default K = L_padded / 5
    plan, ga = gpu_run(dicts, [x], 1e-4, K=0, flags=0)
    assert len(ga[0]) == 1024 // 5


def test_resume_continues_sequence():
    torch = _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 64, 16, 64), (0, 256, 64, 256)]
    x = np.random.default_rng(4).standard_normal(4096)
    plan = mpg.Plan(dicts, [4096], 1e-4, F64)
    plan.analyze(torch.from_numpy(x).cuda())
    plan.run(100)
    plan.run(2000)   # grows the atom log, continues
    ga = plan.atoms(0)
    orc = oracle_run(dicts, x, 1e-4, K=2000)
    assert_identical(ga, orc)


def test_resynth_and_coefs():
    torch = _torch()
    dicts = [(0, 64, 16, 64), (0, 256, 64, 256)]
    L = 4000
    x = np.random.default_rng(5).standard_normal(L)
    plan, ga = gpu_run(dicts, [x], 1e-4, K=500, flags=F64)
    orc = oracle_run(dicts, x, 1e-4, K=500)
    assert_identical(ga[0], orc)
    y = plan.resynth(0).cpu().numpy()
    yr = O.resynth(dicts, orc.L_padded, orc.w, orc.m, orc.n, orc.c)
    assert np.max(np.abs(y - yr)) < 1e-11 * np.abs(yr).max()
    for w, d in enumerate(dicts):
        c = plan.coefs(0, w).cpu().numpy()
        ref = np.zeros_like(c)
        for a in ga[0]:
            if a["w"] == w:
                ref[a["n"], a["m"]] += a["re"] + 1j * a["im"]
        assert np.max(np.abs(c - ref)) < 1e-14 * max(1.0, np.abs(ref).max())


def test_fresh_plan_after_freed_plans():
    # padding leaves must read as empty even when the allocator hands back
    # memory that earlier plans wrote
    torch = _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 64, 16, 64), (0, 256, 64, 256)]
    junk = []
    for i in range(3):
        x = np.random.default_rng(100 + i).standard_normal(8192)
        p = mpg.Plan(dicts, [8192], 1e-4, F64)
        p.analyze(torch.from_numpy(x).cuda())
        p.run(50)
        junk.append(p)
    del junk
    import gc
    gc.collect()
    x = np.random.default_rng(7).standard_normal(4096)
    _, ga = gpu_run(dicts, [x], 1e-4, K=200, flags=F64)
    assert_identical(ga[0], oracle_run(dicts, x, 1e-4, K=200))


# --------------------------------------------------------------------------
# reset procedure (Alg. 2)

@pytest.mark.parametrize("eps,reset_it", [(5e-2, 200), (1e-3, 150)])
def test_resets_fp64_identical(eps, reset_it):
    torch = _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 64, 16, 64), (0, 256, 64, 256)]
    L = 2000
    x = np.random.default_rng(7).standard_normal(L)
    plan = mpg.Plan(dicts, [L], eps, F64)
    plan.analyze(torch.from_numpy(x).cuda())
    plan.run_resets(900, 0.0, reset_it)
    ga = plan.atoms(0)
    orc = O.mp_resets(dicts, x, eps, K=900, reset_it=reset_it)
    assert len(ga) == orc.n_atoms
    assert np.array_equal(ga["w"], orc.w) and np.array_equal(ga["m"], orc.m) and np.array_equal(ga["n"], orc.n)
    c = ga["re"] + 1j * ga["im"]
    assert np.max(np.abs(c - orc.c)) <= 1e-9 * np.abs(orc.c).max()
    assert np.max(np.abs(ga["E_after"] - orc.E)) <= 1e-12 * orc.E0
    inf = plan.info(0)
    assert inf.stop_reason == orc.stop_reason
    assert abs(inf.E - orc.E_true[-1]) <= 1e-12 * orc.E0
    # the planes hold the analysis of the final true residual
    for w, d in enumerate(dicts):
        ref = O.dgt(d, orc.residual)
        got = plan.residual(0, w).cpu().numpy()
        assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("dft", ["f32", "f64", "f16pairs"])
def test_resets_fp32_batch_reach_true_target(dft):
    # dft f64: the re-analyses of the true residual run the FP64 DFT too;
    # f16pairs: they run the split DFT on matrix cores from the FP64 residual
    torch = _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 64, 16, 64), (0, 256, 64, 256)]
    lens = [2048, 3000, 4096]
    xs = [np.random.default_rng(20 + i).standard_normal(L).astype(np.float32) for i, L in enumerate(lens)]
    flags = {"f32": 0, "f64": mpg.MP_DFT_F64, "f16pairs": mpg.MP_DFT_F16SPLIT}[dft]
    plan = mpg.Plan(dicts, lens, 5e-2, flags)
    plan.analyze(torch.from_numpy(np.concatenate(xs)).cuda())
    plan.run_resets(100000, 30.0, 200, -6.0)
    for s, x in enumerate(xs):
        inf = plan.info(s)
        assert inf.stop_reason == mpg.MP_STOP_SNR
        assert inf.E <= 1e-3 * inf.E0
        # the reported error is the energy of the true residual
        xd = x.astype(np.float64)
        Lp = inf.L_padded
        yp = plan.resynth(s).cpu().numpy()
        xp = np.zeros(Lp)
        xp[:len(x)] = xd
        assert abs(np.sum((xp - yp) ** 2) - inf.E) <= 1e-9 * inf.E0
        orc = O.mp_resets(dicts, xd, 5e-2, K=100000, target_db=30.0, reset_it=200, reset_db=-6.0)
        assert_tolerance(plan.atoms(s), orc)
