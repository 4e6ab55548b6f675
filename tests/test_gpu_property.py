"""Property-based parity of the HIP path with the oracle on random small
configurations: one to three Gabor systems with any window, frame lengths
8 .. 256, windows up to twice the frame, hops that divide M or not, ragged
signal lengths.  FP64 plans must select what the oracle selects (up to the
first selection whose oracle top-2 gap is below 1e-10, where rounding may
legitimately decide).  FP32 plans run 150 selections on signals as short as
64 samples, far below the signal's energy; each run is replayed on the oracle
with the GPU planes taken after every selection, so that every selection is
checked to be a maximum within the coefficient error measured right there,
E within 1e-5 ||x||^2; the sequence must agree with the oracle's own up to
the first top-2 gap below 1e-6 or below what the run's largest measured
coefficient error allows (gpu_helpers.measured_floor_agreement)."""
import numpy as np
import pytest
from hypothesis import given, settings, HealthCheck, strategies as st

from oracle import core as O
from gpu_helpers import (gpu_run, gpu_run_staged, oracle_run, first_mismatch, agreement, replay_check,
                         measured_floor_agreement)

pytestmark = pytest.mark.gpu
F64 = 0x1


@st.composite
def _systems(draw):
    W = draw(st.integers(1, 3))
    dicts = []
    while len(dicts) < W:
        M = 2 ** draw(st.integers(3, 8))
        gl = 2 * draw(st.integers(2, M))
        a = draw(st.sampled_from(sorted({M // 8, M // 4, M // 2, M, 3 * M // 8, 3 * M // 4})))
        d = (draw(st.integers(0, 2)), gl, a, M)
        if d not in dicts:
            dicts.append(d)
    L = draw(st.integers(64, 4096))
    return dicts, L, draw(st.integers(0, 2 ** 31 - 1))


def _signal(L, seed):
    return np.random.default_rng(seed).standard_normal(L)


_SETTINGS = settings(max_examples=20, deadline=None, derandomize=True,
                     suppress_health_check=[HealthCheck.too_slow, HealthCheck.filter_too_much])


@_SETTINGS
@given(_systems())
def test_random_configs_fp64_same_selections(cfg):
    pytest.importorskip("torch")
    dicts, L, seed = cfg
    Lp = O.padded_length(dicts, L)
    if Lp < 0 or Lp > 16384:
        return
    x = _signal(L, seed)
    K = 150
    print("fp64 case", dicts, L, seed, flush=True)
    _, ga = gpu_run(dicts, [x], 1e-4, K=K, flags=F64)
    orc = oracle_run(dicts, x, 1e-4, K=K)
    small = np.nonzero(orc.gap < 1e-10)[0]
    upto = int(small[0]) if len(small) else orc.n_atoms
    fm = first_mismatch(ga[0], orc)
    assert fm >= upto, "differs at %d before the first near-tie at %d: %s" % (fm, upto, dicts)
    if upto:
        c = ga[0]["re"][:upto] + 1j * ga[0]["im"][:upto]
        assert np.max(np.abs(c - orc.c[:upto])) <= 1e-9 * np.max(np.abs(orc.c))
        assert np.max(np.abs(ga[0]["E_after"][:upto] - orc.E[:upto])) <= 1e-12 * orc.E0


@_SETTINGS
@given(_systems())
def test_random_configs_fp32_rule(cfg):
    pytest.importorskip("torch")
    dicts, L, seed = cfg
    Lp = O.padded_length(dicts, L)
    if Lp < 0 or Lp > 16384:
        return
    x = _signal(L, seed).astype(np.float32)
    K = 150
    print("fp32 case", dicts, L, seed, flush=True)
    plan, ga, cps = gpu_run_staged(dicts, [x], 1e-4, list(range(1, K + 1)), keep=[0])
    orc = oracle_run(dicts, x, 1e-4, K=K, x_dtype=np.float32)
    rep = replay_check(dicts, x.astype(np.float64), 1e-4, ga[0], cps[0], c_model=None)
    fm, k_lit, _ = agreement(ga[0], orc)
    k_meas = measured_floor_agreement(ga[0], orc, rep["max_error"])
    n = min(len(ga[0]), orc.n_atoms)
    print("agreement: %d of %d (literal 1e-6 rule from %d, measured-error rule from %d)" % (fm, n, k_lit, k_meas))
    if fm < n:
        assert fm >= k_meas, "sequence differs at %d before the gap allowed by the measured error (%d)" % (
            fm, k_meas)
    if fm:
        assert np.max(np.abs(ga[0]["E_after"][:fm] - orc.E[:fm])) <= 1e-5 * orc.E0


@st.composite
def _split_dft_systems(draw):
    # one to three systems of M = 256 .. 4096 (the frame-group split DFT's
    # shapes), any window, windows from M/4 to 2M, hops dividing M or not;
    # a batch of one to three ragged signals
    W = draw(st.integers(1, 3))
    dicts = []
    while len(dicts) < W:
        M = 2 ** draw(st.integers(8, 12))
        gl = 2 * draw(st.integers(M // 8, M))
        a = draw(st.sampled_from(sorted({M // 8, M // 4, M // 2, 3 * M // 8})))
        d = (draw(st.integers(0, 2)), gl, a, M)
        if d not in dicts:
            dicts.append(d)
    lens = draw(st.lists(st.integers(256, 12000), min_size=1, max_size=3))
    return dicts, lens, draw(st.integers(0, 2 ** 31 - 1)), draw(st.sampled_from([0x40, 0x80]))


@settings(max_examples=15, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.filter_too_much])
@given(_split_dft_systems())
def test_random_configs_split_dft_planes(cfg):
    # planes of the split DFT on matrix cores against the oracle's DGT, element
    # by element, relative to each plane's maximum (FP16 pairs 3e-6, BF16 5e-5)
    torch = pytest.importorskip("torch")
    from paper_2202_12380_amd import mpg
    dicts, lens, seed, fmt = cfg
    Lp = [O.padded_length(dicts, L) for L in lens]
    if min(Lp) < 0 or max(Lp) > 65536:
        return
    print("split dft case", dicts, lens, seed, hex(fmt), flush=True)
    xs = [np.random.default_rng(seed + i).standard_normal(L).astype(np.float32).astype(np.float64)
          for i, L in enumerate(lens)]
    plan = mpg.Plan(dicts, lens, 1e-4, fmt)
    plan.analyze(torch.from_numpy(np.concatenate(xs)).to(torch.float32).cuda())
    tol = 3e-6 if fmt == 0x40 else 5e-5
    for s_, (L, v) in enumerate(zip(lens, xs)):
        xp = np.zeros(Lp[s_])
        xp[:L] = v
        for w, d in enumerate(dicts):
            ref = O.dgt(d, xp)
            got = plan.residual(s_, w).cpu().numpy()
            assert np.max(np.abs(got - ref)) <= tol * np.abs(ref).max(), (dicts, lens, s_, w)
    plan.close()
