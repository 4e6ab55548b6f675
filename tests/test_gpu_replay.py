"""Whole-run GPU parity, past the first divergence from the oracle's own
sequence: the oracle replays the GPU's selections (orc_mp_replay), the
coefficient error of the GPU planes is measured at checkpoints, and every GPU
selection must be a maximum of the oracle's scores within that error, with
the error estimates within 1e-5 ||x||^2 of the replay's.

* sampled signals of the 256-signal batch (the two shortest, the median and
  the longest), FP32, to 40 dB: also the FP32 error model (the coefficient
  error stays a small multiple of u32 times the largest initial coefficient);
* a white-noise run that stops on a negative error estimate (Sec. 6.1), FP32,
  against the oracle's own stop.
"""
import numpy as np
import pytest

from oracle import core as O
from paper_2202_12380_amd import signals as S
from gpu_helpers import gpu_run_staged, oracle_run, assert_tolerance, agreement, replay_check

pytestmark = pytest.mark.gpu

def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.mark.parametrize("flags", [0x40, 0x0])
def test_fp32_c3_sampled_signals_whole_run(flags):
    # analysis in FP16 pairs on matrix cores (0x40, as benchmarked) or the FP32 FFT
    _torch()
    wl = S.workload(3)
    xs = S.signals(3)
    order = np.argsort([len(x) for x in xs])
    pick = [int(order[0]), int(order[1]), int(order[len(xs) // 2]), int(order[-1])]
    sub = [xs[i].astype(np.float32) for i in pick]
    plan, ga, cps = gpu_run_staged(wl.dicts, sub, wl.eps, [1000, 6000, 1 << 17], snr_db=40.0,
                                   keep=range(len(sub)), flags=flags)
    for j, i in enumerate(pick):
        x = sub[j].astype(np.float64)
        orc = oracle_run(wl.dicts, x, wl.eps, K=1 << 17, snr_db=40.0)
        print("signal %d (L=%d):" % (i, len(x)), agreement(ga[j], orc))
        rep = replay_check(wl.dicts, x, wl.eps, ga[j], cps[j])
        assert plan.info(j).stop_reason == 2          # 40 dB on the estimate
        # the replay's estimate after the GPU's last selection meets the target too
        assert rep["n"] == len(ga[j])


def test_fp32_white_noise_until_negative_estimate():
    # Sec. 6.1's stop rule on a reduced-scale white-noise signal (2^16
    # samples, the study's three Blackman systems, eps = 1e-3)
    _torch()
    from paper_2202_12380_amd import mpg
    dicts = [(0, 512, 128, 512), (0, 1024, 256, 1024), (0, 2048, 512, 2048)]
    L = 1 << 16
    x = np.random.default_rng(2022).standard_normal(L).astype(np.float32)
    eps = 1e-3
    plan, ga, cps = gpu_run_staged(dicts, [x], eps, [5000, 20000, 1 << 22], keep=[0])
    inf = plan.info(0)
    assert inf.stop_reason == mpg.MP_STOP_ENEG
    orc = oracle_run(dicts, x, eps, K=1 << 22, cap=1 << 22)
    assert orc.stop_reason == O.STOP_ENEG
    k_gpu, k_orc = len(ga[0]), orc.n_atoms
    print("white noise: GPU stops after %d, oracle after %d; %s" % (k_gpu, k_orc, agreement(ga[0], orc)))
    assert abs(k_gpu - k_orc) <= 0.05 * k_orc
    rep = replay_check(dicts, x.astype(np.float64), eps, ga[0], cps[0])
    # along the GPU's own selections the oracle's estimate also reaches zero
    # at the end (within the energy tolerance) and not much earlier
    r = O.mp_replay(dicts, x.astype(np.float64), eps, ga[0]["w"], ga[0]["m"], ga[0]["n"])
    assert r.E[-1] <= 1e-5 * r.E0
    assert np.all(r.E[:-1] >= -1e-5 * r.E0)
