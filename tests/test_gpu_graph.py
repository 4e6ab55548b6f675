"""mp_analyze + mp_run captured into a HIP graph (torch.cuda.CUDAGraph on the
library's C-ABI calls) and replayed: every replay, with eager GPU work and
synchronisations in between, selects exactly what the eager calls select
(the batched configuration's captured loop)."""
import numpy as np
import pytest

from paper_2202_12380_amd import signals as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("flags", [0x40, 0x0])
def test_captured_analysis_and_loop_replay_like_eager(flags):
    # analysis in FP16 pairs on matrix cores (0x40, as benchmarked) or the FP32 FFT
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_12380_amd import mpg
    dicts = [(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)]
    lens = [16384, 9000, 20000, 12288]
    xs = [S.audio_like(L, S.rng(95, i)).astype(np.float32) for i, L in enumerate(lens)]
    x = torch.from_numpy(np.concatenate(xs)).cuda()
    plan = mpg.Plan(dicts, lens, 1e-4, flags)
    K, snr = 4000, 30.0
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.analyze(x, s)                     # eager reference (also sizes the atom logs)
        plan.run(K, snr, s)
    torch.cuda.synchronize()
    ref = [plan.atoms(i) for i in range(len(lens))]
    assert all(len(a) > 100 for a in ref)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.analyze(x, s)
        plan.run(K, snr, s)
    torch.cuda.synchronize()
    for rep in range(3):
        # unrelated eager work between replays
        y = torch.randn(1 << 20, device="cuda")
        _ = (y * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(lens)):
            a = plan.atoms(i)
            print("replay %d signal %d: %d atoms" % (rep, i, len(a)), flush=True)
            assert len(a) == len(ref[i])
            for f in ("w", "m", "n", "re", "im", "E_after"):
                assert np.array_equal(a[f], ref[i][f]), (rep, i, f)
    del g
    plan.close()


def test_capture_before_any_eager_call():
    # a fresh plan whose first mp_analyze / mp_run happen under capture (the
    # launchers' attribute and occupancy queries run inside the capture); the
    # replays select what a second plan selects eagerly
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_12380_amd import mpg
    dicts = [(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)]
    lens = [16384, 9000]
    xs = [S.audio_like(L, S.rng(96, i)).astype(np.float32) for i, L in enumerate(lens)]
    x = torch.from_numpy(np.concatenate(xs)).cuda()
    K, snr = 2000, 25.0
    ref_plan = mpg.Plan(dicts, lens, 1e-4, 0x40)
    ref_plan.analyze(x)
    ref_plan.run(K, snr)
    torch.cuda.synchronize()
    ref = [ref_plan.atoms(i) for i in range(len(lens))]
    ref_plan.close()
    plan = mpg.Plan(dicts, lens, 1e-4, 0x40)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    try:
        with torch.cuda.graph(g, stream=s):
            plan.analyze(x, s)
            plan.run(K, snr, s)
    except mpg.MPError as e:
        # the atom logs cannot grow under capture (MP_E_STATE): size them with
        # one eager run of the loop alone, then capture again
        assert e.code == mpg.MP_E_STATE, e
        del g
        with torch.cuda.stream(s):
            plan.analyze(x, s)
            plan.run(K, snr, s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            plan.analyze(x, s)
            plan.run(K, snr, s)
    torch.cuda.synchronize()
    for rep in range(2):
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(lens)):
            a = plan.atoms(i)
            assert len(a) == len(ref[i]), (rep, i)
            for f in ("w", "m", "n", "re", "im", "E_after"):
                assert np.array_equal(a[f], ref[i][f]), (rep, i, f)
    del g
    plan.close()
