"""The allocation-free synthesis entry point (mp_resynth_static) against the
plan-buffer one (mp_resynth), through the C-ABI: the same samples on two calls
in a row, the second on a shorter signal, so that a stale accumulator from the
first call would show; both also against the oracle's synthesis."""
import numpy as np
import pytest

from oracle import core as O
from paper_2202_12380_amd import signals as S

pytestmark = pytest.mark.gpu


def test_static_resynth_matches_plan_resynth_twice():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_12380_amd import mpg
    dicts = [(0, 256, 64, 256), (0, 1024, 256, 1024), (0, 4096, 1024, 4096)]
    lens = [40000, 17000]                         # the second call is on the shorter signal
    xs = [S.audio_like(L, S.rng(91, i)).astype(np.float32) for i, L in enumerate(lens)]
    plan = mpg.Plan(dicts, lens, 1e-4, 0)
    plan.analyze(torch.from_numpy(np.concatenate(xs)).cuda())
    plan.run(0, 30.0)
    torch.cuda.synchronize()
    for sig, dt, code in ((0, torch.float64, mpg.MP_DTYPE_F64), (1, torch.float32, mpg.MP_DTYPE_F32)):
        inf = plan.info(sig)
        print("signal %d: L_padded %d, %d atoms" % (sig, inf.L_padded, inf.n_atoms), flush=True)
        assert inf.n_atoms > 100
        y_ref = torch.empty(inf.L_padded, dtype=dt, device="cuda")
        y_st = torch.full((inf.L_padded,), float("nan"), dtype=dt, device="cuda")
        mpg.mp_resynth(plan.h, sig, y_ref.data_ptr(), code)
        mpg.mp_resynth_static(plan.h, sig, y_st.data_ptr(), code)
        torch.cuda.synchronize()
        a, b = y_ref.cpu().numpy(), y_st.cpu().numpy()
        assert np.array_equal(a, b), np.max(np.abs(a - b))   # same kernels, same order of sums
        at = plan.atoms(sig)
        ref = O.resynth(dicts, inf.L_padded, at["w"], at["m"], at["n"], at["re"] + 1j * at["im"])
        tol = 1e-11 if dt == torch.float64 else 2e-7
        assert np.max(np.abs(b - ref)) <= tol * np.max(np.abs(ref))
    plan.close()


def test_static_resynth_limit():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2202_12380_amd import mpg
    L = mpg.MP_STATIC_RESYNTH_MAX + 4096
    plan = mpg.Plan([(0, 64, 16, 64)], [L], 1e-4, 0)
    plan.analyze(torch.zeros(L, dtype=torch.float32, device="cuda"))
    y = torch.empty(L, dtype=torch.float32, device="cuda")
    with pytest.raises(mpg.MPError) as e:
        mpg.mp_resynth_static(plan.h, 0, y.data_ptr(), mpg.MP_DTYPE_F32)
    assert e.value.code == mpg.MP_E_LIMIT
    plan.close()
