"""Shared helpers for the GPU parity tests: run the HIP path through the C-ABI
binding and the oracle on the same seeded inputs, and compare under the stated
tolerances."""
import numpy as np

from oracle import core as O


def gpu_run(dicts, xs, eps, K=0, snr_db=0.0, flags=0, x_dtype=None):
    """Runs the HIP path on a batch; returns (plan, list of atom arrays)."""
    import torch
    from paper_2202_12380_amd import mpg
    f64 = bool(flags & mpg.MP_PREC_F64)
    if x_dtype is None:
        x_dtype = torch.float64 if f64 else torch.float32
    plan = mpg.Plan(dicts, [len(x) for x in xs], eps, flags)
    x = torch.from_numpy(np.concatenate([np.asarray(v, np.float64) for v in xs])).to(x_dtype).cuda()
    plan.analyze(x)
    plan.run(K, snr_db)
    torch.cuda.synchronize()
    return plan, [plan.atoms(s) for s in range(len(xs))]


def oracle_run(dicts, x, eps, K=0, snr_db=0.0, flags=0, x_dtype=np.float64, cap=None):
    xv = np.asarray(x).astype(x_dtype).astype(np.float64)
    oflags = 0
    if flags & 0x10:
        oflags |= O.THR_REL
    if flags & 0x20:
        oflags |= O.CONJ_GATE_GAMMA
    if flags & 0x100:
        oflags |= O.PEDANTIC
    return O.mp(dicts, xv, eps, K=K, target_db=snr_db, flags=oflags, cap=cap)


def first_mismatch(ga, orc):
    n = min(len(ga), orc.n_atoms)
    same = (ga["w"][:n] == orc.w[:n]) & (ga["m"][:n] == orc.m[:n]) & (ga["n"][:n] == orc.n[:n])
    if same.all():
        return n
    return int(np.argmin(same))


def assert_identical(ga, orc, c_rel=1e-9, e_rel=1e-12):
    """FP64 path: identical atom sequence (ties broken by lowest index)."""
    fm = first_mismatch(ga, orc)
    assert len(ga) == orc.n_atoms, (len(ga), orc.n_atoms)
    assert fm == orc.n_atoms, "sequence differs at %d (oracle gap there %.3g, min gap %.3g)" % (
        fm, orc.gap[fm] if fm < orc.n_atoms else -1, orc.gap.min() if orc.n_atoms else -1)
    if orc.n_atoms:
        c = ga["re"] + 1j * ga["im"]
        scale = np.max(np.abs(orc.c))
        assert np.max(np.abs(c - orc.c)) <= c_rel * scale
        assert np.max(np.abs(ga["E_after"] - orc.E)) <= e_rel * orc.E0


def fp32_gap_floor(orc, gap_tol=1e-6):
    """Per-selection top-2 gap below which FP32 may legitimately pick the other
    coefficient.  A coefficient keeps an absolute rounding error of about
    u32 |rho_0| sqrt(n) from the n (~16) large early updates that touched it,
    while its value decays with the residual, |rho_k| ~ |rho_0| sqrt(E_k / E0);
    the relative error of |rho_k|^2 is then about 2 u32 sqrt(n) sqrt(E0 / E_k)
    ~ 1e-6 sqrt(E0 / E_k).  The floor is gap_tol at the start and grows as the
    energy falls (1e-4 at 40 dB)."""
    E_before = np.concatenate([[orc.E0], orc.E[:-1]]) if orc.n_atoms else np.zeros(0)
    return np.maximum(gap_tol, 1e-6 * np.sqrt(orc.E0 / np.maximum(E_before, 1e-300)))


def assert_tolerance(ga, orc, gap_tol=1e-6, e_tol=1e-5):
    """FP32 path: same sequence up to the first selection whose top-2 gap is
    below the FP32 floor (gap_tol, growing with the energy decay, see
    fp32_gap_floor), and E within e_tol * ||x||^2 up to there."""
    fm = first_mismatch(ga, orc)
    small = np.nonzero(orc.gap < fp32_gap_floor(orc, gap_tol))[0]
    k_gap = int(small[0]) if len(small) else orc.n_atoms
    if fm < min(len(ga), orc.n_atoms):
        assert fm >= k_gap, "sequence differs at %d before the first small gap at %d (gap %.3g)" % (
            fm, k_gap, orc.gap[fm])
    else:
        # one run may simply be longer (different stop step)
        assert fm == min(len(ga), orc.n_atoms)
    upto = min(fm, len(ga), orc.n_atoms)
    if upto:
        assert np.max(np.abs(ga["E_after"][:upto] - orc.E[:upto])) <= e_tol * orc.E0
    return fm, k_gap
