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


def gpu_run_staged(dicts, xs, eps, stages, snr_db=0.0, flags=0, keep=()):
    """Runs the HIP path on a batch in stages (mp_run resumed with the
    selection caps in `stages`, the last one the real cap).  Returns (plan,
    atoms per signal, checkpoints) where checkpoints[s] maps the selection
    count of signal s (for s in keep) after the analysis (0) and after each
    stage to its residual planes."""
    import torch
    from paper_2202_12380_amd import mpg
    f64 = bool(flags & mpg.MP_PREC_F64)
    x_dtype = torch.float64 if f64 else torch.float32
    plan = mpg.Plan(dicts, [len(x) for x in xs], eps, flags)
    x = torch.from_numpy(np.concatenate([np.asarray(v, np.float64) for v in xs])).to(x_dtype).cuda()
    plan.analyze(x)
    torch.cuda.synchronize()
    cps = {s: {0: planes_of(plan, s, len(dicts))} for s in keep}   # after the analysis
    for K in stages:
        plan.run(K, snr_db)
        torch.cuda.synchronize()
        for s in keep:
            k = int(plan.info(s).n_atoms)
            if k not in cps[s]:
                cps[s][k] = planes_of(plan, s, len(dicts))
    return plan, [plan.atoms(s) for s in range(len(xs))], cps


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


U32 = 2.0 ** -24      # unit roundoff of FP32

# Measured coefficient error of the GPU paths, in units of u32 sqrt(S_0)
# (S_0 the largest initial selection score): max |rho_gpu - rho_oracle| over
# all coefficients stays at 1.7 .. 4.3 for the FP32 FFT and FP16-pair
# analyses and 15 .. 20 for BF16 pairs, from the start of a run to its end
# (40 dB on audio-like signals, 5e4 selections on white noise; replay tests).
# The error model used below takes twice the largest measured value.
C_FP32 = 8.0
C_BF16 = 32.0


def fp32_gap_floor(orc, gap_tol=1e-6, c=C_FP32):
    """Top-2 gap below which the GPU may legitimately select the other
    coefficient: with an error e <= c u32 sqrt(S_0) on every coefficient, two
    scores S_k (1 - g) and S_k may swap when g < 4 e / sqrt(S_k) =
    4 c u32 sqrt(S_0 / S_k) (S_k the selected score at step k).  Reported
    next to the literal rule; asserted only for the cases that name
    themselves (floor=True)."""
    if not orc.n_atoms:
        return np.zeros(0)
    S = np.maximum(orc.best, 1e-300)
    return np.maximum(gap_tol, 4.0 * c * U32 * np.sqrt(S[0] / S))


def agreement(ga, orc, gap_tol=1e-6, c=C_FP32):
    """First difference of the sequences and the first oracle selections
    whose top-2 gap is below the literal tolerance and below the floor."""
    fm = first_mismatch(ga, orc)
    small = np.nonzero(orc.gap < gap_tol)[0]
    k_lit = int(small[0]) if len(small) else orc.n_atoms
    if getattr(orc, "best", None) is None:
        return fm, k_lit, k_lit
    small_f = np.nonzero(orc.gap < fp32_gap_floor(orc, gap_tol, c))[0]
    k_floor = int(small_f[0]) if len(small_f) else orc.n_atoms
    return fm, k_lit, k_floor


def measured_floor_agreement(ga, orc, e, gap_tol=1e-6):
    """First oracle selection at which the GPU may legitimately choose another
    coefficient given a measured error e on every coefficient: its top-2 gap
    is below max(gap_tol, (4 sqrt(S_k) e + 2 e^2) / S_k)."""
    S = np.maximum(orc.best, 1e-300)
    thr = np.maximum(gap_tol, (4.0 * np.sqrt(S) * e + 2.0 * e * e) / S)
    small = np.nonzero(orc.gap < thr)[0]
    return int(small[0]) if len(small) else orc.n_atoms


def assert_tolerance(ga, orc, gap_tol=1e-6, e_tol=1e-5, floor=False, c=C_FP32):
    """FP32 path: the same sequence up to the first selection whose oracle
    top-2 gap is below gap_tol (the literal rule), and E within e_tol ||x||^2
    up to there.  floor=True (cases named as needing it) asserts the floor of
    the measured error model instead; both agreement lengths are printed."""
    fm, k_lit, k_floor = agreement(ga, orc, gap_tol, c)
    n = min(len(ga), orc.n_atoms)
    print("agreement: %d of %d (literal %g rule from %d, floor rule from %d)" % (
        fm, n, gap_tol, k_lit, k_floor))
    k_gap = k_floor if floor else k_lit
    if fm < n:
        assert fm >= k_gap, "sequence differs at %d before the first small gap at %d (gap %.3g)" % (
            fm, k_gap, orc.gap[fm])
    upto = min(fm, n)
    if upto:
        assert np.max(np.abs(ga["E_after"][:upto] - orc.E[:upto])) <= e_tol * orc.E0
    return fm, k_gap


def planes_of(plan, s, n_sys):
    return [plan.residual(s, w).cpu().numpy().astype(np.complex128) for w in range(n_sys)]


def replay_check(dicts, x, eps, ga, plane_checkpoints, flags=0, e_tol=1e-5, c_model=C_FP32):
    """Checks a whole GPU run, past any divergence from the oracle's own
    sequence: the oracle replays the GPU's selections (orc_mp_replay) and
      * at each checkpoint k (GPU planes after k selections, given as
        {k: [plane per system]}) the largest coefficient error
        e_k = max |rho_gpu - rho_oracle| is measured;
      * every GPU selection must be a maximum of the oracle's scores up to
        that error: chosen >= best - 4 sqrt(best) e - 2 e^2 (scores are
        |rho|^2; an error e per coefficient moves a score by at most
        2 |rho| e + e^2, on both sides of the comparison).  Selection i is
        made on the planes after i selections; e is the error measured there
        when a checkpoint sits at i, else the larger of the errors at the two
        checkpoints around i (exact with a checkpoint at every selection; with
        sparse checkpoints it assumes that the error between two checkpoints
        stays within theirs, which c_model backs);
      * the GPU's error estimates follow the replay's within e_tol ||x||^2.
    c_model: if not None, e_k <= c_model u32 sqrt(S_0) is asserted too (S_0
    the largest initial score): the error model of fp32_gap_floor.  Returns a
    report dict."""
    xv = np.asarray(x, np.float64)
    oflags = 0
    if flags & 0x10:
        oflags |= O.THR_REL
    if flags & 0x20:
        oflags |= O.CONJ_GATE_GAMMA
    if flags & 0x100:
        oflags |= O.PEDANTIC
    k_all = len(ga)
    ks = sorted(plane_checkpoints)
    assert ks and ks[-1] == k_all, "the last checkpoint must be the end of the run"
    errs = {}
    rep = None
    for k in ks:
        r = O.mp_replay(dicts, xv, eps, ga["w"][:k], ga["m"][:k], ga["n"][:k], flags=oflags,
                        return_planes=True)
        errs[k] = max(float(np.max(np.abs(g - o))) for g, o in zip(plane_checkpoints[k], r.planes))
        if k == k_all:
            rep = r
    S0 = float(rep.best[0]) if k_all else 0.0
    # error bound per selection: the checkpoint at it, else the larger of the
    # two around it
    ka = np.asarray(ks)
    ea = np.asarray([errs[q] for q in ks])
    idx = np.arange(k_all)
    j1 = np.searchsorted(ka, idx, side="right") - 1      # last checkpoint <= i
    j2 = np.searchsorted(ka, idx, side="left")           # first checkpoint >= i
    e1 = np.where(j1 >= 0, ea[np.clip(j1, 0, len(ka) - 1)], 0.0)
    e2 = np.where(j2 < len(ka), ea[np.clip(j2, 0, len(ka) - 1)], 0.0)
    bound = np.maximum(e1, e2)
    slack = rep.best - rep.chosen
    allowed = 4.0 * np.sqrt(rep.best) * bound + 2.0 * bound ** 2
    bad = np.nonzero(slack > allowed * (1 + 1e-12) + 1e-300)[0]
    dE = float(np.max(np.abs(ga["E_after"] - rep.E))) / rep.E0 if k_all else 0.0
    c_meas = {k: errs[k] / (U32 * np.sqrt(S0)) for k in ks} if S0 > 0 else {}
    report = dict(n=k_all, errors=errs, c_measured=c_meas, invalid=len(bad),
                  first_invalid=int(bad[0]) if len(bad) else -1,
                  worst_ratio=float(np.max(slack / np.maximum(allowed, 1e-300))) if k_all else 0.0,
                  max_dE_over_E0=dE)
    report["max_error"] = float(ea.max())
    if len(ks) > 8:  # dense checkpoints: print the largest ones only
        top = sorted(ks, key=lambda q: -errs[q])[:4]
        shown = dict(report, errors={q: errs[q] for q in top},
                     c_measured={q: c_meas[q] for q in top} if c_meas else {})
        print("replay (%d checkpoints, largest shown):" % len(ks), shown)
    else:
        print("replay:", report)
    assert len(bad) == 0, "GPU selection %d is not a maximum within the measured error (%s)" % (
        bad[0], report)
    assert dE <= e_tol, report
    if c_model is not None:
        assert all(v <= c_model for v in c_meas.values()), report
    return report
