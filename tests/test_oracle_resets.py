"""Pins of the oracle's reset procedure (Alg. 2), which is composed of the
oracle's MP (Alg. 1), synthesis and analysis.  What fixes it:

* with the exact Gram matrix (epsilon = 0) the coefficient-domain residual is
  the analysis of the true residual, so resets cannot change the selections;
* the error after each round is the energy of x minus the synthesis of every
  selection so far, computed here independently in one pass;
* with a coarse threshold the estimate of plain approximate MP says the target
  is reached while the true error is far above it; with resets the true error
  reaches the target (Theorem 2 / Corollary 1 of the paper's Sec. 3);
* a relative inner criterion (reset_db) ends each round once the estimate has
  fallen by that many dB, so every round lowers the true error.
"""
import numpy as np
import pytest

from oracle import core as O


def test_exact_gram_resets_do_not_change_the_selection():
    dicts = [(0, 32, 8, 32), (0, 64, 16, 64)]
    x = np.random.default_rng(6).standard_normal(512)
    a = O.mp(dicts, x, 0.0, K=200)
    b = O.mp_resets(dicts, x, 0.0, K=200, reset_it=37)
    assert np.array_equal(a.w, b.w) and np.array_equal(a.m, b.m) and np.array_equal(a.n, b.n)
    assert np.max(np.abs(a.c - b.c)) < 1e-12 * np.max(np.abs(a.c))
    # at every reset the true error equals the estimate of plain MP there
    for kr, et in zip(b.k_rounds, b.E_true):
        assert abs(et - a.E[kr - 1]) < 1e-10 * a.E0
    assert len(b.k_rounds) == int(np.ceil(200 / 37))


@pytest.mark.parametrize("eps,reset_it", [(5e-2, 200), (1e-3, 150)])
def test_true_error_is_the_synthesis_residual(eps, reset_it):
    dicts = [(0, 64, 16, 64), (0, 256, 64, 256)]
    x = np.random.default_rng(7).standard_normal(2000)
    r = O.mp_resets(dicts, x, eps, K=900, reset_it=reset_it)
    y = O.resynth(dicts, r.L_padded, r.w, r.m, r.n, r.c)
    xp = np.zeros(r.L_padded)
    xp[:len(x)] = x
    res = xp - y
    assert np.max(np.abs(res - r.residual)) < 1e-10 * np.abs(xp).max()
    assert abs(res @ res - r.E_true[-1]) < 1e-10 * r.E0
    # each round's inner estimates start from the previous round's true error
    starts = np.concatenate([[0], r.k_rounds[:-1]])
    prev = np.concatenate([[r.E0], r.E_true[:-1]])
    for s0, ep in zip(starts, prev):
        if s0 < r.n_atoms:
            assert r.E[s0] < ep


def test_resets_reach_the_target_where_the_estimate_misleads():
    dicts = [(0, 64, 16, 64), (0, 256, 64, 256)]
    x = np.random.default_rng(5).standard_normal(2048)
    E0 = float(x @ x)
    plain = O.mp(dicts, x, 5e-2, K=100000, target_db=30.0, cap=100000)
    y = O.resynth(dicts, plain.L_padded, plain.w, plain.m, plain.n, plain.c)[:len(x)]
    true_plain_db = 10 * np.log10(E0 / np.sum((x - y) ** 2))
    assert plain.E[-1] <= 1e-3 * E0          # the estimate claims 30 dB ...
    assert true_plain_db < 20.0               # ... far from the truth
    r = O.mp_resets(dicts, x, 5e-2, K=100000, target_db=30.0, reset_it=200)
    assert r.stop_reason == 2
    assert r.E_true[-1] <= 1e-3 * r.E0 and 10 * np.log10(r.E0 / r.E_true[-1]) >= 30.0
    assert len(r.E_true) > 2


def test_relative_inner_criterion_lowers_the_true_error_every_round():
    dicts = [(0, 64, 16, 64), (0, 256, 64, 256)]
    x = np.random.default_rng(9).standard_normal(2048)
    r = O.mp_resets(dicts, x, 2e-2, K=100000, target_db=25.0, reset_it=100000, reset_db=-3.0)
    assert r.stop_reason == 2 and len(r.E_true) >= 5
    assert np.all(np.diff(r.E_true) < 0)
    # every round ended on the relative criterion: its last estimate is at or
    # below half the error it started from
    starts = np.concatenate([[r.E0], r.E_true[:-1]])
    for kr, ep in zip(r.k_rounds[:-1], starts[:-1]):
        assert r.E[kr - 1] <= ep * 10 ** (-0.3) * (1 + 1e-12)
