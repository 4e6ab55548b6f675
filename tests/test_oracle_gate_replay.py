"""Pins for two oracle paths that the first pin file does not reach:

* the literal conjugate-partner condition of Alg. 3 (the partner term only
  when gamma != 0), against approximate MP written with the truncated Gram
  matrix of explicitly built atoms (no kernels, no grids, no modulation
  table), with and without the condition, on inputs where it matters;
* the replay mode (selections taken from another run): on its own sequence it
  is the oracle's loop bit for bit, and at eps = 0 it equals signal-domain
  projection along ANY selection list, argmax or not.
"""
import numpy as np
import pytest

from oracle import core as O
from oracle import textbook as T


def _planted_low_high(dicts, L, seed, noise=0.05):
    """Real atoms near DC and near Nyquist (where the partner condition
    matters), plus noise."""
    rng = np.random.default_rng(seed)
    x = noise * rng.standard_normal(L)
    for w, d in enumerate(dicts):
        M = d[3]
        for m in (3, 4, 5, M // 2 - 3, M // 2 - 4):
            n = int(rng.integers(0, L // d[2]))
            alpha = complex(rng.standard_normal(), rng.standard_normal())
            x += (alpha * T.atom(d, m, n, L)).real
    return x


GATE_CASES = [
    ([(0, 32, 8, 32), (0, 64, 16, 64)], 256, 1e-3, 60, 11),
    ([(1, 32, 8, 32), (0, 64, 16, 64)], 256, 1e-4, 60, 12),
    ([(1, 16, 4, 32), (2, 32, 8, 32)], 256, 1e-4, 60, 13),   # windows shorter than M: gamma of more bins
]


@pytest.mark.parametrize("dicts,L,eps,K,seed", GATE_CASES)
def test_gamma_gate_matches_truncated_gram(dicts, L, eps, K, seed):
    x = _planted_low_high(dicts, L, seed)
    orcs = {}
    for gate in (False, True):
        orc = O.mp(dicts, x, eps, K=K, flags=O.CONJ_GATE_GAMMA if gate else 0, return_planes=True)
        assert orc.n_atoms >= 20       # K, or the estimate turned negative first
        w, m, n, c, E, rho = T.truncated_gram_mp(dicts, x, eps, orc.n_atoms, gate_gamma=gate)
        assert np.array_equal(orc.w, w) and np.array_equal(orc.m, m) and np.array_equal(orc.n, n), gate
        assert np.max(np.abs(orc.c - c)) <= 1e-12 * np.max(np.abs(c))
        assert np.max(np.abs(orc.E - E)) <= 1e-12 * float(x @ x)
        planes = np.concatenate([p.ravel() for p in orc.planes])
        assert np.max(np.abs(planes - rho)) <= 1e-12 * np.max(np.abs(rho))
        orcs[gate] = (orc, planes)
    # the condition changes the result on these inputs: some selected pair has
    # gamma == 0 while its partner column has surviving entries
    a, b = orcs[False], orcs[True]
    same_seq = np.array_equal(a[0].w, b[0].w) and np.array_equal(a[0].m, b[0].m) and np.array_equal(a[0].n, b[0].n)
    assert not same_seq or np.max(np.abs(a[1] - b[1])) > 1e-6 * np.max(np.abs(a[1]))


def test_gamma_gate_is_inert_where_gamma_never_vanishes():
    # a short Gaussian (narrow in time, broad in frequency): |gamma| exceeds
    # eps at every bin with a partner, so the gated and ungated oracles
    # coincide exactly
    dicts = [(2, 6, 2, 16)]
    L = 128
    D, index = T.dictionary(dicts, L)
    g = np.abs(np.sum(D * D, axis=0))
    assert min(g[i] for i, (_, m, _) in enumerate(index) if 0 < m < 8) > 1e-2
    x = np.random.default_rng(5).standard_normal(L)
    a = O.mp(dicts, x, 1e-3, K=80, return_planes=True)
    b = O.mp(dicts, x, 1e-3, K=80, flags=O.CONJ_GATE_GAMMA, return_planes=True)
    assert a.n_atoms == b.n_atoms > 0
    assert np.array_equal(a.c, b.c) and np.array_equal(a.E, b.E)


@pytest.mark.parametrize("flags", [0, O.CONJ_GATE_GAMMA, O.PEDANTIC])
def test_replay_of_own_sequence_is_the_loop(flags):
    dicts = [(0, 64, 16, 64), (1, 128, 32, 128)]
    x = np.random.default_rng(21).standard_normal(2048)
    r = O.mp(dicts, x, 1e-3, K=400, flags=flags, return_planes=True)
    q = O.mp_replay(dicts, x, 1e-3, r.w, r.m, r.n, flags=flags, return_planes=True)
    assert np.array_equal(q.c, r.c) and np.array_equal(q.E, r.E) and np.array_equal(q.gap, r.gap)
    assert all(np.array_equal(a, b) for a, b in zip(q.planes, r.planes))
    assert np.array_equal(q.best, q.chosen)


def test_replay_any_sequence_at_eps0_is_signal_domain_projection():
    # at eps = 0 the coefficient-domain update is exact for every selection,
    # so a replay along a random list (not the argmax) must equal the
    # signal-domain projections along the same list
    dicts = [(0, 16, 4, 16), (1, 32, 8, 32)]
    L = 128
    x = np.random.default_rng(8).standard_normal(L)
    rng = np.random.default_rng(9)
    seq = []
    for _ in range(40):
        w = int(rng.integers(0, 2))
        d = dicts[w]
        seq.append((w, int(rng.integers(0, d[3] // 2 + 1)), int(rng.integers(0, L // d[2]))))
    w, m, n = (np.array(v) for v in zip(*seq))
    q = O.mp_replay(dicts, x, 0.0, w, m, n, return_planes=True)
    c, E, rho = T.project_sequence(dicts, x, seq)
    E0 = float(x @ x)
    assert np.max(np.abs(q.c - c)) <= 1e-11 * np.max(np.abs(c))
    assert np.max(np.abs(q.E - E)) <= 1e-12 * E0
    planes = np.concatenate([p.ravel() for p in q.planes])
    assert np.max(np.abs(planes - rho)) <= 1e-11 * np.max(np.abs(rho))
    # chosen scores are those of the listed atoms, best the maximum over all
    assert np.all(q.chosen <= q.best * (1 + 1e-15))


def test_replay_rejects_atoms_outside_the_grid():
    dicts = [(0, 16, 4, 16)]
    x = np.ones(64)
    with pytest.raises(RuntimeError):
        O.mp_replay(dicts, x, 1e-4, [0], [9], [0])      # bin above M/2
    with pytest.raises(RuntimeError):
        O.mp_replay(dicts, x, 1e-4, [0], [1], [16])     # frame past N
