"""Textbook matching pursuit in the signal domain (numpy, tiny signals only).

TEST INFRASTRUCTURE ONLY.  Every iteration recomputes all inner products of the
residual with every atom of the reduced multi-Gabor dictionary from explicitly
built atoms, selects the largest |<r, d_p>| (Sec. 2.2, non-pedantic selection
of Sec. 5), and subtracts the least-squares projection onto the real atom pair
{d, conj d} (Sec. 5, the pair treatment of real signals).  No Gram matrix, no
kernel and no truncation is involved, so with a zero kernel threshold the
coefficient-domain oracle must reproduce this sequence exactly.
"""
import numpy as np


def _window(win: int, gl: int, a: int, M: int) -> np.ndarray:
    # independent restatement of the centred windows, unit 2-norm
    t = np.arange(gl) - gl // 2
    if win == 0:
        g = 0.42 + 0.5 * np.cos(2 * np.pi * t / gl) + 0.08 * np.cos(4 * np.pi * t / gl)
    elif win == 1:
        g = 0.5 + 0.5 * np.cos(2 * np.pi * t / gl)
    elif win == 2:
        g = np.exp(-np.pi * t.astype(np.float64) ** 2 / (a * M))
    else:
        raise ValueError(win)
    return g / np.linalg.norm(g)


def atom(d, m: int, n: int, L: int) -> np.ndarray:
    """d_{m,n}(l) = g(l - n a) exp(2 pi i m (l - n a) / M), circular in l (Eq. gabdict)."""
    win, gl, a, M = d
    g = _window(win, gl, a, M)
    out = np.zeros(L, np.complex128)
    t = np.arange(-gl // 2, gl // 2)
    l = (n * a + t) % L
    ph = np.exp(2j * np.pi * ((m * t) % M) / M)
    np.add.at(out, l, g * ph)
    return out


def dictionary(dicts, L: int):
    """All reduced atoms as columns, in global index order p = off_w + n*(M_w/2+1) + m."""
    cols, index = [], []
    for w, d in enumerate(dicts):
        a, M = d[2], d[3]
        for n in range(L // a):
            for m in range(M // 2 + 1):
                cols.append(atom(d, m, n, L))
                index.append((w, m, n))
    return np.stack(cols, axis=1), index


def _pair_projection_energy(D, index, dicts, r):
    """||P r||^2 for the projection of the real residual onto each atom's real
    pair span{Re d, Im d} (span{d} at DC and Nyquist), by least squares per
    atom: the criterion of pedantic selection (Sec. 5)."""
    out = np.zeros(D.shape[1])
    for p, (w, m, n) in enumerate(index):
        d = D[:, p]
        M = dicts[w][3]
        A = d.real[:, None] if (m == 0 or 2 * m == M) else np.stack([d.real, d.imag], axis=1)
        sol, *_ = np.linalg.lstsq(A, r, rcond=None)
        u = A @ sol
        out[p] = float(u @ u)
    return out


def mp(dicts, x: np.ndarray, n_iter: int, stop_rel: float = 0.0, pedantic: bool = False):
    """Returns (w, m, n, c, E) with E[k] = ||r_{k+1}||^2 after each selection.
    pedantic: select the atom whose pair projection removes the most energy
    instead of the largest |<r, d>|."""
    x = np.asarray(x, np.float64)
    L = len(x)
    D, index = dictionary(dicts, L)
    r = x.copy()
    E0 = float(r @ r)
    ws, ms, ns, cs, Es = [], [], [], [], []
    for _ in range(n_iter):
        rho = D.conj().T @ r
        mag = _pair_projection_energy(D, index, dicts, r) if pedantic else rho.real ** 2 + rho.imag ** 2
        p = int(np.argmax(mag))
        w, m, n = index[p]
        M = dicts[w][3]
        d = D[:, p]
        if m == 0 or 2 * m == M:
            c = rho[p]
            r = r - (c * d).real
        else:
            A = np.stack([d, d.conj()], axis=1)
            sol, *_ = np.linalg.lstsq(A, r.astype(np.complex128), rcond=None)
            c = sol[0]
            r = r - (A @ sol).real
        ws.append(w)
        ms.append(m)
        ns.append(n)
        cs.append(c)
        Es.append(float(r @ r))
        if Es[-1] <= stop_rel * E0:
            break
    return (np.array(ws), np.array(ms), np.array(ns), np.array(cs), np.array(Es))


def project_sequence(dicts, x: np.ndarray, seq):
    """Signal-domain MP along a given selection list seq = [(w, m, n), ...]
    (no selection rule): each step subtracts the least-squares projection of
    the real residual onto the atom's real pair (span{d} at DC and Nyquist).
    Returns (c, E, rho) with E[k] = ||r_{k+1}||^2 and rho = D* r after the
    last step, in global index order."""
    x = np.asarray(x, np.float64)
    L = len(x)
    D, index = dictionary(dicts, L)
    pos = {t: i for i, t in enumerate(index)}
    r = x.copy()
    cs, Es = [], []
    for (w, m, n) in seq:
        d = D[:, pos[(w, m, n)]]
        M = dicts[w][3]
        if m == 0 or 2 * m == M:
            c = np.vdot(d, r)       # <r, d>
            r = r - (c * d).real
        else:
            A = np.stack([d, d.conj()], axis=1)
            sol, *_ = np.linalg.lstsq(A, r.astype(np.complex128), rcond=None)
            c = sol[0]
            r = r - (A @ sol).real
        cs.append(c)
        Es.append(float(r @ r))
    return np.array(cs), np.array(Es), D.conj().T @ r


def truncated_gram_mp(dicts, x: np.ndarray, eps: float, n_iter: int, gate_gamma: bool):
    """Approximate coefficient-domain MP written with the Gram matrix of the
    explicitly built reduced dictionary instead of kernels (Eq. approxResDef
    with the truncated Gram matrix of Eq. truncgram, the real-atom pairs of
    Sec. 5 and the pair update of Alg. 3).  G[p, q] = <d_q, d_p> and, for the
    conjugate partner, Gc[p, q] = <conj d_q, d_p>; both are truncated entry by
    entry (|.| > eps).  gamma(q) = <d_q, conj d_q>, truncated the same way.
    gate_gamma: the partner term is applied only when gamma != 0 (the literal
    condition of Alg. 3); otherwise wherever Gc is nonzero.
    Returns (w, m, n, c, E, rho_final)."""
    x = np.asarray(x, np.float64)
    L = len(x)
    D, index = dictionary(dicts, L)
    G = D.conj().T @ D                      # G[p, q] = sum_l d_q(l) conj(d_p(l))
    Gc = D.conj().T @ D.conj()              # Gc[p, q] = sum_l conj(d_q(l)) conj(d_p(l))
    G = np.where(np.abs(G) > eps, G, 0)
    Gc = np.where(np.abs(Gc) > eps, Gc, 0)
    gam = np.sum(D * D, axis=0)             # <d_q, conj d_q>
    gam = np.where(np.abs(gam) > eps, gam, 0)
    rho = D.conj().T @ x
    E = float(x @ x)
    ws, ms, ns, cs, Es = [], [], [], [], []
    for _ in range(n_iter):
        s = rho.real ** 2 + rho.imag ** 2
        p = int(np.argmax(s))
        w, m, n = index[p]
        M = dicts[w][3]
        pair = not (m == 0 or 2 * m == M)
        if pair:
            g = gam[p]
            c = (rho[p] - np.conj(g) * np.conj(rho[p])) / (1.0 - abs(g) ** 2)
            Et = 2.0 * (abs(c) ** 2 + (g * c * c).real)
        else:
            c = rho[p]
            Et = abs(c) ** 2
        E -= Et
        upd = c * G[:, p]
        if pair and (not gate_gamma or gam[p] != 0):
            upd = upd + np.conj(c) * Gc[:, p]
        rho = rho - upd
        ws.append(w)
        ms.append(m)
        ns.append(n)
        cs.append(c)
        Es.append(E)
    return np.array(ws), np.array(ms), np.array(ns), np.array(cs), np.array(Es), rho
