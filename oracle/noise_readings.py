"""Convergence on white noise under readings of the paper (Sec. 6.1, Fig. 4).

The paper runs three Blackman systems (M = 512/1024/2048, a = M/4) on
6.04e6 samples of Gaussian noise until the error estimate turns negative, at
four thresholds, and prints the steps and the final SNR.  This script runs
the FP64 oracle on a shorter seeded noise signal (the counts scale with the
length: steps per sample and the final SNR are what compare) under each
reading of a point the paper leaves open, and prints a markdown table:

  default   absolute threshold |h| > eps, entry by entry, partner term wherever
            the truncated Gram entry is nonzero;
  gate      the partner term only when gamma != 0 (the literal Alg. 3);
  rel       threshold relative to each kernel's peak (the library's parameter
            name, "kernrelthr", and the kernel figure's caption);
  box       every entry of the survivors' bounding box kept (the kernel as a
            box of "fixed size and shape");
  pedantic  selection by the pair projection energy;
  gate+rel  both.

Test infrastructure (calls only the oracle and the seeded input module):
    python -m oracle.noise_readings [log2_length] [processes]
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import core as O  # noqa: E402

DICTS = [(0, 512, 128, 512), (0, 1024, 256, 1024), (0, 2048, 512, 2048)]
EPS = (1e-4, 1e-3, 5e-3, 1e-2)
READINGS = {"default": 0, "gate": O.CONJ_GATE_GAMMA, "rel": O.THR_REL, "box": O.KEEP_BOX,
            "pedantic": O.PEDANTIC, "gate+rel": O.CONJ_GATE_GAMMA | O.THR_REL}


def _run(job):
    L, eps, name = job
    x = np.random.Generator(np.random.PCG64(np.random.SeedSequence([6, 1, L]))).standard_normal(L)
    t0 = time.perf_counter()
    r = O.mp(DICTS, x, eps, K=1 << 24, flags=READINGS[name], cap=4 * L)
    y = O.resynth(DICTS, r.L_padded, r.w, r.m, r.n, r.c)
    e = float(np.sum((x - y[:L]) ** 2) + np.sum(y[L:] ** 2))
    return dict(eps=eps, reading=name, L=L, steps=int(r.n_atoms), stop=int(r.stop_reason),
                steps_per_sample=r.n_atoms / L, true_snr_db=10 * np.log10(r.E0 / e),
                seconds=time.perf_counter() - t0)


def main():
    L = 1 << (int(sys.argv[1]) if len(sys.argv) > 1 else 17)
    procs = int(sys.argv[2]) if len(sys.argv) > 2 else min(8, os.cpu_count() or 1)
    gold = json.load(open(os.path.join(os.path.dirname(HERE), "tests", "golden", "fig4_noise_convergence.json")))
    paper = {r["eps"]: r for r in gold["runs"]}
    jobs = [(L, e, n) for e in EPS for n in READINGS]
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_run, jobs, chunksize=1)
    print("| eps | reading | steps / sample | true SNR (dB) | paper steps / sample | paper SNR (dB) |")
    print("|---|---|---|---|---|---|")
    for r in res:
        p = paper[r["eps"]]
        print("| %g | %s | %.3f | %.2f | %.3f | %.2f |" % (r["eps"], r["reading"], r["steps_per_sample"],
                                                        r["true_snr_db"], p["steps"] / gold["L"], p["snr_db"]))
    print("signal: %d samples of seeded N(0,1) noise; every run stopped on %s" % (
        L, sorted({r["stop"] for r in res})))


if __name__ == "__main__":
    main()
