"""Writes c5_sig0_oracle_20k.npz: the FP64 oracle's first 20000 selections on
signal 0 of the large five-system workload (2^22 samples, Blackman systems
128 .. 32768 taps, a = gl/4, M = gl, threshold 1e-4; the signal rounded to
FP32 as the GPU path receives it).  The oracle needs about two minutes for
this, too long for a GPU test, so the test reads the stored result.

Calls only the oracle and the seeded input module:
    python tests/golden/make_c5_oracle_reference.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import core as O  # noqa: E402
from paper_2202_12380_amd import signals as S  # noqa: E402

K = 20000


def main():
    wl = S.workload(5)
    x = S.signals(5, batch=1)[0].astype(np.float32).astype(np.float64)
    r = O.mp(wl.dicts, x, wl.eps, K=K)
    out = os.path.join(HERE, "c5_sig0_oracle_20k.npz")
    np.savez_compressed(out, w=r.w.astype(np.int32), m=r.m.astype(np.int32), n=r.n.astype(np.int32),
                        E=r.E.astype(np.float64), gap=r.gap.astype(np.float32),
                        E0=np.float64(r.E0), L_padded=np.int64(r.L_padded), eps=np.float64(wl.eps),
                        dicts=np.array(wl.dicts, np.int32), K=np.int64(K))
    print(out, r.n_atoms)


if __name__ == "__main__":
    main()
