"""Writes the expected moments of the crossing-beams-plus-shadow workload
(Sec. 4.1.1 crossing beams, Sec. 4.2.1 shadow) scaled to 64^3 cells with
the 110-direction Lebedev rule, after its full 500 steps from zero, by the
FP64 oracle.  The GPU tests compare FP32, BF16 and FP16 storage runs of the
same workload against this file.

Calls only the oracle and the seeded workload generators:

    python tests/golden/make_beams_golden.py        # ~5 minutes on one core

Output: tests/golden/beams64_500.npz with E [z, y, x] and F [3, z, y, x]
(float64) and the workload parameters.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import lbrt_oracle as orc  # noqa: E402

N, STEPS = 64, 500
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"beams{N}_{STEPS}.npz")


def main():
    prob = wl.beams(n=N, steps=STEPS)
    t0 = time.time()

    def progress(k, I):
        if k % 50 == 0:
            print(f"step {k}: sum E {I.sum():.12e} ({time.time() - t0:.0f} s)", flush=True)

    I = orc.run(prob, callback=progress)
    E, F = orc.moments(I, prob.dirs)
    np.savez_compressed(OUT, E=E, F=F, n=N, steps=STEPS, npoints=prob.ndir, dt=prob.dt,
                        seed=3)
    print(f"wrote {OUT}: sum E {E.sum():.15e}, max E {E.max():.6e} "
          f"({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
