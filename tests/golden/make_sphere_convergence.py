"""Convergence of the FP64 oracle on the homogeneous radiating sphere
(Sec. 4.2.2) towards its analytic solution, at two resolutions of the same
physical setup: kappa R = 80, eta = kappa (B = 1), 50-direction Lebedev
rule, dt = dx / 2, t = 100 R / 16 (steady state):

    32^3 cells, R = 8,  kappa = 10, 100 steps,
    64^3 cells, R = 16, kappa = 5,  200 steps.

For each radial band (in units of R) it records the relative error of the
shell-averaged E against the analytic shell average, and the far-field
fall-off between the shells 10/8 R and 15/8 R.  The oracle's CPU pin
(test_sphere_reaches_analytic_profile) takes its tolerances from the 32^3
errors of this file and checks that they shrink at 64^3 where the error is
discretisation-limited (the staircase sphere, the 50-point rule's ray
effects and the interpolation's diffusion all shrink with the cell size).

Calls only the oracle, the analytic module and the seeded workloads:

    python tests/golden/make_sphere_convergence.py     # ~4 minutes on one core

Output: tests/golden/sphere_convergence.json.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import analytic  # noqa: E402
from oracle import lbrt_oracle as orc  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere_convergence.json")
# radial bands in units of R: the interior, the rim, just inside, the far field
BANDS = [(0.0, 3 / 8), (3 / 8, 5 / 8), (5 / 8, 6 / 8), (10 / 8, 2.0)]


def sphere_errors(n: int) -> dict:
    R = n / 4.0
    kappa = 80.0 / R
    p = wl.sphere(n=n, radius=R, kappa=kappa, steps=int(round(100 * n / 32)))
    t0 = time.time()
    I = orc.run(p)
    E = I.sum(axis=0)
    c = np.arange(n) + 0.5 - n / 2
    r = np.sqrt(c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2)
    r2 = np.round(r ** 2, 6)
    uniq, inv = np.unique(r2, return_inverse=True)
    Ea = np.array([analytic.sphere_moments(np.sqrt(u), R, kappa)[0] for u in uniq])
    Ea = Ea[inv].reshape(r.shape)
    bands = []
    for lo, hi in BANDS:
        m = (r >= lo * R) & (r < hi * R)
        bands.append(float(abs(E[m].mean() / Ea[m].mean() - 1)))
    m1 = (r >= 10 / 8 * R) & (r < 11 / 8 * R)
    m2 = (r >= 15 / 8 * R) & (r < 16 / 8 * R)
    fall = float(abs((E[m2].mean() / E[m1].mean()) / (Ea[m2].mean() / Ea[m1].mean()) - 1))
    centre = float(abs(E[n // 2 - 1, n // 2 - 1, n // 2 - 1] - 1.0))
    print(f"n = {n}: bands {bands}, fall-off {fall:.3e}, centre {centre:.1e} "
          f"({time.time() - t0:.0f} s)", flush=True)
    return {"n": n, "R": R, "kappa": kappa, "steps": p.steps, "band_rel_err": bands,
            "falloff_rel_err": fall, "centre_abs_err": centre}


def main():
    res = {"bands_in_R": BANDS, "runs": [sphere_errors(32), sphere_errors(64)]}
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
