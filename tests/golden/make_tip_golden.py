"""Writes the oracle's tip after 10^4 steps, in FP64 and with the stored
fields rounded to FP32 after every step:
  tip_small_2d_10k.json: the 128 x 128 workload (moving frame at row 64),
    alpha0 = 0 and 30 deg;
  tip_small_3d_10k.json: a 16 x 48 x 16 polycrystal of the 256^3 recipe
    (4 Voronoi grains, uniform random orientations, planar slab, frozen
    gradient, periodic x and z), moving frame at row 16, with a thermal
    length of 6000 W so that F1 of Eq. Thermal_F1 stays above 1/D~ while the
    frame moves (the time step stays within its limit for the whole run).
Calls only the oracle and the seeded input generator.  Usage:
make_tip_golden.py [2d|3d|all] (default all)."""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2110_12448_amd import workloads as wl  # noqa: E402

NSTEPS = 10000
PROBLEM_3D = dict(n=16, ny=48, n_grains=4, seed=3, frame=1, shift_row=16, lT=6000.0)


def _case(pr, r32, extra):
    p = oracle.Params.from_problem(pr, round_f32=r32)
    psi, U, st = oracle.step(p, pr["psi0"], pr["U0"], pr["grain"], NSTEPS)
    phi = np.tanh(psi / math.sqrt(2.0))
    t = oracle.tip(p, phi)
    case = dict(extra)
    case.update({"round_f32": r32, "shift": st.shift, "x": t["x"], "y_frame": t["y"],
                 "y_lab": t["y"] + st.shift * p.h, "solid_fraction": oracle.solid_fraction(p, phi)})
    if pr["dim"] == 3:
        case["z"] = t["z"]
    if p.lT > 0:
        # F1 over the lattice for the shift and time reached: the run must stay
        # within the explicit limit h^2 / (2 dim max(D~, 1/F1))
        off = st.shift * p.h - p.y0 - p.Vp * NSTEPS * p.dt
        f1 = min(1.0 - (1.0 - p.k) * off / p.lT,
                 1.0 - (1.0 - p.k) * ((p.ny - 1) * p.h + off) / p.lT)
        case["F1_min_end"] = f1
        assert p.dt <= p.h ** 2 / (2 * pr["dim"] * max(p.D, 1.0 / f1)), f1
    print(case, flush=True)
    return case


def main2d():
    out = {"_about": "Oracle tip after 10^4 steps of the 128 x 128 workload (moving frame at "
                     "row 64), alpha0 = 0 and 30 deg, FP64 and with the stored fields rounded "
                     "to FP32 after every step (tests/golden/make_tip_golden.py 2d).",
           "nsteps": NSTEPS, "cases": []}
    for a0 in (0.0, 30.0):
        for r32 in (0, 1):
            pr = wl.config_small_2d(a0, frame=1, shift_row=64)
            out["cases"].append(_case(pr, r32, {"alpha0_deg": a0}))
    with open(os.path.join(HERE, "tip_small_2d_10k.json"), "w") as f:
        json.dump(out, f, indent=1)


def main3d():
    out = {"_about": "Oracle tip after 10^4 steps of a 16 x 48 x 16 polycrystal (4 Voronoi "
                     "grains, planar slab, frozen gradient with lT = 6000 W, moving frame at "
                     "row 16), FP64 and with the stored fields rounded to FP32 after every step "
                     "(tests/golden/make_tip_golden.py 3d).",
           "nsteps": NSTEPS, "problem": PROBLEM_3D, "cases": []}
    for r32 in (0, 1):
        pr = wl.config_polycrystal_3d(**PROBLEM_3D)
        out["cases"].append(_case(pr, r32, {}))
    with open(os.path.join(HERE, "tip_small_3d_10k.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("2d", "all"):
        main2d()
    if which in ("3d", "all"):
        main3d()
