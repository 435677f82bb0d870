"""GPU parity of the 3D fused step (through the C ABI) against the FP64 CPU
oracle on identical seeded inputs."""
import functools
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2110_12448_amd import workloads as wl

pytestmark = pytest.mark.gpu
SQ2 = math.sqrt(2.0)
TOL_F64 = 1e-10
TOL_F32 = 1e-5


def _pf():
    from paper_2110_12448_amd import pfiso
    return pfiso


def run_gpu(pr, precision, nsteps, tune=None, chunks=1):
    pf = _pf()
    print("gpu case: 3D %s prec=%d steps=%d tune=%s" % ((pr["nx"], pr["ny"], pr["nz"]),
                                                       precision, nsteps, tune), flush=True)
    s = pf.Solver(pr, precision=precision)
    if tune is not None:
        s.tune(*tune)
    for _ in range(chunks):
        s.step(nsteps // chunks)
    phi, U, psi, g = s.read_fields()
    tip = s.tip_state()
    shift = s.frame_state()
    s.close()
    return phi, U, psi, tip, shift


HERE = os.path.dirname(os.path.abspath(__file__))


@functools.lru_cache(maxsize=4)
def _oracle_c3(n, nsteps, ny=None):
    pr = wl.config_polycrystal_3d(n=n, ny=ny)
    p = oracle.Params.from_problem(pr)
    psi, U, st = oracle.step(p, pr["psi0"], pr["U0"], pr["grain"], nsteps)
    return pr, np.tanh(psi / SQ2), U, st, p


def run_oracle(pr, nsteps, **over):
    p = oracle.Params.from_problem(pr, **over)
    psi, U, st = oracle.step(p, pr["psi0"], pr["U0"], pr["grain"], nsteps)
    return np.tanh(psi / SQ2), U, psi, st, p


def _cmp(a, b):
    return float(np.max(np.abs(a - b)))


def _poly(n, ny=None, n_grains=3, seed=3, **kw):
    return wl.config_polycrystal_3d(n=n, ny=ny, n_grains=n_grains, seed=seed, **kw)


@pytest.mark.parametrize("prec", [1, 0])
def test_polycrystal_small(prec):
    """24^3 (x, z periodic, y no-flux), 3 Voronoi grains with random cubic
    orientations, frozen gradient, planar slab with noise: 30 steps."""
    pr = _poly(24, seed_radius=8.0)
    ophi, oU, _, st, p = run_oracle(pr, 30)
    phi, U, psi, tip, _ = run_gpu(pr, prec, 30)
    d = max(_cmp(phi, ophi), _cmp(U, oU))
    print("max diff %.3e" % d)
    assert d <= (TOL_F64 if prec == 1 else TOL_F32)
    ot = oracle.tip(p, ophi)
    assert tip["found"] and abs(tip["y_frame"] - ot["y"]) <= (1e-9 if prec == 1 else 1e-3)
    assert tip["solid_fraction"] == pytest.approx(oracle.solid_fraction(p, ophi),
                                                  abs=1e-12 if prec == 1 else 1e-6)


EDGE3 = [
    # (shape (nx, ny, nz), bc, thermal, weights, grains, tune (seg, ztile) or None)
    ((61, 19, 13), (0, 0, 0), "isothermal", wl.ISO_3D, 1, None),
    ((70, 24, 9), (1, 1, 1), "isothermal", wl.ISO_3D, 2, (8, 3)),
    ((20, 30, 17), (1, 0, 0), "frozen", wl.STD_3D, 2, (4, 1)),
    ((16, 16, 16), (0, 0, 0), "isothermal", wl.ISO_3D_441, 1, None),
    ((33, 21, 11), (0, 1, 1), "frozen", wl.ISO_3D, 3, (16, 8)),
    ((4, 12, 5), (1, 0, 1), "isothermal", wl.ISO_3D, 1, (4, 2)),
    # <111>-shell schemes: S-bar_{4,4,1} (periodic, ragged tiles, grains) and
    # the weights (2/3, 0, 1/3) of the <100> + <111> combination
    ((45, 20, 14), (1, 1, 1), "isothermal", wl.ISO_3D_441, 3, (8, 4)),
    ((30, 18, 10), (0, 0, 0), "frozen", (2.0 / 3.0, 0.0, 1.0 / 3.0), 2, (5, 3)),
    # 16-wave workgroups with a ragged last z tile (14 + 3 rows)
    ((50, 22, 17), (1, 0, 0), "frozen", wl.ISO_3D, 2, (8, 14)),
    # no-flux walls in every direction with 4-row segments, with and without
    # <111> links: the first link row of the bottom segment lies below the
    # y wall, and every segment start reads rows of the one below
    ((24, 21, 12), (0, 0, 0), "frozen", wl.ISO_3D_441, 2, (4, 3)),
    ((26, 19, 13), (0, 0, 0), "frozen", wl.ISO_3D, 3, (4, 5)),
]


@pytest.mark.parametrize("case", range(len(EDGE3)))
@pytest.mark.parametrize("prec", [1, 0])
def test_edge_cases_3d(case, prec):
    shape, bc, thermal, w, ng, tune = EDGE3[case]
    if prec == 1 and tune is not None and tune[1] > 6:
        tune = (tune[0], 6)               # FP64 tiles are at most 6 z rows
    nx, ny, nz = shape
    rng = np.random.default_rng(20 + case)
    rot = wl.random_rotations(30 + case, ng)
    grain = rng.integers(0, ng, size=(nz, ny, nx)).astype(np.int8) if ng > 1 else None
    pr = wl.problem(3, shape, thermal=thermal, bc=bc, rot=rot, grain=grain, eps4=0.04,
                    seed_radius=min(shape) / 5.0, y_front=(ny // 2) * 0.8, noise=0.02,
                    seed=40 + case)
    pr["w"] = tuple(w)
    ophi, oU, _, st, p = run_oracle(pr, 20)
    assert st.nonfinite == 0
    phi, U, psi, tip, _ = run_gpu(pr, prec, 20, tune=tune)
    d = max(_cmp(phi, ophi), _cmp(U, oU))
    print("max diff %.3e" % d)
    assert d <= (TOL_F64 if prec == 1 else TOL_F32)


@pytest.mark.parametrize("prec", [1, 0])
def test_moving_frame_3d(prec):
    """Moving frame in 3D over 100 steps (8 shifts; the oracle's tip stays at
    least 5e-3 W from the shift threshold at every decision, so FP32 decides
    as FP64 does)."""
    pr = _poly(20, ny=32, n_grains=2, frame=1, shift_row=8, seed_radius=6.0)
    ophi, oU, _, st, p = run_oracle(pr, 100)
    phi, U, psi, tip, (shift, pend) = run_gpu(pr, prec, 100)
    assert st.shift >= 5 and shift == st.shift
    d = max(_cmp(phi, ophi), _cmp(U, oU))
    print("max diff %.3e" % d)
    assert d <= (TOL_F64 if prec == 1 else TOL_F32)


@pytest.mark.parametrize("prec", [1, 0])
def test_polycrystal_c3_recipe_100_steps(prec):
    """The 256^3 polycrystal's recipe (8 Voronoi grains with uniform random
    orientations, planar slab, frozen gradient, periodic x and z,
    S-bar_{1,2,0}) for the 100 steps of the parity gate, on a 76 x 64 x 76
    lattice tiled as the benchmark tiles 256^3 (86-row segments of 14-row
    workgroups): strips of 60 columns plus a thin strip of 16 in three lane
    groups of 21, three segments of 21-22 rows (the thin strip four shorter
    ones), 14-row workgroups with a partial last z tile in FP32 (6 rows in
    FP64, the most its workgroups hold).  Every cell against the oracle, and
    the tip and solid fraction."""
    pr, ophi, oU, st, p = _oracle_c3(76, 100, ny=64)
    tune = (22, 14) if prec == 0 else (22, 6)
    phi, U, psi, tip, _ = run_gpu(pr, prec, 100, tune=tune)
    d = max(_cmp(phi, ophi), _cmp(U, oU))
    print("max diff %.3e" % d)
    assert d <= (TOL_F64 if prec == 1 else TOL_F32)
    ot = oracle.tip(p, ophi)
    assert tip["found"] and abs(tip["y_frame"] - ot["y"]) <= (1e-9 if prec == 1 else 1e-3)
    assert tip["solid_fraction"] == pytest.approx(oracle.solid_fraction(p, ophi),
                                                  abs=1e-12 if prec == 1 else 1e-6)


def test_tip_golden_3d_10k():
    """Tip of a small polycrystal in the moving frame after 10^4 steps within
    0.05 W of the oracle's, FP64 and FP32 (oracle values stored by
    tests/golden/make_tip_golden.py, FP32 against the oracle that rounds its
    stored fields to FP32 after every step)."""
    gold = json.load(open(os.path.join(HERE, "golden", "tip_small_3d_10k.json")))
    pf = _pf()
    for case in gold["cases"]:
        prec = pf.PF_F64 if case["round_f32"] == 0 else pf.PF_F32
        pr = wl.config_polycrystal_3d(**gold["problem"])
        print("gpu case: 3D tip golden prec=%d steps=%d" % (prec, gold["nsteps"]), flush=True)
        s = pf.Solver(pr, precision=prec)
        s.step(gold["nsteps"])
        t = s.tip_state()
        s.close()
        print(case, {k: t[k] for k in ("x", "z", "y_lab", "frame_shift", "solid_fraction")})
        assert t["frame_shift"] >= 100
        assert abs(t["y_lab"] - case["y_lab"]) <= 0.05
        # the oracle's own FP64 and FP32-rounded runs differ by 2.2e-4 in solid
        # fraction after 10^4 steps
        assert abs(t["solid_fraction"] - case["solid_fraction"]) <= (1e-6 if prec == pf.PF_F64
                                                                      else 1e-3)


@pytest.mark.parametrize("w", [wl.ISO_3D, wl.ISO_3D_441])
@pytest.mark.parametrize("n", [40, 76, 64])
def test_tiles_do_not_change_results_fp32(w, n):
    """Bitwise identical fields for every launch geometry.  n = 40: one strip
    of 40 columns; 76: a strip of 60 and a thin strip of 16 columns in 3 lane
    groups per wave; 64: a strip of 60 and a thin strip of 4 in 4 groups."""
    pr = _poly(n, ny=36, n_grains=4, seed_radius=10.0)
    pr["w"] = tuple(w)
    ref = run_gpu(pr, 0, 12, tune=(16, 6))
    for tune in ((4, 1), (8, 3), (32, 8), (12, 5), (16, 14), (8, 11), (24, 10), (36, 14)):
        out = run_gpu(pr, 0, 12, tune=tune)
        assert np.array_equal(out[2], ref[2]) and np.array_equal(out[1], ref[1]), tune
    ophi, oU, _, st, p = run_oracle(pr, 12)
    assert max(_cmp(ref[0], ophi), _cmp(ref[1], oU)) <= TOL_F32


def test_polycrystal_full_size_fp32():
    """256^3, 8 grains, FP32, in the benchmark's launch configuration: every
    cell after 2 steps against the oracle."""
    pr = wl.config_polycrystal_3d()
    ophi, oU, _, st, p = run_oracle(pr, 2)
    phi, U, psi, tip, _ = run_gpu(pr, 0, 2)
    assert max(_cmp(phi, ophi), _cmp(U, oU)) <= TOL_F32


def test_polycrystal_441_size_fp32():
    """S-bar_{4,4,1} (the 27-point <111> scheme) on a 128^3 polycrystal: every
    cell after 3 steps against the oracle."""
    pr = wl.config_polycrystal_3d(n=128, scheme="iso441")
    ophi, oU, _, st, p = run_oracle(pr, 3)
    phi, U, psi, tip, _ = run_gpu(pr, 0, 3)
    assert max(_cmp(phi, ophi), _cmp(U, oU)) <= TOL_F32


def test_polycrystal_full_run_fp32_vs_fp64():
    """The 256^3 polycrystal for the 5000 steps of its workload: the FP32 tip
    within 0.05 W of the FP64 one and the solid fractions within 1e-4 (the
    FP64 GPU path stands in for the oracle, as in the 2D full-run test)."""
    pf = _pf()
    pr = wl.config_polycrystal_3d()
    out = {}
    for prec in (pf.PF_F64, pf.PF_F32):
        print("gpu case: 256^3 polycrystal prec=%d steps=5000" % prec, flush=True)
        s = pf.Solver(pr, precision=prec)
        for _ in range(5):
            s.step(1000)
            s.synchronize()
        out[prec] = s.tip_state()
        s.close()
    t64, t32 = out[pf.PF_F64], out[pf.PF_F32]
    print({k: (t64[k], t32[k]) for k in ("y_lab", "x", "z", "solid_fraction")})
    assert t64["found"] and abs(t32["y_lab"] - t64["y_lab"]) <= 0.05
    assert abs(t32["solid_fraction"] - t64["solid_fraction"]) <= 1e-4
