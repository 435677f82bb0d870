"""pf_tip_fields, the reduction that allocates nothing (its partials live in
a fixed device array of the library), against pf_tip_state on the same
states: two calls in a row, the second on a smaller lattice, FP32 and FP64,
2D and 3D, with and without a pending frame shift.  Both run the same
reduction kernel with the same launch geometry, so every field must agree
exactly."""
import ctypes as C

import numpy as np
import pytest

from paper_2110_12448_amd import workloads as wl

pytestmark = pytest.mark.gpu

KEYS = ("found", "nonfinite", "index", "x", "y_frame", "z", "solid_fraction")


def _pf():
    from paper_2110_12448_amd import pfiso
    return pfiso


def _compare(s):
    want = s.tip_state()
    got = s.tip_fields()
    print({k: (want[k], got[k]) for k in KEYS}, flush=True)
    for k in KEYS:
        assert got[k] == want[k], (k, got[k], want[k])
    assert got["y_lab"] == got["y_frame"]
    assert got["step"] == 0 and got["frame_shift"] == 0 and got["velocity"] == 0.0


@pytest.mark.parametrize("prec", [0, 1])
def test_matches_tip_state_two_calls(prec):
    pf = _pf()
    big = wl.config_polycrystal_3d(n=40, ny=48, n_grains=4, seed_radius=8.0)
    small = wl.config_small_2d(30.0, n=64)
    for pr, steps in ((big, 15), (small, 40)):
        print("gpu case: pf_tip_fields prec=%d %dx%dx%d" % (prec, pr["nx"], pr["ny"], pr["nz"]),
              flush=True)
        s = pf.Solver(pr, precision=prec)
        s.step(steps)
        _compare(s)
        s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_pending_frame_shift(prec):
    """A moving-frame solve read right after a step that decided to shift (the
    arrays owe one row) and right after one that did not."""
    pf = _pf()
    pr = wl.config_directional_2d(nx=96, ny=64, frame=1, shift_row=12)
    s = pf.Solver(pr, precision=prec)
    seen = set()
    for _ in range(400):
        s.step(1)
        _, pend = s.frame_state()
        if pend not in seen:
            print("pending", pend, flush=True)
            _compare(s)
            seen.add(pend)
        if seen == {0, 1}:
            break
    s.close()
    assert seen == {0, 1}


def test_argument_errors():
    pf = _pf()
    lib = pf.load()
    t = pf.pf_tip()
    assert lib.pf_tip_fields(None, None, 0, 8, 8, 1, 0.8, 0, None, C.byref(t)) == pf.PF_ERR_ARG
    pr = wl.config_small_2d(0.0, n=32)
    s = pf.Solver(pr, precision=pf.PF_F32)
    psi, U = s.device_fields()
    args = [C.c_void_p(psi), C.c_void_p(U)]
    assert lib.pf_tip_fields(*args, 0, 32, 1, 1, 0.8, 0, None, C.byref(t)) == pf.PF_ERR_ARG
    assert lib.pf_tip_fields(*args, 2, 32, 32, 1, 0.8, 0, None, C.byref(t)) == pf.PF_ERR_ARG
    assert lib.pf_tip_fields(*args, 0, 32, 32, 1, 0.8, 2, None, C.byref(t)) == pf.PF_ERR_ARG
    assert lib.pf_tip_fields(*args, 0, 1 << 16, 1 << 15, 1, 0.8, 0, None,
                             C.byref(t)) == pf.PF_ERR_ARG
    s.close()
