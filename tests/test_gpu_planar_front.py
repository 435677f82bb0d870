"""The steady planar directional front on the GPU (the oracle's pin in
test_oracle_planar_front): FP64 fields equal the oracle's, and FP32 fields
keep the closed-form liquid profile U = exp(-V~p zeta / D~) - 1 ahead of the
front, through the C ABI with the moving frame on."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_12448_amd import workloads as wl

pytestmark = pytest.mark.gpu
A2 = 47.0 / 75.0
K, EPS4, D, VP, LT, H_DOMAIN, YF0 = 0.15, 0.02, 2.0, 0.05, 400.0, 320.0, 40.0


def planar_problem(h=0.8, nx=4):
    ny = int(round(H_DOMAIN / h))
    y = np.arange(ny) * h
    psi0 = np.repeat((-(y - YF0) / (1.0 + EPS4))[:, None], nx, axis=1)
    U0 = np.repeat(np.where(y < YF0, 0.0, np.exp(-(y - YF0) * VP / D) - 1.0)[:, None], nx, axis=1)
    return dict(dim=2, nx=nx, ny=ny, nz=1, w=wl.ISO_2D, k=K, eps4=EPS4, D=D, lam=D / A2, h=h,
                dt=wl.stable_dt(2, h, D), Vp=VP, lT=LT, y0=YF0, bc=(oracle.PERIODIC, oracle.NOFLUX,
                                                                  oracle.NOFLUX),
                frame=1, shift_row=int(round(YF0 / h)) + 2, rot=wl.rotation_2d(0.0)[None],
                psi0=psi0, U0=U0, grain=np.zeros(psi0.shape, dtype=np.int8), antitrapping=0,
                two_point=0, dynamic_grains=0)


def front_and_profile(pr, psi, U, shift):
    h = pr["h"]
    col = np.tanh(psi[:, 0] / math.sqrt(2.0))
    j = np.nonzero((col[:-1] >= 0) & (col[1:] < 0))[0][0]
    y_front = (j + col[j] / (col[j] - col[j + 1]) + shift) * h
    y_lab = (np.arange(pr["ny"]) + shift) * h
    ahead = (y_lab - y_front >= 5.0) & (y_lab - y_front <= 120.0)
    closed = np.exp(-(y_lab - y_front) * VP / D) - 1.0
    return y_front, float(np.max(np.abs(U[ahead, 0] - closed[ahead])))


@pytest.mark.parametrize("prec", [1, 0])
def test_planar_front_gpu(prec):
    from paper_2110_12448_amd import pfiso
    pr = planar_problem()
    n = int(round(400.0 / pr["dt"]))
    print("gpu case: planar front prec=%d steps=%d" % (prec, n), flush=True)
    s = pfiso.Solver(pr, precision=prec)
    s.step(n)
    phi, U, psi, _ = s.read_fields()
    shift, _ = s.frame_state()
    s.close()
    p = oracle.Params.from_problem(pr)
    opsi, oU, st = oracle.step(p, pr["psi0"], pr["U0"], None, n)
    assert shift == st.shift
    if prec == 1:
        assert np.max(np.abs(U - oU)) <= 1e-10 and np.max(np.abs(psi - opsi)) <= 1e-9
    y_front, err = front_and_profile(pr, psi, U, shift)
    assert err <= 2e-3, err
    assert abs(y_front - YF0 - VP * n * pr["dt"]) <= 0.25
