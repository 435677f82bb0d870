"""GPU parity at the ends of the parameter ranges pf_create accepts: no
anisotropy (eps4 = 0, where a_s = 1 and the torque vanishes; Eq.
anis_function) and eps4 just below 1/15, and partition coefficients near 0
and near 1 (k enters F~1 of Eq. Thermal_F1, the anti-trapping prefactor
1 + (1 - k) U and the U denominator 1 + k - (1 - k) phi of Eq. PF_b).  Frozen
gradient, 40 steps, against the oracle: FP64 within 1e-10, FP32 within 1e-5."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_12448_amd import workloads as wl

pytestmark = pytest.mark.gpu
SQ2 = math.sqrt(2.0)
TOL = {0: 1e-5, 1: 1e-10}


def _pf():
    from paper_2110_12448_amd import pfiso
    return pfiso


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("eps4,k", [(0.0, 0.15), (0.066, 0.15), (0.02, 0.01), (0.02, 0.99)])
def test_parameter_limits(dim, prec, eps4, k):
    if dim == 2:
        pr = wl.problem(2, (70, 48), eps4=eps4, k=k, alpha0_deg=25.0, seed_radius=9.0,
                        y_front=12.0, seed=21)
    else:
        rot = wl.random_rotations(7, 3)
        rng = np.random.default_rng(5)
        grain = rng.integers(0, 3, size=(18, 24, 20)).astype(np.int8)
        pr = wl.problem(3, (20, 24, 18), eps4=eps4, k=k, rot=rot, grain=grain, seed_radius=6.0,
                        y_front=8.0, seed=22)
    pf = _pf()
    print("gpu case: limits dim=%d prec=%d eps4=%g k=%g" % (dim, prec, eps4, k), flush=True)
    s = pf.Solver(pr, precision=prec)
    s.step(40)
    phi, U, _, _ = s.read_fields()
    s.close()
    p = oracle.Params.from_problem(pr)
    opsi, oU, st = oracle.step(p, pr["psi0"], pr["U0"], pr["grain"], 40)
    assert st.nonfinite == 0
    d = max(float(np.max(np.abs(phi - np.tanh(opsi / SQ2)))), float(np.max(np.abs(U - oU))))
    print("max diff %.3e" % d)
    assert d <= TOL[prec]
