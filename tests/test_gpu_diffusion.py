"""GPU parity of the diffusion-only step (pf_step_diffusion) against the oracle
in frozen-psi mode, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_12448_amd import workloads as wl

pytestmark = pytest.mark.gpu
SQ2 = math.sqrt(2.0)


def _pf():
    from paper_2110_12448_amd import pfiso
    return pfiso


def _perturbed(pr, seed=4, amp=0.2):
    pr = dict(pr)
    pr["U0"] = pr["U0"] + amp * np.random.default_rng(seed).uniform(-1, 1, pr["U0"].shape)
    return pr


def run_gpu(pr, prec, nsteps):
    pf = _pf()
    print("gpu case: diffusion %s prec=%d steps=%d" % ((pr["nx"], pr["ny"]), prec, nsteps),
          flush=True)
    s = pf.Solver(pr, precision=prec)
    s.step_diffusion(nsteps)
    phi, U, psi, g = s.read_fields()
    shift, _ = s.frame_state()
    s.close()
    return phi, U, psi, shift


def run_oracle(pr, nsteps):
    p = oracle.Params.from_problem(pr, frozen_psi=1)
    psi, U, st = oracle.step(p, pr["psi0"], pr["U0"], pr["grain"], nsteps)
    return np.tanh(psi / SQ2), U, psi, st


@pytest.mark.parametrize("prec,tol", [(1, 1e-10), (0, 1e-5)])
@pytest.mark.parametrize("scheme", ["iso", "std"])
def test_diffusion_small(prec, tol, scheme):
    pr = _perturbed(wl.config_small_2d(30.0, scheme=scheme))
    phi, U, psi, _ = run_gpu(pr, prec, 100)
    ophi, oU, opsi, st = run_oracle(pr, 100)
    print("max|dU| %.3e" % np.max(np.abs(U - oU)))
    assert np.max(np.abs(U - oU)) <= tol
    want = pr["psi0"] if prec == 1 else pr["psi0"].astype(np.float32).astype(np.float64)
    assert np.array_equal(psi, want)


def test_diffusion_ragged_noflux_grains_fp64():
    nx, ny = 61, 37
    rng = np.random.default_rng(3)
    rot = np.stack([wl.rotation_2d(10.0 + 20.0 * g) for g in range(3)])
    grain = rng.integers(0, 3, size=(ny, nx)).astype(np.int8)
    pr = _perturbed(wl.problem(2, (nx, ny), thermal="frozen", bc=(0, 0, 0), rot=rot, grain=grain,
                               seed_radius=6.0, y_front=(ny // 2) * 0.8, seed=9))
    phi, U, psi, _ = run_gpu(pr, 1, 60)
    ophi, oU, opsi, st = run_oracle(pr, 60)
    assert np.max(np.abs(U - oU)) <= 1e-10


def test_diffusion_moving_frame_fp64():
    """psi does not move, so a tip above the shift row brings the frame down
    one row per step until it is below: shifts and fields as in the oracle."""
    pr = _perturbed(wl.config_small_2d(0.0, n=64, frame=1, shift_row=6))
    phi, U, psi, shift = run_gpu(pr, 1, 12)
    ophi, oU, opsi, st = run_oracle(pr, 12)
    assert st.shift >= 2 and shift == st.shift
    assert np.max(np.abs(U - oU)) <= 1e-10 and np.max(np.abs(phi - ophi)) <= 1e-12


def test_diffusion_full_size_fp32():
    """1024 x 2048, the bench's launch configuration: every cell after 20 steps."""
    pr = _perturbed(wl.config_directional_2d())
    phi, U, psi, _ = run_gpu(pr, 0, 20)
    ophi, oU, opsi, st = run_oracle(pr, 20)
    assert np.max(np.abs(U - oU)) <= 1e-5


def test_diffusion_rejects_3d_and_two_point():
    pf = _pf()
    s3 = pf.Solver(wl.problem(3, (8, 8, 8)), precision=pf.PF_F32)
    with pytest.raises(pf.PFError) as e:
        s3.step_diffusion(1)
    assert e.value.code == pf.PF_ERR_ARG
    s3.close()
    s2 = pf.Solver(wl.config_small_2d(0.0, n=32, **wl.SCHEMES_2D["S10"]), precision=pf.PF_F32)
    with pytest.raises(pf.PFError) as e:
        s2.step_diffusion(1)
    assert e.value.code == pf.PF_ERR_ARG
    s2.close()
