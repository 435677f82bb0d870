"""Pins the oracle's frozen-psi mode: U evolves by Eq. PF_b with d psi/dt = 0,
i.e. (1 + k - (1-k) phi) dU/dt = D~ div[(1 - phi) grad U] through a fixed
phase field (the anti-trapping current and the source vanish with
d psi/dt)."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_12448_amd import workloads as wl

SQ2 = math.sqrt(2.0)


def _problem(n=40, seed=3):
    return wl.problem(2, (n, n), thermal="isothermal", seed_radius=4.0, noise=0.05, seed=seed,
                      y_front=(n // 2) * 0.8)


def test_psi_unchanged():
    pr = _problem()
    p = oracle.Params.from_problem(pr, frozen_psi=1)
    U0 = pr["U0"] + 0.1 * np.random.default_rng(2).uniform(-1, 1, pr["U0"].shape)
    psi, U, st = oracle.step(p, pr["psi0"], U0, None, 7)
    assert np.array_equal(psi, pr["psi0"])
    assert np.max(np.abs(U - U0)) > 1e-6


@pytest.mark.parametrize("w", [wl.ISO_2D, wl.STD_2D])
def test_solute_conserved(w):
    """sum (1 + k - (1-k) phi) U is constant: the divergence is conservative
    and phi does not change (periodic x, no-flux y)."""
    pr = _problem()
    rng = np.random.default_rng(1)
    U0 = -0.5 + 0.3 * rng.uniform(-1, 1, pr["U0"].shape)
    p = oracle.Params.from_problem(pr, frozen_psi=1, w=w)
    phi = np.tanh(pr["psi0"] / SQ2)
    wgt = 1.0 + p.k - (1.0 - p.k) * phi
    psi, U, st = oracle.step(p, pr["psi0"], U0, None, 20)
    a, b = float(np.sum(wgt * U0)), float(np.sum(wgt * U))
    assert abs(a - b) < 1e-12 * np.sum(np.abs(wgt * U0))
    assert np.max(np.abs(U - U0)) > 1e-4


def test_fourier_mode_in_uniform_liquid():
    """phi = -1 everywhere: dU/dt = D~ L_{2,1} U, so a periodic mode decays by
    the exact factor 1 + dt D~ s(k) per step, with s the symbol of L_{2,1}
    (Eqs. 2D_L10, 2D_L01, weights 2/3 and 1/3)."""
    nx, ny, h = 24, 16, 0.8
    p = oracle.Params(dim=2, nx=nx, ny=ny, h=h, bc=(oracle.PERIODIC,) * 3, frozen_psi=1,
                      w=wl.ISO_2D)
    kx, ky = 2 * math.pi * 3 / (nx * h), 2 * math.pi * 2 / (ny * h)
    x = np.arange(nx) * h
    y = np.arange(ny) * h
    X, Y = np.meshgrid(x, y, indexing="xy")
    U0 = 0.1 * np.cos(kx * X + ky * Y)
    psi0 = np.full((ny, nx), -60.0)
    assert np.all(np.tanh(psi0 / SQ2) == -1.0)
    cx, cy = math.cos(kx * h), math.cos(ky * h)
    sym = (2.0 / 3.0) * (2 * cx + 2 * cy - 4) / h ** 2 + (1.0 / 3.0) * (4 * cx * cy - 4) / (2 * h ** 2)
    n = 30
    psi, U, st = oracle.step(p, psi0, U0, None, n)
    want = U0 * (1.0 + p.dt * p.D * sym) ** n
    np.testing.assert_allclose(U, want, rtol=0, atol=1e-13)


def test_one_dimensional_reduction():
    """Fields uniform in x: every shell reduces to the two-point flux
    (alpha_0 + alpha_n)/2 (U_n - U_0)/h^2 along y with alpha = 1 - phi,
    whatever the weights; compared with an independent 1D stepper (mirror
    ghosts at the y walls)."""
    ny, nx, h, k, D, dt = 50, 5, 0.8, 0.15, 2.0, 0.05
    y = np.arange(ny) * h
    rng = np.random.default_rng(8)
    psi1 = (16.0 - y) + 0.2 * rng.uniform(-1, 1, ny)
    U1 = -0.7 + 0.2 * rng.uniform(-1, 1, ny)
    p = oracle.Params(dim=2, nx=nx, ny=ny, h=h, k=k, D=D, dt=dt, frozen_psi=1,
                      w=(0.4, 0.6, 0.0), bc=(oracle.PERIODIC, oracle.NOFLUX, oracle.NOFLUX))
    psi, U, st = oracle.step(p, np.tile(psi1[:, None], (1, nx)), np.tile(U1[:, None], (1, nx)),
                             None, 25)
    phi = np.tanh(psi1 / SQ2)
    a = 1.0 - phi
    u = U1.copy()
    for _ in range(25):
        ue = np.concatenate([u[:1], u, u[-1:]])
        ae = np.concatenate([a[:1], a, a[-1:]])
        div = ((ae[1:-1] + ae[2:]) / 2 * (ue[2:] - ue[1:-1]) +
               (ae[1:-1] + ae[:-2]) / 2 * (ue[:-2] - ue[1:-1])) / h ** 2
        u = u + dt * D * div / (1.0 + k - (1.0 - k) * phi)
    np.testing.assert_allclose(U[:, 2], u, rtol=0, atol=1e-13)
