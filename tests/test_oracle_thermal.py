"""Pins the oracle's frozen-temperature terms (Sec. 2.1, Eqs. Thermal_F1 and
Thermal_F2) and the thermal coordinate zeta = y + s h - y0 - Vp n dt by a
closed form that does not go through any stencil.

In bulk liquid with phi = -1 exactly (psi = -40: tanh(-40/sqrt2) rounds to -1
in FP64) and uniform psi and U, every spatial difference vanishes, the
anisotropy guard gives a_s = 1 with no torque, and 1 - phi^2 = 0.  Eq. PF_a
then reduces to F1 d psi/dt = sqrt2 phi = -sqrt2, so one explicit step moves
row j by exactly -sqrt2 dt / F1(zeta_j), with F1 = 1 - (1 - k) zeta / lT; and
Eq. PF_b has no source, no anti-trapping flux and no diffusion, so U stays
bit for bit.  Over many steps the rows drift apart only by O(dt m (1-k) h/lT),
whose Laplacian and gradient square stay below the stated bound."""
import math

import numpy as np
import pytest

import oracle

SQ2 = math.sqrt(2.0)


def _params(dim, nx, ny, nz, **kw):
    base = dict(dim=dim, nx=nx, ny=ny, nz=nz, k=0.15, eps4=0.05, D=2.0, lam=3.2, h=0.8,
                dt=0.05, Vp=0.7, lT=30.0, y0=-4.0, bc=(oracle.PERIODIC, oracle.NOFLUX,
                                                    oracle.PERIODIC))
    base.update(kw)
    return oracle.Params(**base)


def _F1(p, n, s):
    """Eq. Thermal_F1 at every row for time level n and frame shift s."""
    zeta = np.arange(p.ny) * p.h + s * p.h - p.y0 - p.Vp * n * p.dt
    return 1.0 - (1.0 - p.k) * zeta / p.lT


CASES = [(0, 0), (7, 0), (0, 5), (40, 3), (123, 9)]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("n,s", CASES)
def test_bulk_drift_one_step(dim, n, s):
    nx, ny, nz = 5, 24, (4 if dim == 3 else 1)
    p = _params(dim, nx, ny, nz)
    F1 = _F1(p, n, s)
    assert F1.min() > 0.2 and F1.max() < 1.8      # a strong gradient over the box
    psi0 = np.full(p.shape(), -40.0)
    U0 = np.full(p.shape(), -0.37)
    psi, U, st = oracle.step(p, psi0, U0, None, 1, oracle.State(step=n, shift=s))
    expect_row = -40.0 - SQ2 * p.dt / F1
    expect = np.broadcast_to(expect_row[:, None], p.shape()[-2:])
    if dim == 3:
        expect = np.broadcast_to(expect, p.shape())
    assert np.max(np.abs(psi - expect)) <= 1e-12
    assert np.array_equal(U, U0)
    assert st.step == n + 1 and st.shift == s


def test_bulk_drift_isothermal_limit():
    """lT <= 0: F1 = 1 everywhere, whatever zeta would be."""
    p = _params(2, 5, 16, 1, lT=0.0)
    psi, U, _ = oracle.step(p, np.full(p.shape(), -40.0), np.full(p.shape(), -0.2), None, 1,
                            oracle.State(step=50, shift=9))
    assert np.max(np.abs(psi + 40.0 + SQ2 * p.dt)) <= 1e-13


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("eps4", [0.0, 0.05])
def test_bulk_drift_many_steps(dim, eps4):
    """m steps advance the clock: row j ends near -40 - sum_n sqrt2 dt /
    (F1(zeta_j^n) a^2).  The first step sees no gradient (a = 1 by the guard);
    after it psi decreases along +y, so the centre normal lies along -y and
    a_s = 1 + eps4 cos(4 (-90 deg)) = 1 + eps4 for alpha0 = 0 (Eq.
    anis_function), with no torque on the y faces.  The rows drift apart:
    after n steps neighbouring rows differ by about sqrt2 dt n delta, delta =
    (1 - k) h / (lT F1^2), so the gradient-square term of Eq. PF_a adds about
    sqrt2 dt sum_n (sqrt2 dt n delta / h)^2 = 2 sqrt2 dt^3 delta^2 m^3 /
    (3 h^2), below 3e-4 here, and the Laplacian less; the tolerance is 1e-3.
    Reading F1 with k in place of 1 - k, a clock that does not advance, or a
    bulk term not divided by a^2 moves the rows by more than 1e-2."""
    nx, ny, nz = 5, 40, (4 if dim == 3 else 1)
    m = 40
    p = _params(dim, nx, ny, nz, lT=200.0, Vp=2.0, eps4=eps4)
    psi, U, st = oracle.step(p, np.full(p.shape(), -40.0), np.full(p.shape(), -0.37), None, m,
                             oracle.State(step=0, shift=2))
    assert st.step == m and st.shift == 2
    a2 = [1.0 if n == 0 else (1.0 + eps4) ** 2 for n in range(m)]
    expect = -40.0 - sum(SQ2 * p.dt / (_F1(p, n, 2) * a2[n]) for n in range(m))
    got = psi.reshape(-1, ny, nx)[0, :, 2]
    # rows away from the no-flux walls: the mirrored end rows drift as their
    # images do, and that difference spreads diffusively (about one row per
    # ten steps here), so only rows 10..ny-11 are held to the bulk form
    mid = slice(10, ny - 10)
    err = np.max(np.abs(got[mid] - expect[mid]))
    assert err <= 1e-3, err
    y = np.arange(ny) * p.h
    alts = [
        -40.0 - sum(SQ2 * p.dt / (a2[n] * (1.0 - p.k * (y + 2 * p.h - p.y0 - p.Vp * n * p.dt) /
                                           p.lT)) for n in range(m)),
        -40.0 - sum(SQ2 * p.dt / (_F1(p, 0, 2) * a2[n]) for n in range(m)),
    ]
    if eps4 > 0:
        alts.append(-40.0 - sum(SQ2 * p.dt / _F1(p, n, 2) for n in range(m)))
    for alt in alts:
        assert np.min(np.abs(alt[mid] - expect[mid])) > 1e-2
    assert np.all(U == -0.37)
