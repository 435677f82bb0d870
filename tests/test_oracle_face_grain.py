"""Pins the oracle's reading of which grain a face flux uses at a grain
boundary (the paper rotates a_s per grain, Sec. 2.2 and Eq. anis_function,
and leaves the face between two grains open): a face takes the grain of the
cell on its lower side along the face normal.

On a linear psi every face gradient of the standard <10>/<100> discretisation
(normal difference and four-point tangential averages) equals grad psi
exactly, and the standard Laplacian vanishes.  The anisotropic remainder
N = div J - a_c^2 L_std of a cell is then [J(R_up) - J(R_down)] . e / h
summed over its axes, where R_up and R_down are the rotations its two faces
along e use.  With grain A below a boundary plane and grain B from it on,
the first B cell sees J(B) on its upper face and J(A) on its lower one, and
every other cell sees one grain on both faces: N = [J(B) - J(A)] . e / h at
the first B cell and 0 elsewhere.  Reading the upper cell's grain instead
puts that value on the last A cell.

J is computed here independently of the oracle's quartic form: in 2D from
the angle form a(theta) = 1 + eps4 cos 4(theta - alpha0), J = a^2 g + a a'(theta)
(-g_y, g_x); in 3D by complex-step differentiation of the cubic a_s(g) =
1 - 3 eps4 + 4 eps4 sum_i (R^T g / |g|)_i^4 (J = a^2 g + |g|^2 a da/dg)."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_12448_amd import workloads as wl

EPS4 = 0.05
H = 0.8


def J_2d(g, alpha0_deg):
    th = math.atan2(g[1], g[0])
    al = math.radians(alpha0_deg)
    a = 1.0 + EPS4 * math.cos(4.0 * (th - al))
    da = -4.0 * EPS4 * math.sin(4.0 * (th - al))
    return a * a * np.asarray(g) + a * da * np.array([-g[1], g[0]])


def a_cubic(g, R):
    gl = np.sqrt(np.sum(g * g))
    n = R.T @ (g / gl)
    return 1.0 - 3.0 * EPS4 + 4.0 * EPS4 * np.sum(n ** 4)


def J_3d(g, R):
    g = np.asarray(g, dtype=np.float64)
    a = a_cubic(g.astype(complex), R).real
    grad = np.empty(3)
    step = 1e-30
    for q in range(3):
        e = np.zeros(3, dtype=complex)
        e[q] = 1j * step
        grad[q] = a_cubic(g.astype(complex) + e, R).imag / step
    return a * a * g + np.dot(g, g) * a * grad


@pytest.mark.parametrize("axis", [0, 1])
def test_face_grain_2d(axis):
    n = 12
    angles = (10.0, 35.0)
    g = np.array([0.3, -0.7])
    x = np.arange(n) * H
    X, Y = np.meshgrid(x, x, indexing="xy")
    psi = g[0] * X + g[1] * Y
    grain = np.zeros((n, n), dtype=np.int8)
    b = 6                                    # first cell of grain 1 along the axis
    if axis == 0:
        grain[:, b:] = 1
    else:
        grain[b:, :] = 1
    rot = np.stack([wl.rotation_2d(a) for a in angles])
    p = oracle.Params(dim=2, nx=n, ny=n, eps4=EPS4, h=H, rot=rot, bc=(oracle.NOFLUX,) * 3)
    N = oracle.anis_remainder(p, psi, grain)
    jump = (J_2d(g, angles[1])[axis] - J_2d(g, angles[0])[axis]) / H
    assert abs(jump) > 1e-2
    inner = slice(2, n - 2)
    if axis == 0:
        line = N[inner, :]
        first, before = line[:, b], line[:, b - 1]
        rest = np.delete(line[:, 2:n - 2], [b - 2, b - 1 - 2], axis=1)
    else:
        line = N[:, inner].T
        first, before = line[:, b], line[:, b - 1]
        rest = np.delete(line[:, 2:n - 2], [b - 2, b - 1 - 2], axis=1)
    assert np.max(np.abs(first - jump)) <= 1e-12
    assert np.max(np.abs(before)) <= 1e-12
    assert np.max(np.abs(rest)) <= 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_face_grain_3d(axis):
    n = 9
    rot = wl.random_rotations(11, 2)
    g = np.array([0.41, -0.27, 0.63])
    c = np.arange(n) * H
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    psi = g[0] * X + g[1] * Y + g[2] * Z
    grain = np.zeros((n, n, n), dtype=np.int8)
    b = 4
    sl = [slice(None)] * 3
    sl[2 - axis] = slice(b, None)            # array axes are (z, y, x)
    grain[tuple(sl)] = 1
    p = oracle.Params(dim=3, nx=n, ny=n, nz=n, w=wl.ISO_3D, eps4=EPS4, h=H, rot=rot,
                      bc=(oracle.NOFLUX,) * 3)
    N = oracle.anis_remainder(p, psi, grain)
    jump = (J_3d(g, rot[1])[axis] - J_3d(g, rot[0])[axis]) / H
    assert abs(jump) > 1e-2
    N = np.moveaxis(N, 2 - axis, 0)[:, 2:n - 2, 2:n - 2]   # axis first, interior of the others
    for i in range(2, n - 2):
        want = jump if i == b else 0.0
        assert np.max(np.abs(N[i] - want)) <= 1e-12, (i, np.max(np.abs(N[i] - want)))


def test_face_flux_matches_independent_J():
    """Single grain, linear psi: the remainder vanishes (every face carries the
    same J), and the 2D and 3D J above agree with each other for rotations
    about z and in-plane gradients (the cubic form reduces to the angle form,
    Eq. anis_function)."""
    R = wl.rotation_2d(23.0)
    g2 = np.array([0.5, 0.2])
    assert np.allclose(J_3d(np.array([g2[0], g2[1], 0.0]), R)[:2], J_2d(g2, 23.0), atol=1e-14)
