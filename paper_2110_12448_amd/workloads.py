"""Seeded synthetic inputs for the phase-field step (FP64, host side).

This module builds initial fields, grain maps, grain rotations and the scalar
parameters of each workload.  It holds none of the time step's arithmetic: no
stencil, no anisotropy, no update.  The GPU path and the CPU oracle both take
their inputs from here and from nowhere else.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator keyed by (seed, stream, index); u = (x >> 11) * 2^-53.

Units: lengths in W, times in tau_0.  Arrays are C-ordered (ny, nx) in 2D and
(nz, ny, nx) in 3D, x fastest; cell (i, j, l) sits at (i h, j h, l h); y is
the growth and thermal axis.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np

NOFLUX = 0
PERIODIC = 1

# Model constants of the thin-interface analysis (Sec. 2.1): a1 = 5 sqrt2 / 8,
# a2 = 47 / 75; with W/d0 fixed by D~ = a1 a2 W/d0, the coupling constant is
# lambda = a1 W / d0 = D~ / a2.
A1 = 5.0 * math.sqrt(2.0) / 8.0
A2 = 47.0 / 75.0

ISO_2D = (2.0 / 3.0, 1.0 / 3.0, 0.0)     # L, G, D_{2,1}
STD_2D = (1.0, 0.0, 0.0)                 # <10> shell only
ISO_3D = (1.0 / 3.0, 2.0 / 3.0, 0.0)     # L, G, D_{1,2,0}
STD_3D = (1.0, 0.0, 0.0)                 # <100> shell only
ISO_3D_441 = (4.0 / 9.0, 4.0 / 9.0, 1.0 / 9.0)

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(keys: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to counters (uint64 in, uint64 out)."""
    with np.errstate(over="ignore"):
        z = keys.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, stream: int, n: int) -> np.ndarray:
    """n uniforms in [0, 1) for (seed, stream); counter = index."""
    base = (np.uint64(seed & 0xFFFF) << np.uint64(48)) | (np.uint64(stream & 0xFF) << np.uint64(40))
    keys = base + np.arange(n, dtype=np.uint64)
    return (splitmix64(keys) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def rotation_2d(alpha0_deg: float) -> np.ndarray:
    """Crystal -> lab rotation by +alpha0 about z (x towards y)."""
    a = math.radians(alpha0_deg)
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def quaternion_to_matrix(q: Sequence[float]) -> np.ndarray:
    """Unit quaternion (w, x, y, z), Hamilton convention -> rotation matrix."""
    w, x, y, z = (float(v) for v in q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def random_rotations(seed: int, n: int) -> np.ndarray:
    """n uniformly distributed rotations (Shoemake, Graphics Gems III, 1992)."""
    u = uniform(seed, 7, 3 * n).reshape(n, 3)
    out = np.empty((n, 3, 3))
    for g in range(n):
        u1, u2, u3 = u[g]
        a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
        q = (b * math.cos(2 * math.pi * u3), a * math.sin(2 * math.pi * u2),
             a * math.cos(2 * math.pi * u2), b * math.sin(2 * math.pi * u3))
        out[g] = quaternion_to_matrix(q)
    return out


def voronoi_columns(nx: int, nz: int, n_seeds: int, seed: int) -> np.ndarray:
    """Grain index on the (x, z) plane from n_seeds lattice sites (periodic
    squared distance in integers; ties go to the lowest seed id)."""
    u = uniform(seed, 9, 2 * n_seeds).reshape(n_seeds, 2)
    sx = np.minimum((u[:, 0] * nx).astype(np.int64), nx - 1)
    sz = np.minimum((u[:, 1] * nz).astype(np.int64), nz - 1)
    ii = np.arange(nx, dtype=np.int64)[None, :]
    ll = np.arange(nz, dtype=np.int64)[:, None]
    best = np.full((nz, nx), np.iinfo(np.int64).max, dtype=np.int64)
    gid = np.zeros((nz, nx), dtype=np.int8)
    for g in range(n_seeds):
        dx = np.abs(ii - sx[g]); dx = np.minimum(dx, nx - dx)
        dz = np.abs(ll - sz[g]); dz = np.minimum(dz, nz - dz)
        d2 = dx * dx + dz * dz
        better = d2 < best
        best = np.where(better, d2, best)
        gid = np.where(better, np.int8(g), gid)
    return gid


def _noisy_psi(dist: np.ndarray, seed: int, amp: float) -> np.ndarray:
    """psi from a signed distance (positive in the solid) with uniform phi noise
    of half-width amp inside the interface band |phi| <= 1 - 2 amp only, so the
    noise never saturates phi (outside the band psi stays the signed distance)."""
    psi = dist.astype(np.float64).copy()
    if amp <= 0.0:
        return psi
    phi = np.tanh(psi / math.sqrt(2.0))
    band = np.abs(phi) <= 1.0 - 2.0 * amp
    u = uniform(seed, 1, psi.size).reshape(psi.shape)
    noisy = np.clip(phi + amp * (2.0 * u - 1.0), -1.0 + 1e-12, 1.0 - 1e-12)
    psi[band] = math.sqrt(2.0) * np.arctanh(noisy[band])
    return psi


def supersaturation(phi: np.ndarray, k: float, c_over_cl0: float) -> np.ndarray:
    """U of a uniform concentration c (Eq. Supersaturation), c/c_l^0 given."""
    return (c_over_cl0 / ((1.0 - phi) / 2.0 + k * (1.0 + phi) / 2.0) - 1.0) / (1.0 - k)


def stable_dt(dim: int, h: float, D: float) -> float:
    """The paper's time step rule: 0.8 h^2 / (4 D) in 2D, 0.8 h^2 / (6 D) in 3D."""
    return 0.8 * h * h / (2 * dim * D)


def problem(dim: int, shape: Sequence[int], *, h: float = 0.8, k: float = 0.15,
            eps4: float = 0.02, D: float = 2.0, lam: Optional[float] = None,
            dt: Optional[float] = None, scheme: str = "iso",
            alpha0_deg: float = 0.0, rot: Optional[np.ndarray] = None,
            grain: Optional[np.ndarray] = None, thermal: str = "frozen",
            Vp: float = 0.05, lT: Optional[float] = None, y_front: float = 0.0,
            omega: float = 0.55, bc: Optional[Sequence[int]] = None,
            frame: int = 0, shift_row: Optional[int] = None,
            seed_shape: str = "disc", seed_radius: float = 10.0,
            noise: float = 0.01, seed: int = 1, antitrapping: int = 0,
            two_point: int = 0, dynamic_grains: int = 0) -> dict:
    """One solve: scalar parameters plus initial psi, U and grain arrays.

    shape is (nx, ny) in 2D and (nx, ny, nz) in 3D.  seed_shape 'disc' puts a
    disc (sphere) of radius seed_radius*h centred at ((nx/2) h, 0[, (nz/2) h]);
    'slab' puts the solid at y <= seed_radius*h.  antitrapping 1 selects the
    full current of Eq. Anti_convention (2D), two_point 1 the two-point <10>
    divergences of the standard scheme (2D); dynamic_grains 1 lets grain
    indices follow solidification.  thermal 'frozen' uses the
    frozen-temperature functions with U from a uniform c_inf = k c_l^0 (U = -1 in
    the liquid, 0 in the solid); 'isothermal' uses F1 = 1, F2 = U with U = -omega
    everywhere.
    """
    nx, ny = int(shape[0]), int(shape[1])
    nz = int(shape[2]) if dim == 3 else 1
    lam = D / A2 if lam is None else lam
    dt = stable_dt(dim, h, D) if dt is None else dt
    if scheme == "iso":
        w = ISO_2D if dim == 2 else ISO_3D
    elif scheme == "std":
        w = STD_2D if dim == 2 else STD_3D
    elif scheme == "iso441":
        w = ISO_3D_441
    else:
        raise ValueError(scheme)
    if bc is None:
        bc = (PERIODIC, NOFLUX, PERIODIC if dim == 3 else NOFLUX)
    H = ny * h
    if thermal == "frozen":
        lT = 40.0 * H if lT is None else lT
        y0 = y_front - 0.5 * lT
    else:
        Vp, lT, y0 = 0.0, 0.0, 0.0
    if rot is None:
        rot = rotation_2d(alpha0_deg)[None]
    rot = np.asarray(rot, dtype=np.float64).reshape(-1, 3, 3)

    x = np.arange(nx) * h
    y = np.arange(ny) * h
    if dim == 2:
        X, Y = np.meshgrid(x, y, indexing="xy")
        if seed_shape == "disc":
            dist = seed_radius * h - np.hypot(X - (nx // 2) * h, Y - y_front)
        else:
            dist = seed_radius * h + y_front - Y
    else:
        z = np.arange(nz) * h
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        if seed_shape == "disc":
            dist = seed_radius * h - np.sqrt((X - (nx // 2) * h) ** 2 + (Y - y_front) ** 2 +
                                             (Z - (nz // 2) * h) ** 2)
        else:
            dist = seed_radius * h + y_front - Y
    psi0 = _noisy_psi(dist, seed, noise)
    phi0 = np.tanh(psi0 / math.sqrt(2.0))
    if thermal == "frozen":
        U0 = supersaturation(phi0, k, k)            # c_inf = k c_l^0: -1 liquid, 0 solid
    else:
        U0 = np.full(psi0.shape, -omega)            # uniform supersaturation -Omega
    if grain is None:
        grain = np.zeros(psi0.shape, dtype=np.int8)
    else:
        grain = np.ascontiguousarray(np.broadcast_to(grain, psi0.shape), dtype=np.int8)
    return dict(dim=dim, nx=nx, ny=ny, nz=nz, w=tuple(w), k=k, eps4=eps4, D=D, lam=lam,
                h=h, dt=dt, Vp=Vp, lT=lT, y0=y0, bc=tuple(bc), frame=int(frame),
                shift_row=int(ny // 2 if shift_row is None else shift_row), rot=rot,
                psi0=psi0, U0=U0, grain=grain, antitrapping=int(antitrapping),
                two_point=int(two_point), dynamic_grains=int(dynamic_grains))


# The three 2D schemes compared in Sec. 5 (Table 1), as problem() keywords.
SCHEMES_2D = {
    "S10": dict(scheme="std", antitrapping=1, two_point=1),   # anisotropic, full A
    "S21": dict(scheme="iso", antitrapping=1),                # isotropic, full A (App. B)
    "Sbar21": dict(scheme="iso"),                             # isotropic, approximated A
}


# ------------------------------------------------------------------ configs

def config_small_2d(alpha0_deg: float = 0.0, n: int = 128, seed: int = 1, **kw) -> dict:
    """128 x 128, h = 0.8, k = 0.15, eps4 = 0.02, D = 2, frozen gradient, disc
    seed of radius 10 h at the bottom with +-0.01 phi noise."""
    return problem(2, (n, n), alpha0_deg=alpha0_deg, seed=seed, **kw)


def config_isothermal_2d(alpha0_deg: float = 30.0, n: int = 781, seed: int = 6, **kw) -> dict:
    """Free growth in an isothermal melt as in the runs behind Table 1
    (Sec. 5): W/d0* = 16, h/W = 1.2, eps4 = 0.014, k = 0.1, Omega = 0.43,
    no-flux walls on a square of side 1.5e4 d0* (781 cells), circular seed of
    radius 50 d0* at the centre.  lambda = a1 W/d0*, D~ = a2 lambda
    (Sec. 2.1), dt = 0.8 h^2 / (4 D~).  The whole run, t = 1.5e6 d0*^2/D, is
    ISOTHERMAL_2D_STEPS steps."""
    lam = A1 * 16.0
    D = A2 * lam
    h = 1.2
    kw.setdefault("bc", (NOFLUX, NOFLUX, NOFLUX))
    return problem(2, (n, n), h=h, k=0.1, eps4=0.014, D=D, lam=lam, dt=stable_dt(2, h, D),
                   thermal="isothermal", omega=0.43, alpha0_deg=alpha0_deg,
                   seed_radius=50.0 / 16.0 / h, y_front=(n // 2) * h, seed=seed, **kw)


# t = 1.5e6 d0*^2 / D = 1.5e6 tau_0 / ((W/d0*)^2 D~) since D = D~ W^2 / tau_0
ISOTHERMAL_2D_STEPS = int(round(1.5e6 / (16.0 ** 2 * (A2 * A1 * 16.0) *
                                         stable_dt(2, 1.2, A2 * A1 * 16.0))))


def misorientation(seed: int) -> float:
    """Grain misorientation uniform in [0, 45] degrees."""
    return 45.0 * float(uniform(seed, 3, 1)[0])


def config_directional_2d(nx: int = 1024, ny: int = 2048, seed: int = 2, **kw) -> dict:
    """Directional solidification in a moving frame: nx x ny, misorientation
    uniform in [0, 45] deg, frame shift at row ny/2."""
    kw.setdefault("alpha0_deg", misorientation(seed))
    kw.setdefault("frame", 1)
    return problem(2, (nx, ny), seed=seed, **kw)


def config_polycrystal_3d(n: int = 256, n_grains: int = 8, seed: int = 3, ny: Optional[int] = None,
                          **kw) -> dict:
    """n^3 polycrystal: n_grains Voronoi columns seeded on the bottom plane,
    uniform random cubic orientations, planar solid slab y <= 5 h."""
    ny = n if ny is None else ny
    gid = voronoi_columns(n, n, n_grains, seed)          # (nz, nx)
    grain = np.broadcast_to(gid[:, None, :], (n, ny, n))
    rot = random_rotations(seed, n_grains)
    kw.setdefault("seed_shape", "slab")
    kw.setdefault("seed_radius", 5.0)
    return problem(3, (n, ny, n), rot=rot, grain=grain, seed=seed, **kw)


def config_batched_2d(n_solves: int = 64, seed: int = 4, sides=(256, 384, 512, 768, 1024),
                      **kw) -> list:
    """n_solves independent square 2D solves, side drawn uniformly from
    `sides`, misorientation uniform in [0, 45] deg, frozen gradient, disc seed
    (each solve seeded with its own noise stream)."""
    u = uniform(seed, 5, 2 * n_solves).reshape(n_solves, 2)
    out = []
    for i in range(n_solves):
        side = int(sides[min(int(u[i, 0] * len(sides)), len(sides) - 1)])
        out.append(problem(2, (side, side), alpha0_deg=45.0 * float(u[i, 1]),
                           seed=(seed * 1000 + i) & 0xFFFF, **kw))
    return out
