"""Pins the oracle's L, G and D operators to the Fourier symbols the paper
prints (Sec. 4.2, Sec. 6.1, App. A), to the isotropy constraints and their
solutions, and to exact results on low-order polynomials (Sec. 4.1)."""
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fourier_symbols.json")))

BASES_2D = {"10": (1.0, 0.0, 0.0), "01": (0.0, 1.0, 0.0)}
BASES_3D = {"100": (1.0, 0.0, 0.0), "010": (0.0, 1.0, 0.0), "001": (0.0, 0.0, 1.0)}


def _params(dim, n, w, bc=oracle.PERIODIC, h=1.0):
    return oracle.Params(dim=dim, nx=n, ny=n, nz=n if dim == 3 else 1, w=w, h=h,
                         bc=(bc, bc, bc))


def _grid(dim, n):
    ax = np.arange(n, dtype=np.float64)
    if dim == 2:
        Y, X = np.meshgrid(ax, ax, indexing="ij")
        return (X, Y)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    return (X, Y, Z)


def _mode(f, m):
    """Fourier coefficient of f at integer wave vector m (x, y[, z])."""
    F = np.fft.fftn(f)
    n = f.shape[0]
    idx = tuple(int(v) % n for v in reversed(m))     # arrays are (z,) y, x
    return F[idx]


def symbol(op, dim, n, w, m):
    """Measured symbol of op at k = 2 pi m / n (h = 1), the paper's definition:
    L: F[L psi](k)/F[psi](k); G: F[G](2k)/F[psi psi](2k); D: F[D](2k)/F[alpha beta](2k)
    with psi = alpha = beta = cos(k.r)."""
    p = _params(dim, n, w)
    X = _grid(dim, n)
    k = [2 * math.pi * mi / n for mi in m]
    ph = sum(ki * xi for ki, xi in zip(k, X))
    f = np.cos(ph)
    m2 = [2 * mi for mi in m]
    if op == "L":
        return (_mode(oracle.laplacian(p, f), m) / _mode(f, m)).real, k
    if op == "G":
        return (_mode(oracle.grad_square(p, f), m2) / _mode(f * f, m2)).real, k
    return (_mode(oracle.divergence(p, f, f), m2) / _mode(f * f, m2)).real, k


def k4_coefficient(op, dim, n, w, m):
    """(S(k) - c k^2)/k^4 Richardson-extrapolated from k and 2k, i.e. the k^4
    coefficient along direction m to O(k^4)."""
    cont = GOLD["continuum"][op]
    vals = []
    for s in (1, 2):
        S, k = symbol(op, dim, n, w, [s * v for v in m])
        k2 = sum(v * v for v in k)
        vals.append((S - cont * k2) / (k2 * k2))
    return (4.0 * vals[0] - vals[1]) / 3.0


def printed(a, b, m):
    """a sum k_i^4 + b sum_{i<j} k_i^2 k_j^2 over k^4 along direction m."""
    u = np.asarray(m, dtype=np.float64)
    u = u / np.linalg.norm(u)
    s4 = np.sum(u ** 4)
    cross = sum(u[i] ** 2 * u[j] ** 2 for i in range(len(u)) for j in range(i + 1, len(u)))
    return a * s4 + b * cross


DIRS_2D = [(1, 0), (1, 1), (2, 1)]
DIRS_3D = [(1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 1, 0)]


@pytest.mark.parametrize("op", ["L", "G", "D"])
@pytest.mark.parametrize("base", ["10", "01"])
def test_symbol_2d_bases(op, base):
    g = GOLD["2d"][op + base]
    for m in DIRS_2D:
        c = k4_coefficient(op, 2, 64, BASES_2D[base], m)
        assert c == pytest.approx(printed(g["a"], g["b"], m), rel=2e-3, abs=2e-4), (op, base, m)


@pytest.mark.parametrize("op", ["L", "G", "D"])
def test_symbol_2d_isotropic_mix(op):
    """With weights (2/3, 1/3) the k^4 coefficient is the same in every direction."""
    key = {"L": "L21", "D": "D21", "G": None}[op]
    a = GOLD["2d"][op + "10"]["a"]
    want = a if key is None else GOLD["2d"][key]["a"]
    w = tuple(GOLD["isotropic_weights"]["2d"]["w"]) + (0.0,)
    for m in DIRS_2D + [(3, 1), (3, 2)]:
        c = k4_coefficient(op, 2, 64, w, m)
        assert c == pytest.approx(want, rel=2e-3), (op, m)


def test_unique_isotropic_weights_2d():
    """Solve c1 + c2 = 1 and 'cross coefficient = 2 * quartic coefficient'
    (Eqs. prove1, prove2) from the measured base symbols; the solution is
    (2/3, 1/3) for L, G and D alike."""
    for op in "LGD":
        ab = {}
        for base in ("10", "01"):
            ca = k4_coefficient(op, 2, 64, BASES_2D[base], (1, 0))
            cd = k4_coefficient(op, 2, 64, BASES_2D[base], (1, 1))
            ab[base] = (ca, 4.0 * cd - 2.0 * ca)       # a, b from the two directions
        A = np.array([[1.0, 1.0],
                      [ab["10"][1] - 2 * ab["10"][0], ab["01"][1] - 2 * ab["01"][0]]])
        c = np.linalg.solve(A, [1.0, 0.0])
        np.testing.assert_allclose(c, GOLD["isotropic_weights"]["2d"]["w"], rtol=5e-3)


@pytest.mark.parametrize("op", ["L", "G", "D"])
@pytest.mark.parametrize("base", ["100", "010", "001"])
def test_symbol_3d_bases(op, base):
    g = GOLD["3d"][op + base]
    for m in DIRS_3D:
        c = k4_coefficient(op, 3, 32, BASES_3D[base], m)
        assert c == pytest.approx(printed(g["a"], g["b"], m), rel=5e-3, abs=5e-4), (op, base, m)


@pytest.mark.parametrize("op", ["L", "G", "D"])
def test_symbol_3d_isotropic_families(op):
    """Every weight set on the printed solution family is isotropic at k^4:
    the three zero-weight solutions and L_{5,6,1}, L_{7,6,2}, L_{4,4,1}."""
    sets = (GOLD["isotropic_weights"]["3d_zero_weight_solutions"]["w"] +
            GOLD["isotropic_weights"]["3d_all_shells_examples"]["w"])
    a = GOLD["3d"][op + "100"]["a"]
    for w in sets:
        cs = [k4_coefficient(op, 3, 32, tuple(w), m) for m in DIRS_3D]
        np.testing.assert_allclose(cs, a, rtol=5e-3, err_msg="%s %s" % (op, w))
        # and the printed constraint holds for the weights
        con = GOLD["constraints"][op + "3d"]
        assert sum(c * x for c, x in zip(con["coef"], w)) == pytest.approx(con["rhs"])
        assert sum(w) == pytest.approx(1.0)


def test_standard_3d_bases_are_anisotropic():
    for op in "LGD":
        cs = [k4_coefficient(op, 3, 32, (1.0, 0.0, 0.0), m) for m in DIRS_3D]
        assert max(cs) - min(cs) > 0.05 * abs(cs[0])


# ---------------------------------------------------------------- polynomials


def _interior(dim, n, r=2):
    s = slice(r, n - r)
    return (s, s) if dim == 2 else (s, s, s)


def _poly(dim, n, h, coefs):
    """Random polynomial (degree <= 4) evaluated on the lattice, plus its
    derivatives computed symbolically from the coefficient table."""
    import sympy as sp
    xs = sp.symbols("x y z")[:dim]
    expr = 0
    rng = np.random.default_rng(coefs)
    from itertools import product
    for powers in product(range(5), repeat=dim):
        if sum(powers) <= 4:
            term = 1
            for v, pw in zip(xs, powers):
                term = term * v ** pw
            expr += float(rng.uniform(-1, 1)) * 0.05 * term
    return xs, expr


def _eval(dim, n, h, xs, expr):
    import sympy as sp
    f = sp.lambdify(xs, expr, "numpy")
    X = [g * h for g in _grid(dim, n)]
    out = f(*X)
    return np.broadcast_to(np.asarray(out, dtype=np.float64), X[0].shape).copy()


@pytest.mark.parametrize("dim,w,iso", [(2, (1, 0, 0), False), (2, (2 / 3, 1 / 3, 0), True),
                                       (3, (1 / 3, 2 / 3, 0), True)])
def test_laplacian_taylor_exact_on_quartics(dim, w, iso):
    """Sec. 4.1: L_{1,0} = lap + h^2/12 (psi_xxxx + psi_yyyy) and
    L_{2,1} = lap + h^2/12 bilap, exactly on polynomials of degree 4 (no higher
    derivatives survive); the 3D 18-point L_{1,2,0} has the same isotropic form
    (its symbol is -k^2 + k^4/12)."""
    import sympy as sp
    n, h = 12, 0.7
    xs, e = _poly(dim, n, h, 11 + dim)
    lap = sum(sp.diff(e, v, 2) for v in xs)
    if iso:
        lead = sum(sp.diff(lap, v, 2) for v in xs)
    else:
        lead = sum(sp.diff(e, v, 4) for v in xs)
    want = _eval(dim, n, h, xs, lap + h * h / 12 * lead)
    p = _params(dim, n, w, bc=oracle.NOFLUX, h=h)
    got = oracle.laplacian(p, _eval(dim, n, h, xs, e))
    sl = _interior(dim, n, 1)
    np.testing.assert_allclose(got[sl], want[sl], atol=1e-10)


@pytest.mark.parametrize("dim,bases", [(2, BASES_2D), (3, BASES_3D)])
def test_grad_square_exact_on_quadratics(dim, bases):
    """Every base of G is |grad psi|^2 exactly on quadratic fields (central
    differences along each shell direction are exact there).  With the printed
    1/(144 h^2) the <111> base would return |grad psi|^2 / 9: the 1/(16 h^2)
    reading is the one that passes."""
    import sympy as sp
    n, h = 10, 0.9
    rng = np.random.default_rng(5)
    xs = sp.symbols("x y z")[:dim]
    e = sum(float(rng.uniform(-1, 1)) * v for v in xs) + sum(
        float(rng.uniform(-1, 1)) * a * b for i, a in enumerate(xs) for b in xs[i:])
    g2 = sum(sp.diff(e, v) ** 2 for v in xs)
    want = _eval(dim, n, h, xs, g2)
    f = _eval(dim, n, h, xs, e)
    for name, w in bases.items():
        got = oracle.grad_square(_params(dim, n, w, bc=oracle.NOFLUX, h=h), f)
        sl = _interior(dim, n, 1)
        np.testing.assert_allclose(got[sl], want[sl], atol=1e-11, err_msg=name)


@pytest.mark.parametrize("dim,bases", [(2, BASES_2D), (3, BASES_3D)])
def test_divergence_exact_alpha_linear_beta_quadratic(dim, bases):
    """div(alpha grad beta) is reproduced exactly by every base when alpha is
    linear and beta quadratic: the averaged alpha at a flux point is exact and
    the difference quotient is the exact directional derivative there."""
    import sympy as sp
    n, h = 10, 0.8
    rng = np.random.default_rng(9)
    xs = sp.symbols("x y z")[:dim]
    al = 1.5 + sum(float(rng.uniform(-1, 1)) * v for v in xs)
    be = sum(float(rng.uniform(-1, 1)) * v for v in xs) + sum(
        float(rng.uniform(-1, 1)) * a * b for i, a in enumerate(xs) for b in xs[i:])
    div = sum(sp.diff(al * sp.diff(be, v), v) for v in xs)
    want = _eval(dim, n, h, xs, div)
    A, B = _eval(dim, n, h, xs, al), _eval(dim, n, h, xs, be)
    for name, w in bases.items():
        got = oracle.divergence(_params(dim, n, w, bc=oracle.NOFLUX, h=h), A, B)
        sl = _interior(dim, n, 1)
        np.testing.assert_allclose(got[sl], want[sl], atol=1e-11, err_msg=name)
        # swapping the roles of alpha and beta must not pass
        bad = oracle.divergence(_params(dim, n, w, bc=oracle.NOFLUX, h=h), B, A)
        assert np.max(np.abs(bad[sl] - want[sl])) > 1e-3


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("bc", [oracle.PERIODIC, oracle.NOFLUX])
def test_divergence_conservative(dim, bc):
    """Every flux leaves one cell and enters another, so the divergence sums to
    zero over a periodic box and over a box with mirrored (no-flux) walls."""
    n = 9 if dim == 3 else 17
    rng = np.random.default_rng(3)
    shape = (n,) * dim
    A = 1.0 + rng.uniform(0, 1, shape)
    B = rng.uniform(-1, 1, shape)
    for w in ((1, 0, 0), (0, 1, 0), (0, 0, 1) if dim == 3 else (0.5, 0.5, 0)):
        d = oracle.divergence(_params(dim, n, w, bc=bc), A, B)
        assert abs(d.sum()) < 1e-11 * np.abs(d).sum()
