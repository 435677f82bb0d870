"""The tip / solid-fraction reduction (pf_tip_state) on lattices large enough
that its grid is capped and every wave strides over several column runs:
against the definitions (Sec. 4.3.2, 6.2.1: the most advanced phi = 0
crossing along y, linear interpolation between the two cells, ties to the
smallest linear index; the solid fraction (1/N) sum (1 + phi)/2) evaluated
with numpy on the fields the solve read back.  FP64 fields, so both sides see
the same psi; they differ only in tanh's last bits and in summation order."""
import math

import numpy as np
import pytest

from paper_2110_12448_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _pf():
    from paper_2110_12448_amd import pfiso
    return pfiso


def tip_by_definition(phi, h):
    """(y, linear index) of the most advanced crossing, or None."""
    p = phi if phi.ndim == 3 else phi[None]
    nz, ny, nx = p.shape
    f0, f1 = p[:, :-1, :], p[:, 1:, :]
    l, j, x = np.nonzero((f0 >= 0.0) & (f1 < 0.0))
    if l.size == 0:
        return None
    a, b = f0[l, j, x], f1[l, j, x]
    y = (j + a / (a - b)) * h
    idx = x + nx * (j + ny * l.astype(np.int64))
    order = np.lexsort((idx, -y))          # largest y first, then smallest index
    return float(y[order[0]]), int(idx[order[0]]), y, idx


@pytest.mark.parametrize("case", ["2d_4096x8448", "3d_336cubed"])
def test_reduction_at_grid_cap_matches_definition(case):
    """4096 x 8448 (16 896 column runs of 32 rows) and 336^3 (22 176): more
    than the 4 x 4096 waves of the capped grid, so some waves take a second
    run."""
    pf = _pf()
    if case == "2d_4096x8448":
        pr = wl.config_directional_2d(nx=4096, ny=8448, noise=0.0)
    else:
        pr = wl.config_polycrystal_3d(n=336, noise=0.0)
    print("gpu case: reduction at scale %s FP64" % case, flush=True)
    s = pf.Solver(pr, precision=pf.PF_F64)
    s.step(5)
    t = s.tip_state()
    phi, _, _, _ = s.read_fields()
    s.close()
    h = pr["h"]
    ref = tip_by_definition(phi, h)
    assert ref is not None and t["found"] == 1
    y_ref, idx_ref, ys, idxs = ref
    assert abs(t["y_frame"] - y_ref) <= 1e-9, (t["y_frame"], y_ref)
    if t["index"] != idx_ref:
        # only a near-tie may pick another cell: its own height must equal the maximum
        k = np.nonzero(idxs == t["index"])[0]
        assert k.size == 1 and abs(ys[k[0]] - y_ref) <= 1e-9, (t["index"], idx_ref)
    nx = pr["nx"]
    assert t["x"] == pytest.approx((t["index"] % nx) * h, abs=1e-12)
    fs_ref = float(np.sum((1.0 + phi) * 0.5) / phi.size)
    assert abs(t["solid_fraction"] - fs_ref) <= 1e-10, (t["solid_fraction"], fs_ref)
    assert t["nonfinite"] == 0
    assert 0.0 < fs_ref < 1.0 and math.isfinite(y_ref)
