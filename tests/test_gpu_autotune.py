"""Tile autotuners (pf_autotune, pf_batch_autotune) through the C ABI: the
choice is a legal launch geometry, the trials leave the solve where it was
(fields, step count and frame untouched), and a solve stepped after tuning is
bitwise the one stepped without tuning."""
import numpy as np
import pytest

from paper_2110_12448_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _pf():
    from paper_2110_12448_amd import pfiso
    return pfiso


def _state(s):
    phi, U, psi, g = s.read_fields()
    return psi, U, g, s.frame_state()


def _same(a, b):
    return all(np.array_equal(x, y) if isinstance(x, np.ndarray) else x == y for x, y in zip(a, b))


CASES = [
    # dim, problem builder, precision, steps before tuning, steps after
    (2, lambda: wl.config_small_2d(20.0, n=97), 0, 7, 40),
    (2, lambda: wl.config_small_2d(0.0, n=128, frame=1, shift_row=12), 1, 5, 30),
    (3, lambda: wl.problem(3, (40, 36, 30), seed_radius=5.0), 0, 3, 12),
    (3, lambda: wl.problem(3, (33, 29, 17), seed_radius=4.0, bc=(1, 0, 1)), 1, 2, 10),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_autotune_keeps_state_and_results(case):
    dim, build, prec, before, after = CASES[case]
    pf = _pf()
    pr = build()
    print("autotune case %d: %dD prec=%d" % (case, dim, prec), flush=True)
    ref = pf.Solver(pr, precision=prec)
    ref.step(before + after)
    want = _state(ref)
    ref.close()
    assert np.all(np.isfinite(want[0])) and np.all(np.isfinite(want[1]))

    s = pf.Solver(pr, precision=prec)
    s.step(before)
    pre = _state(s)
    seg, zt = s.autotune(3)
    assert s.geometry() == (seg, zt)
    assert _same(_state(s), pre)
    if dim == 2:
        assert -64 <= seg <= -1 and zt == 1      # waves per SIMD
    else:
        assert 4 <= seg <= 256 and 1 <= zt <= (2 if prec == 1 else 14)
    s.tune(seg, zt)                      # the choice is accepted as a manual setting
    s.step(after)
    assert _same(_state(s), want)
    s.close()


def test_autotune_rejects_bad_trial_count():
    pf = _pf()
    s = pf.Solver(wl.config_small_2d(0.0, n=32), precision=pf.PF_F32)
    for bad in (0, (1 << 20) + 1):
        with pytest.raises(pf.PFError) as e:
            s.autotune(bad)
        assert e.value.code == pf.PF_ERR_ARG
    s.close()


@pytest.mark.parametrize("frame,graph,prec", [(False, 0, 0), (True, 6, 0), (True, 6, 1)])
def test_batch_autotune(frame, graph, prec):
    pf = _pf()
    sizes = [(64, 64), (97, 130), (200, 61), (31, 40)]
    prs = []
    for i, (nx, ny) in enumerate(sizes):
        kw = dict(alpha0_deg=11.0 * i, seed=200 + i, seed_radius=min(nx, ny) / 6.0)
        if frame:
            kw.update(thermal="frozen", frame=1, shift_row=max(2, ny // 5))
        prs.append(wl.problem(2, (nx, ny), **kw))
    print("batch autotune frame=%d graph=%d prec=%d" % (frame, graph, prec), flush=True)
    ss = [pf.Solver(pr, precision=prec) for pr in prs]
    b = pf.Batch(ss, graph_steps=graph)
    b.step(6)
    pre = [_state(s) for s in ss]
    seg = b.autotune(3)
    assert seg in (0, 4, 6, 8, 12, 16, 24, 32)
    assert all(_same(_state(s), p) for s, p in zip(ss, pre))
    b.step(18)
    for pr, s in zip(prs, ss):
        r = pf.Solver(pr, precision=prec)
        r.step(24)
        assert _same(_state(s), _state(r))
        r.close()
    b.close()
    for s in ss:
        s.close()
