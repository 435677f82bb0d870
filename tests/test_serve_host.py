"""Host-side logic of the request loop (no GPU): the seeded trace, the wave
estimate used by the admission cap, and the policy switches."""
import pytest

from paper_2110_12448_amd import serve
from paper_2110_12448_amd import workloads as wl


def test_trace_is_seeded_and_mixed():
    a = serve.poisson_trace(n=24, seed=5)
    b = serve.poisson_trace(n=24, seed=5)
    assert [(r.arrival, r.steps, r.problem["nx"]) for r in a] == \
           [(r.arrival, r.steps, r.problem["nx"]) for r in b]
    assert all(x.arrival < y.arrival for x, y in zip(a, a[1:]))
    dims = {r.problem["dim"] for r in a}
    assert dims == {2, 3}
    for r in a:
        assert 2000 <= r.steps <= 10000
        if r.problem["dim"] == 2:
            assert r.problem["nx"] % 64 == 0 and 256 <= r.problem["nx"] <= 1024
        else:
            assert r.problem["nx"] in (128, 160, 192)


@pytest.mark.parametrize("shape,batched,want", [
    ((256, 256), False, 5 * 204),                # 2D alone: 1 wave per SIMD, 1-2 row segments
    ((1024, 1024), False, 18 * 170),             # 3 waves per SIMD (18^0.4 = 3.2)
    ((1024, 2048), False, 18 * 227),             # 4 (36^0.4 = 4.2)
    ((256, 256), True, 5 * 32),                  # batched: 60-column strips x 8-row segments
    ((1024, 1024), True, 18 * 128),
    ((2048, 2048), True, 35 * 137),              # longer alone (146 segments): 15 rows
    # 3D: 14 z rows in 16 waves; 2 strips of 60 in 10 segments of 13 rows
    # and a thin strip (4 groups of 16 lanes, 62 z rows per tile) in 15
    # segments of at most 9: 245 workgroups in one round
    ((128, 128, 128), False, (2 * 10 * 10 + 3 * 15) * 16),
    # 4 strips of 60 in 3 segments and a thin one (3 groups of 21 lanes, 46
    # z rows per tile) in 4: 252 workgroups in one round
    ((256, 256, 256), False, (4 * 19 * 3 + 6 * 4) * 16),
])
def test_estimated_waves(shape, batched, want):
    pr = wl.problem(len(shape), shape, noise=0.0)
    assert serve.estimated_waves(pr, batched=batched) == want


def test_policy_switches_validated():
    with pytest.raises(ValueError):
        serve.Server(1 << 30, order="lifo")
    s = serve.Server(1 << 30, order="sjf", max_waves=8192, streams=4, autotune_steps=5)
    assert s.order == "sjf" and s.n_streams == 4 and s.max_waves == 8192
