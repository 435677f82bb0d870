"""Continuous-batching server: every served result is bitwise the result of
the same request run alone and matches the FP64 oracle's explicit step on the
same inputs (FP64 within 1e-10, FP32 within 1e-5 in phi and U); admission
respects the HBM budget."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


POLICIES = [dict(), dict(max_waves=64, streams=3, autotune_steps=2),
            dict(streams=2, autotune_steps=2, batching=False),
            dict(max_waves=200, streams=2, order="sjf"),
            dict(streams=2, autotune_steps=2)]   # with mixed precisions


@pytest.mark.parametrize("policy", range(len(POLICIES)))
def test_served_equals_alone(policy):
    """Batching, a wave cap, several streams and autotuned geometries change
    when and where a solve runs, never its result."""
    from paper_2110_12448_amd import pfiso, serve
    reqs = serve.poisson_trace(n=10, rate=200.0, seed=9, frac_3d=0.3, steps=(20, 60),
                               sides_2d=(64, 192), sides_3d=(16, 24))
    if policy == len(POLICIES) - 1:
        # mixed precisions: FP64 and FP32 2D solves form separate batches
        for r in reqs[1::2]:
            r.precision = pfiso.PF_F64
    one = max(serve.workspace_bytes(r.problem, r.precision) for r in reqs)
    srv = serve.Server(hbm_budget_bytes=3 * one, chunk_steps=16, keep_fields=True, graph_steps=2,
                       **POLICIES[policy])
    print("serving %d requests, policy %s" % (len(reqs), POLICIES[policy]), flush=True)
    res = srv.run(reqs, realtime=False)
    assert sorted(r.rid for r in res) == list(range(len(reqs)))
    by = {r.rid: r for r in res}
    for q in reqs:
        r = by[q.rid]
        assert r.arrival <= r.admitted <= r.finished
        s = pfiso.Solver(q.problem, precision=q.precision)
        s.step(q.steps)
        phi, U, psi, _ = s.read_fields()
        s.close()
        assert np.array_equal(r.fields[2], psi) and np.array_equal(r.fields[1], U), q.rid
        pr = q.problem
        opsi, oU, st = oracle.step(oracle.Params.from_problem(pr), pr["psi0"], pr["U0"],
                                   pr["grain"], q.steps)
        d = max(float(np.max(np.abs(r.fields[0] - np.tanh(opsi / math.sqrt(2.0))))),
                float(np.max(np.abs(r.fields[1] - oU))))
        tol = 1e-10 if q.precision == pfiso.PF_F64 else 1e-5
        assert st.nonfinite == 0 and d <= tol, (q.rid, q.precision, d)
    summ = serve.summarize(res, max(r.finished for r in res), srv.busy_s)
    assert summ["p99_latency_s"] >= summ["p50_latency_s"] > 0


@pytest.mark.parametrize("shape", [(256, 256), (512, 768), (1024, 1024), (1024, 2048), (2048, 2048)])
def test_wave_estimate_matches_library_default(shape):
    """serve.estimated_waves restates the library's default 2D geometry (k
    waves per SIMD, k = round(R^0.4)): it must give the waves the library
    actually launches for a solve on its own."""
    import torch
    from paper_2110_12448_amd import pfiso, serve
    from paper_2110_12448_amd import workloads as wl
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    pr = wl.problem(2, shape, noise=0.0)
    s = pfiso.Solver(pr, precision=pfiso.PF_F32)
    k = -s.geometry()[0]
    s.close()
    strips = -(-shape[0] // 60)
    nsegs = max(1, min(shape[1], k * 4 * cus // strips))
    assert serve.estimated_waves(pr, cus=cus) == strips * nsegs
