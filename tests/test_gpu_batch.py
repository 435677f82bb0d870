"""Batched 2D stepping (pf_batch_*): every solve of a batch must be bitwise
identical to the same solve stepped on its own, with and without HIP-graph
replay, the moving frame, multi-grain maps and interleaved single steps, and
every member must match the FP64 oracle's explicit step (Sec. 4.3.1) on the
same inputs: FP64 within 1e-10, FP32 within 1e-5 in phi and U, frame shifts
equal."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_12448_amd import workloads as wl

pytestmark = pytest.mark.gpu

SIZES = [(64, 64), (97, 130), (200, 61), (128, 256), (31, 40), (256, 128)]


def _pf():
    from paper_2110_12448_amd import pfiso
    return pfiso


def problems(frame=False, multi=False, thermal="isothermal"):
    out = []
    for i, (nx, ny) in enumerate(SIZES):
        a0 = 45.0 * float(wl.uniform(4, 3, len(SIZES))[i])
        kw = dict(thermal=thermal, alpha0_deg=a0, seed=100 + i, seed_radius=min(nx, ny) / 6.0)
        if frame:
            kw.update(frame=1, shift_row=max(2, ny // 5))
        if multi:
            rot = np.stack([wl.rotation_2d(a0), wl.rotation_2d(a0 + 20.0)])
            g = np.zeros((ny, nx), dtype=np.int8)
            g[:, nx // 2:] = 1
            kw.update(rot=rot, grain=g)
        out.append(wl.problem(2, (nx, ny), **kw))
    return out


def solo(pr, prec, nsteps):
    pf = _pf()
    s = pf.Solver(pr, precision=prec)
    s.step(nsteps)
    phi, U, psi, _ = s.read_fields()
    fr = s.frame_state()
    s.close()
    return psi, U, fr


TOL = {0: 1e-5, 1: 1e-10}


def against_oracle(pr, prec, nsteps, phi, U, shift):
    p = oracle.Params.from_problem(pr)
    opsi, oU, st = oracle.step(p, pr["psi0"], pr["U0"], pr["grain"], nsteps)
    d = max(float(np.max(np.abs(phi - np.tanh(opsi / math.sqrt(2.0))))),
            float(np.max(np.abs(U - oU))))
    assert st.nonfinite == 0
    assert shift == st.shift, (shift, st.shift)
    assert d <= TOL[prec], (pr["nx"], pr["ny"], nsteps, d)
    return d


def check_batch(prs, prec, plan, graph=0, oracle_check=True):
    """plan: list of ('b', n) batch steps or ('s', i, n) single steps of solve i."""
    pf = _pf()
    print("batch of %d solves prec=%d graph=%d plan=%s" % (len(prs), prec, graph, plan), flush=True)
    ss = [pf.Solver(pr, precision=prec) for pr in prs]
    b = pf.Batch(ss, graph_steps=graph)
    total = [0] * len(prs)
    for item in plan:
        if item[0] == "b":
            b.step(item[1])
            total = [t + item[1] for t in total]
        else:
            ss[item[1]].step(item[2])
            total[item[1]] += item[2]
            ss[0].tip_state()          # eager work between launches
    for i, pr in enumerate(prs):
        phi, U, psi, _ = ss[i].read_fields()
        fr = ss[i].frame_state()
        rpsi, rU, rfr = solo(pr, prec, total[i])
        assert np.array_equal(psi, rpsi) and np.array_equal(U, rU), (i, total[i])
        assert fr == rfr
        if oracle_check:
            d = against_oracle(pr, prec, total[i], phi, U, fr[0])
            print("member %d %dx%d: %d steps, max diff vs oracle %.2e" %
                  (i, pr["nx"], pr["ny"], total[i], d), flush=True)
    b.close()
    for s in ss:
        s.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_equals_solo(prec):
    check_batch(problems(), prec, [("b", 25)])


def test_batch_frozen_moving_frame():
    prs = problems(frame=True, thermal="frozen")
    check_batch(prs, 0, [("b", 30)])


def test_batch_multigrain():
    check_batch(problems(multi=True), 0, [("b", 20)])


@pytest.mark.parametrize("graph,prec", [(2, 0), (6, 0), (6, 1)])
def test_batch_graph_replays(graph, prec):
    """Graph replays interleaved with eager work and direct launches."""
    prs = problems(frame=True, thermal="frozen") if graph == 6 else problems()
    check_batch(prs, prec, [("b", 13), ("s", 2, 1), ("b", 24), ("s", 0, 3), ("b", 7)], graph=graph)


def test_batch_interleaved_single_steps():
    check_batch(problems(), 1, [("b", 10), ("s", 3, 4), ("b", 10), ("s", 1, 1), ("b", 3)])


def test_batch_of_one_replays_a_single_solve():
    """A single small solve replayed from a graph (6-launch epochs, moving
    frame) equals the same solve stepped launch by launch."""
    prs = problems(frame=True, thermal="frozen")[:1]
    check_batch(prs, 0, [("b", 37), ("s", 0, 2), ("b", 12)], graph=6)


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_large_members_frozen_frame_graph_vs_oracle(prec):
    """Members of 512 x 768 and 640 x 512 beside small ones, frozen gradient,
    moving frame, graph replay (6-launch epochs) with eager work between
    replays: 102 steps, every member against the oracle."""
    sizes = [(512, 768), (640, 512), (96, 160), (256, 256)]
    prs = []
    for i, (nx, ny) in enumerate(sizes):
        a0 = 45.0 * float(wl.uniform(4, 11, len(sizes))[i])
        prs.append(wl.problem(2, (nx, ny), alpha0_deg=a0, seed=300 + i, frame=1,
                              shift_row=12, seed_radius=14.0))
    check_batch(prs, prec, [("b", 60), ("s", 3, 2), ("b", 40)], graph=6)


def test_batch_full_workload_autotuned_graph_vs_oracle():
    """The batched workload itself (64 solves, sides 256..1024, 28 M cells, frozen
    gradient) in the launch configuration the benchmark times: the segment
    length pf_batch_autotune picks for the whole batch and 10-launch graph
    epochs.  One replay and 3 eager steps, then every member against the
    oracle (FP32 within 1e-5)."""
    pf = _pf()
    prs = wl.config_batched_2d()
    ss = [pf.Solver(pr, precision=pf.PF_F32) for pr in prs]
    b = pf.Batch(ss, graph_steps=10)
    seg = b.autotune(5)
    print("batched workload: %d solves, rows per segment %d" % (len(prs), seg), flush=True)
    b.step(13)
    worst = 0.0
    for i, pr in enumerate(prs):
        phi, U, _, _ = ss[i].read_fields()
        fr = ss[i].frame_state()
        worst = max(worst, against_oracle(pr, 0, 13, phi, U, fr[0]))
        if i % 16 == 15:
            print("members 0..%d checked, max diff %.2e" % (i, worst), flush=True)
    b.close()
    for s in ss:
        s.close()
