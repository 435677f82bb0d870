"""Continuous-batching request loop over the C ABI.

Requests (one phase-field solve each: a problem dictionary, a step count and a
precision) arrive over time.  The server keeps every admitted solve's fields
resident in HBM and admits queued requests in arrival order while its HBM
budget allows and, optionally, while the active solves occupy fewer waves than
a cap (so that requests run close to first-come first-served instead of all
sharing the GPU at once).  It advances all active solves tick by tick: the
active 2D solves of one kind share one batched launch per step (pf_batch_*);
3D solves and 2D solves on the full anti-trapping current or two-point
divergences are launched on their own, spread over a pool of HIP streams so
that solves too small to fill the chip overlap.  Launch geometries can come
from the autotuners (pf_autotune per shape class, pf_batch_autotune per batch
kind).  A tick stops at the first step count an active solve needs, so every
request receives exactly its steps; finished requests are read back and their
memory released before the next admission.  Because batched stepping is
bitwise identical to solo stepping and results do not depend on the launch
geometry, each result is the same alone and in the mix.

All arithmetic runs in libpfiso.so; this module only schedules.
"""
from __future__ import annotations

import ctypes as C
import sys
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import pfiso
from . import workloads as wl


@dataclass
class Request:
    rid: int
    arrival: float          # seconds on the trace clock
    problem: dict
    steps: int
    precision: int = pfiso.PF_F32


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    cells: int
    dim: int
    fields: Optional[tuple] = None   # (phi, U, psi) if kept
    tip: Optional[dict] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def workspace_bytes(prob: dict, precision: int) -> int:
    lib = pfiso.load()
    p, keep = pfiso.make_params(prob, precision)
    return int(lib.pf_workspace_bytes(C.byref(p)))


def _batchable(prob: dict) -> bool:
    """Batched launches run the approximated current on shell divergences."""
    return prob["dim"] == 2 and not prob.get("antitrapping", 0) and not prob.get("two_point", 0)


def _geom3d_blocks(nx: int, ny: int, nz: int, seg: int, ztile: int) -> int:
    """Workgroups of one 3D step launch (the library's tile layout: strips of
    60 columns, the nx mod 60 remainder as a thin strip of 3 lane groups (13
    to 17 columns) or 4 (up to 12) with (ztile + 2) * groups - 2 z rows per
    tile, z tiles of ztile rows, segments of at most seg rows, 3/4 of that in
    the thin strip)."""
    nw = ztile + 2
    nfull, r = nx // 60, nx % 60
    gr = 0 if r == 0 else (4 if r <= 12 else (3 if r <= 17 else 1))
    thin_nzt = 0
    if r == 0 or gr >= 3:
        nstrips = nfull
        if r > 0:
            thin_nzt = -(-nz // (nw * gr - 2))
    else:
        nstrips = -(-nx // 60)
    thin_nsegs = -(-ny // max(1, seg * 3 // 4)) if thin_nzt else 0
    return nstrips * -(-nz // ztile) * -(-ny // seg) + thin_nzt * thin_nsegs


def estimated_waves(prob: dict, batched: bool = False, cus: int = 256) -> int:
    """Waves one step launch of this solve occupies at the library's default
    FP32 geometry on a device of `cus` compute units: the measure of how much
    of the chip a solve fills.  60 output columns per wave; in 2D k =
    round(R^0.4) waves per SIMD with R = strips * ny / SIMDs, at most one
    segment per row, and inside a batch segments of that length but at least
    8 rows; in 3D workgroups of 14 z rows in 16 waves (one per CU), with the
    segment count that minimises rounds x (rows + 2.5)."""
    strips = -(-prob["nx"] // 60)
    if prob["dim"] == 2:
        ny, simds = prob["ny"], 4 * cus
        k = max(1, int(np.floor((strips * ny / simds) ** 0.4 + 0.5)))
        nsegs = max(1, min(ny, k * simds // strips))
        if batched:
            nsegs = -(-ny // max(8, -(-ny // nsegs)))
        return strips * nsegs
    nx, ny, nz = prob["nx"], prob["ny"], prob["nz"]
    zt = min(14, nz)
    best, best_cost = ny, None
    for n in range(1, max(1, ny // 4) + 1):
        rows = -(-ny // n)
        blocks = _geom3d_blocks(nx, ny, nz, rows, zt)
        cost = -(-blocks // cus) * (rows + 2.5)
        if best_cost is None or cost < best_cost - 1e-9:
            best, best_cost = rows, cost
    return _geom3d_blocks(nx, ny, nz, best, zt) * (zt + 2)


def _work(r: Request) -> int:
    return int(r.problem["nx"]) * int(r.problem["ny"]) * int(r.problem["nz"]) * int(r.steps)


def _shape_class(prob: dict, precision: int):
    return (prob["dim"], prob["nx"], prob["ny"], prob["nz"], precision,
            int(prob.get("antitrapping", 0)), int(prob.get("two_point", 0)))


def _kind(prob: dict, precision: int):
    return (precision, prob["lT"] > 0.0, int(prob["frame"]), np.asarray(prob["rot"]).reshape(-1, 9).shape[0] > 1)


@dataclass
class _Active:
    req: Request
    solver: pfiso.Solver
    admitted: float
    done: int = 0
    nbytes: int = 0
    waves: int = 0


class Server:
    def __init__(self, hbm_budget_bytes: int, chunk_steps: int = 200, device: str = "cuda:0",
                 keep_fields: bool = False, graph_steps: int = 0, batching: bool = True,
                 progress: int = 0, max_waves: Optional[int] = None, streams: int = 1,
                 autotune_steps: int = 0, order: str = "fifo"):
        """max_waves: admit a request only while the active solves occupy fewer
        waves than this (estimated_waves; None: the HBM budget alone decides).
        streams: HIP streams the solves are spread over (batched solves share
        the first, the others take the rest in turn), so that launches of
        solves too small to fill the chip can run side by side.
        autotune_steps > 0: each unbatched solve takes the launch geometry
        pf_autotune finds for its shape class (timed once per class, on the
        first admission), and each batch kind the segment length
        pf_batch_autotune finds for the first batch of 4 or more solves.
        order: "fifo" admits in arrival order, "sjf" the least work first."""
        if order not in ("fifo", "sjf"):
            raise ValueError(order)
        self.order = order
        self.progress = int(progress)    # > 0: a line on stderr every `progress` results
        self.max_waves = max_waves
        self.n_streams = max(1, int(streams))
        self.autotune_steps = int(autotune_steps)
        self.budget = int(hbm_budget_bytes)
        self.batching = bool(batching)
        self.chunk = int(chunk_steps)
        self.device = device
        self.keep_fields = keep_fields
        self.graph_steps = int(graph_steps)
        self.busy_s = 0.0

    def run(self, requests: List[Request], realtime: bool = True) -> List[Result]:
        """Serve a finite trace.  realtime=False advances the trace clock to
        the next arrival whenever the server is idle instead of sleeping, and
        measures service on the wall clock otherwise (arrival times shift)."""
        import torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        queue: List[Request] = []
        active: List[_Active] = []
        results: List[Result] = []
        used = 0
        t0 = time.perf_counter()
        skew = 0.0                       # idle time skipped in simulated mode
        batches: Dict[tuple, tuple] = {}  # kind -> (member rids, pfiso.Batch)
        dev = torch.device(self.device)
        pool = [torch.cuda.current_stream(dev)] + [torch.cuda.Stream(dev)
                                                   for _ in range(self.n_streams - 1)]
        turn = 0
        geo: Dict[tuple, tuple] = {}      # shape class -> (rows per segment, z rows)
        batch_seg: Dict[tuple, int] = {}  # batch kind -> rows per segment (0: members' own)
        waves = 0

        def now():
            return time.perf_counter() - t0 + skew

        while pending or queue or active:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.pop(0))
            # admission by HBM budget, arrival order (a request larger than
            # the whole budget is admitted alone); "sjf" admits the queued
            # request with the least work (cells x steps) first
            if self.order == "sjf":
                queue.sort(key=lambda q: (_work(q), q.arrival, q.rid))
            while queue:
                r = queue[0]
                need = workspace_bytes(r.problem, r.precision)
                if used + need > self.budget and active:
                    break
                if self.max_waves is not None and waves >= self.max_waves and active:
                    break
                queue.pop(0)
                batched = self.batching and _batchable(r.problem)
                if batched or len(pool) == 1:
                    st = pool[0]
                else:
                    st = pool[1 + turn % (len(pool) - 1)]
                    turn += 1
                s = pfiso.Solver(r.problem, precision=r.precision, device=self.device, stream=st)
                if self.autotune_steps and not batched:
                    cls = _shape_class(r.problem, r.precision)
                    if cls not in geo:
                        geo[cls] = s.autotune(self.autotune_steps)
                    else:
                        s.tune(*geo[cls])
                active.append(_Active(r, s, now(), 0, need, estimated_waves(
                    r.problem, batched=self.batching and _batchable(r.problem))))
                used += need
                waves += active[-1].waves
            if not active:
                if pending:
                    wait = pending[0].arrival - now()
                    if wait > 0:
                        if realtime:
                            time.sleep(wait)
                        else:
                            skew += wait
                continue
            # one tick: advance every active solve by the same number of steps
            tick = min(self.chunk, min(a.req.steps - a.done for a in active))
            tb = time.perf_counter()
            groups: Dict[tuple, List[_Active]] = {}
            for a in active:
                if self.batching and _batchable(a.req.problem):
                    groups.setdefault(_kind(a.req.problem, a.req.precision), []).append(a)
            for kind, members in groups.items():
                rids = tuple(m.req.rid for m in members)
                if kind not in batches or batches[kind][0] != rids:
                    if kind in batches:
                        batches[kind][1].close()
                    seg = batch_seg.get(kind, 0)
                    if seg:
                        for m in members:
                            if m.solver.geometry()[0] != seg:
                                m.solver.tune(seg, 1)
                    b = pfiso.Batch([m.solver for m in members], graph_steps=self.graph_steps)
                    if self.autotune_steps and kind not in batch_seg and len(members) >= 4:
                        batch_seg[kind] = b.autotune(self.autotune_steps)
                    batches[kind] = (rids, b)
                batches[kind][1].step(tick)
            for kind in [k for k in batches if k not in groups]:
                batches.pop(kind)[1].close()
            for a in active:
                if not (self.batching and _batchable(a.req.problem)):
                    a.solver.step(tick)
                a.done += tick
            torch.cuda.synchronize()
            self.busy_s += time.perf_counter() - tb
            # retire finished requests
            still = []
            for a in active:
                if a.done < a.req.steps:
                    still.append(a)
                    continue
                fields = None
                if self.keep_fields:
                    phi, U, psi, _ = a.solver.read_fields()
                    fields = (phi, U, psi)
                tip = a.solver.tip_state(allow_nonfinite=True)
                res = Result(a.req.rid, a.req.arrival, a.admitted, now(), a.req.steps,
                             int(np.prod(a.solver.shape)), a.req.problem["dim"], fields, tip)
                results.append(res)
                if self.progress and len(results) % self.progress == 0:
                    print("served %d requests, %.1f s" % (len(results), now()), file=sys.stderr,
                          flush=True)
                for kind in list(batches):
                    if a.req.rid in batches[kind][0]:
                        batches.pop(kind)[1].close()
                a.solver.close()
                used -= a.nbytes
                waves -= a.waves
            active = still
        for _, b in batches.values():
            b.close()
        return results


def poisson_trace(n: int = 300, rate: float = 20.0, seed: int = 5, frac_3d: float = 0.2,
                  steps=(2000, 10000), sides_2d=(256, 1024), sides_3d=(128, 160, 192),
                  precision: int = pfiso.PF_F32) -> List[Request]:
    """Seeded request trace: exponential inter-arrival times (mean 1/rate),
    2D sides uniform on multiples of 64 in sides_2d, 3D sides from sides_3d,
    step counts uniform in `steps`, misorientations uniform in [0, 45] deg."""
    u = wl.uniform(seed, 11, 6 * n).reshape(n, 6)
    t = 0.0
    out = []
    lo, hi = sides_2d[0] // 64, sides_2d[1] // 64
    for i in range(n):
        t += -np.log(1.0 - u[i, 0]) / rate
        nst = int(steps[0] + u[i, 1] * (steps[1] - steps[0] + 1))
        a0 = 45.0 * float(u[i, 2])
        if u[i, 3] < frac_3d:
            side = int(sides_3d[min(int(u[i, 4] * len(sides_3d)), len(sides_3d) - 1)])
            rot = wl.random_rotations((seed * 7919 + i) & 0xFFFF, 1)
            prob = wl.problem(3, (side, side, side), rot=rot, seed=(seed * 101 + i) & 0xFFFF,
                              seed_shape="slab", seed_radius=5.0)
        else:
            side = 64 * (lo + min(int(u[i, 4] * (hi - lo + 1)), hi - lo))
            prob = wl.problem(2, (side, side), alpha0_deg=a0, seed=(seed * 101 + i) & 0xFFFF)
        out.append(Request(i, t, prob, nst, precision))
    return out


def summarize(results: List[Result], makespan: float, busy: float) -> dict:
    """p50/p99 time-to-result, throughput, and the offered load: device-busy
    time over the span of arrivals (> 1 means requests arrive faster than the
    GPU can finish them, so queueing dominates the tail)."""
    lat = np.array([r.latency for r in results])
    work = float(sum(r.cells * r.steps for r in results))
    span = max(r.arrival for r in results) - min(r.arrival for r in results)
    return {"requests": len(results), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "mean_latency_s": float(lat.mean()),
            "makespan_s": makespan, "cell_updates_per_s": work / makespan,
            "busy_fraction": busy / makespan, "arrival_span_s": span,
            "offered_load": busy / span if span > 0 else None}
