"""Throughput benchmark of the fused phase-field step on one MI355X.

Default workload: the 3D polycrystal, 256^3 lattice, FP32 fields, S-bar_{1,2,0}
(isotropic stencils with the approximated anti-trapping current), 8 grains
from a seeded Voronoi tessellation of the bottom plane with uniform random
cubic orientations (int8 grain map), frozen temperature, periodic x and z.
One benchmark step is one full time step of the hot path: one launch of the
fused psi/U kernel, which reads psi, U and the grain map and writes the next
psi and U.  Fields stay resident in HBM for the whole timed region.  The tip,
solid fraction and finiteness check are not part of the step: they come
from pf_tip_state on demand (timed separately, `tip_state_ms`).

Prints one JSON line (cell-updates/s) with a roofline entry for the step
kernel, the FP64 CPU oracle timed on a bounded sample of the same workload,
and the FP32 error against that oracle sample.

--workload directional2d runs the 2D directional solve (1024 x 2048, moving
frame, S-bar_{2,1}) instead; the other workloads are listed under --workload.
--copy-calibration runs a plain device copy of known size (the reference for
the HBM byte counters).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector (published; counts packed FP32 FMAs)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # the same vector units issuing one FP32 FMA per lane
# FP32 operations per cell-update of the 2D step as written in step2d.hip
# (FMA = 2, each transcendental = 1; index math, selects and cross-lane moves
# not counted): tanh 6, y-face flux 30, psi rate 112 (L 10, G 9, centre a_s
# 15, x-face flux 29, remainder 6, thermal 6, bulk, rate and alpha_A 20,
# update 2, the rest 15), U update 61 (links of D 22 and A 18, combined 4,
# sums, rate and update 17).
ALG_FLOPS_2D = 209
# compulsory bytes per cell-update: read psi, U; write psi, U (FP32)
ALG_BYTES_2D_F32 = 16
# FP32 operations per cell-update of the 3D step as written in step3d.hip
# (same counting rules): psi rate 343 (phi 6, L 37, G 30, centre a_s 39, three
# face fluxes 186 (the z face below is the wave below's z face above),
# remainder 17, thermal and rate 28), U update 187 (the alpha sums of the 9
# links a cell owns 2 x 57, their differences 18 and products 27, the
# exchange, sums and update 26, alpha_D 2).
ALG_FLOPS_3D = 530
# with the <111> shell (S-bar_{4,4,1}): + 32 for its Laplacian and gradient
# square terms, + 37 for its 4 owned divergence links (cube sums from the
# plaquette sums, differences, products, exchange)
ALG_FLOPS_3D_441 = 599
# read psi, U, the int8 grain; write psi, U
ALG_BYTES_3D_F32 = 17
# FP32 operations per cell-update of the 2D step under the three schemes of
# Table 1 (same counting rules; the full current adds three App. B gradients,
# the two-point faces replace the shell divergences)
SCHEME_FLOPS_2D = {"S10": 199, "S21": 295, "Sbar21": 209}
# Table 1: wall time of the whole isothermal run on a Tesla P100 (context)
PAPER_TABLE1_S = {"S10": 1359.0, "S21": 4612.0, "Sbar21": 3883.0}


def src_digest(paths):
    """Digest of the kernel sources' code: comments and whitespace removed, so
    that a documentation edit does not retire counters taken on the same
    kernel."""
    import re
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p)) as f:
            code = f.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


WORKLOADS = {
    "directional2d": dict(
        sources=["paper_2110_12448_amd/csrc/step2d.hip", "paper_2110_12448_amd/csrc/pf_device.hpp"],
        counters="profiles/step2d_directional_1024x2048_counters.json",
        kernel="step2d_kernel<float,frozen,frame>", flops=ALG_FLOPS_2D, bytes=ALG_BYTES_2D_F32,
        steps=20000, warmup=500, tune_steps=50, build=lambda wl: wl.config_directional_2d(),
        text="2D directional solidification, moving frame, 1024x2048, S-bar_{2,1}, FP32 "
             "fields"),
    "directional2d_8192": dict(
        sources=["paper_2110_12448_amd/csrc/step2d.hip", "paper_2110_12448_amd/csrc/pf_device.hpp"],
        counters="profiles/step2d_directional_8192x8192_counters.json",
        kernel="step2d_kernel<float,frozen,frame>", flops=ALG_FLOPS_2D, bytes=ALG_BYTES_2D_F32,
        steps=1000, warmup=50, cpu_steps=2, tune_steps=10,
        build=lambda wl: wl.config_directional_2d(nx=8192, ny=8192),
        text="2D directional solidification, moving frame, 8192x8192 (1 GiB of fields, beyond "
             "the 256 MB last-level cache), S-bar_{2,1}, FP32"),
    "polycrystal3d": dict(
        sources=["paper_2110_12448_amd/csrc/step3d.hip", "paper_2110_12448_amd/csrc/pf_device.hpp"],
        counters="profiles/step3d_polycrystal_256cubed_counters.json",
        kernel="step3d_kernel<float,frozen,multigrain>", flops=ALG_FLOPS_3D, bytes=ALG_BYTES_3D_F32,
        steps=1000, warmup=50, cpu_steps=3, tune_steps=10,
        build=lambda wl: wl.config_polycrystal_3d(),
        text="3D polycrystal, 256^3, 8 Voronoi grains with uniform random cubic orientations "
             "(int8 grain map), planar slab, frozen gradient, periodic x and z, "
             "S-bar_{1,2,0}, FP32 fields"),
    "polycrystal3d_441": dict(
        sources=["paper_2110_12448_amd/csrc/step3d.hip", "paper_2110_12448_amd/csrc/pf_device.hpp"],
        counters="profiles/step3d_polycrystal441_256cubed_counters.json",
        kernel="step3d_kernel<float,frozen,multigrain,shell111>", flops=ALG_FLOPS_3D_441,
        bytes=ALG_BYTES_3D_F32, steps=200, warmup=10, cpu_steps=2, tune_steps=8,
        build=lambda wl: wl.config_polycrystal_3d(scheme="iso441"),
        text="3D polycrystal, 256^3, 8 Voronoi grains, S-bar_{4,4,1} (27-point, <111> shell), FP32"),
    "polycrystal3d_512": dict(
        sources=["paper_2110_12448_amd/csrc/step3d.hip", "paper_2110_12448_amd/csrc/pf_device.hpp"],
        counters="profiles/step3d_polycrystal_512cubed_counters.json",
        kernel="step3d_kernel<float,frozen,multigrain>", flops=ALG_FLOPS_3D, bytes=ALG_BYTES_3D_F32,
        steps=40, warmup=4, cpu_steps=1, tune_steps=4, build=lambda wl: wl.config_polycrystal_3d(n=512),
        text="3D polycrystal, 512^3 (2.1 GiB of fields), 8 Voronoi grains, S-bar_{1,2,0}, FP32"),
}


# counter summary of the batched step kernel (64 solves, 32-row segments)
BATCH_COUNTERS = dict(
    sources=["paper_2110_12448_amd/csrc/step2d.hip", "paper_2110_12448_amd/csrc/pf_device.hpp"],
    counters="profiles/batch2d_64solves_counters.json")


def bench_batched(args):
    """64 uneven 2D solves (sides 256..1024) stepped by one launch per step
    (HIP graph of 10 launches), against the same solves stepped one at a time
    in FP32 and in FP64."""
    import torch
    from paper_2110_12448_amd import pfiso
    from paper_2110_12448_amd import workloads as wl
    prs = wl.config_batched_2d()
    cells = sum(p["nx"] * p["ny"] for p in prs)
    steps = args.steps or 500
    warm = args.warmup if args.warmup is not None else 20

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    ss = [pfiso.Solver(p, precision=pfiso.PF_F32) for p in prs]
    if args.batch_rows:
        # one fixed segment length for every member (profiling runs)
        for s in ss:
            s.tune(args.batch_rows, 1)
    b = pfiso.Batch(ss, graph_steps=10)
    b.step(warm)
    t_default = timed(lambda: b.step(steps))
    seg = args.batch_rows or b.autotune(20)
    print("bench: batched2d %d solves FP32, warmup %d, steps %d, geometry (%d, 1)" %
          (len(prs), warm, steps, seg), file=sys.stderr, flush=True)
    b.step(warm)
    t = timed(lambda: b.step(steps))
    batched = cells * steps / t
    b.close()
    solo_steps = max(10, steps // 5)
    t32 = timed(lambda: [s.step(solo_steps) for s in ss])
    for s in ss:
        s.close()
    ss = [pfiso.Solver(p, precision=pfiso.PF_F64) for p in prs]
    for s in ss:
        s.step(2)
    t64 = timed(lambda: [s.step(solo_steps // 2) for s in ss])
    for s in ss:
        s.close()
    out = {"metric": "phi+U cell-updates/s (batched)", "value": batched,
           "unit": "cell-updates/s", "n_gpus": 1, "steps": steps, "warmup": warm,
           "ms_per_step": t / steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "64 independent 2D solves, sides from {256,384,512,768,1024}, "
                                  "misorientation uniform in [0,45] deg, S-bar_{2,1}, one launch "
                                  "per step replayed from a HIP graph", "solves": len(prs),
                      "cells": cells},
           "autotuned_rows_per_segment": seg if not args.batch_rows else None,
           "rows_per_segment": seg,
           "default_segment_value": cells * steps / t_default,
           "one_at_a_time_f32": cells * solo_steps / t32,
           "one_at_a_time_f64": cells * (solo_steps // 2) / t64}
    # the batched step kernel is the same 2D step body: 209 flops and 16 B of
    # algorithmic traffic per cell-update
    tfl = ALG_FLOPS_2D * batched / 1e12
    gbs = ALG_BYTES_2D_F32 * batched / 1e9
    ctr = load_counters(BATCH_COUNTERS, (seg, 1))
    out["roofline"] = {"bound": "alu", "achieved": round(tfl, 3), "peak": PEAK_FP32_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(tfl / PEAK_FP32_TFLOPS, 4),
                       "frac_of_nonpacked_fp32": round(tfl / PEAK_FP32_NONPACKED_TFLOPS, 4),
                       "traffic": None if ctr is None else ctr["hbm_bytes_per_launch"],
                       "kernel": "batch2d_kernel<float,frozen>",
                       "kernel_ms": round(t / steps * 1e3, 5),
                       "counters_kernel_ns": None if ctr is None else ctr["avg_duration_ns"],
                       "hbm_algorithmic_GBs": round(gbs, 1),
                       "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}
    print(json.dumps(out))


# counter summary of the S_{2,1} (full current, App. B) step kernel on 781^2
SCHEMES_COUNTERS = dict(
    sources=["paper_2110_12448_amd/csrc/step2d.hip", "paper_2110_12448_amd/csrc/pf_device.hpp"],
    counters="profiles/step2d_S21_781sq_counters.json")


def bench_schemes(args):
    """The three 2D schemes of Table 1 on the isothermal free-growth run
    (781^2, 20345 steps, FP32): the whole run timed per scheme, with the
    per-launch kernel time and the FP64 oracle of S_{2,1} on a bounded sample."""
    import numpy as np
    import torch
    from paper_2110_12448_amd import pfiso
    from paper_2110_12448_amd import workloads as wl
    steps = args.steps or wl.ISOTHERMAL_2D_STEPS
    warm = args.warmup if args.warmup is not None else 200
    nl = args.launch_sample or 200
    out_s = {}
    names = args.schemes.split(",")
    if "S21" not in names:
        print("schemes2d reports S21: include it in --schemes", file=sys.stderr)
        sys.exit(2)
    geo = None
    for name in [n for n in ("S10", "S21", "Sbar21") if n in names]:
        pr = wl.config_isothermal_2d(**wl.SCHEMES_2D[name])
        cells = pr["nx"] * pr["ny"]
        s = pfiso.Solver(pr, precision=pfiso.PF_F32)
        st = s.stream
        if name == "S21":
            geo = s.geometry()
        print("bench: schemes2d %s %dx%d FP32, warmup %d, steps %d, geometry %s" %
              (name, pr["nx"], pr["ny"], warm, steps, s.geometry()), file=sys.stderr, flush=True)
        s.step(warm)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        s.step(steps)
        e1.record(st)
        torch.cuda.synchronize()
        run_s = e0.elapsed_time(e1) / 1e3
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(nl)]
        for a, b in evs:
            a.record(st)
            s.step(1)
            b.record(st)
        torch.cuda.synchronize()
        kern_ms = sum(a.elapsed_time(b) for a, b in evs) / nl
        tip = s.tip_state()
        s.close()
        # launches run back to back in the timed run: its average step is the
        # kernel's average duration (isolated launches add event overhead)
        step_ms = run_s * 1e3 / steps
        tf = SCHEME_FLOPS_2D[name] * cells / (step_ms / 1e3) / 1e12
        out_s[name] = {"run_s": run_s, "cell_updates_per_s": cells * steps / run_s,
                       "kernel_ms": round(step_ms, 5),
                       "kernel_ms_isolated_launch": round(kern_ms, 5),
                       "flops_per_cell": SCHEME_FLOPS_2D[name],
                       "achieved_TFLOPs": round(tf, 3),
                       "alu_frac": round(tf / PEAK_FP32_TFLOPS, 4),
                       "tip_y": tip["y_lab"], "solid_fraction": tip["solid_fraction"],
                       "paper_p100_run_s": PAPER_TABLE1_S[name]}
    if "S10" in out_s:
        for name in out_s:
            out_s[name]["time_vs_S10"] = round(out_s[name]["run_s"] / out_s["S10"]["run_s"], 3)
    ctr = load_counters(SCHEMES_COUNTERS, geo)
    pr = wl.config_isothermal_2d(**wl.SCHEMES_2D["S21"])
    cells = pr["nx"] * pr["ny"]
    main_s = out_s["S21"]
    cpu = None
    if not args.no_cpu:
        cpu, _, _, _, _ = cpu_baseline(pr, target_s=12.0, max_steps=200,
                                       label="781^2 isothermal S_{2,1}")
    tf = main_s["achieved_TFLOPs"]
    out = {"metric": "phi+U cell-updates/s", "value": main_s["cell_updates_per_s"],
           "unit": "cell-updates/s", "n_gpus": 1, "steps": steps, "warmup": warm,
           "ms_per_step": main_s["run_s"] / steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "2D isothermal free growth, 781x781, h/W 1.2, W/d0* 16, "
                                  "Omega 0.43, eps4 0.014, k 0.1, alpha0 30 deg, S_{2,1} (full "
                                  "anti-trapping, App. B), FP32; S_{1,0} and S-bar_{2,1} beside",
                      "nx": pr["nx"], "ny": pr["ny"], "h": pr["h"], "dt": pr["dt"],
                      "rows_per_segment": geo[0], "z_tile": geo[1]},
           "roofline": {"bound": "alu", "achieved": tf, "peak": PEAK_FP32_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(tf / PEAK_FP32_TFLOPS, 4),
                        "frac_of_nonpacked_fp32": round(tf / PEAK_FP32_NONPACKED_TFLOPS, 4),
                        "traffic": None if ctr is None else ctr["hbm_bytes_per_launch"],
                        "kernel": "step2d_kernel<float,isothermal,full-AT>",
                        "kernel_ms": main_s["kernel_ms"],
                        "counters_kernel_ns": None if ctr is None else ctr["avg_duration_ns"]},
           "cpu_baseline": cpu, "schemes": out_s}
    print(json.dumps(out))


def _copy_GBs(nbytes=1 << 30, reps=10):
    """Read + write bandwidth of a plain device-to-device copy (GB/s)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


# counter summary of the diffusion-only kernel on 8192^2 (HBM regime)
DIFFUSION_ROWS_PER_SEGMENT = 16
DIFFUSION_COUNTERS = dict(
    sources=["paper_2110_12448_amd/csrc/step2d.hip", "paper_2110_12448_amd/csrc/pf_device.hpp"],
    counters="profiles/step2d_diffusion_8192x8192_counters.json")


def bench_diffusion(args):
    """The diffusion-only step (psi held, U by D~ div[(1-phi) grad U]): the same
    16 bytes per cell as the full step with a fraction of its arithmetic, on
    8192^2 (fields beyond the last-level cache) and 1024x2048, FP32."""
    import torch
    from paper_2110_12448_amd import pfiso
    from paper_2110_12448_amd import workloads as wl
    steps = args.steps or 400
    warm = args.warmup if args.warmup is not None else 20
    nl = args.launch_sample or 100
    if "8192x8192" not in args.diffusion_sizes.split(","):
        print("diffusion2d reports the 8192x8192 lattice: include it in --diffusion-sizes",
              file=sys.stderr)
        sys.exit(2)
    res = {}
    geo = None
    sizes = [("8192x8192", wl.config_directional_2d(nx=8192, ny=8192)),
             ("1024x2048", wl.config_directional_2d())]
    for label, pr in [z for z in sizes if z[0] in args.diffusion_sizes.split(",")]:
        cells = pr["nx"] * pr["ny"]
        s = pfiso.Solver(pr, precision=pfiso.PF_F32)
        st = s.stream
        # HBM-bound: many short segments keep more loads in flight than the
        # full step's default (waves per SIMD sized for VALU issue); 16-row
        # segments were the fastest of 16, 32, 64 rows and 16..64 waves per SIMD
        s.tune(DIFFUSION_ROWS_PER_SEGMENT, 1)
        if label == "8192x8192":
            geo = s.geometry()
        print("bench: diffusion2d %s FP32, warmup %d, steps %d, geometry %s" % (
            label, warm, steps, s.geometry()), file=sys.stderr, flush=True)
        s.step_diffusion(warm)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        s.step_diffusion(steps)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(nl)]
        for a, b in evs:
            a.record(st)
            s.step_diffusion(1)
            b.record(st)
        torch.cuda.synchronize()
        kern_ms = sum(a.elapsed_time(b) for a, b in evs) / nl
        s.close()
        # the timed region is back-to-back launches of this one kernel: its
        # average is the kernel's average launch duration
        res[label] = {"ms_per_step": ms, "cell_updates_per_s": cells / (ms * 1e-3),
                      "kernel_ms_isolated_launch": round(kern_ms, 5),
                      "algorithmic_GBs": round(ALG_BYTES_2D_F32 * cells / (ms * 1e-3) / 1e9, 1)}
    copy = _copy_GBs()
    big = res["8192x8192"]
    gbs = big["algorithmic_GBs"]
    ctr = load_counters(DIFFUSION_COUNTERS, geo)
    out = {"metric": "phi+U cell-updates/s", "value": big["cell_updates_per_s"],
           "unit": "cell-updates/s", "n_gpus": 1, "steps": steps, "warmup": warm,
           "ms_per_step": big["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "diffusion-only step (psi held, U by the shell divergence of "
                                  "Eq. PF_b), 8192x8192 FP32, 16 B per cell as the full step",
                      "rows_per_segment": geo[0], "z_tile": geo[1]},
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(gbs / PEAK_HBM_GBS, 4),
                        "traffic": None if ctr is None else ctr["hbm_bytes_per_launch"],
                        "kernel": "step2d_kernel<float,frozen,frame,diffusion-only>",
                        "kernel_ms": round(big["ms_per_step"], 5),
                        "counters_kernel_ns": None if ctr is None else ctr["avg_duration_ns"],
                        "copy_GBs_measured": round(copy, 1),
                        "frac_of_copy": round(gbs / copy, 4)},
           "sizes": res}
    print(json.dumps(out))


def bench_serve(args):
    """Continuous-batching server on seeded Poisson traces of the served mix
    (300 requests; 80% 2D sides 256..1024, 20% 3D sides 128..192, 2000..10000
    steps, FP32) at two operating points: the arrival rate of the workload
    (mean 20 requests/s, several times what one GPU finishes, so queueing
    sets the latencies) and a rate below capacity (offered load about 0.7, so
    admission and batching set them).  Under an HBM budget and a cap of 8192
    active waves, over 4 streams with autotuned geometries; p50/p99
    time-to-result and throughput per point, beside the same trace served one
    request at a time in FP32 and in FP64 (and, at the workload's rate,
    shortest-work-first admission and all admitted solves sharing the GPU)."""
    from paper_2110_12448_amd import serve
    from paper_2110_12448_amd import pfiso
    budget = int(args.hbm_budget_gib * (1 << 30))

    def served(rate, precision, realtime, **kw):
        reqs = serve.poisson_trace(n=args.requests, rate=rate, precision=precision)
        srv = serve.Server(progress=25, **kw)
        t0 = time.perf_counter()
        res = srv.run(reqs, realtime=realtime)
        makespan = time.perf_counter() - t0
        return reqs, serve.summarize(res, makespan, srv.busy_s)

    policy = dict(max_waves=8192, streams=4, autotune_steps=5)
    points = {}
    for name, rate in (("workload_rate", 20.0), ("below_capacity", args.low_rate)):
        # below capacity the server idles between arrivals: the trace clock
        # skips those idle gaps instead of sleeping through them (latencies
        # and throughput are unchanged; the wall time shrinks)
        realtime = name == "workload_rate"
        print("serve: %s, %d requests at %.1f/s" % (name, args.requests, rate), file=sys.stderr,
              flush=True)
        reqs, summ = served(rate, pfiso.PF_F32, realtime, hbm_budget_bytes=budget,
                            chunk_steps=200, graph_steps=10, **policy)
        pt = {"arrival_rate_per_s": rate, "serving": summ}
        if not args.no_serve_baselines:
            if name == "workload_rate":
                pt["serving_shortest_first"] = served(
                    rate, pfiso.PF_F32, realtime, hbm_budget_bytes=budget, chunk_steps=200,
                    graph_steps=10, order="sjf", **policy)[1]
                pt["all_admitted_sharing_f32"] = served(
                    rate, pfiso.PF_F32, realtime, hbm_budget_bytes=budget, chunk_steps=200,
                    graph_steps=10, autotune_steps=5)[1]
            for bname, prec in (("one_at_a_time_f32", pfiso.PF_F32),
                                ("one_at_a_time_f64", pfiso.PF_F64)):
                pt[bname] = served(rate, prec, realtime, hbm_budget_bytes=1,
                                   chunk_steps=1 << 30, batching=False, autotune_steps=5)[1]
        points[name] = pt
    main_pt = points["workload_rate"]["serving"]
    out = {"metric": "served phi+U cell-updates/s; p50/p99 time-to-result", "value":
           main_pt["cell_updates_per_s"], "unit": "cell-updates/s", "n_gpus": 1,
           "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "served mix: Poisson arrivals, %d requests, 80%% 2D "
                                  "256^2-1024^2, 20%% 3D 128^3-192^3, 2000-10000 steps, FP32, HBM "
                                  "budget %.1f GiB; arrival rates 20/s (the workload's) and "
                                  "%.1f/s (below capacity)" % (args.requests, args.hbm_budget_gib,
                                                                args.low_rate),
                      "requests": args.requests,
                      "policy": "admit in arrival order while under the HBM budget and "
                                "under %d active waves; 2D solves batched per kind; other "
                                "solves over %d streams; autotuned geometries"
                                % (policy["max_waves"], policy["streams"])},
           "serving": main_pt, "operating_points": points}
    print(json.dumps(out))


def load_counters(wk, geometry):
    """The committed rocprofv3 counter summary of the workload's step kernel,
    if it was taken on the current kernel source at the launch geometry in use
    (rows per segment, z rows per workgroup); else None."""
    path = os.path.join(ROOT, wk["counters"])
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_digest") != src_digest(wk["sources"]):
        return None
    if d.get("geometry") != list(geometry):
        return None
    return d


def copy_calibration(nbytes=1 << 30, reps=20):
    """Device-to-device copy of nbytes, reps times (the reference kernel for the
    FETCH_SIZE / WRITE_SIZE counters)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps,
                      "ms_per_copy": ms, "GBs_read_plus_write": 2 * nbytes / ms / 1e6}))


def _host_cpu():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def growth_observables(pr, steps=20000, every=500):
    """Tip velocity and growth angle of the same directional solve under the
    isotropic S-bar_{2,1} and the standard (1, 0) shell weights: the tip
    (x, y_lab) every `every` steps; over the second half of the run, V_tip is
    the least-squares slope of y_lab in time and the growth angle that of the
    tip path x(y_lab) from the pulling axis y, positive towards -x, the side to which the
    crystal's <01> axis leans for a misorientation alpha0 > 0 (so a tip
    following the crystal axis shows alpha0, one following the gradient 0)."""
    import numpy as np
    from paper_2110_12448_amd import pfiso
    from paper_2110_12448_amd import workloads as wl
    R = np.asarray(pr["rot"])[0]
    out = {"alpha0_deg": float(np.degrees(np.arctan2(R[1, 0], R[0, 0]))), "steps": steps}
    for name, w in (("Sbar21", wl.ISO_2D), ("std_weights_1_0", wl.STD_2D)):
        q = dict(pr)
        q["w"] = tuple(w)
        s = pfiso.Solver(q, precision=pfiso.PF_F32)
        ts, xs, ys = [], [], []
        for k in range(0, steps + 1, every):
            if k:
                s.step(every)
            t = s.tip_state()
            if t["found"]:
                ts.append(t["t"]), xs.append(t["x"]), ys.append(t["y_lab"])
        s.close()
        ts, xs, ys = np.array(ts), np.array(xs), np.array(ys)
        width = pr["nx"] * pr["h"]
        xs = np.unwrap(xs * (2 * np.pi / width)) * (width / (2 * np.pi))  # periodic x
        h = len(ts) // 2
        if len(ts) - h < 2:
            out[name] = None
            continue
        v = float(np.polyfit(ts[h:], ys[h:], 1)[0])
        ang = float(np.degrees(np.arctan(-np.polyfit(ys[h:], xs[h:], 1)[0])))
        out[name] = {"v_tip": v, "growth_angle_deg": ang, "tip_y_lab": float(ys[-1]),
                     "tip_x": float(xs[-1]) % width}
    return out


def cpu_baseline(pr, target_s=12.0, max_steps=40, label="1024x2048 directional"):
    """The FP64 oracle on the host: steps of the same solve until target_s or
    max_steps, on all OpenMP threads; then a shorter single-thread sample."""
    import oracle
    p = oracle.Params.from_problem(pr)
    psi, U, g = pr["psi0"], pr["U0"], pr["grain"]
    st = oracle.State()
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps and (time.perf_counter() - t0) < target_s:
        psi, U, st = oracle.step(p, psi, U, g, 1, st)
        steps += 1
    dt = time.perf_counter() - t0
    cells = pr["nx"] * pr["ny"] * pr["nz"]
    threads = oracle.num_threads()
    print("cpu baseline: %d oracle steps on %d threads in %.1f s" % (steps, threads, dt),
          file=sys.stderr, flush=True)
    # single thread: at least one step, at most a quarter of the budget; skipped
    # when one step would take over a minute on one thread
    single, single_sample = None, "skipped: one step would exceed 60 s on one thread"
    if dt / steps * threads <= 60.0:
        oracle.set_num_threads(1)
        t1 = time.perf_counter()
        s1 = 0
        q, V, st1 = pr["psi0"], pr["U0"], oracle.State()
        while s1 < 1 or (s1 < max_steps and (time.perf_counter() - t1) < target_s / 4):
            q, V, st1 = oracle.step(p, q, V, g, 1, st1)
            s1 += 1
        dt1 = time.perf_counter() - t1
        oracle.set_num_threads(threads)
        single, single_sample = cells * s1 / dt1, "%d steps (%.1f s)" % (s1, dt1)
    return {"value": cells * steps / dt, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "FP64 oracle, first %d steps of the same %s solve "
                      "(%.1f s)" % (steps, label, dt),
            "single_thread_value": single,
            "single_thread_sample": single_sample,
            "host": _host_cpu()}, steps, psi, U, st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--launch-sample", type=int, default=None)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["batched2d", "serve", "schemes2d",
                                                             "diffusion2d"],
                    default="polycrystal3d")
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--low-rate", type=float, default=3.0,
                    help="serve: arrival rate (requests/s) of the below-capacity point")
    ap.add_argument("--no-serve-baselines", action="store_true",
                    help="serve: skip the one-at-a-time FP32/FP64 runs of the same trace")
    ap.add_argument("--hbm-budget-gib", type=float, default=2.0)
    ap.add_argument("--batch-rows", type=int, default=0,
                    help="batched2d: one fixed segment length for every member instead of "
                         "pf_batch_autotune (profiling runs)")
    ap.add_argument("--schemes", default="S10,S21,Sbar21",
                    help="schemes2d: schemes to run (S21 is the reported one)")
    ap.add_argument("--diffusion-sizes", default="8192x8192,1024x2048",
                    help="diffusion2d: lattices to run (8192x8192 is the reported one)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the untimed extras: CPU oracle baseline, error against the "
                         "oracle and (directional2d) the growth observables")
    ap.add_argument("--geometry", default="auto",
                    help="launch geometry of the step kernel: 'auto' (pf_autotune before the "
                         "warm-up), 'default' (the library's), or 'SEG,ZTILE'")
    ap.add_argument("--copy-calibration", action="store_true")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload in ("batched2d", "serve", "schemes2d", "diffusion2d"):
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        {"batched2d": bench_batched, "serve": bench_serve,
         "schemes2d": bench_schemes, "diffusion2d": bench_diffusion}[args.workload](args)
        return
    wk = WORKLOADS[args.workload]
    if args.steps is None:
        args.steps = wk["steps"]
    if args.warmup is None:
        args.warmup = wk["warmup"]
    if args.launch_sample is None:
        args.launch_sample = min(400, args.steps)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2110_12448_amd import pfiso
    from paper_2110_12448_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pr = wk["build"](wl)
    cells = pr["nx"] * pr["ny"] * pr["nz"]
    s = pfiso.Solver(pr, precision=pfiso.PF_F32, device="cuda:0")
    st = s.stream
    if args.geometry == "auto":
        s.autotune(wk["tune_steps"])
    elif args.geometry != "default":
        s.tune(*[int(v) for v in args.geometry.split(",")])
    geometry = s.geometry()
    print("bench: %s %dx%dx%d FP32, warmup %d, steps %d, geometry %s (%s)" %
          (args.workload, pr["nx"], pr["ny"], pr["nz"], args.warmup, args.steps, geometry,
           args.geometry), file=sys.stderr, flush=True)
    s.step(args.warmup)
    s.tip_state()
    torch.cuda.synchronize()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    s.step(args.steps)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    value = cells * args.steps / (ms / 1e3)

    # average duration of the step kernel itself: one event pair per launch
    n = args.launch_sample
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(n)]
    for a, b in evs:
        a.record(st)
        s.step(1)
        b.record(st)
    torch.cuda.synchronize()
    kern_ms = sum(a.elapsed_time(b) for a, b in evs) / n
    # the on-demand reduction (tip, solid fraction, finiteness): pf_tip_state
    # enqueues the two reduction launches and one 48-byte copy on the
    # solver's stream and waits; timed on that stream
    tip = s.tip_state()
    nt = 20
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(nt)]
    for a, b in evs:
        a.record(st)
        tip = s.tip_state()
        b.record(st)
    torch.cuda.synchronize()
    tip_ms = sum(a.elapsed_time(b) for a, b in evs) / nt
    s.close()

    # every step of the timed region is one launch of the step kernel, back to
    # back on one stream: the region's average is the kernel's average launch
    # duration (the isolated per-launch events add their own overhead)
    step_kernel_ms = ms_per_step
    achieved_tflops = wk["flops"] * cells / (step_kernel_ms / 1e3) / 1e12
    achieved_gbs = wk["bytes"] * cells / (step_kernel_ms / 1e3) / 1e9
    ctr = load_counters(wk, geometry)
    traffic = None if ctr is None else ctr["hbm_bytes_per_launch"]
    roofline = {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4),
                "frac_of_nonpacked_fp32": round(achieved_tflops / PEAK_FP32_NONPACKED_TFLOPS, 4),
                "traffic": traffic,
                "kernel": wk["kernel"], "kernel_ms": round(step_kernel_ms, 5),
                "kernel_ms_isolated_launch": round(kern_ms, 5),
                "hbm_algorithmic_GBs": round(achieved_gbs, 1),
                "hbm_frac": round(achieved_gbs / PEAK_HBM_GBS, 4),
                "flops_per_cell": wk["flops"], "bytes_per_cell": wk["bytes"],
                "valu_lane_instr_per_cell": None if ctr is None else round(ctr["valu_lane_instr_per_cell"], 1),
                "cycles_per_valu_instr_per_simd":
                    None if ctr is None else round(ctr["cycles_per_valu_instr_per_simd"], 2),
                "counters_kernel_ns": None if ctr is None else ctr["avg_duration_ns"]}

    cpu = None
    err = None
    obs = None
    if not args.no_cpu and args.workload == "directional2d":
        print("observables: S-bar_{2,1} and (1, 0) weights, %d steps each" % wk["steps"],
              file=sys.stderr, flush=True)
        obs = growth_observables(pr, steps=wk["steps"])
    if not args.no_cpu:
        if "cpu_steps" not in wk:
            cpu, nst, opsi, oU, ost = cpu_baseline(pr)
        else:
            cpu, nst, opsi, oU, ost = cpu_baseline(pr, target_s=15.0, max_steps=wk["cpu_steps"],
                                                   label=wk["text"].split(",")[0] + " %dx%dx%d" % (
                                                       pr["nx"], pr["ny"], pr["nz"]))
        # the same number of steps on the GPU, compared with the oracle state
        s2 = pfiso.Solver(pr, precision=pfiso.PF_F32, device="cuda:0")
        s2.step(nst)
        phi, U, psi, _ = s2.read_fields()
        s2.close()
        ophi = np.tanh(opsi / math.sqrt(2.0))
        err = {"steps": nst, "max_abs_dphi": float(np.max(np.abs(phi - ophi))),
               "max_abs_dU": float(np.max(np.abs(U - oU)))}
        # the FP32 storage floor beside it: the oracle rounding its stored psi
        # and U to FP32 after every step, against the plain FP64 oracle
        import oracle
        print("fp32 storage floor: %d oracle steps" % nst, file=sys.stderr, flush=True)
        rpsi, rU, _ = oracle.step(oracle.Params.from_problem(pr, round_f32=1), pr["psi0"],
                                  pr["U0"], pr["grain"], nst)
        err["fp32_storage_floor"] = {
            "max_abs_dphi": float(np.max(np.abs(np.tanh(rpsi / math.sqrt(2.0)) - ophi))),
            "max_abs_dU": float(np.max(np.abs(rU - oU)))}

    out = {
        "metric": "phi+U cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wk["text"],
                   "nx": pr["nx"], "ny": pr["ny"], "nz": pr["nz"], "h": pr["h"], "dt": pr["dt"],
                   "k": pr["k"], "eps4": pr["eps4"], "D": pr["D"],
                   "rows_per_segment": geometry[0], "z_tile": geometry[1],
                   "geometry_from": {"auto": "pf_autotune"}.get(args.geometry, args.geometry)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
        "growth": obs,
        "tip": {"y_lab": tip["y_lab"], "x": tip["x"], "z": tip["z"],
                "frame_shift": tip["frame_shift"], "solid_fraction": tip["solid_fraction"]},
        "tip_state_ms": round(tip_ms, 5),
        "tip_state_vs_step": round(tip_ms / ms_per_step, 3),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
