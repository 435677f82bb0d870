"""Throughput benchmark of the fused phase-field step on one MI355X.

Workload: 2D directional solidification in a moving frame, 1024 x 2048
lattice, FP32 fields, S-bar_{2,1} (isotropic stencils with the approximated
anti-trapping current), frozen temperature, misorientation drawn uniformly in
[0, 45] deg (seed 2).  One benchmark step is one full time step of the hot
path: the fused psi/U kernel with its in-pass FP64 tip / solid-fraction
reduction and the moving-frame decision.  Fields stay resident in HBM for the
whole timed region.

Prints one JSON line (cell-updates/s) with a roofline entry for the step
kernel and the FP64 CPU oracle timed on a bounded sample of the same
workload.
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
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector (published)
# FP32 operations per cell-update of the 2D step as written in step2d.hip
# (FMA = 2, each transcendental = 1; index math, selects and cross-lane moves
# not counted); derivation in the design doc.
ALG_FLOPS_2D = 237
# compulsory bytes per cell-update: read psi, U; write psi, U (FP32)
ALG_BYTES_2D_F32 = 16


def src_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = ["paper_2110_12448_amd/csrc/step2d.hip", "paper_2110_12448_amd/csrc/pf_device.hpp"]


def load_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "step2d_directional_1024x2048_counters.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_digest") != src_digest(KERNEL_SOURCES):
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(pr, target_s=12.0, max_steps=40):
    import numpy as np
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
    cells = pr["nx"] * pr["ny"]
    return {"value": cells * steps / dt, "unit": "cell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "FP64 oracle, first %d steps of the same 1024x2048 directional solve "
                      "(%.1f s)" % (steps, dt)}, steps, psi, U, st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--launch-sample", type=int, default=400)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2110_12448_amd import pfiso
    from paper_2110_12448_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pr = wl.config_directional_2d()
    cells = pr["nx"] * pr["ny"]
    s = pfiso.Solver(pr, precision=pfiso.PF_F32, device="cuda:0")
    st = s.stream
    print("bench: %dx%d FP32 directional, alpha0=%.2f deg, warmup %d" %
          (pr["nx"], pr["ny"], math.degrees(math.atan2(pr["rot"][0][1][0], pr["rot"][0][0][0])),
           args.warmup), file=sys.stderr, flush=True)
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
    tip = s.tip_state()
    s.close()

    achieved_tflops = ALG_FLOPS_2D * cells / (kern_ms / 1e3) / 1e12
    achieved_gbs = ALG_BYTES_2D_F32 * cells / (kern_ms / 1e3) / 1e9
    traffic = load_traffic()
    roofline = {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved_tflops / PEAK_FP32_TFLOPS, 4),
                "traffic": traffic,
                "kernel": "step2d_kernel<float,frozen,reduce>", "kernel_ms": round(kern_ms, 5),
                "hbm_algorithmic_GBs": round(achieved_gbs, 1),
                "hbm_frac": round(achieved_gbs / PEAK_HBM_GBS, 4),
                "flops_per_cell": ALG_FLOPS_2D, "bytes_per_cell": ALG_BYTES_2D_F32}

    cpu = None
    err = None
    if not args.no_cpu:
        cpu, nst, opsi, oU, ost = cpu_baseline(pr)
        # the same number of steps on the GPU, compared with the oracle state
        s2 = pfiso.Solver(pr, precision=pfiso.PF_F32, device="cuda:0")
        s2.step(nst)
        phi, U, psi, _ = s2.read_fields()
        s2.close()
        ophi = np.tanh(opsi / math.sqrt(2.0))
        err = {"steps": nst, "max_abs_dphi": float(np.max(np.abs(phi - ophi))),
               "max_abs_dU": float(np.max(np.abs(U - oU)))}

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
        "config": {"workload": "2D directional solidification, moving frame, 1024x2048, "
                               "S-bar_{2,1}, FP32 fields, FP64 tip/fraction reductions",
                   "nx": pr["nx"], "ny": pr["ny"], "h": pr["h"], "dt": pr["dt"],
                   "k": pr["k"], "eps4": pr["eps4"], "D": pr["D"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
        "tip": {"y_lab": tip["y_lab"], "x": tip["x"], "frame_shift": tip["frame_shift"],
                "velocity": tip["velocity"], "solid_fraction": tip["solid_fraction"]},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
