"""Benchmark of the coupled LB/FD step on one MI355X.

Workload: the pseudo 2-D porous burner, D2Q9, 2048 x 512 cells, staggered
cylinders (radius 20, pitch 64) at 400 K, lean inflow at u = 0.02, outflow,
4 species / 1 reaction -- synthetic, seeded inputs built by
``paper_2304_05657_amd.workloads.cylinder_burner``.

Prints one JSON line.  ``value`` is the FP64 step's throughput in MLUPS
(all cells of the box per second), with every input resident in HBM before
the timed region; the mixed-precision forms are reported beside it.
``roofline`` is for the step kernel: algorithmic bytes per launch (per fluid
cell 2 Q b_pop + 2 (1 + N_sp) b_scalar, plus 1 byte of mask per cell) over
the launch duration measured with HIP events on the stream the kernel runs
on.  ``cpu_baseline`` times the FP64 oracle (test infrastructure) on the
host cores for a bounded number of steps of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS of coupled LBM+FD step and % HBM roofline, FP64 vs mixed precision"
HBM_PEAK_GBS = 8000.0
POP_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}
SCALAR_BYTES = {"fp64": 8, "fp32": 4, "fp16": 4}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16": "f32"}


def algorithmic_bytes(prob, precision: str) -> float:
    """Minimum HBM bytes of one step: each population and scalar of a fluid
    cell read and written once, one mask byte per cell."""
    per_fluid = 2 * prob.lattice * POP_BYTES[precision] + 2 * (1 + prob.n_species) * SCALAR_BYTES[precision]
    return float(prob.n_fluid * per_fluid + prob.N)


def run_gpu(prob, precision: str, steps: int, warmup: int) -> dict:
    import torch
    from paper_2304_05657_amd.lbfd import Solver

    s = Solver(prob, precision=precision, stream=int(torch.cuda.current_stream().cuda_stream))
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = s.time_steps(steps)  # HIP events on the solver's stream around exactly `steps` launches
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.sync()
    f = s.fields()
    import numpy as np
    fluid = prob.mask == 0
    ok = bool(np.isfinite(f["T"][fluid]).all() and np.isfinite(f["u"]).all())
    per_step_s = ms * 1e-3 / steps
    nbytes = algorithmic_bytes(prob, precision)
    achieved = nbytes / per_step_s / 1e9
    out = {
        "precision": precision, "ms_per_step": ms / steps, "wall_ms_per_step": wall * 1e3 / steps,
        "mlups": prob.N / per_step_s / 1e6, "mflups": prob.n_fluid / per_step_s / 1e6,
        "algorithmic_bytes_per_step": nbytes, "achieved_GBs": achieved,
        "hbm_frac": achieved / HBM_PEAK_GBS, "finite": ok,
    }
    s.close()
    return out


def run_cpu_baseline(prob, budget_s: float) -> dict:
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    o = oracle.Oracle(prob, threads=threads)
    o.step(1)  # first-touch
    n, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 200:
            break
    return {"value": prob.N * n / el / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d FP64 steps of the same %dx%d burner from its initial state (after one untimed "
                      "step), %.1f s" % (n, prob.nx, prob.ny, el)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precisions", default="fp64,fp32,fp16",
                    help="first entry is the headline value, the others are reported beside it")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 512 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU sharding is a design note, "
              "not an executable path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    from paper_2304_05657_amd import workloads as W

    prob = W.cylinder_burner()
    precs = [p.strip() for p in args.precisions.split(",") if p.strip()]
    results = {}
    for p in precs:
        print("[bench] %s: %d warmup + %d timed steps" % (p, args.warmup, args.steps), file=sys.stderr, flush=True)
        results[p] = run_gpu(prob, p, args.steps, args.warmup)
        print("[bench] %s: %s" % (p, json.dumps(results[p])), file=sys.stderr, flush=True)
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] copy probe: %d bytes read, %d bytes written" % (src.numel() * 8, dst.numel() * 8),
              file=sys.stderr, flush=True)
        del src, dst
    head = results[precs[0]]
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, %.0f s budget)" % args.cpu_seconds, file=sys.stderr, flush=True)
        cpu = run_cpu_baseline(prob, args.cpu_seconds)
    line = {
        "metric": METRIC,
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[precs[0]],
        "data": "synthetic",
        "config": {"workload": prob.name, "lattice": "D2Q9", "cells": prob.N, "fluid_cells": prob.n_fluid,
                   "species": prob.n_species, "reactions": len(prob.reactions), "storage": precs[0]},
        "roofline": {"bound": "hbm", "achieved": head["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["achieved_GBs"] / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": cpu,
        "precisions": {p: {k: v for k, v in r.items() if k != "precision"} for p, r in results.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
