"""Benchmark of the coupled LB/FD step on one MI355X.

Default workload: the pseudo 2-D porous burner, D2Q9, 2048 x 512 cells,
staggered cylinders (radius 20, pitch 64) at 400 K, lean inflow at
u = 0.02, outflow, 4 species / 1 reaction -- synthetic, seeded inputs built
by ``paper_2304_05657_amd.workloads.cylinder_burner``.  ``--workload``
selects another of ``workloads.named`` (``porous``: D3Q27 256^3 sphere
packing; ``porous_mech``: D3Q27 512 x 256^2, 9 species / 20 reactions).

Prints one JSON line.  ``value`` is the FP64 step's throughput in MLUPS
(all cells of the box per second), with every input resident in HBM before
the timed region; the mixed-precision forms are reported beside it.
``roofline`` is for the dominant kernel (the single step launch in 2-D, the
interior-cell launch in 3-D): algorithmic flops per launch against the
vector-ALU peak, with the algorithmic bytes per launch (per fluid cell
2 Q b_pop + 2 (1 + N_sp) b_scalar, plus 1 byte of mask per cell) beside
them, over the launch duration measured with HIP events on the stream the
kernel runs on.  ``cpu_baseline`` times the FP64 oracle (test infrastructure) on the
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
# Vector ALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
# Both FP64 and FP32 issue at this rate: packed FP32 is not used.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# sources that fix what the step kernel reads and writes (device code, the
# host-side launch plan and the boundary-cell list)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2304_05657_amd", "csrc", f)
                  for f in ("lbfd_kernels.h", "lbfd_internal.h", "lbfd_api.hip")]
# HBM bytes per launch of the dominant kernel on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) scaled by
# the same counters on a plain 512 MiB device copy (FETCH_SIZE reads 0.5x,
# WRITE_SIZE 1.0x the copied bytes), valid for the kernel sources whose
# SHA-256 (kernel_sha) is given (profiles/traffic_step_kernels_burner_2048x512.md).
TRAFFIC_WORKLOAD = "cylinder_burner_2048x512"
TRAFFIC = {
    "fp64": {"kernel_sha256": "9d1349d250e5324bb86203a936403069b8b3797f96b9c2043a72caf81abe6588", "bytes_per_launch": 267.0e6},
    "fp32": {"kernel_sha256": "9d1349d250e5324bb86203a936403069b8b3797f96b9c2043a72caf81abe6588", "bytes_per_launch": 168.1e6},
    "fp16": {"kernel_sha256": "9d1349d250e5324bb86203a936403069b8b3797f96b9c2043a72caf81abe6588", "bytes_per_launch": 125.3e6},
}
POP_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}
SCALAR_BYTES = {"fp64": 8, "fp32": 4, "fp16": 4}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16": "f32"}


def algorithmic_bytes(prob, precision: str) -> float:
    """Minimum HBM bytes of one step: each population and scalar of a fluid
    cell read and written once, one mask byte per cell."""
    per_fluid = 2 * prob.lattice * POP_BYTES[precision] + 2 * (1 + prob.n_species) * SCALAR_BYTES[precision]
    return float(prob.n_fluid * per_fluid + prob.N)


def algorithmic_flops_per_cell(prob) -> int:
    """Floating-point operations of one coupled step for one fluid cell
    (FMA = 2, add/mul/div/exp = 1), counted from the minimal form of each
    operation: moments, density, FD operators with WENO3 on 1 + N_sp scalars
    per axis, Arrhenius source, Lambda, Euler update, P_h, source Xi and
    pre-conditioning, per-axis central-moment transforms, relaxation."""
    Q = prob.lattice
    D = 2 if Q == 9 else 3
    ns = prob.n_species
    nrx = len(prob.reactions)
    moments = (Q - 1) + D * (2 * Q // 3 - 1)
    density = 2 * ns + 1
    velocity = 2 + D + 1
    fd = D * (6 + 56 * (1 + ns) + 5 * ns + 1) + (1 + ns)
    chem = nrx * (10 + 2 * ns)
    lam = 6 * ns + 2
    euler = 2 + 2 * ns
    ph = 3
    xi = Q * (16 + 2 * D) + 4
    shift = 1 + 2 * Q
    transforms = 2 * 12 * D * Q // 3
    relax = 3 * (Q - 1 - D)
    out = 4 * Q + 1
    return (moments + density + velocity + fd + chem + lam + euler + ph + xi + shift + transforms + relax
            + out)


def kernel_sha() -> str:
    """SHA-256 over the concatenated KERNEL_SOURCES."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def flame_position(diag, prob) -> float:
    """Front position in cells: the burnt length sum(theta) / (mean fluid
    cells per x column), counted back from the outlet face."""
    return prob.nx - diag["sum_theta"] / (prob.n_fluid / prob.nx)


def accuracy(ref: dict, ref_diag: dict, fields: dict, diag: dict, prob) -> dict:
    """Errors of a mixed-precision run against the FP64 run at the same level."""
    import numpy as np
    fl = prob.mask == 0
    dims = 2 if prob.lattice == 9 else 3
    umag_r = np.sqrt(sum(ref["u"][d][fl] ** 2 for d in range(dims)))
    du = np.sqrt(sum((fields["u"][d][fl] - ref["u"][d][fl]) ** 2 for d in range(dims)))
    dT = np.abs(fields["T"][fl] - ref["T"][fl]) / (prob.T_b - prob.T_u)
    return {"u_max_rel": float(du.max() / umag_r.max()), "u_rms_rel": float(np.sqrt((du ** 2).mean()) / umag_r.max()),
            "T_max_rel": float(dT.max()), "T_rms_rel": float(np.sqrt((dT ** 2).mean())),
            "flame_dx_cells": float(flame_position(diag, prob) - flame_position(ref_diag, prob))}


def run_gpu(prob, precision: str, steps: int, warmup: int, links=None, images=None) -> dict:
    import torch
    from paper_2304_05657_amd.lbfd import Solver

    s = Solver(prob, precision=precision, stream=int(torch.cuda.current_stream().cuda_stream))
    if links is not None:
        s.set_wall_links(*links)
    if images is not None:
        s.set_image_points(*images)
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
    # the dominant kernel alone: interior cells, launches serialised and
    # bracketed by HIP events on the solver's stream
    n_fluid, n_boundary = s.cell_counts()
    n_int = n_fluid - n_boundary
    kms_i, kms_b = s.time_kernels(steps)
    t_int = kms_i * 1e-3 / steps
    per_fluid = algorithmic_bytes(prob, precision) - prob.N
    per_fluid /= prob.n_fluid
    int_bytes = n_int * per_fluid + prob.N
    int_flops = n_int * algorithmic_flops_per_cell(prob)
    launches = s.step_launches()
    fpc = algorithmic_flops_per_cell(prob)
    if launches == 1:
        # one launch per step: the step kernel is the whole step, and its
        # average launch duration is the event-timed step above
        dominant = {"kernel": "step_kernel (one launch per step: boundary and interior cells)",
                    "cells": n_fluid, "ms_per_launch": ms / steps, "flops": n_fluid * fpc,
                    "algorithmic_bytes": nbytes}
    else:
        dominant = {"kernel": "step_kernel (interior cells)", "cells": n_int, "ms_per_launch": kms_i / steps,
                    "flops": int_flops, "algorithmic_bytes": int_bytes}
    t_dom = dominant["ms_per_launch"] * 1e-3
    dominant.update({"flops_per_cell": fpc, "TFLOPs": dominant["flops"] / t_dom / 1e12,
                     "alu_frac": dominant["flops"] / t_dom / 1e12 / VALU_PEAK_TFLOPS,
                     "GBs": dominant["algorithmic_bytes"] / t_dom / 1e9,
                     "hbm_frac": dominant["algorithmic_bytes"] / t_dom / 1e9 / HBM_PEAK_GBS})
    out = {
        "precision": precision, "ms_per_step": ms / steps, "wall_ms_per_step": wall * 1e3 / steps,
        "launches_per_step": launches, "dominant_kernel": dominant,
        "mlups": prob.N / per_step_s / 1e6, "mflups": prob.n_fluid / per_step_s / 1e6,
        "algorithmic_bytes_per_step": nbytes, "achieved_GBs": achieved,
        "hbm_frac": achieved / HBM_PEAK_GBS, "finite": ok,
        "interior_kernel": {"cells": n_int, "ms_per_launch": kms_i / steps, "flops_per_cell":
                            algorithmic_flops_per_cell(prob), "TFLOPs": int_flops / t_int / 1e12,
                            "alu_frac": int_flops / t_int / 1e12 / VALU_PEAK_TFLOPS,
                            "algorithmic_bytes": int_bytes, "GBs": int_bytes / t_int / 1e9,
                            "hbm_frac": int_bytes / t_int / 1e9 / HBM_PEAK_GBS},
        "boundary_kernel": {"cells": n_boundary, "ms_per_launch": kms_b / steps},
    }
    return out, s


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
    # the same oracle on one core, continuing the run, for a quarter of the budget
    o.set_threads(1)
    n1, t1 = 0, time.perf_counter()
    while True:
        o.step(1)
        n1 += 1
        el1 = time.perf_counter() - t1
        if el1 >= budget_s / 4 or n1 >= 50:
            break
    return {"value": prob.N * n / el / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d FP64 steps of the same workload (%s) from its initial state (after one untimed "
                      "step), %.1f s" % (n, prob.name, el),
            "single_core": {"value": prob.N * n1 / el1 / 1e6, "unit": "MLUPS", "cores": 1,
                            "sample": "the next %d steps of that run on one thread, %.1f s" % (n1, el1)}}


def roofline(res: dict, precision: str, workload: str) -> dict:
    """Roofline of the dominant kernel (the one step launch in 2-D, the
    interior-cell launch in 3-D): it is bound by the vector ALU (instruction
    issue), so achieved is algorithmic TFLOP/s against the VALU peak; its
    HBM rate is given beside it."""
    dk = res["dominant_kernel"]
    t = TRAFFIC.get(precision) if workload == TRAFFIC_WORKLOAD else None
    traffic = t["bytes_per_launch"] if t and t.get("kernel_sha256") == kernel_sha() else None
    return {"kernel": dk["kernel"], "bound": "alu", "achieved": dk["TFLOPs"],
            "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": dk["alu_frac"], "traffic": traffic,
            "hbm_achieved_GBs": dk["GBs"], "hbm_peak_GBs": HBM_PEAK_GBS, "hbm_frac": dk["hbm_frac"],
            "launch_ms": dk["ms_per_launch"], "cells_per_launch": dk["cells"],
            "algorithmic_flops_per_cell": dk["flops_per_cell"],
            "algorithmic_bytes_per_launch": dk["algorithmic_bytes"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precisions", default="fp64,fp32,fp16",
                    help="first entry is the headline value, the others are reported beside it")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--collision", default="central_moments", choices=("central_moments", "cumulants"),
                    help="relaxation of the orders >= 4: central moments (default) or cumulants")
    ap.add_argument("--wall-links", action="store_true",
                    help="interpolated bounce-back on the links crossing the workload's cylinders / spheres")
    ap.add_argument("--transport", default="unity_lewis", choices=("unity_lewis", "mixture_averaged"),
                    help="species transport: Fick with unity Lewis numbers (default) or mixture-averaged "
                         "diffusion with synthetic Lewis numbers and heat capacities")
    ap.add_argument("--image-points", action="store_true",
                    help="Shepard-reconstructed image points for the ghost nodes inside the workload's "
                         "cylinders / spheres")
    ap.add_argument("--workload", default="burner",
                    help="burner (default), channel, porous or porous_mech")
    ap.add_argument("--accuracy-steps", type=int, default=None,
                    help="level at which the mixed-precision runs are compared with the FP64 run "
                         "(0: skip; default 20000 for the burner, 2000 otherwise)")
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

    prob = W.named(args.workload).replace(collision=args.collision)
    if args.transport == "mixture_averaged":
        prob = W.mixture_transport(prob)
    links = W.wall_links(prob) if args.wall_links else None
    images = W.image_points(prob) if args.image_points else None
    if args.accuracy_steps is None:
        args.accuracy_steps = 20000 if args.workload == "burner" else 2000
    precs = [p.strip() for p in args.precisions.split(",") if p.strip()]
    results = {}
    ref = None
    for p in precs:
        print("[bench] %s: %d warmup + %d timed steps" % (p, args.warmup, args.steps), file=sys.stderr, flush=True)
        results[p], solver = run_gpu(prob, p, args.steps, args.warmup, links, images)
        print("[bench] %s: %s" % (p, json.dumps(results[p])), file=sys.stderr, flush=True)
        if args.accuracy_steps > 0:
            # continue the same run (outside the timed region) to the
            # comparison level and compare with the FP64 run
            solver.step(max(0, args.accuracy_steps - solver.level))
            solver.sync()
            f, d = solver.fields(), solver.diagnostics()
            results[p]["level"] = solver.level
            results[p]["finite_at_level"] = d["nonfinite"] == 0
            results[p]["flame_x_cells"] = flame_position(d, prob)
            if p == "fp64":
                ref = (f, d)
            elif ref is not None:
                results[p]["error_vs_fp64"] = accuracy(ref[0], ref[1], f, d, prob)
                print("[bench] %s vs fp64 at level %d: %s" % (p, solver.level, json.dumps(results[p]["error_vs_fp64"])),
                      file=sys.stderr, flush=True)
        solver.close()
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
        "config": {"workload": prob.name, "lattice": "D2Q9" if prob.lattice == 9 else "D3Q27", "cells": prob.N, "fluid_cells": prob.n_fluid,
                   "species": prob.n_species, "reactions": len(prob.reactions), "storage": precs[0],
                   "collision": prob.collision, "transport": prob.transport, "wall_links": links is not None,
                   "image_points": images is not None},
        "roofline": roofline(head, precs[0], prob.name),
        "cpu_baseline": cpu,
        "precisions": {p: {k: v for k, v in r.items() if k != "precision"} for p, r in results.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
