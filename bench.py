"""Benchmark of the coupled LB/FD step on one MI355X.

Default workload: the 3-D porous medium with the synthetic mechanism,
D3Q27, 512 x 256 x 256 cells, seeded overlapping spheres of radius 6-12 to
porosity 0.85, 9 species / 20 reactions with FP64 sub-cycled Arrhenius
sources (``paper_2304_05657_amd.workloads.porous_3d_mech``) -- the largest
single-GPU configuration.  ``--workload`` selects another of
``workloads.named`` (``porous``: D3Q27 256^3, 4 species; ``burner``: D2Q9
2048 x 512; ``channel``).  ``--also`` adds further workloads to the same
line (default: the 256^3 packing, FP64 and FP16 populations).

Prints one JSON line.  ``value`` is the first precision's (FP64) step
throughput in MLUPS (all cells of the box per second) with every input
resident in HBM before the timed region; the timed region is exactly
``--steps`` steps with the FP64 conservation / non-finite reductions every
``--check-every`` steps, bracketed by HIP events on the solver's stream.
The mixed-precision forms are reported beside it, each with its step HBM
fraction (algorithmic bytes per step over the step time over 8 TB/s) and
its error against the FP64 run at a common level.

``roofline`` is for the dominant kernel (the launch with the longest
duration per step, timed separately with HIP events on the solver's
stream): its algorithmic flops and bytes per launch over its duration; the
bound is the one its arithmetic intensity selects against the ridge of the
FP64/FP32 vector peak (78.6 TFLOP/s without packed FP32) and 8 TB/s, and
``frac`` is the fraction of that peak; both fractions are given.
``cpu_baseline`` times the FP64 oracle (test infrastructure) on the host
cores for one step of a bounded slab of the same box.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS of coupled LBM+FD step and % HBM roofline, FP64 vs mixed precision"
HBM_PEAK_GBS = 8000.0
# Vector ALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.
# FP64 and FP32 issue at this rate: packed FP32 is not used.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
RIDGE = VALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)  # flop per byte
# sources that fix what the launches read and write (device code, the
# host-side launch plan and the boundary-cell list)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2304_05657_amd", "csrc", f)
                  for f in ("lbfd_kernels.h", "lbfd_internal.h", "lbfd_api.hip", "lbfd_math.h", "lbfd_chemjit.hip")]
# HBM bytes per launch of a kernel on a workload, from two rocprofv3 --pmc
# runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) scaled by the same
# counters on a plain device copy of known size, valid for the kernel
# sources whose SHA-256 is given (summaries under profiles/).
# HBM bytes per launch of the headline's dominant kernel from rocprofv3
# FETCH_SIZE + WRITE_SIZE (each scaled by what a 512 MiB device copy reads
# as), valid only for the kernel sources they were taken on
# (profiles/traffic_porous_mech_512x256x256_and_porous_256.md)
TRAFFIC = {
    ("porous3d_mech_512x256x256", "fp64", "lbfd_chem_jit_f64"): {
        "bytes_per_launch": 7303.2e6,
        "kernel_sha256": "abaa665ca7687a4218bf59cc40c4678ede0fd3324a05bfe3a728042f89330646",
    },
}
POP_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}
SCALAR_BYTES = {"fp64": 8, "fp32": 4, "fp16": 4}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16": "f32"}
CHEM_PASS_MIN_SPECIES = 5  # mechanisms of more than four species: chemistry launch


def chem_pass(prob) -> bool:
    return prob.n_species >= CHEM_PASS_MIN_SPECIES


def step_bytes_per_fluid(prob, precision: str) -> int:
    """Algorithmic bytes of one fluid cell's step: each population and
    scalar read and written once."""
    return 2 * prob.lattice * POP_BYTES[precision] + 2 * (1 + prob.n_species) * SCALAR_BYTES[precision]


def algorithmic_bytes(prob, precision: str) -> float:
    """Minimum HBM bytes of one step: per fluid cell 2 Q b_pop +
    2 (1 + N_sp) b_scalar, plus one mask byte per cell."""
    return float(prob.n_fluid * step_bytes_per_fluid(prob, precision) + prob.N)


def step_flops_per_cell(prob) -> int:
    """Floating-point operations of one coupled step for one fluid cell
    without the Arrhenius source (FMA = 2, add/mul/div = 1), counted from
    the minimal form of each operation: moments, density, FD operators with
    WENO3 on 1 + N_sp scalars per axis, Lambda, Euler update, P_h, source Xi
    and pre-conditioning, per-axis central-moment transforms, relaxation."""
    Q = prob.lattice
    D = 2 if Q == 9 else 3
    ns = prob.n_species
    moments = (Q - 1) + D * (2 * Q // 3 - 1)
    density = 2 * ns + 1
    velocity = 2 + D + 1
    fd = D * (6 + 56 * (1 + ns) + 5 * ns + 1) + (1 + ns)
    lam = 6 * ns + 2
    euler = 2 + 2 * ns
    ph = 3
    xi = Q * (16 + 2 * D) + 4
    shift = 1 + 2 * Q
    transforms = 2 * 12 * D * Q // 3
    relax = 3 * (Q - 1 - D)
    out = 4 * Q + 1
    return moments + density + velocity + fd + lam + euler + ph + xi + shift + transforms + relax + out


def chem_flops_per_substep(prob) -> int:
    """Flops of one chemistry sub-step of one cell (exp and log count 1):
    per reaction the exponent b ln T - Ta/T + ln(A dt) - ln N (5), exp,
    the reactant product (n_react), nu_k r for every species (2 N_sp) and
    q r (2); per sub-step the current state (1 + N_sp), ln T and 1/T (2), the
    limiter (3 N_sp) and the accumulation (2 + 2 N_sp)."""
    ns = prob.n_species
    per_rx = sum(5 + 1 + len(r.reactants) + 2 * ns + 2 for r in prob.reactions)
    return per_rx + (1 + ns) + 2 + 3 * ns + 2 + 2 * ns


def mean_substeps(prob, T_sample) -> float:
    """Mean number of chemistry sub-steps over a sample of cell
    temperatures: N = ceil(max_j k_j / 0.1) capped at chem_substeps_max
    (1 without sub-cycling)."""
    import numpy as np
    if prob.chem_substeps_max <= 1 or not prob.reactions:
        return 1.0
    T = np.asarray(T_sample, dtype=np.float64)
    kmax = np.zeros_like(T)
    for r in prob.reactions:
        kmax = np.maximum(kmax, r.A * prob.dt_phys * np.exp(r.b * np.log(T) - r.Ta / T))
    n = np.clip(np.ceil(kmax / 0.1), 1, prob.chem_substeps_max)
    return float(n.mean())


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
    out = {"u_max_rel": float(du.max() / umag_r.max()), "u_rms_rel": float(np.sqrt((du ** 2).mean()) / umag_r.max()),
           "T_max_rel": float(dT.max()), "T_rms_rel": float(np.sqrt((dT ** 2).mean())),
           "flame_dx_cells": float(flame_position(diag, prob) - flame_position(ref_diag, prob))}
    dY = max(float(np.abs(fields["Y"][k][fl] - ref["Y"][k][fl]).max()) for k in range(prob.n_species))
    out["Y_max_abs"] = dY
    return out


def kernel_record(name, cells, ms, flops, nbytes):
    t = ms * 1e-3
    tf = flops / t / 1e12
    gbs = nbytes / t / 1e9
    intensity = flops / nbytes if nbytes else float("inf")
    return {"kernel": name, "cells": cells, "ms_per_launch": ms, "flops": flops, "algorithmic_bytes": nbytes,
            "intensity_flop_per_byte": intensity, "TFLOPs": tf, "alu_frac": tf / VALU_PEAK_TFLOPS, "GBs": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS, "bound": "alu" if intensity > RIDGE else "hbm"}


def run_gpu(prob, precision: str, steps: int, warmup: int, check_every: int, links=None, images=None):
    import numpy as np
    import torch
    from paper_2304_05657_amd.lbfd import Solver

    s = Solver(prob, precision=precision, check_every=check_every,
               stream=int(torch.cuda.current_stream().cuda_stream))
    if links is not None:
        s.set_wall_links(*links)
    if images is not None:
        s.set_image_points(*images)
    s.step(warmup)
    s.sync()
    # sub-step counts of the chemistry at the level the timed region starts
    # from (a random sample of fluid cells), for the chemistry's flop count
    nsub = 1.0
    if prob.reactions and prob.chem_substeps_max > 1:
        T = s.fields()["T"][prob.mask == 0]
        rng = np.random.default_rng(0)
        nsub = mean_substeps(prob, rng.choice(T, size=min(200000, T.size), replace=False))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = s.time_steps(steps)  # HIP events on the solver's stream around exactly `steps` steps
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.sync()
    per_step_s = ms * 1e-3 / steps
    nbytes = algorithmic_bytes(prob, precision)
    # each launch alone, serialised and bracketed by HIP events on the
    # solver's stream (after the timed region; the state advances)
    n_fluid, n_boundary = s.cell_counts()
    n_int = n_fluid - n_boundary
    kms_i, kms_b, kms_c = s.time_kernels(steps)
    launches = s.step_launches()
    per_fluid = step_bytes_per_fluid(prob, precision)
    sfl = step_flops_per_cell(prob)
    cfl = chem_flops_per_substep(prob) * nsub
    kernels = []
    if chem_pass(prob):
        nsc = (1 + prob.n_species) * SCALAR_BYTES[precision]
        specialised, chem_note = s.chem_kernel()
        if not specialised:
            print("[bench] chemistry kernel: %s" % chem_note, file=sys.stderr, flush=True)
        label = ("lbfd_chem_jit_%s (FP64 Arrhenius source, kernel specialised to the mechanism, one thread per cell)"
                 % ("f64" if precision == "fp64" else "f32")
                 if specialised else "chem_kernel (FP64 Arrhenius source, one thread per cell)")
        kernels.append(kernel_record(label, n_fluid,
                                     kms_c / steps, n_fluid * cfl, float(n_fluid * 2 * nsc + prob.N)))
        step_fl = sfl
    else:
        step_fl = sfl + cfl
    if prob.lattice == 9:
        kernels.append(kernel_record("step_kernel (one launch: boundary and interior cells)", n_fluid,
                                     (kms_i + kms_b) / steps, n_fluid * step_fl, float(n_fluid * per_fluid + prob.N)))
    else:
        kernels.append(kernel_record("step_kernel (interior cells)", n_int, kms_i / steps, n_int * step_fl,
                                     float(n_int * per_fluid + prob.N)))
        kernels.append(kernel_record("step_kernel (boundary cells) + outlet_kernel", n_boundary, kms_b / steps,
                                     n_boundary * step_fl, float(n_boundary * per_fluid)))
    dominant = max(kernels, key=lambda k: k["ms_per_launch"])
    f = s.fields()
    fluid = prob.mask == 0
    ok = bool(np.isfinite(f["T"][fluid]).all() and np.isfinite(f["u"]).all())
    out = {
        "precision": precision, "ms_per_step": ms / steps, "wall_ms_per_step": wall * 1e3 / steps,
        "check_every": check_every, "launches_per_step": launches,
        "mlups": prob.N / per_step_s / 1e6, "mflups": prob.n_fluid / per_step_s / 1e6,
        "algorithmic_bytes_per_step": nbytes, "achieved_GBs": nbytes / per_step_s / 1e9,
        "step_hbm_frac": nbytes / per_step_s / 1e9 / HBM_PEAK_GBS, "finite": ok,
        "chem_mean_substeps": nsub, "kernels": kernels, "dominant_kernel": dominant["kernel"],
    }
    return out, s


def run_cpu_baseline(prob, budget_s: float) -> dict:
    """The FP64 oracle on the host cores, one step from the initial state
    over a slab of z planes of the same box (every cell of the slab
    computed, the rest of the box inactive), sized from a one-plane
    calibration to about `budget_s` seconds; MLUPS = slab cells / time."""
    import numpy as np
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    o = oracle.Oracle(prob, threads=threads)
    plane = prob.nx * prob.ny

    def slab(z0, z1):
        a = np.zeros((prob.nz, prob.ny, prob.nx), np.uint8)
        a[z0:z1] = 1
        return a

    if prob.nz == 1:
        o.step(1)  # first touch
        n, t0 = 0, time.perf_counter()
        while True:
            o.step(1)
            n += 1
            el = time.perf_counter() - t0
            if el >= budget_s or n >= 200:
                break
        cells, what = prob.N * n, "%d FP64 steps of the whole box" % n
    else:
        o.set_active(slab(0, 1))
        t0 = time.perf_counter()
        o.step(1)
        t1 = time.perf_counter() - t0
        k = int(max(1, min(prob.nz - 1, budget_s / max(t1, 1e-3))))
        o.set_active(slab(1, 1 + k))
        t0 = time.perf_counter()
        o.step(1)
        el = time.perf_counter() - t0
        cells, what = plane * k, "one FP64 step of the z planes 1..%d (%d cells, the rest of the box inactive)" % (k, plane * k)
    res = {"value": cells / el / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": "%s of %s, %.1f s" % (what, prob.name, el)}
    del o
    return res


def bench_adjoint(args, W):
    """Cost of the discrete adjoint against the forward step on one workload:
    us per step of lbfd_adjoint (forward pass with checkpoints every K steps,
    the backward sweep with each segment recomputed), of lbfd_objective (the
    steps with the objective's diagnostics) and of plain steps."""
    import time
    import torch
    from paper_2304_05657_amd.lbfd import Solver
    prob = W.named(args.workload)
    s = Solver(prob, "fp64")
    state = s.save_state()
    n, K = args.steps, args.adjoint
    s.objective(min(n, 10))
    s.load_state(state)
    t0 = time.perf_counter()
    s.step(n)
    s.sync()
    plain = (time.perf_counter() - t0) / n * 1e6
    s.load_state(state)
    t0 = time.perf_counter()
    J = s.objective(n)
    obj = (time.perf_counter() - t0) / n * 1e6
    s.load_state(state)
    s.adjoint(min(n, 2 * K), K)
    s.load_state(state)
    t0 = time.perf_counter()
    Ja, gW, gA, gTa = s.adjoint(n, K)
    adj = (time.perf_counter() - t0) / n * 1e6
    torch.cuda.synchronize()
    line = {"metric": "discrete adjoint cost per step", "value": adj, "unit": "us", "higher_is_better": False,
            "steps": n, "checkpoint_every": K, "plain_step_us": plain, "objective_step_us": obj,
            "ratio_to_plain_step": adj / plain, "ratio_to_objective_step": adj / obj, "J": Ja,
            "J_objective": J, "dJ_dA": list(map(float, gA)), "dJ_dTa": list(map(float, gTa)),
            "dtype": "f64", "data": "synthetic", "n_gpus": 1,
            "config": {"workload": prob.name, "lattice": "D%dQ%d" % (2 if prob.lattice == 9 else 3, prob.lattice),
                       "cells": int(prob.mask.size), "objective": "wall_q"}}
    print(json.dumps(line), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--check-every", type=int, default=10,
                    help="FP64 reductions (conservation, non-finite check) every this many steps, in the timed region")
    ap.add_argument("--precisions", default="fp64,fp32,fp16",
                    help="first entry is the headline value, the others are reported beside it")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
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
    ap.add_argument("--workload", default="porous_mech",
                    help="porous_mech (default), porous, burner or channel")
    ap.add_argument("--accuracy-steps", type=int, default=None,
                    help="level at which the mixed-precision runs are compared with the FP64 run "
                         "(0: skip, also for the --also workloads; default 200 for porous_mech, 20000 for the "
                         "burner, 5000 for porous)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 512 MiB device copy (calibrates the HBM byte counters)")
    ap.add_argument("--also", default="porous:fp64,fp16",
                    help="further workloads on the same line, 'name:prec,prec;name:...' ('none' for none)")
    ap.add_argument("--adjoint", type=int, default=0, metavar="K",
                    help="instead of the step benchmark: time lbfd_adjoint (FP64, wall heat flux over every "
                         "level) over --steps steps with checkpoints every K steps on --workload "
                         "(channel_adjoint: the 1024 x 256 channel), against lbfd_objective and plain steps "
                         "over the same steps; prints one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU slab sharding is a design note, "
              "not an executable path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    from paper_2304_05657_amd import workloads as W

    if args.adjoint:
        sys.exit(bench_adjoint(args, W))

    default_acc = {"porous_mech": 200, "burner": 20000, "porous": 5000, "channel": 2000}

    def bench_workload(name, precs, acc_steps, links_flag, images_flag):
        prob = W.named(name).replace(collision=args.collision)
        if args.transport == "mixture_averaged":
            prob = W.mixture_transport(prob)
        links = W.wall_links(prob) if links_flag else None
        images = W.image_points(prob) if images_flag else None
        results, ref = {}, None
        for p in precs:
            print("[bench] %s %s: %d warmup + %d timed steps" % (prob.name, p, args.warmup, args.steps),
                  file=sys.stderr, flush=True)
            results[p], solver = run_gpu(prob, p, args.steps, args.warmup, args.check_every, links, images)
            print("[bench] %s %s: %s" % (prob.name, p, json.dumps(results[p])), file=sys.stderr, flush=True)
            if acc_steps > 0:
                # continue the same run (outside the timed region) to the
                # comparison level and compare with the FP64 run
                solver.step(max(0, acc_steps - solver.level))
                solver.sync()
                f, d = solver.fields(), solver.diagnostics()
                results[p]["level"] = solver.level
                results[p]["finite_at_level"] = d["nonfinite"] == 0
                results[p]["flame_x_cells"] = flame_position(d, prob)
                if p == "fp64":
                    ref = (f, d)
                elif ref is not None:
                    results[p]["error_vs_fp64"] = accuracy(ref[0], ref[1], f, d, prob)
                    print("[bench] %s vs fp64 at level %d: %s" % (p, solver.level,
                          json.dumps(results[p]["error_vs_fp64"])), file=sys.stderr, flush=True)
            solver.close()
            del solver
        return prob, results, links is not None, images is not None

    precs = [p.strip() for p in args.precisions.split(",") if p.strip()]
    acc = args.accuracy_steps if args.accuracy_steps is not None else default_acc.get(args.workload, 2000)
    prob, results, has_links, has_images = bench_workload(args.workload, precs, acc, args.wall_links,
                                                          args.image_points)
    others = {}
    for item in [x for x in args.also.split(";") if x.strip() and x.strip() not in ("none", "''", '""')]:
        name, _, pl = item.partition(":")
        ops = [p.strip() for p in (pl or "fp64").split(",") if p.strip()]
        oacc = args.accuracy_steps if args.accuracy_steps == 0 else default_acc.get(name.strip(), 2000)
        oprob, ores, _, _ = bench_workload(name.strip(), ops, oacc, False, False)
        others[oprob.name] = {"lattice": "D2Q9" if oprob.lattice == 9 else "D3Q27", "cells": oprob.N,
                              "fluid_cells": oprob.n_fluid, "species": oprob.n_species,
                              "reactions": len(oprob.reactions),
                              "precisions": {p: {k: v for k, v in r.items() if k != "precision"}
                                             for p, r in ores.items()}}
        del oprob
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
    dk = max(head["kernels"], key=lambda k: k["ms_per_launch"])
    bound = dk["bound"]
    tkey = (prob.name, precs[0], dk["kernel"].split(" ")[0])
    t = TRAFFIC.get(tkey)
    traffic = t["bytes_per_launch"] if t and t.get("kernel_sha256") == kernel_sha() else None
    roof = {"kernel": dk["kernel"], "bound": bound,
            "achieved": dk["TFLOPs"] if bound == "alu" else dk["GBs"],
            "peak": VALU_PEAK_TFLOPS if bound == "alu" else HBM_PEAK_GBS,
            "unit": "TFLOP/s" if bound == "alu" else "GB/s",
            "frac": dk["alu_frac"] if bound == "alu" else dk["hbm_frac"],
            "traffic": traffic, "intensity_flop_per_byte": dk["intensity_flop_per_byte"], "ridge_flop_per_byte": RIDGE,
            "alu_frac": dk["alu_frac"], "hbm_frac": dk["hbm_frac"], "launch_ms": dk["ms_per_launch"],
            "cells_per_launch": dk["cells"], "algorithmic_flops_per_launch": dk["flops"],
            "algorithmic_bytes_per_launch": dk["algorithmic_bytes"],
            "step_hbm_frac": head["step_hbm_frac"]}
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
        "config": {"workload": prob.name, "lattice": "D2Q9" if prob.lattice == 9 else "D3Q27", "cells": prob.N,
                   "fluid_cells": prob.n_fluid, "species": prob.n_species, "reactions": len(prob.reactions),
                   "chem_substeps_max": prob.chem_substeps_max, "storage": precs[0],
                   "check_every": args.check_every, "collision": prob.collision, "transport": prob.transport,
                   "wall_links": has_links, "image_points": has_images},
        "roofline": roof,
        "cpu_baseline": cpu,
        "precisions": {p: {k: v for k, v in r.items() if k != "precision"} for p, r in results.items()},
        "other_workloads": others,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
