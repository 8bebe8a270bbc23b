#!/usr/bin/env python3
"""Benchmark of the hologram hot path on one MI355X.

One step = forward hologram (cgh_forward) of a 1,024-point cloud on a
1,920 x 1,024 hologram (the paper's headline shape, Table 1 / abstract),
G = I - T against a target hologram T, then the adjoint (cgh_backward) that
yields dL/dx, dL/dy, dL/dz, dL/dA of L = 0.5 ||I - T||^2.  Inputs are seeded
synthetic clouds already resident in HBM.

Prints ONE JSON line: throughput in G point-pixel interactions per second
(N * Nx * Ny / step time) of the compensated variant (the paper's method:
one native cosine per interaction), the roofline record of the dominant
kernel (the adjoint) from HIP events recorded around it, accuracy against the
FP64 GPU forward, and the FP64 CPU oracle's rate on a bounded sample of the
same workload (the cpu_baseline leg, the only part that touches the oracle).
Under "variants" the same step is reported for every variant (plain,
compensated, the recurrence of Eq. (2), the FP32 and 16-bit separable forms):
step time eager and as a replayed HIP graph, mean / median / min kernel
times, roofline fractions and the errors against FP64 (forward) and the
compensated adjoint.

The accuracy checks run first and the other variants are timed before the
headline, so that the headline's warm-up and timed steps run at the clock the
GPU settles at under sustained load (from a cold start it ramps up over the
first tens of milliseconds; --ramp measures that).

Other modes print one report line each: --workload (the other workload
shapes, every variant, and the Adam fitting loop for fit4k), --sweep (the
Table 1 N-sweep), --oracle-timing (the oracle per workload, serial and on all
cores), --copy-bytes (a plain copy, the reference for hardware byte counters),
--ramp (the headline step's kernel times over its first 400 steps from a cold
start).
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

# Roofline of the direct kernels, which are bound by the vector ALU.  MI355X's
# FP32 vector peak, 157.3 TFLOP/s, is 256 CUs x 2.4 GHz x 128 FP32 lanes per
# clock (x 2 flops per FMA): 7.86e13 FP32 lane-operations per second.  Every
# FP32 operation of an interaction takes one slot of that rate and every
# transcendental (v_cos_f32, v_sin_f32: quarter rate) four.  The machine probe
# (profiles/machine_issue_rates_gfx950.md) bears this out: a 64-lane FP32
# instruction with VGPR operands takes 0.61 of a CU clock (0.5 at the peak),
# one reading an SGPR about 1.05, a cosine or sine 2.2 (2 at quarter rate),
# and the transcendentals overlap neither each other nor other FP32 work.
PEAK_FP32_LANE_OPS = 256 * 2.4e9 * 128
TRANS_SLOTS = 4
# Algorithmic FP32 operations (and transcendentals) per point-pixel interaction:
#  fwd plain        dy, r2 (fma), Prev*r2, fract, acc fma  (+ cos)
#  fwd compensated  X+Y add, acc fma                       (+ cos)
#  fwd recurrence   Gamma += delta, acc fma (delta += Delta is shared by the
#                   rows of a lane; seeds are overhead)     (+ cos)
#  adj plain        r2 (fma), Prev*r2, fract, Sc fma, G*sin folded into the
#                   column and row sums (2 fma)             (+ sin, cos)
#  adj compensated  sin and cos of X+Y from the per-axis cosines and sines by
#                   the addition theorem (2 mul, 2 fma), Sc fma, column/row
#                   sums (2 fma); no transcendental per interaction
#  adj recurrence   Gamma += delta_c, Sc fma, column/row sums (2) (+ sin, cos)
FP32_OPS = {"fwd_plain": 5, "fwd_compensated": 2, "fwd_recurrence": 2,
            "adj_plain": 6, "adj_compensated": 7, "adj_recurrence": 4}
TRANS_OPS = {"fwd_plain": 1, "fwd_compensated": 1, "fwd_recurrence": 1,
             "adj_plain": 2, "adj_compensated": 0, "adj_recurrence": 2}
SLOTS = {k: FP32_OPS[k] + TRANS_SLOTS * TRANS_OPS[k] for k in FP32_OPS}
# The practical ceiling: each kernel's per-interaction instruction mix run
# alone by the probe (issue-bound, 8 resident waves per SIMD, operands where
# the kernel holds them), in CU clocks per 64 interactions.  The recurrence
# forward issues Gamma += delta, the cosine and an FMA with A from an SGPR,
# plus one add per 4 interactions (delta += Delta, shared by 4 rows).  The recurrence
# adjoint issues an add of two VGPRs, sine, cosine and three FMAs with G from
# an SGPR; the compensated adjoint two products, two FMAs (sin and cos by the
# addition theorem) and the same three FMAs.
MIX_CLOCKS = {"fwd_plain": 6.116, "fwd_compensated": 3.685, "fwd_recurrence": 3.966,
              "adj_plain": 9.331, "adj_compensated": 4.033, "adj_recurrence": 7.839}
CU_CLOCKS_PER_S = 256 * 2.4e9
# The separable variant is a different algorithm, bound by the FP32 matrix
# cores (dense MFMA FP32 peak 157.3 TFLOP/s): the forward is one GEMM of
# 2 x (2N) flops per pixel (4 flops per interaction), the adjoint two
# (8 flops per interaction).
# The half-precision separable variants run the same GEMMs on the fp16/bf16
# matrix cores (dense peak 2.5 PFLOP/s); f16x3 issues three MFMAs per product
# (hi*hi, hi*lo, lo*hi), so its matrix-core work is three times the flops.
PEAK_MFMA_F32 = 157.3e12
PEAK_MFMA_F16 = 2.5e15
MFMA_FLOPS = {"separable": (4, 8, PEAK_MFMA_F32), "separable_f16x3": (12, 24, PEAK_MFMA_F16),
              "separable_f16": (4, 8, PEAK_MFMA_F16), "separable_bf16": (4, 8, PEAK_MFMA_F16)}
ALL_VARIANTS = ("compensated", "plain", "recurrence", "separable", "separable_f16x3",
                "separable_f16", "separable_bf16")


def peak_interactions(key):
    """Roofline peak (interactions/s) of a kernel ("fwd_<variant>" or
    "adj_<variant>"): VALU issue for the direct variants, the matrix cores of
    the GEMM operand type for the separable ones."""
    op, variant = key.split("_", 1)
    if variant in MFMA_FLOPS:
        f_fwd, f_adj, peak = MFMA_FLOPS[variant]
        return peak / (f_fwd if op == "fwd" else f_adj)
    return PEAK_FP32_LANE_OPS / SLOTS[key]


def mix_interactions(key):
    """Interactions/s of the kernel's instruction mix run alone (the probe),
    or None where the probe has no such mix."""
    c = MIX_CLOCKS.get(key)
    return CU_CLOCKS_PER_S * 64 / c if c else None


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--variant", default="compensated",
                    choices=list(ALL_VARIANTS))
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="target wall seconds of each oracle sample (forward, adjoint)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="time the FP64 CPU oracle per workload (serial and all cores)")
    ap.add_argument("--only", action="store_true",
                    help="time --variant alone (no other variants; its accuracy only)")
    ap.add_argument("--ramp", action="store_true",
                    help="instead of the benchmark, time the headline step's kernels over its "
                         "first 400 steps from a cold start, in blocks of 20")
    ap.add_argument("--workload", default="paper",
                    choices=["paper", "small", "mesh8k", "mesh64k", "adjoint", "fit4k"],
                    help="paper: the headline fwd+adjoint step; the others print one report "
                         "line for that workload instead")
    ap.add_argument("--sweep", action="store_true",
                    help="forward N-sweep at 1920x1024 (N = 512..3584, the Table 1 shapes)")
    ap.add_argument("--fit-iters", type=int, default=100)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of the benchmark, run 5 plain device-to-device copies of this "
                         "many bytes (a known-traffic reference for hardware byte counters)")
    ap.add_argument("--library-gemm", action="store_true",
                    help="instead of the benchmark, time the platform's GEMM (torch.matmul: "
                         "hipBLASLt / rocBLAS) at the separable variants' contraction shapes of "
                         "the headline workload")
    ap.add_argument("--summarize", nargs=2, metavar=("KIND", "DIR"),
                    help="no GPU: write the profiles/ summary of KIND (stats, traffic or "
                         "counters) from the rocprofv3 CSV output under DIR")
    return ap.parse_args()


def copy_reference(nbytes):
    """Plain device copies of a known size: the calibration kernel for the
    FETCH_SIZE / WRITE_SIZE counters (each copy reads and writes nbytes)."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "copies": 5}), flush=True)


def measured_traffic(kernel, path=None, key="traffic_bytes"):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    record, or None when the kernel's sources have changed since the counters
    were taken.  ``traffic_bytes``: FETCH_SIZE and WRITE_SIZE scaled by a
    plain-copy reference; ``traffic_bytes_sized``: reads counted by request
    size (32, 64 and 128 bytes) plus the same writes."""
    if path is None:
        path = os.path.join(ROOT, "profiles", "traffic_paper_1920x1024_n1024.json")
    try:
        with open(path) as f:
            rec = json.load(f)["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None
    if _sources_hash(rec["sources"]) != rec["source_sha256_16"]:
        return None
    return rec.get(key)


# Device-code names of the direct adjoint kernels (the roofline kernel).
ADJ_KERNEL_NAME = {"plain": "adj_partial_kernel<0>", "compensated": "adj_partial_kernel<1>",
                   "recurrence": "adj_partial_kernel<2>"}
FWD_KERNEL = {"plain": 0, "compensated": 1, "recurrence": 7}
ADJ_KERNEL = {"plain": 3, "compensated": 4, "recurrence": 8}
for _v in MFMA_FLOPS:
    FWD_KERNEL[_v], ADJ_KERNEL[_v] = 5, 6


def _launch_stats(prefix, each):
    """Mean (the roofline's figure), median and min of per-launch kernel times."""
    import statistics

    if not each:
        return {prefix + "_kernel_ms": float("nan"), prefix + "_kernel_median_ms": float("nan"),
                prefix + "_kernel_min_ms": float("nan")}
    return {prefix + "_kernel_ms": sum(each) / len(each),
            prefix + "_kernel_median_ms": statistics.median(each),
            prefix + "_kernel_min_ms": min(each)}


def graph_step_ms(step, steps, torch):
    """The same step captured once into a HIP graph (torch.cuda.graph) and
    replayed ``steps`` times: ms per replay, or None if capture fails."""
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        graph.replay()
        ms, _ = timed_steps(graph.replay, steps, torch)
        del graph
        return ms
    except RuntimeError as e:
        print("graph capture failed: %s" % e, file=sys.stderr)
        return None


def timed_steps(step, steps, torch):
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    return e0.elapsed_time(e1) / steps, wall


# The separable variants' contractions at the headline workload (1920x1024,
# N = 1024: 2N = 2048 table columns), as (name, M, N, K) of C[M][N] =
# sum_k A(m, k) B(n, k), and the library kernel each one is compared with:
# this library's GEMM instantiation per operand format (fp16 hi/lo as one
# plain fp16 GEMM of three times the depth: [Ah Ah Al] . [Bh Bl Bh]).
SEP_GEMMS = (("forward I = Y X^T", 1024, 1920, 2048, 0),
             ("adjoint U, K = rows", 2048, 1920, 1024, 1),
             ("adjoint P, K = columns", 2048, 1024, 1920, 2))
SEP_OURS = {"f32": "gemm_f32_kernel<%s>", "f16": "gemm_half_kernel<0, %d>",
            "bf16": "gemm_half_kernel<1, %d>", "f16x3": "gemm_half_kernel<2, %d>"}
SEP_F32_ARGS = {0: "true, true, 0", 1: "false, false, 1", 2: "false, true, 2"}


def library_gemm():
    """torch.matmul (the platform's GEMM library) at the separable contraction
    shapes: mean of 50 launches after 5 warm-up ones, by CUDA events on
    torch's stream (one matmul per launch, so launch gaps are included)."""
    import torch

    dev = torch.device("cuda:0")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = []
    for name, m, n, k, fold in SEP_GEMMS:
        for fmt, dt, depth in (("f32", torch.float32, k), ("f16", torch.float16, k),
                               ("bf16", torch.bfloat16, k), ("f16x3", torch.float16, 3 * k)):
            g = torch.Generator(device=dev).manual_seed(7)
            A = torch.randn(m, depth, device=dev, generator=g).to(dt)
            Bt = torch.randn(depth, n, device=dev, generator=g).to(dt)
            C = torch.empty(m, n, device=dev, dtype=dt)
            for _ in range(5):
                torch.matmul(A, Bt, out=C)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(50):
                torch.matmul(A, Bt, out=C)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / 50 * 1e3
            out.append({"gemm": name, "format": fmt, "M": m, "N": n, "K": k, "depth": depth,
                        "us": us, "flops": 2.0 * m * n * depth, "fold": fold})
    print(json.dumps({"mode": "library_gemm", "torch": torch.__version__, "results": out}),
          flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: no multi-GPU path is implemented "
              "(--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    if args.summarize:
        summarize(*args.summarize)
        return
    if args.copy_bytes > 0:
        copy_reference(args.copy_bytes)
        return
    if args.library_gemm:
        library_gemm()
        return
    if args.sweep:
        report_sweep(args)
        return
    if args.oracle_timing:
        report_oracle_timing(args)
        return
    if args.ramp:
        report_ramp(args)
        return
    if args.workload != "paper":
        report_workload(args)
        return

    import numpy as np
    import torch

    from paper_1002_0916_amd import binding as B
    from paper_1002_0916_amd import workloads as W

    B.load_library()
    dev = torch.device("cuda:0")
    wl = W.WORKLOADS["paper"]
    nx, ny, n = wl.nx, wl.ny, wl.n
    inter = wl.interactions
    cloud = W.paper_cloud()
    target = W.paper_target_cloud()
    x, y, z, a = (torch.from_numpy(v).to(dev) for v in cloud.astuple())
    tx, ty, tz, ta = (torch.from_numpy(v).to(dev) for v in target.astuple())
    T = B.forward_f64(tx, ty, tz, ta, nx, ny).float()
    I = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    G = torch.empty_like(I)
    torch.cuda.synchronize()

    def make_step(variant):
        def step():
            # the forward writes I and G = I - T in one call (cgh_forward_residual)
            B.forward_residual(x, y, z, a, T, nx, ny, wl.pitch, wl.wavelength, variant, out=I,
                               residual=G)
            B.backward(x, y, z, a, G, nx, ny, wl.pitch, wl.wavelength, variant)
        return step

    others = [] if args.only else [v for v in ALL_VARIANTS if v != args.variant]

    # Accuracy of every forward variant against the FP64 GPU forward, and of
    # every adjoint against the compensated one (relative L2 per gradient
    # group, the largest of the four), with G = I64 - T.  Run before the
    # timing, it also starts the GPU's clock ramp.
    I64 = B.forward_f64(x, y, z, a, nx, ny)
    suma = float(np.sum(np.abs(cloud.a.astype(np.float64))))
    errs, adj_errs = {}, {}
    G64 = (I64 - T.double()).float()
    ref = [t.double() for t in B.backward(x, y, z, a, G64, nx, ny, wl.pitch, wl.wavelength,
                                         "compensated")]
    for variant in [args.variant] + others:
        # the step's own call (its I is cgh_forward's, bit for bit), so that
        # every forward launch of a run is the kernel the step times
        Iv, _ = B.forward_residual(x, y, z, a, T, nx, ny, wl.pitch, wl.wavelength, variant)
        errs[variant] = float((Iv.double() - I64).abs().max().item()) / suma
        gv = B.backward(x, y, z, a, G64, nx, ny, wl.pitch, wl.wavelength, variant)
        adj_errs[variant] = max(float((g.double() - r).norm() / r.norm())
                                for g, r in zip(gv, ref))
    torch.cuda.synchronize()

    # The other variants are timed first and the headline last: from a cold
    # start the GPU's clock ramps up over the first tens of milliseconds of
    # sustained load (kernels up to 15% slower over the first 60 steps;
    # `--ramp` measures it), so the headline's W warm-up and K timed steps run
    # at the steady clock that any longer run reaches.
    results = {}
    for variant in others + [args.variant]:
        step = make_step(variant)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        for k in range(B.KERNEL_COUNT):
            B.profile_read(k)  # clear
        B.profile_enable(True)
        ms, wall = timed_steps(step, args.steps, torch)
        B.profile_enable(False)
        fe = B.profile_read_each(FWD_KERNEL[variant])
        ae = B.profile_read_each(ADJ_KERNEL[variant])
        results[variant] = dict(ms_per_step=ms, wall_s=wall, fwd_launches=len(fe),
                                adj_launches=len(ae), **_launch_stats("fwd", fe),
                                **_launch_stats("adj", ae))
        results[variant]["graph_ms_per_step"] = graph_step_ms(step, args.steps, torch)

    main_r = results[args.variant]
    ms = main_r["ms_per_step"]
    value = inter / (ms * 1e-3) / 1e9
    adj_key = "adj_" + args.variant
    adj_ms = main_r["adj_kernel_ms"]
    achieved = inter / (adj_ms * 1e-3) / 1e9
    peak = peak_interactions(adj_key) / 1e9

    def kernel_summary(variant):
        r = results[variant]
        g = r.get("graph_ms_per_step")
        return {
            "ms_per_step": r["ms_per_step"],
            "gpps": inter / (r["ms_per_step"] * 1e-3) / 1e9,
            # the same step replayed from one captured HIP graph
            "graph_ms_per_step": g,
            "graph_gpps": inter / (g * 1e-3) / 1e9 if g else None,
            "fwd_kernel_ms": r["fwd_kernel_ms"],
            "fwd_kernel_median_ms": r["fwd_kernel_median_ms"],
            "fwd_kernel_min_ms": r["fwd_kernel_min_ms"],
            "adj_kernel_ms": r["adj_kernel_ms"],
            "adj_kernel_median_ms": r["adj_kernel_median_ms"],
            "adj_kernel_min_ms": r["adj_kernel_min_ms"],
            "fwd_gpps": inter / (r["fwd_kernel_ms"] * 1e-3) / 1e9,
            "adj_gpps": inter / (r["adj_kernel_ms"] * 1e-3) / 1e9,
            # N nx ny / (t_fwd + t_adj): the two main kernels alone
            "combined_kernel_gpps": inter / ((r["fwd_kernel_ms"] + r["adj_kernel_ms"]) * 1e-3)
                                    / 1e9,
            "fwd_roofline_frac": (inter / (r["fwd_kernel_ms"] * 1e-3)) /
                                 peak_interactions("fwd_" + variant),
            "adj_roofline_frac": (inter / (r["adj_kernel_ms"] * 1e-3)) /
                                 peak_interactions("adj_" + variant),
            "fwd_frac_of_mix": ((inter / (r["fwd_kernel_ms"] * 1e-3)) /
                                mix_interactions("fwd_" + variant)
                                if mix_interactions("fwd_" + variant) else None),
            "adj_frac_of_mix": ((inter / (r["adj_kernel_ms"] * 1e-3)) /
                                mix_interactions("adj_" + variant)
                                if mix_interactions("adj_" + variant) else None),
            "max_err_vs_fp64_over_sum_abs_a": errs[variant],
            "adj_rel_l2_vs_compensated": adj_errs[variant],
        }

    out = {
        "metric": "Gpoint-pixel/s fwd+adjoint at 1920x1024, N=1024; % VALU peak; "
                  "max err vs FP64",
        "value": value,
        "unit": "Gpoint-pixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded uniform point clouds)",
        "config": {
            "workload": "1920x1024 hologram, N=1024 points (x U[0,1920), y U[0,1024), "
                        "z U[0.5,1.0] m, A U[0.5,1.0]), p=8e-6 m, lambda=633e-9 m",
            "step": "forward + (I - T) + adjoint (dL/dx, dL/dy, dL/dz, dL/dA); I and I - T "
                    "from one cgh_forward_residual call",
            "variant": args.variant,
            "nx": nx, "ny": ny, "n_points": n,
        },
        "roofline": {
            "kernel": adj_key,
            "bound": "mfma" if args.variant.startswith("separable") else "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "Ginteraction/s",
            "frac": achieved / peak,
            "traffic": (measured_traffic(ADJ_KERNEL_NAME[args.variant])
                        if args.variant in ADJ_KERNEL_NAME else None),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated)",
            "traffic_sized": (measured_traffic(ADJ_KERNEL_NAME[args.variant],
                                               key="traffic_bytes_sized")
                              if args.variant in ADJ_KERNEL_NAME else None),
            "traffic_sized_unit": "bytes per launch (reads: TCC_EA0_RDREQ_32B/64B/128B x "
                                  "request size; writes: copy-calibrated WRITE_SIZE)",
            "peak_basis": (
                "FP32 vector peak 157.3 TFLOP/s = 7.86e13 FP32 lane-op/s (256 CU x 2.4 GHz x "
                "128 lanes); per interaction %d FP32 ops + %d transcendentals x %d slots "
                "(quarter rate) = %d slots" % (FP32_OPS[adj_key], TRANS_OPS[adj_key],
                                                TRANS_SLOTS, SLOTS[adj_key])
                if adj_key in SLOTS else "matrix-core peak of the GEMM operand type"),
            "slots_per_interaction": SLOTS.get(adj_key),
            "trans_slots": TRANS_SLOTS if adj_key in SLOTS else None,
            # the same instruction mix run alone on this chip (machine probe)
            "mix_peak": (mix_interactions(adj_key) / 1e9 if mix_interactions(adj_key)
                         else None),
            "frac_of_mix": (achieved * 1e9 / mix_interactions(adj_key)
                            if mix_interactions(adj_key) else None),
            "flops_per_interaction": (MFMA_FLOPS[args.variant][1]
                                      if args.variant in MFMA_FLOPS else None),
            "peak_lane_ops_per_s": PEAK_FP32_LANE_OPS if adj_key in SLOTS else None,
            "kernel_ms": adj_ms,
        },
        "variants": {v: kernel_summary(v) for v in [args.variant] + others},
        "paper_context": {
            "note": "forward only, Radeon HD5850, Table 1: 31 ms at N=1024",
            "paper_forward_gpps": inter / 31e-3 / 1e9,
            "this_forward_gpps": inter / (main_r["fwd_kernel_ms"] * 1e-3) / 1e9,
        },
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cloud, target, nx, ny, wl, args.cpu_seconds, x, y,
                                           z, a, T, args.variant, B, torch, np)
    print(json.dumps(out), flush=True)


def cpu_baseline(cloud, target, nx, ny, wl, seconds, x, y, z, a, T, variant, B, torch, np):
    """FP64 CPU oracle on a bounded sample of the same workload (all allowed cores).

    Forward: the first R full rows (all N points); adjoint: P points over the full
    grid, both sized from a short calibration to take about ``seconds`` each.
    Combined rate = 1 / (1/r_fwd + 1/r_adj), the oracle's fwd+adjoint rate.
    """
    import oracle

    cores = len(os.sched_getaffinity(0))
    n = cloud.n
    xs, ys, zs, as_ = cloud.astuple()

    def fwd_rows(rows):
        px = np.tile(np.arange(nx, dtype=np.int64), rows)
        py = np.repeat(np.arange(rows, dtype=np.int64), nx)
        t0 = time.perf_counter()
        v = oracle.forward_at(xs, ys, zs, as_, nx, ny, px, py, wl.pitch, wl.wavelength,
                              threads=cores)
        return time.perf_counter() - t0, v

    t_cal, _ = fwd_rows(max(1, cores // 4))
    rate_f = max(1, cores // 4) * nx * n / t_cal
    rows = int(min(ny, max(cores, seconds * rate_f / (nx * n))))
    t_f, v_f = fwd_rows(rows)
    r_f = rows * nx * n / t_f

    # Adjoint sample with the same G as the GPU step (G = I - T).
    I = B.forward(x, y, z, a, nx, ny, wl.pitch, wl.wavelength, variant)
    Gd = (I - T)
    G = Gd.cpu().numpy().astype(np.float64)
    gg = B.backward(x, y, z, a, Gd.contiguous(), nx, ny, wl.pitch, wl.wavelength, variant)
    gg = [t.cpu().numpy() for t in gg]
    rng = np.random.default_rng(1234)
    cal = np.arange(min(n, cores))
    t0 = time.perf_counter()
    oracle.adjoint(xs, ys, zs, as_, nx, ny, G, idx=cal, pitch=wl.pitch,
                   wavelength=wl.wavelength, threads=cores)
    rate_a = cal.shape[0] * nx * ny / (time.perf_counter() - t0)
    npts = int(min(n, max(cores, seconds * rate_a / (nx * ny))))
    npts = max(cores, (npts // cores) * cores) if npts >= cores else npts
    idx = np.sort(rng.choice(n, size=min(npts, n), replace=False))
    t0 = time.perf_counter()
    ref = oracle.adjoint(xs, ys, zs, as_, nx, ny, G, idx=idx, pitch=wl.pitch,
                         wavelength=wl.wavelength, threads=cores)
    t_a = time.perf_counter() - t0
    r_a = idx.shape[0] * nx * ny / t_a
    combined = 1.0 / (1.0 / r_f + 1.0 / r_a)

    Ig = I.cpu().numpy()[:rows].reshape(-1).astype(np.float64)
    suma = float(np.sum(np.abs(as_.astype(np.float64))))
    rel = {}
    for name, g, r in zip("xyza", gg, ref):
        rel["d" + name] = float(np.linalg.norm(g[idx] - r) / np.linalg.norm(r))
    return {
        "value": combined / 1e9,
        "unit": "Gpoint-pixel/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "forward: first %d of %d rows x all %d points (%.2f s); adjoint: %d of %d "
                  "points x all %d pixels (%.2f s); FP64, libm cos/sin, %d threads"
                  % (rows, ny, n, t_f, idx.shape[0], n, nx * ny, t_a, cores),
        "fwd_gpps": r_f / 1e9,
        "adj_gpps": r_a / 1e9,
        "cpu_model": _cpu_model(),
        "gpu_vs_oracle_on_sample": {
            "variant": variant,
            "fwd_max_err_over_sum_abs_a": float(np.max(np.abs(Ig - v_f)) / suma),
            "grad_rel_l2": rel,
        },
    }


RAMP_STEPS, RAMP_BLOCK = 400, 20


def report_ramp(args):
    """The clock's ramp under load: the headline step (--variant) run
    RAMP_STEPS times straight after start-up, with no warm-up, and the mean
    forward and adjoint kernel times (HIP events) of each block of RAMP_BLOCK
    steps."""
    import numpy as np
    import torch

    from paper_1002_0916_amd import binding as B
    from paper_1002_0916_amd import workloads as W

    B.load_library()
    dev = torch.device("cuda:0")
    wl = W.WORKLOADS["paper"]
    nx, ny = wl.nx, wl.ny
    x, y, z, a = (torch.from_numpy(v).to(dev) for v in W.paper_cloud().astuple())
    tx, ty, tz, ta = (torch.from_numpy(v).to(dev) for v in W.paper_target_cloud().astuple())
    T = B.forward_f64(tx, ty, tz, ta, nx, ny).float()
    I = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    G = torch.empty_like(I)
    torch.cuda.synchronize()
    for k in range(B.KERNEL_COUNT):
        B.profile_read(k)
    B.profile_enable(True)
    for _ in range(RAMP_STEPS):
        B.forward_residual(x, y, z, a, T, nx, ny, wl.pitch, wl.wavelength, args.variant, out=I,
                           residual=G)
        B.backward(x, y, z, a, G, nx, ny, wl.pitch, wl.wavelength, args.variant)
    torch.cuda.synchronize()
    B.profile_enable(False)
    fe = np.array(B.profile_read_each(FWD_KERNEL[args.variant], RAMP_STEPS))
    ae = np.array(B.profile_read_each(ADJ_KERNEL[args.variant], RAMP_STEPS))
    blocks = [{"first_step": i, "fwd_ms": float(fe[i:i + RAMP_BLOCK].mean()),
               "adj_ms": float(ae[i:i + RAMP_BLOCK].mean())}
              for i in range(0, RAMP_STEPS, RAMP_BLOCK)]
    print(json.dumps({"mode": "ramp", "variant": args.variant, "steps": RAMP_STEPS,
                      "block": RAMP_BLOCK, "blocks": blocks}), flush=True)


def summarize_ramp(root):
    line = _json_lines(root, "ramp")[-1]
    cmd = "timeout -k 10 300 python3 bench.py --ramp > <out>/ramp.log"
    b = line["blocks"]
    steady = b[len(b) // 2:]
    fs = sum(r["fwd_ms"] for r in steady) / len(steady)
    as_ = sum(r["adj_ms"] for r in steady) / len(steady)
    lines = ["# Clock ramp: the headline step from a cold start, 1920x1024, N=1024", "",
             "Command (from the repository root on an MI355X machine), then `python bench.py "
             "--summarize ramp <out>`:", "", "```", cmd, "```", "",
             "The %s step (forward, G = I - T, adjoint) run %d times straight after start-up "
             "with no warm-up; mean kernel times (HIP events) per block of %d steps, and "
             "against the mean of the second half (the steady state)."
             % (line["variant"], line["steps"], line["block"]), "",
             "| steps | forward ms | / steady | adjoint ms | / steady |", "|---|---|---|---|---|"]
    for r in b:
        lines.append("| %d-%d | %.4f | %.3f | %.4f | %.3f |"
                     % (r["first_step"], r["first_step"] + line["block"] - 1, r["fwd_ms"],
                        r["fwd_ms"] / fs, r["adj_ms"], r["adj_ms"] / as_))
    _write_md("clock_ramp_paper_1920x1024.md", lines)


def report_oracle_timing(args):
    """The FP64 CPU oracle timed on this host, per workload (part of the
    cpu_baseline leg: the only code here that calls the oracle), beside the
    compensated GPU kernels on the same workload.  Serial (one thread): the
    256x256 N=64 and 1920x1024 N=1024 full grids.  All allowed cores: the
    1920x1024 full grid, the 1920x1080 mesh clouds and the 3840x2160 N=16384
    cloud on 8192 seeded pixels plus the corners and the centre, and the
    1024x1024 N=4096 cloud's full forward and full adjoint."""
    import numpy as np
    import torch

    import oracle
    from paper_1002_0916_amd import binding as B
    from paper_1002_0916_amd import workloads as W

    B.load_library()
    dev = torch.device("cuda:0")
    cores = len(os.sched_getaffinity(0))
    rows = []

    def gpu_rates(cloud, nx, ny, wl, G=None):
        x, y, z, a = (torch.from_numpy(v).to(dev) for v in cloud.astuple())
        inter = cloud.n * nx * ny
        fms = _kernel_ms(B, torch, lambda: B.forward(x, y, z, a, nx, ny, wl.pitch,
                                                     wl.wavelength, "compensated"),
                         B.KERNEL_FWD_COMPENSATED, 5)
        out = {"gpu_fwd_gpps": inter / (fms * 1e-3) / 1e9}
        if G is not None:
            g = torch.from_numpy(np.ascontiguousarray(G, dtype=np.float32)).to(dev)
            ams = _kernel_ms(B, torch, lambda: B.backward(x, y, z, a, g, nx, ny, wl.pitch,
                                                          wl.wavelength, "compensated"),
                             B.KERNEL_ADJ_COMPENSATED, 5)
            out["gpu_adj_gpps"] = inter / (ams * 1e-3) / 1e9
        return out

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    def add(name, what, threads, inter, secs, gpu_gpps):
        rate = inter / secs
        rows.append({"workload": name, "what": what, "threads": threads,
                     "interactions": inter, "seconds": secs, "oracle_gpps": rate / 1e9,
                     "gpu_gpps": gpu_gpps, "gpu_over_oracle": gpu_gpps * 1e9 / rate})
        print("  %-10s %-34s %2d thr %9.3e int %8.2f s %8.4f G/s" %
              (name, what, threads, inter, secs, rate / 1e9), file=sys.stderr, flush=True)

    def full_fwd(name, cloud, wl, threads, gpu):
        t = timed(lambda: oracle.forward(*cloud.astuple(), wl.nx, wl.ny, wl.pitch,
                                         wl.wavelength, threads=threads))
        add(name, "forward, full grid", threads, cloud.n * wl.nx * wl.ny, t,
            gpu["gpu_fwd_gpps"])

    def subset_fwd(name, cloud, wl, seed, gpu):
        px, py = W.sample_pixels(seed, wl.nx, wl.ny, 8192)
        t = timed(lambda: oracle.forward_at(*cloud.astuple(), wl.nx, wl.ny, px, py, wl.pitch,
                                            wl.wavelength, threads=cores))
        add(name, "forward, %d sampled pixels" % px.shape[0], cores, cloud.n * px.shape[0], t,
            gpu["gpu_fwd_gpps"])

    wl0, wl1 = W.WORKLOADS["small"], W.WORKLOADS["paper"]
    c0, c1 = W.small_cloud(), W.paper_cloud()
    g0, g1 = gpu_rates(c0, wl0.nx, wl0.ny, wl0), gpu_rates(c1, wl1.nx, wl1.ny, wl1)
    full_fwd("small", c0, wl0, 1, g0)
    full_fwd("paper", c1, wl1, 1, g1)
    full_fwd("paper", c1, wl1, cores, g1)
    wl2a, wl2b = W.WORKLOADS["mesh8k"], W.WORKLOADS["mesh64k"]
    c2a, c2b = W.mesh_clouds()
    subset_fwd("mesh8k", c2a, wl2a, 81, gpu_rates(c2a, wl2a.nx, wl2a.ny, wl2a))
    subset_fwd("mesh64k", c2b, wl2b, 82, gpu_rates(c2b, wl2b.nx, wl2b.ny, wl2b))
    wl4 = W.WORKLOADS["fit4k"]
    _, c4 = W.fit_clouds()
    subset_fwd("fit4k", c4, wl4, 84, gpu_rates(c4, wl4.nx, wl4.ny, wl4))
    # 1024x1024 N=4096: full forward and full adjoint, G = I - T with I the
    # oracle hologram of the trainable cloud and T that of the hidden one.
    wl3 = W.WORKLOADS["adjoint"]
    h3, c3 = W.adjoint_clouds()
    t0 = time.perf_counter()
    I3 = oracle.forward(*c3.astuple(), wl3.nx, wl3.ny, wl3.pitch, wl3.wavelength, threads=cores)
    tf = time.perf_counter() - t0
    T3 = oracle.forward(*h3.astuple(), wl3.nx, wl3.ny, wl3.pitch, wl3.wavelength, threads=cores)
    G3 = (I3 - T3).astype(np.float32).astype(np.float64)
    g3 = gpu_rates(c3, wl3.nx, wl3.ny, wl3, G3)
    inter3 = c3.n * wl3.nx * wl3.ny
    add("adjoint", "forward, full grid", cores, inter3, tf, g3["gpu_fwd_gpps"])
    ta = timed(lambda: oracle.adjoint(*c3.astuple(), wl3.nx, wl3.ny, G3, pitch=wl3.pitch,
                                      wavelength=wl3.wavelength, threads=cores))
    add("adjoint", "adjoint, all points, full grid", cores, inter3, ta, g3["gpu_adj_gpps"])
    print(json.dumps({"mode": "oracle_timing", "cores": cores, "cpu_model": _cpu_model(),
                      "oracle": "FP64, libm cos/sin, row-parallel (bitwise equal to serial)",
                      "gpu": "compensated kernels, mean of 5 launches after 1 warm-up",
                      "rows": rows}), flush=True)


def _kernel_ms(B, torch, fn, kernel, reps):
    """Average duration of ``kernel`` over ``reps`` calls of fn (library events)."""
    fn()
    torch.cuda.synchronize()
    B.profile_read(kernel)
    B.profile_enable(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    B.profile_enable(False)
    n, ms = B.profile_read(kernel)
    return ms / max(n, 1)


def _clouds(name, W):
    if name == "small":
        return W.small_cloud(), None
    if name == "mesh8k":
        return W.mesh_clouds()[0], None
    if name == "mesh64k":
        return W.mesh_clouds()[1], None
    if name == "adjoint":
        hidden, c = W.adjoint_clouds()
        return c, hidden
    if name == "fit4k":
        hidden, c = W.fit_clouds()
        return c, hidden
    return W.paper_cloud(), W.paper_target_cloud()


def report_workload(args):
    """One JSON report line for a non-headline workload: forward kernel times
    and errors against the FP64 GPU forward for every variant, the adjoint
    kernel times, and for fit4k the Adam fitting loop."""
    import numpy as np
    import torch

    from paper_1002_0916_amd import binding as B
    from paper_1002_0916_amd import workloads as W

    B.load_library()
    dev = torch.device("cuda:0")
    wl = W.WORKLOADS[args.workload]
    nx, ny = wl.nx, wl.ny
    cloud, hidden = _clouds(args.workload, W)
    inter = cloud.n * nx * ny
    x, y, z, a = (torch.from_numpy(v).to(dev) for v in cloud.astuple())
    suma = float(np.sum(np.abs(cloud.a.astype(np.float64))))
    reps = max(1, min(20, int(4e11 // inter)))
    out = {"mode": "workload", "workload": args.workload, "description": wl.description,
           "nx": nx, "ny": ny, "n_points": cloud.n, "interactions": inter, "reps": reps}

    t64 = time.perf_counter()
    I64 = B.forward_f64(x, y, z, a, nx, ny)
    torch.cuda.synchronize()
    out["fwd_f64_ms"] = (time.perf_counter() - t64) * 1e3
    out["fwd_f64_gpps"] = inter / (out["fwd_f64_ms"] * 1e-3) / 1e9
    for variant in ((args.variant,) if args.only else ALL_VARIANTS):
        fk, ak = FWD_KERNEL[variant], ADJ_KERNEL[variant]
        Iv = B.forward(x, y, z, a, nx, ny, wl.pitch, wl.wavelength, variant)
        err = float((Iv.double() - I64).abs().max().item()) / suma
        fms = _kernel_ms(B, torch, lambda: B.forward(x, y, z, a, nx, ny, wl.pitch,
                                                     wl.wavelength, variant, out=Iv), fk, reps)
        G = (Iv - I64.float()).contiguous() if hidden is None else None
        if G is None:
            hx, hy, hz, ha = (torch.from_numpy(v).to(dev) for v in hidden.astuple())
            T = B.forward_f64(hx, hy, hz, ha, nx, ny).float()
            G = (Iv - T).contiguous()
        ams = _kernel_ms(B, torch, lambda: B.backward(x, y, z, a, G, nx, ny, wl.pitch,
                                                      wl.wavelength, variant), ak, reps)
        out[variant] = {
            "fwd_kernel_ms": fms, "fwd_gpps": inter / (fms * 1e-3) / 1e9,
            "fwd_roofline_frac": inter / (fms * 1e-3) / peak_interactions("fwd_" + variant),
            "adj_kernel_ms": ams, "adj_gpps": inter / (ams * 1e-3) / 1e9,
            "adj_roofline_frac": inter / (ams * 1e-3) / peak_interactions("adj_" + variant),
            "fwd_frac_of_mix": (inter / (fms * 1e-3) / mix_interactions("fwd_" + variant)
                                if mix_interactions("fwd_" + variant) else None),
            "adj_frac_of_mix": (inter / (ams * 1e-3) / mix_interactions("adj_" + variant)
                                if mix_interactions("adj_" + variant) else None),
            "max_err_vs_fp64_over_sum_abs_a": err,
        }
    if args.workload == "fit4k" and args.fit_iters > 0:
        from paper_1002_0916_amd import fit as F

        hx, hy, hz, ha = (torch.from_numpy(v).to(dev) for v in hidden.astuple())
        T = B.forward_f64(hx, hy, hz, ha, nx, ny).float()
        res = F.fit(x, y, z, a, T, nx, ny, iters=args.fit_iters, lr=1e-2, pitch=wl.pitch,
                    wavelength=wl.wavelength, variant="compensated")
        It = B.forward_f64(x, y, res.z, res.a, nx, ny)
        Ic = B.forward(x, y, res.z, res.a, nx, ny, wl.pitch, wl.wavelength, "compensated")
        suma_fit = float(res.a.abs().double().sum())
        out["fit"] = {
            "iterations": res.iterations, "seconds": res.seconds,
            "iterations_per_s": res.iterations_per_s, "lr": 1e-2,
            "params": "A and z/pitch (Adam); x, y fixed",
            "loss_first": res.losses[0], "loss_last": res.losses[-1],
            "loss_curve": res.losses,
            "fwd_kernel_ms": res.fwd_ms, "adj_kernel_ms": res.adj_ms,
            "fwd_gpps": inter / (res.fwd_ms * 1e-3) / 1e9,
            "adj_gpps": inter / (res.adj_ms * 1e-3) / 1e9,
            "fitted_fwd_max_err_vs_fp64_over_sum_abs_a":
                float((Ic.double() - It).abs().max().item()) / suma_fit,
        }
    print(json.dumps(out), flush=True)


def report_sweep(args):
    """Forward kernel time against N at 1920x1024 (the Table 1 shapes and
    beyond) for the direct FP32 variants, the recurrence of Eq. (2) (the
    kernel Table 1 times) among them; the paper's HD5850 times are context."""
    import torch

    from paper_1002_0916_amd import binding as B
    from paper_1002_0916_amd import workloads as W

    B.load_library()
    dev = torch.device("cuda:0")
    paper_ms = {512: 19, 1024: 31, 1536: 44, 2048: 56, 2560: 68, 3072: 80, 3584: 93}
    # About 70 ms of untimed load first (20 forwards at N = 16384), so that
    # every point of the sweep runs at the clock the GPU settles at under load.
    c = W.paper_cloud(n=16384)
    x, y, z, a = (torch.from_numpy(v).to(dev) for v in c.astuple())
    I = torch.empty((1024, 1920), dtype=torch.float32, device=dev)
    for _ in range(20):
        B.forward(x, y, z, a, 1920, 1024, variant="compensated", out=I)
    torch.cuda.synchronize()
    rows = []
    for n in (512, 1024, 1536, 2048, 2560, 3072, 3584, 8192, 16384):
        c = W.paper_cloud(n=n)
        x, y, z, a = (torch.from_numpy(v).to(dev) for v in c.astuple())
        I = torch.empty((1024, 1920), dtype=torch.float32, device=dev)
        rec = {"n": n, "paper_hd5850_ms": paper_ms.get(n)}
        for variant, k in (("plain", B.KERNEL_FWD_PLAIN),
                           ("recurrence", B.KERNEL_FWD_RECURRENCE),
                           ("compensated", B.KERNEL_FWD_COMPENSATED)):
            ms = _kernel_ms(B, torch, lambda: B.forward(x, y, z, a, 1920, 1024, variant=variant,
                                                        out=I), k, 10)
            rec[variant + "_ms"] = ms
            rec[variant + "_gpps"] = n * 1920 * 1024 / (ms * 1e-3) / 1e9
        rows.append(rec)
    print(json.dumps({"mode": "sweep", "hologram": "1920x1024", "rows": rows}), flush=True)


# --------------------------------------------------------------------------
# Summaries of rocprofv3 runs for profiles/ (no GPU needed: they read the CSV
# files that the commands listed in each summary wrote).

PROFILES = os.path.join(ROOT, "profiles")
HEADLINE_INTERACTIONS = 1024 * 1920 * 1024
_ROCPROF = "cd /tmp && export TMPDIR=/tmp && "


def _kernel_short(name):
    name = name.replace("void ", "").replace("cgh::(anonymous namespace)::", "")
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(", 1)[0]


def _csv_files(root, pattern):
    import glob

    files = sorted(glob.glob(os.path.join(root, "**", pattern), recursive=True))
    if not files:
        raise SystemExit("no %s under %s" % (pattern, root))
    return files


def _counter_means(files):
    """{kernel: {counter: mean over dispatches}} from counter_collection CSVs."""
    import collections
    import csv

    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                acc[_kernel_short(r["Kernel_Name"])][r["Counter_Name"]].append(
                    float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}


def _write_md(name, lines):
    path = os.path.join(PROFILES, name)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote", path)


def summarize_stats(root):
    """Kernel-duration table from `rocprofv3 --kernel-trace --stats` of the
    default benchmark command."""
    import csv

    rows = []
    for f in _csv_files(root, "*kernel_stats.csv"):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    cmd = (_ROCPROF + "timeout -s KILL 400 rocprofv3 --kernel-trace --stats -f csv -d <out>/stats "
           "-o bench -- python3 bench.py > <out>/stats/bench_stdout.log")
    lines = ["# Kernel stats: bench.py step at 1920x1024, N=1024", "",
             "Command (run from the repository root on an MI355X machine): the default benchmark "
             "command under the kernel tracer, then `python bench.py --summarize stats "
             "<out>/stats`:", "", "```", cmd, "```", "",
             "The run times every variant of the step (50 timed + 5 warm-up steps each, one "
             "graph capture and 50 replays per variant, the accuracy checks and the CPU "
             "baseline).  Kernel "
             "names: fwd_comp_residual_kernel (the step's forward, which also writes G = I - T) "
             "/ adj_partial_kernel<1> (compensated), fwd_plain_kernel / "
             "adj_partial_kernel<0> (plain), fwd_rec_kernel<K, R> / adj_partial_kernel<2> "
             "(recurrence), gemm_f32_kernel (separable FP32), gemm_half_kernel<format, fold> "
             "(format 2 = fp16 hi/lo, 0 = fp16, 1 = bf16; fold 0 = forward, 1 and 2 = the "
             "adjoint contractions).", "", "Durations in microseconds.", "",
             "| kernel | calls | avg us | min us | max us | share |", "|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["Percentage"])):
        lines.append("| %s | %s | %.1f | %.1f | %.1f | %.1f%% |" % (
            _kernel_short(r["Name"])[:70], r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    # The JSON line that the profiled command printed (saved beside the CSVs
    # as *.log): its HIP-event kernel means, taken in the same run.
    def json_line(path):
        found = None
        with open(path) as fh:
            for text in fh:
                if text.startswith("{") and '"variants"' in text:
                    found = json.loads(text)
        return found

    # bench_stdout.log: the profiled command's own line; unprofiled.log
    # (optional): the same command run without the profiler.
    line = unprof = None
    for f in _csv_files(root, "*.log"):
        if os.path.basename(f) == "unprofiled.log":
            unprof = json_line(f)
        else:
            line = json_line(f) or line
    if line is not None:
        traced = {_kernel_short(r["Name"]): float(r["AverageNs"]) / 1e3 for r in rows}
        pairs = [("fwd_comp_residual_kernel", "compensated", "fwd"),
                 ("adj_partial_kernel<1>", "compensated", "adj"),
                 ("fwd_plain_kernel", "plain", "fwd"), ("adj_partial_kernel<0>", "plain", "adj"),
                 ("fwd_rec_kernel<8, 4, 2>", "recurrence", "fwd"),
                 ("adj_partial_kernel<2>", "recurrence", "adj")]
        lines += ["", "Agreement with the HIP events that bench.py records around the same kernels "
                  "in the same profiled run (mean of the timed steps' launches; the trace "
                  "average also covers warm-up, graph-replay and accuracy-check launches)"
                  + (", and with the same command run without the profiler" if unprof else "")
                  + ":", "",
                  "| kernel | traced avg us | HIP-event mean us | traced / event |"
                  + (" unprofiled HIP-event mean us | traced / unprofiled |" if unprof else ""),
                  "|---|---|---|---|" + ("---|---|" if unprof else "")]
        for k, v, op in pairs:
            ev = line["variants"].get(v, {}).get(op + "_kernel_ms")
            if k in traced and ev:
                row = "| %s | %.1f | %.1f | %.3f |" % (k, traced[k], ev * 1e3,
                                                       traced[k] / (ev * 1e3))
                uv = unprof["variants"].get(v, {}).get(op + "_kernel_ms") if unprof else None
                if uv:
                    row += " %.1f | %.3f |" % (uv * 1e3, traced[k] / (uv * 1e3))
                lines.append(row)
        lines += ["", "Profiled step of the headline (compensated) variant: %.3f ms." %
                  line["ms_per_step"]]
        if unprof:
            lines.append("Unprofiled step of the same command: %.3f ms." % unprof["ms_per_step"])
    _write_md("bench_paper_1920x1024_n1024_kernel_stats.md", lines)


# Kernels whose traffic is recorded, with the sources their code comes from
# (bench.py reports a kernel's traffic only while these hash the same) and
# the algorithmic bytes of one launch at the headline workload.
TRAFFIC_KERNELS = {
    "adj_partial_kernel<1>": (["adjoint.hip", "phase.h", "records.h", "cgh_internal.h"],
                              "G 7.86 MB + row table 8.39 MB + column table 7.86 MB + "
                              "inputs 0.02 MB + run partials 9.44 MB (576 runs: three rounds "
                              "of 3 waves per SIMD over 16 point groups) = 33.6 MB"),
    "adj_partial_kernel<0>": (["adjoint.hip", "phase.h", "records.h", "cgh_internal.h"],
                              "G 7.86 MB + inputs 0.02 MB + run partials 12.58 MB (768 runs: "
                              "4 waves per SIMD)"),
    "adj_partial_kernel<2>": (["adjoint.hip", "phase.h", "records.h", "cgh_internal.h"],
                              "G 7.86 MB + inputs 0.02 MB + run partials 9.44 MB (576 runs)"),
    "fwd_comp_residual_kernel": (["forward.hip", "phase.h", "cgh_internal.h"],
                                 "row table 4.19 MB + column table 7.86 MB + amplitudes + "
                                 "hologram 7.86 MB + target 7.86 MB + residual 7.86 MB = 35.6 MB"),
    "fwd_plain_kernel": (["forward.hip", "phase.h", "cgh_internal.h"],
                         "records 0.02 MB + hologram 7.86 MB"),
    "fwd_rec_kernel<8, 4, 2>": (["forward.hip", "phase.h", "cgh_internal.h"],
                             "records 0.02 MB + hologram 7.86 MB"),
    "prep_kernel": (["prep.hip", "phase.h", "records.h", "cgh_internal.h"],
                    "inputs 0.02 MB + records 0.2 MB (+ f64 records)"),
    "gemm_f32_kernel<true, true, 0>": (["gemm.hip", "fold.h", "phase.h", "cgh_internal.h"],
                                       "tables 8.4 + 15.7 MB + split planes (forward)"),
    "gemm_f32_kernel<false, false, 1>": (["gemm.hip", "fold.h", "phase.h", "cgh_internal.h"],
                                         "tables 8.4 MB + G 7.86 MB + fold planes 0.5 MB"),
    "gemm_f32_kernel<false, true, 2>": (["gemm.hip", "fold.h", "phase.h", "cgh_internal.h"],
                                        "tables 15.7 MB + G 7.86 MB + fold planes 0.5 MB"),
    "gemm_half_kernel<2, 0>": (["gemm_half.hip", "fold.h", "phase.h", "cgh_internal.h"],
                               "hi+lo tables 12 MB + split planes (forward)"),
    "gemm_half_kernel<2, 1>": (["gemm_half.hip", "fold.h", "phase.h", "cgh_internal.h"],
                               "hi+lo tables 4.2 MB + hi+lo G 7.9 MB + fold planes 0.5 MB"),
    "gemm_half_kernel<2, 2>": (["gemm_half.hip", "fold.h", "phase.h", "cgh_internal.h"],
                               "hi+lo tables 7.9 MB + hi+lo G 7.9 MB + fold planes 0.5 MB"),
    "gemm_half_kernel<0, 0>": (["gemm_half.hip", "fold.h", "phase.h", "cgh_internal.h"],
                               "fp16 tables 6 MB + split planes (forward)"),
    "sep_sum_slices_kernel": (["separable.hip", "phase.h", "cgh_internal.h"],
                              "split planes + hologram 7.86 MB"),
    "sep_adj_operands_half_kernel<2>": (["separable_half.hip", "phase.h", "cgh_internal.h"],
                                        "G 7.86 MB in; G, Gt, Xt, Yt hi+lo planes 41 MB out"),
}


def _code_text(text):
    """Source text without comments and with whitespace collapsed, so that a
    comment edit leaves a kernel's recorded traffic valid and a code edit
    does not."""
    import re

    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def _sources_hash(sources, base=None):
    import hashlib

    base = base or os.path.join(ROOT, "paper_1002_0916_amd", "csrc")
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(base, name)) as f:
            h.update(_code_text(f.read()).encode())
    return h.hexdigest()[:16]


def summarize_traffic(root):
    """HBM bytes per launch from FETCH_SIZE and WRITE_SIZE runs of the benchmark,
    scaled by what the same counters read for a plain copy of known size."""
    copy_bytes = 268435456
    fe = _counter_means(_csv_files(os.path.join(root, "fetch"), "*counter_collection.csv"))
    wr = _counter_means(_csv_files(os.path.join(root, "write"), "*counter_collection.csv"))
    cf = _counter_means(_csv_files(os.path.join(root, "copy_fetch"), "*counter_collection.csv"))
    cw = _counter_means(_csv_files(os.path.join(root, "copy_write"), "*counter_collection.csv"))
    copy_f = cf["__amd_rocclr_copyBuffer"]["FETCH_SIZE"]
    copy_w = cw["__amd_rocclr_copyBuffer"]["WRITE_SIZE"]
    ff, wf = copy_f * 1024 / copy_bytes, copy_w * 1024 / copy_bytes
    # Read requests by size (optional pass): FETCH_SIZE's gfx950 formula counts
    # a 128-byte request as 64 bytes, so the copy-derived factor is right only
    # for kernels whose reads come in 128-byte requests.
    rq = cq = {}
    if os.path.isdir(os.path.join(root, "rdreq")):
        rq = _counter_means(_csv_files(os.path.join(root, "rdreq"), "*counter_collection.csv"))
        cq = _counter_means(_csv_files(os.path.join(root, "copy_rdreq"),
                                       "*counter_collection.csv"))

    def sized(c):
        return (32 * c["TCC_EA0_RDREQ_32B_sum"] + 64 * c["TCC_EA0_RDREQ_64B_sum"]
                + 128 * c["TCC_EA0_RDREQ_128B_sum"])

    copy_sized = sized(cq["__amd_rocclr_copyBuffer"]) if "__amd_rocclr_copyBuffer" in cq else None
    kernels = {}
    for k, (sources, _) in TRAFFIC_KERNELS.items():
        if k not in fe or k not in wr:
            print("no counters for", k)
            continue
        f_raw, w_raw = fe[k]["FETCH_SIZE"], wr[k]["WRITE_SIZE"]
        kernels[k] = {"fetch_kib_raw": round(f_raw, 1), "write_kib_raw": round(w_raw, 1),
                      "fetch_bytes": f_raw * 1024 / ff, "write_bytes": w_raw * 1024 / wf,
                      "traffic_bytes": f_raw * 1024 / ff + w_raw * 1024 / wf,
                      "source_sha256_16": _sources_hash(sources), "sources": sources}
        if k in rq:
            c = rq[k]
            kernels[k].update({
                "read_requests": {"32B": c["TCC_EA0_RDREQ_32B_sum"],
                                  "64B": c["TCC_EA0_RDREQ_64B_sum"],
                                  "128B": c["TCC_EA0_RDREQ_128B_sum"]},
                "read_bytes_sized": sized(c),
                "traffic_bytes_sized": sized(c) + w_raw * 1024 / wf})
    rec = {"workload": "1920x1024 hologram, N=1024 points (bench.py step)",
           "copy_reference_bytes": copy_bytes, "fetch_factor": ff, "write_factor": wf,
           "copy_read_bytes_sized": copy_sized, "kernels": kernels}
    with open(os.path.join(PROFILES, "traffic_paper_1920x1024_n1024.json"), "w") as f:
        json.dump(rec, f, indent=1)
    runs = [("fetch", "FETCH_SIZE", "bench.py --steps 3 --warmup 1 --no-cpu-baseline"),
            ("write", "WRITE_SIZE", "bench.py --steps 3 --warmup 1 --no-cpu-baseline"),
            ("copy_fetch", "FETCH_SIZE", "bench.py --copy-bytes %d" % copy_bytes),
            ("copy_write", "WRITE_SIZE", "bench.py --copy-bytes %d" % copy_bytes)]
    lines = ["# HBM traffic per launch: bench.py step at 1920x1024, N=1024", "",
             "Commands (from the repository root on an MI355X machine, one counter per run), then "
             "`python bench.py --summarize traffic <out>`:", "", "```", _ROCPROF.rstrip(" &")]
    if rq:
        runs += [("rdreq", RDREQ_COUNTERS, "bench.py --steps 3 --warmup 1 --no-cpu-baseline"),
                 ("copy_rdreq", RDREQ_COUNTERS, "bench.py --copy-bytes %d" % copy_bytes)]
    for d, counter, cmd in runs:
        lines.append("timeout -s KILL 150 rocprofv3 --kernel-trace --pmc %s -f csv -d <out>/%s "
                     "-o %s -- python3 %s" % (counter, d, d, cmd))
    lines += ["```", "",
              "Calibration: a plain %d-byte device copy (`__amd_rocclr_copyBuffer`, reads and "
              "writes that many bytes) reads FETCH_SIZE = %.0f KiB and WRITE_SIZE = %.0f KiB per "
              "dispatch, so bytes = FETCH_SIZE x 1024 / %.5f and WRITE_SIZE x 1024 / %.3f."
              % (copy_bytes, copy_f, copy_w, ff, wf), "",
              "Counter values are averages over the kernel's dispatches in the run (every "
              "variant of the step).  `traffic_paper_1920x1024_n1024.json` holds the same "
              "figures with a hash of each kernel's sources; bench.py reports the traffic of "
              "the roofline kernel only while that hash matches.", "",
              "| kernel | FETCH_SIZE KiB (raw) | WRITE_SIZE KiB (raw) | fetch | write | total | "
              "algorithmic bytes |", "|---|---|---|---|---|---|---|"]
    for k, v in kernels.items():
        lines.append("| %s | %.0f | %.0f | %.2f MB | %.2f MB | %.2f MB | %s |" % (
            k, v["fetch_kib_raw"], v["write_kib_raw"], v["fetch_bytes"] / 1e6,
            v["write_bytes"] / 1e6, v["traffic_bytes"] / 1e6, TRAFFIC_KERNELS[k][1]))
    if rq:
        lines += ["", "## Reads by request size", "",
                  "On gfx950 the FETCH_SIZE expression counts a 128-byte read request as 64 bytes "
                  "(the copy above reads %.4f of its bytes), so the copy factor is exact only for "
                  "128-byte requests.  Scalar loads (the direct kernels' point records and rows "
                  "of G) come in 64-byte requests, which FETCH_SIZE already counts in full, and "
                  "the copy factor doubles them.  Counting each request at its size "
                  "(TCC_EA0_RDREQ_32B, _64B, _128B) gives the reads below; the copy reads %.1f MB "
                  "of its %.1f MB this way."
                  % (ff, (copy_sized or 0) / 1e6, copy_bytes / 1e6), "",
                  "| kernel | 32 B requests | 64 B requests | 128 B requests | reads (sized) | "
                  "reads (copy-scaled FETCH_SIZE) | total (sized reads + writes) |",
                  "|---|---|---|---|---|---|---|"]
        for k, v in kernels.items():
            if "read_bytes_sized" not in v:
                continue
            r = v["read_requests"]
            lines.append("| %s | %.0f | %.0f | %.0f | %.2f MB | %.2f MB | %.2f MB |" % (
                k, r["32B"], r["64B"], r["128B"], v["read_bytes_sized"] / 1e6,
                v["fetch_bytes"] / 1e6, v["traffic_bytes_sized"] / 1e6))
    _write_md("traffic_paper_1920x1024_n1024.md", lines)


RDREQ_COUNTERS = ("TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum "
                  "TCC_EA0_RDREQ_sum")

# Algorithmic bytes of one launch of the compensated kernels at 3840x2160,
# N = 16384 (npad 16384): tables of FP32 per (row or column, point).
FIT4K_ALGORITHMIC = {
    "fwd_comp_kernel": (2160 * 16384 * 4 + 3840 * 16384 * 4 + 2160 * 3840 * 4,
                        "row table 141.6 MB + column table 251.7 MB + hologram 33.2 MB"),
    "adj_partial_kernel<1>": (2160 * 3840 * 4 + 2160 * 16384 * 8 + 3840 * 16384 * 4
                              + 36 * 16384 * 16,
                              "G 33.2 MB + row table 283.1 MB + column table 251.7 MB + "
                              "run partials 9.4 MB (36 runs: three rounds of 3 waves per SIMD "
                              "over 256 point groups)"),
}


def summarize_traffic_fit4k(root):
    """HBM bytes per launch of the compensated kernels at 3840x2160, N=16384
    (copy-calibrated FETCH_SIZE and WRITE_SIZE of `bench.py --workload fit4k
    --only --fit-iters 0`)."""
    copy_bytes = 268435456
    fe = _counter_means(_csv_files(os.path.join(root, "fetch"), "*counter_collection.csv"))
    wr = _counter_means(_csv_files(os.path.join(root, "write"), "*counter_collection.csv"))
    cf = _counter_means(_csv_files(os.path.join(root, "copy_fetch"), "*counter_collection.csv"))
    cw = _counter_means(_csv_files(os.path.join(root, "copy_write"), "*counter_collection.csv"))
    ff = cf["__amd_rocclr_copyBuffer"]["FETCH_SIZE"] * 1024 / copy_bytes
    wf = cw["__amd_rocclr_copyBuffer"]["WRITE_SIZE"] * 1024 / copy_bytes
    cmd = "bench.py --workload fit4k --only --variant compensated --fit-iters 0"
    lines = ["# HBM traffic per launch: compensated kernels at 3840x2160, N=16384", "",
             "Commands (from the repository root on an MI355X machine, one counter per run), then "
             "`python bench.py --summarize traffic_fit4k <out>`:", "", "```",
             _ROCPROF.rstrip(" &")]
    for d, counter, c in (("fetch", "FETCH_SIZE", cmd), ("write", "WRITE_SIZE", cmd),
                          ("copy_fetch", "FETCH_SIZE", "bench.py --copy-bytes %d" % copy_bytes),
                          ("copy_write", "WRITE_SIZE", "bench.py --copy-bytes %d" % copy_bytes)):
        lines.append("timeout -s KILL 300 rocprofv3 --kernel-trace --pmc %s -f csv -d <out>/%s "
                     "-o %s -- python3 %s" % (counter, d, d, c))
    lines += ["```", "", "Copy calibration as for the 1920x1024 record: bytes = FETCH_SIZE x 1024 "
              "/ %.5f and WRITE_SIZE x 1024 / %.3f." % (ff, wf), "",
              "| kernel | fetch | write | total | algorithmic bytes | total / algorithmic |",
              "|---|---|---|---|---|---|"]
    for k, (alg, what) in FIT4K_ALGORITHMIC.items():
        if k not in fe or k not in wr:
            print("no counters for", k)
            continue
        f, w = fe[k]["FETCH_SIZE"] * 1024 / ff, wr[k]["WRITE_SIZE"] * 1024 / wf
        lines.append("| %s | %.1f MB | %.1f MB | %.1f MB | %s = %.1f MB | %.2f |" % (
            k, f / 1e6, w / 1e6, (f + w) / 1e6, what, alg / 1e6, (f + w) / alg))
    _write_md("traffic_fit4k_3840x2160_n16384.md", lines)

COUNTER_PASSES = (
    "SQ_INSTS_VALU SQ_INSTS_VALU_TRANS_F32 SQ_INSTS_SALU SQ_INSTS_SMEM SQ_INSTS_LDS SQ_WAVES "
    "GRBM_GUI_ACTIVE",
    "SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_MFMA SQ_VALU_MFMA_BUSY_CYCLES "
    "GRBM_GUI_ACTIVE GRBM_COUNT",
)
# Direct kernels per variant, with the roofline key of their algorithmic work
# per interaction (FP32_OPS + TRANS_OPS instructions).
COUNTER_KERNELS = {
    "compensated": {"fwd_comp_residual_kernel": "fwd_compensated",
                    "adj_partial_kernel<1>": "adj_compensated"},
    "plain": {"fwd_plain_kernel": "fwd_plain", "adj_partial_kernel<0>": "adj_plain"},
    "recurrence": {"fwd_rec_kernel<8, 4, 2>": "fwd_recurrence",
                   "adj_partial_kernel<2>": "adj_recurrence"},
}


def summarize_counters(root):
    """Per-interaction VALU, transcendental, SALU, SMEM and LDS instruction
    counts and VALU issue rate of the direct kernels, and matrix-core use of the
    fp16 hi/lo GEMM, from two counter passes per variant (DIR/<variant>.<pass>)."""
    variants = list(COUNTER_KERNELS) + ["separable_f16x3"]
    data = {}
    for v in variants:
        files = [f for p in (1, 2)
                 for f in _csv_files(os.path.join(root, "%s.%d" % (v, p)), "*counter_collection.csv")]
        data[v] = _counter_means(files)
    # The fp16 hi/lo GEMM runs as three instantiations per step (forward and
    # the two adjoint contractions, one dispatch each): average them.
    half = [c for k, c in data["separable_f16x3"].items() if k.startswith("gemm_half_kernel<2,")]
    if half:
        data["separable_f16x3"]["gemm_half_kernel<2>"] = {
            name: sum(c[name] for c in half) / len(half) for name in half[0]}
    n = HEADLINE_INTERACTIONS
    lines = ["# Hardware counters of the hot kernels, 1920x1024 hologram, N = 1024", "",
             "Two counter passes per variant (rocprofv3 does not split counters over passes), "
             "from the repository root on an MI355X machine, then `python bench.py --summarize "
             "counters <out>`:", "", "```", _ROCPROF.rstrip(" &")]
    for v in variants:
        for i, counters in enumerate(COUNTER_PASSES, 1):
            lines.append("timeout -s KILL 90 rocprofv3 --pmc %s -f csv -d <out>/%s.%d -o pmc -- "
                         "python3 bench.py --variant %s --only --steps 5 --warmup 1 "
                         "--no-cpu-baseline" % (counters, v, i, v))
    lines += ["```", "",
              "Counter values are averages over the kernel's dispatches.  SQ_INSTS_* count wave "
              "instructions (64 lanes each) over the chip; GRBM_GUI_ACTIVE is summed over the 8 "
              "XCDs.  VALU issue is 4 SQ_ACTIVE_INST_VALU / (1024 SIMDs x GRBM_GUI_ACTIVE / 8): "
              "VALU instructions issued per SIMD per 4 clocks (a transcendental counting about "
              "1.3).  One per 4 clocks (100%) is the single-issue rate; gfx950 issues FP32 "
              "instructions whose operands are all VGPRs faster than that, so a kernel made of "
              "them can exceed 100% (the machine probe: up to 1.6 per CU clock).", "",
              "Per point-pixel interaction (N nx ny = %d; lanes that compute padding count).  "
              "Algorithmic: the FP32 operations and transcendentals the roofline counts; "
              "slots: FP32 ops + 4 per transcendental (quarter rate) of the FP32 vector peak."
              % n, "", "| kernel | VALU instr | of which transcendental | algorithmic instr "
              "(of which transcendental) | algorithmic slots | VALU issue | SALU / VALU | "
              "SMEM / VALU | LDS / VALU |",
              "|---|---|---|---|---|---|---|---|---|"]
    for v, ks in COUNTER_KERNELS.items():
        for k, key in ks.items():
            c = data[v].get(k)
            if c is None:
                print("no counters for", k)
                continue
            valu = c["SQ_INSTS_VALU"] * 64 / n
            tr = c["SQ_INSTS_VALU_TRANS_F32"] * 64 / n
            busy = 4 * c["SQ_ACTIVE_INST_VALU"] / (1024 * c["GRBM_GUI_ACTIVE"] / 8)
            lines.append("| `%s` | %.2f | %.2f | %d (%d) | %d | %.0f%% | %.3f | %.4f | %.4f |" % (
                k, valu, tr, FP32_OPS[key] + TRANS_OPS[key], TRANS_OPS[key], SLOTS[key],
                100 * busy,
                c["SQ_INSTS_SALU"] / c["SQ_INSTS_VALU"], c["SQ_INSTS_SMEM"] / c["SQ_INSTS_VALU"],
                c["SQ_INSTS_LDS"] / c["SQ_INSTS_VALU"]))
    g = data["separable_f16x3"].get("gemm_half_kernel<2>")
    if g is not None:
        mf = g["SQ_VALU_MFMA_BUSY_CYCLES"] / (1024 * g["GRBM_GUI_ACTIVE"] / 8)
        lines += ["", "Matrix-core kernel (`gemm_half_kernel<2>`, the fp16 hi/lo GEMM of the "
                  "separable_f16x3 variant; average over its forward and two adjoint dispatches "
                  "per step):", "",
                  "| MFMA instr / dispatch | MFMA busy cycles / MFMA | MFMA busy | LDS instr / MFMA "
                  "| VALU instr / MFMA |", "|---|---|---|---|---|",
                  "| %.0f | %.1f | %.0f%% | %.2f | %.2f |" % (
                      g["SQ_INSTS_MFMA"], g["SQ_VALU_MFMA_BUSY_CYCLES"] / g["SQ_INSTS_MFMA"],
                      100 * mf, g["SQ_INSTS_LDS"] / g["SQ_INSTS_MFMA"],
                      g["SQ_INSTS_VALU"] / g["SQ_INSTS_MFMA"])]
    lines += ["", "Raw averages per dispatch:", "", "| kernel | counter | value |", "|---|---|---|"]
    for v in variants:
        ks = list(COUNTER_KERNELS.get(v, {})) or ["gemm_half_kernel<2>"]
        for k in ks:
            for name, val in sorted(data[v].get(k, {}).items()):
                lines.append("| `%s` | %s | %.6g |" % (k, name, val))
    _write_md("counters_paper_1920x1024_n1024.md", lines)


def _json_lines(root, mode):
    """The JSON report lines of `mode` in the *.log files under root."""
    found = []
    for f in _csv_files(root, "*.log"):
        with open(f) as fh:
            for text in fh:
                if text.startswith("{"):
                    d = json.loads(text)
                    if d.get("mode") == mode:
                        found.append(d)
    if not found:
        raise SystemExit("no %s report line under %s" % (mode, root))
    return found


def _linear_fit(xs, ys):
    """Least-squares t = a + b N: (a, b, R^2, largest |residual| / t)."""
    n = len(xs)
    mx, my = sum(xs) / n, sum(ys) / n
    sxx = sum((x - mx) ** 2 for x in xs)
    b = sum((x - mx) * (y - my) for x, y in zip(xs, ys)) / sxx
    a = my - b * mx
    res = [y - (a + b * x) for x, y in zip(xs, ys)]
    ss = sum((y - my) ** 2 for y in ys)
    return a, b, 1 - sum(r * r for r in res) / ss, max(abs(r) / y for r, y in zip(res, ys))


def summarize_sweep(root):
    """Table 1's N-sweep at 1920x1024 (forward kernel times against N) with a
    linear fit per variant."""
    d = _json_lines(root, "sweep")[-1]
    rows = d["rows"]
    cmd = "timeout -k 10 300 python3 bench.py --sweep > <out>/sweep.log"
    lines = ["# Table 1 N-sweep: forward kernel at 1920x1024 against N", "",
             "Command (from the repository root on an MI355X machine), then `python bench.py "
             "--summarize sweep <out>`:", "", "```", cmd, "```", "",
             "Forward kernel time per launch (mean of 10 launches after a warm-up, HIP events "
             "around the kernel; the run starts with about 70 ms of untimed forwards, so that "
             "the clock has ramped up) for the seeded paper-shaped cloud of each N (x U[0,1920), "
             "y U[0,1024), z U[0.5,1] m, A U[0.5,1]).  The HD5850 column is the paper's Table 1 "
             "(its recurrence kernel on other hardware): context, not a target.  G/s = "
             "N x 1920 x 1024 / t.", "",
             "| N | HD5850 (paper) ms | plain ms | plain G/s | recurrence ms | recurrence G/s | "
             "compensated ms | compensated G/s | recurrence / paper speed-up |",
             "|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        paper = r.get("paper_hd5850_ms")
        lines.append("| %d | %s | %.3f | %.0f | %.3f | %.0f | %.3f | %.0f | %s |" % (
            r["n"], paper if paper else "-", r["plain_ms"], r["plain_gpps"], r["recurrence_ms"],
            r["recurrence_gpps"], r["compensated_ms"], r["compensated_gpps"],
            "%.0fx" % (paper / r["recurrence_ms"]) if paper else "-"))
    lines += ["", "Linear fit t = a + b N over all rows (time is linear in N at a fixed "
              "hologram, as in Table 1):", "",
              "| variant | a (us) | b (ns per point) | R^2 | largest residual / t |",
              "|---|---|---|---|---|"]
    ns = [r["n"] for r in rows]
    for v in ("plain", "recurrence", "compensated"):
        a, b, r2, worst = _linear_fit(ns, [r[v + "_ms"] for r in rows])
        lines.append("| %s | %.1f | %.2f | %.6f | %.2f%% |" % (v, a * 1e3, b * 1e6, r2,
                                                               100 * worst))
    a, b, r2, worst = _linear_fit([r["n"] for r in rows if r.get("paper_hd5850_ms")],
                                  [r["paper_hd5850_ms"] for r in rows if r.get("paper_hd5850_ms")])
    lines += ["", "The paper's HD5850 column fits t = a + b N with a = %.1f ms and b = %.1f us "
              "per point (R^2 = %.5f)." % (a, b * 1e3, r2)]
    _write_md("sweep_1920x1024.md", lines)


WORKLOAD_FILES = {"mesh8k": "workload_mesh8k_1920x1080.md",
                  "mesh64k": "workload_mesh64k_1920x1080.md",
                  "adjoint": "workload_adjoint_1024x1024.md",
                  "fit4k": "workload_fit4k_3840x2160.md"}


def summarize_workloads(root):
    """One summary per workload report line (--workload W), and the oracle
    timing (--oracle-timing), from the logs under root."""
    for d in _json_lines(root, "workload"):
        w = d["workload"]
        cmd = "timeout -k 10 900 python3 bench.py --workload %s > <out>/workload_%s.log" % (w, w)
        lines = ["# Workload %s: %dx%d hologram, N = %d" % (w, d["nx"], d["ny"], d["n_points"]),
                 "", d["description"], "",
                 "Command (from the repository root on an MI355X machine), then `python bench.py "
                 "--summarize workloads <out>`:", "", "```", cmd, "```", "",
                 "Kernel times are the mean of %d launches (HIP events around the kernel).  "
                 "Errors are max |dI| / sum |A| against the FP64 GPU forward on the full grid.  "
                 "Roofline fractions: of the FP32 vector peak for the direct variants (slots per "
                 "interaction as in bench.py), of the matrix-core peak of the GEMM operand type "
                 "for the separable ones; 'of mix' is the fraction of the same instruction mix run "
                 "alone by the machine probe." % d["reps"], "",
                 "FP64 GPU forward: %.2f ms (%.0f G interactions/s)." % (d["fwd_f64_ms"],
                                                                        d["fwd_f64_gpps"]), "",
                 "| variant | fwd ms | fwd G/s | fwd frac | fwd of mix | adj ms | adj G/s | "
                 "adj frac | adj of mix | max err / sum|A| |",
                 "|---|---|---|---|---|---|---|---|---|---|"]
        for v in ALL_VARIANTS:
            r = d.get(v)
            if not r:
                continue
            fm, am = r.get("fwd_frac_of_mix"), r.get("adj_frac_of_mix")
            if fm is None and mix_interactions("fwd_" + v):
                fm = r["fwd_gpps"] * 1e9 / mix_interactions("fwd_" + v)
            if am is None and mix_interactions("adj_" + v):
                am = r["adj_gpps"] * 1e9 / mix_interactions("adj_" + v)
            lines.append("| %s | %.4g | %.0f | %.2f | %s | %.4g | %.0f | %.2f | %s | %.2e |" % (
                v, r["fwd_kernel_ms"], r["fwd_gpps"], r["fwd_roofline_frac"],
                "%.2f" % fm if fm else "-", r["adj_kernel_ms"], r["adj_gpps"],
                r["adj_roofline_frac"], "%.2f" % am if am else "-",
                r["max_err_vs_fp64_over_sum_abs_a"]))
        f = d.get("fit")
        if f:
            lines += ["", "## Fitting loop (%d Adam iterations, lr %g, %s)" % (
                f["iterations"], f["lr"], f["params"]), "",
                "- %.2f iterations/s (%.2f s in total)" % (f["iterations_per_s"], f["seconds"]),
                "- loss %.4g -> %.4g (%.1f%%)" % (f["loss_first"], f["loss_last"],
                                                   100 * (f["loss_last"] / f["loss_first"] - 1)),
                "- in the loop: forward %.2f ms (%.0f G/s), adjoint %.2f ms (%.0f G/s)" % (
                    f["fwd_kernel_ms"], f["fwd_gpps"], f["adj_kernel_ms"], f["adj_gpps"]),
                "- fitted cloud's compensated hologram against FP64: max |dI| / sum |A| = %.2e" %
                f["fitted_fwd_max_err_vs_fp64_over_sum_abs_a"], "",
                "Loss curve (L = 0.5 ||I - T||^2 before each iteration):", "",
                "| iteration | loss |", "|---|---|"]
            lines += ["| %d | %.6g |" % (i, v) for i, v in enumerate(f["loss_curve"])]
        _write_md(WORKLOAD_FILES.get(w, "workload_%s.md" % w), lines)
    try:
        o = _json_lines(root, "oracle_timing")[-1]
    except SystemExit:
        return
    lines = ["# Oracle timing on the MI355X machine's host CPU", "",
             "Command (from the repository root on an MI355X machine), then `python bench.py "
             "--summarize workloads <out>`:", "", "```",
             "timeout -k 10 900 python3 bench.py --oracle-timing > <out>/oracle_timing.log",
             "```", "",
             "CPU: %s, %d allowed cores.  Oracle: %s.  GPU: %s." % (
                 o["cpu_model"], o["cores"], o["oracle"], o["gpu"]), "",
             "| workload | what | threads | interactions | oracle s | oracle G/s | GPU G/s | "
             "GPU / oracle |", "|---|---|---|---|---|---|---|---|"]
    for r in o["rows"]:
        lines.append("| %s | %s | %d | %.3g | %.3g | %.3g | %.0f | %.3g |" % (
            r["workload"], r["what"], r["threads"], r["interactions"], r["seconds"],
            r["oracle_gpps"], r["gpu_gpps"], r["gpu_over_oracle"]))
    _write_md("oracle_timing.md", lines)


def summarize_library(root):
    """This library's GEMM kernels (average durations from the kernel-stats
    run of the default benchmark, ROOT/stats) against the platform's GEMM at
    the same contraction shapes (ROOT/library.log, `bench.py --library-gemm`)."""
    import csv

    lib = _json_lines(root, "library_gemm")[-1]
    ours = {}
    for f in _csv_files(os.path.join(root, "stats"), "*kernel_stats.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                ours[_kernel_short(r["Name"])] = float(r["AverageNs"]) / 1e3
    lines = ["# The separable GEMMs against the platform's GEMM library, 1920x1024, N = 1024",
             "", "Commands (from the repository root on an MI355X machine): the kernel-stats run "
             "of the default benchmark (`profiles/bench_paper_1920x1024_n1024_kernel_stats.md`) "
             "for this library's kernels, and", "", "```",
             "timeout -k 10 300 python3 bench.py --library-gemm > <out>/library.log", "```", "",
             "then `python bench.py --summarize library <out>`.  The platform's GEMM is "
             "`torch.matmul` (torch %s: hipBLASLt / rocBLAS), timed by events over 50 launches "
             "(launch gaps included, so its figures are upper bounds on its kernel time), on "
             "plain operands of the same shape: its output is in the operand type and has no "
             "epilogue, while this library's kernels write FP32 and the adjoint ones fold "
             "their output per point in the epilogue.  fp16 hi/lo runs as one fp16 GEMM of "
             "three times the depth.  Rates in TFLOP/s of the format's work (f16x3: three "
             "products); %% of the dense peak (FP32 157.3 TFLOP/s, fp16/bf16 2.5 PFLOP/s)."
             % lib["torch"], "",
             "| contraction (M x N x K) | format | library us | library TFLOP/s | % peak | "
             "this library us | TFLOP/s | % peak | speed-up |", "|---|---|---|---|---|---|---|---|---|"]
    for r in lib["results"]:
        peak = 157.3e12 if r["format"] == "f32" else 2.5e15
        key = SEP_OURS[r["format"]] % (SEP_F32_ARGS[r["fold"]] if r["format"] == "f32"
                                       else r["fold"])
        mine = ours.get(key)
        lt = r["flops"] / (r["us"] * 1e-6)
        row = "| %s (%d x %d x %d) | %s | %.1f | %.0f | %.1f%% |" % (
            r["gemm"], r["M"], r["N"], r["K"], r["format"], r["us"], lt / 1e12, 100 * lt / peak)
        if mine:
            mt = r["flops"] / (mine * 1e-6)
            row += " %.1f | %.0f | %.1f%% | %.2fx |" % (mine, mt / 1e12, 100 * mt / peak,
                                                      r["us"] / mine)
        else:
            row += " - | - | - | - |"
        lines.append(row)
    _write_md("gemm_library_comparison_1920x1024.md", lines)


def summarize(kind, root):
    fn = {"stats": summarize_stats, "traffic": summarize_traffic,
          "traffic_fit4k": summarize_traffic_fit4k, "counters": summarize_counters,
          "sweep": summarize_sweep, "workloads": summarize_workloads,
          "library": summarize_library, "ramp": summarize_ramp}.get(kind)
    if fn is None:
        raise SystemExit("--summarize KIND must be stats, traffic, traffic_fit4k, counters, "
                         "sweep, workloads, library or ramp")
    fn(root)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
