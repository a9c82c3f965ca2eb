"""Benchmark of the first-passage hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload srusr_is_fp32|srusr_fp64]
                    [--n-traj N] [--no-cpu-baseline]

One bench step is one full pass of the hot path over the workload's batch of
trajectories: Philox -> Box-Muller -> noise-table lookup -> drift -> bias ->
Euler-Maruyama update -> log-weight -> first passage -> retire/refill ->
LDS histogram, with inputs already resident on the device.  The default
workload is the SR -> USR piecewise-linear potential with the Bessel-ansatz
noise table, FP32 state with FP64 log-weights and a constant importance-sampling
bias A = 2 over 1e8 trajectories (dN = 1e-4, 256 log-spaced bins), the
configuration whose far tail reaches P(deltaN) ~ 1e-10.

Prints one JSON line: trajectory-steps/s (device step counter / wall time), the
ESS-weighted tail-sample rate at the P = 1e-10 tail, the roofline of the EM
kernel (algorithmic FP operations per step x launches / HIP-event kernel time)
and the CPU oracle timed on a bounded sample on the host cores.
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

METRIC = "trajectory-steps/s and ESS-weighted tail samples/s at 5% P(δN) tail error"

# Algorithmic work of one trajectory step (constant bias, phi-indexed table,
# piecewise-linear potential), counted operation by operation from the step's
# definition; FMA = 2 FLOPs, a transcendental = 1.  Derivation in the design doc.
ALG_FLOPS_PER_STEP = {"fp32": 56.5, "fp64": 58.5}
ALG_INT_OPS_PER_STEP = 16.0          # Philox4x32-10 amortised over 4 steps + uniform conversions
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}   # MI355X vector peaks (FP32 figure assumes packed issue)
PEAK_HBM_GBS = 8000.0


def _workload(name: str, n_traj: int | None):
    from paper_2410_13683_amd import workloads as W
    if name == "srusr_is_fp32":
        w = W.srusr_is_fp32(A_bias=2.0)
    elif name == "srusr_fp64":
        w = W.srusr_bessel()
    else:
        raise SystemExit(f"unknown workload {name}")
    if n_traj:
        w = w.with_(n_traj=int(n_traj))
    return w


def cpu_baseline(w, target_s: float = 20.0) -> dict:
    """The CPU oracle, as it stands, on the first trajectories of the same workload."""
    from oracle import oracle as orc
    from tests._glue import oracle_problem
    prob = oracle_problem(w)
    threads = orc.max_threads()
    n0 = max(64, threads * 8)
    t0 = time.perf_counter()
    _, _, st = orc.run(prob, w.dN, w.seed, n0, max_steps=w.max_steps)
    dt0 = time.perf_counter() - t0
    steps0 = int((st & orc.STEP_MASK).astype("uint64").sum())
    n1 = int(min(max(n0, n0 * target_s / max(dt0, 1e-3)), 2_000_000))
    t1 = time.perf_counter()
    _, _, st = orc.run(prob, w.dN, w.seed, n1, traj_offset=n0, max_steps=w.max_steps)
    dt1 = time.perf_counter() - t1
    steps1 = int((st & orc.STEP_MASK).astype("uint64").sum())
    return {"value": steps1 / dt1, "unit": "trajectory-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"trajectories {n0}..{n0 + n1 - 1} of the same workload ({steps1} steps, "
                      f"{dt1:.1f} s, FP64 oracle, OpenMP over trajectories)",
            "seconds": dt1}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="srusr_is_fp32")
    ap.add_argument("--n-traj", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-side", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run one device-to-device copy of BYTES (a known-size kernel that scales the "
                         "profiler's FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(trajectories would shard by index with one histogram all-reduce; see DESIGN.md).",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2410_13683_amd import runner

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = _workload(args.workload, args.n_traj)
    prec = "fp32" if w.precision == 1 else "fp64"
    ctx = runner.context_for(w)
    stream = torch.cuda.current_stream()
    print(f"[bench] workload {w.name}: {w.n_traj:.3g} trajectories, warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        ctx.run(w.n_traj, w.dN, w.seed, 0, stream)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1} done ({ctx.last_kernel_ms():.0f} ms)", file=sys.stderr, flush=True)
    ctx.reset()
    kernel_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        # step k covers trajectories k*n .. (k+1)*n-1: fresh samples every step
        ctx.run(w.n_traj, w.dN, w.seed, k * w.n_traj, stream)
        kernel_ms.append(ctx.last_kernel_ms())
        print(f"[bench] step {k + 1}/{args.steps}: {kernel_ms[-1]:.0f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    hist = ctx.histogram()
    ctx.destroy()

    steps_total = int(hist["n_steps_total"])
    value = steps_total / wall
    x_star, p_star, ess_T, n_T = runner.tail_ess(hist, w.n_bins, w.bins_kind, w.lo, w.hi, 1e-10)
    ess_rate = ess_T / wall
    avg_ms = float(np.mean(kernel_ms))
    steps_per_launch = steps_total / args.steps
    achieved = ALG_FLOPS_PER_STEP[prec] * steps_per_launch / (avg_ms * 1e-3) / 1e12
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "potential": "piecewise-linear slow roll -> ultra-slow roll, V0=1e-10, eps+=0.01, eps-=1e-8",
            "noise": f"Bessel-ansatz table, {w.table_n} phi nodes, sigma={w.sigma}",
            "state": "FP32 pairs + FP64 log-weights" if prec == "fp32" else "FP64",
            "bias_A": w.A_bias,
            "trajectories_per_step": w.n_traj,
            "dN": w.dN,
            "bins": f"{w.n_bins} {'log' if w.bins_kind else 'linear'} over deltaN in [{w.lo:.4g}, {w.hi:.4g})",
        },
        "ess_tail_per_s": ess_rate,
        "tail": {"deltaN_star": x_star, "P_tail": p_star, "ESS_T": ess_T, "samples_in_T": n_T,
                 "t_5pct_s": (400.0 / ess_rate) if ess_rate > 0 else None},
        "trajectory_steps": steps_total,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_TFLOPS[prec],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[prec],
            "traffic": None,
            "kernel": "em_fp32s_kernel" if prec == "fp32" else "em_fp64_kernel",
            "kernel_ms": avg_ms,
            "flops_per_step": ALG_FLOPS_PER_STEP[prec],
            "int_ops_per_step": ALG_INT_OPS_PER_STEP,
        },
    }
    if not args.no_fp64_side and prec == "fp32":
        w64 = _workload("srusr_fp64", None)
        c64 = runner.context_for(w64)
        c64.run(w64.n_traj, w64.dN, w64.seed, 0, stream)
        torch.cuda.synchronize()
        c64.reset()
        t1 = time.perf_counter()
        c64.run(w64.n_traj, w64.dN, w64.seed, w64.n_traj, stream)
        ms64 = c64.last_kernel_ms()
        torch.cuda.synchronize()
        wall64 = time.perf_counter() - t1
        h64 = c64.histogram()
        c64.destroy()
        s64 = int(h64["n_steps_total"])
        result["fp64_srusr"] = {"trajectories": w64.n_traj, "trajectory_steps_per_s": s64 / wall64,
                                "kernel_ms": ms64,
                                "tflops": ALG_FLOPS_PER_STEP["fp64"] * s64 / (ms64 * 1e-3) / 1e12}
        print(f"[bench] fp64 side run: {s64 / wall64:.3e} steps/s", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
