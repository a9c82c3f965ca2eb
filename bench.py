"""Benchmark of the first-passage hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--n-traj N] [--no-cpu-baseline]
                    [--workload srusr_is_fp32|srusr_fp64|srusr_2d|srusr_learned|batched]

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

--workload srusr_learned measures the learned control on the same problem: the
constant-bias fallback A in {0.5, 1, 2} (one pass each; its best ESS_T rate is
the comparison), then training of the 2->64->64->2 network from the constant
A = 1 on 3e7 generated trajectories in 120 iterations (replay gradient of
ln E[w^2 1_T] with T the P = 1e-10 tail found by the A = 2 pass, Adam), then
the timed passes with the trained, tabulated control.  After them (outside the timed region) the trained
network itself, evaluated every 64 and every 16 steps, runs one pass of 1e7 fresh
trajectories each: its rate and tail ESS beside the tabulated control's.

--workload srusr_2d runs the SR -> USR problem with 2D noise (the covariance of the
full Bunch-Davies mode at -k eta = 0.1 on 2048 nodes), FP64 state, 1e6 trajectories.

--workload batched measures many problems in one persistent launch: the 64
SR -> USR instances with eps_- log-uniform in [1e-10, 1e-6], phi_e - phi_end
uniform in [0.1, 1] and trajectory counts log-uniform in [1e4, 1e6] (a tenth of
the [1e5, 1e7] range, so one pass takes seconds), FP32 state, a cap of 2^20
steps per trajectory (most flat-branch runs are censored); the batch is
autotuned, captured as a hipGraph and replayed for the timed passes, and the
same work as 64 consecutive single-problem launches is timed beside it.
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

# Floating-point work of one trajectory step (constant bias, phi-indexed table, piecewise-linear
# potential), the method's algorithmic count with FMA = 2 FLOPs: the drift (3 - pi^2/2)(pi + V'/V) 8,
# the table lookup (coordinate, clamp, fraction, two interpolations) 10, noise and bias 4, the phi
# update 4 plus 4 for its float-pair accumulation, the pi update 6, the crossing and eps_1 tests 2,
# half a Box-Muller pair (log, square root, sine and cosine, scalings) 5, the FP64 log-weight 2:
# 45.  It is the same for every FP32-state kernel revision (the work of the method, not of one
# implementation); the FP64 path's own operation count (54.5 with a bias, 47.5 without) is kept
# for its side run.
ALG_FLOPS_PER_STEP = {"fp32": 45.0, "fp64": 54.5}
# FP64 without a bias: no A S, pi + A S, A S dN + noise or ln w (7 of the 54.5)
ALG_FLOPS_FP64_NO_BIAS = 54.5 - 7.0
# FP32 state without a bias: no log-weight (2 of the 45)
ALG_FLOPS_FP32_NO_BIAS = 45.0 - 2.0
# the tabulated learned control adds its grid coordinates (ln|pi| included), the clamped
# cell and fractions, the bilinear interpolation and the per-step dA = a xi sqrt(dN) + a^2 dN/2
# (31); in FP32 also a S and its separate FMA into the increment (3), less the offset of the
# Box-Muller FMAs, which it does not use (1)
ALG_FLOPS_LEARNED_EXTRA = {"fp32": 33.0, "fp64": 31.0}
# FP64 state with 2D noise, no bias: a Box-Muller pair per step (13), V'/V (9), five interpolated
# table entries (23), the 2x2 noise product (6), the update (12), events (4); a constant bias adds
# B = a S e (8) and dA (10)
ALG_FLOPS_2D = {"none": 67.0, "const": 85.0}
# the Gaussian bump's V'/V (FP64): x, x^2/2, exp, K g, phi (m^2 + phi^2), Sigma (1 + g), the
# numerator 2 m^2 d2 - x g d1, the denominator, its reciprocal with one Newton step and the product
# = 22 FLOPs in place of the linear potentials' 9
ALG_FLOPS_BUMP_FP64 = 54.5 - 9.0 + 22.0
# FP32 state on a time-indexed table: V'/V exactly (phi - phi_T from the float pair, 3; the branch's
# compare, 1; the FMA, 2; the reciprocal, 1) in place of its interpolation and NaN test (3); the last
# node is zero, so the weight tests S > 0 (1)
ALG_FLOPS_TIME_FP32 = 45.0 - 3.0 + 7.0 + 1.0
ALG_INT_OPS_PER_STEP = 16.0          # Philox4x32-10 amortised over 4 steps + uniform conversions
PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}   # MI355X published vector peaks
PEAK_HBM_GBS = 8000.0

# HBM traffic of one launch of the default workload's kernel (FP32 state, constant bias, 1e8
# trajectories), from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch),
# each scaled by what the same counter reads for a 1 GiB device-to-device copy in the same
# process (FETCH_SIZE reads 0.5 GiB: x2.0; WRITE_SIZE reads 1 GiB: x1.0).  Valid only for the
# kernel source it was measured on (hash of the kernel file and its header).
MEASURED_TRAFFIC = {
    "source_sha256": "fdc53c6b19b7b05f38b14be916129ce282f97ac0dc66d910ad5b255d6c16be41",
    "workload": "srusr_is_fp32_A2", "n_traj": 100_000_000,
    "fetch_bytes": 10942.5625 * 1024 * 2.0, "write_bytes": 2127586.59375 * 1024 * 1.0,
}


def _code_tokens(text: str) -> str:
    """The C++ source without its comments and with whitespace runs collapsed: what the compiler
    sees, so that an edit of the comments alone keeps a measurement valid."""
    out, i, n = [], 0, len(text)
    while i < n:
        ch = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif ch in "\"'":
            j = i + 1
            while j < n and text[j] != ch:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(ch)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_sha() -> str:
    """Hash of the EM kernels' code (their source file and headers, comments left out)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("fpt_em.hip", "internal.hpp", "potential.hpp"):
        with open(os.path.join(ROOT, "paper_2410_13683_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(_code_tokens(fh.read()).encode())
    return h.hexdigest()


# rocprofv3's derived VALUBusy = 100 sum(SQ_ACTIVE_INST_VALU) / CU_NUM / GRBM_GUI_ACTIVE, from one
# --pmc VALUBusy VALUUtilization pass of one launch per kernel.  On gfx950 sum(SQ_ACTIVE_INST_VALU)
# equals the VALU instruction count to within a few per cent, so the figure is VALU instructions
# issued per CU per cycle (x100; four SIMDs per CU).  Valid only for the kernel source it was
# measured on, like the traffic.
# "hw_flops_per_step" and "insts_per_step" come from one --pmc pass of eight SQ_INSTS_VALU_*
# counters per kernel (one launch): 64 x wave-instructions / trajectory steps, FLOPs counted as
# 2 FMA + ADD + MUL + TRANS of each precision.  They measure what the compiled kernel executes,
# beside the operation-by-operation count of the method used for "achieved".
MEASURED_VALU = {
    "source_sha256": "fdc53c6b19b7b05f38b14be916129ce282f97ac0dc66d910ad5b255d6c16be41",
    "srusr_is_fp32_A2": {"VALUBusy": 139.295, "VALUUtilization": 98.989,
                         "hw_flops_per_step": {"f32": 27.720, "f64": 0.143},
                         "insts_per_step": {"FMA_F32": 10.352, "ADD_F32": 3.325, "MUL_F32": 1.689,
                                            "TRANS_F32": 2.003, "CVT": 1.263, "INT32": 0.625,
                                            "FMA_F64": 0.025, "ADD_F64": 0.094}},
    "srusr_bessel_fp64": {"VALUBusy": 95.481, "VALUUtilization": 99.712,
                          "hw_flops_per_step": {"f32": 0.0, "f64": 58.024},
                          "insts_per_step": {"FMA_F64": 20.433, "ADD_F64": 4.796, "MUL_F64": 10.848,
                                             "TRANS_F64": 1.514, "INT32": 3.664, "FMA_F32": 0.0,
                                             "ADD_F32": 0.0, "MUL_F32": 0.0}},
}
# the issue rate of independent v_fma_f32 chains, wave-instructions per SIMD per cycle, recorded
# with a register-only micro-kernel (16 waves per SIMD)
FMA_F32_ISSUE_CEILING = 0.352


def measured_valu(name: str):
    m = MEASURED_VALU
    if name not in m or kernel_source_sha() != m["source_sha256"]:
        return None
    v = dict(m[name])
    v["valu_issue_per_simd_cycle"] = v["VALUBusy"] / 100.0 / 4.0
    v["fma_f32_issue_ceiling"] = FMA_F32_ISSUE_CEILING
    return v


def hw_counted_rate(valu, steps_per_s):
    """TFLOP/s of the FLOPs the hardware counters saw the kernel execute (both precisions)."""
    if not valu or "hw_flops_per_step" not in valu:
        return None
    return sum(valu["hw_flops_per_step"].values()) * steps_per_s / 1e12


def measured_traffic(w):
    m = MEASURED_TRAFFIC
    if w.name != m["workload"] or w.n_traj != m["n_traj"] or kernel_source_sha() != m["source_sha256"]:
        return None, None
    detail = {"fetch_bytes": m["fetch_bytes"], "write_bytes": m["write_bytes"],
              "per_trajectory_bytes": (m["fetch_bytes"] + m["write_bytes"]) / m["n_traj"],
              "note": "writes are the work-queue claims (device-scope atomics, performed at the memory side); "
                      "no per-step traffic"}
    return m["fetch_bytes"] + m["write_bytes"], detail


def _workload(name: str, n_traj: int | None):
    from paper_2410_13683_amd import workloads as W
    if name == "srusr_is_fp32":
        w = W.srusr_is_fp32(A_bias=2.0)
    elif name == "srusr_fp64":
        w = W.srusr_bessel()
    elif name == "srusr_learned":
        w = W.srusr_learned(n_traj=100_000_000, A_init=1.0)
    elif name == "srusr_2d":
        w = W.srusr_2d()
    elif name == "srusr_2d_fp32":
        w = W.srusr_2d(n_traj=10_000_000).with_(name="srusr_2d_fp32", precision=1)
    elif name == "srusr_matched":
        w = W.srusr_is_fp32_matched(A_bias=2.0)
    elif name == "srusr_2d_time":
        w = W.srusr_2d_time()
    elif name == "srusr_time":
        w = W.srusr_is_fp32_time(A_bias=2.0)
    elif name == "bump":
        w = W.gaussian_bump_is(A_bias=3.0)
    elif name == "bump_time":
        w = W.gaussian_bump_time_is(A_bias=3.0)
    else:
        raise SystemExit(f"unknown workload {name}")
    if n_traj:
        w = w.with_(n_traj=int(n_traj))
    return w


def cpu_baseline(w, target_s: float = 20.0) -> dict:
    """The CPU oracle, as it stands, on the first trajectories of the same workload (its noise table
    built once, outside the timing)."""
    from oracle import oracle as orc
    from oracle.problems import NOISE_2D, oracle_problem, oracle_problem2d
    threads = orc.max_threads()
    kw = dict(instance=w.extra.get("instance", 0), max_steps=w.max_steps)
    if w.noise in NOISE_2D:
        p2 = oracle_problem2d(w)
        run = lambda n, off, nt=0: orc.run2d(p2, w.dN, w.seed, n, traj_offset=off, n_threads=nt, **kw)
    else:
        p1 = oracle_problem(w)
        run = lambda n, off, nt=0: orc.run(p1, w.dN, w.seed, n, traj_offset=off, n_threads=nt, **kw)
    n0 = max(64, threads * 8)
    t0 = time.perf_counter()
    _, _, st = run(n0, 0)
    dt0 = time.perf_counter() - t0
    n1 = int(min(max(n0, n0 * target_s / max(dt0, 1e-3)), 2_000_000))
    t1 = time.perf_counter()
    _, _, st = run(n1, n0)
    dt1 = time.perf_counter() - t1
    steps1 = int((st & orc.STEP_MASK).astype("uint64").sum())
    # one host thread on the trajectories that follow, for about a tenth of the time
    n2 = max(1, int(n1 * 0.1 / threads))
    t2 = time.perf_counter()
    _, _, st2 = run(n2, n0 + n1, 1)
    dt2 = time.perf_counter() - t2
    steps2 = int((st2 & orc.STEP_MASK).astype("uint64").sum())
    return {"value": steps1 / dt1, "unit": "trajectory-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"trajectories {n0}..{n0 + n1 - 1} of the same workload ({steps1} steps, "
                      f"{dt1:.1f} s, FP64 oracle, OpenMP over trajectories)",
            "seconds": dt1, "cpu_model": _cpu_model(),
            "value_1_thread": steps2 / dt2,
            "sample_1_thread": f"trajectories {n0 + n1}..{n0 + n1 + n2 - 1} ({steps2} steps, {dt2:.1f} s)"}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _tail_slot(hist, w, x):
    """The slot whose lower edge (from the library's bin edges) is nearest to x."""
    import numpy as np
    from paper_2410_13683_amd import fpt
    _, edges, _ = fpt.fpt_density(hist, w.bins_kind, w.n_bins, w.lo, w.hi, moments=False)
    return int(np.argmin(np.abs(edges - x))) + 1     # slot j + 1 starts at edges[j]


def tail_at(hist, w, x):
    """(P(deltaN >= x), ESS over those bins, samples there) for a bin edge x of the workload
    (fpt_tail_at)."""
    from paper_2410_13683_amd import fpt
    t = fpt.fpt_tail_at(hist, w.bins_kind, w.n_bins, w.lo, w.hi, _tail_slot(hist, w, x))
    return t["P"], t["ess"], int(t["count"])


def tail_errors(hist, w, x) -> dict:
    """One-sigma errors of P(deltaN >= x) from fpt_tail_at: the plain standard error of
    sum w 1_T / n, and the per-bin lognormal intervals added in quadrature over the tail bins."""
    from paper_2410_13683_amd import fpt
    t = fpt.fpt_tail_at(hist, w.bins_kind, w.n_bins, w.lo, w.hi, _tail_slot(hist, w, x))
    return {"P_tail_err": t["P_err"], "P_tail_err_lognormal": t["P_err_lognormal"]}


def train_learned(w, stream, train_traj: float = 3e7, iters: int = 120, lr: float = 0.03) -> dict:
    """Constant-bias fallback passes, then GPU training of the learned control (see the module
    docstring).  Returns the context holding the trained network and the figures."""
    import torch
    from paper_2410_13683_amd import fpt, runner
    from paper_2410_13683_amd import workloads as W
    out = {"constant_fallback": []}
    x_star = None
    for A in (0.5, 1.0, 2.0):
        wc = W.srusr_is_fp32(A_bias=A, n_traj=w.n_traj)
        c = runner.context_for(wc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.run(wc.n_traj, wc.dN, wc.seed, 0, stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        h = c.histogram()
        c.destroy()
        if A == 2.0:
            x_star = runner.tail_ess(h, wc.n_bins, wc.bins_kind, wc.lo, wc.hi, 1e-10)[0]
        out["constant_fallback"].append({"A": A, "wall_s": wall, "steps": int(h["n_steps_total"]), "hist": h})
        print(f"[bench] constant A={A}: {wall:.1f} s", file=sys.stderr, flush=True)
    for r in out["constant_fallback"]:
        h = r.pop("hist")
        p, ess, nT = tail_at(h, w, x_star)
        r.update(P_tail=p, ESS_T=ess, samples_in_T=nT, ess_tail_per_s=ess / r["wall_s"])
    out["deltaN_star"] = x_star
    ctx = runner.context_for(w, mlp_params=w.mlp_params, norm=w.mlp_norm, mlp_every=0, grid_n=w.grid_n,
                             grid_range=w.grid_range)
    d_grad = torch.zeros(fpt.FPT_MLP_NPARAM, dtype=torch.float32, device="cuda")
    n_it = int(train_traj) // iters
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Js = []
    for it in range(iters):
        # fresh trajectories every iteration, disjoint from the timed passes (index offset 2^40)
        J, _ = ctx.mlp_grad(n_it, w.dN, w.seed, x_star, d_grad, traj_offset=(1 << 40) + it * n_it, stream=stream,
                            objective=fpt.FPT_MLP_OBJ_LOG_J)
        ctx.mlp_adam(d_grad, lr, stream=stream)
        Js.append(J)
    torch.cuda.synchronize()
    out.update(ctx=ctx, train_trajectories=n_it * iters, train_iterations=iters, lr=lr, A_init=1.0,
               train_s=time.perf_counter() - t0, J_first=Js[0], J_last=Js[-1],
               objective="ln E[w^2 1(deltaN >= deltaN_star)]")
    print(f"[bench] training: {out['train_s']:.1f} s, J {Js[0]:.3e} -> {Js[-1]:.3e}", file=sys.stderr,
          flush=True)
    return out


def exact_network_passes(w, params, x_star, stream, every=(64, 16), n_traj: int = 10_000_000) -> list:
    """After the timed passes of the tabulated control: the trained network itself evaluated every
    k steps (mlp_every = k), one pass of n_traj fresh trajectories per k, each with its own context.
    Reports the rate and the tail ESS at the same deltaN*, beside the tabulated control's."""
    import torch
    from paper_2410_13683_amd import runner
    out = []
    for k in every:
        c = runner.context_for(w, mlp_params=params, mlp_every=k)
        c.run(n_traj // 100, w.dN, w.seed, 1 << 41, stream)          # warm-up, trajectories set apart
        torch.cuda.synchronize()
        c.reset()
        t0 = time.perf_counter()
        c.run(n_traj, w.dN, w.seed, (1 << 41) + k * n_traj, stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        h = c.histogram()
        ms = c.last_kernel_ms()
        c.destroy()
        p, ess, nT = tail_at(h, w, x_star)
        steps = int(h["n_steps_total"])
        out.append({"every": k, "trajectories": n_traj, "trajectory_steps_per_s": steps / wall, "kernel_ms": ms,
                    "P_tail": p, "ESS_T": ess, "samples_in_T": nT, "ess_tail_per_s": ess / wall})
        print(f"[bench] exact network every {k} steps: {steps / wall:.3e} steps/s, ESS_T {ess:.3g}", file=sys.stderr,
              flush=True)
    return out


def bench_multi_amplitude(args) -> dict:
    """Configuration 3 as written: the SR -> USR problem in FP32 state with the bias amplitudes
    A in {0.5, 1, 2}, 1e8 trajectories per amplitude.  A step is one pass at each of the three
    amplitudes (their own contexts and histograms, fresh trajectory indices each step), 3e8
    trajectories in all; at the end the tail masses of the three histograms are merged slot by slot with
    inverse-variance weights (fpt_tail_at for P(deltaN >= e_j) and its error at every slot,
    fpt_merge_bins), as Sec. 4.2 combines amplitudes where they agree."""
    import numpy as np
    import torch
    from paper_2410_13683_amd import fpt, runner
    from paper_2410_13683_amd import workloads as W
    amps = (0.5, 1.0, 2.0)
    n = int(args.n_traj) if args.n_traj else 100_000_000
    ws = [W.srusr_is_fp32(A_bias=A, n_traj=n) for A in amps]
    t_tab = time.perf_counter()
    ctxs = [runner.context_for(w) for w in ws]
    table_s = time.perf_counter() - t_tab
    stream = torch.cuda.current_stream()
    passes = [0, 0, 0]
    print(f"[bench] workload srusr_is_fp32_multiA: A in {amps}, {n:.3g} trajectories per pass, warmup "
          f"{args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        for a in range(3):
            ctxs[a].run(n, ws[a].dN, ws[a].seed, 0, stream)
            torch.cuda.synchronize()
            print(f"[bench] warmup {i + 1} (A={amps[a]:g}) done ({ctxs[a].last_kernel_ms():.0f} ms)",
                  file=sys.stderr, flush=True)
    for c in ctxs:
        c.reset()
    kernel_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for a in range(3):
            ctxs[a].run(n, ws[a].dN, ws[a].seed, passes[a] * n, stream)
            passes[a] += 1
            kernel_ms.append(ctxs[a].last_kernel_ms())
            print(f"[bench] step {k + 1}/{args.steps} (A={amps[a]:g}): {kernel_ms[-1]:.0f} ms", file=sys.stderr,
                  flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    hists = [c.histogram() for c in ctxs]
    for c in ctxs:
        c.destroy()
    w = ws[0]
    steps_total = int(sum(h["n_steps_total"] for h in hists))
    used = [i for i in range(3) if passes[i] > 0]
    # tail mass P(deltaN >= e_j) of every slot j = 1 .. n_bins + 1 and its standard error, per amplitude
    slots = range(1, w.n_bins + 2)
    P = np.full((len(used), len(slots)), np.nan)
    E = np.full_like(P, np.nan)
    for r, i in enumerate(used):
        for j in slots:
            t = fpt.fpt_tail_at(hists[i], w.bins_kind, w.n_bins, w.lo, w.hi, j)
            if t["count"] >= 2:
                P[r, j - 1], E[r, j - 1] = t["P"], t["P_err"]
    Pm, Em = fpt.fpt_merge_bins(P, E)
    _, edges, _ = fpt.fpt_density(hists[used[0]], w.bins_kind, w.n_bins, w.lo, w.hi, moments=False)
    deep = np.flatnonzero(np.isfinite(Pm) & (Pm > 0) & (Pm <= 1e-10))
    merged = None
    if len(deep):
        j = int(deep[0])                                 # lowest edge whose merged tail mass is <= 1e-10
        x_star = float(edges[j]) if j < w.n_bins else float(w.hi)
        ess_eq = (Pm[j] / Em[j]) ** 2                    # equally weighted samples with the same relative error
        merged = {"deltaN_star": x_star, "P_tail": float(Pm[j]), "P_tail_err": float(Em[j]), "ESS_equiv": ess_eq,
                  "ess_tail_per_s": ess_eq / wall, "t_5pct_s": 400.0 / (ess_eq / wall),
                  "per_amplitude": {f"{amps[i]:g}": {"passes": passes[i], "P_tail": float(P[r, j]),
                                                    "P_tail_err": float(E[r, j])}
                                    for r, i in enumerate(used)}}
    avg_ms = float(np.mean(kernel_ms))          # per launch (one amplitude)
    achieved = ALG_FLOPS_PER_STEP["fp32"] * steps_total / (float(np.sum(kernel_ms)) * 1e-3) / 1e12
    return {
        "metric": METRIC, "value": steps_total / wall, "unit": "trajectory-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "srusr_is_fp32_multiA", "amplitudes": list(amps), "trajectories_per_step": 3 * n, "trajectories_per_amplitude": n,
                   "potential": "piecewise-linear slow roll -> ultra-slow roll, V0=1e-10, eps+=0.01, eps-=1e-8",
                   "noise": f"Bessel-ansatz table, {w.table_n} phi nodes, sigma={w.sigma}",
                   "state": "FP32 pairs + FP64 log-weights", "dN": w.dN,
                   "bins": f"{w.n_bins} log over deltaN in [{w.lo:.4g}, {w.hi:.4g})"},
        "ess_tail_per_s": merged["ess_tail_per_s"] if merged else 0.0,
        "tail": merged, "trajectory_steps": steps_total, "table_setup_s": table_s,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["fp32"], "traffic": None,
                     "kernel": "em_kernel<FP32 state, const bias, table>", "kernel_ms": avg_ms,
                     "flops_per_step": ALG_FLOPS_PER_STEP["fp32"]},
    }


def bench_batched(args) -> dict:
    """Timed passes of the 64-instance batch (see the module docstring)."""
    import tempfile
    import numpy as np
    import torch
    from paper_2410_13683_amd import fpt, runner
    from paper_2410_13683_amd import workloads as W
    scale = args.n_traj if args.n_traj else 0.1
    ws = [w.with_(precision=1) for w in W.batched_instances()]
    counts = np.array([max(1, int(round(w.n_traj * scale))) for w in ws], dtype=np.uint64)
    ctxs = [runner.context_for(w) for w in ws]
    stream = torch.cuda.Stream()
    batch = fpt.Batch(ctxs, use_graph=True)
    dN, seed = ws[0].dN, ws[0].seed
    cache = os.path.join(tempfile.gettempdir(), "fpt_batch_tune.txt")
    t0 = time.perf_counter()
    batch.autotune(counts, dN, seed, cache_path=cache, stream=stream)
    tune_s = time.perf_counter() - t0
    block, chunk = batch.config()
    print(f"[bench] batched: {int(counts.sum())} trajectories over {len(ws)} instances; tuned block {block} "
          f"chunk {chunk} in {tune_s:.1f} s", file=sys.stderr, flush=True)
    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            batch.run(counts, dN, seed, 0, stream=stream)
            stream.synchronize()
            print(f"[bench] warmup {i + 1} done ({batch.last_ms():.0f} ms)", file=sys.stderr, flush=True)
        for c in ctxs:
            c.reset()
        kernel_ms = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            batch.run(counts, dN, seed, (k + 1) * (1 << 32), stream=stream)
            kernel_ms.append(batch.last_ms())
            print(f"[bench] step {k + 1}/{args.steps}: {kernel_ms[-1]:.0f} ms", file=sys.stderr, flush=True)
        stream.synchronize()
        wall = time.perf_counter() - t0
    hists = [c.histogram() for c in ctxs]
    steps_total = int(sum(h["n_steps_total"] for h in hists))
    censored = int(sum(h["n_censored"] for h in hists))
    # the same trajectories as consecutive single-problem launches (one pass)
    for c in ctxs:
        c.reset()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    single_ms = 0.0
    for c, w, n in zip(ctxs, ws, counts):
        c.run(int(n), dN, seed, 1 << 32, None)
        single_ms += c.last_kernel_ms()
    torch.cuda.synchronize()
    wall_single = time.perf_counter() - t1
    steps_single = int(sum(c.histogram()["n_steps_total"] for c in ctxs))
    batch.destroy()
    for c in ctxs:
        c.destroy()
    avg_ms = float(np.mean(kernel_ms))
    achieved = ALG_FLOPS_FP32_NO_BIAS * (steps_total / args.steps) / (avg_ms * 1e-3) / 1e12
    return {
        "metric": METRIC, "value": steps_total / wall, "unit": "trajectory-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched_64_fp32", "instances": len(ws),
                   "trajectories_per_step": int(counts.sum()),
                   "counts": "log-uniform in [1e4, 1e6]" if scale == 0.1 else f"batched_instances x {scale}",
                   "step_cap": int(ws[0].max_steps), "dN": dN, "graph": True,
                   "tuned_block": block, "tuned_chunk": chunk, "tune_s": tune_s},
        "trajectory_steps": steps_total, "censored": censored,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["fp32"], "traffic": None, "kernel": "batch_kernel",
                     "kernel_ms": avg_ms, "flops_per_step": ALG_FLOPS_FP32_NO_BIAS},
        "single_launches": {"trajectory_steps_per_s": steps_single / wall_single, "kernel_ms_sum": single_ms,
                            "batch_speedup": (steps_total / wall) / (steps_single / wall_single)},
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="srusr_is_fp32")
    ap.add_argument("--n-traj", type=float, default=None,
                    help="trajectories per step (batched: scale factor of the instance counts, default 0.1)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-side", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run one device-to-device copy of BYTES (a known-size kernel that scales the "
                         "profiler's FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(trajectories would shard by index, with one all-reduce of the histograms at the end).",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2410_13683_amd import runner

    torch.cuda.set_device(0)
    if args.workload == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return 0
    if args.workload == "srusr_is_fp32_multiA":
        print(json.dumps(bench_multi_amplitude(args)), flush=True)
        return 0
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = _workload(args.workload, args.n_traj)
    prec = "fp32" if w.precision == 1 else "fp64"
    stream = torch.cuda.current_stream()
    learned = None
    table_s = None
    if w.bias_kind == 2:
        learned = train_learned(w, stream)
        ctx = learned.pop("ctx")
    else:
        t_tab = time.perf_counter()
        ctx = runner.context_for(w)
        table_s = time.perf_counter() - t_tab
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
    if learned:
        learned["exact_network"] = exact_network_passes(w, ctx.mlp_get(), learned["deltaN_star"], stream)
    ctx.destroy()

    steps_total = int(hist["n_steps_total"])
    value = steps_total / wall
    x_star, p_star, ess_T, n_T = runner.tail_ess(hist, w.n_bins, w.bins_kind, w.lo, w.hi, 1e-10)
    if learned:
        # the same tail as the constant fallback passes
        x_star = learned["deltaN_star"]
        p_star, ess_T, n_T = tail_at(hist, w, x_star)
    ess_rate = ess_T / wall
    avg_ms = float(np.mean(kernel_ms))
    steps_per_launch = steps_total / args.steps
    flops_step = ALG_FLOPS_PER_STEP[prec] + (ALG_FLOPS_LEARNED_EXTRA[prec] if learned else 0.0)
    if prec == "fp64" and not learned and w.bias_kind == 0:     # no bias
        flops_step = ALG_FLOPS_FP64_NO_BIAS
    if w.noise in ("bessel2d", "bessel2d_time"):
        flops_step = ALG_FLOPS_2D["const" if w.bias_kind else "none"]
    if w.kind == 2:
        flops_step = ALG_FLOPS_BUMP_FP64
    if w.noise == "matched_time" and prec == "fp32":
        flops_step = ALG_FLOPS_TIME_FP32
    achieved = flops_step * steps_per_launch / (avg_ms * 1e-3) / 1e12
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
            "potential": ("Gaussian bump, K=1.17e-3, m=0.5, Sigma=1.59e-2, phi0=2.18812, CMB-normalised V0"
                          if w.kind == 2 else
                          "piecewise-linear slow roll -> ultra-slow roll, V0=1e-10, eps+=0.01, eps-=1e-8"),
            "noise": (f"2D noise, full Bunch-Davies mode at -k eta = {w.sigma}, {w.table_n} phi nodes"
                      if w.noise == "bessel2d" else
                      f"2D noise, full Bunch-Davies mode at -k eta = {w.sigma}, {w.table_n} time nodes over tau in "
                      f"[0, {w.table_hi:.6g}] after the reference trajectory passes phi_in, zero after it"
                      if w.noise == "bessel2d_time" else
                      f"Bessel-matched table (B_k from the mode equation), {w.table_n} phi nodes, sigma={w.sigma}"
                      if w.noise == "matched" else
                      f"Bessel-matched table on {w.table_n} time nodes over tau in [0, {w.table_hi:.6g}] after the "
                      f"reference trajectory passes phi_in, zero after it, sigma={w.sigma}"
                      if w.noise == "matched_time" else
                      f"Bessel-ansatz table, {w.table_n} phi nodes, sigma={w.sigma}"),
            "state": "FP32 pairs + FP64 log-weights" if prec == "fp32" else "FP64",
            "bias": "learned 2-64-64-2 tanh network, tabulated" if learned else f"constant A={w.A_bias:g}",
            "trajectories_per_step": w.n_traj,
            "dN": w.dN,
            "bins": f"{w.n_bins} {'log' if w.bins_kind else 'linear'} over deltaN in [{w.lo:.4g}, {w.hi:.4g})",
        },
        "ess_tail_per_s": ess_rate,
        "tail": {"deltaN_star": x_star, "P_tail": p_star, "ESS_T": ess_T, "samples_in_T": n_T,
                 "t_5pct_s": (400.0 / ess_rate) if ess_rate > 0 else None,
                 **(tail_errors(hist, w, x_star) if x_star is not None else {})},
        "trajectory_steps": steps_total,
        "table_setup_s": table_s,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_TFLOPS[prec],
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_TFLOPS[prec],
            "traffic": None,
            "kernel": (f"em2d_kernel<{prec.upper()}, 2D noise>" if w.noise in ("bessel2d", "bessel2d_time") else
                       "em_kernel<FP64, Gaussian bump>" if w.kind == 2 else
                       "em_kernel<FP32 state, learned control, table>" if prec == "fp32" and learned else
                       "em_kernel<FP32 state, const bias, table>" if prec == "fp32" else "em_kernel<FP64>"),
            "kernel_ms": avg_ms,
            "flops_per_step": flops_step,
            "int_ops_per_step": ALG_INT_OPS_PER_STEP,
        },
    }
    result["roofline"]["valu"] = measured_valu(w.name)
    hw = hw_counted_rate(result["roofline"]["valu"], steps_per_launch / (avg_ms * 1e-3))
    if hw:
        result["roofline"]["achieved_hw_counted"] = hw
        result["roofline"]["frac_hw_counted"] = hw / PEAK_TFLOPS[prec]
    if prec == "fp32":
        # the target is half the published FP32 vector peak; the gap to it, stated as is (the
        # published peak counts packed FP32, which these kernels are built without)
        result["roofline"]["frac_target"] = 0.5
        result["roofline"]["frac_gap_to_target"] = 0.5 - achieved / PEAK_TFLOPS[prec]
    if not learned:
        traffic, detail = measured_traffic(w)
        result["roofline"]["traffic"] = traffic
        if detail:
            result["roofline"]["traffic_detail"] = detail
            result["roofline"]["traffic_GBs"] = traffic / (avg_ms * 1e-3) / 1e9
    if learned:
        best = max(learned["constant_fallback"], key=lambda r: r["ess_tail_per_s"])
        learned["ess_tail_per_s_vs_best_constant"] = ess_rate / best["ess_tail_per_s"] if best["ess_tail_per_s"] else None
        # per equal trajectory count: the fallback passes ran one batch each, the timed run `steps` batches
        learned["ESS_T_per_batch_vs_best_constant"] = (ess_T / args.steps) / best["ESS_T"] if best["ESS_T"] else None
        result["learned"] = learned
    if not args.no_fp64_side and prec == "fp32" and not learned:
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
                                "tflops": ALG_FLOPS_FP64_NO_BIAS * s64 / (ms64 * 1e-3) / 1e12,
                                "valu": measured_valu(w64.name)}
        hw64 = hw_counted_rate(result["fp64_srusr"]["valu"], s64 / (ms64 * 1e-3))
        if hw64:
            result["fp64_srusr"]["tflops_hw_counted"] = hw64
        print(f"[bench] fp64 side run: {s64 / wall64:.3e} steps/s", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
