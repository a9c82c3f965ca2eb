"""GPU-side test glue: build a library context from a workload with the
library's own noise-table generator, run it through the C ABI and fetch the
per-trajectory dumps and the histogram."""
from __future__ import annotations

import numpy as np
import torch

from paper_2410_13683_amd import fpt
from paper_2410_13683_amd.workloads import Workload


def gpu_table(w: Workload, pot):
    if w.noise == "xi_const":
        return tuple(np.array([v]) for v in w.noise_Xi), None, 0.0, 0.0
    if w.noise == "bessel2d":
        X = fpt.fpt_noise_table_bessel2d(pot, w.sigma, w.table_n, w.table_lo, w.table_hi)
        return X, None, w.table_lo, w.table_hi
    if w.noise == "bessel2d_time":
        X = fpt.fpt_noise_table_bessel2d_time(pot, w.sigma, w.table_n, w.table_lo, w.table_hi, *w.match_start,
                                              w.phi_in)[:3]
        if w.noise_cut_end:
            for x in X:
                x[-1] = 0.0
        return X, None, w.table_lo, w.table_hi
    if w.noise == "const":
        return np.array([w.noise_S]), np.array([w.noise_tan]), 0.0, 0.0
    if w.noise == "matched":
        S, t, _ = fpt.fpt_noise_table_matched(pot, w.sigma, w.table_n, w.table_lo, w.table_hi, *w.match_start)
        if w.noise_cut_below:
            S[0] = 0.0
        return S, t, w.table_lo, w.table_hi
    if w.noise == "matched_time":
        S, t, _, _ = fpt.fpt_noise_table_matched_time(pot, w.sigma, w.table_n, w.table_lo, w.table_hi,
                                                      *w.match_start, w.phi_in)
        if w.noise_cut_end:
            S[-1] = 0.0
        return S, t, w.table_lo, w.table_hi
    S, t = fpt.fpt_noise_table_bessel(pot, w.sigma, w.table_n, w.table_lo, w.table_hi)
    return S, t, w.table_lo, w.table_hi


def gpu_context(w: Workload, **kw) -> fpt.Context:
    pot = fpt.make_potential(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.phi_in, w.pi_in, w.phi_end, w.bump)
    S, t, lo, hi = gpu_table(w, pot)
    args = dict(bias_kind=w.bias_kind, A=w.A_bias, precision=w.precision, bins_kind=w.bins_kind,
                n_bins=w.n_bins, lo=w.lo, hi=w.hi, N_ref=w.N_ref, max_steps=w.max_steps,
                instance=w.extra.get("instance", 0),
                axis=fpt.FPT_AXIS_TIME if w.noise in ("matched_time", "bessel2d_time") else fpt.FPT_AXIS_PHI)
    if w.bias_kind == 2:
        args.update(mlp_params=w.mlp_params, norm=w.mlp_norm, mlp_every=0, grid_n=w.grid_n,
                    grid_range=w.grid_range)
    if t is None:
        args["Xi"] = S
        S = None
    args.update(kw)
    return fpt.Context(pot, S, t, lo, hi, **args)


def gpu_run(w: Workload, n_traj=None, traj_offset=0, dumps=True, ctx=None, **kw):
    n = w.n_traj if n_traj is None else n_traj
    own = ctx is None
    if own:
        ctx = gpu_context(w, **kw)
    dev = torch.device("cuda")
    N = lnw = steps = None
    if dumps and n > 0:
        N = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
        lnw = torch.zeros(n, dtype=torch.float64, device=dev)
        steps = torch.zeros(n, dtype=torch.int32, device=dev)
    ctx.run(n, w.dN, w.seed, traj_offset, torch.cuda.current_stream(), N, lnw, steps)
    torch.cuda.synchronize()
    hist = ctx.histogram()
    out = None
    if dumps and n > 0:
        out = (N.cpu().numpy(), lnw.cpu().numpy(), steps.cpu().numpy().view(np.uint32))
    if own:
        ctx.destroy()
    return out, hist
