"""Build a library context for a workload description and run it.

Argument marshalling only: the noise table comes from the library's own device
kernels (fpt_noise_table_bessel, _bessel2d, _matched) and every trajectory step
runs in libfpt.so.
"""
from __future__ import annotations

import numpy as np

from . import fpt
from .workloads import Workload


def potential_of(w: Workload) -> fpt.fpt_potential:
    return fpt.make_potential(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.phi_in, w.pi_in, w.phi_end, w.bump)


def table_of(w: Workload, pot=None):
    """(S, tan_theta, phi_lo, phi_hi) of the workload's noise; for 2D noise S is the tuple
    (Xi_pp, Xi_pq, Xi_qq) and tan_theta is None."""
    if w.noise == "xi_const":
        return tuple(np.array([v]) for v in w.noise_Xi), None, 0.0, 0.0
    if w.noise == "bessel2d":
        X = fpt.fpt_noise_table_bessel2d(pot or potential_of(w), w.sigma, w.table_n, w.table_lo, w.table_hi)
        return X, None, w.table_lo, w.table_hi
    if w.noise == "bessel2d_time":
        X = fpt.fpt_noise_table_bessel2d_time(pot or potential_of(w), w.sigma, w.table_n, w.table_lo, w.table_hi,
                                              *w.match_start, w.phi_in)[:3]
        if w.noise_cut_end:
            for x in X:
                x[-1] = 0.0
        return X, None, w.table_lo, w.table_hi
    if w.noise == "const":
        return np.array([w.noise_S]), np.array([w.noise_tan]), 0.0, 0.0
    if w.noise == "bessel":
        S, t = fpt.fpt_noise_table_bessel(pot or potential_of(w), w.sigma, w.table_n, w.table_lo, w.table_hi)
        return S, t, w.table_lo, w.table_hi
    if w.noise == "matched":
        S, t, _ = fpt.fpt_noise_table_matched(pot or potential_of(w), w.sigma, w.table_n, w.table_lo, w.table_hi,
                                              *w.match_start)
        if w.noise_cut_below:
            S[0] = 0.0
        return S, t, w.table_lo, w.table_hi
    if w.noise == "matched_time":
        S, t, _, _ = fpt.fpt_noise_table_matched_time(pot or potential_of(w), w.sigma, w.table_n, w.table_lo,
                                                      w.table_hi, *w.match_start, w.phi_in)
        if w.noise_cut_end:
            S[-1] = 0.0
        return S, t, w.table_lo, w.table_hi
    raise ValueError(f"unknown noise kind {w.noise!r}")


def context_for(w: Workload, **overrides) -> fpt.Context:
    pot = potential_of(w)
    S, t, lo, hi = table_of(w, pot)
    kw = dict(bias_kind=w.bias_kind, A=w.A_bias, precision=w.precision, bins_kind=w.bins_kind, n_bins=w.n_bins,
              lo=w.lo, hi=w.hi, N_ref=w.N_ref, max_steps=w.max_steps, instance=w.extra.get("instance", 0),
              axis=fpt.FPT_AXIS_TIME if w.noise in ("matched_time", "bessel2d_time") else fpt.FPT_AXIS_PHI)
    if w.bias_kind == 2:
        kw.update(mlp_params=w.mlp_params, norm=w.mlp_norm, mlp_every=0, grid_n=w.grid_n, grid_range=w.grid_range)
    if t is None:
        kw["Xi"] = S
        S = None
    kw.update(overrides)
    return fpt.Context(pot, S, t, lo, hi, **kw)


def tail_set(hist: dict, n_bins: int, bins_kind: int, lo: float, hi: float, p_tail: float = 1e-10) -> dict:
    """The library's tail set at probability p_tail (fpt_tail_find): the bins from the lowest edge
    x* whose weighted tail mass P(deltaN >= x*) (overflow included) is at most p_tail, with P, its
    errors, ESS_T and the samples in T (slot -1 when no edge qualifies)."""
    return fpt.fpt_tail_find(hist, bins_kind, n_bins, lo, hi, p_tail)


def tail_ess(hist: dict, n_bins: int, bins_kind: int, lo: float, hi: float, p_tail: float = 1e-10):
    """(x*, P(deltaN >= x*), ESS_T, samples in T) of tail_set, or (None, 0, 0, 0)."""
    t = tail_set(hist, n_bins, bins_kind, lo, hi, p_tail)
    if t["slot"] < 0:
        return None, 0.0, 0.0, 0
    return t["x_star"], t["P"], t["ess"], int(t["count"])


def run_blocks(ctx: fpt.Context, w: Workload, n_blocks: int, stream, traj_offset: int = 0):
    """Run w.n_traj trajectories as n_blocks consecutive blocks (trajectories traj_offset + b*m ..),
    reading and clearing the context's histogram after each.  Returns the per-block n_traj and
    sum_w arrays (inputs of fpt_jackknife) and the histogram of all blocks together."""
    m = w.n_traj // n_blocks
    ctx.reset()
    n_b, sw_b, total = [], [], None
    for b in range(n_blocks):
        ctx.run(m, w.dN, w.seed, traj_offset + b * m, stream)
        h = ctx.histogram()
        ctx.reset()
        n_b.append(int(h["n_traj"]))
        sw_b.append(np.asarray(h["sum_w"], dtype=np.float64))
        if total is None:
            total = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in h.items()}
        else:
            for k, v in h.items():
                total[k] = total[k] + v
    return np.asarray(n_b, dtype=np.uint64), np.stack(sw_b), total
