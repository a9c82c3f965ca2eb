"""Normalisation and error bars of the weighted first-passage histogram (Sec. 4.1) --
test infrastructure.

Plain numpy versions of what the library computes from its histogram
accumulators.  They share no code with the library.  Only tests/ and bench.py's
CPU baseline use this module.

* Normalisation: Sec. 4.1 reconstructs P(deltaN) from the weighted runs.  A bin's
  density is its sum of weights over n_traj (every trajectory run) times its width;
  a tail set T = {deltaN >= x*} has P = sum_T w / n_traj, standard error
  sqrt((sum_T w^2/n - P^2)/n) and ESS_T = (sum_T w)^2 / sum_T w^2.  The whole run has
  mean_w = sum w / n, the weighted mean and variance of N and ESS = (sum w)^2 / sum w^2.

* Direct sampling (no bias): delete-one jackknife over B blocks of trajectories.
  The paper treats each simulation run as an independent sample and resamples them.
* Importance sampling: the error of a per-bin lognormal mean.  Within slot j, ln w of
  the n_j trajectories there is treated as normal with mean mu and variance s^2.  The
  slot's mass is (n_j/n) exp(mu + s^2/2).  Its one-standard-deviation interval in
  ln(mass) combines two independent parts:
  - Cox's standard error of ln(mean w), s^2/n_j + s^4/(2(n_j - 1));
  - the binomial fluctuation of the count, (1 - n_j/n)/n_j.
  Without weights the interval is the binomial one.
* Several bias amplitudes: the inverse-variance weighted mean per slot.

Masses are per histogram slot (slot 0 underflow, 1..n_bins the bins, n_bins + 1
overflow), sum_w/n_traj.  Dividing by the bin width gives the density.
"""
from __future__ import annotations

import numpy as np


def jackknife(n_traj_blocks, sum_w_blocks):
    """(p, err) per slot from B blocks: p = sum_b sw_b / sum_b n_b; the delete-one estimates
    p_(b) = (sum sw - sw_b)/(N - n_b); err^2 = (B - 1)/B sum_b (p_(b) - mean_b p_(b))^2."""
    n = np.asarray(n_traj_blocks, dtype=np.float64)
    sw = np.asarray(sum_w_blocks, dtype=np.float64)        # (B, n_slots)
    B = len(n)
    N, SW = n.sum(), sw.sum(axis=0)
    p = SW / N
    loo = np.empty_like(sw)
    for b in range(B):
        loo[b] = (SW - sw[b]) / (N - n[b])
    mean = loo.mean(axis=0)
    err = np.sqrt((B - 1) / B * ((loo - mean) ** 2).sum(axis=0))
    return p, err


def lognormal(n_traj, count, sum_lnw, sum_lnw2):
    """(p, lo, hi) per slot: (n_j/n) exp(mu + s^2/2), and exp(-+se) times it with
    se^2 = s^2/n_j + s^4/(2(n_j - 1)) + (1 - n_j/n)/n_j; NaN where n_j < 2."""
    c = np.asarray(count, dtype=np.float64)
    p = np.full(len(c), np.nan)
    lo = np.full(len(c), np.nan)
    hi = np.full(len(c), np.nan)
    for j in range(len(c)):
        nj = c[j]
        if nj < 2:
            continue
        mu = sum_lnw[j] / nj
        s2 = max((sum_lnw2[j] - nj * mu * mu) / (nj - 1.0), 0.0)
        theta = mu + 0.5 * s2
        f = nj / n_traj
        se = np.sqrt(s2 / nj + s2 * s2 / (2.0 * (nj - 1.0)) + (1.0 - f) / nj)
        p[j], lo[j], hi[j] = f * np.exp(theta), f * np.exp(theta - se), f * np.exp(theta + se)
    return p, lo, hi


def merge(p_runs, err_runs):
    """Inverse-variance weighted mean per slot over runs; runs with a non-finite or non-positive
    error in a slot are left out there; NaN where none is left."""
    P = np.asarray(p_runs, dtype=np.float64)
    E = np.asarray(err_runs, dtype=np.float64)
    out_p = np.full(P.shape[1], np.nan)
    out_e = np.full(P.shape[1], np.nan)
    for j in range(P.shape[1]):
        ok = np.isfinite(P[:, j]) & np.isfinite(E[:, j]) & (E[:, j] > 0)
        if not ok.any():
            continue
        wgt = 1.0 / E[ok, j] ** 2
        out_p[j] = (wgt * P[ok, j]).sum() / wgt.sum()
        out_e[j] = 1.0 / np.sqrt(wgt.sum())
    return out_p, out_e


def _edges(bins_kind, n_bins, lo, hi):
    """e_j = lo + j (hi - lo)/n_bins (linear) or lo (hi/lo)^(j/n_bins) (log), j = 0..n_bins."""
    e = np.empty(n_bins + 1)
    for j in range(n_bins + 1):
        t = j / n_bins
        e[j] = lo + (hi - lo) * t if bins_kind == 0 else lo * (hi / lo) ** t
    e[n_bins] = hi
    return e


def density(hist, bins_kind, n_bins, lo, hi):
    """(density per bin, edges): sum_w of bin j over n_traj (e_{j+1} - e_j)."""
    e = _edges(bins_kind, n_bins, lo, hi)
    n = float(hist["n_traj"])
    d = np.empty(n_bins)
    for j in range(n_bins):
        d[j] = float(hist["sum_w"][j + 1]) / (n * (e[j + 1] - e[j]))
    return d, e


def moments(hist):
    """mean_w, mean_N, var_N, ess, mass_under, mass_over of a histogram dict."""
    n = float(hist["n_traj"])
    sw, sw2 = float(hist["sum_w_total"]), float(hist["sum_w2_total"])
    mean_N = float(hist["sum_wN"]) / sw
    return {"mean_w": sw / n, "mean_N": mean_N, "var_N": float(hist["sum_wN2"]) / sw - mean_N ** 2,
            "ess": sw * sw / sw2 if sw2 > 0 else 0.0,
            "mass_under": float(hist["sum_w"][0]) / n, "mass_over": float(hist["sum_w"][-1]) / n}


def tail_at(hist, bins_kind, n_bins, lo, hi, slot):
    """The tail set of slots slot .. n_bins + 1 (deltaN >= e_{slot-1}; the overflow slot starts at hi)."""
    e = _edges(bins_kind, n_bins, lo, hi)
    n = float(hist["n_traj"])
    sw = float(np.sum(np.asarray(hist["sum_w"], dtype=np.float64)[slot:]))
    sw2 = float(np.sum(np.asarray(hist["sum_w2"], dtype=np.float64)[slot:]))
    P = sw / n
    # the lognormal intervals of the slots of T, half-widths added in quadrature
    _, lo_j, hi_j = lognormal(n, hist["count"], hist["sum_lnw"], hist["sum_lnw2"])
    half = 0.5 * (hi_j - lo_j)[slot:]
    half = half[np.isfinite(half)]
    return {"slot": slot, "x_star": float(e[slot - 1]), "P": P,
            "P_err": float(np.sqrt(max(sw2 / n - P * P, 0.0) / n)),
            "P_err_lognormal": float(np.sqrt(np.sum(half ** 2))),
            "ess": sw * sw / sw2 if sw2 > 0 else 0.0,
            "count": int(np.sum(np.asarray(hist["count"], dtype=np.uint64)[slot:]))}


def tail_find(hist, bins_kind, n_bins, lo, hi, p_target):
    """The lowest slot j >= 1 whose tail mass sum_{slots >= j} w / n_traj is positive and at most
    p_target, as tail_at; slot -1 when there is none."""
    n = float(hist["n_traj"])
    for j in range(1, n_bins + 2):
        p = float(np.sum(np.asarray(hist["sum_w"], dtype=np.float64)[j:])) / n
        if 0.0 < p <= p_target:
            return tail_at(hist, bins_kind, n_bins, lo, hi, j)
    return {"slot": -1, "x_star": 0.0, "P": 0.0, "P_err": 0.0, "P_err_lognormal": 0.0, "ess": 0.0, "count": 0}

