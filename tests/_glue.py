"""Test-side glue: turn a workload description into an oracle problem.

The oracle builds its own noise table with its own generator; the GPU side
builds its table with the library's generator (see tests/_gpu.py).  Nothing
here computes any step of the method.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc
from paper_2410_13683_amd.workloads import Workload


def oracle_table(w: Workload):
    if w.noise == "const":
        return np.array([w.noise_S]), np.array([w.noise_tan]), 0.0, 0.0
    if w.noise == "bessel":
        S, t = orc.noise_table_bessel(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.sigma,
                                      w.table_n, w.table_lo, w.table_hi, bump=w.bump)
        return S, t, w.table_lo, w.table_hi
    if w.noise == "matched":
        S, t, _ = orc.noise_table_matched(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.sigma, w.table_n,
                                          w.table_lo, w.table_hi, *w.match_start, bump=w.bump)
        if w.noise_cut_below:
            S[0] = 0.0
        return S, t, w.table_lo, w.table_hi
    if w.noise == "matched_time":
        S, t, _, _ = orc.noise_table_matched_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.sigma, w.table_n,
                                                  w.table_lo, w.table_hi, *w.match_start, w.phi_in, bump=w.bump)
        if w.noise_cut_end:
            S[-1] = 0.0
        return S, t, w.table_lo, w.table_hi
    raise ValueError(w.noise)


def oracle_problem(w: Workload, mlp_params=None, mlp_norm=None) -> orc.Problem:
    """The oracle problem of a workload.  A learned control given by the workload
    (w.mlp_params) is the tabulated network on the workload's grid; parameters passed
    here instead select the network evaluated at every step."""
    S, t, lo, hi = oracle_table(w)
    p = orc.Problem(kind=w.kind, V0=w.V0, phi_T=w.phi_T, A_plus=w.A_plus, A_minus=w.A_minus,
                    phi_in=w.phi_in, pi_in=w.pi_in, phi_end=w.phi_end, S=S, tan_theta=t,
                    phi_lo=lo, phi_hi=hi, bias_kind=w.bias_kind, A_bias=w.A_bias,
                    mlp_params=mlp_params, mlp_norm=mlp_norm, bump=w.bump,
                    tab_axis=1 if w.noise == "matched_time" else 0)
    if mlp_params is None and w.mlp_params is not None:
        p.mlp_params = np.ascontiguousarray(w.mlp_params, dtype=np.float32)
        p.mlp_norm = np.asarray(w.mlp_norm, dtype=np.float64)
        p.mlp_every = 0
        p.grid_n = tuple(w.grid_n)
        p.grid_range = tuple(w.grid_range)
    return p


def assert_fp64_parity(gpu, ora, max_step_mismatch=0.002):
    """Per-trajectory FP64 parity: same flags, N within 1e-9 relative, the same crossing step
    except at floating-point near-ties with phi_end (at most max_step_mismatch of them, and
    then off by one step), ln w within 1e-9 relative to 1 + |ln w| where the steps agree.
    The interpolated N = (n - 1 + f) dN, f = (phi_(n-1) - phi_end)/(phi_(n-1) - phi_n), turns a
    rounding difference in phi into dN/|phi_(n-1) - phi_n| times it: a rare short last step (the
    drift and the noise nearly cancel) is a near-tie of the same kind, and up to max_step_mismatch
    of the trajectories (at least one) may then differ up to 1e-7 relative."""
    Ng, lg, sg = gpu
    No, lo_, so = ora
    assert Ng.shape == No.shape
    flags = orc.FLAG_CENSORED | orc.FLAG_ENDED_EARLY
    assert np.array_equal(sg & flags, so & flags)
    fin = (so & flags) == 0
    same = sg == so
    assert (1.0 - same.mean()) <= max_step_mismatch, f"{(~same).sum()} crossing steps differ"
    diff_steps = np.abs((sg & orc.STEP_MASK).astype(np.int64) - (so & orc.STEP_MASK).astype(np.int64))
    assert diff_steps.max(initial=0) <= 1
    rel = np.abs(Ng[fin] - No[fin]) / np.abs(No[fin])
    loose = rel > 1e-9
    worst = int(np.flatnonzero(fin)[np.argmax(rel)]) if rel.size else -1
    assert loose.sum() <= max(1, int(max_step_mismatch * len(rel))), (loose.sum(), rel.max(), worst)
    assert rel.max(initial=0.0) <= 1e-7, (rel.max(), worst)
    ok = same & fin
    assert np.all(np.abs(lg[ok] - lo_[ok]) <= 1e-9 * (1.0 + np.abs(lo_[ok])))


def oracle_problem2d(w: Workload) -> orc.Problem2D:
    if w.noise == "xi_const":
        X, lo, hi = tuple(np.array([v]) for v in w.noise_Xi), 0.0, 0.0
    elif w.noise == "bessel2d_time":
        X = orc.noise_table_bessel2d_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.sigma, w.table_n,
                                          w.table_lo, w.table_hi, *w.match_start, w.phi_in)[:3]
        if w.noise_cut_end:
            for x in X:
                x[-1] = 0.0
        lo, hi = w.table_lo, w.table_hi
    else:
        X = orc.noise_table_bessel2d(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.sigma, w.table_n,
                                     w.table_lo, w.table_hi)
        lo, hi = w.table_lo, w.table_hi
    return orc.Problem2D(kind=w.kind, V0=w.V0, phi_T=w.phi_T, A_plus=w.A_plus, A_minus=w.A_minus,
                         phi_in=w.phi_in, pi_in=w.pi_in, phi_end=w.phi_end, Xpp=X[0], Xpq=X[1], Xqq=X[2],
                         phi_lo=lo, phi_hi=hi, bias_kind=w.bias_kind, A_bias=w.A_bias,
                         tab_axis=1 if w.noise == "bessel2d_time" else 0)


def oracle_run(w: Workload, n_traj=None, traj_offset=0, n_threads=0, **kw):
    if w.noise in ("xi_const", "bessel2d", "bessel2d_time"):
        return orc.run2d(oracle_problem2d(w), w.dN, w.seed, w.n_traj if n_traj is None else n_traj,
                         traj_offset=traj_offset, instance=w.extra.get("instance", 0), max_steps=w.max_steps,
                         n_threads=n_threads)
    p = oracle_problem(w, **kw)
    return orc.run(p, w.dN, w.seed, w.n_traj if n_traj is None else n_traj, traj_offset=traj_offset,
                   instance=w.extra.get("instance", 0), max_steps=w.max_steps, n_threads=n_threads)
