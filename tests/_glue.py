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


def phi_drift(w: Workload) -> float:
    """Bound on how far the HIP path's phi and the oracle's phi may drift apart along a path.  Both
    take the same steps in FP64 but round in a different order (fused multiply-adds, the reciprocal
    of V/V', table-driven log and sincos): a few ulp of the largest |phi| per step.  Over 1e5 steps
    that is some 300 ulp as a random walk and 1e5 ulp if every rounding went the same way; the bound
    is 1e4 ulp (1.1e-13 for |phi| <= 0.0486, the SR -> USR workloads)."""
    return 1e4 * 2.0 ** -52 * max(abs(w.phi_in), abs(w.phi_end))


def assert_fp64_parity(gpu, ora, w):
    """Per-trajectory FP64 parity with the oracle (ora from oracle_run(..., last_phi=True), which
    adds phi before and after each trajectory's last step): the same flags; N within 1e-9
    relative; the same crossing step; ln w within 1e-9 relative to 1 + |ln w| where the steps
    agree.  Two exemptions, each tied to its mechanism and checked per trajectory:
      * a crossing step one apart only at a near-tie with phi_end, where the oracle's phi before
        or after its last step lies within phi_drift(w) of phi_end (N is continuous there);
      * N may miss 1e-9 only by what a phi difference of phi_drift(w) becomes through the
        interpolation N = (n - 1 + f) dN, f = (phi_(n-1) - phi_end)/(phi_(n-1) - phi_n): by
        dN phi_drift / |phi_(n-1) - phi_n| (a short last step, where drift and noise nearly
        cancel)."""
    drift = phi_drift(w)
    Ng, lg, sg = gpu
    No, lo_, so, phi2 = ora
    assert Ng.shape == No.shape == lg.shape == sg.shape and phi2.shape == (len(No), 2)
    flags = orc.FLAG_CENSORED | orc.FLAG_ENDED_EARLY
    assert np.array_equal(sg & flags, so & flags), "flags differ"
    fin = (so & flags) == 0
    ng = (sg & orc.STEP_MASK).astype(np.int64)
    no = (so & orc.STEP_MASK).astype(np.int64)
    tie = np.min(np.abs(phi2 - w.phi_end), axis=1) < drift
    bad_step = (ng != no) & ~(fin & tie & (np.abs(ng - no) == 1))
    assert not bad_step.any(), ("crossing steps differ", np.flatnonzero(bad_step)[:10], ng[bad_step][:10],
                                no[bad_step][:10], phi2[bad_step][:10] - w.phi_end)
    rel = np.zeros(len(No))
    rel[fin] = np.abs(Ng[fin] - No[fin]) / np.abs(No[fin])
    last = np.abs(phi2[:, 0] - phi2[:, 1])
    with np.errstate(divide="ignore"):
        allowed = np.maximum(1e-9, np.where(fin, w.dN * drift / (last * np.abs(No)), 0.0))
    over = fin & (rel > allowed)
    assert not over.any(), ("N differs", np.flatnonzero(over)[:10], rel[over][:10], last[over][:10])
    # ended early: N = n dN on both sides
    early = (so & orc.FLAG_ENDED_EARLY) != 0
    assert np.array_equal(Ng[early], No[early])
    ok = (ng == no) & ((so & orc.FLAG_CENSORED) == 0)
    assert np.all(np.abs(lg[ok] - lo_[ok]) <= 1e-9 * (1.0 + np.abs(lo_[ok]))), "ln w differs"
    return {"step_ties": int((ng != no).sum()), "short_last_step": int((fin & (rel > 1e-9)).sum())}


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


def oracle_run(w: Workload, n_traj=None, traj_offset=0, n_threads=0, last_phi=False, **kw):
    """The oracle's (N, ln w, steps) for the workload's trajectories, plus phi before and after
    each last step with last_phi (the form assert_fp64_parity takes)."""
    if w.noise in ("xi_const", "bessel2d", "bessel2d_time"):
        return orc.run2d(oracle_problem2d(w), w.dN, w.seed, w.n_traj if n_traj is None else n_traj,
                         traj_offset=traj_offset, instance=w.extra.get("instance", 0), max_steps=w.max_steps,
                         n_threads=n_threads, last_phi=last_phi)
    p = oracle_problem(w, **kw)
    return orc.run(p, w.dN, w.seed, w.n_traj if n_traj is None else n_traj, traj_offset=traj_offset,
                   instance=w.extra.get("instance", 0), max_steps=w.max_steps, n_threads=n_threads,
                   last_phi=last_phi)


def oracle_sampled(w: Workload, idx, prob=None):
    """oracle_run(..., last_phi=True) of the trajectories at the given (sorted) indices, one oracle
    call per run of consecutive indices; prob: the oracle problem (1D or 2D) if already built."""
    idx = np.asarray(idx, dtype=np.int64)
    two_d = w.noise in ("xi_const", "bessel2d", "bessel2d_time")
    if prob is None:
        prob = oracle_problem2d(w) if two_d else oracle_problem(w)
    run = orc.run2d if two_d else orc.run
    parts = []
    start = 0
    for k in range(1, len(idx) + 1):
        if k == len(idx) or idx[k] != idx[k - 1] + 1:
            parts.append(run(prob, w.dN, w.seed, k - start, traj_offset=int(idx[start]),
                             instance=w.extra.get("instance", 0), max_steps=w.max_steps, last_phi=True))
            start = k
    return tuple(np.concatenate([p[i] for p in parts]) for i in range(4))
