"""Test-side glue: the oracle's runs of a workload description and the per-trajectory FP64
parity check.

The oracle builds its own noise table with its own generator (oracle/problems.py); the GPU side
builds its table with the library's generator (see tests/_gpu.py).  Nothing here computes any
step of the method.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc
from oracle.problems import NOISE_2D, oracle_problem, oracle_problem2d, oracle_table  # noqa: F401
from paper_2410_13683_amd.workloads import Workload


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


def oracle_run(w: Workload, n_traj=None, traj_offset=0, n_threads=0, last_phi=False, **kw):
    """The oracle's (N, ln w, steps) for the workload's trajectories, plus phi before and after
    each last step with last_phi (the form assert_fp64_parity takes)."""
    if w.noise in NOISE_2D:
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
    two_d = w.noise in NOISE_2D
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
