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
                                      w.table_n, w.table_lo, w.table_hi)
        return S, t, w.table_lo, w.table_hi
    raise ValueError(w.noise)


def oracle_problem(w: Workload, mlp_params=None, mlp_norm=None) -> orc.Problem:
    S, t, lo, hi = oracle_table(w)
    return orc.Problem(kind=w.kind, V0=w.V0, phi_T=w.phi_T, A_plus=w.A_plus, A_minus=w.A_minus,
                       phi_in=w.phi_in, pi_in=w.pi_in, phi_end=w.phi_end, S=S, tan_theta=t,
                       phi_lo=lo, phi_hi=hi, bias_kind=w.bias_kind, A_bias=w.A_bias,
                       mlp_params=mlp_params, mlp_norm=mlp_norm)


def oracle_run(w: Workload, n_traj=None, traj_offset=0, n_threads=0, **kw):
    p = oracle_problem(w, **kw)
    return orc.run(p, w.dN, w.seed, w.n_traj if n_traj is None else n_traj, traj_offset=traj_offset,
                   instance=w.extra.get("instance", 0), max_steps=w.max_steps, n_threads=n_threads)
