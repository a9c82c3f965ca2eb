"""Test infrastructure, not part of the product.

The oracle's problem for a workload description: any object with the workload fields (kind, V0,
phi_T, A_plus, A_minus, phi_in, pi_in, phi_end, the noise kind and its table parameters, the bias,
the learned control's parameters, bump).  The oracle builds its noise tables with its own
generators (Sec. 3.2 and 3.4 for the Bessel tables, Sec. 3.3 for the matched ones, Sec. 4.1 for
tables in time).  This module reads the description's attributes only: it imports nothing from
the GPU package.  Only tests/ and the CPU-baseline leg of bench.py use it.
"""
from __future__ import annotations

import numpy as np

from . import oracle as orc

NOISE_2D = ("xi_const", "bessel2d", "bessel2d_time")


def oracle_table(w):
    """(S, tan_theta, phi_lo, phi_hi) of the description's 1D noise, from the oracle's generators."""
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


def oracle_problem(w, mlp_params=None, mlp_norm=None) -> orc.Problem:
    """The oracle problem of a 1D description.  A learned control given by the description
    (w.mlp_params) is the tabulated network on its grid; parameters passed here instead select
    the network evaluated at every step."""
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


def oracle_problem2d(w) -> orc.Problem2D:
    """The oracle problem of a 2D description (constant covariance or the 2D Bessel tables)."""
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
