"""Derive the stored workload constants with the CPU oracle only (test infrastructure).

Prints DELTA_E (phi_e - phi_end with a noise-free Euler-Maruyama passage time of
exactly 10 e-folds from phi_e at dN = 1e-4) and the noise-free reference
passage times N_REF_SRUSR and N_REF_LINEAR stored in the workloads module.

    python -m oracle.derive_constants
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import oracle as orc  # noqa: E402

V0 = 1e-10
A_PLUS = V0 * math.sqrt(2.0 * 0.01)
A_MINUS = V0 * math.sqrt(2.0 * 1e-8)


def noise_free_N(phi_end: float, dN: float = 1e-4) -> float:
    p = orc.Problem(kind=orc.POT_PIECEWISE_LINEAR, V0=V0, phi_T=0.0, A_plus=A_PLUS, A_minus=A_MINUS,
                    phi_in=0.0, pi_in=-math.sqrt(0.02), phi_end=phi_end,
                    S=np.zeros(1), tan_theta=np.zeros(1))
    N, _, steps = orc.run(p, dN, seed=0, n_traj=1)
    assert steps[0] & (orc.FLAG_CENSORED | orc.FLAG_ENDED_EARLY) == 0
    return float(N[0])


def derive_delta_e(target: float = 10.0) -> float:
    lo, hi = 0.0475, 0.06          # N(lo) < target < N(hi)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if noise_free_N(-mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def linear_N_ref() -> float:
    alpha = math.sqrt(0.02)
    p = orc.Problem(kind=orc.POT_PIECEWISE_LINEAR, V0=V0, phi_T=0.0, A_plus=V0 * alpha, A_minus=V0 * alpha,
                    phi_in=1.0, pi_in=-alpha / (1.0 + alpha), phi_end=0.0,
                    S=np.zeros(1), tan_theta=np.zeros(1))
    N, _, _ = orc.run(p, 1e-3, seed=0, n_traj=1)
    return float(N[0])


def hubble_noise() -> float:
    """S = H/(2 pi) with H^2 = V0/3: the oracle's table at a node where nu = 3/2 exactly
    (exponential potential, V''/V = (V'/V)^2) and V = V0."""
    S, t = orc.noise_table_bessel(orc.POT_EXPONENTIAL, V0, 0.0, 0.3, 0.0, 1.0, 1, 0.0, 0.0)
    assert t[0] == 0.0
    return float(S[0])


if __name__ == "__main__":
    print(f"NOISE_S_HUBBLE = {hubble_noise()!r}")
    d = derive_delta_e()
    print(f"DELTA_E = {d!r}")
    print(f"N_REF_SRUSR = {noise_free_N(-d)!r}")
    print(f"N_REF_LINEAR = {linear_N_ref()!r}")
