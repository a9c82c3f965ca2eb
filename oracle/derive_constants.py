"""Derive the stored workload constants with the CPU oracle only (test infrastructure).

Prints DELTA_E (phi_e - phi_end with a noise-free Euler-Maruyama passage time of
exactly 10 e-folds from phi_e at dN = 1e-4) and the noise-free reference
passage times N_REF_SRUSR and N_REF_LINEAR stored in the workloads module.

    python -m oracle.derive_constants
    python -m oracle.derive_constants --bump     (the Gaussian-bump workload's constants)
    python -m oracle.derive_constants --time     (the time-indexed SR -> USR workload's start)
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


if __name__ == "__main__" and "--bump" not in sys.argv and "--time" not in sys.argv:
    print(f"NOISE_S_HUBBLE = {hubble_noise()!r}")
    d = derive_delta_e()
    print(f"DELTA_E = {d!r}")
    print(f"N_REF_SRUSR = {noise_free_N(-d)!r}")
    print(f"N_REF_LINEAR = {linear_N_ref()!r}")


# ---------------------------------------------------------------------------
# Gaussian bump, eq. (potential_swagat)
# ---------------------------------------------------------------------------
BUMP = (0.5, 1.17e-3, 1.59e-2)     # m, K, Sigma
BUMP_PHI0 = 2.18812
BUMP_PHI_START = 3.2               # on the slow-roll attractor, ~42 e-folds before the transition


def _bump_background():
    """Classical trajectory of the bump from the slow-roll attractor at BUMP_PHI_START (scipy DOP853
    on eqs. klein_gordon + Friedmann in e-folds, with the oracle's V'/V) until eps1 = 1."""
    from scipy.integrate import solve_ivp

    def dlnV(p):
        V, dV, _ = orc.potential(orc.POT_GAUSSIAN_BUMP, 1.0, BUMP_PHI0, 0.0, 0.0, p, bump=BUMP)
        return dV / V

    def rhs(N, s):
        return [s[1], -(3.0 - 0.5 * s[1] ** 2) * (s[1] + dlnV(s[0]))]

    end = lambda N, s: 0.5 * s[1] ** 2 - 1.0
    end.terminal = True
    sol = solve_ivp(rhs, [0.0, 200.0], [BUMP_PHI_START, -dlnV(BUMP_PHI_START)], events=end, rtol=1e-12,
                    atol=1e-16, method="DOP853", dense_output=True)
    return sol, rhs, dlnV


def bump_constants():
    """N_T (first eps2 < -3), the USR interval, the noise window and the CMB-normalised V0."""
    from scipy.optimize import brentq
    sol, rhs, dlnV = _bump_background()
    N_end = float(sol.t_events[0][0])

    def eps2(N):
        p, q = sol.sol(N)
        return 2.0 * rhs(N, [p, q])[1] / q

    grid = np.arange(0.0, N_end, 0.01)
    e2 = np.array([eps2(N) for N in grid])
    i = int(np.argmax(e2 < -3.0))
    N_T = brentq(lambda N: eps2(N) + 3.0, grid[i - 1], grid[i], xtol=1e-13)
    k = i + int(np.argmax(e2[i:] > -3.0))
    N_usr_end = brentq(lambda N: eps2(N) + 3.0, grid[k - 1], grid[k], xtol=1e-13)
    # noise window (sigma = 1): from the middle of ultra-slow roll to N_T + 4.7, in the constant-eps2 phase
    N_lo, N_hi = 0.5 * (N_T + N_usr_end), N_T + 4.7
    phi_in, pi_in = (float(x) for x in sol.sol(N_lo))
    phi_lo = float(sol.sol(N_hi)[0])
    # CMB normalisation P_R = V/(24 pi^2 eps_V) = 2.1e-9 at N_end - 55
    p_star = float(sol.sol(N_end - 55.0)[0])
    u = orc.potential(orc.POT_GAUSSIAN_BUMP, 1.0, BUMP_PHI0, 0.0, 0.0, p_star, bump=BUMP)[0]
    eps_V = 0.5 * dlnV(p_star) ** 2
    V0 = 2.1e-9 * 24.0 * math.pi ** 2 * eps_V / u
    return dict(N_T=N_T, N_usr_end=N_usr_end, N_end=N_end, eps2_hi=eps2(N_hi), phi_in=phi_in, pi_in=pi_in,
                phi_lo=phi_lo, V0=V0, phi_star=p_star, tau_hi=N_hi - N_lo)


def bump_noise_free_N(c, phi_end: float, dN: float) -> float:
    p = orc.Problem(kind=orc.POT_GAUSSIAN_BUMP, V0=c["V0"], phi_T=BUMP_PHI0, A_plus=0.0, A_minus=0.0,
                    phi_in=c["phi_in"], pi_in=c["pi_in"], phi_end=phi_end, S=np.zeros(1), tan_theta=np.zeros(1),
                    bump=BUMP)
    N, _, steps = orc.run(p, dN, seed=0, n_traj=1)
    assert steps[0] & (orc.FLAG_CENSORED | orc.FLAG_ENDED_EARLY) == 0
    return float(N[0])


if __name__ == "__main__" and "--bump" in sys.argv:
    c = bump_constants()
    for k_, v_ in c.items():
        print(f"BUMP_{k_.upper()} = {v_!r}")
    print(f"BUMP_N_REF = {bump_noise_free_N(c, 2.0, 1e-3)!r}   # phi_end = 2.0, dN = 1e-3")


# ---------------------------------------------------------------------------
# Noise indexed by time on the SR -> USR problem (Sec. 4.1)
# ---------------------------------------------------------------------------
MATCH_PHI_START = 1.0      # the matched table's classical trajectory starts here, pi = -V'/V


def time_start():
    """(pi_ref, N_ref): the momentum with which the classical trajectory from (MATCH_PHI_START,
    -V'/V) reaches the transition phi = 0 (scipy DOP853 on eq. klein_gordon in e-folds, slope A_+
    above the transition), and the noise-free Euler-Maruyama passage from (0, pi_ref) to
    -DELTA_E at dN = 1e-4."""
    from scipy.integrate import solve_ivp

    def rhs(N, s):
        return [s[1], -(3.0 - 0.5 * s[1] ** 2) * (s[1] + A_PLUS / (V0 + A_PLUS * s[0]))]

    hit = lambda N, s: s[0]
    hit.terminal = True
    sol = solve_ivp(rhs, [0.0, 50.0], [MATCH_PHI_START, -A_PLUS / (V0 + A_PLUS * MATCH_PHI_START)], events=hit,
                    rtol=1e-13, atol=1e-16, method="DOP853")
    pi_ref = float(sol.y_events[0][0][1])
    d = derive_delta_e()
    p = orc.Problem(kind=orc.POT_PIECEWISE_LINEAR, V0=V0, phi_T=0.0, A_plus=A_PLUS, A_minus=A_MINUS,
                    phi_in=0.0, pi_in=pi_ref, phi_end=-d, S=np.zeros(1), tan_theta=np.zeros(1))
    N, _, steps = orc.run(p, 1e-4, seed=0, n_traj=1)
    assert steps[0] & (orc.FLAG_CENSORED | orc.FLAG_ENDED_EARLY) == 0
    return pi_ref, float(N[0]), float(sol.t_events[0][0])


if __name__ == "__main__" and "--time" in sys.argv:
    pi_ref, n_ref, n_to_kink = time_start()
    print(f"TIME_PI_IN = {pi_ref!r}   # {n_to_kink:.4f} e-folds from phi = {MATCH_PHI_START}")
    print(f"N_REF_TIME = {n_ref!r}")
