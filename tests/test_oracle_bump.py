"""Pins of the oracle's Gaussian-bump potential (eq. potential_swagat) and of the
workload built on it.
- The shape: the bump multiplies the base potential by 1 + K e^(-x^2/2), centred at phi_0
  with width Sigma.  The base potential tends to V0 far out and is V0/2 at phi = m.
- V' and V'' against finite differences of the oracle's own V.
- The background: the paper prints eps2 = 0.732 at N_T + 4.7 and eps2 = 1.02 at N_T + 9.3
  (N_T the first time eps2 < -3), in the constant-eps2 phase after ultra-slow roll.  A scipy
  solve of the Klein-Gordon equation with the oracle's V'/V reproduces both.
- The Euler-Maruyama drift: the noise-free passage against a cosmic-time Klein-Gordon solve,
  Richardson-extrapolated.
- The matched table on the bump: the separate-universe criterion within 1 % in the window
  the workload uses, and B_k continuous where nu crosses 2 (the Wronskian form needs no Y_nu).
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

from paper_2410_13683_amd import workloads as W
from tests.golden.printed import printed
from tests.test_oracle_dynamics import _kg_passage

GOLD = printed()

KIND = 2
M, K, SIG = W.BUMP
PHI0 = W.BUMP_PHI0


def _pot(orc, phi, V0=1.0, bump=W.BUMP):
    return orc.potential(KIND, V0, PHI0, 0.0, 0.0, phi, bump=bump)


def test_bump_shape(orc):
    for phi in (PHI0 - 3 * SIG, PHI0 - SIG, PHI0, PHI0 + 0.5 * SIG, PHI0 + 2 * SIG):
        x = (phi - PHI0) / SIG
        ratio = _pot(orc, phi)[0] / _pot(orc, phi, bump=(M, 0.0, SIG))[0]
        assert math.isclose(ratio - 1.0, K * math.exp(-0.5 * x * x), rel_tol=1e-9)
    assert math.isclose(_pot(orc, M, bump=(M, 0.0, SIG))[0], 0.5, rel_tol=1e-15)
    assert math.isclose(_pot(orc, 1e4, bump=(M, 0.0, SIG))[0], 1.0, rel_tol=1e-8)
    assert _pot(orc, PHI0, V0=3.0)[0] == pytest.approx(3.0 * _pot(orc, PHI0)[0], rel=1e-15)


@pytest.mark.parametrize("phi", [0.6, 1.3, PHI0 - 2.1 * SIG, PHI0 - 0.3 * SIG, PHI0 + 0.9 * SIG, PHI0 + 2.7 * SIG, 3.1])
def test_bump_derivatives_match_finite_differences(orc, phi):
    h = 1e-4 * SIG
    V = lambda p: _pot(orc, p)[0]
    dV = lambda p: _pot(orc, p)[1]
    fd1 = (-V(phi + 2 * h) + 8 * V(phi + h) - 8 * V(phi - h) + V(phi - 2 * h)) / (12 * h)
    fd2 = (-dV(phi + 2 * h) + 8 * dV(phi + h) - 8 * dV(phi - h) + dV(phi - 2 * h)) / (12 * h)
    _, d1, d2 = _pot(orc, phi)
    assert abs(d1 - fd1) < 1e-7 * (abs(d1) + 1e-3)
    assert abs(d2 - fd2) < 1e-6 * (abs(d2) + 1e-2)


def _background(orc, phi_start=3.2):
    def dlnV(p):
        V, dV, _ = _pot(orc, p)
        return dV / V

    def rhs(N, s):
        return [s[1], -(3.0 - 0.5 * s[1] ** 2) * (s[1] + dlnV(s[0]))]

    sol = integrate.solve_ivp(rhs, [0.0, 60.0], [phi_start, -dlnV(phi_start)], rtol=1e-12, atol=1e-16,
                              method="DOP853", dense_output=True)

    def eps2(N):
        p, q = sol.sol(N)
        return 2.0 * rhs(N, [p, q])[1] / q

    grid = np.arange(0.0, 59.0, 0.01)
    e2 = np.array([eps2(N) for N in grid])
    i = int(np.argmax(e2 < -3.0))
    N_T = optimize.brentq(lambda N: eps2(N) + 3.0, grid[i - 1], grid[i], xtol=1e-13)
    return sol, eps2, N_T


def test_bump_parameters_are_the_printed_ones():
    """The workload's potential is the one Sec. 4.3 prints (tests/golden/printed_values.txt), and the
    two printed times are ln(sigma1/sigma2) apart to their printed precision."""
    assert W.BUMP == (GOLD["bump.m"], GOLD["bump.K"], GOLD["bump.Sigma"])
    assert W.BUMP_PHI0 == GOLD["bump.phi0"]
    gap = GOLD["bump.N2_minus_NT"] - GOLD["bump.N1_minus_NT"]
    assert abs(gap - math.log(GOLD["bump.sigma1"] / GOLD["bump.sigma2"])) < 0.05


def test_bump_background_reproduces_printed_eps2(orc):
    """eps2(N_T + 4.7) = 0.732 and eps2(N_T + 9.3) = 1.02 as printed (three figures; values from
    tests/golden/printed_values.txt)."""
    sol, eps2, N_T = _background(orc)
    N1, N2 = N_T + GOLD["bump.N1_minus_NT"], N_T + GOLD["bump.N2_minus_NT"]
    assert abs(eps2(N1) - GOLD["bump.eps2_1"]) < 0.001, eps2(N1)
    assert abs(eps2(N2) - GOLD["bump.eps2_2"]) < 0.005, eps2(N2)
    # ultra-slow roll in between: eps2 near -6
    assert min(eps2(N) for N in np.arange(N_T, N_T + 2.5, 0.05)) < -5.5
    # the workload's stored constants come from this background
    assert math.isclose(eps2(N1), W.BUMP_EPS2, rel_tol=1e-6)
    assert math.isclose(sol.sol(N_T + 4.7)[0], W.BUMP_PHI_LO, rel_tol=1e-9)


def test_bump_noise_free_passage_matches_klein_gordon(orc):
    w = W.gaussian_bump()
    V = lambda p: _pot(orc, p, V0=w.V0)[0]
    dV = lambda p: _pot(orc, p, V0=w.V0)[1]
    N_kg = _kg_passage(V, dV, w.phi_in, w.pi_in, w.phi_end)
    p = orc.Problem(kind=KIND, V0=w.V0, phi_T=PHI0, A_plus=0.0, A_minus=0.0, phi_in=w.phi_in, pi_in=w.pi_in,
                    phi_end=w.phi_end, S=np.zeros(1), tan_theta=np.zeros(1), bump=W.BUMP)
    N1 = orc.run(p, 1e-3, 1, 1)[0][0]
    N2 = orc.run(p, 5e-4, 1, 1)[0][0]
    assert math.isclose(N1, W.BUMP_N_REF, rel_tol=1e-12)
    N_rich = 2 * N2 - N1
    assert abs(N_rich - N_kg) < 2e-4, (N1, N2, N_rich, N_kg)
    assert abs(N1 - N_kg) > 5 * abs(N_rich - N_kg)


def _bump_mode_check(orc, w, phi_j, sigma, N_after):
    """(relative App. A criterion error, 4|B|^2/pi) of the node phi_j: the full mode equation with
    scipy to N_T + N_after, against P_R from the matched growing mode via
    eqs. (separate_universe_constants), (separate_universe_power_spectrum)."""
    phi_s, pi_s = w.match_start
    V = lambda p: _pot(orc, p, V0=w.V0)

    def bg(N, s):
        Vv, dV, _ = V(s[0])
        return [s[1], -(3.0 - 0.5 * s[1] ** 2) * (s[1] + dV / Vv)]

    b = integrate.solve_ivp(bg, [0.0, 45.0], [phi_s, pi_s], rtol=1e-12, atol=1e-18, method="DOP853",
                            dense_output=True)
    H = lambda N: math.sqrt(V(b.sol(N)[0])[0] / (3.0 - 0.5 * b.sol(N)[1] ** 2))
    grid = np.arange(0.0, 44.0, 0.01)
    i = int(np.argmax(np.array([b.sol(N)[0] for N in grid]) < phi_j))
    Ns = optimize.brentq(lambda N: b.sol(N)[0] - phi_j, grid[i - 1], grid[i], xtol=1e-14)
    p, q = b.sol(Ns)
    Hs = H(Ns)
    k = sigma * math.exp(Ns) * Hs
    N0 = optimize.brentq(lambda N: k - 100.0 * math.exp(N) * H(N), 0.0, Ns)
    a0, y0 = math.exp(N0), k / (math.exp(N0) * H(N0))
    Vv, dV, d2V = V(b.sol(N0)[0])
    c = (4.0 * (2.25 - 3.0 * (d2V / Vv - (dV / Vv) ** 2)) - 1.0) / 8.0
    F = (1 + 1j * c / y0) / (a0 * math.sqrt(2 * k))
    G = ((-1 - 1j * y0) * (1 + 1j * c / y0) + 1j * c / y0) / (a0 * math.sqrt(2 * k))

    def full(N, s):
        pp, qq, fr, fi, gr, gi = s
        e = 0.5 * qq * qq
        Vv, dV, d2V = V(pp)
        dq = -(3 - e) * (qq + dV / Vv)
        m2 = (k * k * math.exp(-2 * N) + d2V) * (3 - e) / Vv - qq * qq * (3 - e) - 2 * qq * dq
        return [qq, dq, gr, gi, -(3 - e) * gr - m2 * fr, -(3 - e) * gi - m2 * fi]

    _, _, N_T = _background(orc, phi_s)
    N_end = N_T + N_after
    m = integrate.solve_ivp(full, [N0, N_end], [*b.sol(N0), F.real, F.imag, G.real, G.imag], rtol=1e-10,
                            atol=1e-40, method="DOP853", dense_output=True)
    e = m.y[:, -1]
    PR_full = k ** 3 * (e[2] ** 2 + e[3] ** 2) / (4 * math.pi ** 2 * 0.5 * e[1] ** 2)
    S, t, fac = orc.noise_table_matched(KIND, w.V0, PHI0, 0.0, 0.0, sigma, 1, phi_j, phi_j, phi_s, pi_s,
                                        bump=W.BUMP)
    e1 = 0.5 * q * q
    dq = bg(Ns, [p, q])[1]
    e2 = 2 * dq / q
    eps1 = lambda N: 0.5 * m.sol(N)[1] ** 2
    Hm = lambda N: math.sqrt(V(m.sol(N)[0])[0] / (3.0 - eps1(N)))
    integral = integrate.quad(lambda N: 1.0 / (2 * eps1(N) * math.exp(3 * N) * Hm(N)), Ns, N_end, limit=800,
                              epsrel=1e-9)[0]
    dphi_h = S[0] * math.sqrt(2 * math.pi ** 2 / k ** 3)
    ddphi_h = t[0] * dphi_h
    C = dphi_h / math.sqrt(2 * e1) - math.exp(3 * Ns) * Hs * math.sqrt(2 * e1) * (e2 / 2 * dphi_h - ddphi_h) * integral
    PR_su = k ** 3 / (2 * math.pi ** 2) * C * C
    return (PR_su - PR_full) / PR_full, fac[0]


@pytest.mark.parametrize("where", [0.25, 0.75])
def test_bump_matched_table_obeys_consistency_relation(orc, where):
    """Nodes of the workload's window (sigma = 1), a quarter and three quarters of the way down."""
    w = W.gaussian_bump()
    phi_j = w.table_hi - where * (w.table_hi - w.table_lo)
    rel, fac = _bump_mode_check(orc, w, phi_j, 1.0, 18.0)
    assert abs(rel) <= 0.01, (rel, fac)
    assert abs(fac - 1.0) > 0.05     # the matched factor is not the Bunch-Davies one


def test_bump_matched_table_across_nu_equal_two(orc):
    """Later in the constant-eps2 phase nu(phi) passes 2: B_k (from J_nu alone) stays smooth."""
    w = W.gaussian_bump()
    lo, hi, n = 2.2024, 2.2029, 21
    S, t, fac = orc.noise_table_matched(KIND, w.V0, PHI0, 0.0, 0.0, 1.0, n, lo, hi, *w.match_start, bump=W.BUMP)
    nu = t + 1.5
    assert nu.min() < 2.0 < nu.max()
    assert np.all(np.isfinite(fac)) and np.all(fac > 0)
    d2 = np.abs(np.diff(np.log(fac), 2))
    assert d2.max() < 10 * np.median(d2) + 1e-6
