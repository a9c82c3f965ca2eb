"""Pins of the oracle's random numbers and noise table against things other
than itself: rocRAND's Philox4x32-10, Box-Muller invariants, the normal law,
the de Sitter limit of the noise (eq. covariance_de_sitter) and the Bessel-
function solution of the mode equation (eqs. delta_phi_bessel, A_k_and_B_k)
evaluated with scipy."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate, special, stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_words(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_words")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "helpers", "rocrand_philox_words.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(triples):
        inp = "".join(f"{s} {sub} {off}\n" for s, sub, off in triples)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)

    return run


def test_philox_matches_rocrand(orc, rocrand_words):
    rng = np.random.default_rng(123)
    cases = []
    for seed in [0, 1, 0xDEADBEEFCAFEF00D, 2**64 - 1, 42]:
        for _ in range(20):
            ctr = rng.integers(0, 2**32, 4, dtype=np.uint64)
            cases.append((seed, ctr))
    cases.append((0, np.zeros(4, dtype=np.uint64)))
    cases.append((2**64 - 1, np.full(4, 2**32 - 1, dtype=np.uint64)))
    triples = []
    for seed, c in cases:
        sub = int(c[2]) | (int(c[3]) << 32)
        triples.append((seed, sub, int(c[0]) | (int(c[1]) << 32)))
    ref = rocrand_words(triples)
    for (seed, c), r in zip(cases, ref):
        key = [seed & 0xFFFFFFFF, seed >> 32]
        got = orc.philox4x32_10(c.astype(np.uint32), key)
        assert np.array_equal(got.astype(np.uint64), r), (seed, c, got, r)


def test_counter_layout_and_uniforms(orc):
    """u_j * 2^32 - 1/2 are the Philox words of counter (traj lo, m, traj hi, instance)."""
    for seed, inst, traj, m in [(5, 0, 0, 0), (5, 3, 2**40 + 17, 123456), (2**63 + 9, 7, 99, 2**31 + 5)]:
        u = orc.uniforms(seed, inst, traj, m)
        w = orc.philox4x32_10([traj & 0xFFFFFFFF, m & 0xFFFFFFFF, traj >> 32, inst],
                              [seed & 0xFFFFFFFF, seed >> 32])
        assert np.array_equal(u * 2.0**32 - 0.5, w.astype(np.float64))
        assert np.all((u > 0) & (u < 1))


def test_box_muller_invariants(orc):
    """(xi_{4m}, xi_{4m+1}) has squared radius -2 ln u0 and angle 2 pi u1; likewise (u2, u3)."""
    rng = np.random.default_rng(9)
    for _ in range(200):
        seed = int(rng.integers(0, 2**63))
        traj = int(rng.integers(0, 2**40))
        m = int(rng.integers(0, 2**30))
        u = orc.uniforms(seed, 1, traj, m)
        z = orc.normals(seed, 1, traj, 4 * m, 4)
        for a, b, ur, ua in [(z[0], z[1], u[0], u[1]), (z[2], z[3], u[2], u[3])]:
            assert math.isclose(a * a + b * b, -2.0 * math.log(ur), rel_tol=1e-13)
            ang = math.atan2(b, a) % (2 * math.pi)
            d = abs(ang - 2 * math.pi * ua)
            d = min(d, 2 * math.pi - d)
            assert d < 1e-12


def test_normals_are_standard_normal(orc):
    z = np.concatenate([orc.normals(11, 0, t, 0, 4000) for t in range(100)])
    assert abs(z.mean()) < 4 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 4 * math.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # consecutive draws are uncorrelated (step n and n+1 of a trajectory)
    r = np.corrcoef(z[:-1], z[1:])[0, 1]
    assert abs(r) < 4 / math.sqrt(z.size)


# --------------------------------------------------------------------------
# noise table
# --------------------------------------------------------------------------
def test_de_sitter_limit(orc):
    """nu = 3/2 exactly for V = V0 exp(alpha phi) (V''/V = (V'/V)^2): the table reduces to
    Xi = (H/2pi)^2 diag(1, 0), H^2 = V/3, independent of sigma (eq. covariance_de_sitter)."""
    V0, alpha = 3e-10, 0.7
    phis = np.linspace(-0.5, 0.5, 11)
    for sigma in (1.0, 0.01):
        S, t = orc.noise_table_bessel(orc.POT_EXPONENTIAL, V0, 0.0, alpha, 0.0, sigma, 11, -0.5, 0.5)
        H = np.sqrt(V0 * np.exp(alpha * phis) / 3.0)
        np.testing.assert_allclose(S, H / (2 * np.pi), rtol=1e-13)
        assert np.all(np.abs(t) < 1e-14)


def _bd_mode_power(nu, x, H):
    """(k^3/2pi^2)|delta phi_k|^2 for the Bessel solution with Bunch-Davies coefficients
    in de Sitter (a = -1/(H eta)), as a function of x = -k eta."""
    A = math.sqrt(math.pi) / 2 * np.exp(1j * (nu + 0.5) * math.pi / 2)
    B = math.sqrt(math.pi) / 2 * np.exp(1j * (nu + 1.5) * math.pi / 2)
    amp = A * special.jv(nu, x) + B * special.yv(nu, x)
    return H**2 * x**3 * np.abs(amp) ** 2 / (2 * math.pi**2)


def test_bd_mode_normalisation_sanity():
    """The test's own Bessel solution tends to the Bunch-Davies vacuum |delta phi|^2 = 1/(2 k a^2)
    deep inside the horizon (eq. bunch_davies), i.e. (k^3/2pi^2)|dphi|^2 -> H^2 x^2 / (4 pi^2)."""
    H = 1.3
    for nu in (1.5, 1.62):
        x = 3000.0
        assert math.isclose(_bd_mode_power(nu, x, H), H**2 * x**2 / (4 * math.pi**2), rel_tol=1e-3)


@pytest.mark.parametrize("sigma", [1.0, 0.3, 0.01])
def test_table_is_growing_mode_of_bessel_solution(orc, sigma):
    """S^2 equals the super-horizon growing mode of the Bunch-Davies Bessel solution extrapolated
    to -k eta = sigma, and tan(theta_n) = d ln(delta phi_h)/dN (eqs. delta_phi_bessel, A_k_and_B_k,
    covariance_matrix, noise_phase_space_angle_1D), computed here from scipy's J_nu, Y_nu."""
    V0 = 1e-10
    Ap, Am = V0 * 0.1414213562373095, V0 * 0.0204  # steep and moderately flat branches
    n, lo, hi = 9, -0.004, 0.004
    S, t = orc.noise_table_bessel(orc.POT_PIECEWISE_LINEAR, V0, 0.0, Ap, Am, sigma, n, lo, hi)
    phis = lo + (hi - lo) * np.arange(n) / (n - 1)
    for phi, Sj, tj in zip(phis, S, t):
        nu = tj + 1.5
        V = V0 + (Ap if phi >= 0 else Am) * phi
        H = math.sqrt(V / 3.0)
        x = 1e-5
        grow = _bd_mode_power(nu, x, H) * x ** (2 * nu - 3)   # x-independent growing-mode amplitude
        assert math.isclose(Sj**2, grow * sigma ** (3 - 2 * nu), rel_tol=1e-7)
        # d ln|delta phi_h| / dN with x proportional to e^-N, delta phi proportional to x^{3/2} |A J + B Y|
        def lnamp(lx):
            xx = math.exp(lx)
            return 1.5 * lx + 0.5 * math.log(_bd_mode_power(nu, xx, 1.0) / xx**3)
        h = 1e-3
        dlnphi_dN = -(lnamp(math.log(x) + h) - lnamp(math.log(x) - h)) / (2 * h)
        assert abs(dlnphi_dN - tj) < 1e-6


def test_table_nu_matches_hubble_flow_form(orc):
    """nu^2 of the table (eq. nu_squared_approximation, a function of phi only) agrees to O(eps_1)
    with eq. nu_squared, evaluated from the Hubble-flow parameters eps_1..eps_3 of a background
    solved in cosmic time from eqs. klein_gordon and Friedmann (scipy)."""
    V0, r = 1e-10, 0.2
    Ap = V0 * r
    # background on the slow-roll attractor of V = V0 + Ap phi (same slope on both sides)
    def rhs(t, y):
        phi, dphi = y
        V = V0 + Ap * phi
        H = math.sqrt((V + 0.5 * dphi**2) / 3.0)
        return [dphi, -3 * H * dphi - Ap]
    phi0 = 2.0
    V = V0 + Ap * phi0
    H0 = math.sqrt(V / 3.0)
    sol = integrate.solve_ivp(rhs, [0, 8 / H0], [phi0, -Ap / (3 * H0)], rtol=1e-11, atol=1e-20,
                              dense_output=True)
    ts = np.linspace(3 / H0, 6 / H0, 4001)
    phi, dphi = sol.sol(ts)
    Vt = V0 + Ap * phi
    H = np.sqrt((Vt + 0.5 * dphi**2) / 3.0)
    N = integrate.cumulative_trapezoid(H, ts, initial=0.0)
    e1 = dphi**2 / (2 * H**2)
    e2 = np.gradient(np.log(e1), N)
    e3 = np.gradient(np.log(np.abs(e2)), N)
    nu2_flow = 9 / 4 - e1 + 1.5 * e2 - 0.5 * e1 * e2 + 0.25 * e2**2 + 0.5 * e2 * e3
    k = len(ts) // 2
    S, t = orc.noise_table_bessel(orc.POT_PIECEWISE_LINEAR, V0, 0.0, Ap, Ap, 1.0, 1, phi[k], phi[k])
    nu2_table = (t[0] + 1.5) ** 2
    assert abs(nu2_table - nu2_flow[k]) < 1.5 * e1[k]
    assert nu2_table - 9 / 4 > 0.5 * (nu2_flow[k] - 9 / 4)
