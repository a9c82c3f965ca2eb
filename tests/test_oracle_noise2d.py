"""Pins of the oracle's two-dimensional noise: the covariance of the full mode
function at -k eta = sigma against scipy's Bessel functions, the massless de
Sitter closed form and the Wronskian; the symmetric square root; the 2D random
stream; and the 2D dynamics against closed-form sums, the inverse-Gaussian law
and unit-mean weights."""
import math

import numpy as np
import pytest
from scipy import linalg, signal, special, stats

from paper_2410_13683_amd import workloads as W


def _bd_mode(nu, y):
    """F = y^(3/2) [A J_nu + B Y_nu] and -y F' with scipy's Bessel functions (A, B Bunch-Davies)."""
    A = 0.5 * math.sqrt(math.pi) * np.exp(1j * (nu + 0.5) * math.pi / 2)
    B = 0.5 * math.sqrt(math.pi) * np.exp(1j * (nu + 1.5) * math.pi / 2)
    Z = A * special.jv(nu, y) + B * special.yv(nu, y)
    dZ = A * special.jvp(nu, y) + B * special.yvp(nu, y)
    F = y ** 1.5 * Z
    dF = 1.5 * y ** 0.5 * Z + y ** 1.5 * dZ
    return F, -y * dF


@pytest.mark.parametrize("sigma", [0.01, 0.1, 0.7, 1.5])
def test_table2d_matches_bessel_functions(orc, sigma):
    """Xi from the oracle's power series equals Xi from scipy's J_nu, Y_nu and their derivatives."""
    w = W.srusr_bessel()
    n = 7
    X = orc.noise_table_bessel2d(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, sigma, n, w.table_lo, w.table_hi)
    h = (w.table_hi - w.table_lo) / (n - 1)
    for j in range(n):
        phi = w.table_lo + j * h
        V, dV, d2V = orc.potential(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, phi)
        nu = math.sqrt(9 / 4 - 3 * (d2V / V - (dV / V) ** 2))
        F, G = _bd_mode(nu, sigma)
        c = V / 3 / (2 * math.pi ** 2)
        ref = (c * abs(F) ** 2, c * (F * np.conj(G)).real, c * abs(G) ** 2)
        for k in range(3):
            assert math.isclose(X[k][j], ref[k], rel_tol=1e-10, abs_tol=1e-12 * ref[0]), (j, k, X[k][j], ref[k])


@pytest.mark.parametrize("sigma", [0.02, 0.4, 1.0, 2.0])
def test_table2d_de_sitter_closed_form(orc, sigma):
    """Exponential potential: nu = 3/2 exactly, the massless mode H/sqrt(2k^3) (1 - i k eta) e^(-i k eta)
    gives Xi = H^2/(4 pi^2) [[1 + s^2, -s^2], [-s^2, s^4]] at -k eta = s."""
    V0, alpha, phi = 1e-10, 0.3, 0.4
    X = orc.noise_table_bessel2d(1, V0, 0.0, alpha, 0.0, sigma, 1, phi, phi)
    c = V0 * math.exp(alpha * phi) / 3 / (4 * math.pi ** 2)
    ref = (c * (1 + sigma ** 2), -c * sigma ** 2, c * sigma ** 4)
    for k in range(3):
        assert math.isclose(X[k][0], ref[k], rel_tol=1e-12), (k, X[k][0], ref[k])


@pytest.mark.parametrize("sigma", [0.01, 0.3, 1.0])
def test_table2d_determinant_is_the_wronskian(orc, sigma):
    """Canonical normalisation: Im(dphi dpi*) = sigma^3/2 in units H^2/k^3 for every nu, so
    det Xi = (H^2 sigma^3 / (4 pi^2))^2 at every node (both branches of the potential)."""
    w = W.srusr_bessel()
    n = 9
    X = orc.noise_table_bessel2d(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, sigma, n, w.table_lo, w.table_hi)
    h = (w.table_hi - w.table_lo) / (n - 1)
    for j in range(n):
        V = orc.potential(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.table_lo + j * h)[0]
        det = X[0][j] * X[2][j] - X[1][j] ** 2
        ref = (V / 3 * sigma ** 3 / (4 * math.pi ** 2)) ** 2
        assert math.isclose(det, ref, rel_tol=1e-6 if sigma < 0.1 else 1e-9), (j, det, ref)


def test_table2d_growing_mode_limit(orc):
    """sigma -> 0: the growing mode dominates, Xi_pp -> the 1D table's S^2 and Xi_pq/Xi_pp -> tan theta_n
    (eq. covariance_constant_nu); the gradient corrections are O(sigma^2) (relative in Xi_pp, absolute in
    the ratio, which is tan theta_n ~ 2e-8 on the flat branch)."""
    w = W.srusr_bessel()
    n, sigma = 5, 1e-6
    X = orc.noise_table_bessel2d(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, sigma, n, w.table_lo, w.table_hi)
    S, t = orc.noise_table_bessel(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, sigma, n, w.table_lo, w.table_hi)
    np.testing.assert_allclose(X[0], S ** 2, rtol=1e-10)
    np.testing.assert_allclose(X[1] / X[0], t, rtol=1e-8, atol=3 * sigma ** 2)


def test_sqrt_sym2_is_the_matrix_square_root(orc):
    rng = np.random.default_rng(0)
    for _ in range(50):
        M = rng.standard_normal((2, 2)) * 10.0 ** rng.uniform(-7, -5)
        Xi = M @ M.T + np.eye(2) * 10.0 ** rng.uniform(-16, -12)
        Spp, Spq, Sqq = orc.sqrt_sym2(Xi[0, 0], Xi[0, 1], Xi[1, 1])
        S = np.array([[Spp, Spq], [Spq, Sqq]])
        np.testing.assert_allclose(S, linalg.sqrtm(Xi).real, rtol=1e-7, atol=1e-12 * np.abs(S).max())
        np.testing.assert_allclose(S @ S, Xi, rtol=1e-10, atol=1e-12 * Xi.max())
    assert orc.sqrt_sym2(0.0, 0.0, 0.0) == (0.0, 0.0, 0.0)
    with pytest.raises(ValueError):
        orc.sqrt_sym2(1.0, 2.0, 1.0)             # indefinite


def test_normals2d_are_the_1d_stream_in_pairs(orc):
    """Step n of a 2D trajectory takes (xi_1, xi_2) = normals 2n and 2n+1 of the 1D stream."""
    z2 = orc.normals2d(11, 3, 12345, 5, 40)
    z1 = orc.normals(11, 3, 12345, 10, 80)
    assert np.array_equal(z2.reshape(-1), z1)


def _flat_problem(orc, Xi, phi_in, phi_end, A_bias):
    return orc.Problem2D(kind=1, V0=1e-10, phi_T=0.0, A_plus=0.0, A_minus=0.0, phi_in=phi_in, pi_in=0.0,
                         phi_end=phi_end, Xpp=np.array([Xi[0]]), Xpq=np.array([Xi[1]]), Xqq=np.array([Xi[2]]),
                         bias_kind=1 if A_bias else 0, A_bias=A_bias)


def _axis(Xi):
    """Unit eigenvector of the largest eigenvalue with a non-negative phi component (numpy)."""
    vals, vecs = np.linalg.eigh(np.array([[Xi[0], Xi[1]], [Xi[1], Xi[2]]]))
    e = vecs[:, int(np.argmax(vals))]
    return e if e[0] >= 0 else -e


def test_principal_axis_matches_eigh(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, c = rng.uniform(0, 2, 2)
        b = rng.uniform(-1, 1) * math.sqrt(a * c)
        e = orc.principal_axis(a, b, c)
        ref = _axis((a, b, c))
        assert abs(e[0] * ref[0] + e[1] * ref[1]) > 1 - 1e-12 and e[0] >= 0
    assert orc.principal_axis(0.0, 0.0, 0.0) == (1.0, 0.0)
    assert orc.principal_axis(2.0, 0.0, 2.0) == (1.0, 0.0)
    assert orc.principal_axis(1.0, 0.0, 2.0) == (0.0, 1.0)


def test_2d_linear_regime_closed_form(orc):
    """Flat potential (V'/V = 0), constant 2D noise S, constant bias B = A S e (e the principal axis) and
    pi so small that pi^2/2 is negligible: pi_{n+1} = (1 - 3 dN) pi_n + B_pi dN + (S_pq xi1 + S_qq xi2) sqrt(dN),
    phi_n = phi_0 + sum_{k<n} (pi_k + B_phi) dN + sqrt(dN) sum_{k<n} (S_pp xi1 + S_pq xi2).  The passage step,
    the interpolated N and ln w = -A sqrt(dN) sum (e . xi) - n A^2 dN / 2 must match these sums."""
    Xi = (1.0e-12, 4.0e-13, 6.0e-13)
    S = linalg.sqrtm(np.array([[Xi[0], Xi[1]], [Xi[1], Xi[2]]])).real
    e = _axis(Xi)
    A, dN, phi_in, phi_end = -1e4, 1e-4, 1e-3, 0.0
    B = A * S @ e
    p = _flat_problem(orc, Xi, phi_in, phi_end, A)
    n_check = 6
    N, lnw, steps = orc.run2d(p, dN, 33, n_check)
    for i in range(n_check):
        n = int(steps[i] & orc.STEP_MASK)
        z = orc.normals2d(33, 0, i, 0, n + 1)
        noise = (z @ S.T) * math.sqrt(dN)                     # rows: S xi sqrt(dN)
        pis = np.concatenate([[0.0], signal.lfilter([1.0], [1.0, -(1.0 - 3.0 * dN)], B[1] * dN + noise[:, 1])])
        incr = (pis[:-1] + B[0]) * dN + noise[:, 0]
        phis = phi_in + np.concatenate([[0.0], np.cumsum(incr)])
        assert int(np.argmax(phis <= phi_end)) == n
        N_ref = (n - 1) * dN + dN * (phis[n - 1] - phi_end) / (phis[n - 1] - phis[n])
        assert abs(N[i] - N_ref) < 1e-12 + 1e-10 * N_ref
        l_ref = -A * math.sqrt(dN) * (z[:n] @ e).sum() - n * A * A * dN / 2
        assert abs(lnw[i] - l_ref) < 1e-9 * max(1.0, abs(l_ref))


def _ig_sf(x, mu, lam):
    A = math.sqrt(lam / x) * (x / mu - 1.0)
    B = math.sqrt(lam / x) * (x / mu + 1.0)
    return 0.5 * math.exp(-A * A / 2.0) * (special.erfcx(A / math.sqrt(2)) - special.erfcx(B / math.sqrt(2)))


def _ig2d(orc, S, delta, A_bias):
    """Exponential potential, pi_in = -alpha, 2D noise diag(S^2, delta^2) with delta << S."""
    alpha, dphi = 0.5, 1.0
    return orc.Problem2D(kind=1, V0=1e-10, phi_T=0.0, A_plus=alpha, A_minus=0.0, phi_in=dphi, pi_in=-alpha,
                         phi_end=0.0, Xpp=np.array([S * S]), Xpq=np.array([0.0]), Xqq=np.array([delta * delta]),
                         bias_kind=1 if A_bias else 0, A_bias=A_bias), dphi / alpha, dphi ** 2 / S ** 2


def test_2d_inverse_gaussian_law_and_tail(orc):
    """With noise along phi and a vanishing pi component the 2D system is the 1D Brownian motion with
    drift: N is inverse-Gaussian; with the bias B = A S e_phi the weighted tail matches the closed form."""
    S = 0.05
    p, mu, lam = _ig2d(orc, S, 1e-7 * S, 0.0)
    N, lnw, _ = orc.run2d(p, 1e-4, 7, 20_000)
    assert np.all(lnw == 0.0)
    ks = stats.kstest(N, stats.invgauss(mu / lam, scale=lam).cdf)
    assert ks.pvalue > 1e-3, ks
    p, mu, lam = _ig2d(orc, S, 1e-7 * S, 2.6)
    N, lnw, _ = orc.run2d(p, 1e-4, 17, 20_000)
    sd = math.sqrt(mu ** 3 / lam)
    for k in (5.0, 6.5, 8.0):
        x = mu + k * sd
        wts = np.exp(lnw) * (N > x)
        est, se, exact = wts.mean(), wts.std() / math.sqrt(len(N)), _ig_sf(x, mu, lam)
        assert abs(est / exact - 1.0) < 0.05 + 4 * se / exact, (k, est, exact, se)


def test_2d_weights_have_unit_mean_with_correlated_noise(orc):
    """E_Q[w] = 1 with a strongly correlated, non-singular 2D noise acting on both phi and pi."""
    S = 0.05
    p = orc.Problem2D(kind=1, V0=1e-10, phi_T=0.0, A_plus=0.5, A_minus=0.0, phi_in=1.0, pi_in=-0.5, phi_end=0.0,
                      Xpp=np.array([S * S]), Xpq=np.array([0.8 * S * S]), Xqq=np.array([S * S]),
                      bias_kind=1, A_bias=1.2)
    N, lnw, _ = orc.run2d(p, 1e-3, 5, 20_000)
    wt = np.exp(lnw)
    assert abs(wt.mean() - 1.0) < 4 * wt.std() / math.sqrt(len(wt))
    assert np.std(lnw) > 0.5


def test_2d_rank_one_limit_is_the_1d_law(orc):
    """Xi = s s^T + tiny identity with s = S (1, t): the principal axis is s/|s|, the bias A S e = A s is the
    1D bias and dA = A (e . xi) sqrt(dN) + A^2 dN/2 the 1D weight with the 1D normal e . xi.  The 2D process
    then has the law of the 1D process (two-sample KS on N and on ln w, different random numbers)."""
    from tests._glue import oracle_problem
    w = W.linear_slow_roll(n_traj=6000).with_(noise_tan=0.4)
    S, t = w.noise_S, 0.4
    eps = (1e-4 * S) ** 2
    for A in (0.0, 1.5):
        w1 = w.with_(bias_kind=1 if A else 0, A_bias=A)
        N1, l1, _ = orc.run(oracle_problem(w1), w.dN, 3, w.n_traj)
        p2 = orc.Problem2D(kind=w.kind, V0=w.V0, phi_T=w.phi_T, A_plus=w.A_plus, A_minus=w.A_minus,
                           phi_in=w.phi_in, pi_in=w.pi_in, phi_end=w.phi_end, Xpp=np.array([S * S + eps]),
                           Xpq=np.array([S * S * t]), Xqq=np.array([S * S * t * t + eps]),
                           bias_kind=1 if A else 0, A_bias=A)
        N2, l2, _ = orc.run2d(p2, w.dN, 4, w.n_traj)
        assert stats.ks_2samp(N1, N2).pvalue > 1e-3
        if A:
            assert stats.ks_2samp(l1, l2).pvalue > 1e-3
