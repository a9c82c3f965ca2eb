"""Pins of the oracle's trajectories against closed forms, exact laws and
independent solvers:

* the slow-roll fixed point pi = -V'/V of the exponential potential (exact),
* the linear relaxation rate 3 - pi^2/2 around it (geometric series),
* the noise-free passage time against eqs. klein_gordon + Friedmann solved in
  cosmic time by scipy (Richardson-extrapolated Euler-Maruyama),
* the inverse-Gaussian first-passage law of a Brownian motion with drift
  (textbook; KS test), and its far tail under importance sampling (closed form),
* ln w of a constant bias as a closed-form sum of the same Gaussian numbers,
* phi and pi of a linear (Ornstein-Uhlenbeck) regime as closed-form sums
  (scipy.signal.lfilter), which fixes the tan(theta_n) factors, the bias
  direction and the sqrt(dN) noise scaling,
* E_Q[w] = 1 (unbiasedness of the weights, eq. weight),
* the linear-theory spread of N for the linear slow-roll workload.
"""
import math

import numpy as np
import pytest
from scipy import integrate, signal, special, stats

from paper_2410_13683_amd import workloads as W
from tests._glue import oracle_problem, oracle_run


def _exp_problem(orc, alpha, S, phi_in, phi_end, pi_in, A_bias=0.0, tan=0.0):
    return orc.Problem(kind=orc.POT_EXPONENTIAL, V0=1e-10, phi_T=0.0, A_plus=alpha, A_minus=0.0,
                       phi_in=phi_in, pi_in=pi_in, phi_end=phi_end, S=np.array([S]), tan_theta=np.array([tan]),
                       bias_kind=orc.BIAS_CONST if A_bias else orc.BIAS_NONE, A_bias=A_bias)


def test_fixed_point_is_exact(orc):
    """pi = -V'/V is a fixed point of the drift; with no noise phi moves at exactly alpha per e-fold."""
    for alpha in (0.1, 0.5, 1.3):
        p = _exp_problem(orc, alpha, 0.0, 1.0, 0.0, -alpha)
        N, lnw, steps = orc.run(p, 1e-3, 1, 1)
        assert abs(N[0] - 1.0 / alpha) < 1e-9
        assert lnw[0] == 0.0


def test_relaxation_rate(orc):
    """A small offset delta of pi from -alpha decays geometrically with factor 1 - (3 - alpha^2/2) dN,
    so the extra distance covered is delta / (3 - alpha^2/2) and N = (dphi + delta/lambda)/alpha."""
    alpha, delta, dN, dphi = 1.0, 1e-5, 1e-4, 6.0   # e^{-lambda N} ~ 3e-7 left at the passage
    p = _exp_problem(orc, alpha, 0.0, dphi, 0.0, -alpha + delta)
    N, _, _ = orc.run(p, dN, 1, 1)
    lam = 3.0 - alpha**2 / 2.0
    expected = (dphi + delta / lam) / alpha
    assert abs((N[0] - dphi / alpha) / (expected - dphi / alpha) - 1.0) < 2e-3


def _kg_passage(V, dV, phi_in, pi_in, phi_end):
    """e-folds from (phi_in, dphi/dN = pi_in) to phi_end from eqs. klein_gordon and Friedmann in
    cosmic time (3H^2 = V + phidot^2/2, phidot = pi H)."""
    H0 = math.sqrt(V(phi_in) / (3.0 - pi_in**2 / 2.0))

    def rhs(t, y):
        phi, dphi, N = y
        H = math.sqrt((V(phi) + 0.5 * dphi**2) / 3.0)
        return [dphi, -3.0 * H * dphi - dV(phi), H]

    ev = lambda t, y: y[0] - phi_end
    ev.terminal = True
    sol = integrate.solve_ivp(rhs, [0, 1e4 / H0], [phi_in, pi_in * H0, 0.0], events=ev,
                              rtol=1e-12, atol=[1e-16, 1e-22, 1e-14], method="DOP853")
    return float(sol.y_events[0][0][2])


@pytest.mark.parametrize("which", ["linear", "srusr"])
def test_noise_free_passage_matches_klein_gordon(orc, which):
    if which == "linear":
        w = W.linear_slow_roll()
        dNs, tol = (1e-3, 5e-4), 2e-6
    else:
        w = W.srusr_bessel()
        dNs, tol = (1e-4, 5e-5), 5e-3
    Ap, Am, V0, phiT = w.A_plus, w.A_minus, w.V0, w.phi_T
    V = lambda phi: V0 + (Ap if phi >= phiT else Am) * (phi - phiT)
    dV = lambda phi: Ap if phi >= phiT else Am
    N_kg = _kg_passage(V, dV, w.phi_in, w.pi_in, w.phi_end)
    p = orc.Problem(kind=w.kind, V0=V0, phi_T=phiT, A_plus=Ap, A_minus=Am, phi_in=w.phi_in, pi_in=w.pi_in,
                    phi_end=w.phi_end, S=np.zeros(1), tan_theta=np.zeros(1))
    N1 = orc.run(p, dNs[0], 1, 1)[0][0]
    N2 = orc.run(p, dNs[1], 1, 1)[0][0]
    N_rich = 2 * N2 - N1          # Euler-Maruyama is first order in dN
    assert abs(N_rich - N_kg) < tol, (N1, N2, N_rich, N_kg)
    assert abs(N1 - N_kg) > abs(N_rich - N_kg)


def _ig_params(w):
    mu = (w.phi_in - w.phi_end) / w.A_plus
    lam = (w.phi_in - w.phi_end) ** 2 / w.noise_S**2
    return mu, lam


def _ig_sf(x, mu, lam):
    """P(N > x) of the inverse-Gaussian law, written with erfcx to stay finite far in the tail."""
    A = math.sqrt(lam / x) * (x / mu - 1.0)
    B = math.sqrt(lam / x) * (x / mu + 1.0)
    return 0.5 * math.exp(-A * A / 2.0) * (special.erfcx(A / math.sqrt(2)) - special.erfcx(B / math.sqrt(2)))


def test_inverse_gaussian_law(orc):
    """Constant V'/V = alpha, pi = -alpha, constant noise along phi only: N ~ IG(dphi/alpha, dphi^2/S^2)."""
    w = W.exponential_ig(n_traj=20_000)
    N, lnw, steps = oracle_run(w)
    assert np.all(steps & (orc.FLAG_CENSORED | orc.FLAG_ENDED_EARLY) == 0)
    assert np.all(lnw == 0.0)
    mu, lam = _ig_params(w)
    ks = stats.kstest(N, stats.invgauss(mu / lam, scale=lam).cdf)
    assert ks.pvalue > 1e-3, ks
    # closed-form check of the survival function used below
    x = mu * 1.3
    assert math.isclose(_ig_sf(x, mu, lam), stats.invgauss(mu / lam, scale=lam).sf(x), rel_tol=1e-9)


def test_importance_sampled_tail(orc):
    """With a constant bias the weighted estimate of P(N > x) far in the tail matches the
    inverse-Gaussian closed form (eqs. weight, weight_A; bias parallel to the noise)."""
    A_bias = 2.6
    w = W.exponential_ig(n_traj=20_000, A_bias=A_bias, seed=17)
    N, lnw, steps = oracle_run(w)
    mu, lam = _ig_params(w)
    sd = math.sqrt(mu**3 / lam)
    for k in (5.0, 6.5, 8.0):
        x = mu + k * sd
        ind = N > x
        wts = np.exp(lnw) * ind
        est = wts.mean()
        se = wts.std() / math.sqrt(len(N))
        exact = _ig_sf(x, mu, lam)
        assert exact < 1e-4
        assert abs(est / exact - 1.0) < 0.05 + 4 * se / exact, (k, est, exact, se)


def test_log_weight_closed_form(orc):
    """ln w = -A sqrt(dN) sum_{k<n} xi_k - n A^2 dN / 2 for a constant amplitude and S > 0."""
    w = W.linear_slow_roll().with_(bias_kind=W.BIAS_CONST, A_bias=1.7, seed=21)
    N, lnw, steps = oracle_run(w, n_traj=8)
    for i in range(8):
        n = int(steps[i] & orc.STEP_MASK)
        z = orc.normals(w.seed, 0, i, 0, n)
        ref = -w.A_bias * math.sqrt(w.dN) * z.sum() - n * w.A_bias**2 * w.dN / 2.0
        assert abs(lnw[i] - ref) < 1e-9 * max(1.0, abs(ref))


def test_linear_regime_closed_form(orc):
    """Flat potential (V'/V = 0), constant noise S along (1, t), constant bias A, and pi so small that
    pi^2/2 is negligible: pi_n is the linear filter pi_{n+1} = (1 - 3 dN) pi_n + t S (A dN + xi_n sqrt(dN))
    and phi_n = phi_0 + sum_{k<n} (pi_k + A S) dN + S sqrt(dN) sum_{k<n} xi_k.  The passage step and the
    interpolated N must match these sums."""
    S, t, A, dN = 1e-6, 0.35, -1e4, 1e-4
    phi_in, phi_end = 1e-3, 0.0
    p = _exp_problem(orc, 0.0, S, phi_in, phi_end, 0.0, A_bias=A, tan=t)
    n_check = 6
    N, lnw, steps = orc.run(p, dN, 33, n_check)
    for i in range(n_check):
        n = int(steps[i] & orc.STEP_MASK)
        z = orc.normals(33, 0, i, 0, n + 1)
        b = t * S * (A * dN + z * math.sqrt(dN))
        pis = np.concatenate([[0.0], signal.lfilter([1.0], [1.0, -(1.0 - 3.0 * dN)], b)])  # pi_0..pi_{n+1}
        phis = phi_in + np.concatenate([[0.0], np.cumsum((pis[:-1] + A * S) * dN + S * math.sqrt(dN) * z)])
        first = int(np.argmax(phis <= phi_end))
        assert first == n
        N_ref = (n - 1) * dN + dN * (phis[n - 1] - phi_end) / (phis[n - 1] - phis[n])
        assert abs(N[i] - N_ref) < 1e-12 + 1e-10 * N_ref
        # the pi contribution matters at the level tested: dropping it moves N by far more
        phis_nopi = phi_in + np.concatenate([[0.0], np.cumsum(A * S * dN + S * math.sqrt(dN) * z)])
        n2 = int(np.argmax(phis_nopi <= phi_end))
        N_nopi = (n2 - 1) * dN + dN * (phis_nopi[n2 - 1] - phi_end) / (phis_nopi[n2 - 1] - phis_nopi[n2])
        assert abs(N_nopi - N_ref) > 1e3 * abs(N[i] - N_ref) + 1e-9


def test_weights_have_unit_mean(orc):
    """E_Q[w] = 1: the weights reweight the biased paths to the unbiased measure."""
    w = W.exponential_ig(n_traj=20_000, A_bias=1.0, seed=5)
    N, lnw, steps = oracle_run(w)
    wt = np.exp(lnw)
    assert abs(wt.mean() - 1.0) < 4 * wt.std() / math.sqrt(len(wt))


def test_linear_workload_mean_and_spread(orc):
    """Linear slow roll with constant noise: <N> equals the noise-free Euler-Maruyama value and the
    spread equals the linear-theory value S sqrt(int dphi / v^3) = 1.918e-5 (v = V'/V on the attractor)."""
    w = W.linear_slow_roll(n_traj=10_000)
    N, lnw, steps = oracle_run(w)
    sd = N.std()
    assert abs(N.mean() - W.N_REF_LINEAR) < 5 * sd / math.sqrt(len(N))
    assert abs(sd / W.SIGMA_LIN_LINEAR - 1.0) < 0.04


def test_censoring_and_early_end_flags(orc):
    w = W.linear_slow_roll(n_traj=4).with_(max_steps=1000)
    N, lnw, steps = oracle_run(w)
    assert np.all(steps == (1000 | orc.FLAG_CENSORED))
    assert np.all(np.isnan(N))
    # pi_in^2/2 > 1 from the start: the first step ends inflation before phi_end
    p = _exp_problem(orc, 0.1, 1e-6, 1.0, 0.0, -1.6)
    N, lnw, steps = orc.run(p, 1e-3, 1, 3)
    assert np.all(steps == (1 | orc.FLAG_ENDED_EARLY))
    np.testing.assert_allclose(N, 1e-3)


def test_last_step_phi_values(orc):
    """The oracle's phi before and after each trajectory's last step (what the per-trajectory
    parity check uses to recognise near-ties): phi before it is the state a run capped one step
    earlier ends in, the step crosses phi_end, and the interpolation N = (n - 1 + f) dN with
    f = (phi_(n-1) - phi_end)/(phi_(n-1) - phi_n) gives the oracle's N."""
    w = W.srusr_bessel(n_traj=40, seed=29).with_(bias_kind=W.BIAS_CONST, A_bias=1.0)
    N, lnw, st, phi2 = oracle_run(w, last_phi=True)
    n = (st & orc.STEP_MASK).astype(np.int64)
    assert np.all((st & (orc.FLAG_CENSORED | orc.FLAG_ENDED_EARLY)) == 0)
    assert np.all(phi2[:, 0] > w.phi_end) and np.all(phi2[:, 1] <= w.phi_end)
    f = (phi2[:, 0] - w.phi_end) / (phi2[:, 0] - phi2[:, 1])
    np.testing.assert_allclose(N, (n - 1) * w.dN + w.dN * f, rtol=1e-15)
    for i in (0, 17, 39):
        _, _, st_c, phi2_c = oracle_run(w.with_(max_steps=int(n[i] - 1)), n_traj=1, traj_offset=i, last_phi=True)
        assert st_c[0] == (n[i] - 1) | orc.FLAG_CENSORED
        assert phi2_c[0, 0] == phi2_c[0, 1] == phi2[i, 0]
