"""Pins of the oracle's noise indexed by time (the paper's scheme, Sec. 4.1: noise
precomputed along the classical trajectory, indexed by time and switched off after
a fixed number of steps).
- The time-node matched table equals the phi-node one at the trajectory's phi.
- With a switch-off, ln w follows its closed form, which counts exactly the steps
  with n dN inside the noisy part of the table.
- With vanishing noise, a time-indexed run and a phi-indexed run along the same
  classical trajectory coincide."""
import math

import numpy as np
import pytest

from paper_2410_13683_amd import workloads as W


def test_time_nodes_equal_phi_nodes(orc):
    w = W.srusr_matched()
    taus = np.array([0.3, 1.2, 2.4, 4.0, 7.0])
    for tau in taus:
        S, t, fac, ph = orc.noise_table_matched_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, 1, tau, tau,
                                                     *w.match_start, w.phi_in)
        Sp, tp, fp = orc.noise_table_matched(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, 1, ph[0], ph[0],
                                             *w.match_start)
        assert ph[0] < w.phi_in
        np.testing.assert_allclose([S[0], t[0], fac[0]], [Sp[0], tp[0], fp[0]], rtol=1e-12, atol=1e-15)
    # the node at tau = 0 is the reference point: on the kink (phi_ref = phi_T = 0) it is the phi node
    # at phi_T exactly, on the branch before the kink, whatever the rounding of the trajectory
    S, t, fac, ph = orc.noise_table_matched_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, 2, 0.0, 0.01,
                                                 *w.match_start, w.phi_T)
    Sp, tp, fp = orc.noise_table_matched(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, 1, w.phi_T, w.phi_T,
                                         *w.match_start)
    assert ph[0] == w.phi_T and ph[1] < w.phi_T
    np.testing.assert_allclose([S[0], t[0], fac[0]], [Sp[0], tp[0], fp[0]], rtol=1e-12, atol=1e-15)
    assert abs(fac[0] - 1.0) < 1e-3 and fac[1] < 0.5      # before and after the kink's kick
    # a node outside the followed trajectory, and a reference the trajectory never passes, are errors
    with pytest.raises(ValueError):
        orc.noise_table_matched_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, 3, -50.0, 1.0,
                                     *w.match_start, w.phi_in)
    with pytest.raises(ValueError):
        orc.noise_table_matched_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, 3, 0.0, 1.0,
                                     *w.match_start, 5.0)


@pytest.mark.parametrize("A", [0.0, 1.3])
def test_switch_off_log_weight_closed_form(orc, A):
    """Exponential potential on its fixed point, time table S = S0 up to the node before
    tau_off and 0 at tau_off (noise and bias switched off after it): ln w = -A sqrt(dN) sum z_n
    - m A^2 dN/2 over the m steps with S(n dN) > 0."""
    alpha, S0, dN = 0.5, 0.05, 1e-3
    n_nodes, tau_off = 11, 0.4137
    S = np.full(n_nodes, S0)
    S[-1] = 0.0
    p = orc.Problem(kind=orc.POT_EXPONENTIAL, V0=1e-10, phi_T=0.0, A_plus=alpha, A_minus=0.0, phi_in=1.0,
                    pi_in=-alpha, phi_end=0.0, S=S, tan_theta=np.zeros(n_nodes), phi_lo=0.0, phi_hi=tau_off,
                    bias_kind=orc.BIAS_CONST if A else orc.BIAS_NONE, A_bias=A, tab_axis=1)
    N, lnw, steps = orc.run(p, dN, 41, 12)
    for i in range(12):
        n = int(steps[i] & orc.STEP_MASK)
        z = orc.normals(41, 0, i, 0, n)
        # the oracle's S(n dN) > 0 exactly for n dN < tau_off: the last interval ramps to 0 at tau_off
        on = np.array([k * dN < tau_off for k in range(n)])
        m = int(on.sum())
        ref = -A * math.sqrt(dN) * z[on].sum() - m * A * A * dN / 2.0
        assert abs(lnw[i] - ref) < 1e-10 * max(1.0, abs(ref))
        assert n * dN > tau_off          # the run outlasts the noise


def test_vanishing_noise_time_axis_equals_phi_axis(orc):
    """The SR -> USR problem with the matched noise scaled by 1e-9: the trajectories stay on the
    classical path, where the time table and the phi table give the same noise."""
    w = W.srusr_matched()
    Sp, tp, _ = orc.noise_table_matched(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, w.table_n,
                                        w.table_lo, w.table_hi, *w.match_start)
    St, tt, _, _ = orc.noise_table_matched_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, 2049, 0.0, 10.5,
                                                *w.match_start, w.phi_in)
    common = dict(kind=w.kind, V0=w.V0, phi_T=w.phi_T, A_plus=w.A_plus, A_minus=w.A_minus, phi_in=w.phi_in,
                  pi_in=w.pi_in, phi_end=w.phi_end, bias_kind=orc.BIAS_CONST, A_bias=1.0)
    pp = orc.Problem(S=Sp * 1e-9, tan_theta=tp, phi_lo=w.table_lo, phi_hi=w.table_hi, **common)
    pt = orc.Problem(S=St * 1e-9, tan_theta=tt, phi_lo=0.0, phi_hi=10.5, tab_axis=1, **common)
    Np, lp, sp, php = orc.run(pp, w.dN, 5, 6, last_phi=True)
    Nt, lt, st = orc.run(pt, w.dN, 5, 6)
    # phi_end sits where the noise-free passage falls on a step boundary (N = 10 at this dN), so a
    # path with vanishing noise ends within ~1e-15 of phi_end and its crossing step is a near-tie
    # (the identity of the crossing step, reading 16): it may move by one step there, N may not
    tie = np.minimum(np.abs(php[:, 0] - w.phi_end), np.abs(php[:, 1] - w.phi_end)) < 1e-12
    same = (sp & orc.STEP_MASK) == (st & orc.STEP_MASK)
    d = (sp & orc.STEP_MASK).astype(np.int64) - (st & orc.STEP_MASK).astype(np.int64)
    assert np.all(same | (tie & (np.abs(d) == 1))) and same.sum() >= 3
    assert np.all((sp & ~np.uint32(orc.STEP_MASK)) == (st & ~np.uint32(orc.STEP_MASK)))
    np.testing.assert_allclose(Nt, Np, rtol=1e-12)
    np.testing.assert_allclose(lt[same], lp[same], rtol=1e-12)


def test_linear_in_time_noise_closed_form(orc):
    """Exponential potential on its fixed point (pi = -alpha stays exact: tan theta = 0), noise
    S(tau) = S0 + S1 tau on a time table (exact under linear interpolation), constant bias A:
    phi_n = phi_in - alpha n dN + sum_{k<n} S(k dN) (A dN + xi_k sqrt(dN)).  The crossing step and
    the interpolated N follow from these sums; a table read at phi instead of at k dN would not."""
    alpha, S0, S1, A, dN = 0.5, 0.02, 0.05, 0.7, 1e-3
    tau_hi, n_nodes = 4.0, 9
    taus = np.linspace(0.0, tau_hi, n_nodes)
    p = orc.Problem(kind=orc.POT_EXPONENTIAL, V0=1e-10, phi_T=0.0, A_plus=alpha, A_minus=0.0, phi_in=1.0,
                    pi_in=-alpha, phi_end=0.0, S=S0 + S1 * taus, tan_theta=np.zeros(n_nodes), phi_lo=0.0,
                    phi_hi=tau_hi, bias_kind=orc.BIAS_CONST, A_bias=A, tab_axis=1)
    N, lnw, steps = orc.run(p, dN, 77, 8)
    for i in range(8):
        n = int(steps[i] & orc.STEP_MASK)
        assert n * dN < tau_hi                     # the whole run lies inside the table
        z = orc.normals(77, 0, i, 0, n)
        k = np.arange(n)
        Sk = S0 + S1 * (k * dN)
        phis = 1.0 + np.concatenate([[0.0], np.cumsum(-alpha * dN + Sk * (A * dN + z * math.sqrt(dN)))])
        assert int(np.argmax(phis <= 0.0)) == n
        N_ref = (n - 1) * dN + dN * phis[n - 1] / (phis[n - 1] - phis[n])
        assert abs(N[i] - N_ref) < 1e-10 * N_ref


def test_bump_time_nodes_equal_phi_nodes(orc):
    """The Gaussian bump: a time node is the phi node at the trajectory's phi there, and the window's
    length in e-folds (from the scipy background) ends at the phi window's lower edge.  On the
    plateau pi ~ 1e-4, so the phi node's root in N carries 1e-16/|pi| ~ 1e-12 e-folds of rounding
    and k = sigma e^N H with it: 1e-10 here (1e-12 on the steeper SR -> USR trajectory)."""
    w = W.gaussian_bump_time()
    for tau in (0.0, 0.7, 2.1, W.BUMP_TAU_HI):
        S, t, fac, ph = orc.noise_table_matched_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, 1, tau, tau,
                                                     *w.match_start, w.phi_in, bump=w.bump)
        Sp, tp, fp = orc.noise_table_matched(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, 1, ph[0], ph[0],
                                             *w.match_start, bump=w.bump)
        np.testing.assert_allclose([S[0], t[0], fac[0]], [Sp[0], tp[0], fp[0]], rtol=1e-10, atol=1e-15)
        if tau == 0.0:
            assert ph[0] == w.phi_in
    assert abs(ph[0] - W.BUMP_PHI_LO) < 1e-12


def test_2d_time_nodes_equal_phi_nodes(orc):
    """2D covariance on time nodes: the phi node at the trajectory's phi there, bit for bit (the
    same covariance routine at the same phi)."""
    w = W.srusr_2d_time()
    taus = np.array([0.0, 0.9, 3.3, 11.0])
    for tau in taus:
        X = orc.noise_table_bessel2d_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.sigma, 1, tau, tau,
                                          *w.match_start, w.phi_in)
        Xp = orc.noise_table_bessel2d(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.sigma, 1, X[3][0], X[3][0])
        assert [X[0][0], X[1][0], X[2][0]] == [Xp[0][0], Xp[1][0], Xp[2][0]]
        if tau == 0.0:
            assert X[3][0] == w.phi_in
    # and its phi nodes are those of the 1D time table (one trajectory, one interpolation)
    S, t, fac, ph = orc.noise_table_matched_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, 4, 0.5, 9.5,
                                                 *w.match_start, w.phi_in)
    X = orc.noise_table_bessel2d_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.sigma, 4, 0.5, 9.5,
                                      *w.match_start, w.phi_in)
    assert np.array_equal(X[3], ph)
    with pytest.raises(ValueError):
        orc.noise_table_bessel2d_time(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, w.sigma, 3, -50.0, 1.0,
                                      *w.match_start, w.phi_in)


@pytest.mark.parametrize("A", [0.0, 1.1])
def test_2d_switch_off_log_weight_closed_form(orc, A):
    """Exponential potential, constant diagonal 2D noise Xi = diag(a, c) (a > c: principal axis (1, 0)
    at every node, the zero node included) up to tau_off, zero there: dA = A xi_1 sqrt(dN) + A^2 dN/2
    on exactly the steps with n dN < tau_off, whatever the path; the noise moves pi, so a table read
    at phi would switch off elsewhere."""
    alpha, dN, n_nodes, tau_off = 0.5, 1e-3, 9, 0.3217
    a, c = 0.04 ** 2, 0.01 ** 2
    Xpp, Xpq, Xqq = np.full(n_nodes, a), np.zeros(n_nodes), np.full(n_nodes, c)
    Xpp[-1] = Xqq[-1] = 0.0
    p = orc.Problem2D(kind=orc.POT_EXPONENTIAL, V0=1e-10, phi_T=0.0, A_plus=alpha, A_minus=0.0, phi_in=1.0,
                      pi_in=-alpha, phi_end=0.0, Xpp=Xpp, Xpq=Xpq, Xqq=Xqq, phi_lo=0.0, phi_hi=tau_off,
                      bias_kind=orc.BIAS_CONST if A else orc.BIAS_NONE, A_bias=A, tab_axis=1)
    N, lnw, steps = orc.run2d(p, dN, 29, 10)
    for i in range(10):
        n = int(steps[i] & orc.STEP_MASK)
        assert n * dN > tau_off
        z = orc.normals2d(29, 0, i, 0, n)          # (n, 2)
        on = np.array([k * dN < tau_off for k in range(n)])
        m = int(on.sum())
        ref = -A * math.sqrt(dN) * z[on, 0].sum() - m * A * A * dN / 2.0
        assert abs(lnw[i] - ref) < 1e-10 * max(1.0, abs(ref)), (i, lnw[i], ref)
