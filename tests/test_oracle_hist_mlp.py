"""Pins of the oracle's histogram (against numpy.histogram) and of its learned-bias
network and replay gradient (against a numpy forward pass, the constant-bias
path, and central finite differences of the objective)."""
import math

import numpy as np
import pytest

from paper_2410_13683_amd import workloads as W
from tests._glue import oracle_problem, oracle_run


@pytest.mark.parametrize("kind", [0, 1])
def test_histogram_matches_numpy(orc, kind):
    rng = np.random.default_rng(3)
    n_bins, lo, hi = 37, 0.013, 0.171
    x = rng.uniform(-0.01, 0.2, 200_000)
    lnw = rng.normal(-3, 2, x.size)
    N_ref = 10.0
    N = x + N_ref
    steps = np.full(x.size, 5, dtype=np.uint32)
    h = orc.histogram(N, lnw, steps, N_ref, kind, n_bins, lo, hi)
    edges = orc.bin_edges(kind, n_bins, lo, hi)
    xin = N - N_ref
    inside = (xin >= lo) & (xin < hi)
    c, _ = np.histogram(xin[inside], bins=edges)
    sw, _ = np.histogram(xin[inside], bins=edges, weights=np.exp(lnw[inside]))
    sl2, _ = np.histogram(xin[inside], bins=edges, weights=lnw[inside] ** 2)
    assert np.array_equal(h["count"][1:-1], c.astype(np.uint64))
    np.testing.assert_allclose(h["sum_w"][1:-1], sw, rtol=1e-12)
    np.testing.assert_allclose(h["sum_lnw2"][1:-1], sl2, rtol=1e-12)
    assert h["count"][0] == np.count_nonzero(xin < lo)
    assert h["count"][-1] == np.count_nonzero(xin >= hi)


def test_histogram_flags_and_totals(orc):
    N = np.array([10.01, np.nan, 10.5, 10.02])
    lnw = np.array([0.1, 0.0, -0.2, 0.3])
    steps = np.array([100, 50 | orc.FLAG_CENSORED, 7 | orc.FLAG_ENDED_EARLY, 101], dtype=np.uint32)
    h = orc.histogram(N, lnw, steps, 10.0, 0, 4, 0.0, 0.04)
    assert h["n_traj"] == 4 and h["n_censored"] == 1 and h["n_ended_early"] == 1
    assert h["n_steps_total"] == 100 + 50 + 7 + 101
    assert int(h["count"].sum()) == 2
    assert math.isclose(h["sum_w_total"], math.exp(0.1) + math.exp(0.3))


# --------------------------------------------------------------------------
# learned bias
# --------------------------------------------------------------------------
def _random_params(rng, scale=0.3, out_bias=1.0):
    p = (rng.standard_normal(4482) * scale).astype(np.float32)
    p[4480] = out_bias       # b3[0]
    return p


def _numpy_mlp(p, x):
    W1 = p[:128].reshape(64, 2).astype(np.float64)
    b1 = p[128:192].astype(np.float64)
    W2 = p[192:4288].reshape(64, 64).astype(np.float64)
    b2 = p[4288:4352].astype(np.float64)
    W3 = p[4352:4480].reshape(2, 64).astype(np.float64)
    b3 = p[4480:4482].astype(np.float64)
    h1 = np.tanh(W1 @ x + b1)
    h2 = np.tanh(W2 @ h1 + b2)
    return W3 @ h2 + b3


def test_mlp_forward_matches_numpy(orc):
    rng = np.random.default_rng(0)
    p = _random_params(rng)
    norm = np.array([0.01, 0.02, -5.0, 2.0])
    for phi, pi_ in [(0.0, -0.1), (-0.03, -1e-4), (0.02, 0.05), (0.001, 0.0)]:
        x = np.array([(phi - norm[0]) / norm[1], (math.log(max(abs(pi_), 1e-30)) - norm[2]) / norm[3]])
        ref = _numpy_mlp(p, x)[0]
        assert math.isclose(orc.mlp_eval(p, norm, phi, pi_), ref, rel_tol=1e-12, abs_tol=1e-14)


def test_constant_network_reproduces_constant_bias(orc):
    """W3 = 0, b3 = (A, 0): the learned amplitude is exactly A, so every trajectory equals the
    constant-bias one."""
    rng = np.random.default_rng(1)
    p = _random_params(rng)
    p[4352:4480] = 0.0
    A = 1.5
    p[4480] = A
    w = W.linear_slow_roll(n_traj=64).with_(bias_kind=W.BIAS_CONST, A_bias=A)
    Nc, lc, sc = oracle_run(w)
    wm = w.with_(bias_kind=W.BIAS_MLP)
    Nm, lm, sm = oracle_run(wm, mlp_params=p, mlp_norm=np.array([0.5, 0.5, -2.0, 1.0]))
    assert np.array_equal(sc, sm)
    assert np.array_equal(Nc, Nm)
    assert np.array_equal(lc, lm)


def _mlp_problem():
    w = W.exponential_ig(n_traj=96, dN=2e-3, seed=29).with_(bias_kind=W.BIAS_MLP)
    norm = np.array([0.5, 0.5, math.log(0.5), 1.0])
    return w, norm


def test_replay_objective_matches_forward_weights(orc):
    """At theta = theta_old the replayed objective is (1/n) sum_T w^2 of the forward run."""
    rng = np.random.default_rng(2)
    theta = _random_params(rng, scale=0.2, out_bias=1.0)
    w, norm = _mlp_problem()
    prob = oracle_problem(w, mlp_params=theta, mlp_norm=norm)
    N, lnw, steps = orc.run(prob, w.dN, w.seed, w.n_traj)
    tail_lo = 0.05
    T = (N - w.N_ref) >= tail_lo
    J_fwd = np.sum(np.exp(2 * lnw[T])) / w.n_traj
    grad, J = orc.mlp_replay_grad(prob, theta, theta, w.dN, w.seed, w.n_traj, w.N_ref, tail_lo)
    assert T.sum() > 5
    assert math.isclose(J, J_fwd, rel_tol=1e-10)
    assert np.all(np.isfinite(grad))


def test_replay_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(4)
    theta_old = _random_params(rng, scale=0.2, out_bias=1.0)
    theta = theta_old.copy()
    theta[4480] += np.float32(0.25)        # evaluate away from theta_old
    w, norm = _mlp_problem()
    prob = oracle_problem(w, mlp_params=theta_old, mlp_norm=norm)
    tail_lo = 0.0
    grad, J = orc.mlp_replay_grad(prob, theta_old, theta, w.dN, w.seed, w.n_traj, w.N_ref, tail_lo)
    for k in [4480, 4352 + 5, 4288 + 7, 192 + 64 * 3 + 11, 128 + 9, 2 * 17 + 1]:
        h = np.float32(1e-2) if k >= 4352 else np.float32(2e-2)
        tp = theta.copy(); tp[k] += h
        tm = theta.copy(); tm[k] -= h
        hp = float(tp[k]) - float(theta[k])
        hm = float(theta[k]) - float(tm[k])
        _, Jp = orc.mlp_replay_grad(prob, theta_old, tp, w.dN, w.seed, w.n_traj, w.N_ref, tail_lo)
        _, Jm = orc.mlp_replay_grad(prob, theta_old, tm, w.dN, w.seed, w.n_traj, w.N_ref, tail_lo)
        fd = (Jp - Jm) / (hp + hm)
        assert abs(fd - grad[k]) <= 2e-3 * abs(grad[k]) + 1e-6 * abs(J), (k, fd, grad[k])


# --------------------------------------------------------------------------
# tabulated learned control
# --------------------------------------------------------------------------
GRID_N = (24, 12)
GRID_RANGE = (-0.2, 1.2, -1.5, 1.5)


def test_tabulation_matches_numpy(orc):
    rng = np.random.default_rng(7)
    p = _random_params(rng)
    a = orc.mlp_tabulate(p, GRID_N, GRID_RANGE)
    x0 = np.linspace(GRID_RANGE[0], GRID_RANGE[1], GRID_N[0])
    x1 = np.linspace(GRID_RANGE[2], GRID_RANGE[3], GRID_N[1])
    for i in (0, 5, GRID_N[0] - 1):
        for j in (0, 7, GRID_N[1] - 1):
            assert math.isclose(a[i, j], _numpy_mlp(p, np.array([x0[i], x1[j]]))[0], rel_tol=1e-12, abs_tol=1e-14)


def test_tabulated_constant_network_is_the_constant_bias(orc):
    rng = np.random.default_rng(8)
    p = _random_params(rng)
    p[4352:4480] = 0.0
    p[4480] = 1.25
    w = W.linear_slow_roll(n_traj=48).with_(bias_kind=W.BIAS_CONST, A_bias=1.25)
    Nc, lc, sc = oracle_run(w)
    prob = oracle_problem(w.with_(bias_kind=W.BIAS_MLP), mlp_params=p, mlp_norm=np.array([0.5, 0.5, -2.0, 1.0]))
    for every in (0, 1, 5):
        prob.mlp_every = every
        prob.grid_n, prob.grid_range = GRID_N, GRID_RANGE
        Nm, lm, sm = orc.run(prob, w.dN, w.seed, w.n_traj)
        assert np.array_equal(sc, sm)
        np.testing.assert_allclose(Nm, Nc, rtol=1e-13)
        np.testing.assert_allclose(lm, lc, rtol=1e-12, atol=1e-12)


def _grid_problem(theta):
    w, norm = _mlp_problem()
    prob = oracle_problem(w, mlp_params=theta, mlp_norm=norm)
    prob.mlp_every = 0
    prob.grid_n, prob.grid_range = GRID_N, GRID_RANGE
    return w, prob


def test_grid_replay_objective_matches_forward_weights(orc):
    rng = np.random.default_rng(12)
    theta = _random_params(rng, scale=0.2, out_bias=1.0)
    w, prob = _grid_problem(theta)
    N, lnw, steps = orc.run(prob, w.dN, w.seed, w.n_traj)
    tail_lo = 0.05
    T = (N - w.N_ref) >= tail_lo
    J_fwd = np.sum(np.exp(2 * lnw[T])) / w.n_traj
    grad, J, G = orc.grid_replay_grad(prob, theta, theta, w.dN, w.seed, w.n_traj, w.N_ref, tail_lo)
    assert T.sum() > 5
    assert math.isclose(J, J_fwd, rel_tol=1e-10)
    assert np.count_nonzero(G) > 4 and np.all(np.isfinite(grad))


def test_grid_replay_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(13)
    theta_old = _random_params(rng, scale=0.2, out_bias=1.0)
    theta = theta_old.copy()
    theta[4480] += np.float32(0.2)
    w, prob = _grid_problem(theta_old)
    tail_lo = 0.0
    grad, J, _ = orc.grid_replay_grad(prob, theta_old, theta, w.dN, w.seed, w.n_traj, w.N_ref, tail_lo)
    for k in [4480, 4352 + 9, 4288 + 3, 192 + 64 * 5 + 17, 128 + 30, 2 * 40 + 1]:
        h = np.float32(1e-2) if k >= 4352 else np.float32(2e-2)
        tp = theta.copy(); tp[k] += h
        tm = theta.copy(); tm[k] -= h
        _, Jp, _ = orc.grid_replay_grad(prob, theta_old, tp, w.dN, w.seed, w.n_traj, w.N_ref, tail_lo)
        _, Jm, _ = orc.grid_replay_grad(prob, theta_old, tm, w.dN, w.seed, w.n_traj, w.N_ref, tail_lo)
        fd = (Jp - Jm) / ((float(tp[k]) - float(theta[k])) + (float(theta[k]) - float(tm[k])))
        assert abs(fd - grad[k]) <= 2e-3 * abs(grad[k]) + 1e-6 * abs(J), (k, fd, grad[k])


# --------------------------------------------------------------------------
# Adam
# --------------------------------------------------------------------------
def test_adam_first_step_is_the_signed_learning_rate(orc):
    """From zero moments the bias-corrected first step is lr g / (|g| + eps) against the gradient."""
    rng = np.random.default_rng(21)
    g = (rng.standard_normal(50) * 10.0 ** rng.uniform(-4, 2, 50)).astype(np.float32)
    th0 = rng.standard_normal(50).astype(np.float32)
    th, m, v = th0.copy(), np.zeros(50, np.float32), np.zeros(50, np.float32)
    lr, eps = 1e-2, 1e-8
    orc.adam_step(th, m, v, g, 1, lr, 0.9, 0.999, eps)
    gd = g.astype(np.float64)
    expect = th0.astype(np.float64) - lr * gd / (np.abs(gd) + eps)
    np.testing.assert_allclose(th, expect.astype(np.float32), rtol=2e-7, atol=1e-9)
    np.testing.assert_allclose(m, (0.1 * gd).astype(np.float32), rtol=1e-6)
    np.testing.assert_allclose(v, (0.001 * gd * gd).astype(np.float32), rtol=1e-6)


def test_adam_constant_gradient_moves_linearly(orc):
    """A constant gradient keeps the bias-corrected moments at g and g^2, so after t steps the
    parameter has moved by t lr g/(|g| + eps); a zero gradient afterwards only decays m and v."""
    g = np.array([3.0, -0.5, 1e-3, -20.0], dtype=np.float32)
    th = np.zeros(4, np.float32)
    m, v = np.zeros(4, np.float32), np.zeros(4, np.float32)
    lr, eps, T = 1e-3, 1e-8, 40
    for t in range(1, T + 1):
        orc.adam_step(th, m, v, g, t, lr, 0.8, 0.99, eps)
    gd = g.astype(np.float64)
    np.testing.assert_allclose(th, -T * lr * gd / (np.abs(gd) + eps), rtol=2e-5)
    m0, v0 = m.copy(), v.copy()
    th_before = th.copy()
    orc.adam_step(th, m, v, np.zeros(4, np.float32), T + 1, lr, 0.8, 0.99, eps)
    np.testing.assert_allclose(m, 0.8 * m0.astype(np.float64), rtol=1e-6)
    np.testing.assert_allclose(v, 0.99 * v0.astype(np.float64), rtol=1e-6)
    assert np.all(np.sign(th - th_before) == -np.sign(gd))      # momentum keeps moving downhill
