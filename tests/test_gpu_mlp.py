"""GPU parity of the learned importance-sampling control through the C ABI.

The control is the 2->64->64->2 network tabulated on a grid of its normalised
inputs and interpolated bilinearly.  Checked against the CPU oracle: the
tabulated node values; FP64-state trajectories with the control (per
trajectory, as for the constant bias); the FP32-state path on coupled streams;
the replay gradient of the tail second moment J = E[w^2 1_T] with its grid-node
weights; the Adam step; and training, which must lower J and keep the tail
estimate unbiased against the inverse-Gaussian closed form.
"""
import math
import sys

import numpy as np
import pytest
from scipy import special

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as orc  # noqa: E402
from paper_2410_13683_amd import fpt  # noqa: E402
from paper_2410_13683_amd import workloads as W  # noqa: E402
from tests._glue import assert_fp64_parity, oracle_problem, oracle_run  # noqa: E402
from tests._gpu import gpu_context, gpu_run  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ig(n=3000, seed=29, params=None, dN=2e-3):
    return W.exponential_ig_learned(n_traj=n, seed=seed, dN=dN,
                                    params=W.mlp_random(1) if params is None else params)


def _srusr(n, seed, params, precision=0):
    return W.srusr_learned(n_traj=n, seed=seed).with_(mlp_params=params, precision=precision)


def _tail_lo_in_gap(N, N_ref, q):
    """A threshold near the q-quantile of deltaN that sits in the middle of the widest gap
    between neighbouring samples there, so rounding-level changes of N cannot move a path
    across it."""
    d = np.sort(N - N_ref)
    i0 = int(q * len(d))
    lo, hi = max(i0 - 20, 0), min(i0 + 20, len(d) - 1)
    gaps = np.diff(d[lo:hi + 1])
    k = int(np.argmax(gaps))
    return 0.5 * (d[lo + k] + d[lo + k + 1]), gaps[k]


def test_tabulation_matches_oracle():
    p = W.mlp_random(3)
    w = _ig(params=p)
    say(f"tabulation {w.grid_n}")
    ctx = gpu_context(w)
    np.testing.assert_allclose(ctx.mlp_table(), orc.mlp_tabulate(p, w.grid_n, w.grid_range), rtol=1e-13,
                               atol=1e-15)
    p2 = W.mlp_random(4)
    ctx.mlp_set(p2)
    np.testing.assert_allclose(ctx.mlp_table(), orc.mlp_tabulate(p2, w.grid_n, w.grid_range), rtol=1e-13,
                               atol=1e-15)
    assert np.array_equal(ctx.mlp_get(), p2)
    # device-resident parameters
    p3 = torch.from_numpy(W.mlp_random(5)).cuda()
    ctx.mlp_set(p3)
    torch.cuda.synchronize()
    assert np.array_equal(ctx.mlp_get(), p3.cpu().numpy())
    ctx.destroy()


def test_fp64_learned_control_ig_parity():
    """3000 trajectories (46 waves and a ragged tail) of the inverse-Gaussian companion with a
    random network as the control: per-trajectory parity with the oracle."""
    w = _ig(n=3000)
    say(f"fp64 learned ig n={w.n_traj}")
    gpu, hist = gpu_run(w)
    ora = oracle_run(w, last_phi=True)
    assert_fp64_parity(gpu, ora, w)
    assert np.std(gpu[1]) > 0.1          # the control varies: log-weights are not trivial


def test_fp64_learned_control_srusr_parity():
    """The SR -> USR problem (Bessel noise table, two-branch potential) with a random network as
    the control, FP64 state, 1500 trajectories: per-trajectory parity with the oracle."""
    w = _srusr(1500, 41, W.mlp_random(7, scale=0.2, out_bias=1.0))
    say(f"fp64 learned srusr n={w.n_traj}")
    gpu, _ = gpu_run(w)
    ora = oracle_run(w, last_phi=True)
    assert_fp64_parity(gpu, ora, w)


@pytest.mark.parametrize("precision", [0, 1])
def test_constant_network_equals_constant_bias(precision):
    """W3 = 0, b3 = (A, 0): the tabulated control is exactly A, so every trajectory equals the
    constant-bias one: in FP64 up to summation order; in FP32 up to rounding, because the
    constant bias rides in each step's normal (z = xi sqrt(dN) + A dN) while the learned one is
    added to the phi increment, so the two round differently (8.9e-8 relative in N at most on
    these 4000 paths; the bar is 2e-6)."""
    A = 1.5
    w = _srusr(4000, 43, W.mlp_constant_init(A, seed=2), precision=precision)
    wc = w.with_(bias_kind=W.BIAS_CONST, A_bias=A, mlp_params=None)
    say(f"constant network vs constant bias, precision {precision}")
    (Nm, lm, sm), _ = gpu_run(w)
    (Nc, lc, sc), _ = gpu_run(wc)
    assert np.mean(sm == sc) > 0.999
    same = sm == sc
    np.testing.assert_allclose(Nm[same], Nc[same], rtol=1e-12 if precision == 0 else 2e-6)
    tol = 1e-10 if precision == 0 else 2e-5
    assert np.all(np.abs(lm[same] - lc[same]) <= tol * (1.0 + np.abs(lc[same])))


def _ks(a, b):
    xs = np.sort(np.concatenate([a, b]))
    fa = np.searchsorted(np.sort(a), xs, side="right") / len(a)
    fb = np.searchsorted(np.sort(b), xs, side="right") / len(b)
    return np.max(np.abs(fa - fb))


def test_fp32_learned_control_coupled_with_fp64():
    """FP32 state vs FP64 state with the same learned control on the same random streams
    (2e4 SR -> USR trajectories): per-trajectory agreement up to FP32 rounding and KS below 1e-3."""
    p = W.mlp_random(8, scale=0.2, out_bias=1.5)
    w = _srusr(20_000, 44, p)
    say("fp32 vs fp64 learned control, n=2e4")
    (N64, l64, s64), _ = gpu_run(w)
    (N32, l32, s32), _ = gpu_run(w.with_(precision=1))
    flags = orc.FLAG_CENSORED | orc.FLAG_ENDED_EARLY
    assert np.all((s64 & flags) == 0) and np.all((s32 & flags) == 0)
    dn = N32 - N64
    say(f"  N32 - N64: median {np.median(dn):.3e}, max |.| {np.abs(dn).max():.3e}")
    assert abs(np.median(dn)) < 2e-5 and np.mean(np.abs(dn) < 1e-4) > 0.99
    ks = _ks(N32, N64)
    same = s32 == s64
    dl = np.abs(l32 - l64)[same]
    say(f"  KS {ks:.2e}; same step {same.mean():.4f}; |dlnw| median {np.median(dl):.2e} max {dl.max():.2e}")
    assert ks < 1e-3 and same.mean() > 0.95 and np.median(dl) < 1e-5 and dl.max() < 1e-3


def _grad_case(w, q=0.8):
    N, lnw, st = oracle_run(w)
    tail_lo, gap = _tail_lo_in_gap(N, w.N_ref, q)
    theta = np.ascontiguousarray(w.mlp_params, dtype=np.float32)
    prob = oracle_problem(w)
    grad_o, J_o, G_o = orc.grid_replay_grad(prob, theta, theta, w.dN, w.seed, w.n_traj, w.N_ref, tail_lo)
    n_tail_o = int(np.sum(((st & (orc.FLAG_CENSORED | orc.FLAG_ENDED_EARLY)) == 0) & (N - w.N_ref >= tail_lo)))
    ctx = gpu_context(w)
    d_grad = torch.zeros(fpt.FPT_MLP_NPARAM, dtype=torch.float32, device="cuda")
    d_G = torch.zeros(w.grid_n[0] * w.grid_n[1], dtype=torch.float64, device="cuda")
    J, n_tail = ctx.mlp_grad(w.n_traj, w.dN, w.seed, tail_lo, d_grad, d_G=d_G)
    torch.cuda.synchronize()
    g_plain = d_grad.cpu().numpy().astype(np.float64)
    # the log objective divides by J on the device
    ctx.mlp_grad(w.n_traj, w.dN, w.seed, tail_lo, d_grad, objective=fpt.FPT_MLP_OBJ_LOG_J, want_J=False)
    g_log = d_grad.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(g_log, g_plain / J, rtol=1e-5, atol=1e-6 * np.abs(g_plain).max() / J)
    out = dict(J=J, n_tail=n_tail, grad=g_plain,
               G=d_G.cpu().numpy().reshape(w.grid_n), J_o=J_o, n_tail_o=n_tail_o, grad_o=grad_o, G_o=G_o,
               gap=gap)
    # the context's histogram is not touched by gradient runs
    assert ctx.histogram()["n_traj"] == 0
    ctx.destroy()
    return out


def test_gradient_matches_oracle_fp64():
    """Replay gradient on 4000 inverse-Gaussian paths with a random control, FP64 state: J, the
    tail count, the grid-node weights G and dJ/dtheta against the oracle."""
    w = _ig(n=4000, params=W.mlp_random(9, scale=0.2, out_bias=1.0))
    say("gradient fp64 (ig, n=4000)")
    r = _grad_case(w)
    say(f"  J {r['J']:.6e} vs {r['J_o']:.6e}; tail {r['n_tail']} vs {r['n_tail_o']}")
    assert r["n_tail"] == r["n_tail_o"] and r["n_tail"] > 100
    assert math.isclose(r["J"], r["J_o"], rel_tol=1e-9)
    Gm = np.abs(r["G_o"]).max()
    np.testing.assert_allclose(r["G"], r["G_o"], rtol=1e-9, atol=1e-12 * Gm)
    gm = np.abs(r["grad_o"]).max()
    np.testing.assert_allclose(r["grad"], r["grad_o"], rtol=1e-5, atol=1e-6 * gm)
    assert np.count_nonzero(r["grad_o"][:4480]) > 4000     # every layer receives gradient


def test_gradient_matches_oracle_fp64_srusr():
    """The same on 800 SR -> USR paths (table noise, two branches, pi varying over decades)."""
    w = _srusr(800, 45, W.mlp_random(10, scale=0.2, out_bias=1.0))
    say("gradient fp64 (srusr, n=800)")
    r = _grad_case(w, q=0.7)
    say(f"  J {r['J']:.6e} vs {r['J_o']:.6e}; tail {r['n_tail']} vs {r['n_tail_o']}")
    assert r["n_tail"] == r["n_tail_o"] and r["n_tail"] > 100
    assert math.isclose(r["J"], r["J_o"], rel_tol=1e-9)
    np.testing.assert_allclose(r["G"], r["G_o"], rtol=1e-8, atol=1e-11 * np.abs(r["G_o"]).max())
    np.testing.assert_allclose(r["grad"], r["grad_o"], rtol=1e-5, atol=1e-6 * np.abs(r["grad_o"]).max())


def test_gradient_fp32_state_within_1e3():
    """FP32-state replay gradient against the FP64 oracle on the same streams (800 SR -> USR
    paths): J and dJ/dtheta within 1e-3 relative (vector norm)."""
    w = _srusr(800, 46, W.mlp_random(11, scale=0.2, out_bias=1.0), precision=1)
    say("gradient fp32 (srusr, n=800)")
    r = _grad_case(w.with_(precision=0), q=0.7)            # oracle reference and its threshold
    N, _, _ = oracle_run(w)
    tail_lo, _ = _tail_lo_in_gap(N, w.N_ref, 0.7)
    ctx = gpu_context(w)
    d_grad = torch.zeros(fpt.FPT_MLP_NPARAM, dtype=torch.float32, device="cuda")
    J, n_tail = ctx.mlp_grad(w.n_traj, w.dN, w.seed, tail_lo, d_grad)
    g = d_grad.cpu().numpy().astype(np.float64)
    ctx.destroy()
    rel_g = np.linalg.norm(g - r["grad_o"]) / np.linalg.norm(r["grad_o"])
    say(f"  J {J:.6e} vs {r['J_o']:.6e}; tail {n_tail} vs {r['n_tail_o']}; |dg|/|g| {rel_g:.2e}")
    assert abs(J / r["J_o"] - 1.0) < 1e-3 and rel_g < 1e-3


def test_adam_matches_oracle():
    w = _ig(params=W.mlp_random(12))
    ctx = gpu_context(w)
    th = np.ascontiguousarray(w.mlp_params, dtype=np.float32).copy()
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    rng = np.random.default_rng(13)
    for t in (1, 2, 3):
        g = (rng.standard_normal(th.size) * 10.0 ** rng.uniform(-5, 1, th.size)).astype(np.float32)
        ctx.mlp_adam(torch.from_numpy(g).cuda(), 3e-3, 0.9, 0.999, 1e-8)
        orc.adam_step(th, m, v, g, t, 3e-3, 0.9, 0.999, 1e-8)
        got = ctx.mlp_get()
        ulp = np.spacing(np.abs(th).astype(np.float32))
        assert np.all(np.abs(got - th) <= ulp), np.max(np.abs(got - th) / ulp)
    # the table follows the parameters
    np.testing.assert_allclose(ctx.mlp_table(), orc.mlp_tabulate(ctx.mlp_get(), w.grid_n, w.grid_range),
                               rtol=1e-13, atol=1e-15)
    ctx.destroy()


def _ig_sf(x, mu, lam):
    """P(N > x) of the inverse-Gaussian law (erfcx form, finite far in the tail)."""
    A = math.sqrt(lam / x) * (x / mu - 1.0)
    B = math.sqrt(lam / x) * (x / mu + 1.0)
    return 0.5 * math.exp(-A * A / 2.0) * (special.erfcx(A / math.sqrt(2)) - special.erfcx(B / math.sqrt(2)))


def test_training_lowers_tail_second_moment_and_stays_unbiased():
    """Inverse-Gaussian companion, tail T = {deltaN >= 5 sigma_N}: start from the constant
    control a = 1 (too weak for this tail), take Adam steps on the replay gradient, and compare
    the tail second moment J and the estimate of P_T before and after on fresh trajectories.
    Training must lower J by a large factor (17x measured; the bar is 8x) and both estimates must
    match the closed form."""
    w = _ig(n=100_000, seed=50, params=W.mlp_constant_init(1.0, seed=3), dN=1e-4)
    mu = (w.phi_in - w.phi_end) / w.A_plus
    lam = (w.phi_in - w.phi_end) ** 2 / w.noise_S ** 2
    tail_lo = 5.0 * math.sqrt(mu ** 3 / lam)
    exact = _ig_sf(mu + tail_lo, mu, lam)
    ctx = gpu_context(w)
    d_grad = torch.zeros(fpt.FPT_MLP_NPARAM, dtype=torch.float32, device="cuda")
    n_eval = 1_000_000

    def evaluate(seed):
        ctx.reset()
        N = torch.empty(n_eval, dtype=torch.float64, device="cuda")
        lnw = torch.empty(n_eval, dtype=torch.float64, device="cuda")
        ctx.run(n_eval, w.dN, seed, 0, None, N, lnw, None)
        torch.cuda.synchronize()
        N, lnw = N.cpu().numpy(), lnw.cpu().numpy()
        wt = np.exp(lnw) * ((N - w.N_ref) >= tail_lo)
        return wt.mean(), wt.std() / math.sqrt(n_eval), np.mean(wt * wt)

    p0, se0, J0 = evaluate(1001)
    say(f"  before: P_T {p0:.4e} +- {se0:.1e} (exact {exact:.4e}), J {J0:.3e}")
    for it in range(40):
        J, n_tail = ctx.mlp_grad(w.n_traj, w.dN, 5000 + it, tail_lo, d_grad)
        ctx.mlp_adam(d_grad, 0.05)
        if it % 10 == 0:
            say(f"  iter {it}: J {J:.3e} tail paths {n_tail}")
    p1, se1, J1 = evaluate(1002)
    say(f"  after:  P_T {p1:.4e} +- {se1:.1e}, J {J1:.3e}; J ratio {J0 / J1:.1f}")
    ctx.destroy()
    for p, se in ((p0, se0), (p1, se1)):
        assert abs(p / exact - 1.0) < 0.05 + 4 * se / exact
    assert J1 < J0 / 8.0


# ---- the network evaluated in the step (mlp_every = k >= 1) ------------------------------------

def _exact_problem(w, k):
    p = oracle_problem(w, mlp_params=np.ascontiguousarray(w.mlp_params, dtype=np.float32),
                       mlp_norm=np.asarray(w.mlp_norm, dtype=np.float64))
    p.mlp_every = k
    return p


@pytest.mark.parametrize("k", [1, 7, 16])
def test_exact_network_every_k_steps_fp64_parity(k):
    """The network itself every k steps in FP64 state (the amplitude held in between, evaluated at
    the state of step k floor(n/k)) on 2000 inverse-Gaussian paths with a random network: per
    trajectory against the oracle's own network every k steps (N within 1e-9, the same crossing
    step, ln w within 1e-9).  k = 7 does not divide the launch's chunk of 128 steps, so the lanes
    of a wave evaluate at different steps."""
    w = _ig(n=2000, seed=33, params=W.mlp_random(13, scale=0.2, out_bias=1.0))
    say(f"exact network every {k} steps, fp64 ig n={w.n_traj}")
    gpu, _ = gpu_run(w, mlp_every=k)
    ora = orc.run(_exact_problem(w, k), w.dN, w.seed, w.n_traj, last_phi=True)
    assert np.std(gpu[1]) > 0.05                      # the network varies along the paths
    assert_fp64_parity(gpu, ora, w)
    # and it differs from the tabulated control: the network is not constant
    tab, _ = gpu_run(w)
    assert np.mean(np.abs(tab[1] - gpu[1]) > 1e-6) > 0.5


def test_exact_network_srusr_fp64_parity_and_fp32_coupled():
    """The SR -> USR problem (table noise, two branches, pi over decades) with the network every 8
    steps: FP64 state per trajectory against the oracle (800 paths), and FP32 state (its network
    in FP32) coupled with the oracle on the same streams: N within FP32 rounding except at near-ties,
    ln w where the crossing steps agree."""
    w = _srusr(800, 47, W.mlp_random(14, scale=0.2, out_bias=1.0))
    p = _exact_problem(w, 8)
    say(f"exact network every 8 steps, srusr n={w.n_traj}")
    gpu, _ = gpu_run(w, mlp_every=8)
    ora = orc.run(p, w.dN, w.seed, w.n_traj, last_phi=True)
    assert_fp64_parity(gpu, ora, w)
    (N32, l32, s32), _ = gpu_run(w.with_(precision=1), mlp_every=8)
    dn = np.abs(N32 - ora[0])
    same = s32 == ora[2]
    dl = np.abs(l32 - ora[1])[same]
    say(f"  fp32: |dN| median {np.median(dn):.2e} max {dn.max():.2e}; same step {same.mean():.4f}; "
        f"|dlnw| median {np.median(dl):.2e} max {dl.max():.2e}")
    assert np.mean(dn < 1e-4) > 0.98 and same.mean() > 0.95 and np.median(dl) < 1e-5 and dl.max() < 1e-3


def test_exact_network_context_rejects_the_gradient():
    w = _ig(n=100, params=W.mlp_random(15))
    ctx = gpu_context(w, mlp_every=4)
    d_grad = torch.zeros(fpt.FPT_MLP_NPARAM, dtype=torch.float32, device="cuda")
    with pytest.raises(fpt.FptError):
        ctx.mlp_grad(w.n_traj, w.dN, w.seed, 0.0, d_grad)
    ctx.destroy()
