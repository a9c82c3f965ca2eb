"""GPU parity of the Bessel-matched noise table (Sec. 3.4) against the CPU oracle
through the C ABI.  Cases:
- the SR -> USR table on the full 4096-node grid, at sigma = 1 and 0.1;
- a sudden kink in near de Sitter, also checked against its closed form;
- power-law inflation (exponential potential);
- single nodes at and around the transition, and nodes the trajectory never reaches;
- the late-start error;
- FP64 trajectories on the matched table: per-trajectory parity with the oracle
  driven by its own table.
FP32 trajectories are checked on the matched table too: the mean and spread of
the passage time against the FP64 run."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as orc  # noqa: E402
from paper_2410_13683_amd import fpt  # noqa: E402
from paper_2410_13683_amd import workloads as W  # noqa: E402
from tests._glue import assert_fp64_parity, oracle_run  # noqa: E402
from tests._gpu import gpu_run  # noqa: E402

# near de Sitter piecewise-linear potential: eps_+ = 1e-8, A_- = A_+/10
V0 = 1e-10
AP = V0 * math.sqrt(2e-8)
AM = 0.1 * AP
PI_T = -AP / V0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _both(kind, V0_, phi_T, Ap, Am, sigma, n, lo, hi, phi_start, pi_start):
    pot = fpt.make_potential(kind, V0_, phi_T, Ap, Am, 0.0, 0.0, -1.0)
    g = fpt.fpt_noise_table_matched(pot, sigma, n, lo, hi, phi_start, pi_start)
    o = orc.noise_table_matched(kind, V0_, phi_T, Ap, Am, sigma, n, lo, hi, phi_start, pi_start)
    return g, o


def _assert_tables_close(g, o, rtol=1e-9):
    S, t, fac = g
    So, to, faco = o
    np.testing.assert_allclose(fac, faco, rtol=rtol, atol=0)
    np.testing.assert_allclose(S, So, rtol=rtol, atol=0)
    np.testing.assert_allclose(t, to, rtol=0, atol=1e-14)


@pytest.mark.parametrize("sigma", [1.0, 0.1])
def test_srusr_matched_table_matches_oracle(sigma):
    w = W.srusr_matched(sigma=sigma)
    say(f"matched table srusr sigma={sigma}")
    phi_start, pi_start = w.match_start
    if sigma == 0.1:
        phi_start = 1.5     # ln(100/0.1) = 6.9 e-folds before the highest node
        pi_start = -w.A_plus / (w.V0 + w.A_plus * phi_start)
    g, o = _both(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, sigma, w.table_n, w.table_lo, w.table_hi,
                 phi_start, pi_start)
    _assert_tables_close(g, o)
    # the transition changes the noise.  sigma = 1: factors from ~0.1 to ~2.6 after it.  sigma = 0.1:
    # the modes matched in ultra-slow roll left the Hubble radius before the transition, and their
    # dphi falls with sqrt(eps1) towards (A_-/A_+)^2 = 1e-6 of the Bunch-Davies value
    phis = w.table_lo + np.arange(w.table_n) * (w.table_hi - w.table_lo) / (w.table_n - 1)
    post = g[2][(phis < 0) & (phis > -0.045)]
    if sigma == 1.0:
        assert post.min() < 0.5 and post.max() > 1.5
    else:
        assert post.max() < 0.01 and post.min() > 1e-7


@pytest.mark.parametrize("sigma", [1.0, 0.1])
def test_sudden_kink_matches_oracle_and_closed_form(sigma):
    n = 48
    lo, hi = -0.288 * abs(PI_T), 0.4 * abs(PI_T)
    phi_start = 10 * abs(PI_T)
    say(f"matched table kink sigma={sigma}")
    g, o = _both(0, V0, 0.0, AP, AM, sigma, n, lo, hi, phi_start, -AP / (V0 + AP * phi_start))
    _assert_tables_close(g, o)
    c = AM / V0
    kappa = -3.0 * (AP - AM) / (V0 * abs(PI_T))
    phis = lo + np.arange(n) * (hi - lo) / (n - 1)
    for j in np.nonzero(phis < 0)[0]:
        x = 0.1
        for _ in range(100):   # Newton: time after the kink at which phi_j is reached
            f = -c * x + (PI_T + c) * (1 - math.exp(-3 * x)) / 3 - phis[j]
            x -= f / (-c + (PI_T + c) * math.exp(-3 * x))
        y = sigma * math.exp(x)
        gg = np.exp(1j * y) * (1 + 1j / y)
        ref = abs(1 + 1j * kappa * gg * gg.real / y) ** 2
        assert abs(g[2][j] - ref) < 1e-6 * ref, (j, g[2][j], ref)


def test_power_law_matches_oracle():
    say("matched table power law")
    g, o = _both(1, V0, 0.0, 0.3, 0.0, 0.3, 9, 0.0, 1.2, 4.0, -0.3)
    _assert_tables_close(g, o)
    assert np.all(np.abs(g[2] - 1) > 1e-3)


@pytest.mark.parametrize("case", ["at_kink", "just_below", "above_start", "unreached", "single"])
def test_edge_nodes(case):
    w = W.srusr_matched()
    phi_start, pi_start = w.match_start
    say(f"matched table edge {case}")
    if case == "at_kink":            # the node at phi_T takes the mode before the kick
        lo, hi, n = -2.0 ** -10, 2.0 ** -10, 3
    elif case == "just_below":
        lo, hi, n = -2.0 ** -30, 0.0, 2
    elif case == "above_start":      # nodes at or above phi_start keep factor 1
        lo, hi, n = 1.0, 1.2, 5
    elif case == "unreached":        # beyond N = 200 on the flat branch: never reached
        lo, hi, n = -0.09, -0.08, 5
    else:
        lo, hi, n = -0.03, -0.03, 1
    g, o = _both(w.kind, w.V0, w.phi_T, w.A_plus, w.A_minus, 1.0, n, lo, hi, phi_start, pi_start)
    _assert_tables_close(g, o)
    if case in ("above_start", "unreached"):
        assert g[2].tolist() == [1.0] * n
    if case == "at_kink":
        assert abs(g[2][1] - 1.0) < 1e-3 and g[2][0] < 0.5


def test_late_start_is_an_error():
    pot = fpt.make_potential(0, V0, 0.0, AP, AM, 0.0, 0.0, -1.0)
    with pytest.raises(fpt.FptError) as e:
        fpt.fpt_noise_table_matched(pot, 1.0, 5, -1e-5, 1e-5, 2 * abs(PI_T), PI_T)
    assert e.value.status == fpt.FPT_EINVAL


def test_fp64_trajectories_on_matched_table():
    """1500 SR -> USR trajectories on the matched table: per-trajectory parity."""
    w = W.srusr_matched(n_traj=1500)
    say("fp64 trajectories matched table")
    gpu, _ = gpu_run(w)
    ora = oracle_run(w, last_phi=True)
    assert_fp64_parity(gpu, ora, w)


def test_fp32_trajectories_on_matched_table():
    """FP32 state on the matched table: mean and spread of N within the statistical error of the
    FP64 run on the same seeds."""
    w = W.srusr_matched(n_traj=200_000)
    say("fp32 vs fp64 trajectories matched table")
    g64, _ = gpu_run(w)
    g32, _ = gpu_run(w.with_(precision=1))
    N64, N32 = g64[0], g32[0]
    assert np.isfinite(N32).all()
    s = N64.std()
    assert abs(N32.mean() - N64.mean()) < 5 * s / math.sqrt(len(N64))
    assert abs(N32.std() / s - 1) < 0.02
