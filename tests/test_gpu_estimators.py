"""Error bars of the weighted histogram (Sec. 4.1) through the C ABI:
- the library's jackknife, lognormal (Cox) and merge entry points equal the oracle's
  estimators (host computation);
- on the GPU, with the inverse-Gaussian companion problem:
  - the jackknife error of direct sampling matches the spread of independent replicate runs;
  - Cox's interval of importance-sampled slots matches the replicate spread of the estimates;
  - runs with several bias amplitudes merge consistently, and the merged far tail follows the
    closed-form inverse-Gaussian law."""
import math
import sys

import numpy as np
import pytest
from scipy import stats

pytestmark = pytest.mark.gpu

from oracle import estimators as E  # noqa: E402
from paper_2410_13683_amd import fpt  # noqa: E402
from paper_2410_13683_amd import workloads as W  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_estimators_match_oracle():
    """Host-only entry points: no device needed."""
    rng = np.random.default_rng(3)
    B, ns = 13, 40
    n = rng.integers(1000, 5000, size=B).astype(np.uint64)
    sw = rng.gamma(1.5, 2.0, size=(B, ns)) * 100
    sw[:, 3] = 0.0
    p, e = fpt.fpt_jackknife(n, sw)
    po, eo = E.jackknife(n, sw)
    np.testing.assert_allclose(p, po, rtol=1e-14)
    np.testing.assert_allclose(e, eo, rtol=1e-12, atol=1e-300)
    count = rng.integers(0, 400, size=ns).astype(np.uint64)
    count[:3] = [0, 1, 2]
    mu = rng.normal(-20, 5, size=ns)
    s = rng.uniform(0, 1.5, size=ns)
    slnw = count * mu
    slnw2 = count * (mu ** 2 + s ** 2)
    g = fpt.fpt_lognormal_bins(10 ** 6, count, slnw, slnw2)
    o = E.lognormal(10 ** 6, count, slnw, slnw2)
    for a, b in zip(g, o):
        np.testing.assert_allclose(a, b, rtol=1e-13, equal_nan=True)
    P = rng.uniform(0, 1, size=(4, ns))
    Er = rng.uniform(0.01, 0.1, size=(4, ns))
    Er[0, 5] = np.inf
    Er[:, 7] = 0.0
    P[2, 9] = np.nan
    g = fpt.fpt_merge_bins(P, Er)
    o = E.merge(P, Er)
    for a, b in zip(g, o):
        np.testing.assert_allclose(a, b, rtol=1e-13, equal_nan=True)


def test_estimator_argument_errors():
    with pytest.raises(fpt.FptError):
        fpt.fpt_jackknife(np.array([10], dtype=np.uint64), np.ones((1, 4)))        # one block
    with pytest.raises(fpt.FptError):
        fpt.fpt_jackknife(np.array([10, 0], dtype=np.uint64), np.ones((2, 4)))     # an empty block
    with pytest.raises(fpt.FptError):
        fpt.fpt_lognormal_bins(0, np.ones(3), np.zeros(3), np.zeros(3))            # no trajectories


@pytest.fixture(scope="module")
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


def test_jackknife_error_matches_replicate_spread(_gpu):
    """Direct sampling of the inverse-Gaussian problem: 8 replicates of 16 blocks x 2e4."""
    from paper_2410_13683_amd import runner
    torch = _gpu
    w = W.exponential_ig(n_traj=16 * 20_000, dN=2e-4)
    stream = torch.cuda.current_stream()
    ctx = runner.context_for(w, bins_kind=0, n_bins=40, lo=-0.5, hi=1.0)
    P, ERR = [], []
    for r in range(8):
        n_b, sw_b, _ = runner.run_blocks(ctx, w, 16, stream, traj_offset=r * w.n_traj)
        p, e = fpt.fpt_jackknife(n_b, sw_b)
        P.append(p)
        ERR.append(e)
    ctx.destroy()
    P, ERR = np.array(P), np.array(ERR)
    ok = P.mean(0) > 2e-3
    ratio = P.std(0, ddof=1)[ok] / ERR.mean(0)[ok]
    say(f"jackknife: replicate spread / jackknife error over {ok.sum()} bins: mean {ratio.mean():.3f}")
    assert ok.sum() >= 10
    assert 0.8 < ratio.mean() < 1.25, ratio
    # and against the binomial error of a count fraction
    binom = np.sqrt(P.mean(0) * (1 - P.mean(0)) / w.n_traj)[ok]
    assert 0.8 < np.mean(ERR.mean(0)[ok] / binom) < 1.2


def test_lognormal_error_matches_replicate_spread(_gpu):
    """Importance sampling (A = 2) into the far tail, 48 log bins over deltaN in [0.3, 3):
    8 replicates of 2e5 trajectories."""
    from paper_2410_13683_amd import runner
    torch = _gpu
    w = W.exponential_ig(n_traj=200_000, dN=2e-4, A_bias=2.0)
    stream = torch.cuda.current_stream()
    ctx = runner.context_for(w, bins_kind=1, n_bins=48, lo=0.3, hi=3.0)
    PL, HW, PP, CNT = [], [], [], []
    for r in range(8):
        ctx.reset()
        ctx.run(w.n_traj, w.dN, w.seed, r * w.n_traj, stream)
        h = ctx.histogram()
        p, lo, hi = fpt.fpt_lognormal_bins(h["n_traj"], h["count"], h["sum_lnw"], h["sum_lnw2"])
        PL.append(p)
        HW.append(0.5 * (hi - lo))
        PP.append(np.asarray(h["sum_w"]) / h["n_traj"])
        CNT.append(np.asarray(h["count"]))
    ctx.destroy()
    PL, HW, PP, CNT = map(np.array, (PL, HW, PP, CNT))
    ok = CNT.min(0) >= 200
    ok[0] = ok[-1] = False     # under- and overflow slots span a wide range of ln w: not a bin
    assert ok.sum() >= 10
    spread = PP.std(0, ddof=1)[ok]
    ratio = spread / HW.mean(0)[ok]
    say(f"lognormal: replicate spread / Cox half-width over {ok.sum()} slots: mean {ratio.mean():.3f}")
    assert 0.75 < ratio.mean() < 1.3, ratio
    # the lognormal mass and the plain mass estimate agree within the interval
    assert np.all(np.abs(PL.mean(0)[ok] / PP.mean(0)[ok] - 1) < 3 * HW.mean(0)[ok] / PP.mean(0)[ok] + 0.01)


def test_merge_across_bias_amplitudes_follows_closed_form(_gpu):
    """A in {1, 2, 3}, 4e5 trajectories each at dN = 1e-4, 40 log bins over deltaN in [0.1, 3):
    every run agrees with the merge where it has data, and the merged slot masses follow the
    inverse-Gaussian law (mean 2, shape 400) out to deltaN = 1, 1e-6 below the peak."""
    from paper_2410_13683_amd import runner
    torch = _gpu
    stream = torch.cuda.current_stream()
    lo, hi, nb = 0.1, 3.0, 40
    P, ERR = [], []
    for A in (1.0, 2.0, 3.0):
        w = W.exponential_ig(n_traj=400_000, dN=1e-4, A_bias=A)
        ctx = runner.context_for(w, bins_kind=1, n_bins=nb, lo=lo, hi=hi)
        ctx.run(w.n_traj, w.dN, w.seed, 0, stream)
        h = ctx.histogram()
        ctx.destroy()
        n = h["n_traj"]
        p = np.asarray(h["sum_w"]) / n
        e = np.sqrt(np.maximum(np.asarray(h["sum_w2"]) / n - p ** 2, 0.0) / n)
        e[np.asarray(h["count"]) < 100] = np.inf      # too few samples for a variance
        P.append(p)
        ERR.append(e)
    pm, em = fpt.fpt_merge_bins(np.array(P), np.array(ERR))
    for p, e in zip(P, ERR):
        both = np.isfinite(e) & np.isfinite(em) & (e > 0)
        zz = (p[both] - pm[both]) / e[both]
        assert np.all(np.abs(zz) < 5), zz
    mu, lam = 2.0, 400.0
    edges = 2.0 + lo * (hi / lo) ** (np.arange(nb + 1) / nb)
    law = stats.invgauss(mu / lam, scale=lam)
    exact = law.sf(edges[:-1]) - law.sf(edges[1:])
    ok = np.isfinite(pm[1:-1]) & (edges[1:] <= 3.0) & (exact > 0)
    rel = np.abs(pm[1:-1][ok] / exact[ok] - 1)
    z = (pm[1:-1][ok] - exact[ok]) / em[1:-1][ok]
    say(f"merge: {ok.sum()} bins down to {exact[ok].min():.1e}, chi2/n {np.mean(z ** 2):.2f}, max rel {rel.max():.3f}")
    assert ok.sum() >= 15 and exact[ok].min() < 1e-6
    # the Euler-Maruyama overshoot (O(S sqrt(dN))) shifts the law slightly; allow 5 % beside the errors
    assert np.all(rel < 0.05 + 4 * em[1:-1][ok] / exact[ok]), rel


def test_normalisation_of_gpu_histogram_matches_oracle():
    """Sec. 4.1's reconstruction of P(deltaN) end to end: the library's normalisation
    (fpt_density, fpt_tail_find, fpt_tail_at) of a GPU histogram against the oracle's
    normalisation of the oracle's histogram of its own trajectories.  SR -> USR problem, FP64,
    bias A = 2, 2e4 trajectories, the 256 log bins of the FP32 benchmark: the densities and tail
    sets agree to 1e-9 wherever the two histograms hold the same trajectories (an FP64 near-tie
    may move one across an edge)."""
    import torch
    from oracle import oracle as orc
    from tests._glue import oracle_run
    from tests._gpu import gpu_run
    w = W.srusr_is_fp32(2.0, n_traj=20_000).with_(precision=0, seed=51)
    say(f"normalisation of a GPU histogram: {w.n_traj} trajectories")
    torch.cuda.set_device(0)
    _, h = gpu_run(w, dumps=False)
    ho = orc.histogram(*oracle_run(w), w.N_ref, w.bins_kind, w.n_bins, w.lo, w.hi)
    cg, co = h["count"].astype(np.int64), ho["count"].astype(np.int64)
    assert np.abs(cg - co).sum() <= 2
    d, edges, m = fpt.fpt_density(h, w.bins_kind, w.n_bins, w.lo, w.hi)
    d_o, e_o = E.density(ho, w.bins_kind, w.n_bins, w.lo, w.hi)
    m_o = E.moments(ho)
    np.testing.assert_allclose(edges, e_o, rtol=1e-15)
    same = (cg == co)[1:-1]
    np.testing.assert_allclose(d[same], d_o[same], rtol=1e-9, atol=1e-300)
    for k in ("mean_w", "mean_N", "ess"):
        np.testing.assert_allclose(m[k], m_o[k], rtol=1e-6 if k == "ess" else 1e-9, err_msg=k)
    suffix_same = np.cumsum((cg != co)[::-1])[::-1] == 0       # slots j.. hold the same trajectories
    checked = 0
    for p in (1e-4, 1e-6, 1e-8):
        t, t_o = fpt.fpt_tail_find(h, w.bins_kind, w.n_bins, w.lo, w.hi, p), \
            E.tail_find(ho, w.bins_kind, w.n_bins, w.lo, w.hi, p)
        if t["slot"] > 0 and suffix_same[t["slot"]] and t["slot"] == t_o["slot"]:
            for k in ("P", "P_err", "ess"):
                np.testing.assert_allclose(t[k], t_o[k], rtol=1e-8, err_msg=(p, k))
            assert t["count"] == t_o["count"]
            checked += 1
        say(f"  p = {p:g}: slot {t['slot']} (oracle {t_o['slot']}), P = {t['P']:.4e}, ESS_T = {t['ess']:.1f}")
    assert checked >= 2
