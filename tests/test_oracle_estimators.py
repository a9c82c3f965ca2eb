"""Pins of the oracle's error-bar estimators (Sec. 4.1).
- The delete-one jackknife equals the textbook standard error of a mean of equal blocks,
  and on direct-sampling counts it reproduces the binomial error.
- Without weights the lognormal estimator is the count fraction with the binomial interval.
- On lognormal samples Cox's interval covers the true mean at the one-sigma rate; the
  interval without its s^4 term does not.
- With random counts and lognormal weights, the combined interval covers the true slot mass
  at the one-sigma rate; Cox's part alone does not.
- The inverse-variance merge against closed forms."""
import math

import numpy as np
import pytest

from oracle import estimators as E


def test_jackknife_equals_standard_error_of_equal_blocks():
    rng = np.random.default_rng(1)
    B, m = 17, 1000
    sw = rng.gamma(2.0, 3.0, size=(B, 5)) * m
    p, err = E.jackknife(np.full(B, m), sw)
    block_means = sw / m
    np.testing.assert_allclose(p, block_means.mean(axis=0), rtol=1e-14)
    np.testing.assert_allclose(err, block_means.std(axis=0, ddof=1) / math.sqrt(B), rtol=1e-12)


def test_jackknife_reproduces_binomial_error():
    """Direct sampling: w = 1, slot masses are count fractions; 40 blocks of 2.5e4."""
    rng = np.random.default_rng(2)
    probs = np.array([0.5, 0.2, 0.05, 0.01, 0.002])
    B, m = 40, 25_000
    counts = np.stack([rng.multinomial(m, np.append(probs, 1 - probs.sum()))[:-1] for _ in range(B)])
    p, err = E.jackknife(np.full(B, m), counts.astype(float))
    binom = np.sqrt(probs * (1 - probs) / (B * m))
    # the jackknife variance has a chi^2_(B-1) spread: +-23 % at 1 sigma for B = 40
    assert np.all(np.abs(err / binom - 1) < 0.6), err / binom
    assert abs(np.mean(err / binom) - 1) < 0.25


def test_jackknife_unequal_blocks_brute_force():
    n = np.array([10.0, 30.0, 7.0])
    sw = np.array([[1.0, 4.0], [2.0, 9.0], [0.5, 1.5]])
    p, err = E.jackknife(n, sw)
    loo = [(sw.sum(0) - sw[b]) / (n.sum() - n[b]) for b in range(3)]
    mean = np.mean(loo, axis=0)
    np.testing.assert_allclose(err, np.sqrt(2 / 3 * sum((x - mean) ** 2 for x in loo)), rtol=1e-14)
    np.testing.assert_allclose(p, sw.sum(0) / n.sum(), rtol=1e-15)


def test_lognormal_without_weights_is_the_count_fraction():
    count = np.array([0, 1, 5, 300])
    p, lo, hi = E.lognormal(1000, count, np.zeros(4), np.zeros(4))
    assert np.isnan(p[0]) and np.isnan(p[1])
    f = count[2:] / 1000
    np.testing.assert_allclose(p[2:], f, rtol=1e-15)
    rel = np.sqrt((1 - f) / count[2:])          # binomial relative error of a count fraction
    np.testing.assert_allclose(np.log(hi[2:] / p[2:]), rel, rtol=1e-14)
    np.testing.assert_allclose(np.log(p[2:] / lo[2:]), rel, rtol=1e-14)
    # a slot holding every trajectory has no count fluctuation
    p, lo, hi = E.lognormal(50, [50], [0.0], [0.0])
    assert lo[0] == hi[0] == p[0] == 1.0


@pytest.mark.parametrize("s", [0.5, 1.0])
def test_cox_interval_covers_the_lognormal_mean_at_one_sigma(s):
    """2000 replicate slots of 60 lognormal weights (mu = -7), each slot holding every trajectory
    (no count fluctuation): the interval holds the true mean e^(mu + s^2/2) in 68.3 % of them
    (binomial +-1 %).  Dropping the s^4 term of the standard error takes the coverage visibly lower."""
    rng = np.random.default_rng(int(s * 10))
    R, nj, mu = 2000, 60, -7.0
    lnw = rng.normal(mu, s, size=(R, nj))
    truth = math.exp(mu + 0.5 * s * s)
    cover = 0
    cover_short = 0
    for r in range(R):
        # n_traj = n_j: the slot holds every trajectory, so only Cox's part is left
        p, lo, hi = E.lognormal(nj, [nj], [lnw[r].sum()], [(lnw[r] ** 2).sum()])
        cover += lo[0] <= truth <= hi[0]
        m_ = lnw[r].mean()
        s2 = lnw[r].var(ddof=1)
        th, se = m_ + s2 / 2, math.sqrt(s2 / nj)
        cover_short += math.exp(th - se) <= truth <= math.exp(th + se)
    assert abs(cover / R - 0.6827) < 0.035, cover / R
    if s == 1.0:
        assert cover_short / R < cover / R - 0.03


def test_merge_closed_forms():
    p, e = E.merge([[1.0, 5.0, np.nan], [3.0, 5.0, 2.0]], [[1.0, 1.0, 1.0], [1.0, 2.0, 0.5]])
    assert p[0] == pytest.approx(2.0) and e[0] == pytest.approx(1 / math.sqrt(2))
    assert p[1] == pytest.approx(5.0) and e[1] == pytest.approx(1 / math.sqrt(1.25))
    assert p[2] == pytest.approx(2.0) and e[2] == pytest.approx(0.5)          # the NaN run is left out
    p, e = E.merge([[1.0], [4.0]], [[0.0], [np.inf]])                          # no usable run
    assert np.isnan(p[0]) and np.isnan(e[0])
    p, e = E.merge([[1.0], [4.0]], [[1.0], [2.0]])
    assert p[0] == pytest.approx((1.0 + 4.0 / 4) / 1.25)


@pytest.mark.parametrize("s", [0.05, 0.7])
def test_combined_interval_covers_the_slot_mass_at_one_sigma(s):
    """1500 replicates of n = 4000 trajectories, each in the slot with probability 0.03, with
    lognormal weights (mu = -5) there: the interval holds the true mass 0.03 e^(mu + s^2/2) in
    68.3 % of replicates.  With nearly constant weights (s = 0.05) Cox's part alone is far too
    narrow: the count fluctuation dominates."""
    rng = np.random.default_rng(int(100 * s))
    R, n, q, mu = 1500, 4000, 0.03, -5.0
    truth = q * math.exp(mu + 0.5 * s * s)
    cover = cover_cox = 0
    for r in range(R):
        nj = rng.binomial(n, q)
        lnw = rng.normal(mu, s, size=nj)
        p, lo, hi = E.lognormal(n, [nj], [lnw.sum()], [(lnw ** 2).sum()])
        cover += lo[0] <= truth <= hi[0]
        th = math.log(p[0])
        s2 = lnw.var(ddof=1)
        se = math.sqrt(s2 / nj + s2 * s2 / (2 * (nj - 1)))
        cover_cox += math.exp(th - se) <= truth <= math.exp(th + se)
    assert abs(cover / R - 0.6827) < 0.04, cover / R
    if s == 0.05:
        assert cover_cox / R < 0.2


# ---- normalisation (Sec. 4.1: P(deltaN) from the weighted runs) --------------------------------

def _samples(rng, n, bins_kind):
    """Synthetic per-trajectory outputs: N, ln w and flags (3 % censored, 2 % ended early)."""
    from oracle import oracle as orc
    x = rng.gamma(3.0, 0.02, size=n) - (0.01 if bins_kind == 0 else 0.0)
    lnw = rng.normal(-1.0, 0.8, size=n)
    steps = np.full(n, 1000, dtype=np.uint32)
    u = rng.random(n)
    steps[u < 0.03] |= orc.FLAG_CENSORED
    steps[(u >= 0.03) & (u < 0.05)] |= orc.FLAG_ENDED_EARLY
    return 10.0 + x, lnw, steps


@pytest.mark.parametrize("bins_kind", [0, 1])
def test_normalisation_equals_sums_over_samples(bins_kind):
    """Brute force from the samples themselves, not from the histogram: the mass of each bin, of
    every tail set and of the whole run, with n_traj counting every trajectory run (censored and
    ended-early ones included), against the oracle's normalisation of its histogram."""
    from oracle import oracle as orc
    rng = np.random.default_rng(40 + bins_kind)
    n, nb, lo, hi, N_ref = 20_000, 37, (0.005 if bins_kind else -0.02), 0.15, 10.0
    N, lnw, steps = _samples(rng, n, bins_kind)
    h = orc.histogram(N, lnw, steps, N_ref, bins_kind, nb, lo, hi)
    crossed = (steps & (orc.FLAG_CENSORED | orc.FLAG_ENDED_EARLY)) == 0
    x, w = N[crossed] - N_ref, np.exp(lnw[crossed])
    e = lo + (hi - lo) * np.arange(nb + 1) / nb if bins_kind == 0 else lo * (hi / lo) ** (np.arange(nb + 1) / nb)
    d, edges = E.density(h, bins_kind, nb, lo, hi)
    np.testing.assert_allclose(edges, e, rtol=1e-15)
    for j in range(nb):
        inside = (x >= e[j]) & (x < e[j + 1])
        np.testing.assert_allclose(d[j] * n * (e[j + 1] - e[j]), w[inside].sum(), rtol=1e-12, atol=1e-300)
    m = E.moments(h)
    np.testing.assert_allclose(m["mean_w"], w.sum() / n, rtol=1e-12)
    np.testing.assert_allclose(m["mean_N"], (w * N[crossed]).sum() / w.sum(), rtol=1e-13)
    var = (w * (N[crossed] - (w * N[crossed]).sum() / w.sum()) ** 2).sum() / w.sum()
    np.testing.assert_allclose(m["var_N"], var, rtol=1e-6)
    np.testing.assert_allclose(m["ess"], w.sum() ** 2 / (w * w).sum(), rtol=1e-12)
    np.testing.assert_allclose(m["mass_under"], w[x < lo].sum() / n, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(m["mass_over"], w[x >= hi].sum() / n, rtol=1e-12, atol=1e-300)
    # every bin's mass plus the two outer slots is the whole weight
    np.testing.assert_allclose((d * np.diff(e)).sum() + m["mass_under"] + m["mass_over"], w.sum() / n, rtol=1e-12)
    for slot in (1, 5, nb, nb + 1):
        t = E.tail_at(h, bins_kind, nb, lo, hi, slot)
        x_star = e[slot - 1]
        wt = w[x >= x_star]
        assert abs(t["x_star"] - x_star) <= 4e-16 * abs(x_star) and t["count"] == len(wt)
        np.testing.assert_allclose(t["P"], wt.sum() / n, rtol=1e-12, atol=1e-300)
        # the plain standard error of the mean of w 1_T over all n trajectories
        full = np.zeros(n)
        full[np.flatnonzero(crossed)[x >= x_star]] = wt
        np.testing.assert_allclose(t["P_err"], full.std() / math.sqrt(n), rtol=1e-9)
        np.testing.assert_allclose(t["ess"], wt.sum() ** 2 / (wt * wt).sum(), rtol=1e-12)
    checked = 0
    for p in (1e-3, 1e-2, 0.1, 0.3):
        t = E.tail_find(h, bins_kind, nb, lo, hi, p)
        mass = [w[x >= e[j - 1]].sum() / n for j in range(1, nb + 2)]
        want = next((j for j in range(1, nb + 2) if 0.0 < mass[j - 1] <= p), -1)
        assert t["slot"] == want, (p, t["slot"], want)
        checked += want > 0
    assert checked >= 2
    assert E.tail_find(h, bins_kind, nb, lo, hi, 1e-12)["slot"] == -1


def test_density_closed_form():
    """One sample at the centre of each linear bin j with weight j + 1, n = 2 n_bins trajectories
    (half of them censored): density_j = (j + 1) / (n width)."""
    from oracle import oracle as orc
    nb, lo, hi = 12, -0.3, 0.9
    width = (hi - lo) / nb
    centres = lo + width * (np.arange(nb) + 0.5)
    N = np.concatenate([centres, np.full(nb, np.nan)])
    lnw = np.concatenate([np.log(np.arange(1, nb + 1, dtype=float)), np.zeros(nb)])
    steps = np.concatenate([np.full(nb, 7, dtype=np.uint32), np.full(nb, 7 | orc.FLAG_CENSORED, dtype=np.uint32)])
    h = orc.histogram(N, lnw, steps, 0.0, 0, nb, lo, hi)
    d, _ = E.density(h, 0, nb, lo, hi)
    np.testing.assert_allclose(d, np.arange(1, nb + 1) / (2 * nb * width), rtol=1e-13)
    t = E.tail_at(h, 0, nb, lo, hi, nb)                 # the last bin alone
    assert t["count"] == 1 and abs(t["P"] - nb / (2 * nb)) < 1e-15 and t["ess"] == 1.0
