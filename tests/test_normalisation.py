"""The library's normalisation entry points (fpt_density, fpt_tail_at, fpt_tail_find; Sec. 4.1:
P(deltaN) reconstructed from the weighted runs) against the oracle's plain versions
(oracle/estimators.py, pinned on sample sums in tests/test_oracle_estimators.py), on histograms
the oracle builds from synthetic per-trajectory outputs.  Host code: no GPU needed."""
import numpy as np
import pytest

from oracle import estimators as E
from oracle import oracle as orc
from paper_2410_13683_amd import fpt


def _hist(seed, bins_kind, n_bins, lo, hi, n=30_000):
    rng = np.random.default_rng(seed)
    x = rng.gamma(2.5, 0.025, size=n) - (0.0 if bins_kind else 0.02)
    lnw = rng.normal(-3.0, 1.5, size=n) - 20.0 * x          # heavier bins carry smaller weights
    steps = np.full(n, 99, dtype=np.uint32)
    steps[rng.random(n) < 0.02] |= orc.FLAG_CENSORED
    return orc.histogram(5.0 + x, lnw, steps, 5.0, bins_kind, n_bins, lo, hi)


CASES = [(0, 64, -0.02, 0.2), (1, 256, 0.01, 0.3), (1, fpt.FPT_MAX_BINS, 1e-3, 0.5), (0, 1, 0.0, 0.1)]


@pytest.mark.parametrize("bins_kind,n_bins,lo,hi", CASES)
def test_density_and_moments_match_oracle(bins_kind, n_bins, lo, hi):
    h = _hist(7, bins_kind, n_bins, lo, hi)
    d, e, m = fpt.fpt_density(h, bins_kind, n_bins, lo, hi)
    d_o, e_o = E.density(h, bins_kind, n_bins, lo, hi)
    m_o = E.moments(h)
    np.testing.assert_allclose(e, e_o, rtol=1e-15)
    np.testing.assert_allclose(d, d_o, rtol=1e-13, atol=0)
    for k, v in m_o.items():
        np.testing.assert_allclose(m[k], v, rtol=1e-13, atol=0, err_msg=k)


@pytest.mark.parametrize("bins_kind,n_bins,lo,hi", CASES)
def test_tail_sets_match_oracle(bins_kind, n_bins, lo, hi):
    h = _hist(8, bins_kind, n_bins, lo, hi)
    for slot in sorted({1, 2, n_bins // 2 + 1, n_bins, n_bins + 1}):
        t, t_o = fpt.fpt_tail_at(h, bins_kind, n_bins, lo, hi, slot), E.tail_at(h, bins_kind, n_bins, lo, hi, slot)
        assert t["slot"] == slot and t["count"] == t_o["count"]
        for k in ("x_star", "P", "P_err", "P_err_lognormal", "ess"):
            np.testing.assert_allclose(t[k], t_o[k], rtol=1e-12, atol=0, err_msg=(slot, k))
    found = 0
    for p in (1e-12, 1e-6, 1e-4, 1e-3, 1e-2, 0.1, 0.5):
        t, t_o = fpt.fpt_tail_find(h, bins_kind, n_bins, lo, hi, p), E.tail_find(h, bins_kind, n_bins, lo, hi, p)
        assert t["slot"] == t_o["slot"], p
        found += t["slot"] > 0
        if t["slot"] > 0:
            assert 0 < t["P"] <= p
            np.testing.assert_allclose([t["P"], t["ess"]], [t_o["P"], t_o["ess"]], rtol=1e-12)
    assert found >= 1


def test_normalisation_rejects_bad_arguments():
    h = _hist(9, 0, 16, 0.0, 0.2)
    for args in [(0, 0, 0.0, 0.2), (0, 16, 0.2, 0.2), (1, 16, 0.0, 0.2), (0, fpt.FPT_MAX_BINS + 1, 0.0, 0.2)]:
        with pytest.raises(fpt.FptError):
            fpt.fpt_density(h, *args)
    for slot in (0, 18):
        with pytest.raises(fpt.FptError):
            fpt.fpt_tail_at(h, 0, 16, 0.0, 0.2, slot)
    for p in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(fpt.FptError):
            fpt.fpt_tail_find(h, 0, 16, 0.0, 0.2, p)
    empty = dict(h, n_traj=0)
    with pytest.raises(fpt.FptError):
        fpt.fpt_density(empty, 0, 16, 0.0, 0.2)
    bad = dict(h, sum_w=np.where(np.arange(18) == 3, np.nan, h["sum_w"]))
    with pytest.raises(fpt.FptError):
        fpt.fpt_tail_at(bad, 0, 16, 0.0, 0.2, 1)
