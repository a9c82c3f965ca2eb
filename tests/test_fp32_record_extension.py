"""The FP32 kernels evaluate a 16-step group on the linear piece of the interval where the group
starts, an approximation of the FP32 variant (the method, the oracle and the FP64 kernels
interpolate in every step's own interval): where a path passes a node, the piece is extended
instead of switched.  These checks bound that extension on the noise tables the FP32 workloads
use, computed from the oracle's own table generators (no GPU): early in the ultra-slow roll a path
moves about one node spacing per step, so a group can run 16 intervals past its start."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from _glue import oracle_table  # noqa: E402
from paper_2410_13683_amd import workloads as W  # noqa: E402


def _extension_error(q, k, skip):
    """max over intervals j (outside `skip`) of |q_j - k (q_j+1 - q_j) - q_j-k| / |q_j-k|: the
    start interval's piece extended k nodes below its lower node, against the table there."""
    n = len(q)
    j = np.arange(k, n - 1)
    j = j[~np.isin(j, skip)]
    ext = q[j] - k * (q[j + 1] - q[j])
    return float(np.max(np.abs(ext - q[j - k]) / np.abs(q[j - k])))


def _tables(w):
    S, t, lo, hi = oracle_table(w)
    n = len(S)
    h = (hi - lo) / (n - 1)
    x = lo + h * np.arange(n)
    A = np.where(x >= w.phi_T, w.A_plus, w.A_minus)
    r = A / (w.V0 + A * (x - w.phi_T))        # V'/V at the nodes
    return S, t, r, x, h


def test_record_extension_on_the_bessel_table():
    """Default table (4096 nodes, spacing 2^-16): over 16 intervals, away from the kink's NaN-marked
    intervals, the extension stays within 1e-9 (S), 5e-7 (tan theta) and 1e-8 (V'/V) relative."""
    w = W.srusr_is_fp32(2.0)
    S, t, r, x, h = _tables(w)
    jT = int(round((w.phi_T - x[0]) / h))
    skip = np.arange(jT - 18, jT + 18)
    # a path moves |pi| dN per step, at most ~0.92 of a spacing here (|pi| <= sqrt(2 eps_+))
    assert np.sqrt(2 * 0.01) * w.dN / h < 1.0
    assert _extension_error(S, 16, skip) < 1e-9
    assert _extension_error(t, 16, skip) < 5e-7
    assert _extension_error(r, 16, skip) < 1e-8


def _group_extension_error(q, x, h, dN, phi_T, speed):
    """max over intervals below the kink of the relative difference, over the distance a 16-step
    group moves there (16 |pi| dN, |pi| from `speed`), between the start interval's extended piece
    and the table's linear interpolation."""
    worst, where = 0.0, None
    jT = int(round((phi_T - x[0]) / h))
    for j in range(1, jT - 2):
        d = 16.0 * speed(x[j]) * dN / h            # group displacement in node spacings
        ks = np.arange(1, int(np.ceil(d)) + 1).astype(float)
        ks[-1] = d
        kk = np.minimum(np.floor(ks).astype(int), j)
        fr = ks - kk
        tab = q[j - kk] + fr * (q[np.maximum(j - kk - 1, 0)] - q[j - kk])
        e = float(np.max(np.abs(q[j] - ks * (q[j + 1] - q[j]) - tab) / np.abs(tab)))
        if e > worst:
            worst, where = e, x[j]
    return worst, where


def test_record_extension_on_the_matched_table():
    """Bessel-matched table: sharp features near phi_end (slope changes of tens of per cent of S
    between neighbouring intervals), where paths are slow.  At the distance a 16-step group moves
    along the classical ultra-slow-roll path (|pi| = sqrt(2 eps_+) - 3 |phi - phi_T|, not below
    sqrt(2 eps_-)), the extension stays within 5e-3 of S, the worst just above phi_end, and
    within 2e-7 of tan theta; on the default table the same measure stays below 1e-9 (S)."""
    speed = lambda phi: max(np.sqrt(2 * 0.01) - 3.0 * abs(phi), np.sqrt(2 * 1e-8))
    w = W.srusr_is_fp32_matched(2.0)
    S, t, r, x, h = _tables(w)
    eS, at = _group_extension_error(S, x, h, w.dN, w.phi_T, speed)
    et, _ = _group_extension_error(t, x, h, w.dN, w.phi_T, speed)
    assert 1e-4 < eS < 5e-3 and at < w.phi_end + 0.003
    assert et < 2e-7
    wd = W.srusr_is_fp32(2.0)
    Sd, _, _, xd, hd = _tables(wd)
    assert _group_extension_error(Sd, xd, hd, wd.dN, wd.phi_T, speed)[0] < 1e-9
