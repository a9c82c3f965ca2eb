"""The per-trajectory FP64 parity check (tests/_glue.assert_fp64_parity) on the CPU, with the
oracle on both sides: it accepts a rounding-level difference of the start (phi_in moved by a few
ulp, which is how two FP64 implementations that round differently drift apart), and rejects a
wrong random stream, an N off by 1e-8 and a crossing step off by one away from a near-tie."""
import numpy as np
import pytest

from paper_2410_13683_amd import workloads as W
from tests._glue import assert_fp64_parity, oracle_run


@pytest.fixture(scope="module")
def runs():
    w = W.srusr_bessel(n_traj=1200, seed=23).with_(bias_kind=W.BIAS_CONST, A_bias=1.5)
    ref = oracle_run(w, last_phi=True)
    moved = oracle_run(w.with_(phi_in=w.phi_in + 4e-18), last_phi=True)    # 4e-18: below 1 ulp of 0.05
    return w, ref, moved


def test_accepts_rounding_level_drift(runs):
    w, ref, moved = runs
    assert_fp64_parity(ref[:3], ref, w)
    assert_fp64_parity(moved[:3], ref, w)


def test_rejects_a_wrong_stream(runs):
    w, ref, _ = runs
    other = oracle_run(w.with_(seed=w.seed + 1), n_traj=1, traj_offset=5)
    gpu = tuple(a.copy() for a in ref[:3])
    for k in range(3):
        gpu[k][5] = other[k][0]
    with pytest.raises(AssertionError):
        assert_fp64_parity(gpu, ref, w)


def test_rejects_small_n_and_step_errors(runs):
    w, ref, _ = runs
    # the trajectory whose last step is the longest: no exemption can apply to it
    i = int(np.argmax(np.abs(ref[3][:, 0] - ref[3][:, 1])))
    gpu = tuple(a.copy() for a in ref[:3])
    gpu[0][i] *= 1.0 + 1e-8
    with pytest.raises(AssertionError):
        assert_fp64_parity(gpu, ref, w)
    gpu = tuple(a.copy() for a in ref[:3])
    gpu[2][i] += 1
    with pytest.raises(AssertionError):
        assert_fp64_parity(gpu, ref, w)
    gpu = tuple(a.copy() for a in ref[:3])
    gpu[1][i] += 1e-6
    with pytest.raises(AssertionError):
        assert_fp64_parity(gpu, ref, w)
