"""The stored workload constants are what the oracle-only derivation script produces."""
import math

from oracle import derive_constants as dc
from paper_2410_13683_amd import workloads as W


def test_stored_constants_rederive():
    assert math.isclose(dc.hubble_noise(), W.NOISE_S_HUBBLE, rel_tol=1e-14)
    assert math.isclose(dc.noise_free_N(-W.DELTA_E), W.N_REF_SRUSR, rel_tol=1e-12)
    assert math.isclose(dc.linear_N_ref(), W.N_REF_LINEAR, rel_tol=1e-12)
    assert abs(W.N_REF_SRUSR - 10.0) < 1e-9


def test_table_grid_is_dyadic():
    assert W.TABLE_PHI_LO + W.TABLE_J_T * W.TABLE_H == 0.0
    assert (W.TABLE_PHI_HI - W.TABLE_PHI_LO) / (W.TABLE_N - 1) == W.TABLE_H
    w = W.srusr_bessel()
    assert w.table_lo < w.phi_end - 1e-3 and w.table_hi > w.phi_in + 1e-3


def test_time_workload_start_rederives():
    """The time-indexed workload starts on the matched table's reference trajectory: the stored
    momentum at the transition and the noise-free passage from there."""
    pi_ref, n_ref, n_to_kink = dc.time_start()
    assert math.isclose(pi_ref, W.TIME_PI_IN, rel_tol=1e-10)
    assert math.isclose(n_ref, W.N_REF_TIME, rel_tol=1e-10)
    assert dc.MATCH_PHI_START == W.MATCH_PHI_START
    # the reference trajectory relaxes for ~7.6 e-folds and arrives slower than sqrt(2 eps_+)
    assert 7.0 < n_to_kink < 8.0 and abs(pi_ref) < math.sqrt(0.02)
    w = W.srusr_time()
    assert w.pi_in == W.TIME_PI_IN and w.N_ref == W.N_REF_TIME and w.table_hi > W.N_REF_TIME
