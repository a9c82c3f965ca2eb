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
