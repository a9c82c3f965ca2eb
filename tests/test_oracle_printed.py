"""The oracle on the piecewise-linear model with the parameters Sec. 4.2 prints (eq.
potential_starobinsky; tests/golden/printed_values.txt): V0 = 2.8719e-12 and A_+ = 1e-14 are said
to give a scale-invariant spectrum with the CMB amplitude on large scales.  On the slow-roll side
the oracle's Bessel-ansatz noise (eq. covariance_constant_nu with nu from eq.
nu_squared_approximation, sigma = 0.01) must then be the de Sitter H/2pi to O(sigma^2) and eps_V,
and the spectrum S^2/(2 eps_1) on the slow-roll attractor must sit at the measured 2.1e-9 (the
Planck amplitude the paper cites, to 10 %)."""
import math

import numpy as np

from tests.golden.printed import printed

GOLD = printed()


def test_printed_starobinsky_parameters_give_the_cmb_amplitude(orc):
    V0, Ap = GOLD["starobinsky.V0"], GOLD["starobinsky.A_plus"]
    Am = Ap * GOLD["starobinsky.A_minus_over_A_plus"]
    phi = np.linspace(0.05, 0.5, 10)
    S, t = orc.noise_table_bessel(0, V0, 0.0, Ap, Am, 0.01, len(phi), phi[0], phi[-1])
    V = np.array([orc.potential(0, V0, 0.0, Ap, Am, p)[0] for p in phi])
    H = np.sqrt(V / 3.0)
    np.testing.assert_allclose(S, H / (2.0 * math.pi), rtol=1e-3)   # de Sitter on the slow-roll side
    eps1 = 0.5 * (Ap / V) ** 2                                      # attractor: pi = -V'/V
    P_R = S ** 2 / (2.0 * eps1)
    assert np.all(np.abs(P_R / 2.1e-9 - 1.0) < 0.1), P_R
    # scale invariance: the spectrum changes by less than 1 % over the slow-roll range
    assert P_R.max() / P_R.min() < 1.01
