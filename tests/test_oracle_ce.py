"""Pins of the oracle's Chapman-Enskog viscosity chain (section "Macroscopic
Validation: Viscosity and Transport Coefficients"): transport cross-section,
collision integral and viscosity against hard-sphere closed forms and the
inverse-square potential, whose deflection angle is known in closed form."""
import math

import numpy as np
import pytest

import workloads as W


def test_hard_sphere_cross_section_and_viscosity(orc):
    d = 3.0                                   # Angstrom
    P = orc.potential_hs(d)
    Q = orc.transport_q2(P, [50.0, 500.0, 5e4], 4e-10, n_panels=64, n_gl=8)
    # sin^2(2 arccos(b/d)) = 4 (b/d)^2 (1 - (b/d)^2): Q2 = (2/3) pi d^2, any E
    np.testing.assert_allclose(Q, 2.0 / 3.0 * math.pi * (d * 1e-10) ** 2, rtol=1e-12)
    T = np.array([300.0, 3000.0])
    om = orc.collision_integral(P, T, 4e-10, n_lag=8, n_panels=64, n_gl=8)
    np.testing.assert_allclose(om, math.pi * (d * 1e-10) ** 2, rtol=1e-12)
    mu = orc.viscosity_ce(om, T, W.AR_MASS)
    want = 5.0 / 16.0 * np.sqrt(math.pi * W.AR_MASS * W.KB * T) / (math.pi * (d * 1e-10) ** 2)
    np.testing.assert_allclose(mu, want, rtol=1e-12)
    # the average as printed weights E^2 / (2 (kT)^3): constant Q2 comes back
    om_p = orc.collision_integral(P, T, 4e-10, n_lag=8, printed=True, n_panels=64, n_gl=8)
    np.testing.assert_allclose(om_p, Q[0], rtol=1e-12)


def _q2_inverse_square(K, E, b_cut):
    """2 pi int_0^b_cut sin^2(pi (1 - b / sqrt(b^2 + K/E))) b db, b in Angstrom,
    by scipy quad on the closed-form angle (independent of the oracle)."""
    from scipy.integrate import quad
    a = math.sqrt(K / E)

    def f(b):
        return math.sin(math.pi * (1.0 - b / math.sqrt(b * b + a * a))) ** 2 * b

    val, err = quad(f, 0.0, b_cut, limit=400, epsabs=1e-14, epsrel=1e-13)
    return 2.0 * math.pi * val * 1e-20        # Angstrom^2 -> m^2


def test_inverse_square_cross_section_against_closed_form_angle(orc):
    K = 2000.0                                 # K Angstrom^2
    P = orc.potential_invpow(K, 2)
    E = np.array([100.0, 1000.0, 20000.0])
    b_cut = 30.0
    got = orc.transport_q2(P, E, b_cut * 1e-10, n_panels=512, n_gl=16)
    want = np.array([_q2_inverse_square(K, e, b_cut) for e in E])
    np.testing.assert_allclose(got, want, rtol=1e-8)


def test_collision_integral_of_a_one_over_E_cross_section(orc):
    # inverse square: Q2 = c / E up to the b cut-off; with b_cut far beyond
    # sqrt(K/E) the standard average gives Omega = c / (2 T)
    K = 50.0
    P = orc.potential_invpow(K, 2)
    b_cut = 400.0
    T = np.array([400.0])
    q1 = orc.transport_q2(P, [1000.0], b_cut * 1e-10, n_panels=2048, n_gl=8)[0]
    c = q1 * 1000.0
    om = orc.collision_integral(P, T, b_cut * 1e-10, n_lag=12, n_panels=2048, n_gl=8)
    assert om[0] == pytest.approx(c / (2.0 * T[0]), rel=2e-4)
