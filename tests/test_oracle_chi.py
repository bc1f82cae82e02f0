"""Pins of the oracle's deflection angle chi(b, E).

Checked against: the hard-sphere closed form chi = 2 arccos(b/d); V = 0;
the inverse-square and Coulomb closed forms; a 40-digit mpmath evaluation of
the deflection integral for the Jager-form potential; and brute-force
integration of the pair trajectory (relative-motion ODE) on a few inputs.
"""
import math

import numpy as np
import pytest

import workloads as W


def test_hard_sphere_closed_form(orc):
    P = orc.potential_hs(3.0)
    for b in [0.0, 0.3, 1.5, 2.9, 2.999, 3.0, 3.2, 9.0]:
        for E in (10.0, 3e4):
            ref = 2.0 * math.acos(min(b / 3.0, 1.0))
            assert abs(orc.chi(P, b, E) - ref) < 1e-13


def test_free_motion(orc):
    P = orc.potential_invpow(0.0, 2)
    for b in [0.1, 1.0, 7.0]:
        assert abs(orc.chi(P, b, 100.0)) < 1e-13


@pytest.mark.parametrize("K,E", [(500.0, 300.0), (5e4, 20.0), (10.0, 1e5)])
def test_inverse_square_closed_form(orc, K, E):
    P = orc.potential_invpow(K, 2)
    for b in [0.05, 0.5, 2.0, 6.0, 10.0]:
        ref = math.pi * (1.0 - b / math.sqrt(b * b + K / E))
        assert abs(orc.chi(P, b, E) - ref) < 1e-12


@pytest.mark.parametrize("K,E", [(800.0, 300.0), (2e4, 50.0)])
def test_coulomb_closed_form(orc, K, E):
    P = orc.potential_invpow(K, 1)
    for b in [0.05, 0.5, 2.0, 6.0, 10.0]:
        ref = 2.0 * math.atan(K / (2.0 * E * b))
        assert abs(orc.chi(P, b, E) - ref) < 1e-12


def test_jager_potential_anchors(orc):
    P = orc.potential_jager(W.JAGER_PLACEHOLDER)
    p = W.JAGER_PLACEHOLDER
    # well of the placeholder set at R_eps with depth 143.2 K
    r = np.linspace(3.0, 5.0, 20001)
    V = np.array([orc.potential_V(P, x) for x in r])
    i = int(np.argmin(V))
    assert abs(r[i] - p.R_eps) < 2e-4 and abs(V[i] + 143.2) < 1e-3
    # continuity (value and slope) at the short-range switch 0.4 R_eps
    r0 = 0.4 * p.R_eps
    h = 1e-7
    lo, hi = orc.potential_V(P, r0 - h), orc.potential_V(P, r0 + h)
    assert abs(hi - lo) / abs(hi) < 1e-6
    s_lo = (orc.potential_V(P, r0 - h) - orc.potential_V(P, r0 - 3 * h)) / (2 * h)
    s_hi = (orc.potential_V(P, r0 + 3 * h) - orc.potential_V(P, r0 + h)) / (2 * h)
    assert abs(s_hi - s_lo) / abs(s_hi) < 1e-4


def _mp_chi(b, E, dps=40):
    """chi by mpmath at high precision, straight from the integral in r."""
    import mpmath as mp
    mp.mp.dps = dps
    p = W.JAGER_PLACEHOLDER

    def V(r):
        if r < mp.mpf("0.4") * p.R_eps:
            return p.A_sr / r * mp.e ** (-p.a_sr * r)
        rep = p.A * mp.e ** (p.a1 * r + p.a2 * r * r + p.am1 / r + p.am2 / (r * r))
        disp = 0
        x = p.beta_tt * r
        for n in range(3, 9):
            s = sum(x ** k / mp.factorial(k) for k in range(2 * n + 1))
            disp += (1 - mp.e ** (-x) * s) * p.C[n - 3] / r ** (2 * n)
        return rep - disp

    b = mp.mpf(b)
    E = mp.mpf(E)

    def D(r):
        return 1 - b * b / (r * r) - V(r) / E

    r = max(b, mp.findroot(V, 3.25))
    while D(r * mp.mpf("0.999")) > 0:
        r *= mp.mpf("0.999")
    rmin = mp.findroot(D, (r * mp.mpf("0.999"), r), solver="anderson")
    # integral over r of dr / (r^2 sqrt(D(r))) with r = rmin / u
    # split at the short-range switch, where V'' jumps
    r0 = mp.mpf("0.4") * p.R_eps
    pts = [0, rmin / r0, 1] if rmin < r0 else [0, 1]
    I = mp.quad(lambda u: 1 / mp.sqrt(D(rmin / u)), pts)
    return float(mp.pi - 2 * (b / rmin) * I)


@pytest.mark.parametrize("g,b", [(2743.87, 9.472), (498.07, 5.2766), (120.81, 7.176),
                                 (312.92, 4.003), (2567.27, 2.096), (19528.8, 0.7)])
def test_jager_against_mpmath(orc, g, b):
    P = orc.potential_jager(W.JAGER_PLACEHOLDER)
    E = 0.5 * (W.AR_MASS / 2) * g * g / W.KB
    ref = _mp_chi(b, E)
    assert abs(orc.chi(P, b, E) - ref) < 1e-11


def _ode_chi(Vp, b, E, X0=400.0):
    """Deflection from the pair trajectory: relative motion under -V'(r) r_hat,
    units where the reduced mass is 2 and E = g^2 (V in K, r in Angstrom)."""
    from scipy.integrate import solve_ivp
    g = math.sqrt(E)
    mu = 2.0

    def rhs(t, y):
        x, yy, vx, vy = y
        r = math.hypot(x, yy)
        f = -Vp(r) / mu / r
        return [vx, vy, f * x, f * yy]

    def out(t, y):
        return math.hypot(y[0], y[1]) - X0 * 1.0001
    out.terminal = True
    out.direction = 1
    T = 4.0 * X0 / g * 50
    sol = solve_ivp(rhs, (0, T), [-X0, b, g, 0.0], method="DOP853", rtol=1e-12,
                    atol=1e-12, events=out, max_step=X0 / g / 20)
    vx, vy = sol.y[2, -1], sol.y[3, -1]
    return math.atan2(vy, vx)


def test_ode_brute_force_inverse_square():
    K, E = 500.0, 300.0
    for b in [0.5, 2.0, 5.0]:
        ref = math.pi * (1.0 - b / math.sqrt(b * b + K / E))
        got = _ode_chi(lambda r: -2.0 * K / r ** 3, b, E, X0=3000.0)
        assert abs(got - ref) < 2e-6


def test_ode_brute_force_jager(orc):
    P = orc.potential_jager(W.JAGER_PLACEHOLDER)

    def Vp(r, h=1e-6):
        return (orc.potential_V(P, r + h) - orc.potential_V(P, r - h)) / (2 * h)

    for g, b in [(2000.0, 2.5), (800.0, 4.0), (5000.0, 1.0)]:
        E = 0.5 * (W.AR_MASS / 2) * g * g / W.KB
        got = _ode_chi(Vp, b, E, X0=200.0)
        ref = orc.chi(P, b, E)
        # compare angles modulo 2 pi (atan2 folds to (-pi, pi])
        d = (got - ref + math.pi) % (2 * math.pi) - math.pi
        assert abs(d) < 1e-6, (g, b, got, ref)


def test_batch_matches_single_and_is_well_behaved(orc):
    P = orc.potential_jager(W.JAGER_PLACEHOLDER)
    b, g, mr = W.deflection_batch(seed=2, n=400)
    ch, st = orc.chi_batch(P, b, g, mr, n_threads=4)
    assert np.all(st == 0) and np.all(np.isfinite(ch))
    for q in range(0, 400, 37):
        E = 0.5 * mr * g[q] ** 2 / W.KB
        assert abs(ch[q] - orc.chi(P, b[q] * 1e10, E)) < 1e-11
    # head-on collisions reflect, grazing ones barely deflect
    assert abs(orc.chi(P, 0.0, 1000.0) - math.pi) < 1e-13
    assert abs(orc.chi(P, 10.0, 1e5)) < 1e-3
