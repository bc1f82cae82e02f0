"""Pins of the oracle's deflection angle chi(b, E).

Checked against: the hard-sphere closed form chi = 2 arccos(b/d); V = 0;
the inverse-square and Coulomb closed forms; a 30-digit mpmath evaluation of
the deflection integral for the Jager-form potential (a different
substitution and quadrature), also on orbiting pairs (|chi| > pi); and
brute-force integration of the pair trajectory (relative-motion ODE) on a
few inputs.  Also the impact parameter from the latents and the rotation of
v_r by chi.
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


def _mp_V(r):
    """The Jager-form potential (placeholder coefficients) in mpmath
    arithmetic, written out from eqs. jager_potential and damping."""
    import mpmath as mp
    p = W.JAGER_PLACEHOLDER
    if r < mp.mpf("0.4") * p.R_eps:
        return p.A_sr / r * mp.exp(-p.a_sr * r)
    rep = p.A * mp.exp(p.a1 * r + p.a2 * r * r + p.am1 / r + p.am2 / (r * r))
    x = p.beta_tt * r
    sums, term, s = [mp.mpf(1)], mp.mpf(1), mp.mpf(1)
    for k in range(1, 17):  # partial sums of the series of e^x
        term = term * x / k
        s = s + term
        sums.append(s)
    ex = mp.exp(-x)
    disp = 0
    for n in range(3, 9):
        disp += (1 - ex * sums[2 * n]) * p.C[n - 3] / r ** (2 * n)
    return rep - disp


def _mp_chi(b, E, dps=30, n_pan=32):
    """chi(b, E) at 30 digits, independent of the oracle's scheme.

    r_min is the largest zero of D(r) = 1 - b^2/r^2 - V(r)/E: a downward scan
    (steps of 2e-4 relative) that also minimises D at every local minimum it
    passes, so a dip of D below zero narrower than a step (the outer root of
    a nearly orbiting pair) is not stepped over; then a high-precision root.
    The integral over r is taken with u = r_min / r = sin(phi), phi in
    [0, pi/2], which leaves the smooth integrand cos(phi) / sqrt(D(r_min /
    sin phi)) (a different substitution from the oracle's), by tanh-sinh on
    n_pan equal panels.  At the pairs below, 32 and 128 panels agree to all
    printed digits, also where the integrand has the sharp interior peak of a
    nearly orbiting pair."""
    import mpmath as mp
    mp.mp.dps = dps
    b = mp.mpf(b)
    E = mp.mpf(E)

    def D(r):
        return 1 - b * b / (r * r) - _mp_V(r) / E

    r = max(b, mp.findroot(_mp_V, 3.3)) * mp.mpf("1.0001")  # beyond it D > 0
    q = 1 - mp.mpf("2e-4")
    d2, d1, r1 = None, D(r), r
    while True:
        r0 = r1 * q
        d0 = D(r0)
        if d0 <= 0:
            lo, hi = r0, r1
            break
        if d2 is not None and d1 < d2 and d1 < d0:  # local minimum of D near r1
            rm = mp.findroot(lambda x: mp.diff(D, x), r1)
            if r0 < rm < r1 / q and D(rm) < 0:
                lo, hi = rm, r1 / q
                break
        d2, d1, r1 = d1, d0, r0
    rmin = mp.findroot(D, (lo, hi), solver="anderson")

    def f(ph):
        if ph <= 0:
            return mp.mpf(0)
        d = D(rmin / mp.sin(ph))
        return mp.cos(ph) / mp.sqrt(d) if d > 0 else mp.mpf(0)

    I = mp.quad(f, mp.linspace(0, mp.pi / 2, n_pan + 1))
    return float(mp.pi - 2 * (b / rmin) * I)


# The last two: high-energy pairs of the 2^20-pair batch of seed 2 whose
# turning point lies just inside the switch between the two branches of the
# potential (0.4 R_eps), so the integrand's first nodes straddle it.
@pytest.mark.parametrize("g,b", [(2743.87, 9.472), (498.07, 5.2766), (120.81, 7.176),
                                 (312.92, 4.003), (2567.27, 2.096), (19528.8, 0.7),
                                 (15687.361230336597, 0.925757711954615),
                                 (14749.692948604592, 0.8179355689506196)])
def test_jager_against_mpmath(orc, g, b):
    P = orc.potential_jager(W.JAGER_PLACEHOLDER)
    E = 0.5 * (W.AR_MASS / 2) * g * g / W.KB
    ref = _mp_chi(b, E)
    assert abs(orc.chi(P, b, E) - ref) < 1e-11


# Pairs with |chi| > pi (orbiting): the four deepest of the 8192-pair
# deflection batch of seed 21 (inner turning point, D has a positive minimum
# just outside it), and two of the 2^20-pair batch of seed 2 whose turning
# point is the outer root of a narrow dip of D below zero.
ORBITING = [(103.57376810723666, 8.079814274291563), (137.77047932098122, 7.3909200524353995),
            (329.61966362185007, 5.6092124815582896), (158.3846329044944, 7.0679805139823095),
            (103.39603267872018, 8.089059700682917), (109.73764407706153, 7.939459649590853)]


@pytest.mark.parametrize("g,b", ORBITING)
def test_jager_orbiting_against_mpmath(orc, g, b):
    """chi beyond a half-turn.  Bound 1e-10 rad: near orbiting chi is
    ill-conditioned in the potential (at the first pair a relative change of V
    by 1e-13 moves chi by 3e-11 rad, from the mpmath reference), and the
    oracle's FP64 V carries relative rounding of ~1e-14 near r_min."""
    P = orc.potential_jager(W.JAGER_PLACEHOLDER)
    E = 0.5 * (W.AR_MASS / 2) * g * g / W.KB
    ref = _mp_chi(b, E)
    got = orc.chi(P, b, E)
    assert abs(ref) > math.pi
    assert abs(got - ref) < 1e-10, (g, b, got, ref)


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


def test_impact_from_z_closed_form(orc):
    """b = b_max sqrt(1 - exp(-|z|^2/2)): hand values, and b^2 / b_max^2
    uniform on [0, 1) for z ~ N(0, I_2) (|z|^2 / 2 is Exp(1))."""
    from scipy import stats
    bm = 1e-9
    assert orc.impact_from_z(np.array([0.0, 0.0]), bm) == 0.0
    # |z|^2 = 2 ln 2 -> b^2 = b_max^2 / 2
    z = np.array([math.sqrt(2 * math.log(2.0)), 0.0])
    assert abs(orc.impact_from_z(z, bm) - bm / math.sqrt(2.0)) < 1e-24
    z = np.array([0.6, -0.8])  # |z|^2 = 1
    assert abs(orc.impact_from_z(z, bm) - bm * math.sqrt(1 - math.exp(-0.5))) < 1e-24
    assert abs(orc.impact_from_z(np.array([40.0, 0.0]), bm) - bm) < 1e-24
    rng = np.random.default_rng(8)
    zz = rng.standard_normal((200_000, 2))
    b = orc.impact_from_z(zz, bm)
    assert b.shape == (200_000,) and np.all((b >= 0) & (b < bm))
    assert stats.kstest((b / bm) ** 2, "uniform").pvalue > 1e-3


def test_rotate_against_pair_update(orc):
    """rotate(v_r, chi, xi) against the oracle's Phase-B pair update with
    angles (C code): one pair per cell, v_i' - v_j' must equal the rotated
    v_r; plus the geometry of the rotation: |v_r'| = g, the angle between v_r
    and v_r' is |chi| folded to [0, pi], v_r' lies in the plane of v_r and xi
    on the side of xi for 0 < chi < pi, chi = 0 and pi give v_r and -v_r."""
    rng = np.random.default_rng(5)
    m = 500
    vr = rng.standard_normal((m, 3)) * 300.0
    xi = rng.standard_normal((m, 3))
    chi_ = rng.uniform(-7.0, 7.0, m)
    chi_[:3] = [0.0, math.pi, 0.5 * math.pi]
    out = orc.rotate(vr, chi_, xi)
    # the pair update: particles 2p, 2p+1 with v_i - v_j = vr, pair p in cell p
    v = np.zeros((3, 2 * m))
    vcm = rng.standard_normal((m, 3)) * 100.0
    v[:, 0::2] = (vcm + 0.5 * vr).T
    v[:, 1::2] = (vcm - 0.5 * vr).T
    sel = {"pair_off": np.arange(m, dtype=np.int32), "pair_cnt": np.ones(m, np.int32),
           "pair_i": np.arange(0, 2 * m, 2, dtype=np.int32),
           "pair_j": np.arange(1, 2 * m, 2, dtype=np.int32),
           "pair_cell": np.arange(m, dtype=np.int32)}
    vn = orc.apply_chi(sel, v, np.cos(chi_), np.sin(chi_), xi)
    vr_new = (vn[:, 0::2] - vn[:, 1::2]).T
    np.testing.assert_allclose(vr_new, out, rtol=0, atol=1e-9)
    g = np.linalg.norm(vr, axis=1)
    assert np.max(np.abs(np.linalg.norm(out, axis=1) - g) / g) < 1e-14
    cosang = np.sum(out * vr, axis=1) / (g * g)
    ang = np.arccos(np.clip(cosang, -1, 1))
    assert np.max(np.abs(ang - orc.fold(chi_))) < 1e-7
    nrm = np.cross(vr, xi)
    assert np.max(np.abs(np.sum(out * nrm, axis=1)) / (g * np.linalg.norm(nrm, axis=1))) < 1e-13
    s = np.sin(chi_)
    side = np.sum(out * xi, axis=1) - np.cos(chi_) * np.sum(vr * xi, axis=1)
    ok = np.abs(s) > 1e-6
    assert np.all(np.sign(side[ok]) == np.sign(s[ok]))
    np.testing.assert_allclose(out[0], vr[0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(out[1], -vr[1], rtol=0, atol=1e-10)
