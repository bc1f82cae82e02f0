"""Pins of the oracle's flow loop around the collision step (section "Results
and Discussion": Couette channel and lid-driven cavity): free flight and wall
events against closed forms and the wall Maxwellian, sampling and the
macroscopic-field formulas against direct computation, and the Couette
profile's qualitative shape."""
import math

import numpy as np
import pytest

import workloads as W


def _dom(orc, nx, ny, L, kinds, T=273.0, u_w=((0, 0, 0),) * 4):
    return orc.domain(nx, ny, L, L, kinds, (T,) * 4, u_w, W.AR_MASS)


def test_free_flight_periodic_box(orc):
    rng = np.random.default_rng(1)
    n, L, dt = 5000, 1e-3, 3e-6
    dom = _dom(orc, 7, 5, L, (W.WALL_PERIODIC,) * 4)
    pos = rng.uniform(0, L, (2, n))
    v = rng.normal(0, 400, (3, n))
    p2, v2, cell, stuck, hits = orc.move(dom, pos, v, dt, 3, 4)
    assert stuck == 0
    assert np.array_equal(v2, v)
    want = np.mod(pos + v[:2] * dt, L)
    d = np.abs(p2 - want)
    d = np.minimum(d, L - d)                       # the same point across the seam
    assert d.max() < 1e-15
    ix = np.minimum((p2[0] * 7 / L).astype(int), 6)
    iy = np.minimum((p2[1] * 5 / L).astype(int), 4)
    assert np.array_equal(cell, iy * 7 + ix)


def test_specular_walls_closed_form(orc):
    L = 1.0
    dom = _dom(orc, 4, 4, L, (W.WALL_SPECULAR,) * 4)
    # x: 0.3 + 1.0 t hits x = 1 at t = 0.7, returns for 0.3 -> 0.7 (velocity -1);
    # y: 0.9 - 0.25 t stays inside
    pos = np.array([[0.3], [0.9]])
    v = np.array([[1.0], [-0.25], [3.0]])
    p2, v2, cell, stuck, hits = orc.move(dom, pos, v, 1.0, 0, 0)
    assert hits == 1
    assert p2[0, 0] == pytest.approx(0.7, abs=1e-15) and p2[1, 0] == pytest.approx(0.65, abs=1e-15)
    assert np.array_equal(v2[:, 0], [-1.0, -0.25, 3.0])
    # many particles and bounces: speeds kept exactly, positions inside
    rng = np.random.default_rng(2)
    pos = rng.uniform(0, L, (2, 4000))
    v = rng.normal(0, 1.3, (3, 4000))
    p2, v2, cell, stuck, hits = orc.move(dom, pos, v, 1.0, 0, 0)
    assert stuck == 0 and hits > 1000
    assert np.array_equal(np.abs(v2), np.abs(v))
    assert p2.min() >= 0.0 and p2.max() <= L


def test_diffuse_wall_draws_the_wall_maxwellian(orc):
    from scipy import stats
    n, L, T = 200_000, 1.0, 350.0
    uw = ((0, 0, 0), (0, 0, 0), (120.0, 0.0, 0.0), (0, 0, 0))
    dom = _dom(orc, 1, 1, L, (W.WALL_PERIODIC, W.WALL_PERIODIC, W.WALL_DIFFUSE,
                              W.WALL_SPECULAR), T=T, u_w=uw)
    # every particle reaches y = 0 within dt and leaves it once (no second hit)
    pos = np.stack([np.linspace(0.1, 0.9, n), np.full(n, 1e-6)])
    v = np.stack([np.zeros(n), np.full(n, -1.0), np.zeros(n)])
    dt = 2e-6
    p2, v2, cell, stuck, hits = orc.move(dom, pos, v, dt, 11, 5)
    assert hits == n
    sw = math.sqrt(W.KB * T / W.AR_MASS)
    assert np.all(v2[1] > 0)
    # normal component: Rayleigh(sigma_w) (flux-weighted half-range Maxwellian)
    assert stats.kstest(v2[1] / sw, "rayleigh").pvalue > 1e-3
    # tangential: N(u_w, sigma_w^2) in x, N(0, sigma_w^2) in z
    for comp, mean in ((0, 120.0), (2, 0.0)):
        x = v2[comp]
        assert abs(x.mean() - mean) < 5 * sw / math.sqrt(n)
        assert abs(x.var() / sw ** 2 - 1.0) < 5 * math.sqrt(2.0 / n)
        assert stats.kstest((x - mean) / sw, "norm").pvalue > 1e-3


def test_closed_diffuse_box_stays_at_wall_temperature(orc):
    rng = np.random.default_rng(4)
    n, L, T = 40_000, 1e-3, 300.0
    dom = _dom(orc, 4, 4, L, (W.WALL_DIFFUSE,) * 4, T=T)
    pos = rng.uniform(0, L, (2, n))
    v = rng.normal(0, math.sqrt(W.KB * T / W.AR_MASS), (3, n))
    dt = 2e-7
    acc = None
    for step in range(60):
        pos, v, cell, stuck, hits = orc.move(dom, pos, v, dt, 9, step)
        assert stuck == 0
        cs, perm, _ = orc.sort_cells(cell, 16)
        pos, v = pos[:, perm], v[:, perm]
        if step >= 20:
            acc = orc.sample(cs, v, acc)
    f = orc.fields(acc.sum(axis=0, keepdims=True), 40, W.AR_MASS, 1.0)
    assert f[0, 4] == pytest.approx(T, rel=0.01)
    assert np.all(np.abs(f[0, 1:4]) < 5.0)
    counts = acc[:, 0] / 40
    assert np.all(np.abs(counts / counts.mean() - 1) < 0.05)


def test_sampling_sums_and_field_formulas(orc):
    rng = np.random.default_rng(5)
    n_cells = 30
    counts = rng.integers(0, 200, n_cells)
    cs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    v = rng.normal(0, 300, (3, cs[-1])) + rng.normal(0, 80, (3, 1))
    v[1] += 0.4 * v[0]                                 # sheared, correlated
    acc = orc.sample(cs, v)
    acc = orc.sample(cs, v, acc)                       # two identical samples
    fpv = 7.0
    f = orc.fields(acc, 2, W.AR_MASS, fpv)
    for k in range(n_cells):
        a, b = cs[k], cs[k + 1]
        if b == a:
            assert np.all(f[k] == 0)
            continue
        vk = v[:, a:b]
        N = b - a
        assert acc[k, 0] == 2 * N
        np.testing.assert_allclose(acc[k, 1:4], 2 * vk.sum(axis=1), rtol=1e-12, atol=1e-9)
        u = vk.mean(axis=1)
        c = vk - u[:, None]
        c2 = np.sum(c * c, axis=0)
        dens = N * fpv
        rho = dens * W.AR_MASS
        np.testing.assert_allclose(f[k, 0], dens, rtol=1e-14)
        np.testing.assert_allclose(f[k, 1:4], u, rtol=1e-10, atol=1e-9)
        np.testing.assert_allclose(f[k, 4], W.AR_MASS * c2.mean() / (3 * W.KB), rtol=1e-9)
        np.testing.assert_allclose(f[k, 5], -rho * np.mean(c[0] * c[1]),
                                   rtol=1e-7, atol=1e-9 * rho * c2.mean())
        q = 0.5 * rho * np.mean(c2 * c, axis=1)
        scale = 0.5 * rho * np.mean(c2 ** 1.5)
        np.testing.assert_allclose(f[k, 6:9], q, rtol=0, atol=1e-8 * scale)


def test_maxwellian_has_no_stress_or_heat_flux(orc):
    rng = np.random.default_rng(6)
    n, T = 400_000, 300.0
    s = math.sqrt(W.KB * T / W.AR_MASS)
    v = rng.normal(0, s, (3, n))
    v[0] += 50.0
    cs = np.array([0, n], np.int32)
    f = orc.fields(orc.sample(cs, v), 1, W.AR_MASS, 1.0)[0]
    assert f[4] == pytest.approx(T, rel=5 * math.sqrt(2.0 / (3 * n)))
    p = W.AR_MASS * s * s * n
    assert abs(f[5]) < 5 * p / math.sqrt(n)
    assert np.all(np.abs(f[6:9]) < 5 * W.AR_MASS * s ** 3 * n * math.sqrt(15.0 / n))


@pytest.mark.timeout(300)
def test_couette_profile_shape(orc):
    """Short oracle run of the Couette case: antisymmetric velocity profile,
    slip at both walls, shear heating above the wall temperature."""
    fl = W.couette_flow(seed=3, ny=16, ppc=60, kn=0.5, u_wall=500.0)
    dom = orc.domain(fl.nx, fl.ny, fl.Lx, fl.Ly, fl.kinds, fl.T_w, fl.u_w, W.AR_MASS)
    pos, v = fl.pos, fl.v
    acc = None
    for step in range(900):
        pos, v, cs, info = orc.flow_step(dom, pos, v, fl.xs, fl.lam, fl.dt, 21, step)
        if step >= 500:
            acc = orc.sample(cs, v, acc)
    f = orc.fields(acc, 400, W.AR_MASS, fl.fnum_per_volume)
    ux, T = f[:, 1], f[:, 4]
    assert ux[0] < -100 and ux[-1] > 100              # dragged by the walls
    assert ux[0] > -500 and ux[-1] < 500              # velocity slip at both walls
    assert np.all(np.diff(ux) > -60)                  # increasing across the channel
    assert abs(ux.mean()) < 40                        # antisymmetric about the middle
    assert T[len(T) // 2] > 290                       # viscous heating above 273 K
