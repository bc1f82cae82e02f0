"""Pins of the oracle's angle network, Huber loss, deflection-angle table and
table rule (sections "Neural Network Architecture", "Neural Surrogate
Training" and "Runtime Acceleration via Neural Table Look-up") against closed
forms, finite differences and special cases."""
import math

import numpy as np
import pytest

import workloads as W


def test_softplus_and_sigmoid_closed_forms(orc):
    assert orc.softplus(0.0) == pytest.approx(math.log(2.0), abs=1e-15)
    assert orc.softplus(50.0) == pytest.approx(50.0, abs=1e-15)
    assert orc.softplus(-50.0) == pytest.approx(math.exp(-50.0), rel=1e-12)
    z = np.linspace(-8, 8, 41)
    h = 1e-6
    fd = (orc.softplus(z + h) - orc.softplus(z - h)) / (2 * h)
    np.testing.assert_allclose(orc.sigmoid(z), fd, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(orc.sigmoid(z), 1.0 / (1.0 + np.exp(-z)), rtol=1e-14, atol=1e-18)


def test_huber_piecewise_values_and_gradient(orc):
    # small residuals: 0.5 d^2; large: |d| - 0.5; continuous at |d| = 1
    assert orc.huber_loss([0.25], [0.0]) == pytest.approx(0.03125, abs=1e-16)
    assert orc.huber_loss([0.0], [3.0]) == pytest.approx(2.5, abs=1e-16)
    assert orc.huber_loss([1.0 - 1e-12], [0.0]) == pytest.approx(0.5, abs=1e-11)
    assert orc.huber_loss([1.0 + 1e-12], [0.0]) == pytest.approx(0.5, abs=1e-11)
    rng = np.random.default_rng(3)
    yh = rng.normal(0, 2, 64)
    y = rng.normal(0, 2, 64)
    g = orc.huber_grad(yh, y)
    h = 1e-6
    for q in range(0, 64, 7):
        e = np.zeros(64)
        e[q] = h
        fd = (orc.huber_loss(yh + e, y) - orc.huber_loss(yh - e, y)) / (2 * h)
        assert g[q] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_angle_net_hand_worked(orc):
    # 2 -> 2 (SiLU) -> 1 (Softplus), worked by hand
    W1 = np.array([[1.0, -2.0], [0.5, 0.0]])
    b1 = np.array([0.0, 1.0])
    W2 = np.array([[2.0, -1.0]])
    b2 = np.array([0.25])
    x = np.array([[0.5, 0.25]])
    z1 = np.array([0.5 - 0.5, 0.25 + 1.0])      # [0, 1.25]
    h1 = z1 / (1.0 + np.exp(-z1))                # [0, 1.25 sigmoid(1.25)]
    z2 = 2.0 * h1[0] - h1[1] + 0.25
    want = math.log1p(math.exp(z2))
    assert orc.angle_net_forward([W1, W2], [b1, b2], x)[0] == pytest.approx(want, abs=1e-15)


def test_angle_net_backward_matches_finite_differences(orc):
    Ws, bs = W.mlp_init(5, (2, 7, 5, 1))
    rng = np.random.default_rng(8)
    x = rng.uniform(-1, 1, (9, 2))
    dy = rng.normal(0, 1, 9)
    dW, db, dx = orc.angle_net_backward(Ws, bs, x, dy)

    def f(Ws_, bs_, x_):
        return float(np.sum(dy * orc.angle_net_forward(Ws_, bs_, x_)))

    h = 1e-6
    for l in range(len(Ws)):
        for (a, c) in [(0, 0), (Ws[l].shape[0] - 1, Ws[l].shape[1] - 1)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][a, c] += h
            Wm[l][a, c] -= h
            fd = (f(Wp, bs, x) - f(Wm, bs, x)) / (2 * h)
            assert dW[l][a, c] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][0] += h
        bm[l][0] -= h
        fd = (f(Ws, bp, x) - f(Ws, bm, x)) / (2 * h)
        assert db[l][0] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    xp = x.copy()
    xm = x.copy()
    xp[3, 1] += h
    xm[3, 1] -= h
    assert dx[3, 1] == pytest.approx((f(Ws, bs, xp) - f(Ws, bs, xm)) / (2 * h), rel=1e-6, abs=1e-9)


def test_angle_input_normalisation(orc):
    lo, hi = math.log(5.0), math.log(5e5)
    x = orc.angle_net_input([5.0, 5e5, math.sqrt(5.0 * 5e5)], [0.0, 1.0, 0.5], lo, hi)
    np.testing.assert_allclose(x[:, 0], [-1.0, 1.0, 0.0], atol=1e-14)
    np.testing.assert_allclose(x[:, 1], [0.0, 1.0, 0.5], atol=0)


def test_angle_rows_energy_and_target(orc):
    m_red = W.AR_MASS / 2
    g = np.array([1000.0])
    E = 0.5 * m_red * 1e6 / W.KB
    x, y = orc.angle_rows([2e-10], g, np.array([-0.3]), m_red, 0.0, 2 * math.log(E), 1e-9)
    assert x[0, 0] == pytest.approx(0.0, abs=1e-13)      # ln E at the middle of [0, 2 ln E]
    assert x[0, 1] == pytest.approx(0.2, abs=1e-15)
    assert y[0] == pytest.approx(math.log1p(0.3), abs=1e-15)   # theta = |chi| for |chi| <= pi


def test_chi_table_of_constant_network(orc):
    # zero hidden weights: y = softplus(b_out) everywhere, theta = e^{b_out}
    Ws, bs = W.mlp_init(2, (2, 6, 4, 1))
    Ws = [np.zeros_like(w) for w in Ws]
    bs = [np.zeros_like(b) for b in bs]
    bs[-1][0] = math.log(0.7)
    t = orc.chi_table(Ws, bs, 5, 4, 0.0, 3.0)
    np.testing.assert_allclose(t, 0.7, rtol=1e-14)
    bs[-1][0] = 5.0     # e^5 > pi: clipped
    np.testing.assert_allclose(orc.chi_table(Ws, bs, 3, 3, 0.0, 3.0), math.pi, rtol=0)


def test_table_lookup_reproduces_bilinear_functions(orc):
    n_e, n_b, lo, hi = 33, 17, math.log(3.0), math.log(3e4)
    lnE, brel = orc.table_grid(n_e, n_b, lo, hi)
    a, b, c, d = 0.3, 0.01, -0.2, 0.05
    f = lambda le, br: a + b * le + c * br + d * le * br
    T = f(lnE[:, None], brel[None, :])
    rng = np.random.default_rng(4)
    E = np.exp(rng.uniform(lo, hi, 500))
    br = rng.uniform(0, 1, 500)
    np.testing.assert_allclose(orc.table_lookup(T, lo, hi, E, br), f(np.log(E), br), atol=1e-13)
    # nodes give the entries; outside the grid the edge values
    np.testing.assert_allclose(orc.table_lookup(T, lo, hi, np.exp(lnE[5]) * np.ones(n_b), brel),
                               T[5], atol=1e-13)
    assert orc.table_lookup(T, lo, hi, [1e-3], [2.0])[0] == pytest.approx(T[0, -1], abs=1e-14)
    assert orc.table_lookup(T, lo, hi, [1e9], [-1.0])[0] == pytest.approx(T[-1, 0], abs=1e-14)


def test_table_rule_special_angles(orc):
    pop = W.ragged_population(12, 40, 30, empty_frac=0.1)
    cs, perm, _ = orc.sort_cells(pop.cell_of, pop.n_cells)
    v = pop.v[:, perm]
    m_red = W.AR_MASS / 2
    zero = {"theta": np.zeros((4, 4)), "lne_lo": 0.0, "lne_hi": 12.0}
    vn, info = orc.step(cs, v, pop.xs, pop.lam, 3, 1, rule="table", table=zero, m_red=m_red)
    assert int(info["sel"]["pair_cnt"].sum()) > 0
    np.testing.assert_allclose(vn, v, rtol=0, atol=1e-9)       # theta = 0: no change
    flip = {"theta": np.full((4, 4), math.pi), "lne_lo": 0.0, "lne_hi": 12.0}
    vn, info = orc.step(cs, v, pop.xs, pop.lam, 3, 1, rule="table", table=flip, m_red=m_red)
    # theta = pi: v_r' = -v_r, so a cell with one accepted pair swaps the two
    # particles' velocities
    sel = info["sel"]
    one = np.flatnonzero(sel["pair_cnt"] == 1)
    assert len(one) > 0
    for k in one:
        p = sel["pair_off"][k]
        i, j = sel["pair_i"][p], sel["pair_j"][p]
        np.testing.assert_allclose(vn[:, i], v[:, j], rtol=1e-12, atol=1e-9)
        np.testing.assert_allclose(vn[:, j], v[:, i], rtol=1e-12, atol=1e-9)
