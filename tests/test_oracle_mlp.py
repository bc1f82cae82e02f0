"""Pins of the oracle's network parts: forward, projection, loss, gradients,
moment-match adjoint, Adam and the cosine schedule.

Gradients are checked by central finite differences; the forward pass by a
hand-worked example and by a special case that must reproduce the isotropic
scattering law exactly.
"""
import math

import numpy as np
import pytest

import workloads as W


def test_forward_hand_worked(orc):
    # 2 -> 2 -> 1.  x=(3,1): z1 = (3-1, 6+0.5-1) = (2, 5.5)
    W1 = np.array([[1.0, -1.0], [2.0, 0.5]])
    b1 = np.array([0.0, -1.0])
    W2 = np.array([[1.0, -2.0]])
    b2 = np.array([0.5])
    x = np.array([[3.0, 1.0], [-1.0, 2.0]])
    y = orc.mlp_forward([W1, W2], [b1, b2], x, act="relu")
    assert y[0, 0] == 2.0 - 11.0 + 0.5
    assert y[1, 0] == 0.5            # both hidden units negative -> output = bias
    ys = orc.mlp_forward([W1, W2], [b1, b2], x, act="silu")
    silu = lambda t: t / (1.0 + math.exp(-t))
    assert abs(ys[0, 0] - (silu(2.0) - 2.0 * silu(5.5) + 0.5)) < 1e-15
    assert abs(ys[1, 0] - (silu(-3.0) - 2.0 * silu(-2.0) + 0.5)) < 1e-15


def test_relu_passthrough_reproduces_isotropic_rule(orc):
    # Weights that route xi through unchanged (xi = relu(xi) - relu(-xi)) make
    # the surrogate output u = xi/|xi|, an isotropic direction independent of
    # v_r: cos(chi) must be uniform (KS), as for the VHS law.
    from scipy import stats
    W1 = np.zeros((6, 8))
    W1[0:3, 3:6] = np.eye(3)
    W1[3:6, 3:6] = -np.eye(3)
    W2 = np.concatenate([np.eye(3), -np.eye(3)], axis=1)
    rows = W.training_rows(seed=5, n=20000)
    x = orc.network_input(rows["vr"], rows["xi"], rows["z"], rows["sigma_v"])
    y = orc.mlp_forward([W1, W2], [np.zeros(6), np.zeros(3)], x, act="relu")
    np.testing.assert_allclose(y, rows["xi"], rtol=0, atol=1e-15)
    vn, u, _ = orc.project(y, rows["g"])
    cosc = np.sum(u * rows["vr"], axis=1) / rows["g"]
    assert stats.kstest(cosc, "uniform", args=(-1, 2)).pvalue > 1e-3
    np.testing.assert_allclose(np.linalg.norm(vn, axis=1), rows["g"], rtol=1e-14)


def _loss(orc, Ws, bs, x, g, target, sv, act, kind="velocity"):
    y = orc.mlp_forward(Ws, bs, x, act)
    vn, _, _ = orc.project(y, g)
    if kind == "direction":
        return orc.direction_loss(vn, target)
    return orc.surrogate_loss(vn, target, sv)


def test_direction_loss_closed_form(orc):
    """Two unit-speed directions at angle a: |u - u*|^2 / 4 = (1 - cos a) / 2,
    whatever the common speed g; the mean over rows; gradient by central
    differences."""
    rng = np.random.default_rng(3)
    a = rng.uniform(0, np.pi, 50)
    g = 10 ** rng.uniform(2, 4, 50)
    t = np.stack([g, np.zeros(50), np.zeros(50)], axis=1)
    v = np.stack([g * np.cos(a), g * np.sin(a), np.zeros(50)], axis=1)
    assert orc.direction_loss(v, t) == pytest.approx(np.mean((1 - np.cos(a)) / 2), rel=1e-13)
    G = orc.direction_loss_grad(v, t)
    h = 1e-3
    for (i, d) in [(0, 0), (7, 1), (49, 2)]:
        vp, vm = v.copy(), v.copy()
        vp[i, d] += h
        vm[i, d] -= h
        fd = (orc.direction_loss(vp, t) - orc.direction_loss(vm, t)) / (2 * h)
        assert abs(fd - G[i, d]) < 1e-9 * max(1.0, abs(fd)) + 1e-14


@pytest.mark.parametrize("act,kind", [("silu", "velocity"), ("relu", "velocity"),
                                      ("silu", "direction")])
def test_gradients_against_finite_differences(orc, act, kind):
    rng = np.random.default_rng(12)
    Ws, bs = W.mlp_init(3, W.FD_DIMS)
    rows = W.training_rows(seed=6, n=64)
    x = orc.network_input(rows["vr"], rows["xi"], rows["z"], rows["sigma_v"])
    g = rows["g"]
    target = rng.normal(0, 1, (64, 3)) * g[:, None]
    sv = rows["sigma_v"]
    y = orc.mlp_forward(Ws, bs, x, act)
    vn, _, _ = orc.project(y, g)
    G = (orc.direction_loss_grad(vn, target) if kind == "direction"
         else orc.surrogate_loss_grad(vn, target, sv))
    dy = orc.project_backward(G, y, g)
    dW, db, dx = orc.mlp_backward(Ws, bs, x, dy, act)
    h = 1e-6
    for l in range(len(Ws)):
        for (i, j) in [(0, 0), (1, 3), (Ws[l].shape[0] - 1, Ws[l].shape[1] - 1), (2, 5)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][i, j] += h
            Wm[l][i, j] -= h
            fd = (_loss(orc, Wp, bs, x, g, target, sv, act, kind) -
                  _loss(orc, Wm, bs, x, g, target, sv, act, kind)) / (2 * h)
            assert abs(fd - dW[l][i, j]) <= 1e-6 * max(1.0, abs(fd)), (l, i, j, fd, dW[l][i, j])
        for i in [0, bs[l].shape[0] - 1]:
            bp = [b.copy() for b in bs]
            bm = [b.copy() for b in bs]
            bp[l][i] += h
            bm[l][i] -= h
            fd = (_loss(orc, Ws, bp, x, g, target, sv, act, kind) -
                  _loss(orc, Ws, bm, x, g, target, sv, act, kind)) / (2 * h)
            assert abs(fd - db[l][i]) <= 1e-6 * max(1.0, abs(fd))
    # input gradient
    for (r, c) in [(0, 0), (5, 7), (63, 3)]:
        xp = x.copy()
        xm = x.copy()
        xp[r, c] += h
        xm[r, c] -= h
        fd = (_loss(orc, Ws, bs, xp, g, target, sv, act, kind) -
              _loss(orc, Ws, bs, xm, g, target, sv, act, kind)) / (2 * h)
        assert abs(fd - dx[r, c]) <= 1e-6 * max(1.0, abs(fd))


def test_moment_match_adjoint_against_finite_differences(orc):
    rng = np.random.default_rng(4)
    v_pre = rng.normal(0, 300, (7, 3))
    v = v_pre + rng.normal(0, 40, (7, 3))
    w = rng.normal(0, 1, (7, 3))

    def L(vv):
        return float(np.sum(w * orc.moment_match_group(vv, v_pre)))

    G = orc.moment_match_group_backward(w, v, v_pre)
    h = 1e-4
    for m in range(7):
        for q in range(3):
            vp = v.copy()
            vm = v.copy()
            vp[m, q] += h
            vm[m, q] -= h
            fd = (L(vp) - L(vm)) / (2 * h)
            assert abs(fd - G[m, q]) < 1e-8 * max(1.0, abs(fd))


def test_adam_first_step_and_cosine_schedule(orc):
    rng = np.random.default_rng(1)
    p = [rng.normal(size=(4, 3))]
    g = [rng.normal(size=(4, 3))]
    m = [np.zeros((4, 3))]
    s = [np.zeros((4, 3))]
    p0 = p[0].copy()
    orc.adam_step(p, g, m, s, t=1, lr=1e-3, eps=1e-8)
    # bias correction makes the first step lr * g / (|g| + eps)
    np.testing.assert_allclose(p[0], p0 - 1e-3 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-14)
    assert orc.cosine_lr(0, 100, 1e-3) == 1e-3
    assert abs(orc.cosine_lr(100, 100, 1e-3) - 1e-6) < 1e-18
    assert abs(orc.cosine_lr(50, 100, 1e-3) - 0.5 * (1e-3 + 1e-6)) < 1e-15
