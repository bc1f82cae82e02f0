"""GPU parity of the flow loop around the collision step (Couette channel,
lid-driven cavity): move with wall events, gather, sampling and fields
against the FP64 oracle, a multi-step cavity run step by step against the
oracle's loop, and the Couette profile shape from a longer GPU run."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_21244_amd import _lib
    _lib.load()
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def api(dev):
    from paper_2602_21244_amd import api as A
    return A


CASES = {
    "couette": ((W.WALL_PERIODIC, W.WALL_PERIODIC, W.WALL_DIFFUSE, W.WALL_DIFFUSE),
                ((0, 0, 0), (0, 0, 0), (-500.0, 0, 0), (500.0, 0, 0))),
    "cavity": ((W.WALL_DIFFUSE,) * 4, ((0, 0, 0), (0, 0, 0), (0, 0, 0), (100.0, 0, 0))),
    "specular": ((W.WALL_SPECULAR,) * 4, ((0, 0, 0),) * 4),
    "mixed": ((W.WALL_SPECULAR, W.WALL_DIFFUSE, W.WALL_PERIODIC, W.WALL_PERIODIC),
              ((0, 0, 0), (0, 40.0, 10.0), (0, 0, 0), (0, 0, 0))),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_move_matches_oracle(orc, dev, api, case, dtype):
    say("move", case, dtype)
    kinds, uw = CASES[case]
    rng = np.random.default_rng(list(CASES).index(case) + 40)
    n, L, nx, ny = 60_000, 1e-3, 13, 9
    T = (273.0, 300.0, 250.0, 350.0)
    pos = rng.uniform(0, L, (2, n))
    v = rng.normal(0, 400, (3, n))
    v[0] += 200.0
    if dtype == torch.float32:
        pos = pos.astype(np.float32).astype(np.float64)
        v = v.astype(np.float32).astype(np.float64)
    dt = 1.5e-6                                   # ~0.6 box widths: many wall events
    dom_o = orc.domain(nx, ny, L, L, kinds, T, uw, W.AR_MASS)
    p_o, v_o, c_o, stuck_o, hits_o = orc.move(dom_o, pos, v, dt, 12, 34)
    dom = api.domain(nx, ny, L, L, kinds, T, uw, W.AR_MASS)
    pg = torch.as_tensor(pos, dtype=dtype, device=dev).contiguous()
    vg = torch.as_tensor(v, dtype=dtype, device=dev).contiguous()
    st = api.new_status(dev)
    cg = api.move(pg, vg, dom, dt, 12, 34, st=st).cpu().numpy()
    s = api.read_status(st)
    say(f"  wall events {s.wall_events} (oracle {hits_o}), limit {s.wall_limit} ({stuck_o})")
    pg, vg = pg.double().cpu().numpy(), vg.double().cpu().numpy()
    if dtype == torch.float64:
        assert s.wall_events == hits_o and s.wall_limit == stuck_o
        assert np.array_equal(cg, c_o)
        np.testing.assert_allclose(pg, p_o, rtol=0, atol=1e-12 * L)
        np.testing.assert_allclose(vg, v_o, rtol=1e-12, atol=1e-9)
    else:
        # FP32 storage of the FP64 result; a few wall events may differ in the
        # last bit of a stored input, so compare particle by particle
        np.testing.assert_allclose(pg, p_o.astype(np.float32), rtol=0, atol=4e-7 * L)
        np.testing.assert_allclose(vg, v_o.astype(np.float32), rtol=2e-6, atol=1e-3)
        ix = np.minimum((pg[0].astype(np.float32).astype(np.float64) * (nx / L)).astype(int), nx - 1)
        iy = np.minimum((pg[1].astype(np.float32).astype(np.float64) * (ny / L)).astype(int), ny - 1)
        assert np.array_equal(cg, iy * nx + ix)
        assert np.mean(cg == c_o) > 0.999
    assert pg.min() >= 0 and pg.max() <= L


def test_gather_bitexact(dev, api):
    rng = np.random.default_rng(3)
    n = 100_003
    perm = torch.as_tensor(rng.permutation(n).astype(np.int32), device=dev)
    for rows in (2, 3):
        src = torch.as_tensor(rng.normal(size=(rows, n)), device=dev).contiguous()
        out = api.gather(perm, src)
        assert torch.equal(out, src[:, perm.long()])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sample_and_fields_match_oracle(orc, dev, api, dtype):
    rng = np.random.default_rng(5)
    n_cells = 700
    counts = rng.integers(0, 300, n_cells)
    counts[::17] = 0
    cs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    v = rng.normal(0, 300, (3, cs[-1])) + rng.normal(0, 60, (3, 1))
    v[1] += 0.3 * v[0]
    if dtype == torch.float32:
        v = v.astype(np.float32).astype(np.float64)
    csg = torch.as_tensor(cs, device=dev)
    vg = torch.as_tensor(v, dtype=dtype, device=dev).contiguous()
    acc = api.sample(csg, vg)
    api.sample(csg, vg, acc)
    acc_o = orc.sample(cs, v)
    acc_o = orc.sample(cs, v, acc_o)
    scale = np.abs(acc_o).max(axis=0) + 1e-300
    assert np.max(np.abs(acc.cpu().numpy() - acc_o) / scale) < 1e-12
    f = api.sample_fields(acc, 2, W.AR_MASS, 5.0).cpu().numpy()
    f_o = orc.fields(acc_o, 2, W.AR_MASS, 5.0)
    fs = np.abs(f_o).max(axis=0) + 1e-300
    err = np.abs(f - f_o) / fs
    say(f"  field max rel err {err.max():.2e}")
    assert err.max() < 1e-9


@pytest.mark.parametrize("rule", ["vhs", "neural"])
def test_cavity_loop_matches_oracle_step_by_step(orc, dev, api, rule):
    """A small lid-driven cavity run for 12 steps on the GPU (FP64) and in the
    oracle: every step the same cell_start, and positions and velocities equal
    to round-off."""
    say("cavity loop", rule)
    from paper_2602_21244_amd.flow import FlowSim
    fl = W.cavity_flow(seed=9, nx=10, ny=8, ppc=40)
    net = None
    net_o = None
    if rule == "neural":
        Ws, bs = W.mlp_init(4, W.FD_DIMS)
        net = api.Net(Ws, bs, act="silu", wdtype="f64", sigma_v=600.0, device=dev)
        net_o = {"Ws": Ws, "bs": bs, "act": "silu", "sigma_v": 600.0}
    sim = FlowSim(fl, dtype=torch.float64, rule=rule, net=net, seed=17, device=dev)
    dom_o = orc.domain(fl.nx, fl.ny, fl.Lx, fl.Ly, fl.kinds, fl.T_w, fl.u_w, W.AR_MASS)
    pos, v = fl.pos, fl.v
    for step in range(12):
        sim.step()
        pos, v, cs, info = orc.flow_step(dom_o, pos, v, fl.xs, fl.lam, fl.dt, 17, step,
                                         rule=rule, net=net_o)
        assert np.array_equal(sim.cs.cpu().numpy(), cs), step
        vscale = np.max(np.abs(v))
        ev = np.max(np.abs(sim.v.cpu().numpy() - v)) / vscale
        ep = np.max(np.abs(sim.pos.cpu().numpy() - pos)) / fl.Lx
        assert ev < 1e-9 and ep < 1e-12, (step, ev, ep)
    st = sim.status()
    say(f"  12 steps: velocity rel err {ev:.2e}, position {ep:.2e}, wall events {st.wall_events}")


def test_couette_profile_on_gpu(dev, api):
    """Couette channel (walls at -500 / +500 m/s, Kn = 0.2) for 3000 steps on
    the GPU: linear-in-the-bulk, antisymmetric velocity profile with slip at
    both walls, shear heating above the wall temperature, uniform density."""
    from paper_2602_21244_amd.flow import FlowSim
    fl = W.couette_flow(seed=4, ny=40, ppc=200, kn=0.2, u_wall=500.0)
    sim = FlowSim(fl, dtype=torch.float32, rule="vhs", seed=3, device=dev)
    sim.run(3000, sample_from=1500)
    sim.status()
    f = sim.fields().cpu().numpy()
    ux, T, nd = f[:, 1], f[:, 4], f[:, 0] / fl.n_density
    say(f"  u_x at walls {ux[0]:.1f} / {ux[-1]:.1f} m/s, T max {T.max():.1f} K, "
        f"density {nd.min():.3f}..{nd.max():.3f}")
    assert -500 < ux[0] < -150 and 150 < ux[-1] < 500
    assert abs(ux.mean()) < 15
    assert np.all(np.diff(ux) > -25)
    assert T.max() > 320 and T[len(T) // 2] > T[0]
    # uniform pressure across the channel: the cooler gas at the walls is denser
    p = nd * T
    assert np.all(np.abs(p / p.mean() - 1) < 0.08)
    assert nd[0] > nd[len(nd) // 2]
