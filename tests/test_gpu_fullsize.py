"""Parity at full workload sizes, in the launch configuration the benchmark
times, checked on sampled contiguous cell ranges (the random numbers are
keyed by the global cell id, so the oracle can step a range on its own).

* Mach-10 cylinder step (~30 M particles, FP32 velocities, BF16 network):
  sort bit-exact over all particles; pair lists bit-exact on sampled ranges;
  network directions within the BF16 bound of FP64 inference of the same
  weights; Phase B + moment matching to FP32 tolerance given those directions.
* Cavity step with the isotropic rule (~1 M particles, FP64): velocities to
  1e-12 on sampled ranges.
* Cylinder step through the persistent one-launch isotropic kernel: bit for
  bit the separate entry points over all 30 M particles.
* Cylinder step with the neural table rule (table from the angle network,
  Phase B fused with the matching): velocities to the FP32 bound on sampled
  ranges.
* Cylinder step with the ab initio quadrature rule: chi of every sampled pair
  to the FP32 bounds, velocities to the FP32 bound.
"""
import itertools
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


def _ranges(cs, picks, width):
    out = []
    for k0 in picks:
        k1 = min(k0 + width, len(cs) - 1)
        out.append((k0, k1))
    return out


def _surrogate_nets():
    """The seeded-init network and the shipped trained weights the benchmark
    loads (when present), each as (name, Ws, bs, sigma_v)."""
    import os
    nets = []
    Ws, bs = W.mlp_init(0, W.SURROGATE_DIMS)
    nets.append(("seeded", Ws, bs, 3547.0))
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2602_21244_amd", "weights", "jager_surrogate_8x128x4.npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        L = int(z["n_layers"])
        nets.append(("trained", [z[f"W{l}"] for l in range(L)], [z[f"b{l}"] for l in range(L)],
                     float(z["sigma_v"])))
    return nets


def test_cylinder_fullsize_neural_step(orc, dev, api):
    """Both the seeded network and the trained weights the benchmark times:
    BF16 directions against FP64 inference of the same bf16-rounded weights
    (the bound of the BF16 arithmetic), and the shift the rounding itself
    causes against the unrounded weights (reported)."""
    say("full-size cylinder step (bench configuration)")
    _cylinder_neural_case(orc, dev, api, "realistic", torch.float32,
                          list(itertools.product(_surrogate_nets(), ("all", "front", "first"))))


@pytest.mark.parametrize("order,vdtype", [("shuffled", torch.float32), ("realistic", torch.float64)])
def test_cylinder_fullsize_variants(orc, dev, api, order, vdtype):
    """The two other forms of the step the benchmark times: particles fully
    shuffled (FP32) and FP64 velocities, with the trained weights and the
    benchmark's activation split."""
    say("full-size cylinder step", order, vdtype)
    nets = [n for n in _surrogate_nets() if n[0] == "trained"] or _surrogate_nets()[:1]
    _cylinder_neural_case(orc, dev, api, order, vdtype, [(nets[0], "first")])


def _cylinder_neural_case(orc, dev, api, order, vdtype, cases):
    pop = W.cylinder_grid(seed=5, order=order)
    n, nc = pop.n, pop.n_cells
    lowp = vdtype == torch.float32
    es = 4 if lowp else 8
    cell_of = torch.as_tensor(pop.cell_of, device=dev)
    v_in = torch.as_tensor(pop.v, dtype=vdtype, device=dev).contiguous()
    lam = torch.as_tensor(pop.lam, device=dev)
    st = api.new_status(dev)
    cs, perm, v = api.sort_cells(cell_of, nc, v_in, st=st)
    ref_perm = np.argsort(pop.cell_of, kind="stable")
    assert np.array_equal(perm.cpu().numpy(), ref_perm)
    ocs = np.concatenate([[0], np.cumsum(np.bincount(pop.cell_of, minlength=nc))]).astype(np.int32)
    assert np.array_equal(cs.cpu().numpy(), ocs)
    mom = torch.zeros(nc * 6, dtype=torch.float64, device=dev)
    api.moment_match(cs, v, mom, api.L.MM_CAPTURE)
    probe = api.PairList(nc, 1, dev)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, probe, st=st)
    cap = int(api.read_status(st).n_cand * 1.02) + 1024
    pairs = api.PairList(nc, cap, dev)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, pairs, st=st)
    v_pre = v.clone()
    vp = v_pre.double().cpu().numpy()
    off = pairs.off.cpu().numpy()
    cnt = pairs.cnt.cpu().numpy()
    band = 150 * 400 + 95     # row 150 crosses the shock band and the empty disc
    rng_cells = _ranges(ocs, [0, band, 80_000, nc - 60], 60)
    sels = {}
    for k0, k1 in rng_cells:
        a, b = ocs[k0], ocs[k1]
        sub_cs = (ocs[k0:k1 + 1] - a).astype(np.int32)
        sub_v = vp[:, a:b]
        omom = orc.moments(sub_cs, sub_v)
        sel = orc.select_ntc(sub_cs, sub_v, pop.xs, pop.lam[k0:k1], omom, 11, 0, cell_base=k0)
        m = int(sel["pair_cnt"].sum())
        p0 = int(off[k0])
        assert np.array_equal(cnt[k0:k1], sel["pair_cnt"])
        assert np.array_equal(pairs.i[p0:p0 + m].cpu().numpy(), sel["pair_i"] + a)
        assert np.array_equal(pairs.j[p0:p0 + m].cpu().numpy(), sel["pair_j"] + a)
        sels[k0] = (sub_cs, sub_v, omom, sel, m, p0, a, b)
    ws = api.collide_ws(cap, v)
    for (name, Ws, bs, sigma_v), split in cases:
        v.copy_(v_pre)
        net = api.Net(Ws, bs, act="silu", wdtype="bf16", sigma_v=sigma_v, device=dev, split=split)
        name = f"{name}, split {split}"
        Wr = [w.float().double().cpu().numpy() for w in net.W]   # as the GPU holds them
        br = [np.asarray(b_, np.float32).astype(np.float64) for b_ in bs]
        api.neural_collide(net, v, pairs, 11, 0, schedule=api.L.SCHED_DEFER, ws=ws, st=st)
        # the fused Phase B + matching pass the timed step runs
        api.apply_pairs_match(cs, v, pairs, api.L.APPLY_DIRECTIONS, mom, ws, st=st)
        torch.cuda.synchronize()
        say(f"  [{name}] {n} particles, {int(api.read_status(st).n_pairs)} pairs")
        vout = v.double().cpu().numpy()
        gdirs = ws[: 3 * (cap + 1) * es].view(vdtype).view(3, cap + 1)
        sq_r, sq_u, cnt_a, worst_v = 0.0, 0.0, 0, 0.0
        for k0, k1 in rng_cells:
            sub_cs, sub_v, omom, sel, m, p0, a, b = sels[k0]
            if m == 0:
                continue
            U, xi, z = orc.pair_latents(sel, 11, 0, lowp=lowp)
            vr = (sub_v[:, sel["pair_i"]] - sub_v[:, sel["pair_j"]]).T
            xin = orc.network_input(vr, xi, z, sigma_v)
            u_gpu = gdirs[:, p0:p0 + m].T.double().cpu().numpy()
            for ref_W, ref_b, acc in ((Wr, br, "r"), (Ws, bs, "u")):
                y = orc.mlp_forward(ref_W, ref_b, xin, "silu")
                c = np.sum(u_gpu * y, axis=1) / (np.linalg.norm(u_gpu, axis=1) * np.linalg.norm(y, axis=1))
                ang2 = float(np.sum(np.arccos(np.clip(c, -1, 1)) ** 2))
                if acc == "r":
                    sq_r += ang2
                else:
                    sq_u += ang2
            cnt_a += m
            # Phase B + matching from the GPU's directions, in FP64
            u = u_gpu / np.linalg.norm(u_gpu, axis=1, keepdims=True)
            vb = orc.apply_dirs(sel, sub_v, u)
            vm, _ = orc.moment_match(sub_cs, omom, sel["pair_cnt"], vb)
            scale = np.sqrt(W.KB * 200.0 / W.AR_MASS)
            err = np.max(np.abs(vout[:, a:b] - vm)) / max(scale, np.max(np.abs(sub_v)))
            worst_v = max(worst_v, float(err))
        rms_r, rms_u = np.sqrt(sq_r / cnt_a), np.sqrt(sq_u / cnt_a)
        say(f"  [{name}] sampled ranges ({cnt_a} pairs): direction rms {rms_r:.3e} rad against "
            f"the bf16-rounded weights ({rms_u:.3e} against the unrounded), velocity rel err "
            f"{worst_v:.3e}")
        assert rms_r <= 1e-2
        if split == "all":
            # every activation a bf16 pair: the result is that of the weights
            assert rms_r <= 1e-3
        assert worst_v < (1e-5 if lowp else 1e-11)


def test_cavity_fullsize_vhs_fp64(orc, dev, api):
    say("full-size cavity step, isotropic rule, FP64")
    pop = W.cavity_grid(seed=3)
    nc = pop.n_cells
    cell_of = torch.as_tensor(pop.cell_of, device=dev)
    v_in = torch.as_tensor(pop.v, device=dev).contiguous()
    lam = torch.as_tensor(pop.lam, device=dev)
    cs, perm, v = api.sort_cells(cell_of, nc, v_in)
    vp = v.cpu().numpy()
    mom = torch.zeros(nc * 6, dtype=torch.float64, device=dev)
    api.moment_match(cs, v, mom, api.L.MM_CAPTURE)
    pairs = api.PairList(nc, 1 << 21, dev)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 3, 7, pairs)
    api.collide_vhs(v, pairs, 3, 7)
    api.moment_match(cs, v, mom, api.L.MM_APPLY, pair_cnt=pairs.cnt)
    vout = v.cpu().numpy()
    ocs = cs.cpu().numpy()
    worst = 0.0
    for k0, k1 in _ranges(ocs, [0, 20_000, nc - 200], 200):
        a, b = ocs[k0], ocs[k1]
        sub_cs = (ocs[k0:k1 + 1] - a).astype(np.int32)
        ref, _ = orc.step(sub_cs, vp[:, a:b], pop.xs, pop.lam[k0:k1], 3, 7, rule="vhs",
                          match=True, cell_base=k0)
        worst = max(worst, float(np.max(np.abs(vout[:, a:b] - ref))))
    err = worst / math.sqrt(W.KB * 273.15 / W.AR_MASS)
    say(f"  sampled ranges: velocity rel err {err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_deflection_batch_fullsize(orc, dev, api, dtype):
    """The deflection batch at its full size (2^20 pairs, g log-uniform
    100-20 000 m/s, b^2 uniform on [0, (1 nm)^2]) against the oracle on every
    pair, FP64 and FP32 (the FP32 kernel against the oracle on the
    FP32-rounded inputs).  RMS, max, 99.9th percentile and the orbiting
    pairs (|chi| > pi) are reported separately; bounds as for the 8192-pair
    case."""
    import os
    from test_gpu_parity import check_chi
    say("deflection batch 2^20", dtype)
    b, g, mr = W.deflection_batch(seed=2, n=1 << 20)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        b = b.astype(np.float32).astype(np.float64)
        g = g.astype(np.float32).astype(np.float64)
    P = orc.potential_jager(W.JAGER_PLACEHOLDER)
    ref, ost = orc.chi_batch(P, b, g, mr, n_threads=min(16, os.cpu_count() or 1))
    assert np.all(ost == 0)
    st = api.new_status(dev)
    chi = api.deflect_jager(torch.as_tensor(b, dtype=tdt, device=dev),
                            torch.as_tensor(g, dtype=tdt, device=dev), mr,
                            api.potential_jager(W.JAGER_PLACEHOLDER), st=st)
    got = chi.double().cpu().numpy()
    assert api.read_status(st).root_fail == 0 and np.all(np.isfinite(got))
    check_chi(got, ref, dtype, "batch 2^20")


def test_cylinder_fullsize_fused_vhs_step(dev, api):
    """The persistent one-launch VHS step (`dsmc_step_vhs_fused`, timed by
    the benchmark) on the whole Mach-10 cylinder: pair counts and every
    matched velocity bit-identical to the separate entry points (capture,
    NTC selection, isotropic collision, moment matching), with every cell
    staged (the shock-band cells hold ~2 200 particles)."""
    say("full-size cylinder step, fused isotropic step against separate calls")
    pop = W.cylinder_grid(seed=5, order="realistic")
    nc = pop.n_cells
    cell_of = torch.as_tensor(pop.cell_of, device=dev)
    v_in = torch.as_tensor(pop.v, dtype=torch.float32, device=dev).contiguous()
    lam = torch.as_tensor(pop.lam, device=dev)
    st = api.new_status(dev)
    cs, _, v0 = api.sort_cells(cell_of, nc, v_in, st=st)
    v1 = v0.clone()
    mom = torch.zeros(nc * 6, dtype=torch.float64, device=dev)
    api.moment_match(cs, v1, mom, api.L.MM_CAPTURE)
    probe = api.PairList(nc, 1, dev)
    api.select_pairs_ntc(cs, v1, pop.xs, lam, mom, 17, 3, probe, st=st)
    cap = int(api.read_status(st).n_cand * 1.02) + 1024
    pairs = api.PairList(nc, cap, dev)
    api.select_pairs_ntc(cs, v1, pop.xs, lam, mom, 17, 3, pairs, st=st)
    api.collide_vhs(v1, pairs, 17, 3)
    api.moment_match(cs, v1, mom, api.L.MM_APPLY, pair_cnt=pairs.cnt)
    v2 = v0.clone()
    cnt = torch.zeros(nc, dtype=torch.int32, device=dev)
    lib = api.lib()
    ws = api.workspace(lib.dsmc_step_vhs_ws(nc, 0), dev)
    st2 = api.new_status(dev)
    api.check(lib.dsmc_step_vhs_fused(nc, api._ptr(cs), api._dtype(v2), api._vec3(v2),
                                      api.xs_struct(pop.xs), api._ptr(lam),
                                      api.rng_struct(17, 3), 1, api._ptr(cnt), api._ptr(ws),
                                      int(ws.numel()), api._ptr(st2), api._stream()),
              "dsmc_step_vhs_fused")
    c = cnt.cpu().numpy()
    say(f"  {int(c.clip(min=0).sum())} pairs, cells not staged {int((c < 0).sum())}, "
        f"max pairs in a cell {int(c.max())}")
    assert (c >= 0).all()
    assert np.array_equal(c, pairs.cnt.cpu().numpy())
    assert torch.equal(v1, v2)


def test_cylinder_fullsize_table_step(orc, dev, api):
    """The table rule as the benchmark runs it on the Mach-10 cylinder: the
    512 x 512 table synthesised from the angle network (the shipped weights
    when present), Phase A by bilinear lookup (deferred), Phase B fused with
    the moment matching; against the oracle's table step with the same table
    on sampled cell ranges (shock band, free stream, disc edge): velocities to
    the FP32 bound."""
    import os
    say("full-size cylinder step, table rule")
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2602_21244_amd", "weights", "jager_anet.npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        L = int(z["n_layers"])
        Ws, bs = [z[f"W{l}"] for l in range(L)], [z[f"b{l}"] for l in range(L)]
        lo, hi = float(z["lne_lo"]), float(z["lne_hi"])
    else:
        Ws, bs = W.mlp_init(11, api.ANGLE_DIMS)
        lo, hi = math.log(5.0), math.log(5.0e5)
    net = api.AngleNet(Ws, bs, device=dev)
    tab = api.ChiTable(512, 512, lo, hi, device=dev)
    api.chi_table_build(net, tab)
    table = {"theta": tab.theta.double().cpu().numpy(), "lne_lo": lo, "lne_hi": hi}
    pop = W.cylinder_grid(seed=5, order="realistic")
    nc = pop.n_cells
    cell_of = torch.as_tensor(pop.cell_of, device=dev)
    v_in = torch.as_tensor(pop.v, dtype=torch.float32, device=dev).contiguous()
    lam = torch.as_tensor(pop.lam, device=dev)
    st = api.new_status(dev)
    cs, _, v = api.sort_cells(cell_of, nc, v_in, st=st)
    mom = torch.zeros(nc * 6, dtype=torch.float64, device=dev)
    api.moment_match(cs, v, mom, api.L.MM_CAPTURE)
    probe = api.PairList(nc, 1, dev)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, probe, st=st)
    cap = int(api.read_status(st).n_cand * 1.02) + 1024
    pairs = api.PairList(nc, cap, dev)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, pairs, st=st)
    vp = v.double().cpu().numpy()
    ws = api.collide_ws(cap, v)
    api.collide_table(tab, v, pairs, 11, 0, W.AR_MASS / 2, schedule=api.L.SCHED_DEFER, ws=ws)
    api.apply_pairs_match(cs, v, pairs, api.L.APPLY_ANGLES, mom, ws, st=st)
    vout = v.double().cpu().numpy()
    ocs = cs.cpu().numpy()
    band = 150 * 400 + 95
    worst, n_pairs = 0.0, 0
    for k0, k1 in _ranges(ocs, [0, band, 80_000, nc - 60], 60):
        a, b = ocs[k0], ocs[k1]
        sub_cs = (ocs[k0:k1 + 1] - a).astype(np.int32)
        ref, info = orc.step(sub_cs, vp[:, a:b], pop.xs, pop.lam[k0:k1], 11, 0, rule="table",
                             table=table, m_red=W.AR_MASS / 2, lowp=True, match=True,
                             cell_base=k0)
        n_pairs += int(info["sel"]["pair_cnt"].sum())
        scale = max(float(np.max(np.abs(vp[:, a:b]))), math.sqrt(W.KB * 200.0 / W.AR_MASS))
        worst = max(worst, float(np.max(np.abs(vout[:, a:b] - ref))) / scale)
    say(f"  sampled ranges ({n_pairs} pairs): velocity rel err {worst:.3e}")
    assert n_pairs > 10_000 and worst < 1e-5


def _theta_err(got, ref):
    return np.abs(np.arccos(np.clip(np.cos(got), -1, 1)) - np.arccos(np.clip(np.cos(ref), -1, 1)))


def test_cylinder_fullsize_quadrature_step(orc, dev, api):
    """The ab initio rule as the benchmark runs it on the Mach-10 cylinder
    (FP32 lane quadrature with the FP64 refinement pass, Phase A deferred,
    Phase B fused with the moment matching): on sampled cell ranges, chi of
    every accepted pair against the oracle's quadrature (the FP32 bounds of
    the batch test: theta 1e-4, RMS 1e-5) and the velocities against the
    oracle's rotation, pair update and matching from the GPU's angles."""
    say("full-size cylinder step, quadrature rule")
    pop = W.cylinder_grid(seed=5, order="realistic")
    nc = pop.n_cells
    cell_of = torch.as_tensor(pop.cell_of, device=dev)
    v_in = torch.as_tensor(pop.v, dtype=torch.float32, device=dev).contiguous()
    lam = torch.as_tensor(pop.lam, device=dev)
    st = api.new_status(dev)
    cs, _, v = api.sort_cells(cell_of, nc, v_in, st=st)
    mom = torch.zeros(nc * 6, dtype=torch.float64, device=dev)
    api.moment_match(cs, v, mom, api.L.MM_CAPTURE)
    probe = api.PairList(nc, 1, dev)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, probe, st=st)
    cap = int(api.read_status(st).n_cand * 1.02) + 1024
    pairs = api.PairList(nc, cap, dev)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, pairs, st=st)
    vp = v.double().cpu().numpy()
    pot = api.potential_jager(W.JAGER_PLACEHOLDER)
    ws = api.collide_ws(cap, v)
    api.collide_jager(v, pairs, 11, 0, W.AR_MASS / 2, W.B_MAX, pot, schedule=api.L.SCHED_DEFER,
                      ws=ws, st=st)
    buf = ws[: 6 * (cap + 1) * 4].view(torch.float32).view(6, cap + 1)
    ang = buf[:5].double().cpu().numpy()     # cos chi, sin chi, xi
    api.apply_pairs_match(cs, v, pairs, api.L.APPLY_ANGLES, mom, ws, st=st)
    assert api.read_status(st).root_fail == 0
    vout = v.double().cpu().numpy()
    ocs = cs.cpu().numpy()
    off = pairs.off.cpu().numpy()
    P = orc.potential_jager(W.JAGER_PLACEHOLDER)
    band = 150 * 400 + 95
    d_all, worst_v = [], 0.0
    for k0, k1 in _ranges(ocs, [0, band, 80_000, nc - 60], 60):
        a, b = ocs[k0], ocs[k1]
        sub_cs = (ocs[k0:k1 + 1] - a).astype(np.int32)
        sub_v = vp[:, a:b]
        omom = orc.moments(sub_cs, sub_v)
        sel = orc.select_ntc(sub_cs, sub_v, pop.xs, pop.lam[k0:k1], omom, 11, 0, cell_base=k0)
        m, p0 = int(sel["pair_cnt"].sum()), int(off[k0])
        cc, sc, xi = ang[0, p0:p0 + m], ang[1, p0:p0 + m], ang[2:5, p0:p0 + m].T.copy()
        U, _, _ = orc.pair_latents(sel, 11, 0, lowp=True)
        vr = sub_v[:, sel["pair_i"]] - sub_v[:, sel["pair_j"]]
        g = np.sqrt(np.sum(vr * vr, axis=0))
        ref, _ = orc.chi_batch(P, W.B_MAX * np.sqrt(U[:, 4]), g, W.AR_MASS / 2, n_threads=8)
        d_all.append((_theta_err(np.arctan2(sc, cc), ref), np.abs(ref) <= np.pi))
        vb = orc.apply_chi(sel, sub_v, cc, sc, xi)
        vm, _ = orc.moment_match(sub_cs, omom, sel["pair_cnt"], vb)
        scale = max(float(np.max(np.abs(sub_v))), math.sqrt(W.KB * 200.0 / W.AR_MASS))
        worst_v = max(worst_v, float(np.max(np.abs(vout[:, a:b] - vm))) / scale)
    d = np.concatenate([x for x, _ in d_all])
    tame = np.concatenate([t for _, t in d_all])
    rms = float(np.sqrt(np.mean(d * d)))
    orb = float(d[~tame].max()) if (~tame).any() else 0.0
    say(f"  {len(d)} pairs: theta err rms {rms:.3e}, max |chi|<=pi {d[tame].max():.3e}, "
        f"orbiting ({int((~tame).sum())}) max {orb:.3e}; velocity rel err {worst_v:.3e}")
    assert len(d) > 10_000
    assert d[tame].max() < 1e-4 and orb < 1e-4 and rms < 1e-5
    assert worst_v < 1e-5
