"""Benchmark of the DSMC collision step on one MI355X.

One step = the whole collision path on the Mach-10 cylinder-shaped workload
(400 x 300 cells, ~30 M particles, uneven populations): stable counting sort
of the post-streaming particle order into cells, FP64 cell moments, NTC pair
selection, the neural collision operator (BF16 MFMA MLP + energy-shell
projection, Phase B pair updates) and FP64 cell-wise moment matching.  The
metric is accepted collision pairs per second.  The same step with the ab
initio quadrature rule in place of the network is timed beside it, with the
network's angle error against the quadrature on the same pairs.

Prints ONE JSON line.  --gpus above 1 exits: the path is measured on one GPU.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MLP_FLOP_PER_PAIR = 2 * (8 * 128 + 3 * 128 * 128 + 128 * 3)  # 101,120 (unpadded)
PEAK_BF16 = 2.5e15
PEAK_HBM = 8.0e12
PEAK_FP32 = 157.3e12   # vector FP32
PEAK_FP64 = 78.6e12    # vector FP64


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="cylinder", choices=["cylinder", "cavity"])
    p.add_argument("--order", default="realistic", choices=["realistic", "shuffled", "sorted"])
    p.add_argument("--quad-steps", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-variants", action="store_true",
                   help="skip the shuffled-order and FP64-velocity neural step timings")
    p.add_argument("--no-cavity-loop", action="store_true",
                   help="skip the cavity flow-loop timing (profiling runs of the step kernels)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run a plain 1 GiB device copy first (reference for counter scaling)")
    p.add_argument("--cpu-sample-pairs", type=int, default=4_000_000)
    p.add_argument("--weights", default=os.path.join(ROOT, "paper_2602_21244_amd", "weights",
                                                     "jager_surrogate_8x128x4.npz"))
    p.add_argument("--anet-weights", default=os.path.join(ROOT, "paper_2602_21244_amd", "weights",
                                                          "jager_anet.npz"))
    p.add_argument("--table-steps", type=int, default=5)
    p.add_argument("--split", default="first", choices=["first", "front", "all"],
                   help="activations entering the matrix cores as bf16 pairs: the input and "
                        "the first hidden activation (first), the first two (front), or all")
    return p.parse_args()


def load_weights(path, workloads):
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        L = int(z["n_layers"])
        Ws = [z[f"W{l}"] for l in range(L)]
        bs = [z[f"b{l}"] for l in range(L)]
        return Ws, bs, float(z["sigma_v"]), "trained"
    Ws, bs = workloads.mlp_init(0, workloads.SURROGATE_DIMS)
    return Ws, bs, 3547.0, "seeded-init"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the collision step is measured on one GPU only (asked for --gpus "
              f"{args.gpus}); sharding it across GPUs is described, not implemented.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import workloads as W
    from paper_2602_21244_amd import api
    L = api.L

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    if args.workload == "cylinder":
        pop = W.cylinder_grid(seed=5, order=args.order)
        wname = f"mach10_cylinder_400x300_{args.order}"
    else:
        pop = W.cavity_grid(seed=3)
        wname = "cavity_200x200"
    log(f"workload {wname}: {pop.n} particles, {pop.n_cells} cells ({time.time() - t0:.1f}s)")

    stream = torch.cuda.current_stream()
    hbm_ceiling = copy_ceiling(dev)
    log(f"measured copy ceiling: {hbm_ceiling / 1e9:.0f} GB/s ({hbm_ceiling / PEAK_HBM:.2f} of 8 TB/s)")
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    cell_of = torch.as_tensor(pop.cell_of, device=dev)
    v_in = torch.as_tensor(pop.v, dtype=torch.float32, device=dev).contiguous()
    lam = torch.as_tensor(pop.lam, device=dev)
    n, n_cells = pop.n, pop.n_cells
    v = torch.empty_like(v_in)
    cs = torch.empty(n_cells + 1, dtype=torch.int32, device=dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    mom = torch.zeros(n_cells * 6, dtype=torch.float64, device=dev)
    st = api.new_status(dev)
    lib = api.lib()
    sort_ws_b = lib.dsmc_sort_cells_ws(n, n_cells)
    sort_ws = api.workspace(sort_ws_b, dev)

    def do_sort():
        api.check(lib.dsmc_sort_cells(n, n_cells, api._ptr(cell_of), L.F32, api._vec3(v_in),
                                      api._vec3(v), api._ptr(cs), api._ptr(perm), api._ptr(sort_ws),
                                      sort_ws_b, api._ptr(st), api._stream()), "sort")

    # size the pair capacity from a first selection
    do_sort()
    api.moment_match(cs, v, mom, L.MM_CAPTURE)
    probe = api.PairList(n_cells, 1, dev)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, probe, st=st)
    n_cand = api.read_status(st).n_cand
    cap = int(n_cand * 1.02) + 1024
    pairs = api.PairList(n_cells, cap, dev)
    sel_ws = api.workspace(lib.dsmc_select_pairs_ntc_ws(n_cells, cap), dev)

    Ws, bs, sigma_v, wkind = load_weights(args.weights, W)
    net = api.Net(Ws, bs, act="silu", wdtype="bf16", sigma_v=sigma_v, device=dev, split=args.split)
    # the other activation splits, timed beside it on the same pairs
    nets_other = {sp: api.Net(Ws, bs, act="silu", wdtype="bf16", sigma_v=sigma_v, device=dev,
                              split=sp)
                  for sp in ("all", "front", "first") if sp != args.split}
    col_ws = api.collide_ws(cap, v)
    pot = api.potential_jager(W.JAGER_PLACEHOLDER)
    quad = api.quad_struct(64)

    # neural deflection-angle table: angle network -> 512 x 512 table
    anet, lne_lo, lne_hi, akind = load_anet(args.anet_weights, W, api, dev)
    tab = api.ChiTable(512, 512, lne_lo, lne_hi, device=dev)
    tab_ws = api.chi_table_build(anet, tab)
    torch.cuda.synchronize()
    tb0, tb1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tb0.record(stream)
    for _ in range(3):
        api.chi_table_build(anet, tab, ws=tab_ws)
    tb1.record(stream)
    torch.cuda.synchronize()
    table_build_ms = tb0.elapsed_time(tb1) / 3
    log(f"chi table 512x512 build: {table_build_ms:.3f} ms ({akind} angle network)")

    # launch shape of the fused Phase B + moment matching, tuned on this
    # step's own pair list (Phase A of the network, deferred)
    from paper_2602_21244_amd import autotune
    do_sort()
    api.moment_match(cs, v, mom, L.MM_CAPTURE)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, pairs, ws=sel_ws, st=st)
    api.neural_collide(net, v, pairs, 11, 0, schedule=L.SCHED_DEFER, ws=col_ws, st=st)
    match_shape, match_times = autotune.tune_match_schedule(cs, v, pairs, L.APPLY_DIRECTIONS, mom,
                                                            col_ws, use_cache=False)
    log(f"autotuned phase B + match launch shape {match_shape}: {match_times[match_shape]:.4f} ms "
        f"(default 40/2/1: {match_times[(40, 2, 1)]:.4f} ms)")

    def stage_events(k):
        return [torch.cuda.Event(enable_timing=True) for _ in range(k)]

    def step(rule, ev=None):
        """One collision step; ev: list of 6 events bracketing the stages."""
        if ev: ev[0].record(stream)
        do_sort()
        if ev: ev[1].record(stream)
        api.moment_match(cs, v, mom, L.MM_CAPTURE)
        if ev: ev[2].record(stream)
        api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, pairs, ws=sel_ws, st=st)
        if ev: ev[3].record(stream)
        if rule == "neural":
            api.neural_collide(net, v, pairs, 11, 0, schedule=L.SCHED_DEFER, ws=col_ws, st=st)
            kind = L.APPLY_DIRECTIONS
        elif rule == "vhs":
            api.collide_vhs(v, pairs, 11, 0, schedule=L.SCHED_DEFER, ws=col_ws)
            kind = L.APPLY_DIRECTIONS
        elif rule == "table":
            api.collide_table(tab, v, pairs, 11, 0, W.AR_MASS / 2, schedule=L.SCHED_DEFER,
                              ws=col_ws)
            kind = L.APPLY_ANGLES
        else:
            api.collide_jager(v, pairs, 11, 0, W.AR_MASS / 2, W.B_MAX, pot, quad=quad,
                              schedule=L.SCHED_DEFER, ws=col_ws, st=st)
            kind = L.APPLY_ANGLES
        if ev: ev[4].record(stream)
        # Phase B and the cell-wise moment matching in one pass
        api.apply_pairs_match(cs, v, pairs, kind, mom, col_ws, mode=L.MM_APPLY, st=st)
        if ev: ev[5].record(stream)

    names = ["sort", "moments", "select", "phaseA", "phaseB_match"]

    def run(rule, warm, steps):
        for _ in range(warm):
            step(rule)
        torch.cuda.synchronize()
        evs = [stage_events(6) for _ in range(steps)]
        # no collector pause while the steps are queued: the GPU would idle
        # between two events and the gap would count as stage time
        gc.collect()
        gc.disable()
        t_start = time.perf_counter()
        for q in range(steps):
            step(rule, evs[q])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        gc.enable()
        per = {nm: float(np.mean([evs[q][s].elapsed_time(evs[q][s + 1]) for q in range(steps)]))
               for s, nm in enumerate(names)}
        tot = float(np.mean([evs[q][0].elapsed_time(evs[q][5]) for q in range(steps)]))
        return wall, tot, per

    api.status_clear(st)
    wall_n, ms_n, per_n = run("neural", args.warmup, args.steps)
    s = api.read_status(st)
    n_pairs = int(s.n_pairs)
    log(f"neural: {ms_n:.3f} ms/step (events), wall {wall_n / args.steps * 1e3:.3f} ms/step, "
        f"pairs {n_pairs}, stages {json.dumps({k: round(x, 4) for k, x in per_n.items()})}")

    # the same step captured as one HIP graph and replayed (the launch
    # sequence of a production loop); every replay recomputes the step from
    # the same post-streaming input, so its result must equal the eager one
    graph = graph_replay_timing(step, v, args.steps)
    log(f"neural step as a HIP graph: {graph}")

    # neural directions of this step for the angle comparison
    es = 4
    dirs = col_ws[: 3 * (cap + 1) * es].view(torch.float32).view(3, cap + 1)[:, :n_pairs].clone()

    # Phase A with every activation split on the same pairs (the step's last
    # selection): their times, and each one's angle to split "all" (every
    # activation a bf16 pair, ~1e-4 rad from exact activations)
    split_cmp = phase_a_split_compare(api, L, {args.split: net, **nets_other}, v, pairs, col_ws,
                                      st, stream, cap, n_pairs, args.steps)
    split_cmp["timed_split"] = args.split
    log(f"activation split: {split_cmp}")

    wall_q, ms_q, per_q = run("quadrature", 1, args.quad_steps)
    log(f"quadrature: {ms_q:.3f} ms/step, stages {json.dumps({k: round(x, 4) for k, x in per_q.items()})}")

    # angle error of the network against the quadrature on the same pairs:
    # rebuild the quadrature direction from (cos chi, sin chi, xi) and the
    # pre-collision v_r (sorted velocities before Phase B of that step)
    do_sort()
    api.moment_match(cs, v, mom, L.MM_CAPTURE)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, pairs, ws=sel_ws, st=st)
    api.collide_jager(v, pairs, 11, 0, W.AR_MASS / 2, W.B_MAX, pot, quad=quad,
                      schedule=L.SCHED_DEFER, ws=col_ws, st=st)
    torch.cuda.synchronize()
    m = min(n_pairs, 200_000)
    sel_idx = torch.linspace(0, n_pairs - 1, m, device=dev).long()
    buf = col_ws[: 6 * (cap + 1) * es].view(torch.float32).view(6, cap + 1)
    cc, sc = buf[0, sel_idx].double(), buf[1, sel_idx].double()
    xi = buf[2:5, sel_idx].double()
    pi_, pj_ = pairs.i[sel_idx].long(), pairs.j[sel_idx].long()
    vr = (v[:, pi_] - v[:, pj_]).double()
    vh = vr / vr.norm(dim=0, keepdim=True)
    w = xi - (xi * vh).sum(0, keepdim=True) * vh
    e = w / w.norm(dim=0, keepdim=True)
    uq = cc * vh + sc * e
    un = dirs[:, sel_idx].double()
    un = un / un.norm(dim=0, keepdim=True)
    ang = torch.arccos(torch.clamp((uq * un).sum(0), -1, 1)).cpu().numpy()
    chi_rms = float(np.sqrt(np.mean(ang ** 2)))
    log(f"network vs quadrature direction error: rms {chi_rms:.4f} rad ({wkind} weights)")

    # the table rule on the same step, and its angle error against the
    # quadrature on the same pairs (folded angles)
    wall_t, ms_t, per_t = run("table", 1, args.table_steps)
    log(f"table: {ms_t:.3f} ms/step, stages {json.dumps({k: round(x, 4) for k, x in per_t.items()})}")
    th_q = torch.arccos(torch.clamp(cc, -1, 1))
    do_sort()
    api.moment_match(cs, v, mom, L.MM_CAPTURE)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, pairs, ws=sel_ws, st=st)
    api.collide_table(tab, v, pairs, 11, 0, W.AR_MASS / 2, schedule=L.SCHED_DEFER, ws=col_ws)
    torch.cuda.synchronize()
    th_t = torch.arccos(torch.clamp(buf[0, sel_idx].double(), -1, 1))
    dth = (th_t - th_q).cpu().numpy()
    table_rms = float(np.sqrt(np.mean(dth ** 2)))
    log(f"table vs quadrature folded-angle error: rms {table_rms:.4f} rad ({akind} angle network)")
    table_flop = 512 * 512 * anet_flop_per_row(anet.dims)

    # the isotropic VHS rule (the plain rule the network replaces) on the same
    # step: its Phase A reads the pair list and writes one direction per pair
    wall_v, ms_v, per_v = run("vhs", 1, args.table_steps)
    log(f"vhs: {ms_v:.3f} ms/step, stages {json.dumps({k: round(x, 4) for k, x in per_v.items()})}")

    # the isotropic rule as one persistent launch per step (cell work queue:
    # moments, selection, Phase A/B and matching with the cell in LDS)
    fused = fused_vhs_timing(api, lib, L, pop, cs, v, do_sort, lam, args.table_steps)
    log(f"isotropic rule, persistent fused step: {fused}")

    # SBT selection (the alternative rate control) on the same sorted input,
    # beside the NTC selection's stage time
    st_sbt = api.new_status(dev)
    sbt_ws = api.workspace(lib.dsmc_select_pairs_sbt_ws(n_cells, cap), dev)
    do_sort()
    api.moment_match(cs, v, mom, L.MM_CAPTURE)
    api.select_pairs_sbt(cs, v, pop.xs, lam, 11, 0, pairs, ws=sbt_ws, st=st_sbt)
    torch.cuda.synchronize()
    s0_, s1_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0_.record(stream)
    for _ in range(5):
        api.select_pairs_sbt(cs, v, pop.xs, lam, 11, 0, pairs, ws=sbt_ws, st=st_sbt)
    s1_.record(stream)
    torch.cuda.synchronize()
    sbt_ms = s0_.elapsed_time(s1_) / 5
    sbt_pairs = int(pairs.cnt.sum())
    log(f"sbt selection: {sbt_ms:.3f} ms, {sbt_pairs} pairs (NTC stage {per_n['select']:.3f} ms)")

    # Chapman-Enskog viscosity from the quadrature chi: 64 temperatures
    T_ce = torch.linspace(300.0, 3000.0, 64, dtype=torch.float64, device=dev)
    api.viscosity_ce(T_ce, W.AR_MASS, 2.5e-9, pot)
    torch.cuda.synchronize()
    c0_, c1_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0_.record(stream)
    for _ in range(3):
        api.viscosity_ce(T_ce, W.AR_MASS, 2.5e-9, pot)
    c1_.record(stream)
    torch.cuda.synchronize()
    ce_ms = c0_.elapsed_time(c1_) / 3
    log(f"Chapman-Enskog viscosity, 64 temperatures: {ce_ms:.3f} ms")

    # deflection batch (2^20 pairs, g log-uniform 100-20 000 m/s, b^2 uniform):
    # quadrature FP64 / FP32 against the angle network evaluated per pair
    batch = deflection_batch_timing(api, W, dev, pot, quad, anet, lne_lo, lne_hi)
    log(f"deflection batch: {batch}")

    # roofline of the dominant kernel (the fused MLP, Phase A of the network)
    t_mlp = per_n["phaseA"] * 1e-3
    achieved = n_pairs * MLP_FLOP_PER_PAIR / t_mlp
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_BF16 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_BF16,
                "traffic": counter_traffic(MLP_KERNEL[args.split]),
                "kernel": "k_mlp_bf16 (Phase A of dsmc_neural_collide)",
                "sq_counters": mlp_sq_counters(MLP_KERNEL[args.split]),
                "algorithmic_flop_per_pair": MLP_FLOP_PER_PAIR}
    sort_bytes = n * (4 + 4 + 12 + 12 + 4)  # cell id twice, v read + write, perm
    extra = {
        "quadrature_pairs_per_s": n_pairs / (ms_q * 1e-3),
        "quadrature_ms_per_step": ms_q,
        "neural_over_quadrature": (ms_q / ms_n),
        "chi_rms_vs_quadrature_rad": chi_rms,
        "network_weights": wkind,
        "stage_ms_neural": per_n,
        "stage_ms_quadrature": per_q,
        "quadrature_valu_roofline": quadrature_valu_roofline(per_q["phaseA"]),
        "sort_GBps_algorithmic": sort_bytes / (per_n["sort"] * 1e-3) / 1e9,
        "hbm_copy_ceiling_GBps": hbm_ceiling / 1e9,
        "stage_hbm": stage_rooflines({**per_n, "phaseA_vhs": per_v["phaseA"]}, n, n_cells,
                                     n_pairs, hbm_ceiling),
        "table_pairs_per_s": n_pairs / (ms_t * 1e-3),
        "table_ms_per_step": ms_t,
        "stage_ms_table": per_t,
        "table_theta_rms_vs_quadrature_rad": table_rms,
        "sbt_select_ms": sbt_ms,
        "sbt_pairs": sbt_pairs,
        "ntc_select_ms": per_n["select"],
        "ce_viscosity_ms_64_temperatures": ce_ms,
        "eager_ms_per_step": ms_n,
        "activation_split": split_cmp,
        "graph": graph,
        "match_schedule": {"shape_wave_medium_big_per_cu": list(match_shape),
                           "ms": match_times[match_shape], "default_ms": match_times[(40, 2, 1)]},
        "vhs_fused_step": fused,
        "vhs_pairs_per_s": n_pairs / (ms_v * 1e-3),
        "vhs_ms_per_step": ms_v,
        "stage_ms_vhs": per_v,
        "angle_network_weights": akind,
        "table_build_ms_512x512": table_build_ms,
        "table_build_TFLOPs": table_flop / (table_build_ms * 1e-3) / 1e12,
        "pairs_per_step": n_pairs,
        "particles": n,
        "cells": n_cells,
        "deflection_batch_2p20": batch,
    }

    # the same neural step with the particles fully shuffled (worst case for
    # the sort and the gathers) and with FP64 velocities
    if args.workload == "cylinder" and not args.no_variants:
        for tag, order, vdt in (("shuffled_fp32", "shuffled", torch.float32),
                                ("realistic_fp64", "realistic", torch.float64)):
            extra[f"neural_step_{tag}"] = variant_step_timing(W, api, L, dev, net, order, vdt,
                                                              max(3, args.steps // 2))
            log(f"neural step, {tag}: {extra[f'neural_step_{tag}']}")

    # surrogate training step (batch 65 536 harvested rows): forward (MFMA),
    # MSE, hand-written backward, Adam on every parameter
    train = train_step_timing(api, W, dev, net, sigma_v)
    extra["train_step"] = train
    log(f"training step: {train}")

    # the flow loop around the step on the paper's lid-driven cavity (50 x 50
    # cells, 250 000 particles, Kn = 0.1, lid 100 m/s): move with diffuse
    # walls, binning, selection, the per-pair network, fused Phase B + moment
    # matching and sampling every step
    if not args.no_cavity_loop:
        cav = cavity_loop_timing(W, dev, net)
        extra["cavity_loop"] = cav
        log(f"cavity loop: {cav}")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(pop, Ws, bs, sigma_v, args.cpu_sample_pairs)
        log(f"cpu baseline: {cpu}")

    # the step as launched eagerly and as a replayed HIP graph does the same
    # work; the faster of the two (graph only when its result matched)
    ms_step = ms_n
    if graph.get("bit_identical_to_eager") and graph.get("ms_per_step", ms_n) < ms_n:
        ms_step = graph["ms_per_step"]
    out = {
        "metric": "collision pairs/s: neural vs quadrature \u03c7 at stated angle error; "
                  "% HBM/MFMA peak",
        "value": n_pairs / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": wname, "particles": n, "cells": n_cells,
                   "pairs_per_step": n_pairs, "velocities": "fp32 SoA",
                   "mlp": "8-128x4-3 SiLU bf16/fp32-acc", "mlp_split": args.split,
                   "moments": "fp64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


def variant_step_timing(W, api, L, dev, net, order, vdtype, steps, warm=2):
    """The timed neural step (sort, capture, NTC select, network Phase A,
    fused Phase B + matching) on the cylinder population in another particle
    order and/or velocity precision: mean event time per step and stage."""
    import torch
    pop = W.cylinder_grid(seed=5, order=order)
    code = L.F64 if vdtype == torch.float64 else L.F32
    cell_of = torch.as_tensor(pop.cell_of, device=dev)
    v_in = torch.as_tensor(pop.v, dtype=vdtype, device=dev).contiguous()
    lam = torch.as_tensor(pop.lam, device=dev)
    n, nc = pop.n, pop.n_cells
    v = torch.empty_like(v_in)
    cs = torch.empty(nc + 1, dtype=torch.int32, device=dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    mom = torch.zeros(nc * 6, dtype=torch.float64, device=dev)
    st = api.new_status(dev)
    lib = api.lib()
    swb = lib.dsmc_sort_cells_ws(n, nc)
    sws = api.workspace(swb, dev)
    stream = torch.cuda.current_stream()

    def do_sort():
        api.check(lib.dsmc_sort_cells(n, nc, api._ptr(cell_of), code, api._vec3(v_in), api._vec3(v),
                                      api._ptr(cs), api._ptr(perm), api._ptr(sws), swb, api._ptr(st),
                                      api._stream()), "sort")

    do_sort()
    api.moment_match(cs, v, mom, L.MM_CAPTURE)
    probe = api.PairList(nc, 1, dev)
    api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, probe, st=st)
    cap = int(api.read_status(st).n_cand * 1.02) + 1024
    pairs = api.PairList(nc, cap, dev)
    sel_ws = api.workspace(lib.dsmc_select_pairs_ntc_ws(nc, cap), dev)
    col_ws = api.collide_ws(cap, v)

    def step(ev=None):
        if ev: ev[0].record(stream)
        do_sort()
        if ev: ev[1].record(stream)
        api.moment_match(cs, v, mom, L.MM_CAPTURE)
        if ev: ev[2].record(stream)
        api.select_pairs_ntc(cs, v, pop.xs, lam, mom, 11, 0, pairs, ws=sel_ws, st=st)
        if ev: ev[3].record(stream)
        api.neural_collide(net, v, pairs, 11, 0, schedule=L.SCHED_DEFER, ws=col_ws, st=st)
        if ev: ev[4].record(stream)
        api.apply_pairs_match(cs, v, pairs, L.APPLY_DIRECTIONS, mom, col_ws, mode=L.MM_APPLY, st=st)
        if ev: ev[5].record(stream)

    for _ in range(warm):
        step()
    torch.cuda.synchronize()
    api.status_clear(st)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
    gc.collect()
    gc.disable()
    for q in range(steps):
        step(evs[q])
    torch.cuda.synchronize()
    gc.enable()
    names = ["sort", "moments", "select", "phaseA", "phaseB_match"]
    per = {nm: float(np.mean([evs[q][k].elapsed_time(evs[q][k + 1]) for q in range(steps)]))
           for k, nm in enumerate(names)}
    ms = float(np.mean([evs[q][0].elapsed_time(evs[q][5]) for q in range(steps)]))
    s = api.read_status(st)
    n_pairs = int(pairs.cnt.sum())
    out = {"order": order, "velocities": "fp64" if code == L.F64 else "fp32", "particles": n,
           "pairs_per_step": n_pairs, "ms_per_step": ms, "pairs_per_s": n_pairs / (ms * 1e-3),
           "stage_ms": per, "status_flags": int(s.flags)}
    del v_in, v, pairs, col_ws, sel_ws, sws
    torch.cuda.empty_cache()
    return out


def graph_replay_timing(step, v, reps):
    """Capture step("neural") as one HIP graph on a side stream, replay it
    `reps` times between events, and check a replay against the eager step."""
    import torch
    out = {}
    try:
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step("neural")
        torch.cuda.synchronize()
        eager = v.clone()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            step("neural")
        v.zero_()
        g.replay()
        torch.cuda.synchronize()
        out["bit_identical_to_eager"] = bool(torch.equal(v, eager))
        for _ in range(2):
            g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        out["ms_per_step"] = e0.elapsed_time(e1) / reps
        out["replays"] = reps
    except Exception as e:  # pragma: no cover - reported, the eager number stands
        out["error"] = repr(e)
    return out


def fused_vhs_timing(api, lib, L, pop, cs, v, do_sort, lam, reps):
    """dsmc_step_vhs_fused (one persistent launch: moments, NTC, isotropic
    Phase A/B and moment matching per cell in LDS) after the sort, timed
    against nothing else; cells it cannot stage (> 3072 particles) counted."""
    import torch
    dev = v.device
    n_cells = pop.n_cells
    cnt = torch.zeros(n_cells, dtype=torch.int32, device=dev)
    ws = api.workspace(lib.dsmc_step_vhs_ws(n_cells, 0), dev)
    st = api.new_status(dev)

    def one():
        api.check(lib.dsmc_step_vhs_fused(n_cells, api._ptr(cs), L.F32, api._vec3(v),
                                          api.xs_struct(pop.xs), api._ptr(lam),
                                          api.rng_struct(11, 0), 1, api._ptr(cnt), api._ptr(ws),
                                          int(ws.numel()), api._ptr(st), api._stream()),
                  "dsmc_step_vhs_fused")
    do_sort()
    one()
    torch.cuda.synchronize()
    ms_sort = []
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tot = 0.0
    for _ in range(reps):
        e[0].record()
        do_sort()
        e[1].record()
        one()
        e[2].record()
        torch.cuda.synchronize()
        ms_sort.append(e[0].elapsed_time(e[1]))
        tot += e[1].elapsed_time(e[2])
    c = cnt.cpu()
    return {"fused_kernel_ms": tot / reps, "step_ms_with_sort": tot / reps + float(np.mean(ms_sort)),
            "pairs": int(c.clamp(min=0).sum()), "cells_not_staged": int((c < 0).sum()),
            "max_pairs_in_a_cell": int(c.max())}


MLP_KERNEL = {"all": "k_mlp_bf16<128, true, float, 0, false, 1, 512, 0>",
              "front": "k_mlp_bf16<128, true, float, 0, false, 1, 512, 1>",
              "first": "k_mlp_bf16<128, true, float, 0, false, 1, 512, 2>"}


def phase_a_split_compare(api, L, nets, v, pairs, col_ws, st, stream, cap, n_pairs, reps):
    """Phase A (the network on every pair, directions deferred) with each
    activation split in `nets`: mean event time of each, and the RMS / max
    angle between its directions and those of split "all" on the same
    pairs."""
    import torch
    out = {"phaseA_ms": {}, "angle_rms_vs_all_rad": {}, "angle_max_vs_all_rad": {}}
    dirs = {}
    for tag, nt in nets.items():
        api.neural_collide(nt, v, pairs, 11, 0, schedule=L.SCHED_DEFER, ws=col_ws, st=st)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            api.neural_collide(nt, v, pairs, 11, 0, schedule=L.SCHED_DEFER, ws=col_ws, st=st)
        e1.record(stream)
        torch.cuda.synchronize()
        out["phaseA_ms"][tag] = e0.elapsed_time(e1) / reps
        dirs[tag] = col_ws[: 3 * (cap + 1) * 4].view(torch.float32).view(3, cap + 1)[:, :n_pairs].double()
    b = dirs["all"]
    for tag, a in dirs.items():
        if tag == "all":
            continue
        c = (a * b).sum(0) / (a.norm(dim=0) * b.norm(dim=0))
        ang = torch.arccos(torch.clamp(c, -1.0, 1.0))
        out["angle_rms_vs_all_rad"][tag] = float(torch.sqrt(torch.mean(ang ** 2)))
        out["angle_max_vs_all_rad"][tag] = float(ang.max())
    return out


def quadrature_valu_roofline(ms_phase_a):
    """Executed VALU flop of the in-step quadrature (lane rule plus its FP64
    refinement pass) from the committed rocprofv3 operation counts, over the
    live event time of that Phase A; null when the counts were taken on
    another build of deflect.hip."""
    from paper_2602_21244_amd.build import compile_signature
    path = os.path.join(ROOT, "profiles", "valu_flops_quadrature_mach10_cylinder_400x300.md")
    if not os.path.exists(path):
        return None
    try:
        blob = json.loads(open(path).read().split("```json", 1)[1].split("```", 1)[0])
        ks = [blob["kernels"]["k_phaseA_jager_f32"], blob["kernels"]["k_refine<PhaseAJagerJob<float> >"]]
    except (IndexError, KeyError, ValueError):
        return None
    if blob.get("compile_signature") != compile_signature(blob.get("source", "deflect.hip")):
        return None
    f32 = sum(k["fp32_flop"] for k in ks)
    f64 = sum(k["fp64_flop"] for k in ks)
    t = ms_phase_a * 1e-3
    r32, r64 = f32 / t, f64 / t
    return {"bound": "alu", "kernels": "k_phaseA_jager_f32 + k_refine (FP64)",
            "fp32_flop": f32, "fp64_flop": f64, "ms": ms_phase_a,
            "achieved_fp32_TFLOPs": r32 / 1e12, "achieved_fp64_TFLOPs": r64 / 1e12,
            "peak_fp32_TFLOPs": PEAK_FP32 / 1e12, "peak_fp64_TFLOPs": PEAK_FP64 / 1e12,
            "frac": r32 / PEAK_FP32 + r64 / PEAK_FP64}


def mlp_sq_counters(kernel):
    """Matrix-core utilisation of `kernel` from the committed rocprofv3 SQ
    counter summary (SQ_VALU_MFMA_BUSY_CYCLES over the SIMD cycles at the
    clock measured in the same pass), or None for another build."""
    from paper_2602_21244_amd.build import compile_signature
    path = os.path.join(ROOT, "profiles", "sq_counters_k_mlp_bf16_mach10_cylinder_400x300.md")
    if not os.path.exists(path):
        return None
    try:
        blob = json.loads(open(path).read().split("```json", 1)[1].split("```", 1)[0])
        k = blob["kernels"][kernel]
    except (IndexError, KeyError, ValueError):
        return None
    if blob.get("compile_signature") != compile_signature(blob.get("source", "mlp.hip")):
        return None
    return k


def counter_traffic(kernel, source="mlp.hip"):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (scaled by a plain copy), or None when the
    summary is missing or was taken on a different build of the kernel."""
    from paper_2602_21244_amd.build import compile_signature
    path = os.path.join(ROOT, "profiles", "hbm_counters_mach10_cylinder_400x300_bench.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    try:
        blob = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
        k = blob["kernels"][kernel]
    except (IndexError, KeyError, ValueError):
        return None
    if k.get("compile_signature") != compile_signature(source):
        return None
    return k["hbm_bytes"]


def deflection_batch_timing(api, W, dev, pot, quad, anet, lne_lo, lne_hi, reps=3):
    import torch
    b, g, mr = W.deflection_batch(seed=2, n=1 << 20)
    out = {"pairs": int(b.size)}
    th, raw = {}, {}
    for name, dt in (("quadrature_fp64", torch.float64), ("quadrature_fp32", torch.float32)):
        bt = torch.as_tensor(b, dtype=dt, device=dev)
        gt = torch.as_tensor(g, dtype=dt, device=dev)
        chi = api.deflect_jager(bt, gt, mr, pot, quad)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            chi = api.deflect_jager(bt, gt, mr, pot, quad)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": ms, "pairs_per_s": b.size / (ms * 1e-3)}
        th[name] = torch.arccos(torch.clamp(torch.cos(chi.double()), -1, 1))
        raw[name] = chi.double()
    b64 = torch.as_tensor(b, device=dev)
    g64 = torch.as_tensor(g, device=dev)
    chi64 = torch.as_tensor(th["quadrature_fp64"], device=dev)
    x, _ = api.anet_rows(b64, g64, chi64, mr, lne_lo, lne_hi, W.B_MAX)
    y, ws = api.anet_forward(anet, x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        api.anet_forward(anet, x, y, ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out["angle_network_per_pair"] = {"ms": ms, "pairs_per_s": b.size / (ms * 1e-3)}
    th_net = torch.clamp(torch.expm1(y.double()), 0, math.pi)
    ref = th["quadrature_fp64"]
    out["theta_rms_fp32_vs_fp64_rad"] = float(torch.sqrt(((th["quadrature_fp32"] - ref) ** 2).mean()))
    out["theta_rms_network_vs_fp64_rad"] = float(torch.sqrt(((th_net - ref) ** 2).mean()))
    # chi itself (not folded into [0, pi]): FP32 against FP64, all pairs and
    # the orbiting ones (|chi| > pi) separately
    c64, c32 = raw["quadrature_fp64"], raw["quadrature_fp32"]
    d = (c32 - c64).abs()
    orb = c64.abs() > math.pi

    def dist(x):
        if x.numel() == 0:
            return {"pairs": 0}
        return {"pairs": int(x.numel()), "rms": float(torch.sqrt((x ** 2).mean())),
                "max": float(x.max()), "p99_9": float(torch.quantile(x.float(), 0.999))}

    out["chi_fp32_vs_fp64_rad"] = {"all": dist(d), "orbiting": dist(d[orb]),
                                   "not_orbiting": dist(d[~orb])}
    return out


def anet_flop_per_row(dims):
    return 2 * sum(dims[l] * dims[l + 1] for l in range(len(dims) - 1))


def load_anet(path, workloads, api, dev):
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        L = int(z["n_layers"])
        Ws = [z[f"W{l}"] for l in range(L)]
        bs = [z[f"b{l}"] for l in range(L)]
        return (api.AngleNet(Ws, bs, device=dev), float(z["lne_lo"]), float(z["lne_hi"]),
                "trained")
    Ws, bs = workloads.mlp_init(11, api.ANGLE_DIMS)
    return api.AngleNet(Ws, bs, device=dev), math.log(5.0), math.log(5.0e5), "seeded-init"


def cavity_loop_timing(W, dev, net, warm=20, steps=200):
    import torch
    from paper_2602_21244_amd.flow import FlowSim
    fl = W.cavity_flow()
    sim = FlowSim(fl, dtype=torch.float32, rule="neural", net=net, seed=5, device=dev)
    sim.run(warm, sample_from=0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.run(steps, sample_from=0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = sim.status()
    f = sim.fields().cpu().numpy()
    return {"particles": fl.n, "cells": fl.n_cells, "ms_per_step": ms,
            "particle_steps_per_s": fl.n / (ms * 1e-3),
            "pairs_per_step": float(st.n_pairs), "wall_events_per_step":
            float(st.wall_events) / (warm + steps),
            "lid_row_mean_ux": float(f[-fl.nx:, 1].mean()), "mean_T": float(f[:, 4].mean())}


def train_step_timing(api, W, dev, net, sigma_v, B=65536, steps=5):
    import ctypes

    import torch
    rows = W.training_rows(seed=4, n=B)
    pot = api.potential_jager(W.JAGER_PLACEHOLDER)
    x, g, tgt, chi = api.harvest_rows(torch.as_tensor(rows["vr"], device=dev),
                                      torch.as_tensor(rows["xi"], device=dev),
                                      torch.as_tensor(rows["z"], device=dev), rows["sigma_v"],
                                      W.B_MAX, W.AR_MASS / 2, pot, api.quad_struct(64))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    api.harvest_rows(torch.as_tensor(rows["vr"], device=dev), torch.as_tensor(rows["xi"], device=dev),
                     torch.as_tensor(rows["z"], device=dev), rows["sigma_v"], W.B_MAX,
                     W.AR_MASS / 2, pot, api.quad_struct(64))
    e1.record()
    torch.cuda.synchronize()
    harvest_ms = e0.elapsed_time(e1)
    from paper_2602_21244_amd.train import FlatParams
    Ws = [w.float().cpu().numpy() for w in net.W]
    bs = [b.cpu().numpy() for b in net.b]
    net = api.Net(Ws, bs, act="silu", wdtype="bf16", sigma_v=sigma_v, device=dev)
    params = FlatParams(net, Ws, bs, dev)
    act = api.workspace(api.neural_act_bytes(net, B), dev)
    bws = api.workspace(api.lib().dsmc_neural_backward_ws(ctypes.byref(net.struct), B), dev)
    dvr = torch.empty(B, 3, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    evs = []

    def one(t):
        y, vr = api.neural_forward_rows(net, x, g, act_save=act)
        api.mse_loss(vr, tgt, sigma_v, dvr, loss)
        api.neural_backward(net, x, act, y, g, dvr, params.dW, params.db, ws=bws)
        params.step(t, 1e-4)

    one(1)
    torch.cuda.synchronize()
    a, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for t in range(steps):
        one(t + 2)
    b_.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b_) / steps
    flop = 3 * MLP_FLOP_PER_PAIR * B
    return {"batch": B, "ms_per_step": ms, "algorithmic_TFLOPs": flop / (ms * 1e-3) / 1e12,
            "harvest_ms_65536_rows": harvest_ms}


def cpu_baseline(pop, Ws, bs, sigma_v, sample_pairs):
    """The oracle's neural step timed on the host on a bounded sample of the
    same workload: a contiguous range of cells starting at grid row 120 (so it
    holds free-stream, shock-band and empty disc cells) with about
    `sample_pairs` pairs.  Timed twice: one thread, and the same cells split
    into contiguous ranges stepped concurrently on all usable cores (threads:
    the oracle's C loops and numpy release the interpreter lock; its random
    numbers are keyed by the global cell id, so the ranges give the same
    result), BLAS pinned to one thread in both."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    cs, perm, _ = oracle.sort_cells(pop.cell_of, pop.n_cells)
    v = pop.v[:, perm]
    nx = int(pop.meta.get("nx", 1))
    k0 = min(120 * nx, pop.n_cells - 1)
    # about P_COLL pairs per particle: take cells until the sample is reached
    target_particles = int(sample_pairs / 0.5)
    k1 = int(np.searchsorted(cs, cs[k0] + target_particles))
    k1 = max(k0 + 1, min(k1, pop.n_cells))
    net = {"Ws": Ws, "bs": bs, "act": "silu", "sigma_v": sigma_v}

    def run_range(a, b):
        sub_cs = (cs[a: b + 1] - cs[a]).astype(np.int32)
        sub_v = v[:, cs[a]: cs[b]].copy()
        _, info = oracle.step(sub_cs, sub_v, pop.xs, pop.lam[a:b].copy(), 11, 0, rule="neural",
                              net=net, cell_base=a)
        return int(info["sel"]["pair_cnt"].sum())

    try:
        n_cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n_cores = os.cpu_count() or 1
    n_cores = max(1, min(n_cores, 16))   # the host share of one GPU
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        if ctx:
            ctx.__enter__()
        t = time.perf_counter()
        npairs = run_range(k0, k1)
        dt1 = time.perf_counter() - t
        bounds = np.linspace(k0, k1, 4 * n_cores + 1).astype(int)
        t = time.perf_counter()
        with ThreadPoolExecutor(n_cores) as ex:
            counts = list(ex.map(lambda ab: run_range(*ab), zip(bounds[:-1], bounds[1:])))
        dtn = time.perf_counter() - t
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    assert sum(counts) == npairs
    sample = (f"cells {k0}..{k1 - 1} of {pop.n_cells} ({int(cs[k1] - cs[k0])} particles, "
              f"{npairs} pairs), one oracle neural step")
    return {"value": npairs / dtn, "unit": "pairs/s", "cores": n_cores, "kind": "oracle",
            "sample": f"{sample}, {4 * n_cores} cell ranges on {n_cores} threads, {dtn:.1f} s",
            "one_thread": {"value": npairs / dt1, "cores": 1, "seconds": dt1}}


def copy_ceiling(dev, nbytes=1 << 30, reps=5):
    """Measured HBM ceiling: a plain device-to-device copy (read + write)."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3)


def stage_rooflines(per, n, n_cells, n_pairs, ceiling):
    """Algorithmic HBM bytes of the memory-bound stages of the FP32 step and
    their rate against the datasheet peak and the measured copy ceiling.
    sort: 36 B/particle (cell id twice, v read + write, perm); moment capture:
    12 B/particle + 48 B/cell; selection: 12 B/particle (velocities) + 12 B per
    accepted pair (i, j, cell) + 8 B/cell (offset, count); isotropic Phase A:
    48 B/pair (pair record 12, velocities 24, direction 12); Phase B + match:
    24 B/particle + 24 B/pair (record 12, Phase-A result 12) + 56 B/cell
    (moments 48, cell bounds 8)."""
    bytes_ = {
        "sort": 36.0 * n,
        "moments": 12.0 * n + 48.0 * n_cells,
        "select": 12.0 * n + 12.0 * n_pairs + 8.0 * n_cells,
        "phaseA_vhs": 48.0 * n_pairs,
        "phaseB_match": 24.0 * n + 24.0 * n_pairs + 56.0 * n_cells,
    }
    out = {}
    for k, b in bytes_.items():
        ms = per[k]
        gbs = b / (ms * 1e-3) / 1e9
        out[k] = {"bytes": b, "ms": ms, "GBps": gbs, "frac_datasheet": gbs * 1e9 / PEAK_HBM,
                  "frac_copy_ceiling": gbs * 1e9 / ceiling}
    return out


if __name__ == "__main__":
    main()
