"""Autotuner of the Phase-B schedules.

Phase B can walk a cell's pairs in one lane (LANE) or spread a cell over a
workgroup in dependency rounds (BLOCK).  AUTO uses BLOCK for cells with more
pairs than a threshold.  The best threshold depends on the cell-size
histogram, so it is measured on the actual pair list: each candidate
threshold is timed with HIP events on a scratch copy of the velocities and the
fastest is installed with dsmc_set_block_threshold.  The fused Phase B +
moment matching of the timed step (dsmc_apply_pairs_match) runs three
persistent kernels (wave per cell, medium and big block per cell) whose grid
sizes are tuned the same way (dsmc_set_match_schedule).  Results are cached
per (device name, pair-count histogram signature) in a JSON file.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import api

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dsmc_gfx950_autotune.json")
CANDIDATES = (8, 16, 32, 48, 64, 128, 256, 1 << 30)


def _signature(pairs):
    cnt = pairs.cnt.cpu().numpy()
    edges = [0, 1, 8, 32, 128, 512, 2048, 1 << 30]
    h, _ = np.histogram(cnt, bins=edges)
    # coarse (log2) histogram so similar workloads share an entry
    return ",".join(str(int(np.log2(x + 1))) for x in h)


def _load_cache():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except Exception:
        return {}


def _save_cache(c):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(c, f, indent=1)
    except OSError:
        pass


def tune_block_threshold(v, pairs, ws, kind=api.L.APPLY_DIRECTIONS, reps=3, use_cache=True):
    """Measure Phase B for each threshold; install and return the fastest.

    v: sorted velocities [3, N]; pairs/ws: a selection and the Phase-A results
    of a collide call made with schedule DSMC_SCHED_DEFER."""
    key = f"{torch.cuda.get_device_name(v.device)}|{kind}|{_signature(pairs)}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        api.set_block_threshold(cache[key]["threshold"])
        return cache[key]["threshold"], cache[key]["ms"]
    scratch = torch.empty_like(v)
    times = {}
    for thr in CANDIDATES:
        api.set_block_threshold(thr)
        best = float("inf")
        for _ in range(reps):
            scratch.copy_(v)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            api.apply_pairs(scratch, pairs, kind, ws, schedule=api.L.SCHED_AUTO)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        times[thr] = best
    thr = min(times, key=times.get)
    api.set_block_threshold(thr)
    cache[key] = {"threshold": int(thr), "ms": {str(k): v_ for k, v_ in times.items()}}
    if use_cache:
        _save_cache(cache)
    return thr, times


MATCH_CANDIDATES = tuple((w, m, b) for w in (8, 16, 24, 40, 64) for m in (1, 2, 4) for b in (1, 2))


def tune_match_schedule(cell_start, v, pairs, kind, mom, ws, reps=3, use_cache=True):
    """Time dsmc_apply_pairs_match for each launch shape on a scratch copy of
    the velocities; install and return the fastest (wave, medium, big
    workgroups per CU) and the times.

    v: sorted velocities [3, N]; pairs/ws: a selection and the Phase-A results
    of a collide call made with schedule DSMC_SCHED_DEFER; mom: the captured
    pre-collision moments."""
    key = f"{torch.cuda.get_device_name(v.device)}|match{kind}|{_signature(pairs)}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        shape = tuple(cache[key]["shape"])
        api.set_match_schedule(*shape)
        return shape, cache[key]["ms"]
    scratch = torch.empty_like(v)
    times = {}
    for shape in MATCH_CANDIDATES:
        api.set_match_schedule(*shape)
        best = float("inf")
        for _ in range(reps):
            scratch.copy_(v)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            api.apply_pairs_match(cell_start, scratch, pairs, kind, mom, ws)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        times[shape] = best
    shape = min(times, key=times.get)
    api.set_match_schedule(*shape)
    cache[key] = {"shape": list(shape), "ms": {"/".join(map(str, k)): t for k, t in times.items()}}
    if use_cache:
        _save_cache(cache)
    return shape, times
