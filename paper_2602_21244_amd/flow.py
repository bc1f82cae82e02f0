"""The DSMC flow loop around the collision step (section "Results and
Discussion": the Couette channel and the lid-driven cavity), on one GPU.

Each step runs, on the library's kernels only: move (free flight, wall
events, cell index) -> bin by cell (sort, gather of positions) -> cell moments
-> NTC selection -> the collision rule (isotropic, per-pair network, angle
table) -> Phase B (fused with the cell-wise moment matching for the network
rule) -> optional sampling of the macroscopic fields.  This module allocates
the buffers once and orders the calls.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from . import api


class FlowSim:
    def __init__(self, flow, dtype=torch.float64, rule="vhs", net=None, table=None,
                 seed=0, device=None, cap=None):
        self.dev = device or torch.device("cuda:0")
        self.rule = rule
        self.net = net
        self.table = table
        self.seed = int(seed)
        self.dt = float(flow.dt)
        self.m = float(flow.xs["m"])
        self.xs = flow.xs
        self.n = flow.n
        self.n_cells = flow.n_cells
        self.fnum_per_volume = float(flow.fnum_per_volume)
        self.dom = api.domain(flow.nx, flow.ny, flow.Lx, flow.Ly, flow.kinds, flow.T_w,
                              flow.u_w, self.m)
        d = self.dev
        self.pos = torch.as_tensor(flow.pos, dtype=dtype, device=d).contiguous()
        self.v = torch.as_tensor(flow.v, dtype=dtype, device=d).contiguous()
        self.pos_b = torch.empty_like(self.pos)
        self.v_b = torch.empty_like(self.v)
        self.cell_of = torch.empty(self.n, dtype=torch.int32, device=d)
        self.cs = torch.zeros(self.n_cells + 1, dtype=torch.int32, device=d)
        self.perm = torch.empty(max(self.n, 1), dtype=torch.int32, device=d)
        self.sort_ws_b = L.load().dsmc_sort_cells_ws(self.n, self.n_cells)
        self.sort_ws = api.workspace(self.sort_ws_b, d)
        self.lam = torch.as_tensor(flow.lam, dtype=torch.float64, device=d)
        self.mom = torch.zeros(self.n_cells * 6, dtype=torch.float64, device=d)
        self.cap = int(cap or max(4 * self.n, 1 << 16))
        self.pairs = api.PairList(self.n_cells, self.cap, d)
        self.sel_ws = api.workspace(L.load().dsmc_select_pairs_ntc_ws(self.n_cells, self.cap), d)
        if rule == "neural":
            self.col_ws = api.neural_ws(net, self.pairs, self.v)
        else:
            self.col_ws = api.collide_ws(self.cap, self.v)
        self.st = api.new_status(d)
        self.acc = torch.zeros(self.n_cells, 13, dtype=torch.float64, device=d)
        self.n_samples = 0
        self.step_no = 0

    def _sort(self):
        lib = L.load()
        api.check(lib.dsmc_sort_cells(self.n, self.n_cells, api._ptr(self.cell_of),
                                      api._dtype(self.v), api._vec3(self.v),
                                      api._vec3(self.v_b), api._ptr(self.cs),
                                      api._ptr(self.perm), api._ptr(self.sort_ws),
                                      self.sort_ws_b, api._ptr(self.st), api._stream()),
                  "dsmc_sort_cells")
        api.gather(self.perm[: self.n], self.pos, self.pos_b)
        self.pos, self.pos_b = self.pos_b, self.pos
        self.v, self.v_b = self.v_b, self.v

    def step(self, sample=False):
        k, s = self.step_no, self.seed
        api.move(self.pos, self.v, self.dom, self.dt, s, k, cell_of=self.cell_of, st=self.st)
        self._sort()
        api.moment_match(self.cs, self.v, self.mom, L.MM_CAPTURE)
        api.select_pairs_ntc(self.cs, self.v, self.xs, self.lam, self.mom, s, k, self.pairs,
                             ws=self.sel_ws, st=self.st)
        if self.rule == "vhs":
            api.collide_vhs(self.v, self.pairs, s, k, ws=self.col_ws)
        elif self.rule == "neural":
            api.neural_collide(self.net, self.v, self.pairs, s, k, schedule=L.SCHED_DEFER,
                               ws=self.col_ws, st=self.st)
            api.apply_pairs_match(self.cs, self.v, self.pairs, L.APPLY_DIRECTIONS, self.mom,
                                  self.col_ws, st=self.st)
        elif self.rule == "table":
            api.collide_table(self.table, self.v, self.pairs, s, k, self.m / 2,
                              ws=self.col_ws)
        else:
            raise ValueError(self.rule)
        if sample:
            api.sample(self.cs, self.v, self.acc)
            self.n_samples += 1
        self.step_no += 1

    def run(self, steps, sample_from=None):
        for _ in range(steps):
            self.step(sample=sample_from is not None and self.step_no >= sample_from)

    def status(self):
        st = api.read_status(self.st)
        if st.flags & L.ST_PAIR_OVERFLOW:
            raise RuntimeError(f"pair capacity {self.cap} exceeded (needed {st.n_cand})")
        return st

    def fields(self):
        if self.n_samples == 0:
            raise RuntimeError("no samples taken")
        return api.sample_fields(self.acc, self.n_samples, self.m, self.fnum_per_volume)
