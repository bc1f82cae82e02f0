"""Python binding of the C-ABI with the same names (argument marshalling only).

Device memory and streams come from PyTorch (ROCm build): arrays are torch
tensors on a HIP device, the stream is torch's current stream.  Every step of
the collision path runs in the library's HIP kernels; nothing here computes.
Velocities are passed as one contiguous [3, N] tensor (SoA rows vx, vy, vz).
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from . import _lib as L
from ._lib import check

_DT = {torch.float32: L.F32, torch.float64: L.F64}


def lib():
    return L.load()


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _vec3(v):
    assert v.dim() == 2 and v.shape[0] == 3 and v.is_contiguous()
    return L.Vec3(v[0].data_ptr(), v[1].data_ptr(), v[2].data_ptr())


def _dtype(v):
    if v.dtype not in _DT:
        raise TypeError(f"velocities must be float32 or float64, got {v.dtype}")
    return _DT[v.dtype]


def workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def new_status(device):
    st = torch.zeros(C.sizeof(L.Status), dtype=torch.uint8, device=device)
    return st


def read_status(st):
    raw = st.cpu().numpy().tobytes()
    return L.Status.from_buffer_copy(raw)


def status_clear(st, stream=None):
    check(lib().dsmc_status_clear(_ptr(st), _stream(stream)), "dsmc_status_clear")


# ---------------------------------------------------------------------------
# Parameter structs
# ---------------------------------------------------------------------------
def xs_struct(xs: dict):
    x = L.Xs()
    if xs["kind"] == "vhs":
        x.kind = L.XS_VHS
        x.m, x.d_ref, x.omega, x.T_ref = xs["m"], xs["d_ref"], xs["omega"], xs["T_ref"]
    elif xs["kind"] == "const":
        x.kind = L.XS_CONST
        x.sigma = xs["sigma"]
        x.m = xs.get("m", 0.0)
    else:
        raise ValueError(xs["kind"])
    return x


def rng_struct(seed, step):
    return L.Rng(int(seed) & 0xFFFFFFFFFFFFFFFF, int(step) & 0xFFFFFFFF, 0)


def potential_jager(p):
    P = L.Potential()
    P.kind = L.POT_JAGER
    P.A, P.a1, P.a2, P.am1, P.am2, P.beta_tt = p.A, p.a1, p.a2, p.am1, p.am2, p.beta_tt
    for q in range(6):
        P.C[q] = p.C[q]
    P.R_eps, P.A_sr, P.a_sr = p.R_eps, p.A_sr, p.a_sr
    return P


def potential_hs(d_angstrom):
    P = L.Potential()
    P.kind = L.POT_HS
    P.d = d_angstrom
    return P


def potential_invpow(K, n):
    P = L.Potential()
    P.kind = L.POT_INVPOW
    P.K = K
    P.n = n
    return P


def quad_struct(n_nodes=64, max_iter=60, scan_ratio=0.95, refine=0):
    return L.Quad(int(n_nodes), int(max_iter), float(scan_ratio), int(refine), 0)


_SPLITS = {"all": L.SPLIT_ALL, "front": L.SPLIT_FRONT, "first": L.SPLIT_FIRST}


class Net:
    """Device copy of an MLP for the C-ABI (keeps the tensors alive)."""

    def __init__(self, Ws, bs, act="silu", wdtype="bf16", sigma_v=1.0, device="cuda",
                 split="all"):
        """split: "all" (every activation a bf16 pair), "front" (the input
        and the first two hidden activations only) or "first" (the input and
        the first hidden activation), see dsmc_mlp.split."""
        if split not in _SPLITS:
            raise ValueError(split)
        self.dims = [int(Ws[0].shape[1])] + [int(w.shape[0]) for w in Ws]
        self.split = split
        self.act = act
        self.wdtype = wdtype
        self.sigma_v = float(sigma_v)
        if wdtype == "bf16":
            self.W = [torch.as_tensor(w, dtype=torch.float32).to(device).to(torch.bfloat16).contiguous() for w in Ws]
            self.b = [torch.as_tensor(b, dtype=torch.float32).to(device).contiguous() for b in bs]
            self.code = L.BF16
        elif wdtype == "f64":
            self.W = [torch.as_tensor(w, dtype=torch.float64).to(device).contiguous() for w in Ws]
            self.b = [torch.as_tensor(b, dtype=torch.float64).to(device).contiguous() for b in bs]
            self.code = L.F64
        elif wdtype == "f32":
            self.W = [torch.as_tensor(w, dtype=torch.float32).to(device).contiguous() for w in Ws]
            self.b = [torch.as_tensor(b, dtype=torch.float32).to(device).contiguous() for b in bs]
            self.code = L.F32
        else:
            raise ValueError(wdtype)
        self.refresh()

    def refresh(self):
        m = L.Mlp()
        m.n_layers = len(self.W)
        for q, d in enumerate(self.dims):
            m.dims[q] = d
        m.act = L.ACT_SILU if self.act == "silu" else L.ACT_RELU
        m.wdtype = self.code
        for q in range(len(self.W)):
            m.W[q] = self.W[q].data_ptr()
            m.b[q] = self.b[q].data_ptr()
        m.sigma_v = self.sigma_v
        m.split = _SPLITS[self.split]
        self.struct = m
        return m


# ---------------------------------------------------------------------------
# Entry points
# ---------------------------------------------------------------------------
def sort_cells(cell_of, n_cells, v_in, st=None, stream=None):
    """Returns (cell_start[n_cells+1], perm[n], v_sorted[3, n])."""
    dev = cell_of.device
    n = int(cell_of.numel())
    v_out = torch.empty_like(v_in)
    cs = torch.empty(n_cells + 1, dtype=torch.int32, device=dev)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    ws_b = lib().dsmc_sort_cells_ws(n, n_cells)
    ws = workspace(ws_b, dev)
    check(lib().dsmc_sort_cells(n, n_cells, _ptr(cell_of), _dtype(v_in), _vec3(v_in), _vec3(v_out),
                                _ptr(cs), _ptr(perm), _ptr(ws), ws_b, _ptr(st), _stream(stream)),
          "dsmc_sort_cells")
    return cs, perm[:n], v_out


def moment_match(cell_start, v, mom, mode, pair_cnt=None, st=None, stream=None):
    n_cells = int(cell_start.numel()) - 1
    check(lib().dsmc_moment_match(n_cells, _ptr(cell_start), _dtype(v), _vec3(v), _ptr(mom),
                                  int(mode), _ptr(pair_cnt), _ptr(st), _stream(stream)),
          "dsmc_moment_match")


def sort_cells_noalloc(cell_of, n_cells, v_in, cs, perm, v_out, st=None, stream=None):
    """dsmc_sort_cells_noalloc into caller-provided outputs (the library's
    static scratch; n and n_cells at most 2^20)."""
    check(lib().dsmc_sort_cells_noalloc(int(cell_of.numel()), int(n_cells), _ptr(cell_of),
                                        _dtype(v_in), _vec3(v_in), _vec3(v_out), _ptr(cs),
                                        _ptr(perm), _ptr(st), _stream(stream)),
          "dsmc_sort_cells_noalloc")


class PairList:
    def __init__(self, n_cells, cap, device):
        self.cap = int(cap)
        self.off = torch.zeros(n_cells, dtype=torch.int32, device=device)
        self.cnt = torch.zeros(n_cells, dtype=torch.int32, device=device)
        self.i = torch.zeros(self.cap + 1, dtype=torch.int32, device=device)
        self.j = torch.zeros(self.cap + 1, dtype=torch.int32, device=device)
        self.cell = torch.zeros(self.cap + 1, dtype=torch.int32, device=device)

    def struct(self):
        return L.Pairs(self.off.data_ptr(), self.cnt.data_ptr(), self.i.data_ptr(),
                       self.j.data_ptr(), self.cell.data_ptr(), self.cap)


def select_pairs_ntc(cell_start, v, xs, lam, mom, seed, step, pairs, ws=None, st=None,
                     stream=None):
    n_cells = int(cell_start.numel()) - 1
    need = lib().dsmc_select_pairs_ntc_ws(n_cells, pairs.cap)
    if ws is None or ws.numel() < need:
        ws = workspace(need, v.device)
    check(lib().dsmc_select_pairs_ntc(n_cells, _ptr(cell_start), _dtype(v), _vec3(v),
                                      xs_struct(xs), _ptr(lam), _ptr(mom), rng_struct(seed, step),
                                      pairs.struct(), _ptr(ws), int(ws.numel()), _ptr(st),
                                      _stream(stream)),
          "dsmc_select_pairs_ntc")
    return ws


def select_pairs_sbt(cell_start, v, xs, lam, seed, step, pairs, ws=None, st=None, stream=None):
    n_cells = int(cell_start.numel()) - 1
    need = lib().dsmc_select_pairs_sbt_ws(n_cells, pairs.cap)
    if ws is None or ws.numel() < need:
        ws = workspace(need, v.device)
    check(lib().dsmc_select_pairs_sbt(n_cells, _ptr(cell_start), _dtype(v), _vec3(v),
                                      xs_struct(xs), _ptr(lam), rng_struct(seed, step),
                                      pairs.struct(), _ptr(ws), int(ws.numel()), _ptr(st),
                                      _stream(stream)),
          "dsmc_select_pairs_sbt")
    return ws


def collide_ws(cap, v, extra=0):
    return workspace(lib().dsmc_collide_ws(int(cap), _dtype(v)) + int(extra), v.device)


def collide_vhs(v, pairs, seed, step, schedule=L.SCHED_AUTO, ws=None, stream=None):
    n_cells = int(pairs.off.numel())
    if ws is None:
        ws = collide_ws(pairs.cap, v)
    check(lib().dsmc_collide_vhs(n_cells, _dtype(v), _vec3(v), pairs.struct(),
                                 rng_struct(seed, step), int(schedule), _ptr(ws), int(ws.numel()),
                                 _stream(stream)),
          "dsmc_collide_vhs")
    return ws


def apply_pairs(v, pairs, kind, ws, schedule=L.SCHED_AUTO, stream=None):
    n_cells = int(pairs.off.numel())
    check(lib().dsmc_apply_pairs(n_cells, _dtype(v), _vec3(v), pairs.struct(), int(kind),
                                 int(schedule), _ptr(ws), int(ws.numel()), _stream(stream)),
          "dsmc_apply_pairs")


def apply_pairs_match(cell_start, v, pairs, kind, mom, ws, mode=L.MM_APPLY, st=None,
                      stream=None):
    n_cells = int(cell_start.numel()) - 1
    if n_cells != int(pairs.off.numel()):
        raise ValueError("apply_pairs_match: cell_start and pairs cover different cell counts")
    check(lib().dsmc_apply_pairs_match(n_cells, _ptr(cell_start), _dtype(v), _vec3(v),
                                       pairs.struct(), int(kind), _ptr(mom), int(mode), _ptr(ws),
                                       int(ws.numel()), _ptr(st), _stream(stream)),
          "dsmc_apply_pairs_match")


def deflect_jager(b, g, m_red, pot, quad=None, fold=False, st=None, stream=None):
    chi = torch.empty_like(g)
    q = quad if quad is not None else quad_struct()
    check(lib().dsmc_deflect_jager(int(b.numel()), _dtype(b), _ptr(b), _ptr(g), _ptr(chi),
                                   float(m_red), C.byref(pot), q, int(bool(fold)), _ptr(st),
                                   _stream(stream)),
          "dsmc_deflect_jager")
    return chi


def collide_jager(v, pairs, seed, step, m_red, b_max, pot, quad=None, schedule=L.SCHED_AUTO,
                  ws=None, st=None, stream=None):
    n_cells = int(pairs.off.numel())
    if ws is None:
        ws = collide_ws(pairs.cap, v)
    q = quad if quad is not None else quad_struct()
    check(lib().dsmc_collide_jager(n_cells, _dtype(v), _vec3(v), pairs.struct(),
                                   rng_struct(seed, step), float(m_red), float(b_max), C.byref(pot),
                                   q, int(schedule), _ptr(ws), int(ws.numel()), _ptr(st),
                                   _stream(stream)),
          "dsmc_collide_jager")
    return ws


def neural_ws(net, pairs, v):
    extra = 0
    if net.wdtype != "bf16":
        extra = lib().dsmc_neural_act_bytes(C.byref(net.struct), int(pairs.cap))
    return collide_ws(pairs.cap, v, extra)


def neural_collide(net, v, pairs, seed, step, schedule=L.SCHED_AUTO, ws=None, st=None,
                   stream=None):
    n_cells = int(pairs.off.numel())
    if ws is None:
        ws = neural_ws(net, pairs, v)
    check(lib().dsmc_neural_collide(C.byref(net.struct), n_cells, _dtype(v), _vec3(v),
                                    pairs.struct(), rng_struct(seed, step), int(schedule),
                                    _ptr(ws), int(ws.numel()), _ptr(st), _stream(stream)),
          "dsmc_neural_collide")
    return ws


def neural_act_bytes(net, B):
    return int(lib().dsmc_neural_act_bytes(C.byref(net.struct), int(B)))


def neural_forward_rows(net, x, g, act_save=None, stream=None):
    """Rows form: returns (y_raw [B, dout], vr_out [B, 3])."""
    B = int(x.shape[0])
    y = torch.empty(B, net.dims[-1], dtype=x.dtype, device=x.device)
    vr = torch.empty(B, 3, dtype=x.dtype, device=x.device)
    ab = int(act_save.numel()) if act_save is not None else 0
    check(lib().dsmc_neural_forward_rows(C.byref(net.struct), B, _ptr(x), _ptr(g), _ptr(y),
                                         _ptr(vr), _ptr(act_save), ab, _stream(stream)),
          "dsmc_neural_forward_rows")
    return y, vr


def neural_backward(net, x, act_save, y_raw, g, dL_dvr, dW, db, dx=None, accumulate=False,
                    ws=None, stream=None):
    B = int(x.shape[0])
    need = lib().dsmc_neural_backward_ws(C.byref(net.struct), B)
    if ws is None or ws.numel() < need:
        ws = workspace(need, x.device)
    nl = len(net.W)
    dWp = (C.c_void_p * nl)(*[t.data_ptr() for t in dW])
    dbp = (C.c_void_p * nl)(*[t.data_ptr() for t in db])
    check(lib().dsmc_neural_backward(C.byref(net.struct), B, _ptr(x), _ptr(act_save),
                                     _ptr(y_raw), _ptr(g), _ptr(dL_dvr), dWp, dbp, _ptr(dx),
                                     int(bool(accumulate)), _ptr(ws), int(ws.numel()),
                                     _stream(stream)),
          "dsmc_neural_backward")
    return ws


def moment_match_backward(cell_start, mom_pre, v_post, G, stream=None):
    out = torch.empty_like(G)
    n_cells = int(cell_start.numel()) - 1
    check(lib().dsmc_moment_match_backward(n_cells, _ptr(cell_start), _ptr(mom_pre),
                                           _ptr(v_post[0]), _ptr(v_post[1]), _ptr(v_post[2]),
                                           _ptr(G[0]), _ptr(G[1]), _ptr(G[2]), _ptr(out[0]),
                                           _ptr(out[1]), _ptr(out[2]), _stream(stream)),
          "dsmc_moment_match_backward")
    return out


def direction_loss(vr_new, vr_target, dL_dvr, loss, stream=None):
    check(lib().dsmc_direction_loss(int(vr_new.shape[0]), _ptr(vr_new), _ptr(vr_target),
                                    _ptr(dL_dvr), _ptr(loss), _stream(stream)),
          "dsmc_direction_loss")


def mse_loss(vr_new, vr_target, sigma_v, dL_dvr, loss, stream=None):
    check(lib().dsmc_mse_loss(int(vr_new.shape[0]), _ptr(vr_new), _ptr(vr_target),
                              float(sigma_v), _ptr(dL_dvr), _ptr(loss), _stream(stream)),
          "dsmc_mse_loss")


def cosine_lr(t, T, lr_max, lr_min=1e-6):
    return float(lib().dsmc_cosine_lr(int(t), int(T), float(lr_max), float(lr_min)))


def adam_step(param, grad, m, v, t, lr, param_bf16=None, beta1=0.9, beta2=0.999, eps=1e-8,
              stream=None):
    check(lib().dsmc_adam_step(int(param.numel()), _ptr(param), _ptr(param_bf16), _ptr(grad),
                               _ptr(m), _ptr(v), int(t), float(lr), float(beta1), float(beta2),
                               float(eps), _stream(stream)),
          "dsmc_adam_step")


def harvest_rows(vr, xi, z, sigma_v, b_max, m_red, pot, quad=None, st=None, stream=None):
    B = int(vr.shape[0])
    dev = vr.device
    x = torch.empty(B, 8, dtype=torch.float32, device=dev)
    g = torch.empty(B, dtype=torch.float32, device=dev)
    tgt = torch.empty(B, 3, dtype=torch.float32, device=dev)
    chi = torch.empty(B, dtype=torch.float64, device=dev)
    q = quad if quad is not None else quad_struct()
    check(lib().dsmc_harvest_rows(B, _ptr(vr), _ptr(xi), _ptr(z), float(sigma_v), float(b_max),
                                  float(m_red), C.byref(pot), q, _ptr(x), _ptr(g), _ptr(tgt),
                                  _ptr(chi), _ptr(st), _stream(stream)),
          "dsmc_harvest_rows")
    return x, g, tgt, chi


def transport_q2(E_kelvin, b_cut, pot, n_panels=256, n_gl=8, quad=None, st=None, stream=None):
    n = int(E_kelvin.numel())
    Q = torch.empty(n, dtype=torch.float64, device=E_kelvin.device)
    ws = workspace(lib().dsmc_transport_q2_ws(n, int(n_panels), int(n_gl)), E_kelvin.device)
    q = quad if quad is not None else quad_struct()
    check(lib().dsmc_transport_q2(n, _ptr(E_kelvin), float(b_cut), int(n_panels), int(n_gl),
                                  C.byref(pot), q, _ptr(Q), _ptr(ws), int(ws.numel()), _ptr(st),
                                  _stream(stream)),
          "dsmc_transport_q2")
    return Q


def viscosity_ce(T, m, b_cut, pot, n_panels=256, n_gl=8, n_lag=16, mode=L.CE_STANDARD,
                 quad=None, st=None, stream=None):
    n = int(T.numel())
    omega = torch.empty(n, dtype=torch.float64, device=T.device)
    mu = torch.empty_like(omega)
    ws = workspace(lib().dsmc_viscosity_ce_ws(n, int(n_panels), int(n_gl), int(n_lag)), T.device)
    q = quad if quad is not None else quad_struct()
    check(lib().dsmc_viscosity_ce(n, _ptr(T), float(m), float(b_cut), int(n_panels), int(n_gl),
                                  int(n_lag), int(mode), C.byref(pot), q, _ptr(omega), _ptr(mu),
                                  _ptr(ws), int(ws.numel()), _ptr(st), _stream(stream)),
          "dsmc_viscosity_ce")
    return omega, mu


def set_block_threshold(pairs):
    check(lib().dsmc_set_block_threshold(int(pairs)), "dsmc_set_block_threshold")


def get_block_threshold():
    return int(lib().dsmc_get_block_threshold())


def set_match_schedule(wave_per_cu, medium_per_cu, big_per_cu):
    m = L.MatchSchedule(int(wave_per_cu), int(medium_per_cu), int(big_per_cu), 0)
    check(lib().dsmc_set_match_schedule(C.byref(m)), "dsmc_set_match_schedule")


def get_match_schedule():
    m = L.MatchSchedule()
    check(lib().dsmc_get_match_schedule(C.byref(m)), "dsmc_get_match_schedule")
    return (m.wave_per_cu, m.medium_per_cu, m.big_per_cu)


# ---------------------------------------------------------------------------
# Angle network and deflection-angle table
# ---------------------------------------------------------------------------
ANGLE_DIMS = (2, 512, 512, 512, 256, 128, 1)


class AngleNet:
    """Device copy of the angle network (bf16 weights for the matrix cores,
    fp32 biases; FP32 master copies for training)."""

    def __init__(self, Ws, bs, device="cuda"):
        self.dims = [int(Ws[0].shape[1])] + [int(w.shape[0]) for w in Ws]
        self.master_W = [torch.as_tensor(w, dtype=torch.float32).to(device).contiguous() for w in Ws]
        self.b = [torch.as_tensor(b, dtype=torch.float32).to(device).contiguous() for b in bs]
        self.W = [w.to(torch.bfloat16).contiguous() for w in self.master_W]
        self.refresh()

    def refresh(self):
        a = L.Anet()
        a.n_layers = len(self.W)
        for q, d in enumerate(self.dims):
            a.dims[q] = d
        for q in range(len(self.W)):
            a.W[q] = self.W[q].data_ptr()
            a.b[q] = self.b[q].data_ptr()
        self.struct = a
        return a


def anet_ws(net, rows, device):
    return workspace(lib().dsmc_anet_ws(C.byref(net.struct), int(rows)), device)


def anet_forward(net, x, y=None, ws=None, stream=None):
    R = int(x.shape[0])
    if y is None:
        y = torch.empty(R, dtype=torch.float32, device=x.device)
    if ws is None:
        ws = anet_ws(net, R, x.device)
    check(lib().dsmc_anet_forward(C.byref(net.struct), R, _ptr(x), _ptr(y), _ptr(ws),
                                  int(ws.numel()), _stream(stream)),
          "dsmc_anet_forward")
    return y, ws


def anet_backward(net, dy, dW, db, ws, stream=None):
    R = int(dy.shape[0])
    pw = (C.c_void_p * len(dW))(*[t.data_ptr() for t in dW])
    pb = (C.c_void_p * len(db))(*[t.data_ptr() for t in db])
    check(lib().dsmc_anet_backward(C.byref(net.struct), R, _ptr(dy), pw, pb, _ptr(ws),
                                   int(ws.numel()), _stream(stream)),
          "dsmc_anet_backward")


def huber_loss(yhat, y, dy, loss, stream=None):
    check(lib().dsmc_huber_loss(int(yhat.numel()), _ptr(yhat), _ptr(y), _ptr(dy), _ptr(loss),
                                _stream(stream)),
          "dsmc_huber_loss")


def anet_rows(b, g, chi, m_red, lne_lo, lne_hi, b_max, stream=None):
    n = int(b.numel())
    x = torch.empty(n, 2, dtype=torch.float32, device=b.device)
    y = torch.empty(n, dtype=torch.float32, device=b.device)
    check(lib().dsmc_anet_rows(n, _ptr(b), _ptr(g), _ptr(chi), float(m_red), float(lne_lo),
                               float(lne_hi), float(b_max), _ptr(x), _ptr(y), _stream(stream)),
          "dsmc_anet_rows")
    return x, y


class ChiTable:
    """theta[n_e][n_b] on the (ln E, b / b_max) grid (device)."""

    def __init__(self, n_e, n_b, lne_lo, lne_hi, device="cuda", theta=None):
        self.theta = (torch.zeros(n_e, n_b, dtype=torch.float32, device=device) if theta is None
                      else torch.as_tensor(theta, dtype=torch.float32).to(device).contiguous())
        self.struct = L.ChiTable(int(n_e), int(n_b), float(lne_lo), float(lne_hi),
                                 self.theta.data_ptr())


def chi_table_build(net, tab, ws=None, stream=None):
    if ws is None:
        ws = workspace(lib().dsmc_chi_table_ws(C.byref(net.struct), C.byref(tab.struct)),
                       tab.theta.device)
    check(lib().dsmc_chi_table_build(C.byref(net.struct), C.byref(tab.struct), _ptr(ws),
                                     int(ws.numel()), _stream(stream)),
          "dsmc_chi_table_build")
    return ws


def collide_table(tab, v, pairs, seed, step, m_red, schedule=L.SCHED_AUTO, ws=None, stream=None):
    if ws is None:
        ws = collide_ws(pairs.cap, v)
    check(lib().dsmc_collide_table(C.byref(tab.struct), int(pairs.off.numel()), _dtype(v), _vec3(v),
                                   pairs.struct(), rng_struct(seed, step), float(m_red),
                                   int(schedule), _ptr(ws), int(ws.numel()), _stream(stream)),
          "dsmc_collide_table")
    return ws


# ---------------------------------------------------------------------------
# Flow loop around the collision step: move, gather, sampling, fields
# ---------------------------------------------------------------------------
def domain(nx, ny, Lx, Ly, kinds, T_w, u_w, m):
    """dsmc_domain; kinds / T_w / u_w per side (x = 0, x = Lx, y = 0, y = Ly)."""
    d = L.Domain()
    d.nx, d.ny, d.Lx, d.Ly, d.m = int(nx), int(ny), float(Lx), float(Ly), float(m)
    for q in range(4):
        d.kind[q] = int(kinds[q])
        d.T_w[q] = float(T_w[q])
        for c in range(3):
            d.u_w[q][c] = float(u_w[q][c])
    return d


def _vec2(p):
    assert p.dim() == 2 and p.shape[0] == 2 and p.is_contiguous()
    return L.Vec3(p[0].data_ptr(), p[1].data_ptr(), None)


def move(pos, v, dom, dt, seed, step, cell_of=None, st=None, stream=None):
    """Free flight over dt with wall events, in place on pos[2, n] and
    v[3, n] (same dtype); returns cell_of[n] (int32)."""
    n = int(v.shape[1])
    if pos.dtype != v.dtype or int(pos.shape[1]) != n:
        raise ValueError("move: positions and velocities must match in dtype and count")
    if cell_of is None:
        cell_of = torch.empty(n, dtype=torch.int32, device=v.device)
    check(lib().dsmc_move(n, _dtype(v), _vec2(pos), _vec3(v), C.byref(dom), float(dt),
                          rng_struct(seed, step), _ptr(cell_of), _ptr(st), _stream(stream)),
          "dsmc_move")
    return cell_of


def gather(perm, src, out=None, stream=None):
    """out[:, s] = src[:, perm[s]] for a [2, n] or [3, n] array."""
    if out is None:
        out = torch.empty_like(src)
    rows = int(src.shape[0])
    if rows not in (2, 3):
        raise ValueError("gather: 2 or 3 rows")
    vin = _vec2(src) if rows == 2 else _vec3(src)
    vout = _vec2(out) if rows == 2 else _vec3(out)
    check(lib().dsmc_gather(int(src.shape[1]), _dtype(src), _ptr(perm), vin, vout,
                            _stream(stream)), "dsmc_gather")
    return out


def sample(cell_start, v, acc=None, stream=None):
    """acc[n_cells, 13] += the raw per-cell moment sums of v (FP64)."""
    n_cells = int(cell_start.numel()) - 1
    if acc is None:
        acc = torch.zeros(n_cells, 13, dtype=torch.float64, device=v.device)
    check(lib().dsmc_sample(n_cells, _ptr(cell_start), _dtype(v), _vec3(v), _ptr(acc),
                            _stream(stream)), "dsmc_sample")
    return acc


def sample_fields(acc, n_samples, mass, fnum_per_volume, out=None, stream=None):
    """Fields [n_cells, 9]: n, ux, uy, uz, T, tau_xy, qx, qy, qz."""
    n_cells = int(acc.shape[0])
    if out is None:
        out = torch.empty(n_cells, 9, dtype=torch.float64, device=acc.device)
    check(lib().dsmc_sample_fields(n_cells, _ptr(acc), float(n_samples), float(mass),
                                   float(fnum_per_volume), _ptr(out), _stream(stream)),
          "dsmc_sample_fields")
    return out
