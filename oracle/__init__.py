"""CPU FP64 oracle of the DSMC collision step -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct implementation of what the GPU library
computes, used to check it.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package; the product
package never does.  It shares no code with the GPU path: the per-cell loops
live in ``dsmc_oracle.c`` (plain C, FP64, built with gcc) and the network parts
below are plain numpy in FP64.

Parity status of each function is recorded next to it; every function is
pinned by a CPU test against something other than itself (closed forms,
library routines, published test vectors, brute force, finite differences).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dsmc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_dsmc_oracle.so")
_lib = None

KB = 1.380649e-23


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build(force=True)
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")


class Potential(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("A", C.c_double),
                ("a1", C.c_double), ("a2", C.c_double), ("am1", C.c_double),
                ("am2", C.c_double), ("beta_tt", C.c_double), ("C", C.c_double * 6),
                ("R_eps", C.c_double), ("A_sr", C.c_double), ("a_sr", C.c_double),
                ("d", C.c_double), ("K", C.c_double)]


POT_JAGER, POT_HS, POT_INVPOW = 0, 1, 2


class Domain(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("Lx", C.c_double), ("Ly", C.c_double),
                ("kind", C.c_int32 * 4), ("T_w", C.c_double * 4),
                ("u_w", (C.c_double * 3) * 4), ("m", C.c_double)]


WALL_PERIODIC, WALL_SPECULAR, WALL_DIFFUSE = 0, 1, 2


def _declare(L):
    L.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.orc_sort_cells.argtypes = [C.c_int32, C.c_int32, _i32p, _i32p, _i32p]
    L.orc_sort_cells.restype = C.c_int
    L.orc_moments.argtypes = [C.c_int32, _i32p, _f64p, _f64p, _f64p, _f64p]
    L.orc_select_ntc.argtypes = [C.c_int32, _i32p, _f64p, _f64p, _f64p, C.c_double,
                                 C.c_double, _f64p, _f64p, C.c_uint64, C.c_uint32, C.c_int32,
                                 _i32p, _i32p, _i32p, _i32p, _i32p, C.c_int64,
                                 C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.orc_select_ntc.restype = C.c_int
    L.orc_select_sbt.argtypes = [C.c_int32, _i32p, _f64p, _f64p, _f64p, C.c_double,
                                 C.c_double, _f64p, C.c_uint64, C.c_uint32, C.c_int32,
                                 _i32p, _i32p, _i32p, _i32p, _i32p, C.c_int64,
                                 C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int32)]
    L.orc_select_sbt.restype = C.c_int
    L.orc_pair_latents.argtypes = [C.c_int64, _i32p, _i32p, C.c_uint64, C.c_uint32,
                                   C.c_int32, C.c_int, _f64p, _f64p, _f64p]
    L.orc_vhs_dirs.argtypes = [C.c_int64, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p,
                               _f64p, _f64p]
    L.orc_apply_dirs.argtypes = [C.c_int32, _i32p, _i32p, _i32p, _i32p, _f64p, _f64p,
                                 _f64p, _f64p]
    L.orc_apply_chi.argtypes = [C.c_int32, _i32p, _i32p, _i32p, _i32p, _f64p, _f64p,
                                _f64p, _f64p, _f64p, _f64p]
    L.orc_moment_match.argtypes = [C.c_int32, _i32p, _f64p, C.c_void_p, C.c_int, _f64p,
                                   _f64p, _f64p]
    L.orc_moment_match.restype = C.c_int32
    L.orc_potential_V.argtypes = [C.POINTER(Potential), C.c_double]
    L.orc_potential_V.restype = C.c_double
    L.orc_chi.argtypes = [C.POINTER(Potential), C.c_double, C.c_double,
                          C.POINTER(C.c_int), C.POINTER(C.c_int64)]
    L.orc_chi.restype = C.c_double
    L.orc_chi_batch.argtypes = [C.POINTER(Potential), C.c_int64, _f64p, _f64p, C.c_double,
                                _f64p, _i32p, C.c_int]
    L.orc_step_vhs.argtypes = [C.c_int32, _i32p, _f64p, _f64p, _f64p, C.c_double,
                               C.c_double, _f64p, C.c_uint64, C.c_uint32, C.c_int, C.c_int,
                               C.c_int]
    L.orc_step_vhs.restype = C.c_int64
    L.orc_move.argtypes = [C.c_int32, C.POINTER(Domain), C.c_double, C.c_uint64, C.c_uint32,
                           _f64p, _f64p, _f64p, _f64p, _f64p, _i32p, C.POINTER(C.c_int64)]
    L.orc_move.restype = C.c_int64
    L.orc_sample.argtypes = [C.c_int32, _i32p, _f64p, _f64p, _f64p, _f64p]


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# RNG, sort, moments
# ---------------------------------------------------------------------------
def philox(ctr, key):
    """Philox4x32-10 of one (ctr[4], key[2]) -> 4 uint32 words."""
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_c(ctr, np.uint32), _c(key, np.uint32), out)
    return out


def sort_cells(cell_of, n_cells):
    """Stable counting sort: (cell_start[n_cells+1], perm[n], n_bad)."""
    cell_of = _c(cell_of, np.int32)
    n = cell_of.shape[0]
    cs = np.zeros(n_cells + 1, np.int32)
    perm = np.zeros(max(n, 1), np.int32)
    bad = lib().orc_sort_cells(n, n_cells, cell_of, cs, perm)
    return cs, perm[: n - bad], bad


def moments(cell_start, v):
    """Per-cell (ux, uy, uz, S, cmax, E) for SoA v[3, n] in sorted order."""
    n_cells = len(cell_start) - 1
    mom = np.zeros(max(n_cells, 1) * 6)
    v = _c(v, np.float64)
    lib().orc_moments(n_cells, _c(cell_start, np.int32), _c(v[0], np.float64),
                      _c(v[1], np.float64), _c(v[2], np.float64), mom)
    return mom[: n_cells * 6].reshape(n_cells, 6)


# ---------------------------------------------------------------------------
# Cross sections (Bird 1994; the paper keeps the cross-section model of the
# selection stage unchanged): sigma_T(g) g = C g^e.
# ---------------------------------------------------------------------------
def sigma_g_law(xs):
    """(C, e) with sigma_T(g) * g = C * g**e for a cross-section description.

    VHS: sigma_T = pi d_ref^2 (2 k T_ref / (m_r g^2))^(omega - 1/2) / Gamma(5/2 - omega)
         with m_r = m/2, so C = pi d_ref^2 (2 k T_ref / m_r)^(omega-1/2) / Gamma(5/2-omega)
         and e = 2 - 2 omega.
    constant sigma: C = sigma, e = 1.
    """
    if xs["kind"] == "vhs":
        mr = xs["m"] / 2.0
        om = xs["omega"]
        Cc = (math.pi * xs["d_ref"] ** 2 * (2.0 * KB * xs["T_ref"] / mr) ** (om - 0.5)
              / math.gamma(2.5 - om))
        return Cc, 2.0 - 2.0 * om
    if xs["kind"] == "const":
        return float(xs["sigma"]), 1.0
    raise ValueError(xs["kind"])


def select_ntc(cell_start, v, xs, lam, mom, seed, step, cap=None, cell_base=0):
    """NTC selection; returns dict with pair_off, pair_cnt, pair_i, pair_j,
    pair_cell (dense, cell-major, candidate order), n_cand, overflow.
    cell_base: global id of the first cell (keys the random numbers)."""
    cs = _c(cell_start, np.int32)
    n_cells = len(cs) - 1
    Cc, e = sigma_g_law(xs)
    v = _c(v, np.float64)
    if cap is None:
        cap = 1 << 26
    # candidates bound the accepted pairs; allocate lazily by a first count
    nc, npair = C.c_int64(0), C.c_int64(0)
    off = np.zeros(max(n_cells, 1), np.int32)
    cnt = np.zeros(max(n_cells, 1), np.int32)
    probe = np.zeros(1, np.int32)
    rc = lib().orc_select_ntc(n_cells, cs, _c(v[0], np.float64), _c(v[1], np.float64),
                              _c(v[2], np.float64), Cc, e, _c(lam, np.float64),
                              _c(mom, np.float64).reshape(-1), int(seed), int(step),
                              int(cell_base), off, cnt, probe, probe, probe, -1, C.byref(nc),
                              C.byref(npair))
    total = nc.value
    if total > cap:
        return {"overflow": True, "n_cand": total, "pair_off": np.zeros(n_cells, np.int32),
                "pair_cnt": np.zeros(n_cells, np.int32),
                "pair_i": np.zeros(0, np.int32), "pair_j": np.zeros(0, np.int32),
                "pair_cell": np.zeros(0, np.int32), "cell_base": int(cell_base)}
    pi = np.zeros(max(total, 1), np.int32)
    pj = np.zeros(max(total, 1), np.int32)
    pc = np.zeros(max(total, 1), np.int32)
    rc = lib().orc_select_ntc(n_cells, cs, _c(v[0], np.float64), _c(v[1], np.float64),
                              _c(v[2], np.float64), Cc, e, _c(lam, np.float64),
                              _c(mom, np.float64).reshape(-1), int(seed), int(step),
                              int(cell_base), off, cnt, pi, pj, pc, total, C.byref(nc),
                              C.byref(npair))
    assert rc == 0
    m = npair.value
    return {"overflow": False, "n_cand": total, "pair_off": off[:n_cells],
            "pair_cnt": cnt[:n_cells], "pair_i": pi[:m], "pair_j": pj[:m],
            "pair_cell": pc[:m], "cell_base": int(cell_base)}


def select_sbt(cell_start, v, xs, lam, seed, step, cap=None, cell_base=0):
    """Simplified Bernoulli Trials selection (same dict as select_ntc, with
    n_cand = trials and n_clamped = trials whose probability exceeded 1)."""
    cs = _c(cell_start, np.int32)
    n_cells = len(cs) - 1
    Cc, e = sigma_g_law(xs)
    v = _c(v, np.float64)
    counts = np.diff(cs)
    total = int(np.sum(np.maximum(counts - 1, 0)))
    if cap is None:
        cap = 1 << 26
    m = max(total, 1)
    off = np.zeros(max(n_cells, 1), np.int32)
    cnt = np.zeros(max(n_cells, 1), np.int32)
    pi = np.zeros(m, np.int32)
    pj = np.zeros(m, np.int32)
    pc = np.zeros(m, np.int32)
    nt, npair, ncl = C.c_int64(0), C.c_int64(0), C.c_int32(0)
    rc = lib().orc_select_sbt(n_cells, cs, _c(v[0], np.float64), _c(v[1], np.float64),
                              _c(v[2], np.float64), Cc, e, _c(lam, np.float64), int(seed),
                              int(step), int(cell_base), off, cnt, pi, pj, pc, int(cap),
                              C.byref(nt), C.byref(npair), C.byref(ncl))
    k = npair.value
    return {"overflow": rc != 0, "n_cand": nt.value, "n_clamped": ncl.value,
            "pair_off": off[:n_cells], "pair_cnt": cnt[:n_cells], "pair_i": pi[:k],
            "pair_j": pj[:k], "pair_cell": pc[:k], "cell_base": int(cell_base)}


def pair_latents(sel, seed, step, lowp=False):
    """(U[np,6], xi[np,3], z[np,2]) for the accepted pairs of a selection."""
    m = len(sel["pair_i"])
    U = np.zeros(max(m, 1) * 6)
    xi = np.zeros(max(m, 1) * 3)
    z = np.zeros(max(m, 1) * 2)
    off = _c(sel["pair_off"], np.int32)
    if len(off) == 0:
        off = np.zeros(1, np.int32)
    lib().orc_pair_latents(m, _c(sel["pair_cell"], np.int32) if m else np.zeros(1, np.int32),
                           off, int(seed), int(step), int(sel.get("cell_base", 0)),
                           int(bool(lowp)), U, xi, z)
    return U[: 6 * m].reshape(m, 6), xi[: 3 * m].reshape(m, 3), z[: 2 * m].reshape(m, 2)


def vhs_dirs(sel, v, U, xi):
    """Phase A of the isotropic rule: unit post-collision directions u[np,3]."""
    m = len(sel["pair_i"])
    u = np.zeros(max(m, 1) * 3)
    v = _c(v, np.float64)
    if m:
        lib().orc_vhs_dirs(m, _c(sel["pair_i"], np.int32), _c(sel["pair_j"], np.int32),
                           _c(v[0], np.float64), _c(v[1], np.float64), _c(v[2], np.float64),
                           _c(U, np.float64).reshape(-1), _c(xi, np.float64).reshape(-1), u)
    return u[: 3 * m].reshape(m, 3)


def _pairs_args(sel):
    def nz(a):
        a = _c(a, np.int32)
        return a if a.size else np.zeros(1, np.int32)
    return nz(sel["pair_off"]), nz(sel["pair_cnt"]), nz(sel["pair_i"]), nz(sel["pair_j"])


def apply_dirs(sel, v, u):
    """Phase B with directions: returns the updated copy of v[3, n]."""
    v = np.array(v, dtype=np.float64, order="C", copy=True)
    vx, vy, vz = [np.ascontiguousarray(v[q]) for q in range(3)]
    n_cells = len(sel["pair_cnt"])
    uu = _c(u, np.float64).reshape(-1)
    if uu.size == 0:
        uu = np.zeros(3)
    lib().orc_apply_dirs(n_cells, *_pairs_args(sel), uu, vx, vy, vz)
    return np.stack([vx, vy, vz])


def apply_chi(sel, v, cos_chi, sin_chi, xi):
    """Phase B with deflection angles: returns the updated copy of v[3, n]."""
    v = np.array(v, dtype=np.float64, order="C", copy=True)
    vx, vy, vz = [np.ascontiguousarray(v[q]) for q in range(3)]
    n_cells = len(sel["pair_cnt"])
    m = len(sel["pair_i"])
    cc = _c(cos_chi, np.float64) if m else np.zeros(1)
    sc = _c(sin_chi, np.float64) if m else np.zeros(1)
    xx = _c(xi, np.float64).reshape(-1) if m else np.zeros(3)
    lib().orc_apply_chi(n_cells, *_pairs_args(sel), cc, sc, xx, vx, vy, vz)
    return np.stack([vx, vy, vz])


def moment_match(cell_start, mom_pre, pair_cnt, v, centred=True):
    """Cell-wise moment matching; returns (v_new[3, n], n_skipped)."""
    v = np.array(v, dtype=np.float64, order="C", copy=True)
    vx, vy, vz = [np.ascontiguousarray(v[q]) for q in range(3)]
    n_cells = len(cell_start) - 1
    pc = None if pair_cnt is None else _c(pair_cnt, np.int32)
    skipped = lib().orc_moment_match(
        n_cells, _c(cell_start, np.int32), _c(mom_pre, np.float64).reshape(-1),
        None if pc is None else pc.ctypes.data_as(C.c_void_p), int(bool(centred)),
        vx, vy, vz)
    return np.stack([vx, vy, vz]), int(skipped)


# ---------------------------------------------------------------------------
# Deflection angle (section "Computational Implementation: The Exact vs.
# Neural Paradigm").
# ---------------------------------------------------------------------------
def potential_jager(p):
    P = Potential()
    P.kind = POT_JAGER
    P.A, P.a1, P.a2, P.am1, P.am2, P.beta_tt = p.A, p.a1, p.a2, p.am1, p.am2, p.beta_tt
    for q in range(6):
        P.C[q] = p.C[q]
    P.R_eps, P.A_sr, P.a_sr = p.R_eps, p.A_sr, p.a_sr
    return P


def potential_hs(d_angstrom):
    P = Potential()
    P.kind = POT_HS
    P.d = d_angstrom
    return P


def potential_invpow(K, n):
    P = Potential()
    P.kind = POT_INVPOW
    P.K = K
    P.n = n
    return P


def potential_V(P, r):
    return lib().orc_potential_V(C.byref(P), float(r))


def chi(P, b_angstrom, E_kelvin, with_evals=False):
    """chi(b, E) for b in Angstrom and E/k_B in K."""
    st = C.c_int(0)
    ne = C.c_int64(0)
    x = lib().orc_chi(C.byref(P), float(b_angstrom), float(E_kelvin), C.byref(st),
                      C.byref(ne))
    if with_evals:
        return x, st.value, ne.value
    return x


def chi_batch(P, b_m, g, m_red, n_threads=1):
    """chi for SI inputs (b in m, g in m/s, reduced mass in kg)."""
    b_m = _c(b_m, np.float64)
    g = _c(g, np.float64)
    n = b_m.shape[0]
    out = np.zeros(max(n, 1))
    st = np.zeros(max(n, 1), np.int32)
    lib().orc_chi_batch(C.byref(P), n, b_m if n else np.zeros(1), g if n else np.zeros(1),
                        float(m_red), out, st, int(n_threads))
    return out[:n], st[:n]


def fold(chi_):
    """Folded deflection angle theta = arccos(cos chi) in [0, pi]."""
    return np.arccos(np.clip(np.cos(chi_), -1.0, 1.0))


def impact_from_z(z, b_max):
    """b = b_max * sqrt(1 - exp(-|z|^2 / 2)) (b^2 uniform for normal z)."""
    z = np.asarray(z, np.float64)
    return b_max * np.sqrt(-np.expm1(-0.5 * np.sum(z * z, axis=-1)))


def rotate(vr, chi_, xi):
    """v_r' = g (cos chi vhat + sin chi e_perp(xi, vhat)) for rows."""
    vr = np.asarray(vr, np.float64)
    g = np.linalg.norm(vr, axis=1)
    vh = vr / np.where(g > 0, g, 1.0)[:, None]
    w = xi - np.sum(xi * vh, axis=1, keepdims=True) * vh
    e = w / np.linalg.norm(w, axis=1, keepdims=True)
    return g[:, None] * (np.cos(chi_)[:, None] * vh + np.sin(chi_)[:, None] * e)


# ---------------------------------------------------------------------------
# Chapman-Enskog viscosity from the deflection angle (section "Macroscopic
# Validation: Viscosity and Transport Coefficients").
# ---------------------------------------------------------------------------
def transport_q2(P, E_kelvin, b_cut, n_panels=256, n_gl=8, n_threads=8):
    """Q2(E) = 2 pi int_0^b_cut (1 - cos^2 chi(b, E)) b db in m^2 (eq.
    transport cross-section), composite Gauss-Legendre in b: n_panels equal
    panels of n_gl nodes.  E in K (E_r / k_B), b_cut in m."""
    x, w = np.polynomial.legendre.leggauss(n_gl)
    edges = np.linspace(0.0, b_cut, n_panels + 1)
    mid = 0.5 * (edges[:-1] + edges[1:])
    half = 0.5 * np.diff(edges)
    b = (mid[:, None] + half[:, None] * x[None, :]).ravel()
    wb = (half[:, None] * w[None, :]).ravel()
    m_red = 1.0          # chi depends on E only: any reduced mass with g = sqrt(2 E k / m_red)
    out = []
    for E in np.atleast_1d(E_kelvin):
        g = np.full(b.shape, math.sqrt(2.0 * E * KB / m_red))
        ch, _ = chi_batch(P, b, g, m_red, n_threads=n_threads)
        out.append(2.0 * math.pi * np.sum(wb * (1.0 - np.cos(ch) ** 2) * b))
    return np.array(out)


def collision_integral(P, T, b_cut, n_lag=24, printed=False, **kw):
    """Omega(T) in m^2.  Standard Chapman-Cowling average (reading of the
    printed average): Omega = 1/(4 (kT)^4) int E^3 Q2(E) exp(-E/kT) dE
    = 1/4 int x^3 e^-x Q2(x kT) dx (generalised Gauss-Laguerre, alpha = 3),
    which makes the hard-sphere viscosity come out right.  printed=True:
    the average as printed, 1/(2 (kT)^3) int E^2 Q2 exp(-E/kT) dE (alpha = 2)."""
    from scipy.special import roots_genlaguerre
    alpha, scale = (2, 0.5) if printed else (3, 0.25)
    x, w = roots_genlaguerre(n_lag, alpha)
    out = []
    for t in np.atleast_1d(T):
        q = transport_q2(P, x * t, b_cut, **kw)
        out.append(scale * np.sum(w * q))
    return np.array(out)


def viscosity_ce(omega, T, m):
    """mu = 5/16 sqrt(pi m k T) / Omega (eq. chapman_enskog), Pa s."""
    return 5.0 / 16.0 * np.sqrt(math.pi * m * KB * np.asarray(T, np.float64)) / omega


# ---------------------------------------------------------------------------
# Conditional MLP, projection, loss and gradients (sections "Cell-Based
# Neural Collision Operator" and "Hard Conservation via Projection").
# ---------------------------------------------------------------------------
def act_fn(name, zz):
    if name == "silu":
        # exp(-z) overflows to inf for z < -709 and z / inf = -0 is the limit
        with np.errstate(over="ignore"):
            return zz / (1.0 + np.exp(-zz))
    if name == "relu":
        return np.maximum(zz, 0.0)
    raise ValueError(name)


def act_grad(name, zz):
    if name == "silu":
        s = 1.0 / (1.0 + np.exp(-zz))
        return s * (1.0 + zz * (1.0 - s))
    if name == "relu":
        return (zz > 0.0).astype(np.float64)
    raise ValueError(name)


def mlp_forward(Ws, bs, x, act="silu", keep=False):
    """h_l = act(W_l h_{l-1} + b_l) for hidden layers, linear output layer."""
    h = np.asarray(x, np.float64)
    zs, hs = [], [h]
    L = len(Ws)
    for l in range(L):
        zz = h @ np.asarray(Ws[l], np.float64).T + np.asarray(bs[l], np.float64)
        if l < L - 1:
            zs.append(zz)
            h = act_fn(act, zz)
            hs.append(h)
        else:
            h = zz
    return (h, zs, hs) if keep else h


def network_input(vr, xi, z, sigma_v):
    """x = [v_r / sigma_v, xi, z] (eq. mlp_input plus the impact latents)."""
    return np.concatenate([np.asarray(vr) / sigma_v, xi, z], axis=1)


def project(y, g, eps=1e-30):
    """Energy-shell projection (eq. energy_shell_projection) with a floor on
    the norm: u = y / max(|y|, eps), v_r' = g u."""
    n = np.linalg.norm(y, axis=1)
    u = y / np.maximum(n, eps)[:, None]
    return g[:, None] * u, u, n


def surrogate_loss(vr_new, vr_target, sigma_v):
    """MSE on the post-collision velocities of the pair, written through v_r:
    (1/B) sum 1/2 (|v_i'-v_i*|^2 + |v_j'-v_j*|^2)/sigma_v^2 = (1/B) sum |dv_r|^2/(4 sigma_v^2)."""
    d = vr_new - vr_target
    return float(np.sum(d * d) / (4.0 * sigma_v ** 2 * d.shape[0]))


def surrogate_loss_grad(vr_new, vr_target, sigma_v):
    d = vr_new - vr_target
    return d / (2.0 * sigma_v ** 2 * d.shape[0])


def direction_loss(vr_new, vr_target):
    """MSE on the scattering directions (section "Neural Surrogate Training"
    names the surrogate's loss as one on the scattering directions): with
    u = v_r'/g and g = |v_r'*| = |v_r'|, (1/B) sum |u - u*|^2 / 4, i.e. the
    velocity MSE with each pair normalised by its own g^2 instead of sigma_v^2."""
    d = vr_new - vr_target
    g2 = np.sum(vr_target * vr_target, axis=1)
    return float(np.sum(np.sum(d * d, axis=1) / (4.0 * g2)) / d.shape[0])


def direction_loss_grad(vr_new, vr_target):
    d = vr_new - vr_target
    g2 = np.sum(vr_target * vr_target, axis=1)
    return d / (2.0 * g2[:, None] * d.shape[0])


def project_backward(G, y, g):
    """dL/dy from dL/dv_r' for v_r' = g y/|y|: (g/|y|)(G - (G.u) u)."""
    n = np.linalg.norm(y, axis=1)
    u = y / n[:, None]
    Gu = np.sum(G * u, axis=1, keepdims=True)
    return (g / n)[:, None] * (G - Gu * u)


def mlp_backward(Ws, bs, x, dy, act="silu"):
    """Gradients (dW list, db list, dx) of sum(dy * mlp(x)) in FP64."""
    _, zs, hs = mlp_forward(Ws, bs, x, act, keep=True)
    L = len(Ws)
    dW = [None] * L
    db = [None] * L
    delta = np.asarray(dy, np.float64)
    for l in range(L - 1, -1, -1):
        dW[l] = delta.T @ hs[l]
        db[l] = delta.sum(axis=0)
        dh = delta @ np.asarray(Ws[l], np.float64)
        if l > 0:
            delta = dh * act_grad(act, zs[l - 1])
        else:
            dx = dh
    return dW, db, dx


def moment_match_group(v, v_pre):
    """Centred moment matching of one group of velocities v[N,3] to the
    moments of v_pre[N,3] (differentiable form used by the adjoint)."""
    up = v_pre.mean(axis=0)
    Sp = np.sum((v_pre - up) ** 2)
    uq = v.mean(axis=0)
    c = v - uq
    Sq = np.sum(c * c)
    a = math.sqrt(Sp / Sq)
    return up + a * c


def moment_match_group_backward(G, v, v_pre):
    """Adjoint of moment_match_group w.r.t. v (v_pre held fixed):
    dL/dv_m = a (G_m - mean G) - (a / S_post) (sum_i G_i . c_i) c_m."""
    up = v_pre.mean(axis=0)
    Sp = np.sum((v_pre - up) ** 2)
    c = v - v.mean(axis=0)
    Sq = np.sum(c * c)
    a = math.sqrt(Sp / Sq)
    Gc = float(np.sum(G * c))
    return a * (G - G.mean(axis=0)) - (a / Sq) * Gc * c


def adam_step(params, grads, m, s, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015), bias-corrected, in FP64; updates in place."""
    for q in range(len(params)):
        m[q] = beta1 * m[q] + (1 - beta1) * grads[q]
        s[q] = beta2 * s[q] + (1 - beta2) * grads[q] ** 2
        mh = m[q] / (1 - beta1 ** t)
        sh = s[q] / (1 - beta2 ** t)
        params[q] = params[q] - lr * mh / (np.sqrt(sh) + eps)
    return params, m, s


def cosine_lr(t, T, lr_max, lr_min=1e-6):
    """Cosine annealing from lr_max to lr_min over T steps."""
    return lr_min + 0.5 * (lr_max - lr_min) * (1.0 + math.cos(math.pi * min(t, T) / T))


# ---------------------------------------------------------------------------
# Angle network and deflection-angle table (sections "Neural Network
# Architecture", "Neural Surrogate Training" and "Runtime Acceleration via
# Neural Table Look-up").  The network maps (normalised ln E_r, b / b_max) to
# a prediction of ln(1 + theta), theta the folded deflection angle; hidden
# layers SiLU, output Softplus.
# ---------------------------------------------------------------------------
def softplus(zz):
    """ln(1 + e^z), evaluated without overflow."""
    return np.logaddexp(0.0, np.asarray(zz, np.float64))


def sigmoid(zz):
    """1 / (1 + e^-z), with e^z / (1 + e^z) for z < 0 (no overflow)."""
    zz = np.asarray(zz, np.float64)
    ez = np.exp(-np.abs(zz))
    return np.where(zz >= 0, 1.0 / (1.0 + ez), ez / (1.0 + ez))


def angle_net_input(E_kelvin, b_rel, lne_lo, lne_hi):
    """x = [2 (ln E - lnE_lo) / (lnE_hi - lnE_lo) - 1, b / b_max]."""
    lnE = np.log(np.asarray(E_kelvin, np.float64))
    x0 = 2.0 * (lnE - lne_lo) / (lne_hi - lne_lo) - 1.0
    return np.stack([x0, np.asarray(b_rel, np.float64)], axis=1)


def angle_net_forward(Ws, bs, x, keep=False):
    """SiLU hidden layers, Softplus output; returns y[B] (= predicted
    ln(1 + theta))."""
    h = np.asarray(x, np.float64)
    zs, hs = [], [h]
    L = len(Ws)
    for l in range(L):
        zz = h @ np.asarray(Ws[l], np.float64).T + np.asarray(bs[l], np.float64)
        zs.append(zz)
        if l < L - 1:
            h = act_fn("silu", zz)
            hs.append(h)
        else:
            h = softplus(zz)
    y = h[:, 0]
    return (y, zs, hs) if keep else y


def angle_net_backward(Ws, bs, x, dy):
    """Gradients (dW list, db list, dx) of sum(dy * angle_net(x)) in FP64."""
    _, zs, hs = angle_net_forward(Ws, bs, x, keep=True)
    L = len(Ws)
    dW = [None] * L
    db = [None] * L
    delta = np.asarray(dy, np.float64)[:, None] * sigmoid(zs[L - 1])
    dx = None
    for l in range(L - 1, -1, -1):
        dW[l] = delta.T @ hs[l]
        db[l] = delta.sum(axis=0)
        dh = delta @ np.asarray(Ws[l], np.float64)
        if l > 0:
            delta = dh * act_grad("silu", zs[l - 1])
        else:
            dx = dh
    return dW, db, dx


def huber_loss(yhat, y):
    """Mean smooth-L1 (Huber, threshold 1) loss of eq. huber_loss."""
    d = np.asarray(yhat, np.float64) - np.asarray(y, np.float64)
    a = np.abs(d)
    return float(np.mean(np.where(a < 1.0, 0.5 * d * d, a - 0.5)))


def huber_grad(yhat, y):
    """d huber_loss / d yhat."""
    d = np.asarray(yhat, np.float64) - np.asarray(y, np.float64)
    return np.clip(d, -1.0, 1.0) / d.shape[0]


def angle_rows(b, g, chi_, m_red, lne_lo, lne_hi, b_max):
    """Training rows from quadrature results: x (angle_net_input) and the
    target ln(1 + theta), theta = fold(chi)."""
    E = 0.5 * m_red * np.asarray(g, np.float64) ** 2 / KB
    x = angle_net_input(E, np.asarray(b, np.float64) / b_max, lne_lo, lne_hi)
    return x, np.log1p(fold(chi_))


def table_grid(n_e, n_b, lne_lo, lne_hi):
    """Grid node coordinates: ln E_i = lnE_lo + i (lnE_hi - lnE_lo)/(n_e - 1),
    b_j / b_max = j / (n_b - 1)."""
    lnE = lne_lo + (lne_hi - lne_lo) * np.arange(n_e) / (n_e - 1)
    brel = np.arange(n_b) / (n_b - 1)
    return lnE, brel


def chi_table(Ws, bs, n_e, n_b, lne_lo, lne_hi):
    """theta[n_e, n_b] = clip(exp(y) - 1, 0, pi) of the angle network at the
    grid nodes."""
    lnE, brel = table_grid(n_e, n_b, lne_lo, lne_hi)
    E = np.repeat(np.exp(lnE), n_b)
    B = np.tile(brel, n_e)
    y = angle_net_forward(Ws, bs, angle_net_input(E, B, lne_lo, lne_hi))
    return np.clip(np.expm1(y), 0.0, math.pi).reshape(n_e, n_b)


def table_lookup(theta, lne_lo, lne_hi, E_kelvin, b_rel):
    """Bilinear interpolation of the table in (ln E, b / b_max), with both
    coordinates clamped to the grid."""
    theta = np.asarray(theta, np.float64)
    n_e, n_b = theta.shape
    fe = (np.log(np.asarray(E_kelvin, np.float64)) - lne_lo) / (lne_hi - lne_lo) * (n_e - 1)
    fb = np.asarray(b_rel, np.float64) * (n_b - 1)
    fe = np.clip(fe, 0.0, n_e - 1)
    fb = np.clip(fb, 0.0, n_b - 1)
    i0 = np.minimum(np.floor(fe).astype(np.int64), n_e - 2)
    j0 = np.minimum(np.floor(fb).astype(np.int64), n_b - 2)
    te = fe - i0
    tb = fb - j0
    t00 = theta[i0, j0]
    t01 = theta[i0, j0 + 1]
    t10 = theta[i0 + 1, j0]
    t11 = theta[i0 + 1, j0 + 1]
    return (1 - te) * ((1 - tb) * t00 + tb * t01) + te * ((1 - tb) * t10 + tb * t11)


def table_angles(sel, v, U, table, b_max, m_red):
    """Phase A of the table rule: theta per accepted pair from the pre-step
    relative speed (E = m_r g^2 / 2) and b = b_max sqrt(U4)."""
    vr = v[:, sel["pair_i"]] - v[:, sel["pair_j"]]
    g = np.sqrt(np.sum(vr * vr, axis=0))
    E = 0.5 * m_red * g * g / KB
    b_rel = np.sqrt(U[:, 4])
    return table_lookup(table["theta"], table["lne_lo"], table["lne_hi"], E, b_rel)


# ---------------------------------------------------------------------------
# Whole-step compositions (sorted arrays in, sorted arrays out)
# ---------------------------------------------------------------------------
def step(cell_start, v, xs, lam, seed, step_no, rule="vhs", lowp=False,
         match=None, net=None, pot=None, b_max=1e-9, m_red=None, cap=None, cell_base=0,
         table=None, selection="ntc"):
    """One collision step on sorted velocities: select (pre-step velocities),
    Phase A per pair, Phase B in candidate order per cell, then moment matching.

    rule: "vhs" | "jager" | "neural" | "table".  net: dict(Ws, bs, act,
    sigma_v) for the neural rule; table: dict(theta, lne_lo, lne_hi) for the
    table rule.  match: None -> on for "neural", off otherwise.
    selection: "ntc" | "sbt" (Simplified Bernoulli Trials).
    cell_base: global id of cell 0 of these arrays (a contiguous range of a
    larger population can be stepped on its own: the random numbers are keyed
    by the global cell id).
    Returns (v_new, info dict).
    """
    v = np.asarray(v, np.float64)
    mom = moments(cell_start, v)
    if selection == "sbt":
        sel = select_sbt(cell_start, v, xs, lam, seed, step_no, cap=cap, cell_base=cell_base)
    else:
        sel = select_ntc(cell_start, v, xs, lam, mom, seed, step_no, cap=cap, cell_base=cell_base)
    if sel["overflow"]:
        return v.copy(), {"sel": sel, "mom": mom}
    U, xi, z = pair_latents(sel, seed, step_no, lowp=lowp)
    info = {"sel": sel, "mom": mom, "U": U, "xi": xi, "z": z}
    if match is None:
        match = rule == "neural"
    if rule == "vhs":
        u = vhs_dirs(sel, v, U, xi)
        vn = apply_dirs(sel, v, u)
        info["u"] = u
    elif rule == "jager":
        vr = v[:, sel["pair_i"]] - v[:, sel["pair_j"]]
        g = np.sqrt(np.sum(vr * vr, axis=0))
        b = b_max * np.sqrt(U[:, 4])
        ch, st = chi_batch(pot, b, g, m_red)
        info["chi"] = ch
        info["chi_status"] = st
        vn = apply_chi(sel, v, np.cos(ch), np.sin(ch), xi)
    elif rule == "neural":
        vr = (v[:, sel["pair_i"]] - v[:, sel["pair_j"]]).T
        g = np.linalg.norm(vr, axis=1)
        x = network_input(vr, xi, z, net["sigma_v"])
        y = mlp_forward(net["Ws"], net["bs"], x, net.get("act", "silu"))
        n = np.linalg.norm(y, axis=1)
        u = y / np.maximum(n, 1e-30)[:, None]
        small = n <= 1e-30
        if np.any(small):
            uv = vhs_dirs(sel, v, U, xi)
            u[small] = uv[small]
        info["u"] = u
        info["y"] = y
        vn = apply_dirs(sel, v, u)
    elif rule == "table":
        th = table_angles(sel, v, U, table, b_max, m_red)
        info["theta"] = th
        vn = apply_chi(sel, v, np.cos(th), np.sin(th), xi)
    else:
        raise ValueError(rule)
    if match:
        vn, sk = moment_match(cell_start, mom, sel["pair_cnt"], vn, centred=True)
        info["skipped"] = sk
    return vn, info


def step_vhs_fast(cell_start, v, xs, lam, seed, step_no, lowp=False, match=False,
                  n_threads=1):
    """Same as step(rule="vhs") but the whole step runs in C (for timing)."""
    Cc, e = sigma_g_law(xs)
    vx, vy, vz = [np.array(v[q], np.float64) for q in range(3)]
    npairs = lib().orc_step_vhs(len(cell_start) - 1, _c(cell_start, np.int32), vx, vy, vz,
                                Cc, e, _c(lam, np.float64), int(seed), int(step_no),
                                int(bool(lowp)), int(bool(match)), int(n_threads))
    return np.stack([vx, vy, vz]), int(npairs)


# ---------------------------------------------------------------------------
# Flow loop around the collision step (section "Results and Discussion": the
# Couette channel and the lid-driven cavity).  Move: free flight, wall events,
# cell index (dsmc_oracle.c, orc_move); sampling of the macroscopic fields.
# ---------------------------------------------------------------------------
def domain(nx, ny, Lx, Ly, kinds, T_w, u_w, m):
    """kinds / T_w / u_w per side (x = 0, x = Lx, y = 0, y = Ly)."""
    d = Domain()
    d.nx, d.ny, d.Lx, d.Ly, d.m = int(nx), int(ny), float(Lx), float(Ly), float(m)
    for q in range(4):
        d.kind[q] = int(kinds[q])
        d.T_w[q] = float(T_w[q])
        for c in range(3):
            d.u_w[q][c] = float(u_w[q][c])
    return d


def move(dom, pos, v, dt, seed, step_no):
    """Free flight over dt with wall events (FP64).  pos[2, n], v[3, n] are
    copied; returns (pos', v', cell_of, n_at_event_limit, n_wall_events)."""
    pos = np.array(pos, np.float64)
    v = np.array(v, np.float64)
    px, py = [np.ascontiguousarray(pos[q]) for q in range(2)]
    vx, vy, vz = [np.ascontiguousarray(v[q]) for q in range(3)]
    n = px.size
    cell = np.zeros(max(n, 1), np.int32)
    hits = C.c_int64(0)
    stuck = lib().orc_move(n, C.byref(dom), float(dt), int(seed), int(step_no),
                           px if n else np.zeros(1), py if n else np.zeros(1),
                           vx if n else np.zeros(1), vy if n else np.zeros(1),
                           vz if n else np.zeros(1), cell, C.byref(hits))
    return np.stack([px, py]), np.stack([vx, vy, vz]), cell[:n], int(stuck), int(hits.value)


def sample(cell_start, v, acc=None):
    """Accumulate the 13 raw moment sums per cell (orc_sample): count, v_i,
    v_i v_j (xx, yy, zz, xy, xz, yz), |v|^2 v_i."""
    n_cells = len(cell_start) - 1
    if acc is None:
        acc = np.zeros((n_cells, 13))
    a = np.ascontiguousarray(acc, np.float64).reshape(-1)
    v = np.asarray(v, np.float64)
    lib().orc_sample(n_cells, _c(cell_start, np.int32), _c(v[0], np.float64),
                     _c(v[1], np.float64), _c(v[2], np.float64), a)
    return a.reshape(n_cells, 13)


def fields(acc, n_samples, m, fnum_per_volume):
    """Macroscopic fields from the raw sums: number density, mean velocity,
    temperature T = m <|c|^2> / (3 k), shear stress tau_xy = -rho <c_x c_y>,
    heat flux q_i = rho <|c|^2 c_i> / 2 (c = v - u, rho = n m); per cell,
    columns (n, ux, uy, uz, T, tau_xy, qx, qy, qz).  fnum_per_volume =
    F_N / V_cell.  Cells never sampled give zeros."""
    acc = np.asarray(acc, np.float64)
    N = acc[:, 0]
    out = np.zeros((acc.shape[0], 9))
    ok = N > 0
    Nn = np.where(ok, N, 1.0)
    u = acc[:, 1:4] / Nn[:, None]
    vv = {"xx": acc[:, 4], "yy": acc[:, 5], "zz": acc[:, 6], "xy": acc[:, 7], "xz": acc[:, 8],
          "yz": acc[:, 9]}
    m2 = {k: x / Nn for k, x in vv.items()}
    e2 = m2["xx"] + m2["yy"] + m2["zz"]
    cc = e2 - np.sum(u * u, axis=1)
    dens = N / n_samples * fnum_per_volume
    rho = dens * m
    # <|c|^2 c_i> = <|v|^2 v_i> - u_i <|v|^2> - 2 u_j <v_j v_i> + 2 |u|^2 u_i
    vij = np.stack([np.stack([m2["xx"], m2["xy"], m2["xz"]], 1),
                    np.stack([m2["xy"], m2["yy"], m2["yz"]], 1),
                    np.stack([m2["xz"], m2["yz"], m2["zz"]], 1)], 1)
    e3 = acc[:, 10:13] / Nn[:, None]
    uu = np.sum(u * u, axis=1)
    c3 = e3 - u * e2[:, None] - 2.0 * np.einsum("kj,kji->ki", u, vij) + 2.0 * uu[:, None] * u
    out[:, 0] = dens
    out[:, 1:4] = u
    out[:, 4] = m * cc / (3.0 * KB)
    out[:, 5] = -rho * (m2["xy"] - u[:, 0] * u[:, 1])
    out[:, 6:9] = 0.5 * rho[:, None] * c3
    out[~ok] = 0.0
    return out


def flow_step(dom, pos, v, xs, lam, dt, seed, step_no, rule="vhs", **kw):
    """One DSMC step of the flow cases: move (wall events), bin by cell with
    positions and velocities gathered into cell order, then the collision
    step of `step` on the sorted velocities.  Returns (pos, v, cell_start,
    info)."""
    pos2, v2, cell_of, stuck, hits = move(dom, pos, v, dt, seed, step_no)
    cs, perm, bad = sort_cells(cell_of, dom.nx * dom.ny)
    pos3 = pos2[:, perm]
    v3 = v2[:, perm]
    vn, info = step(cs, v3, xs, lam, seed, step_no, rule=rule, **kw)
    info.update({"stuck": stuck, "hits": hits, "perm": perm})
    return pos3, vn, cs, info
