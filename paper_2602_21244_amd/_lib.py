"""ctypes declarations of the C-ABI in include/dsmc.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsmc.so")

DSMC_OK, DSMC_E_ARG, DSMC_E_HIP, DSMC_E_UNSUPPORTED = 0, -1, -2, -3
F32, F64, BF16 = 0, 1, 2
ST_PAIR_OVERFLOW, ST_BAD_CELL, ST_ROOT_FAIL, ST_NONFINITE, ST_PROB_CLAMP = 1, 2, 4, 8, 16
ST_WALL_LIMIT = 32
WALL_PERIODIC, WALL_SPECULAR, WALL_DIFFUSE = 0, 1, 2
XS_VHS, XS_CONST = 0, 1
POT_JAGER, POT_HS, POT_INVPOW = 0, 1, 2
ACT_SILU, ACT_RELU = 0, 1
SPLIT_ALL, SPLIT_FRONT, SPLIT_FIRST = 0, 1, 2
SCHED_AUTO, SCHED_LANE, SCHED_BLOCK, SCHED_DEFER, SCHED_WAVE = 0, 1, 2, 3, 4
APPLY_DIRECTIONS, APPLY_ANGLES = 0, 1
MM_CAPTURE, MM_APPLY, MM_APPLY_LITERAL = 0, 1, 2
CE_STANDARD, CE_AS_PRINTED = 0, 1


class Vec3(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p)]


class Rng(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("step", C.c_uint32), ("reserved", C.c_uint32)]


class Status(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("bad_cell", C.c_int32), ("n_cand", C.c_int64),
                ("n_pairs", C.c_int64), ("root_fail", C.c_int32), ("nonfinite", C.c_int32),
                ("mm_skipped", C.c_int32), ("prob_clamped", C.c_int32),
                ("wall_events", C.c_int64), ("wall_limit", C.c_int32), ("reserved", C.c_int32)]


class Domain(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("Lx", C.c_double), ("Ly", C.c_double),
                ("kind", C.c_int32 * 4), ("T_w", C.c_double * 4),
                ("u_w", (C.c_double * 3) * 4), ("m", C.c_double)]


class Pairs(C.Structure):
    _fields_ = [("off", C.c_void_p), ("cnt", C.c_void_p), ("i", C.c_void_p),
                ("j", C.c_void_p), ("cell", C.c_void_p), ("cap", C.c_int64)]


class Xs(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("m", C.c_double),
                ("d_ref", C.c_double), ("omega", C.c_double), ("T_ref", C.c_double),
                ("sigma", C.c_double)]


class Potential(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("A", C.c_double), ("a1", C.c_double),
                ("a2", C.c_double), ("am1", C.c_double), ("am2", C.c_double),
                ("beta_tt", C.c_double), ("C", C.c_double * 6), ("R_eps", C.c_double),
                ("A_sr", C.c_double), ("a_sr", C.c_double), ("d", C.c_double),
                ("K", C.c_double)]


class MatchSchedule(C.Structure):
    _fields_ = [("wave_per_cu", C.c_int32), ("medium_per_cu", C.c_int32),
                ("big_per_cu", C.c_int32), ("reserved", C.c_int32)]


class Quad(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("max_iter", C.c_int32), ("scan_ratio", C.c_double),
                ("refine", C.c_int32), ("reserved", C.c_int32)]


class Mlp(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("dims", C.c_int32 * 7), ("act", C.c_int32),
                ("wdtype", C.c_int32), ("W", C.c_void_p * 6), ("b", C.c_void_p * 6),
                ("sigma_v", C.c_double), ("split", C.c_int32), ("reserved", C.c_int32)]


ANET_MAX_LAYERS = 8


class Anet(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("dims", C.c_int32 * (ANET_MAX_LAYERS + 1)),
                ("W", C.c_void_p * ANET_MAX_LAYERS), ("b", C.c_void_p * ANET_MAX_LAYERS)]


class ChiTable(C.Structure):
    _fields_ = [("n_e", C.c_int32), ("n_b", C.c_int32), ("lne_lo", C.c_double),
                ("lne_hi", C.c_double), ("theta", C.c_void_p)]


_vp, _i32, _i64, _u64, _sz, _d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_size_t, C.c_double

# name: (restype, argtypes)
SIGNATURES = {
    "dsmc_init": (C.c_int, [C.c_int]),
    "dsmc_last_error": (C.c_char_p, []),
    "dsmc_version": (C.c_char_p, []),
    "dsmc_status_clear": (C.c_int, [_vp, _vp]),
    "dsmc_sort_cells_ws": (_sz, [_i32, _i32]),
    "dsmc_sort_cells": (C.c_int, [_i32, _i32, _vp, _i32, Vec3, Vec3, _vp, _vp, _vp, _sz, _vp, _vp]),
    "dsmc_sort_cells_noalloc": (C.c_int, [_i32, _i32, _vp, _i32, Vec3, Vec3, _vp, _vp, _vp, _vp]),
    "dsmc_moment_match": (C.c_int, [_i32, _vp, _i32, Vec3, _vp, _i32, _vp, _vp, _vp]),
    "dsmc_select_pairs_ntc_ws": (_sz, [_i32, _i64]),
    "dsmc_select_pairs_ntc": (C.c_int, [_i32, _vp, _i32, Vec3, Xs, _vp, _vp, Rng, Pairs, _vp,
                                        _sz, _vp, _vp]),
    "dsmc_select_pairs_sbt_ws": (_sz, [_i32, _i64]),
    "dsmc_select_pairs_sbt": (C.c_int, [_i32, _vp, _i32, Vec3, Xs, _vp, Rng, Pairs, _vp, _sz, _vp,
                                        _vp]),
    "dsmc_collide_ws": (_sz, [_i64, _i32]),
    "dsmc_collide_vhs": (C.c_int, [_i32, _i32, Vec3, Pairs, Rng, _i32, _vp, _sz, _vp]),
    "dsmc_apply_pairs": (C.c_int, [_i32, _i32, Vec3, Pairs, _i32, _i32, _vp, _sz, _vp]),
    "dsmc_move": (C.c_int, [_i32, _i32, Vec3, Vec3, _vp, C.c_double, Rng, _vp, _vp, _vp]),
    "dsmc_gather": (C.c_int, [_i32, _i32, _vp, Vec3, Vec3, _vp]),
    "dsmc_sample": (C.c_int, [_i32, _vp, _i32, Vec3, _vp, _vp]),
    "dsmc_sample_fields": (C.c_int, [_i32, _vp, C.c_double, C.c_double, C.c_double, _vp, _vp]),
    "dsmc_apply_pairs_match": (C.c_int, [_i32, _vp, _i32, Vec3, Pairs, _i32, _vp, _i32, _vp, _sz,
                                         _vp, _vp]),
    "dsmc_deflect_jager": (C.c_int, [_i64, _i32, _vp, _vp, _vp, _d, C.POINTER(Potential), Quad,
                                     _i32, _vp, _vp]),
    "dsmc_collide_jager": (C.c_int, [_i32, _i32, Vec3, Pairs, Rng, _d, _d, C.POINTER(Potential),
                                     Quad, _i32, _vp, _sz, _vp, _vp]),
    "dsmc_neural_collide": (C.c_int, [C.POINTER(Mlp), _i32, _i32, Vec3, Pairs, Rng, _i32, _vp,
                                      _sz, _vp, _vp]),
    "dsmc_neural_act_bytes": (_sz, [C.POINTER(Mlp), _i64]),
    "dsmc_neural_forward_rows": (C.c_int, [C.POINTER(Mlp), _i64, _vp, _vp, _vp, _vp, _vp, _sz,
                                           _vp]),
    "dsmc_neural_backward_ws": (_sz, [C.POINTER(Mlp), _i64]),
    "dsmc_neural_backward": (C.c_int, [C.POINTER(Mlp), _i64, _vp, _vp, _vp, _vp, _vp,
                                       C.POINTER(_vp), C.POINTER(_vp), _vp, _i32, _vp, _sz, _vp]),
    "dsmc_moment_match_backward": (C.c_int, [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                             _vp, _vp, _vp]),
    "dsmc_mse_loss": (C.c_int, [_i64, _vp, _vp, _d, _vp, _vp, _vp]),
    "dsmc_direction_loss": (C.c_int, [_i64, _vp, _vp, _vp, _vp, _vp]),
    "dsmc_cosine_lr": (_d, [_i64, _i64, _d, _d]),
    "dsmc_adam_step": (C.c_int, [_i64, _vp, _vp, _vp, _vp, _vp, _i64, _d, _d, _d, _d, _vp]),
    "dsmc_harvest_rows": (C.c_int, [_i64, _vp, _vp, _vp, _d, _d, _d, C.POINTER(Potential), Quad,
                                    _vp, _vp, _vp, _vp, _vp, _vp]),
    "dsmc_step_vhs_ws": (_sz, [_i32, _i64]),
    "dsmc_step_vhs_fused": (C.c_int, [_i32, _vp, _i32, Vec3, Xs, _vp, Rng, _i32, _vp, _vp, _sz,
                                      _vp, _vp]),
    "dsmc_anet_ws": (_sz, [C.POINTER(Anet), _i64]),
    "dsmc_anet_forward": (C.c_int, [C.POINTER(Anet), _i64, _vp, _vp, _vp, _sz, _vp]),
    "dsmc_anet_backward": (C.c_int, [C.POINTER(Anet), _i64, _vp, C.POINTER(_vp), C.POINTER(_vp),
                                     _vp, _sz, _vp]),
    "dsmc_huber_loss": (C.c_int, [_i64, _vp, _vp, _vp, _vp, _vp]),
    "dsmc_anet_rows": (C.c_int, [_i64, _vp, _vp, _vp, _d, _d, _d, _d, _vp, _vp, _vp]),
    "dsmc_chi_table_ws": (_sz, [C.POINTER(Anet), C.POINTER(ChiTable)]),
    "dsmc_chi_table_build": (C.c_int, [C.POINTER(Anet), C.POINTER(ChiTable), _vp, _sz, _vp]),
    "dsmc_collide_table": (C.c_int, [C.POINTER(ChiTable), _i32, _i32, Vec3, Pairs, Rng, _d, _i32,
                                     _vp, _sz, _vp]),
    "dsmc_transport_q2_ws": (_sz, [_i64, _i32, _i32]),
    "dsmc_transport_q2": (C.c_int, [_i64, _vp, _d, _i32, _i32, C.POINTER(Potential), Quad, _vp,
                                    _vp, _sz, _vp, _vp]),
    "dsmc_viscosity_ce_ws": (_sz, [_i32, _i32, _i32, _i32]),
    "dsmc_viscosity_ce": (C.c_int, [_i32, _vp, _d, _d, _i32, _i32, _i32, _i32,
                                    C.POINTER(Potential), Quad, _vp, _vp, _vp, _sz, _vp, _vp]),
    "dsmc_set_block_threshold": (C.c_int, [_i32]),
    "dsmc_get_block_threshold": (_i32, []),
    "dsmc_set_match_schedule": (C.c_int, [_vp]),
    "dsmc_get_match_schedule": (C.c_int, [_vp]),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def load(path: str = LIB_PATH):
    """Load libdsmc.so; raises LibraryMissing if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LibraryMissing(
            f"{path} not found: build the HIP library first "
            "(python -m paper_2602_21244_amd.build or __graft_entry__.build())")
    L = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        if not hasattr(L, name):
            continue
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class DsmcError(RuntimeError):
    pass


def check(rc: int, what: str):
    if rc != DSMC_OK:
        msg = load().dsmc_last_error()
        raise DsmcError(f"{what} failed with code {rc}: {msg.decode() if msg else ''}")
