"""CPU oracle for hierarchical process mapping -- TEST INFRASTRUCTURE ONLY.

A ctypes binding over ``pmo.c`` (plain single-threaded C written from the
paper).  Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg may import this package; the GPU library never does, and the
two share no code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pmo.c")
_LIB = os.path.join(_HERE, "libpmo.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile pmo.c into libpmo.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_POSIX_C_SOURCE=199309L",
                               "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class RefineStats(ctypes.Structure):
    _fields_ = [("j_initial", ctypes.c_int64), ("j_final", ctypes.c_int64),
                ("maxw_initial", ctypes.c_int64), ("maxw_final", ctypes.c_int64),
                ("iterations", ctypes.c_int32), ("lp_iterations", ctypes.c_int32),
                ("weak_iterations", ctypes.c_int32), ("strong_iterations", ctypes.c_int32),
                ("feasible", ctypes.c_int32), ("pad_", ctypes.c_int32)]


MAX_LEVELS = 64


class MapStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("feasible", ctypes.c_int32),
                ("j_final", ctypes.c_int64), ("lmax", ctypes.c_int64),
                ("level_n", ctypes.c_int32 * MAX_LEVELS),
                ("level_nnz", ctypes.c_int64 * MAX_LEVELS),
                ("level_iterations", ctypes.c_int32 * MAX_LEVELS),
                ("level_hem_rounds", ctypes.c_int32 * MAX_LEVELS),
                ("refine_seconds", ctypes.c_double),
                ("total_seconds", ctypes.c_double)]


_P = ctypes.c_void_p
_I32, _I64, _U64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64

_SIGS = {
    "pmo_num_pes": (_I64, [_I32, _P]),
    "pmo_distance": (_I32, [_I32, _P, _P, _I32, _I32]),
    "pmo_comm_cost": (_I64, [_I32, _P, _P, _P, _P, _I32, _P, _P]),
    "pmo_block_weights": (None, [_I32, _P, _P, _I64, _P]),
    "pmo_lmax": (_I64, [_I64, _I64, _I64]),
    "pmo_gain": (_I64, [_P, _P, _P, _P, _I32, _P, _P, _I32, _I32]),
    "pmo_hash": (_U64, [_U64, _U64]),
    "pmo_lp_round": (None, [_I32, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "pmo_rebalance": (None, [_I32, _P, _P, _P, _P, _I64, _I32, _I64, _I64, _U64,
                             _I32, _I32, _P, _P]),
    "pmo_sigma": (_I64, [_I64, _I64, _I64]),
    "pmo_refine": (_I32, [_I32, _P, _P, _P, _P, _I32, _P, _P, _I64, _U64, _I32, _P, _P]),
    "pmo_hem": (_I32, [_I32, _P, _P, _P, _P, _I64, _U64, _I32, _P]),
    "pmo_coarse_map": (_I32, [_I32, _P, _P]),
    "pmo_contract": (_I64, [_I32, _P, _P, _P, _P, _P, _I32, _P, _P, _P, _P]),
    "pmo_initial_partition": (None, [_I32, _P, _P, _P, _I32, _P, _P]),
    "pmo_map": (_I32, [_I32, _P, _P, _P, _P, _I32, _P, _P, _I64, _U64, _P, _P]),
    "pmo_subgraphs": (_I64, [_I32, _P, _P, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "pmo_adaptive_eps_ppm": (_I64, [_I64, _I64, _I64, _I64, _I64, _I32]),
    "pmo_hm": (_I32, [_I32, _P, _P, _P, _P, _I32, _P, _I64, _U64, _P]),
    "pmo_hm_v": (_I32, [_I32, _P, _P, _P, _P, _I32, _P, _I64, _U64, _P, _P]),
    "pmo_lp_round_v": (None, [_I32, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P, _P]),
    "pmo_rebalance_v": (None, [_I32, _P, _P, _P, _P, _I32, _P, _P, _I64, _I32, _I64, _I64,
                               _U64, _I32, _I32, _P, _P, _P]),
    "pmo_refine_v": (_I32, [_I32, _P, _P, _P, _P, _I32, _P, _P, _I64, _U64, _I32, _P, _P,
                            _P]),
    "pmo_refine_trace": (_I32, [_I32, _P, _P, _P, _P, _I32, _P, _P, _I64, _U64, _I32, _P,
                                _P, _P, _I32, _P, _P, _P, _P]),
    "pmo_map_v": (_I32, [_I32, _P, _P, _P, _P, _I32, _P, _P, _I64, _U64, _P, _P, _P]),
}


class Variants(ctypes.Structure):
    """Refinement variants (pmo_variants): jet_c = (num, den) enables Jet's
    relaxed first filter with c = num/den; j_rebalance rebalances by J."""
    _fields_ = [("jet_c_num", ctypes.c_int32), ("jet_c_den", ctypes.c_int32),
                ("j_rebalance", ctypes.c_int32), ("refine_repeats", ctypes.c_int32)]


def variants(jet_c=None, j_rebalance=False, repeats=0):
    """repeats: the "ultra" repetition (Algorithm 6 runs this many times per
    level of a multilevel map; 0 or 1: once)."""
    v = Variants()
    if jet_c:
        v.jet_c_num, v.jet_c_den = int(jet_c[0]), int(jet_c[1])
    else:
        v.jet_c_num, v.jet_c_den = 0, 1
    v.j_rebalance = 1 if j_rebalance else 0
    v.refine_repeats = int(repeats)
    return v


def _var(v):
    return ctypes.byref(v) if v is not None else None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(arr: np.ndarray):
    assert arr.flags["C_CONTIGUOUS"]
    return arr.ctypes.data_as(ctypes.c_void_p)


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32))


def _i64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


def _hier(a, d):
    a = _i32(a)
    d = _i32(d)
    assert a.shape == d.shape and 1 <= a.shape[0] <= 8
    return int(a.shape[0]), a, d


def eps_to_ppm(eps: float) -> int:
    return int(round(eps * 1e6))


def num_pes(a) -> int:
    a = _i32(a)
    return int(lib().pmo_num_pes(a.shape[0], _ptr(a)))


def distance(a, d, x: int, y: int) -> int:
    lv, a, d = _hier(a, d)
    return int(lib().pmo_distance(lv, _ptr(a), _ptr(d), x, y))


def comm_cost(g, part, a, d) -> int:
    lv, a, d = _hier(a, d)
    part = _i32(part)
    return int(lib().pmo_comm_cost(g.n, _ptr(g.xadj), _ptr(g.adjncy), _ptr(g.adjwgt),
                                   _ptr(part), lv, _ptr(a), _ptr(d)))


def block_weights(g, part, k: int) -> np.ndarray:
    part = _i32(part)
    w = np.zeros(k, dtype=np.int64)
    lib().pmo_block_weights(g.n, _ptr(g.vwgt), _ptr(part), k, _ptr(w))
    return w


def lmax(total_weight: int, k: int, eps: float) -> int:
    return int(lib().pmo_lmax(total_weight, k, eps_to_ppm(eps)))


def sigma(lmax_: int, total_weight: int, k: int) -> int:
    return int(lib().pmo_sigma(lmax_, total_weight, k))


def gain(g, part, a, d, v: int, b: int) -> int:
    lv, a, d = _hier(a, d)
    part = _i32(part)
    return int(lib().pmo_gain(_ptr(g.xadj), _ptr(g.adjncy), _ptr(g.adjwgt), _ptr(part),
                              lv, _ptr(a), _ptr(d), v, b))


def hash64(seed: int, word: int) -> int:
    return int(lib().pmo_hash(seed & (2**64 - 1), word & (2**64 - 1)))


def lp_round(g, a, d, part, lock, var=None):
    """One label-propagation round.  Returns (part', lock', target, gain, moved).
    var: Variants or None."""
    lv, a, d = _hier(a, d)
    part = _i32(part).copy()
    lock = np.ascontiguousarray(np.asarray(lock, dtype=np.uint8)).copy()
    n = g.n
    target = np.empty(n, np.int32)
    gn = np.empty(n, np.int64)
    moved = np.empty(n, np.uint8)
    lib().pmo_lp_round_v(n, _ptr(g.xadj), _ptr(g.adjncy), _ptr(g.adjwgt), lv, _ptr(a),
                         _ptr(d), _ptr(part), _ptr(lock), _ptr(target), _ptr(gn),
                         _ptr(moved), _var(var))
    return part, lock, target, gn, moved


def rebalance(g, k, part, strong: bool, lmax_: int, sigma_: int, seed: int,
              level: int, it: int, a=None, d=None, var=None):
    """One weak/strong rebalancing round.  Returns (part', moved).  a, d (the
    hierarchy) are needed by the J-objective variant only."""
    part = _i32(part).copy()
    moved = np.empty(g.n, np.uint8)
    if a is None:
        lv, ap, dp = 0, None, None
    else:
        lv, a, d = _hier(a, d)
        ap, dp = _ptr(a), _ptr(d)
    lib().pmo_rebalance_v(g.n, _ptr(g.xadj), _ptr(g.adjncy), _ptr(g.adjwgt), _ptr(g.vwgt),
                          lv, ap, dp, k, int(bool(strong)), lmax_, sigma_,
                          seed & (2**64 - 1), level, it, _ptr(part), _ptr(moved), _var(var))
    return part, moved


def refine(g, a, d, eps, seed, part, level: int = 0, var=None):
    """Algorithm-6 refinement.  Returns (status, part, RefineStats)."""
    lv, a, d = _hier(a, d)
    part = _i32(part).copy()
    st = RefineStats()
    rc = lib().pmo_refine_v(g.n, _ptr(g.xadj), _ptr(g.adjncy), _ptr(g.adjwgt), _ptr(g.vwgt),
                            lv, _ptr(a), _ptr(d), eps_to_ppm(eps), seed & (2**64 - 1), level,
                            _ptr(part), ctypes.byref(st), _var(var))
    return int(rc), part, st


def refine_trace(g, a, d, eps, seed, part, level: int = 0, var=None, cap: int = 4096):
    """refine() with a record of the loop bodies.  Returns (status, part,
    RefineStats, kinds, j_after, imb_after, counter): kinds is a string of
    'L' / 'w' / 'S' per body; j_after, imb_after and counter are J, the
    heaviest block and Algorithm 6's counter i after each body."""
    lv, a, d = _hier(a, d)
    part = _i32(part).copy()
    st = RefineStats()
    kinds = ctypes.create_string_buffer(cap)
    ja = np.zeros(cap, np.int64)
    ia = np.zeros(cap, np.int64)
    ct = np.zeros(cap, np.int32)
    rc = lib().pmo_refine_trace(g.n, _ptr(g.xadj), _ptr(g.adjncy), _ptr(g.adjwgt),
                                _ptr(g.vwgt), lv, _ptr(a), _ptr(d), eps_to_ppm(eps),
                                seed & (2**64 - 1), level, _ptr(part), ctypes.byref(st),
                                _var(var), cap, kinds, _ptr(ja), _ptr(ia), _ptr(ct))
    m = min(st.iterations, cap)
    return (int(rc), part, st, kinds.raw[:m].decode(), ja[:m].copy(), ia[:m].copy(),
            ct[:m].copy())


def hem(g, lmax_: int, seed: int, level: int = 0):
    """Heavy-edge matching.  Returns (rounds, match)."""
    match = np.empty(g.n, np.int32)
    r = lib().pmo_hem(g.n, _ptr(g.xadj), _ptr(g.adjncy), _ptr(g.adjwgt), _ptr(g.vwgt),
                      lmax_, seed & (2**64 - 1), level, _ptr(match))
    return int(r), match


def coarse_map(match):
    match = _i32(match)
    cmap = np.empty(match.shape[0], np.int32)
    nc = lib().pmo_coarse_map(match.shape[0], _ptr(match), _ptr(cmap))
    return int(nc), cmap


def contract(g, cmap, nc: int):
    """Contract g along cmap.  Returns a gen.Graph-like tuple of arrays."""
    cmap = _i32(cmap)
    nnz = max(g.nnz, 1)
    cx = np.empty(nc + 1, np.int64)
    ca = np.empty(nnz, np.int32)
    cw = np.empty(nnz, np.int32)
    cv = np.empty(max(nc, 1), np.int32)
    m = lib().pmo_contract(g.n, _ptr(g.xadj), _ptr(g.adjncy), _ptr(g.adjwgt), _ptr(g.vwgt),
                           _ptr(cmap), nc, _ptr(cx), _ptr(ca), _ptr(cw), _ptr(cv))
    return cx, ca[:m].copy(), cw[:m].copy(), cv[:nc].copy()


def initial_partition(g, a):
    a = _i32(a)
    part = np.empty(g.n, np.int32)
    lib().pmo_initial_partition(g.n, _ptr(g.xadj), _ptr(g.adjncy), _ptr(g.vwgt),
                                a.shape[0], _ptr(a), _ptr(part))
    return part


def map_graph(g, a, d, eps, seed, var=None):
    """Full multilevel mapping.  Returns (status, part, MapStats)."""
    lv, a, d = _hier(a, d)
    part = np.empty(g.n, np.int32)
    st = MapStats()
    rc = lib().pmo_map_v(g.n, _ptr(g.xadj), _ptr(g.adjncy), _ptr(g.adjwgt), _ptr(g.vwgt),
                         lv, _ptr(a), _ptr(d), eps_to_ppm(eps), seed & (2**64 - 1),
                         _ptr(part), ctypes.byref(st), _var(var))
    return int(rc), part, st


def subgraphs(g, part, parts: int):
    """Induced subgraphs of a partition (Algorithm 1).  Returns a dict with
    vstart, estart, order, xadj, adjncy, adjwgt, vwgt (blocks concatenated)."""
    part = _i32(part)
    n = g.n
    vstart = np.empty(parts + 1, np.int32)
    estart = np.empty(parts + 1, np.int64)
    order = np.empty(max(n, 1), np.int32)
    xo = np.empty(n + parts, np.int64)
    ao = np.empty(max(g.nnz, 1), np.int32)
    wo = np.empty(max(g.nnz, 1), np.int32)
    vo = np.empty(max(n, 1), np.int32)
    m = lib().pmo_subgraphs(n, _ptr(g.xadj), _ptr(g.adjncy), _ptr(g.adjwgt), _ptr(g.vwgt),
                            _ptr(part), parts, _ptr(vstart), _ptr(estart), _ptr(order),
                            _ptr(xo), _ptr(ao), _ptr(wo), _ptr(vo))
    return {"vstart": vstart, "estart": estart, "order": order[:n], "xadj": xo,
            "adjncy": ao[:m], "adjwgt": wo[:m], "vwgt": vo[:n]}


def adaptive_eps_ppm(eps_ppm: int, kp: int, k: int, cv: int, cvp: int, d: int) -> int:
    return int(lib().pmo_adaptive_eps_ppm(eps_ppm, kp, k, cv, cvp, d))


def hm(g, a, eps, seed, var=None):
    """Recursive hierarchical multisection (Algorithm 2); var: refinement
    variants of every partitioning call.  Returns (status, part)."""
    a = _i32(a)
    part = np.empty(max(g.n, 1), np.int32)
    rc = lib().pmo_hm_v(g.n, _ptr(g.xadj), _ptr(g.adjncy), _ptr(g.adjwgt), _ptr(g.vwgt),
                        a.shape[0], _ptr(a), eps_to_ppm(eps), seed & (2**64 - 1), _ptr(part),
                        _var(var))
    return int(rc), part[: g.n]
