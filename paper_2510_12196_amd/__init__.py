"""MI355X (gfx950) hierarchical process mapping -- Python binding.

A thin ctypes layer over ``libpm.so`` (C ABI declared in ``include/pm.h``).
Every function has the name of its C entry point and only marshals
arguments: device arrays are torch tensors on a ROCm device, passed by
``data_ptr()``, with torch's current stream.  All computation runs in the
library's HIP kernels; there is no CPU fallback -- if ``libpm.so`` is missing
or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpm.so")

PM_OK = 0
PM_WARN_IMBALANCED = 1
PM_EINVAL = -1
PM_EGRAPH = -2
PM_EOVERFLOW = -3
PM_ENOMEM = -4
PM_EHIP = -5
PM_ENODEVICE = -6
PM_FLAG_VALIDATE = 1
PM_FLAG_KERNEL_TIMES = 2
PM_FLAG_KERNEL_COUNTS = 4
TIMED_KERNELS = ("lp_phase1", "lp_phase2", "apply_moves", "hem_prefer", "reb_select")
MAX_LEVELS = 8
MAX_GRAPH_LEVELS = 64


class PmError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {_strerror(code)} ({code})")


class PmGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("xadj", ctypes.c_void_p), ("adjncy", ctypes.c_void_p),
                ("adjwgt", ctypes.c_void_p), ("vwgt", ctypes.c_void_p)]


class PmHierarchy(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("a", ctypes.c_int32 * MAX_LEVELS),
                ("d", ctypes.c_int32 * MAX_LEVELS)]


class PmRefineStats(ctypes.Structure):
    _fields_ = [("j_initial", ctypes.c_int64), ("j_final", ctypes.c_int64),
                ("maxw_initial", ctypes.c_int64), ("maxw_final", ctypes.c_int64),
                ("iterations", ctypes.c_int32), ("lp_iterations", ctypes.c_int32),
                ("weak_iterations", ctypes.c_int32), ("strong_iterations", ctypes.c_int32),
                ("feasible", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("refine_ms", ctypes.c_double), ("arcs_processed", ctypes.c_int64)]


class PmMapStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("feasible", ctypes.c_int32),
                ("j_final", ctypes.c_int64), ("lmax", ctypes.c_int64),
                ("level_n", ctypes.c_int32 * MAX_GRAPH_LEVELS),
                ("level_nnz", ctypes.c_int64 * MAX_GRAPH_LEVELS),
                ("level_iterations", ctypes.c_int32 * MAX_GRAPH_LEVELS),
                ("level_hem_rounds", ctypes.c_int32 * MAX_GRAPH_LEVELS),
                ("coarsen_ms", ctypes.c_double), ("contract_ms", ctypes.c_double),
                ("initial_ms", ctypes.c_double), ("uncoarsen_ms", ctypes.c_double),
                ("refine_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("refine_arcs", ctypes.c_int64),
                ("kernel_launches", ctypes.c_int64 * 5), ("kernel_ms", ctypes.c_double * 5),
                ("kernel_bytes", ctypes.c_double * 5), ("kernel_units", (ctypes.c_int64 * 3) * 5)]


class PmMapJob(ctypes.Structure):
    _fields_ = [("graph", PmGraph), ("hierarchy", PmHierarchy), ("eps", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("part_out", ctypes.c_void_p),
                ("status", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("j_final", ctypes.c_int64), ("ms", ctypes.c_double)]


_P = ctypes.c_void_p
_I32, _I64, _U32, _U64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
_SIGS = {
    "pm_version": (ctypes.c_char_p, []),
    "pm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pm_release": (None, []),
    "pm_comm_cost": (ctypes.c_int, [_P, _P, _P, _P, _U32, _P]),
    "pm_comm_cost_noalloc": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "pm_block_weights": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "pm_lp_round": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "pm_rebalance": (ctypes.c_int, [_P, _P, _I32, _I64, _I64, _U64, _I32, _I32, _P, _P, _P]),
    "pm_refine": (ctypes.c_int, [_P, _P, ctypes.c_double, _U64, _I32, _P, _P, _P]),
    "pm_hem": (ctypes.c_int, [_P, _I64, _U64, _I32, _P, _P, _P]),
    "pm_contract": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "pm_initial_partition": (ctypes.c_int, [_P, _P, _P, _P]),
    "pm_map": (ctypes.c_int, [_P, _P, ctypes.c_double, _U64, _P, _P, _U32, _P]),
    "pm_lp_round_ex": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "pm_rebalance_ex": (ctypes.c_int, [_P, _P, _I32, _I64, _I64, _U64, _I32, _I32, _P, _P, _P,
                                       _P]),
    "pm_refine_ex": (ctypes.c_int, [_P, _P, ctypes.c_double, _U64, _I32, _P, _P, _P, _P]),
    "pm_map_ex": (ctypes.c_int, [_P, _P, ctypes.c_double, _U64, _P, _P, _U32, _P, _P]),
    "pm_subgraphs": (ctypes.c_int, [_P, _P, _I32, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "pm_map_hm": (ctypes.c_int, [_P, _P, ctypes.c_double, _U64, _I32, _P, _P, _P, _P]),
    "pm_map_hm_ex": (ctypes.c_int, [_P, _P, ctypes.c_double, _U64, _I32, _P, _P, _P, _P, _P]),
    "pm_get_tuning": (ctypes.c_int, [_P]),
    "pm_set_tuning": (ctypes.c_int, [_P]),
    "pm_map_batch": (ctypes.c_int, [_P, _I32, _I32, _P]),
    "pm_job_footprint": (_I64, [_P, _P]),
    "pm_server_create": (_P, [_I64, _I32]),
    "pm_server_submit": (_I64, [_P, _P]),
    "pm_server_poll": (ctypes.c_int, [_P, _I64]),
    "pm_server_wait": (ctypes.c_int, [_P, _I64, _P, _P]),
    "pm_server_destroy": (None, [_P]),
}
_lib = None


def lib():
    """Load libpm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2510_12196_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().pm_strerror(code).decode()
    except Exception:  # library not loadable: still produce a message
        return "error"


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise PmError(rc, where)
    return rc


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


PM_VARIANT_JET_FILTER = 1
PM_VARIANT_J_REBALANCE = 2


class PmOptions(ctypes.Structure):
    _fields_ = [("variants", ctypes.c_uint32), ("jet_c_num", ctypes.c_int32),
                ("jet_c_den", ctypes.c_int32), ("refine_repeats", ctypes.c_int32)]


def options(jet_c=None, j_rebalance: bool = False, repeats: int = 0) -> PmOptions:
    """Refinement variants: jet_c = (num, den) enables Jet's relaxed first
    filter with c = num/den; j_rebalance ranks rebalancing moves by the J
    gain; repeats runs Algorithm 6 that many times per level ("ultra": 18)."""
    o = PmOptions()
    o.refine_repeats = int(repeats)
    if jet_c:
        o.variants |= PM_VARIANT_JET_FILTER
        o.jet_c_num, o.jet_c_den = int(jet_c[0]), int(jet_c[1])
    if j_rebalance:
        o.variants |= PM_VARIANT_J_REBALANCE
    return o


class PmTuning(ctypes.Structure):
    _fields_ = [("group_v", ctypes.c_int32), ("wave_min_count", ctypes.c_int32),
                ("hem_compact_min_n", ctypes.c_int32), ("reb_compact_min_n", ctypes.c_int32),
                ("contract_rows_min_nnz", ctypes.c_int32), ("contract_rows_long_pct", ctypes.c_int32),
                ("lp_cache", ctypes.c_int32), ("graph_bodies", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def get_tuning() -> dict:
    """The process-wide launch parameters (never change a result)."""
    t = PmTuning()
    _check(lib().pm_get_tuning(ctypes.byref(t)), "pm_get_tuning")
    return t.as_dict()


def set_tuning(**kw) -> dict:
    """Sets some launch parameters; returns the previous ones."""
    old = get_tuning()
    t = PmTuning(**{**old, **{k: int(v) for k, v in kw.items()}})
    _check(lib().pm_set_tuning(ctypes.byref(t)), "pm_set_tuning")
    return old


class tuned:
    """Context manager: launch parameters for the duration of a block."""

    def __init__(self, **kw):
        self.kw = kw
        self.old = None

    def __enter__(self):
        self.old = set_tuning(**self.kw)
        return self

    def __exit__(self, *exc):
        set_tuning(**self.old)
        return False


def _opt(o):
    return ctypes.byref(o) if o is not None else None


def hierarchy(a, d) -> PmHierarchy:
    a = list(a)
    d = list(d)
    if not (1 <= len(a) <= MAX_LEVELS) or len(a) != len(d):
        raise ValueError("hierarchy needs 1..8 levels and one distance per level")
    h = PmHierarchy()
    h.levels = len(a)
    for i, (x, y) in enumerate(zip(a, d)):
        h.a[i] = int(x)
        h.d[i] = int(y)
    return h


@dataclass
class DeviceGraph:
    """CSR graph in device memory (torch tensors)."""
    xadj: object      # int64[n+1]
    adjncy: object    # int32[nnz]
    adjwgt: object    # int32[nnz]
    vwgt: object      # int32[n]

    @property
    def n(self) -> int:
        return int(self.vwgt.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.adjncy.shape[0])

    @classmethod
    def from_host(cls, g, device="cuda") -> "DeviceGraph":
        torch = _torch()

        def t(x, dt):
            return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=dt))).to(device)
        return cls(t(g.xadj, np.int64), t(g.adjncy, np.int32), t(g.adjwgt, np.int32),
                   t(g.vwgt, np.int32))

    def struct(self) -> PmGraph:
        for x in (self.xadj, self.adjncy, self.adjwgt, self.vwgt):
            if not x.is_cuda or not x.is_contiguous():
                raise ValueError("graph arrays must be contiguous device tensors")
        s = PmGraph()
        s.n = self.n
        s.nnz = self.nnz
        s.xadj = self.xadj.data_ptr()
        s.adjncy = self.adjncy.data_ptr() if self.nnz else None
        s.adjwgt = self.adjwgt.data_ptr() if self.nnz else None
        s.vwgt = self.vwgt.data_ptr() if self.n else None
        return s


def _dev(t, dtype_name, n=None):
    if not t.is_cuda or not t.is_contiguous() or str(t.dtype) != f"torch.{dtype_name}":
        raise ValueError(f"expected a contiguous device tensor of {dtype_name}")
    if n is not None and t.shape[0] != n:
        raise ValueError("array length does not match the graph")
    return ctypes.c_void_p(t.data_ptr())


def pm_version() -> str:
    return lib().pm_version().decode()


def pm_release() -> None:
    lib().pm_release()


def pm_comm_cost(g: DeviceGraph, a, d, part, validate: bool = False) -> int:
    """J = sum over all arcs of w * D(part[u], part[v])."""
    out = ctypes.c_int64(0)
    gs, hs = g.struct(), hierarchy(a, d)
    _check(lib().pm_comm_cost(ctypes.byref(gs), ctypes.byref(hs), _dev(part, "int32", g.n),
                              ctypes.byref(out), PM_FLAG_VALIDATE if validate else 0, _stream()),
           "pm_comm_cost")
    return int(out.value)


def pm_comm_cost_noalloc(g: DeviceGraph, a, d, part) -> int:
    """pm_comm_cost through the entry point that allocates nothing."""
    out = ctypes.c_int64(0)
    gs, hs = g.struct(), hierarchy(a, d)
    _check(lib().pm_comm_cost_noalloc(ctypes.byref(gs), ctypes.byref(hs),
                                      _dev(part, "int32", g.n), ctypes.byref(out), _stream()),
           "pm_comm_cost_noalloc")
    return int(out.value)


def pm_block_weights(g: DeviceGraph, a, d, part):
    torch = _torch()
    k = int(np.prod(a))
    w = torch.empty(k, dtype=torch.int64, device=part.device)
    gs, hs = g.struct(), hierarchy(a, d)
    _check(lib().pm_block_weights(ctypes.byref(gs), ctypes.byref(hs), _dev(part, "int32", g.n),
                                  _dev(w, "int64"), _stream()), "pm_block_weights")
    return w


def pm_lp_round(g: DeviceGraph, a, d, part, lock, opts: PmOptions = None):
    """One label-propagation round; part and lock are updated in place.
    Returns (target, gain, moved)."""
    torch = _torch()
    target = torch.empty(g.n, dtype=torch.int32, device=part.device)
    gain = torch.empty(g.n, dtype=torch.int64, device=part.device)
    moved = torch.empty(g.n, dtype=torch.uint8, device=part.device)
    gs, hs = g.struct(), hierarchy(a, d)
    _check(lib().pm_lp_round_ex(ctypes.byref(gs), ctypes.byref(hs), _dev(part, "int32", g.n),
                                _dev(lock, "uint8", g.n), _dev(target, "int32"),
                                _dev(gain, "int64"), _dev(moved, "uint8"), _opt(opts), _stream()),
           "pm_lp_round")
    return target, gain, moved


def pm_rebalance(g: DeviceGraph, a, d, part, strong: bool, lmax: int, sigma: int, seed: int,
                 level: int, it: int, opts: PmOptions = None):
    """One rebalancing round; part is updated in place.  Returns moved flags."""
    torch = _torch()
    moved = torch.empty(g.n, dtype=torch.uint8, device=part.device)
    gs, hs = g.struct(), hierarchy(a, d)
    _check(lib().pm_rebalance_ex(ctypes.byref(gs), ctypes.byref(hs), int(bool(strong)),
                                 int(lmax), int(sigma), seed & (2**64 - 1), int(level), int(it),
                                 _dev(part, "int32", g.n), _dev(moved, "uint8"), _opt(opts),
                                 _stream()), "pm_rebalance")
    return moved


def pm_refine(g: DeviceGraph, a, d, eps: float, seed: int, part, level: int = 0,
              opts: PmOptions = None):
    """Refinement (Algorithm 6) in place.  Returns (status, PmRefineStats)."""
    st = PmRefineStats()
    gs, hs = g.struct(), hierarchy(a, d)
    rc = _check(lib().pm_refine_ex(ctypes.byref(gs), ctypes.byref(hs), float(eps),
                                   seed & (2**64 - 1), int(level), _dev(part, "int32", g.n),
                                   ctypes.byref(st), _opt(opts), _stream()), "pm_refine")
    return rc, st


def pm_hem(g: DeviceGraph, lmax: int, seed: int, level: int = 0):
    """Heavy-edge matching.  Returns (match, rounds)."""
    torch = _torch()
    match = torch.empty(g.n, dtype=torch.int32, device=g.vwgt.device)
    rounds = ctypes.c_int32(0)
    gs = g.struct()
    _check(lib().pm_hem(ctypes.byref(gs), int(lmax), seed & (2**64 - 1), int(level),
                        _dev(match, "int32"), ctypes.byref(rounds), _stream()), "pm_hem")
    return match, int(rounds.value)


def pm_contract(g: DeviceGraph, match):
    """Coarse numbering + contraction.  Returns (cmap, coarse DeviceGraph)."""
    torch = _torch()
    dev = g.vwgt.device
    n, nnz = g.n, g.nnz
    cmap = torch.empty(n, dtype=torch.int32, device=dev)
    cx = torch.empty(n + 1, dtype=torch.int64, device=dev)
    ca = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    cw = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    cv = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    nc = ctypes.c_int32(0)
    cnnz = ctypes.c_int64(0)
    gs = g.struct()
    _check(lib().pm_contract(ctypes.byref(gs), _dev(match, "int32", n), _dev(cmap, "int32"),
                             _dev(cx, "int64"), _dev(ca, "int32"), _dev(cw, "int32"),
                             _dev(cv, "int32"), ctypes.byref(nc), ctypes.byref(cnnz), _stream()),
           "pm_contract")
    k, m = int(nc.value), int(cnnz.value)
    return cmap, DeviceGraph(cx[: k + 1].clone(), ca[:m].clone(), cw[:m].clone(), cv[:k].clone())


def pm_initial_partition(g: DeviceGraph, a, d):
    torch = _torch()
    part = torch.empty(g.n, dtype=torch.int32, device=g.vwgt.device)
    gs, hs = g.struct(), hierarchy(a, d)
    _check(lib().pm_initial_partition(ctypes.byref(gs), ctypes.byref(hs), _dev(part, "int32"),
                                      _stream()), "pm_initial_partition")
    return part


def pm_map(g: DeviceGraph, a, d, eps: float, seed: int, part=None, validate: bool = False,
           kernel_times: bool = False, opts: PmOptions = None, kernel_counts: bool = False):
    """Full multilevel mapping.  Returns (status, part, PmMapStats).
    kernel_times / kernel_counts: per-launch device times / unit counts of
    the timed kernels (TIMED_KERNELS) in the stats."""
    torch = _torch()
    if part is None:
        part = torch.empty(g.n, dtype=torch.int32, device=g.vwgt.device)
    st = PmMapStats()
    gs, hs = g.struct(), hierarchy(a, d)
    flags = ((PM_FLAG_VALIDATE if validate else 0) | (PM_FLAG_KERNEL_TIMES if kernel_times else 0)
             | (PM_FLAG_KERNEL_COUNTS if kernel_counts else 0))
    if opts is None:
        rc = lib().pm_map(ctypes.byref(gs), ctypes.byref(hs), float(eps), seed & (2**64 - 1),
                          _dev(part, "int32", g.n), ctypes.byref(st), flags, _stream())
    else:
        rc = lib().pm_map_ex(ctypes.byref(gs), ctypes.byref(hs), float(eps), seed & (2**64 - 1),
                             _dev(part, "int32", g.n), ctypes.byref(st), flags, _opt(opts),
                             _stream())
    _check(rc, "pm_map")
    return rc, part, st


def pm_subgraphs(g: DeviceGraph, part, parts: int):
    """Induced subgraphs of every block of `part` (device tensors).  Returns a
    dict with vstart, estart, order, xadj, adjncy, adjwgt, vwgt (the layout
    the C-ABI documents; arcs trimmed to the ones kept)."""
    torch = _torch()
    dev = g.vwgt.device
    n, nnz, parts = g.n, g.nnz, int(parts)
    vstart = torch.empty(parts + 1, dtype=torch.int32, device=dev)
    estart = torch.empty(parts + 1, dtype=torch.int64, device=dev)
    order = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    xadj = torch.empty(n + parts, dtype=torch.int64, device=dev)
    adj = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    wgt = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    vw = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    arcs = ctypes.c_int64(0)
    gs = g.struct()
    _check(lib().pm_subgraphs(ctypes.byref(gs), _dev(part, "int32", n), parts,
                              _dev(vstart, "int32"), _dev(estart, "int64"), _dev(order, "int32"),
                              _dev(xadj, "int64"), _dev(adj, "int32"), _dev(wgt, "int32"),
                              _dev(vw, "int32"), ctypes.byref(arcs), _stream()), "pm_subgraphs")
    m = int(arcs.value)
    return {"vstart": vstart, "estart": estart, "order": order[:n], "xadj": xadj,
            "adjncy": adj[:m], "adjwgt": wgt[:m], "vwgt": vw[:n]}


def pm_map_hm(g: DeviceGraph, a, d, eps: float, seed: int, workers: int = 8, part=None,
              opts: PmOptions = None):
    """Hierarchical multisection with the multilevel mapper as partitioner
    (opts: refinement variants of every partitioning call).
    Returns (status, part, J under (a, d), number of partitioning calls)."""
    torch = _torch()
    if part is None:
        part = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.vwgt.device)
    j = ctypes.c_int64(0)
    calls = ctypes.c_int32(0)
    gs, hs = g.struct(), hierarchy(a, d)
    rc = lib().pm_map_hm_ex(ctypes.byref(gs), ctypes.byref(hs), float(eps), seed & (2**64 - 1),
                            int(workers), ctypes.c_void_p(part.data_ptr()), ctypes.byref(j),
                            ctypes.byref(calls), _opt(opts), _stream())
    _check(rc, "pm_map_hm")
    return rc, part[: g.n], int(j.value), int(calls.value)


def make_job(g: DeviceGraph, a, d, eps: float, seed: int, part=None):
    """A PmMapJob for one instance; returns (job, part) -- keep g and part
    alive until the job is done."""
    torch = _torch()
    if part is None:
        part = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.vwgt.device)
    job = PmMapJob()
    job.graph = g.struct()
    job.hierarchy = hierarchy(a, d)
    job.eps = float(eps)
    job.seed = seed & (2**64 - 1)
    job.part_out = part.data_ptr()
    return job, part


def pm_job_footprint(g: DeviceGraph, a, d) -> int:
    gs, hs = g.struct(), hierarchy(a, d)
    return int(_check(lib().pm_job_footprint(ctypes.byref(gs), ctypes.byref(hs)),
                      "pm_job_footprint"))


def pm_map_batch(instances, workers: int = 8):
    """instances: list of (DeviceGraph, a, d, eps, seed).  Maps them all with
    the batched executor.  Returns a list of (status, part, PmMapJob)."""
    made = [make_job(*inst) for inst in instances]
    arr = (PmMapJob * max(len(made), 1))()
    for i, (job, _) in enumerate(made):
        arr[i] = job
    rc = lib().pm_map_batch(arr, len(made), int(workers), _stream())
    out = []
    for i, (_, part) in enumerate(made):
        j = arr[i]
        out.append((int(j.status), part, j))
    if rc < 0 and all(o[0] >= 0 for o in out):
        raise PmError(rc, "pm_map_batch")
    return out


class PmServer:
    """Continuous-batching server (C ABI pm_server_*).  Jobs are admitted in
    FIFO order against an HBM footprint budget and overlap on the device."""

    def __init__(self, budget_bytes: int, workers: int = 8):
        self._h = lib().pm_server_create(int(budget_bytes), int(workers))
        if not self._h:
            raise PmError(PM_EINVAL, "pm_server_create")
        self._keep = {}

    def submit(self, g: DeviceGraph, a, d, eps: float, seed: int, part=None) -> int:
        job, part = make_job(g, a, d, eps, seed, part)
        t = lib().pm_server_submit(self._h, ctypes.byref(job))
        if t < 0:
            raise PmError(int(t), "pm_server_submit")
        self._keep[t] = (g, part)
        return int(t)

    def poll(self, ticket: int) -> bool:
        return _check(lib().pm_server_poll(self._h, ticket), "pm_server_poll") == 1

    def wait(self, ticket: int):
        """Returns (status, part, PmMapJob, latency_ms)."""
        out = PmMapJob()
        lat = ctypes.c_double(0.0)
        rc = lib().pm_server_wait(self._h, ticket, ctypes.byref(out), ctypes.byref(lat))
        _, part = self._keep.pop(ticket)
        return int(rc), part, out, float(lat.value)

    def close(self):
        if self._h:
            lib().pm_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


__all__ = ["PmOptions", "options", "PM_VARIANT_JET_FILTER", "PM_VARIANT_J_REBALANCE",
           "DeviceGraph", "PmError", "PmGraph", "PmHierarchy", "PmMapStats", "PmRefineStats",
           "hierarchy", "lib", "pm_version", "pm_release", "pm_comm_cost", "pm_comm_cost_noalloc",
           "pm_block_weights",
           "pm_lp_round", "pm_rebalance", "pm_refine", "pm_hem", "pm_contract",
           "pm_initial_partition", "pm_map", "PmMapJob", "make_job", "pm_map_batch",
           "pm_job_footprint", "PmServer"]
