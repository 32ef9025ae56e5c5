"""ctypes binding of libdottt.so (include/dottt.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does no counting of its own;
a missing library raises instead of falling back to anything else.  Host inputs are numpy arrays;
device inputs are torch tensors on the context's device (PyTorch is used only for device memory
and streams).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdottt.so")

DT_OK = 0
DT_EINVAL = -22
DT_ENOMEM = -12
DT_EOVERFLOW = -75
DT_EBUSY = -16
DT_ETIMEDOUT = -110
DT_EDEVICE = -5
DT_ENOTBUILT = -38
DT_INF = (1 << 63) - 1
INT64_MIN = -(1 << 63)

# the exported entry points, as declared in include/dottt.h
ENTRY_POINTS = (
    "dt_strerror", "dt_last_error", "dt_ctx_create", "dt_ctx_destroy", "dt_ctx_memory",
    "dt_graph_load", "dt_graph_load_device", "dt_graph_build", "dt_graph_set_tuning",
    "dt_graph_stats", "dt_count", "dt_count_async", "dt_count_noalloc", "dt_count_visits", "dt_count_cells", "dt_count_oneshot", "dt_count_sweep", "dt_count_batch",
    "dt_graph_order", "dt_graph_triangles", "dt_graph_free", "dt_server_start",
    "dt_server_add_graph", "dt_server_submit", "dt_server_wait", "dt_server_stats",
    "dt_server_graph_info", "dt_server_stop", "dt_ctx_set_profiling", "dt_ctx_last_profile", "dt_ctx_batch_tuning",
)
PROFILE_SLOTS = ("peel", "relayout", "tri_count", "tri_fill", "light", "heavy_prefix",
                 "heavy_count", "reduce", "medium", "unit", "peel_adj", "peel_tail", "core")


class DtError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


class dt_query(ctypes.Structure):
    _fields_ = [("d13", ctypes.c_int64), ("d12", ctypes.c_int64), ("d23", ctypes.c_int64),
                ("t_lo", ctypes.c_int64), ("t_hi", ctypes.c_int64)]


class dt_stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64), ("m", ctypes.c_uint64), ("m_loaded", ctypes.c_uint64),
        ("self_loops_dropped", ctypes.c_uint64), ("m_static", ctypes.c_uint64),
        ("n_static_triangles", ctypes.c_uint64), ("degeneracy", ctypes.c_uint32),
        ("max_multiplicity", ctypes.c_uint32), ("t_min", ctypes.c_int64), ("t_max", ctypes.c_int64),
        ("max_out_degree", ctypes.c_uint32), ("peel_rounds", ctypes.c_uint32),
        ("sum_sigma3_lo", ctypes.c_uint64), ("sum_sigma3_hi", ctypes.c_uint64),
        ("n_light_triangles", ctypes.c_uint64), ("n_heavy_triangles", ctypes.c_uint64),
        ("n_medium_triangles", ctypes.c_uint64), ("n_unit_triangles", ctypes.c_uint64),
        ("alg_bytes", ctypes.c_uint64), ("alg_bytes_light", ctypes.c_uint64),
        ("alg_bytes_medium", ctypes.c_uint64), ("alg_bytes_unit", ctypes.c_uint64),
        ("alg_bytes_peel", ctypes.c_uint64), ("alg_bytes_triangles", ctypes.c_uint64),
        ("tri_candidates", ctypes.c_uint64), ("heavy_slots", ctypes.c_uint64),
        ("ms_load", ctypes.c_double), ("ms_peel", ctypes.c_double),
        ("ms_orient", ctypes.c_double), ("ms_triangles", ctypes.c_double),
        ("ms_schedule", ctypes.c_double),
        ("n_contested_triangles", ctypes.c_uint64),
        ("light_pair_cap_used", ctypes.c_uint32), ("medium_cost_pct_used", ctypes.c_uint32),
        ("light_blocks_per_cu", ctypes.c_uint32), ("medium_blocks_per_cu", ctypes.c_uint32),
        ("autotuned", ctypes.c_uint32), ("reserved0", ctypes.c_uint32),
    ]


class dt_tuning(ctypes.Structure):
    _fields_ = [("light_pair_cap", ctypes.c_uint32), ("heavy_chunk", ctypes.c_uint32),
                ("medium_pair_cap", ctypes.c_uint32), ("force_path", ctypes.c_uint32),
                ("peel_tail", ctypes.c_uint32), ("order_method", ctypes.c_uint32),
                ("medium_cost_pct", ctypes.c_uint32), ("autotune", ctypes.c_uint32)]


class dt_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_inflight_queries", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("deadline_ns", ctypes.c_int64),
                ("swap_to_host", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class dt_server_info(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in (
        "graphs", "resident_graphs", "resident_bytes", "budget_bytes", "swap_outs", "swap_ins",
        "swap_out_bytes", "swap_in_bytes", "queries_done")]


_lib = None


def library():
    """Load libdottt.so (built by paper_2106_02762_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2106_02762_amd.build.build()")
    # torch ships its own HIP runtime; loaded first, it is the one the library binds to as well, so a
    # process that also uses torch's device memory holds a single runtime (with the system runtime
    # loaded first, torch's own copy then finds no GPU)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, U32, U64, I64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "dt_strerror": (ctypes.c_char_p, [I]),
        "dt_last_error": (ctypes.c_char_p, []),
        "dt_ctx_create": (I, [I, U64, PP]),
        "dt_ctx_destroy": (I, [P]),
        "dt_ctx_memory": (I, [P, ctypes.POINTER(U64), ctypes.POINTER(U64)]),
        "dt_graph_load": (I, [P, U32, U64, P, P, P, PP]),
        "dt_graph_load_device": (I, [P, U32, U64, P, P, P, PP]),
        "dt_graph_build": (I, [P]),
        "dt_graph_set_tuning": (I, [P, ctypes.POINTER(dt_tuning)]),
        "dt_graph_stats": (I, [P, ctypes.POINTER(dt_stats)]),
        "dt_count": (I, [P, ctypes.POINTER(dt_query), P]),
        "dt_count_async": (I, [P, ctypes.POINTER(dt_query), P, P]),
        "dt_count_noalloc": (I, [P, ctypes.POINTER(dt_query), P, P]),
        "dt_count_visits": (I, [P, ctypes.POINTER(dt_query), P, ctypes.POINTER(U64)]),
        "dt_count_cells": (I, [P, ctypes.POINTER(dt_query), P]),
        "dt_count_oneshot": (I, [P, ctypes.POINTER(dt_query), P]),
        "dt_count_sweep": (I, [P, U64, P, P]),
        "dt_count_batch": (I, [P, U64, P, P, P]),
        "dt_graph_order": (I, [P, P, P]),
        "dt_graph_triangles": (I, [P, P, U64, ctypes.POINTER(U64)]),
        "dt_graph_free": (I, [P]),
        "dt_server_start": (I, [P, ctypes.POINTER(dt_server_cfg), PP]),
        "dt_server_add_graph": (I, [P, P, ctypes.POINTER(U32)]),
        "dt_server_submit": (I, [P, U32, ctypes.POINTER(dt_query), ctypes.POINTER(U64)]),
        "dt_server_wait": (I, [P, U64, P, I64]),
        "dt_server_stats": (I, [P, ctypes.POINTER(dt_server_info)]),
        "dt_server_graph_info": (I, [P, U32, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(U64)]),
        "dt_server_stop": (I, [P]),
        "dt_ctx_set_profiling": (I, [P, I]),
        "dt_ctx_last_profile": (I, [P, P]),
        "dt_ctx_batch_tuning": (I, [P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc, where):
    if rc != DT_OK:
        lib = library()
        raise DtError(rc, where, lib.dt_last_error().decode() or lib.dt_strerror(rc).decode())


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def make_query(d13, d12, d23, t_lo=INT64_MIN, t_hi=DT_INF):
    return dt_query(int(d13), int(d12), int(d23), int(t_lo), int(t_hi))


# --- entry points ------------------------------------------------------------------------------

def dt_strerror(code):
    return library().dt_strerror(int(code)).decode()


def dt_last_error():
    return library().dt_last_error().decode()


def dt_ctx_create(hip_device=0, hbm_budget_bytes=0):
    h = ctypes.c_void_p()
    _check(library().dt_ctx_create(int(hip_device), int(hbm_budget_bytes), ctypes.byref(h)),
           "dt_ctx_create")
    return h


def dt_ctx_destroy(ctx):
    _check(library().dt_ctx_destroy(ctx), "dt_ctx_destroy")


def dt_ctx_memory(ctx):
    used, budget = ctypes.c_uint64(), ctypes.c_uint64()
    _check(library().dt_ctx_memory(ctx, ctypes.byref(used), ctypes.byref(budget)), "dt_ctx_memory")
    return used.value, budget.value


def dt_graph_load(ctx, n, src, dst, t):
    src, dst, t = _u32(src), _u32(dst), _i64(t)
    if not (src.shape == dst.shape == t.shape):
        raise ValueError("src, dst and t must have the same length")
    h = ctypes.c_void_p()
    m = int(src.shape[0])
    _check(library().dt_graph_load(ctx, int(n), m, src.ctypes.data if m else None,
                                   dst.ctypes.data if m else None, t.ctypes.data if m else None,
                                   ctypes.byref(h)), "dt_graph_load")
    return h


def dt_graph_load_device(ctx, n, src, dst, t):
    """src, dst (torch.int32 holding uint32 ids) and t (torch.int64) on the context's device."""
    m = int(src.numel())
    if not (src.is_cuda and dst.is_cuda and t.is_cuda):
        raise ValueError("dt_graph_load_device takes device tensors")
    if src.element_size() != 4 or dst.element_size() != 4 or t.element_size() != 8:
        raise ValueError("src/dst must be 32-bit and t 64-bit tensors")
    if not (src.is_contiguous() and dst.is_contiguous() and t.is_contiguous()):
        raise ValueError("tensors must be contiguous")
    h = ctypes.c_void_p()
    _check(library().dt_graph_load_device(ctx, int(n), m, src.data_ptr(), dst.data_ptr(),
                                          t.data_ptr(), ctypes.byref(h)), "dt_graph_load_device")
    return h


def dt_graph_build(g):
    _check(library().dt_graph_build(g), "dt_graph_build")


def dt_graph_set_tuning(g, light_pair_cap=0, heavy_chunk=0, medium_pair_cap=0, force_path=0,
                        peel_tail=0, order_method=0, medium_cost_pct=0, autotune=0):
    """force_path: 0 unit records and the split, 1 all light, 2 all heavy, 3 all medium.
    peel_tail: vertices the level peel leaves to one workgroup (next build; 0 keeps the setting).
    order_method: 0 the level-by-level peel, 1 h-index core numbers and shell rounds.
    medium_cost_pct: weight of the prefix procedures' cost in the medium / heavy split (percent).
    autotune: 0 tune per size class when not cached, 1 never, 2 tune again now."""
    tu = dt_tuning(int(light_pair_cap), int(heavy_chunk), int(medium_pair_cap), int(force_path),
                   int(peel_tail), int(order_method), int(medium_cost_pct), int(autotune))
    _check(library().dt_graph_set_tuning(g, ctypes.byref(tu)), "dt_graph_set_tuning")


def dt_graph_stats(g):
    st = dt_stats()
    _check(library().dt_graph_stats(g, ctypes.byref(st)), "dt_graph_stats")
    d = {k: getattr(st, k) for k, _ in dt_stats._fields_}
    d["sum_sigma3"] = (d.pop("sum_sigma3_hi") << 64) | d.pop("sum_sigma3_lo")
    return d


def dt_count(g, d13, d12, d23, t_lo=INT64_MIN, t_hi=DT_INF):
    q = make_query(d13, d12, d23, t_lo, t_hi)
    out = np.zeros(8, dtype=np.int64)
    _check(library().dt_count(g, ctypes.byref(q), out.ctypes.data), "dt_count")
    return out


def dt_count_async(g, query, out8_ptr, stream_ptr=None):
    """Enqueue a count; out8_ptr is a device (or pinned host) address of 8 int64."""
    _check(library().dt_count_async(g, ctypes.byref(query), ctypes.c_void_p(int(out8_ptr)),
                                    ctypes.c_void_p(int(stream_ptr)) if stream_ptr else None),
           "dt_count_async")


def dt_count_visits(g, d13, d12, d23, t_lo=INT64_MIN, t_hi=DT_INF):
    """The count with instrumented kernels: (int64[8] counts, visits)."""
    q = make_query(d13, d12, d23, t_lo, t_hi)
    out = np.zeros(8, dtype=np.int64)
    v = ctypes.c_uint64()
    _check(library().dt_count_visits(g, ctypes.byref(q), out.ctypes.data, ctypes.byref(v)), "dt_count_visits")
    return out, v.value


def dt_count_noalloc(g, query, out8_ptr, stream_ptr=None):
    """dt_count_async with the scratch in the library's fixed per-device array (no allocation)."""
    _check(library().dt_count_noalloc(g, ctypes.byref(query), ctypes.c_void_p(int(out8_ptr)),
                                      ctypes.c_void_p(int(stream_ptr)) if stream_ptr else None),
           "dt_count_noalloc")


def dt_count_cells(g, d13, d12, d23, t_lo=INT64_MIN, t_hi=DT_INF):
    q = make_query(d13, d12, d23, t_lo, t_hi)
    out = np.zeros(48, dtype=np.int64)
    _check(library().dt_count_cells(g, ctypes.byref(q), out.ctypes.data), "dt_count_cells")
    return out.reshape(6, 8)


def dt_count_oneshot(g, d13, d12, d23, t_lo=INT64_MIN, t_hi=DT_INF):
    """Ordering, orientation and a fused enumerate-and-count pass for one query; int64[8]."""
    q = make_query(d13, d12, d23, t_lo, t_hi)
    out = np.zeros(8, dtype=np.int64)
    _check(library().dt_count_oneshot(g, ctypes.byref(q), out.ctypes.data), "dt_count_oneshot")
    return out


def dt_count_sweep(g, deltas, t_lo=INT64_MIN, t_hi=DT_INF):
    """Counts of several (d13, d12, d23) triples over one window; returns int64[k][8]."""
    k = len(deltas)
    qarr = (dt_query * max(k, 1))(*[make_query(*d, t_lo, t_hi) for d in deltas])
    out = np.zeros((max(k, 1), 8), dtype=np.int64)
    _check(library().dt_count_sweep(g, k, qarr, out.ctypes.data), "dt_count_sweep")
    return out[:k]


def dt_count_batch(ctx, graphs, queries):
    k = len(graphs)
    garr = (ctypes.c_void_p * max(k, 1))(*[g.value if hasattr(g, "value") else g for g in graphs])
    qarr = (dt_query * max(k, 1))(*queries)
    out = np.zeros((max(k, 1), 8), dtype=np.int64)
    _check(library().dt_count_batch(ctx, k, garr, qarr, out.ctypes.data), "dt_count_batch")
    return out[:k]


def dt_graph_order(g, n):
    core = np.zeros(max(int(n), 1), dtype=np.uint32)
    rank = np.zeros(max(int(n), 1), dtype=np.uint32)
    _check(library().dt_graph_order(g, core.ctypes.data, rank.ctypes.data), "dt_graph_order")
    return core[: int(n)], rank[: int(n)]


def dt_graph_triangles(g):
    cnt = ctypes.c_uint64()
    _check(library().dt_graph_triangles(g, None, 0, ctypes.byref(cnt)), "dt_graph_triangles")
    k = cnt.value
    out = np.zeros((max(k, 1), 3), dtype=np.uint32)
    _check(library().dt_graph_triangles(g, out.ctypes.data, k, ctypes.byref(cnt)), "dt_graph_triangles")
    return out[:k]


def dt_graph_free(g):
    _check(library().dt_graph_free(g), "dt_graph_free")


def dt_ctx_batch_tuning(ctx):
    """(light triangles, medium entries) per item of the context's last batched launch."""
    out = np.zeros(2, dtype=np.uint32)
    _check(library().dt_ctx_batch_tuning(ctx, out.ctypes.data), "dt_ctx_batch_tuning")
    return int(out[0]), int(out[1])


def dt_ctx_set_profiling(ctx, enable=True):
    _check(library().dt_ctx_set_profiling(ctx, 1 if enable else 0), "dt_ctx_set_profiling")


def dt_ctx_last_profile(ctx):
    """{slot: ms} of the event-timed kernels of the last build and count (0 if not run)."""
    ms = np.zeros(len(PROFILE_SLOTS), dtype=np.float32)
    _check(library().dt_ctx_last_profile(ctx, ms.ctypes.data), "dt_ctx_last_profile")
    return {k: float(v) for k, v in zip(PROFILE_SLOTS, ms)}


def dt_server_start(ctx, hbm_budget_bytes=0, max_inflight_queries=0, max_batch=0, deadline_ns=0,
                    swap_to_host=0):
    cfg = dt_server_cfg(int(hbm_budget_bytes), int(max_inflight_queries), int(max_batch),
                        int(deadline_ns), int(swap_to_host), 0)
    h = ctypes.c_void_p()
    _check(library().dt_server_start(ctx, ctypes.byref(cfg), ctypes.byref(h)), "dt_server_start")
    return h


def dt_server_add_graph(server, g):
    gid = ctypes.c_uint32()
    _check(library().dt_server_add_graph(server, g, ctypes.byref(gid)), "dt_server_add_graph")
    return gid.value


def dt_server_submit(server, graph_id, d13, d12, d23, t_lo=INT64_MIN, t_hi=DT_INF):
    q = make_query(d13, d12, d23, t_lo, t_hi)
    ticket = ctypes.c_uint64()
    _check(library().dt_server_submit(server, int(graph_id), ctypes.byref(q), ctypes.byref(ticket)),
           "dt_server_submit")
    return ticket.value


def dt_server_wait(server, ticket, timeout_ns=-1):
    out = np.zeros(8, dtype=np.int64)
    _check(library().dt_server_wait(server, int(ticket), out.ctypes.data, int(timeout_ns)),
           "dt_server_wait")
    return out


def dt_server_stats(server):
    st = dt_server_info()
    _check(library().dt_server_stats(server, ctypes.byref(st)), "dt_server_stats")
    return {k: getattr(st, k) for k, _ in dt_server_info._fields_}


def dt_server_graph_info(server, graph_id):
    """(resident, device bytes) of an admitted graph."""
    r = ctypes.c_int()
    b = ctypes.c_uint64()
    _check(library().dt_server_graph_info(server, int(graph_id), ctypes.byref(r), ctypes.byref(b)),
           "dt_server_graph_info")
    return bool(r.value), b.value


def dt_server_stop(server):
    _check(library().dt_server_stop(server), "dt_server_stop")
