"""Python access to the plain CPU oracle (dottt_oracle.c) and to CPU DOTTT (cpu_dottt.c), the
paper's own method run sequentially on the CPU.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's CPU-baseline leg are
the only callers.  The GPU library never imports or links this package, and this package never
imports the GPU library.  The two C files share no code with each other either.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dottt_oracle.c")
_LIB = os.path.join(_HERE, "libdottt_oracle.so")
_SRC_CPU = os.path.join(_HERE, "cpu_dottt.c")
_LIB_CPU = os.path.join(_HERE, "libcpu_dottt.so")
_lib = None
_lib_cpu = None

INT64_MAX = (1 << 63) - 1
INT64_MIN = -(1 << 63)


class OracleError(RuntimeError):
    pass


class _Stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64), ("m", ctypes.c_uint64), ("self_loops", ctypes.c_uint64),
        ("m_window", ctypes.c_uint64), ("m_static", ctypes.c_uint64),
        ("n_triangles", ctypes.c_uint64), ("degeneracy", ctypes.c_uint32),
        ("max_multiplicity", ctypes.c_uint32), ("t_min", ctypes.c_int64),
        ("t_max", ctypes.c_int64), ("sum_sigma3_lo", ctypes.c_uint64),
        ("sum_sigma3_hi", ctypes.c_uint64),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP) into oracle/libdottt_oracle.so and CPU DOTTT (one
    thread) into oracle/libcpu_dottt.so."""
    global _lib, _lib_cpu
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
        _lib = None
    if force or not os.path.exists(_LIB_CPU):
        tmp = _LIB_CPU + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC_CPU])
        os.replace(tmp, _LIB_CPU)
        _lib_cpu = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_count.argtypes = [ctypes.c_uint32, ctypes.c_uint64, P, P, P,
                                     ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_int64, ctypes.c_int, P, P]
        lib.oracle_count.restype = ctypes.c_int
        lib.oracle_stats_compute.argtypes = [ctypes.c_uint32, ctypes.c_uint64, P, P, P,
                                             ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                             ctypes.POINTER(_Stats), P]
        lib.oracle_stats_compute.restype = ctypes.c_int
        lib.oracle_triangles.argtypes = [ctypes.c_uint32, ctypes.c_uint64, P, P, P,
                                         ctypes.c_int64, ctypes.c_int64, P, ctypes.c_uint64]
        lib.oracle_triangles.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _arrs(src, dst, t):
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    t = np.ascontiguousarray(t, dtype=np.int64)
    if not (src.shape == dst.shape == t.shape):
        raise OracleError("src, dst and t must have the same length")
    return src, dst, t


def _ptr(a):
    return a.ctypes.data if a.size else None


def count(n, src, dst, t, d13, d12, d23, t_lo=INT64_MIN, t_hi=INT64_MAX, nthreads=0,
          cells=False):
    """Per-type counts (int64[8], index k = type T(k+1)) and optionally the 48 cells
    (int64[6, 8], [pi-1, rho-1], vertices named u < v < w by node id)."""
    src, dst, t = _arrs(src, dst, t)
    ty = np.zeros(8, dtype=np.int64)
    ce = np.zeros(48, dtype=np.int64)
    rc = _load().oracle_count(int(n), int(src.shape[0]), _ptr(src), _ptr(dst), _ptr(t),
                              int(d13), int(d12), int(d23), int(t_lo), int(t_hi), int(nthreads),
                              ty.ctypes.data, ce.ctypes.data)
    if rc != 0:
        raise OracleError(f"oracle_count failed: {rc}")
    return (ty, ce.reshape(6, 8)) if cells else ty


def stats(n, src, dst, t, t_lo=INT64_MIN, t_hi=INT64_MAX, nthreads=0, core=False):
    """Graph statistics as a dict (Table 1's columns); with core=True also the core numbers."""
    src, dst, t = _arrs(src, dst, t)
    st = _Stats()
    cr = np.zeros(max(int(n), 1), dtype=np.uint32)
    rc = _load().oracle_stats_compute(int(n), int(src.shape[0]), _ptr(src), _ptr(dst), _ptr(t),
                                      int(t_lo), int(t_hi), int(nthreads), ctypes.byref(st),
                                      cr.ctypes.data if core else None)
    if rc != 0:
        raise OracleError(f"oracle_stats_compute failed: {rc}")
    d = {k: getattr(st, k) for k, _ in _Stats._fields_}
    d["sum_sigma3"] = (d.pop("sum_sigma3_hi") << 64) | d.pop("sum_sigma3_lo")
    return (d, cr[: int(n)]) if core else d


def triangles(n, src, dst, t, t_lo=INT64_MIN, t_hi=INT64_MAX):
    """Static triangles as a lexicographically sorted uint32[k, 3] array of ids a < b < c."""
    src, dst, t = _arrs(src, dst, t)
    lib = _load()
    k = lib.oracle_triangles(int(n), int(src.shape[0]), _ptr(src), _ptr(dst), _ptr(t),
                             int(t_lo), int(t_hi), None, 0)
    if k < 0:
        raise OracleError(f"oracle_triangles failed: {k}")
    out = np.zeros((max(k, 1), 3), dtype=np.uint32)
    k2 = lib.oracle_triangles(int(n), int(src.shape[0]), _ptr(src), _ptr(dst), _ptr(t),
                              int(t_lo), int(t_hi), out.ctypes.data, int(k))
    if k2 != k:
        raise OracleError("triangle count changed between calls")
    return out[:k]


def _load_cpu():
    global _lib_cpu
    if _lib_cpu is None:
        if not os.path.exists(_LIB_CPU):
            build(force=True)
        lib = ctypes.CDLL(_LIB_CPU)
        P = ctypes.c_void_p
        lib.cpu_dottt_count.argtypes = [ctypes.c_uint32, ctypes.c_uint64, P, P, P, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                        ctypes.c_int64, P, ctypes.POINTER(ctypes.c_double)]
        lib.cpu_dottt_count.restype = ctypes.c_int
        _lib_cpu = lib
    return _lib_cpu


def cpu_dottt(n, src, dst, t, d13, d12, d23, t_lo=INT64_MIN, t_hi=INT64_MAX, seconds=False):
    """Per-type counts (int64[8]) by the paper's own algorithm on one CPU thread; with
    seconds=True also the time of its ordering, enumeration and counting steps."""
    src, dst, t = _arrs(src, dst, t)
    ty = np.zeros(8, dtype=np.int64)
    sec = ctypes.c_double(0.0)
    rc = _load_cpu().cpu_dottt_count(int(n), int(src.shape[0]), _ptr(src), _ptr(dst), _ptr(t),
                                     int(d13), int(d12), int(d23), int(t_lo), int(t_hi),
                                     ty.ctypes.data, ctypes.byref(sec))
    if rc != 0:
        raise OracleError(f"cpu_dottt_count failed: {rc}")
    return (ty, sec.value) if seconds else ty
