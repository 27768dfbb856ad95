"""CPU oracle for triangle counting, per-edge support, k-truss and truss
decomposition -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1708_06866_amd``) and the GPU library never imports it.

The arithmetic lives in plain single-threaded C (``oracle.c``, built with gcc
into ``liboracle.so``); this module only marshals numpy arrays.  ``dense``
holds the paper's own array formulations (Alg. 2, 3 and 4) in numpy, used as
independent cross-checks on tiny graphs.

Function map (paper passage -> function)
  normalisation, Sec. II                      -> normalise
  triangle count, Sec. III-A                  -> triangle_count
  the same count over host threads            -> triangle_count_threads
  per-edge support, Sec. III-B (EA, R == 2)   -> support(method="definition")
  per-edge support by triangle listing        -> support(method="listing")
  k-truss, Sec. III-B / Alg. 4 (bulk rounds)  -> ktruss(method="bulk")
  k-truss, one-at-a-time peeling              -> ktruss(method="peel")
  k-truss, peeling by list search (no index)  -> ktruss(method="search")
  truss decomposition, Sec. III-B last para.  -> truss_decomposition
                                                 (method "bulk", "peel" or
                                                 "search")
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` (plain C, -O2, no OpenMP, no -march; pthreads
    for the threaded count only)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    """Load ``liboracle.so``; the environment variable ORACLE_LIB names another
    build of ``oracle.c`` instead (the mutation tests load planted mistakes
    this way, to show that the pins catch them)."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB") or _LIB_PATH
        if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.oracle_normalise.argtypes = [P, P, i64, i32, i32, P, P]
        lib.oracle_normalise.restype = i64
        lib.oracle_triangle_count.argtypes = [i32, i64, P, P]
        lib.oracle_triangle_count.restype = i64
        lib.oracle_triangle_count_threads.argtypes = [i32, i64, P, P, i32]
        lib.oracle_triangle_count_threads.restype = i64
        lib.oracle_support.argtypes = [i32, i64, P, P, P]
        lib.oracle_support.restype = ctypes.c_int
        lib.oracle_support_listing.argtypes = [i32, i64, P, P, P]
        lib.oracle_support_listing.restype = ctypes.c_int
        lib.oracle_ktruss_bulk.argtypes = [i32, i64, P, P, i32, P]
        lib.oracle_ktruss_bulk.restype = i32
        lib.oracle_ktruss_peel.argtypes = [i32, i64, P, P, i32, P]
        lib.oracle_ktruss_peel.restype = i32
        lib.oracle_ktruss_search.argtypes = [i32, i64, P, P, i32, P]
        lib.oracle_ktruss_search.restype = i32
        lib.oracle_truss_decomposition.argtypes = [i32, i64, P, P, i32, P, P]
        lib.oracle_truss_decomposition.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.int32)


def _check_canonical(u: np.ndarray, v: np.ndarray, n: int):
    if len(u) != len(v):
        raise ValueError("u and v differ in length")
    if len(u) == 0:
        return
    if (u < 0).any() or (v >= n).any() or not (u < v).all():
        raise ValueError("not a canonical edge list (need 0 <= u < v < n)")
    key = u.astype(np.int64) * (1 << 32) + v.astype(np.int64)
    if not (np.diff(key) > 0).all():
        raise ValueError("canonical edge list must be sorted and duplicate-free")


def normalise(src, dst, n: int, one_based: bool = False):
    """Raw pairs -> canonical edge list ``(u, v)`` (Sec. II)."""
    src, dst = _i32(src), _i32(dst)
    if len(src) != len(dst):
        raise ValueError("src and dst differ in length")
    u = np.empty(max(len(src), 1), np.int32)
    v = np.empty(max(len(src), 1), np.int32)
    m = _load().oracle_normalise(_p(src), _p(dst), len(src), int(n),
                                 1 if one_based else 0, _p(u), _p(v))
    if m == -1:
        raise ValueError("vertex id out of range")
    if m < 0:
        raise MemoryError("oracle_normalise failed")
    return u[:m].copy(), v[:m].copy()


def triangle_count(n: int, u, v) -> int:
    u, v = _i32(u), _i32(v)
    _check_canonical(u, v, n)
    t = _load().oracle_triangle_count(int(n), len(u), _p(u), _p(v))
    if t < 0:
        raise MemoryError("oracle_triangle_count failed")
    return int(t)


def triangle_count_threads(n: int, u, v, threads: int) -> int:
    """The forward-listing count with its outer loop dealt over `threads`
    host threads (per-thread int64 partials); equal to triangle_count."""
    u, v = _i32(u), _i32(v)
    _check_canonical(u, v, n)
    t = _load().oracle_triangle_count_threads(int(n), len(u), _p(u), _p(v), int(threads))
    if t == -1:
        raise ValueError("threads must be in 1..1024")
    if t < 0:
        raise MemoryError("oracle_triangle_count_threads failed")
    return int(t)


def support(n: int, u, v, method: str = "definition") -> np.ndarray:
    """Per-edge support.  ``definition``: |N(u) cap N(v)| edge by edge;
    ``listing``: every triangle listed once and scattered to its 3 edges."""
    u, v = _i32(u), _i32(v)
    _check_canonical(u, v, n)
    s = np.zeros(max(len(u), 1), np.int32)
    fn = {"definition": _load().oracle_support,
          "listing": _load().oracle_support_listing}[method]
    if fn(int(n), len(u), _p(u), _p(v), _p(s)) != 0:
        raise MemoryError("oracle support failed")
    return s[:len(u)].copy()


def ktruss(n: int, u, v, k: int, method: str = "bulk", start=None):
    """Mask (uint8, canonical order) of the maximal k-truss.  With
    ``method="bulk"`` also returns the number of removing rounds."""
    u, v = _i32(u), _i32(v)
    _check_canonical(u, v, n)
    if k < 2:
        raise ValueError("k must be >= 2")
    mask = np.ones(max(len(u), 1), np.uint8) if start is None else \
        np.ascontiguousarray(np.asarray(start), dtype=np.uint8).copy()
    if len(mask) < len(u):
        raise ValueError("start holds %d entries, %d edges" % (len(mask), len(u)))
    lib = _load()
    if method == "bulk":
        r = lib.oracle_ktruss_bulk(int(n), len(u), _p(u), _p(v), int(k), _p(mask))
    elif method == "peel":
        r = lib.oracle_ktruss_peel(int(n), len(u), _p(u), _p(v), int(k), _p(mask))
    elif method == "search":
        r = lib.oracle_ktruss_search(int(n), len(u), _p(u), _p(v), int(k), _p(mask))
    else:
        raise ValueError(method)
    if r < 0:
        raise RuntimeError("oracle ktruss failed (%d)" % r)
    mask = mask[:len(u)].copy()
    return (mask, int(r)) if method == "bulk" else mask


def truss_decomposition(n: int, u, v, method: str = "peel"):
    """``(tau, kmax)``: truss number per canonical edge and the largest k with a
    non-empty k-truss.  ``bulk``: Alg. 4's rounds per level; ``peel``:
    one-at-a-time peeling over a triangle index (3T edge pairs in memory);
    ``search``: the same peeling with each removed edge's triangles found by
    searching adjacency lists (memory O(n + m), for the largest graphs)."""
    u, v = _i32(u), _i32(v)
    _check_canonical(u, v, n)
    tau = np.zeros(max(len(u), 1), np.int32)
    kmax = ctypes.c_int32(0)
    meth = {"bulk": 0, "peel": 1, "search": 2}[method]
    rc = _load().oracle_truss_decomposition(int(n), len(u), _p(u), _p(v), meth,
                                            _p(tau), ctypes.byref(kmax))
    if rc != 0:
        raise RuntimeError("oracle truss decomposition failed (%d)" % rc)
    return tau[:len(u)].copy(), int(kmax.value)
