"""Seeded synthetic graph inputs shared by the GPU tests, the oracle tests and
the benchmark.

This package holds no triangle, support or truss arithmetic: it only produces
raw edge pairs (``int32`` arrays ``src``, ``dst``), possibly with duplicates,
both directions and self-loops, exactly as the challenge's inputs may arrive
before normalisation (Sec. II: ids are integers, loops removed, directed graphs
symmetrised).

Families
  * ``rmat``   Kronecker / R-MAT power-law graphs (Graph500-style initiator),
               the synthetic family the paper lists in Sec. II.
  * ``er``     Erdos-Renyi G(n, M), a low-clustering contrast.
  * ``rgg``    random geometric graphs on the unit torus (high clustering).
  * ``king``   the M x M 8-neighbour image graphs of Table II.
  * closed-form families (complete, complete tripartite, wheel, windmill,
    book, diamond, trees, stars, cycles) whose counts are known in closed form.

The bulk generators are C (``graphgen.c``, built into ``libgraphgen.so``);
``rmat_numpy`` is an independent numpy transcription of the same sampling rule
used to pin the C code on small sizes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)


def build(force: bool = True) -> str:
    """Compile ``libgraphgen.so`` with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "graphgen.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double,
                                ctypes.c_uint64, ctypes.c_int, P, P]
        lib.gg_rmat.restype = ctypes.c_int
        lib.gg_er.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                              P, P]
        lib.gg_er.restype = ctypes.c_int
        lib.gg_rgg.argtypes = [ctypes.c_int32, ctypes.c_double,
                               ctypes.c_uint64, P, P, ctypes.c_int64]
        lib.gg_rgg.restype = ctypes.c_int64
        lib.gg_rgg_points.argtypes = [ctypes.c_int32, ctypes.c_uint64, P, P]
        lib.gg_rgg_points.restype = None
        lib.gg_mix64.argtypes = [ctypes.c_uint64]
        lib.gg_mix64.restype = ctypes.c_uint64
        lib.gg_permute_vertex.argtypes = [ctypes.c_uint64, ctypes.c_int,
                                          ctypes.c_uint32]
        lib.gg_permute_vertex.restype = ctypes.c_uint32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# ----------------------------------------------------------------------------
# Bulk generators (C)
# ----------------------------------------------------------------------------

def rmat(scale: int, edge_factor: int = 16, seed: int = 1,
         abcd=RMAT_ABCD, permute: bool = True):
    """R-MAT pairs: ``edge_factor * 2**scale`` samples on ``2**scale`` vertices.

    Returns ``(src, dst, n)`` with int32 arrays."""
    a, b, c, _ = abcd
    n_samples = int(edge_factor) << int(scale)
    src = np.empty(n_samples, dtype=np.int32)
    dst = np.empty(n_samples, dtype=np.int32)
    rc = _load().gg_rmat(int(scale), n_samples, float(a), float(b), float(c),
                         int(seed) & (2**64 - 1), 1 if permute else 0,
                         _ptr(src), _ptr(dst))
    if rc != 0:
        raise ValueError("bad R-MAT arguments")
    return src, dst, 1 << int(scale)


def er(n: int, n_samples: int, seed: int = 2):
    """Erdos-Renyi G(n, M) with M = n_samples independent uniform pairs."""
    src = np.empty(n_samples, dtype=np.int32)
    dst = np.empty(n_samples, dtype=np.int32)
    rc = _load().gg_er(int(n), int(n_samples), int(seed) & (2**64 - 1),
                       _ptr(src), _ptr(dst))
    if rc != 0:
        raise ValueError("bad ER arguments")
    return src, dst, int(n)


def rgg_radius2(n: int, mean_degree: float) -> float:
    """Squared radius giving expected degree ``mean_degree`` on the unit torus:
    pi r^2 (n - 1) = mean_degree."""
    return float(mean_degree) / (math.pi * (n - 1))


def rgg(n: int, mean_degree: float = 20.0, seed: int = 3):
    """Random geometric graph on the unit torus, expected degree ``mean_degree``."""
    r2 = rgg_radius2(n, mean_degree)
    cap = int(n * mean_degree) + 1024
    lib = _load()
    while True:
        src = np.empty(cap, dtype=np.int32)
        dst = np.empty(cap, dtype=np.int32)
        cnt = lib.gg_rgg(int(n), r2, int(seed) & (2**64 - 1), _ptr(src),
                         _ptr(dst), cap)
        if cnt < 0:
            raise ValueError("bad RGG arguments")
        if cnt <= cap:
            return src[:cnt].copy(), dst[:cnt].copy(), int(n)
        cap = int(cnt)


def rgg_points(n: int, seed: int = 3):
    x = np.empty(n, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    _load().gg_rgg_points(int(n), int(seed) & (2**64 - 1), _ptr(x), _ptr(y))
    return x, y


# ----------------------------------------------------------------------------
# Independent numpy transcription of the R-MAT rule (pins the C code)
# ----------------------------------------------------------------------------
_M64 = (1 << 64) - 1


def mix64_py(z: int) -> int:
    z = (z + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z + np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _stream_base_py(seed: int, tag: int) -> int:
    return mix64_py(mix64_py(seed & _M64) ^ ((tag * 0xD1B54A32D192ED03) & _M64))


def _perm_keys_py(seed: int, scale: int):
    base = _stream_base_py(seed, 2)
    mask = (1 << scale) - 1
    k1, k2 = [], []
    for r in range(4):
        x = (mix64_py(base ^ (2 * r)) | 1) & mask
        k1.append(x if x != 0 else 1)
        k2.append(mix64_py(base ^ (2 * r + 1)) & mask)
    return k1, k2


def permute_numpy(x: np.ndarray, scale: int, seed: int) -> np.ndarray:
    if scale == 0:
        return np.zeros_like(x)
    k1, k2 = _perm_keys_py(seed, scale)
    mask = np.uint64((1 << scale) - 1)
    sh = np.uint64((scale + 1) // 2)
    y = x.astype(np.uint64)
    for r in range(4):
        y = (y * np.uint64(k1[r]) + np.uint64(k2[r])) & mask
        y = y ^ (y >> sh)
    return y.astype(np.int32)


def rmat_numpy(scale: int, edge_factor: int = 16, seed: int = 1,
               abcd=RMAT_ABCD, permute: bool = True):
    """Same sampling rule as ``rmat`` written with numpy (slow; small sizes)."""
    a, b, c, _ = abcd
    two32 = 4294967296.0
    ta = np.uint64(math.floor(a * two32))
    tab = np.uint64(math.floor((a + b) * two32))
    tabc = np.uint64(math.floor((a + b + c) * two32))
    n_samples = int(edge_factor) << int(scale)
    base = np.uint64(_stream_base_py(seed, 1))
    i = np.arange(n_samples, dtype=np.uint64)
    u = np.zeros(n_samples, dtype=np.uint64)
    v = np.zeros(n_samples, dtype=np.uint64)
    with np.errstate(over="ignore"):
        for lvl in range(scale):
            r = _mix64_np(base ^ ((i << np.uint64(6)) | np.uint64(lvl))) >> np.uint64(32)
            bu = (r >= tab).astype(np.uint64)
            bv = (((r >= ta) & (r < tab)) | (r >= tabc)).astype(np.uint64)
            u = (u << np.uint64(1)) | bu
            v = (v << np.uint64(1)) | bv
        if permute:
            u = permute_numpy(u, scale, seed).astype(np.uint64)
            v = permute_numpy(v, scale, seed).astype(np.uint64)
    return u.astype(np.int32), v.astype(np.int32), 1 << int(scale)


# ----------------------------------------------------------------------------
# Closed-form families (edge lists, int32)
# ----------------------------------------------------------------------------

def _pairs(edges):
    if len(edges) == 0:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    e = np.asarray(edges, dtype=np.int64)
    return e[:, 0].astype(np.int32), e[:, 1].astype(np.int32)


def king(M: int):
    """M x M image graph, each pixel joined to its 8 neighbours (Table II).
    Vertex (i, j) has id i*M + j."""
    idx = np.arange(M * M, dtype=np.int64).reshape(M, M)
    parts = []
    if M >= 2:
        parts.append((idx[:, :-1].ravel(), idx[:, 1:].ravel()))     # right
        parts.append((idx[:-1, :].ravel(), idx[1:, :].ravel()))     # down
        parts.append((idx[:-1, :-1].ravel(), idx[1:, 1:].ravel()))  # down-right
        parts.append((idx[:-1, 1:].ravel(), idx[1:, :-1].ravel()))  # down-left
    if not parts:
        return np.zeros(0, np.int32), np.zeros(0, np.int32), M * M
    s = np.concatenate([p[0] for p in parts]).astype(np.int32)
    d = np.concatenate([p[1] for p in parts]).astype(np.int32)
    return s, d, M * M


def complete(n: int):
    e = [(i, j) for i in range(n) for j in range(i + 1, n)]
    return (*_pairs(e), n)


def complete_tripartite(a: int, b: int, c: int):
    parts = [list(range(0, a)), list(range(a, a + b)), list(range(a + b, a + b + c))]
    e = []
    for p in range(3):
        for q in range(p + 1, 3):
            e += [(x, y) for x in parts[p] for y in parts[q]]
    return (*_pairs(e), a + b + c)


def wheel(r: int):
    """Hub 0 joined to every vertex of the cycle 1..r."""
    e = [(0, i) for i in range(1, r + 1)]
    e += [(i, i % r + 1) for i in range(1, r + 1)]
    return (*_pairs(e), r + 1)


def windmill(t: int):
    """t triangles sharing the centre 0 (friendship graph)."""
    e = []
    for i in range(t):
        x, y = 1 + 2 * i, 2 + 2 * i
        e += [(0, x), (0, y), (x, y)]
    return (*_pairs(e), 2 * t + 1)


def book(p: int):
    """p triangles sharing the spine edge (0, 1)."""
    e = [(0, 1)]
    for i in range(p):
        e += [(0, 2 + i), (1, 2 + i)]
    return (*_pairs(e), p + 2)


def diamond():
    """Two triangles {a,b,c} and {b,c,d} sharing edge bc (a=0,b=1,c=2,d=3)."""
    return (*_pairs([(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)]), 4)


def star(k: int):
    return (*_pairs([(0, i) for i in range(1, k + 1)]), k + 1)


def path(n: int):
    return (*_pairs([(i, i + 1) for i in range(n - 1)]), n)


def cycle(n: int):
    return (*_pairs([(i, (i + 1) % n) for i in range(n)]), n)


def random_tree(n: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    e = [(int(rng.integers(0, i)), i) for i in range(1, n)]
    return (*_pairs(e), n)


def complete_bipartite(a: int, b: int):
    e = [(x, a + y) for x in range(a) for y in range(b)]
    return (*_pairs(e), a + b)


def disjoint_union(*graphs):
    """Union of (src, dst, n) graphs with ids shifted apart."""
    ss, dd, off = [], [], 0
    for s, d, n in graphs:
        ss.append(s.astype(np.int64) + off)
        dd.append(d.astype(np.int64) + off)
        off += n
    if not ss:
        return np.zeros(0, np.int32), np.zeros(0, np.int32), 0
    return (np.concatenate(ss).astype(np.int32),
            np.concatenate(dd).astype(np.int32), off)


def scramble(src, dst, n, seed: int = 0, reverse_frac: float = 0.5,
             dup_frac: float = 0.3, loops: int = 3):
    """Same graph, presented differently: random pair order, random direction,
    duplicated pairs and injected self-loops (normalisation must undo all)."""
    rng = np.random.default_rng(seed)
    s = src.astype(np.int64)
    d = dst.astype(np.int64)
    m = len(s)
    if m:
        flip = rng.random(m) < reverse_frac
        s, d = np.where(flip, d, s), np.where(flip, s, d)
        k = int(dup_frac * m)
        if k:
            pick = rng.integers(0, m, k)
            s = np.concatenate([s, d[pick]])
            d = np.concatenate([d, s[pick]])
    if n > 0 and loops:
        lv = rng.integers(0, n, loops)
        s = np.concatenate([s, lv])
        d = np.concatenate([d, lv])
    order = rng.permutation(len(s))
    return s[order].astype(np.int32), d[order].astype(np.int32), n


def relabel(src, dst, n, seed: int = 0):
    """Apply a random vertex permutation; returns (src, dst, n, perm)."""
    perm = np.random.default_rng(seed).permutation(n).astype(np.int64)
    return perm[src].astype(np.int32), perm[dst].astype(np.int32), n, perm
