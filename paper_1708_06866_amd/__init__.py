"""Python binding of libgc (include/gc.h): exact triangle counting, per-edge
support, k-truss and truss decomposition on an MI355X.

This module only marshals arguments: torch tensors (device memory) become raw
pointers, the current torch stream becomes the ``hipStream_t``, and status
codes become exceptions.  Before any library call it checks what the C ABI
cannot see: caller-supplied output tensors (dtype, layout, device, length
where the C call takes no capacity), equal lengths of host pair arrays, and
ids that fit int32.  Every step of the computation runs in libgc's HIP
kernels; there is no CPU fallback -- if ``libgc.so`` is missing, or no GPU is
visible, the calls raise.

The functions carry the C names::

    g = gc_build_csr(src, dst, n_vertices)          # raw pairs (int32, cuda)
    gc_triangle_count(g)                            # -> int
    gc_edge_support(g)                              # -> int32[m] (cuda)
    gc_ktruss(g, k)                                 # -> (uint8[m] mask, m_k)
    gc_truss_decomposition(g)                       # -> (int32[m] tau, kmax)
    gc_read_edges(path)                             # TSV / Matrix Market file -> pairs

``Graph`` wraps a handle with the same operations as methods.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgc.so")

GC_OK = 0
GC_EINVAL = -1
GC_ERANGE = -2
GC_ECAPACITY = -3
GC_ENOMEM = -4
GC_EDEVICE = -5
GC_EOVERFLOW = -6
GC_INPUT_ONE_BASED = 0x1
GC_FILE_AUTO = 0
GC_FILE_TSV = 1
GC_FILE_MMIO = 2

GC_PENDING = 1

# count strategies: N_BINS degree bins, N_STRATEGIES strategies (include/gc.h)
N_BINS = 5
N_STRATEGIES = 7

_lib = None


class GCRequest(ctypes.Structure):
    _fields_ = [("graph_id", ctypes.c_int32), ("kind", ctypes.c_int32), ("k", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class GCResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("kind", ctypes.c_int32), ("value", ctypes.c_int64),
                ("edges", ctypes.c_int64), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class GCError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__("%s failed: %s (%s)" % (what, _status_str(status), detail))
        self.status = status


def lib():
    """Load libgc.so (after torch, so both share torch's HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgc.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        L.gc_build_csr.argtypes = [P, P, i64, i32, u32, P, ctypes.POINTER(P)]
        L.gc_graph_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.gc_graph_edges.argtypes = [P, P, P, i64, P]
        L.gc_graph_oriented.argtypes = [P, P, P, P, P, i64, i64, P]
        L.gc_triangle_count.argtypes = [P, P, ctypes.POINTER(i64)]
        L.gc_edge_support.argtypes = [P, P, i64, P]
        L.gc_edge_support_noalloc.argtypes = [P, P, i64, P]
        L.gc_ktruss.argtypes = [P, i32, P, i64, P, ctypes.POINTER(i64)]
        L.gc_truss_decomposition.argtypes = [P, P, i64, P, ctypes.POINTER(i32)]
        L.gc_graph_autotune.argtypes = [P, P, P, P]
        L.gc_graph_set_strategy.argtypes = [P, P]
        L.gc_graph_set_tile.argtypes = [P, P]
        L.gc_graph_set_tile.restype = i32
        L.gc_graph_count_config.argtypes = [P, P, P]
        L.gc_graph_count_config.restype = i32
        L.gc_graph_autotune.restype = i32
        L.gc_graph_set_strategy.restype = i32
        L.gc_graph_truss_stats.argtypes = [P, P, i32]
        L.gc_graph_truss_stats.restype = i32
        L.gc_graph_count_times.argtypes = [P, P, i32]
        L.gc_graph_count_times.restype = i32
        L.gc_graph_free.argtypes = [P]
        L.gc_graph_free.restype = None
        L.gc_status_str.argtypes = [i32]
        L.gc_status_str.restype = ctypes.c_char_p
        L.gc_last_error.argtypes = []
        L.gc_last_error.restype = ctypes.c_char_p
        L.gc_batch_build.argtypes = [P, P, P, P, i32, u32, P, ctypes.POINTER(P)]
        L.gc_batch_info.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                    ctypes.POINTER(i64)]
        L.gc_batch_edge_offsets.argtypes = [P, P]
        L.gc_batch_graph.argtypes = [P]
        L.gc_batch_graph.restype = P
        L.gc_batch_triangle_count.argtypes = [P, P, P]
        L.gc_batch_edge_support.argtypes = [P, P, i64, P]
        L.gc_batch_ktruss.argtypes = [P, i32, P, i64, P, P]
        L.gc_batch_autotune.argtypes = [P, P, P, P]
        L.gc_batch_set_strategy.argtypes = [P, P]
        L.gc_batch_free.argtypes = [P]
        L.gc_batch_free.restype = None
        L.gc_server_create.argtypes = [i64, ctypes.POINTER(P)]
        L.gc_server_set_mode.argtypes = [P, i32]
        L.gc_server_add_graph.argtypes = [P, P, P, i64, i32, ctypes.POINTER(i32)]
        L.gc_server_submit.argtypes = [P, ctypes.POINTER(GCRequest), ctypes.POINTER(i64)]
        L.gc_server_poll.argtypes = [P, i64, ctypes.POINTER(GCResult)]
        L.gc_server_wait.argtypes = [P, i64, ctypes.POINTER(GCResult)]
        L.gc_server_stats.argtypes = [P, P]
        L.gc_server_destroy.argtypes = [P]
        L.gc_server_destroy.restype = None
        L.gc_read_edges.argtypes = [ctypes.c_char_p, i32, P, P, i64, ctypes.POINTER(i64),
                                    ctypes.POINTER(i64)]
        L.gc_read_edges.restype = i32
        for name in ("gc_server_create", "gc_server_set_mode", "gc_server_add_graph",
                     "gc_server_submit", "gc_server_poll", "gc_server_wait", "gc_server_stats"):
            getattr(L, name).restype = i32
        for name in ("gc_build_csr", "gc_graph_info", "gc_graph_edges", "gc_graph_oriented",
                     "gc_triangle_count", "gc_edge_support", "gc_edge_support_noalloc",
                     "gc_ktruss",
                     "gc_truss_decomposition", "gc_batch_build", "gc_batch_info",
                     "gc_batch_edge_offsets", "gc_batch_triangle_count",
                     "gc_batch_edge_support", "gc_batch_ktruss", "gc_batch_autotune",
                     "gc_batch_set_strategy"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def _status_str(st: int) -> str:
    try:
        return lib().gc_status_str(st).decode()
    except Exception:  # pragma: no cover
        return str(st)


def _check(st: int, what: str):
    if st != GC_OK:
        raise GCError(st, what, lib().gc_last_error().decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_i32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a cuda tensor" % name)
    if t.dtype != torch.int32:
        raise TypeError("%s must be int32" % name)
    return t.contiguous()


def _dev_out(t, dtype: torch.dtype, need: int, name: str, device: torch.device) -> torch.Tensor:
    """A caller-supplied output that the kernels write in place: a contiguous
    cuda tensor of ``dtype`` with at least ``need`` entries on ``device``.
    Checked before any library call, so a wrong buffer raises here instead
    of reaching a kernel."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, not %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < need:
        raise ValueError("%s holds %d entries, %d needed" % (name, t.numel(), need))
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise TypeError("%s must be a cuda tensor on %s, not on %s" % (name, device, t.device))
    return t


def _host_ids(a, name: str):
    """Host or device integer ids -> int32 tensor; ids that do not fit int32
    raise instead of wrapping."""
    t = torch.as_tensor(a)
    if t.dtype == torch.int32:
        return t
    if t.dtype.is_floating_point or t.dtype.is_complex or t.dtype == torch.bool:
        raise TypeError("%s must hold integer ids, not %s" % (name, t.dtype))
    if t.numel() and (int(t.min()) < -(1 << 31) or int(t.max()) >= (1 << 31)):
        raise ValueError("%s holds ids outside int32" % name)
    return t.to(torch.int32)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Graph:
    """Owning wrapper of a gc_graph* handle."""

    def __init__(self, handle: ctypes.c_void_p, device: torch.device):
        self._h = handle
        self.device = device

    @property
    def handle(self):
        if not self._h:
            raise ValueError("graph handle already freed")
        return self._h

    def free(self):
        if self._h:
            lib().gc_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # sizes ---------------------------------------------------------------
    def info(self):
        n, m, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gc_graph_info(self.handle, ctypes.byref(n), ctypes.byref(m),
                                   ctypes.byref(b)), "gc_graph_info")
        return int(n.value), int(m.value), int(b.value)

    @property
    def n(self) -> int:
        return self.info()[0]

    @property
    def m(self) -> int:
        return self.info()[1]

    # outputs -------------------------------------------------------------
    def edges(self, stream=None):
        return gc_graph_edges(self, stream)

    def oriented(self, stream=None):
        return gc_graph_oriented(self, stream)

    def triangle_count(self, stream=None) -> int:
        return gc_triangle_count(self, stream)

    def edge_support(self, out=None, stream=None) -> torch.Tensor:
        return gc_edge_support(self, out, stream)

    def edge_support_noalloc(self, out, stream=None) -> torch.Tensor:
        return gc_edge_support_noalloc(self, out, stream)

    def ktruss(self, k: int, out=None, stream=None):
        return gc_ktruss(self, k, out, stream)

    def truss_decomposition(self, out=None, stream=None):
        return gc_truss_decomposition(self, out, stream)

    def autotune(self, stream=None):
        """Per-bin count strategies chosen by timing: (strategy[5], ms[5, 7])."""
        import numpy as np
        st = np.zeros(5, dtype=np.int32)
        ms = np.zeros(N_BINS * N_STRATEGIES, dtype=np.float32)
        _check(lib().gc_graph_autotune(self.handle, _stream(stream),
                                       ctypes.c_void_p(st.ctypes.data),
                                       ctypes.c_void_p(ms.ctypes.data)), "gc_graph_autotune")
        return st, ms.reshape(N_BINS, N_STRATEGIES)

    def count_times(self):
        """Kernel time (ms) of each degree bin's count launch in the last
        triangle_count() on this handle (HIP events; -1 before one)."""
        import numpy as np
        v = np.zeros(N_BINS, dtype=np.float32)
        _check(lib().gc_graph_count_times(self.handle, ctypes.c_void_p(v.ctypes.data), N_BINS),
               "gc_graph_count_times")
        return v

    def truss_stats(self) -> dict:
        """Counters of the last truss decomposition on this handle."""
        import numpy as np
        v = np.zeros(41, dtype=np.int64)
        _check(lib().gc_graph_truss_stats(self.handle, ctypes.c_void_p(v.ctypes.data), 41),
               "gc_graph_truss_stats")
        return {"levels": int(v[0]), "rounds": int(v[1]), "removed": int(v[2]),
                "largest_round": int(v[3]), "compactions": int(v[4]),
                "rounds_by_log2_size": [int(x) for x in v[5:37]],
                "candidates": int(v[37]), "searches": int(v[38]),
                "triangles_found": int(v[39]), "triangles_destroyed": int(v[40])}

    def set_strategy(self, strategy):
        import numpy as np
        st = np.ascontiguousarray(strategy, dtype=np.int32)
        _check(lib().gc_graph_set_strategy(self.handle, ctypes.c_void_p(st.ctypes.data)),
               "gc_graph_set_strategy")

    def set_tile(self, tile):
        """Per-bin count tiles (in-edges per work unit: 32, 64 or 128)."""
        import numpy as np
        t = np.ascontiguousarray(tile, dtype=np.int32)
        if t.shape != (N_BINS,):
            raise ValueError("set_tile: %d tiles needed" % N_BINS)
        _check(lib().gc_graph_set_tile(self.handle, ctypes.c_void_p(t.ctypes.data)),
               "gc_graph_set_tile")

    def count_config(self):
        """(strategy[5], tile[5]) the count uses on this handle."""
        import numpy as np
        st = np.zeros(N_BINS, dtype=np.int32)
        t = np.zeros(N_BINS, dtype=np.int32)
        _check(lib().gc_graph_count_config(self.handle, ctypes.c_void_p(st.ctypes.data),
                                           ctypes.c_void_p(t.ctypes.data)),
               "gc_graph_count_config")
        return st, t


def _handle(g):
    return g.handle if isinstance(g, Graph) else g


def gc_build_csr(src: torch.Tensor, dst: torch.Tensor, n_vertices: int, flags: int = 0,
                 stream=None) -> Graph:
    src = _dev_i32(src, "src")
    dst = _dev_i32(dst, "dst")
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in length")
    h = ctypes.c_void_p()
    st = lib().gc_build_csr(_ptr(src), _ptr(dst), src.numel(), int(n_vertices), int(flags),
                            _stream(stream), ctypes.byref(h))
    _check(st, "gc_build_csr")
    return Graph(h, src.device)


def gc_graph_info(g):
    return g.info()


def gc_graph_edges(g: Graph, stream=None):
    _, m, _ = g.info()
    u = torch.empty(max(m, 1), dtype=torch.int32, device=g.device)
    v = torch.empty(max(m, 1), dtype=torch.int32, device=g.device)
    _check(lib().gc_graph_edges(g.handle, _ptr(u), _ptr(v), m, _stream(stream)), "gc_graph_edges")
    return u[:m], v[:m]


def gc_graph_oriented(g: Graph, stream=None):
    n, m, _ = g.info()
    rank = torch.empty(max(n, 1), dtype=torch.int32, device=g.device)
    row_ptr = torch.empty(n + 1, dtype=torch.int32, device=g.device)
    col = torch.empty(max(m, 1), dtype=torch.int32, device=g.device)
    eid = torch.empty(max(m, 1), dtype=torch.int32, device=g.device)
    _check(lib().gc_graph_oriented(g.handle, _ptr(rank), _ptr(row_ptr), _ptr(col), _ptr(eid),
                                   n + 1, m, _stream(stream)), "gc_graph_oriented")
    return rank[:n], row_ptr, col[:m], eid[:m]


def gc_triangle_count(g: Graph, stream=None) -> int:
    t = ctypes.c_int64()
    _check(lib().gc_triangle_count(g.handle, _stream(stream), ctypes.byref(t)),
           "gc_triangle_count")
    return int(t.value)


def gc_edge_support(g: Graph, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if out is not None:
        _dev_out(out, torch.int32, 0, "out", g.device)
    _, m, _ = g.info()
    if out is None:
        out = torch.empty(max(m, 1), dtype=torch.int32, device=g.device)
    _check(lib().gc_edge_support(g.handle, _ptr(out), out.numel(), _stream(stream)),
           "gc_edge_support")
    return out[:m]


def gc_edge_support_noalloc(g: Graph, out: torch.Tensor, stream=None) -> torch.Tensor:
    """gc_edge_support into a caller-supplied int32 tensor, with no allocation
    by the library (nor here: `out` is required)."""
    _dev_out(out, torch.int32, 0, "out", g.device)
    _check(lib().gc_edge_support_noalloc(g.handle, _ptr(out), out.numel(), _stream(stream)),
           "gc_edge_support_noalloc")
    return out[:g.m]


def gc_ktruss(g: Graph, k: int, out: torch.Tensor | None = None, stream=None):
    if out is not None:
        _dev_out(out, torch.uint8, 0, "out", g.device)
    _, m, _ = g.info()
    if out is None:
        out = torch.empty(max(m, 1), dtype=torch.uint8, device=g.device)
    mk = ctypes.c_int64()
    _check(lib().gc_ktruss(g.handle, int(k), _ptr(out), out.numel(), _stream(stream),
                           ctypes.byref(mk)), "gc_ktruss")
    return out[:m], int(mk.value)


def gc_truss_decomposition(g: Graph, out: torch.Tensor | None = None, stream=None):
    if out is not None:
        _dev_out(out, torch.int32, 0, "out", g.device)
    _, m, _ = g.info()
    if out is None:
        out = torch.empty(max(m, 1), dtype=torch.int32, device=g.device)
    kmax = ctypes.c_int32()
    _check(lib().gc_truss_decomposition(g.handle, _ptr(out), out.numel(), _stream(stream),
                                        ctypes.byref(kmax)), "gc_truss_decomposition")
    return out[:m], int(kmax.value)


def build_graph(src, dst, n_vertices: int, device="cuda", one_based: bool = False) -> Graph:
    """Convenience: host or device int32 pairs -> Graph on ``device``."""
    s = _host_ids(src, "src").to(device)
    d = _host_ids(dst, "dst").to(device)
    return gc_build_csr(s, d, n_vertices, GC_INPUT_ONE_BASED if one_based else 0)


# ----------------------------------------------------------------------------
# edge files
# ----------------------------------------------------------------------------
import numpy as _np  # noqa: E402


def gc_read_edges(path: str, fmt: int = GC_FILE_AUTO):
    """Read a TSV or Matrix Market edge file (host): returns (src, dst, n),
    int32 numpy arrays with 0-based ids and the vertex count."""
    L = lib()
    bpath = os.fsencode(path)
    n_pairs = ctypes.c_int64(0)
    n_vertices = ctypes.c_int64(0)
    _check(L.gc_read_edges(bpath, fmt, None, None, 0, ctypes.byref(n_pairs),
                           ctypes.byref(n_vertices)), "gc_read_edges")
    src = _np.empty(n_pairs.value, dtype=_np.int32)
    dst = _np.empty(n_pairs.value, dtype=_np.int32)
    _check(L.gc_read_edges(bpath, fmt, src.ctypes.data_as(ctypes.c_void_p),
                           dst.ctypes.data_as(ctypes.c_void_p), len(src),
                           ctypes.byref(n_pairs), ctypes.byref(n_vertices)), "gc_read_edges")
    return src, dst, int(n_vertices.value)


def read_graph(path: str, fmt: int = GC_FILE_AUTO, device="cuda") -> Graph:
    """Convenience: edge file -> Graph on ``device`` (reading is on the host)."""
    src, dst, n = gc_read_edges(path, fmt)
    return build_graph(src, dst, n, device=device)


# ----------------------------------------------------------------------------
# batches
# ----------------------------------------------------------------------------


class Batch:
    """Owning wrapper of a gc_batch* (many graphs, one device structure)."""

    def __init__(self, handle, device):
        self._h = handle
        self.device = device
        n_graphs, m, _ = self.info()
        self.n_graphs = n_graphs
        off = _np.zeros(n_graphs + 1, dtype=_np.int64)
        _check(lib().gc_batch_edge_offsets(self.handle, ctypes.c_void_p(off.ctypes.data)),
               "gc_batch_edge_offsets")
        self.edge_offsets = off

    @property
    def handle(self):
        if not self._h:
            raise ValueError("batch already freed")
        return self._h

    def free(self):
        if self._h:
            lib().gc_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self):
        g, m, b = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().gc_batch_info(self.handle, ctypes.byref(g), ctypes.byref(m), ctypes.byref(b)),
               "gc_batch_info")
        return int(g.value), int(m.value), int(b.value)

    def graph(self) -> Graph:
        """The union graph (owned by the batch: do not free it)."""
        g = Graph(ctypes.c_void_p(lib().gc_batch_graph(self.handle)), self.device)
        g.free = lambda: None  # the batch owns it
        return g

    def triangle_count(self, out=None, stream=None) -> torch.Tensor:
        # the C call has no capacity argument: out must hold one count per graph
        if out is not None:
            _dev_out(out, torch.int64, self.n_graphs, "out", self.device)
        if out is None:
            out = torch.empty(max(self.n_graphs, 1), dtype=torch.int64, device=self.device)
        _check(lib().gc_batch_triangle_count(self.handle, _ptr(out), _stream(stream)),
               "gc_batch_triangle_count")
        return out[:self.n_graphs]

    def edge_support(self, out=None, stream=None) -> torch.Tensor:
        m = int(self.edge_offsets[-1])
        if out is not None:
            _dev_out(out, torch.int32, 0, "out", self.device)
        if out is None:
            out = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        _check(lib().gc_batch_edge_support(self.handle, _ptr(out), out.numel(), _stream(stream)),
               "gc_batch_edge_support")
        return out[:m]

    def ktruss(self, k: int, stream=None):
        m = int(self.edge_offsets[-1])
        mask = torch.empty(max(m, 1), dtype=torch.uint8, device=self.device)
        mk = torch.empty(max(self.n_graphs, 1), dtype=torch.int64, device=self.device)
        _check(lib().gc_batch_ktruss(self.handle, int(k), _ptr(mask), mask.numel(), _ptr(mk),
                                     _stream(stream)), "gc_batch_ktruss")
        return mask[:m], mk[:self.n_graphs]

    def autotune(self, stream=None):
        st = _np.zeros(N_BINS, dtype=_np.int32)
        ms = _np.zeros(N_BINS * N_STRATEGIES, dtype=_np.float32)
        _check(lib().gc_batch_autotune(self.handle, _stream(stream), ctypes.c_void_p(st.ctypes.data),
                                       ctypes.c_void_p(ms.ctypes.data)), "gc_batch_autotune")
        return st, ms.reshape(N_BINS, N_STRATEGIES)

    def set_strategy(self, strategy):
        st = _np.ascontiguousarray(strategy, dtype=_np.int32)
        _check(lib().gc_batch_set_strategy(self.handle, ctypes.c_void_p(st.ctypes.data)),
               "gc_batch_set_strategy")


def gc_batch_build(src: torch.Tensor, dst: torch.Tensor, pair_offsets, n_vertices,
                   flags: int = 0, stream=None) -> Batch:
    """src/dst: concatenated raw pairs (int32, cuda); pair_offsets: G+1 host
    offsets; n_vertices: G vertex counts."""
    src = _dev_i32(src, "src")
    dst = _dev_i32(dst, "dst")
    off = _np.ascontiguousarray(pair_offsets, dtype=_np.int64)
    nv = _np.ascontiguousarray(n_vertices, dtype=_np.int32)
    G = len(nv)
    if len(off) != G + 1:
        raise ValueError("pair_offsets must have G+1 entries")
    if int(off[-1]) != src.numel() or src.numel() != dst.numel():
        raise ValueError("pair_offsets[-1] must equal the number of pairs")
    h = ctypes.c_void_p()
    _check(lib().gc_batch_build(_ptr(src), _ptr(dst), ctypes.c_void_p(off.ctypes.data),
                                ctypes.c_void_p(nv.ctypes.data), G, int(flags), _stream(stream),
                                ctypes.byref(h)), "gc_batch_build")
    return Batch(h, src.device)


def build_batch(graphs, device="cuda") -> Batch:
    """Convenience: list of host (src, dst, n) -> Batch on ``device``."""
    srcs = [_host_ids(g[0], "src").cpu().numpy().reshape(-1) for g in graphs]
    dsts = [_host_ids(g[1], "dst").cpu().numpy().reshape(-1) for g in graphs]
    off = _np.zeros(len(graphs) + 1, dtype=_np.int64)
    off[1:] = _np.cumsum([len(x) for x in srcs])
    nv = [int(g[2]) for g in graphs]
    s = torch.from_numpy(_np.concatenate(srcs) if srcs else _np.zeros(0, _np.int32)).to(device)
    d = torch.from_numpy(_np.concatenate(dsts) if dsts else _np.zeros(0, _np.int32)).to(device)
    return gc_batch_build(s, d, off, nv)


# ----------------------------------------------------------------------------
# serving
# ----------------------------------------------------------------------------
TRIANGLE_COUNT = 0
KTRUSS_EDGES = 1


class Server:
    """A gc_server: registered graphs, queries with continuous batching."""

    STAT_NAMES = ("completed", "batches", "max_batch", "builds", "evictions", "bytes_charged",
                  "peak_bytes_charged", "deferred", "resident_graphs", "budget",
                  "truss_batches", "max_truss_batch")

    def __init__(self, budget_bytes: int, mode: int = 0):
        torch.cuda.current_device()  # make sure the HIP runtime is up on this device
        h = ctypes.c_void_p()
        _check(lib().gc_server_create(int(budget_bytes), ctypes.byref(h)), "gc_server_create")
        self._h = h
        if mode:
            self.set_mode(mode)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("server already destroyed")
        return self._h

    def close(self):
        if self._h:
            lib().gc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mode(self, mode: int):
        _check(lib().gc_server_set_mode(self.handle, int(mode)), "gc_server_set_mode")

    def add_graph(self, src, dst, n_vertices: int) -> int:
        s = _np.ascontiguousarray(_host_ids(src, "src").cpu().numpy().reshape(-1))
        d = _np.ascontiguousarray(_host_ids(dst, "dst").cpu().numpy().reshape(-1))
        if len(s) != len(d):
            raise ValueError("src and dst differ in length")
        gid = ctypes.c_int32()
        _check(lib().gc_server_add_graph(self.handle, ctypes.c_void_p(s.ctypes.data),
                                         ctypes.c_void_p(d.ctypes.data), len(s), int(n_vertices),
                                         ctypes.byref(gid)), "gc_server_add_graph")
        return int(gid.value)

    def submit(self, graph_id: int, kind: int = TRIANGLE_COUNT, k: int = 0) -> int:
        req = GCRequest(int(graph_id), int(kind), int(k), 0)
        t = ctypes.c_int64()
        _check(lib().gc_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)),
               "gc_server_submit")
        return int(t.value)

    @staticmethod
    def _res(r: GCResult) -> dict:
        return {"status": r.status, "kind": r.kind, "value": r.value, "edges": r.edges,
                "t_submit": r.t_submit, "t_start": r.t_start, "t_done": r.t_done}

    def poll(self, ticket: int):
        r = GCResult()
        st = lib().gc_server_poll(self.handle, int(ticket), ctypes.byref(r))
        if st == GC_PENDING:
            return None
        _check(st, "gc_server_poll")
        return self._res(r)

    def wait(self, ticket: int) -> dict:
        r = GCResult()
        _check(lib().gc_server_wait(self.handle, int(ticket), ctypes.byref(r)), "gc_server_wait")
        return self._res(r)

    def stats(self) -> dict:
        v = _np.zeros(len(self.STAT_NAMES), dtype=_np.int64)
        _check(lib().gc_server_stats(self.handle, ctypes.c_void_p(v.ctypes.data)),
               "gc_server_stats")
        return dict(zip(self.STAT_NAMES, (int(x) for x in v)))
