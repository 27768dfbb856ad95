"""The C ABI library loads and exports every function include/gc.h declares;
host-side argument checks answer without touching a GPU.  CPU only."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gc.h")
LIB = os.path.join(ROOT, "paper_1708_06866_amd", "libgc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1708_06866_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_core_calls():
    names = declared_functions()
    for core in ("gc_build_csr", "gc_triangle_count", "gc_edge_support", "gc_ktruss",
                 "gc_truss_decomposition", "gc_graph_free", "gc_last_error"):
        assert core in names


def test_every_declared_symbol_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    lib.gc_status_str.restype = ctypes.c_char_p
    lib.gc_status_str.argtypes = [ctypes.c_int32]
    for st in range(-6, 1):
        assert lib.gc_status_str(st).decode().startswith("GC_")
    assert b"unknown" in lib.gc_status_str(-99)


def test_host_argument_checks(lib):
    P = ctypes.c_void_p
    lib.gc_build_csr.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, P,
                                 ctypes.POINTER(P)]
    lib.gc_build_csr.restype = ctypes.c_int32
    lib.gc_last_error.restype = ctypes.c_char_p
    out = P(1234)
    # NULL out
    assert lib.gc_build_csr(None, None, 0, 1, 0, None, None) == -1
    # negative pair count; *out is cleared
    assert lib.gc_build_csr(None, None, -1, 1, 0, None, ctypes.byref(out)) == -1
    assert not out.value
    # unknown flag
    assert lib.gc_build_csr(None, None, 0, 1, 0x80, None, ctypes.byref(out)) == -1
    # pairs but NULL arrays
    assert lib.gc_build_csr(None, None, 5, 10, 0, None, ctypes.byref(out)) == -1
    # too many pairs
    assert lib.gc_build_csr(P(8), P(8), 1 << 31, 10, 0, None, ctypes.byref(out)) == -6
    # pairs on an empty vertex set
    assert lib.gc_build_csr(P(8), P(8), 3, 0, 0, None, ctypes.byref(out)) == -2
    assert len(lib.gc_last_error()) > 0
    for fn, args in (("gc_triangle_count", [None, None, None]),
                     ("gc_ktruss", [None, 3, None, 0, None, None]),
                     ("gc_truss_decomposition", [None, None, 0, None, None])):
        f = getattr(lib, fn)
        f.restype = ctypes.c_int32
        assert f(*args) == -1


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1708_06866_amd as gc
    monkeypatch.setattr(gc, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(gc, "_lib", None)
    with pytest.raises(ImportError):
        gc.lib()


def test_null_handles_rejected_on_the_host(lib):
    """Every entry point that takes a handle answers GC_EINVAL for a NULL one
    before any device work; the free calls accept NULL."""
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    calls = (
        ("gc_graph_info", [P, P, P, P], [None, None, None, None]),
        ("gc_graph_edges", [P, P, P, I64, P], [None, None, None, 0, None]),
        ("gc_graph_oriented", [P, P, P, P, P, I64, I64, P], [None] * 5 + [0, 0, None]),
        ("gc_edge_support", [P, P, I64, P], [None, None, 0, None]),
        ("gc_edge_support_noalloc", [P, P, I64, P], [None, None, 0, None]),
        ("gc_graph_autotune", [P, P, P, P], [None, None, None, None]),
        ("gc_graph_set_strategy", [P, P], [None, None]),
        ("gc_graph_set_tile", [P, P], [None, None]),
        ("gc_graph_count_config", [P, P, P], [None, None, None]),
        ("gc_graph_truss_stats", [P, P, I32], [None, None, 0]),
        ("gc_graph_count_times", [P, P, I32], [None, None, 0]),
        ("gc_batch_info", [P, P, P, P], [None, None, None, None]),
        ("gc_batch_edge_offsets", [P, P], [None, None]),
        ("gc_batch_triangle_count", [P, P, P], [None, None, None]),
        ("gc_batch_edge_support", [P, P, I64, P], [None, None, 0, None]),
        ("gc_batch_ktruss", [P, I32, P, I64, P, P], [None, 3, None, 0, None, None]),
        ("gc_batch_set_strategy", [P, P], [None, None]),
        ("gc_server_set_mode", [P, I32], [None, 0]),
        ("gc_server_submit", [P, P, P], [None, None, None]),
        ("gc_server_poll", [P, I64, P], [None, 0, None]),
        ("gc_server_stats", [P, P], [None, None]),
        ("gc_server_create", [I64, P], [0, None]),
        ("gc_read_edges", [P, I32, P, P, I64, P, P], [None, 0, None, None, 0, None, None]),
    )
    for name, argtypes, args in calls:
        f = getattr(lib, name)
        f.argtypes = argtypes
        f.restype = ctypes.c_int32
        assert f(*args) == -1, name
    for name in ("gc_graph_free", "gc_batch_free", "gc_server_destroy"):
        f = getattr(lib, name)
        f.argtypes = [P]
        f.restype = None
        f(None)
    lib.gc_batch_graph.argtypes = [P]
    lib.gc_batch_graph.restype = P
    assert lib.gc_batch_graph(None) is None


@pytest.fixture
def no_library(monkeypatch):
    """The binding with its library replaced by a tripwire: any call into
    libgc fails the test, so a check that passes here ran on the host first."""
    import paper_1708_06866_amd as gc

    def tripwire():
        raise AssertionError("the library was called")
    monkeypatch.setattr(gc, "lib", tripwire)
    return gc


def test_output_buffers_checked_before_any_library_call(no_library):
    """Caller-supplied outputs are written in place by the kernels: wrong
    dtype, layout, length or device is refused by the binding."""
    import torch
    gc = no_library

    class NoGraph(gc.Graph):
        def info(self):
            raise AssertionError("the handle was queried")
    g = NoGraph(ctypes.c_void_p(None), torch.device("cuda", 0))
    cases = (
        (gc.gc_edge_support, torch.int32), (gc.gc_truss_decomposition, torch.int32),
        (gc.gc_edge_support_noalloc, torch.int32),
        (lambda g_, out: gc.gc_ktruss(g_, 3, out), torch.uint8))
    for call, dtype in cases:
        other = torch.int64 if dtype != torch.int64 else torch.int32
        with pytest.raises(TypeError):
            call(g, [0] * 8)                                      # not a tensor
        with pytest.raises(TypeError):
            call(g, torch.zeros(8, dtype=other))                  # wrong dtype
        with pytest.raises(ValueError):
            call(g, torch.zeros(8, 2, dtype=dtype)[:, 0])         # strided view
        with pytest.raises(TypeError):
            call(g, torch.zeros(8, dtype=dtype))                  # host memory

    b = gc.Batch.__new__(gc.Batch)
    b._h, b.device, b.n_graphs = ctypes.c_void_p(None), torch.device("cuda", 0), 5
    b.edge_offsets = np.zeros(6, np.int64)
    with pytest.raises(ValueError):
        b.triangle_count(out=torch.zeros(4, dtype=torch.int64))   # one short
    with pytest.raises(TypeError):
        b.triangle_count(out=torch.zeros(5, dtype=torch.int64))   # host memory
    with pytest.raises(TypeError):
        b.edge_support(out=torch.zeros(5, dtype=torch.int64))     # wrong dtype


def test_host_inputs_checked_before_any_library_call(no_library):
    """Host pair arrays: unequal lengths and ids beyond int32 are refused
    instead of being read past the end or wrapped."""
    import torch
    gc = no_library
    srv = gc.Server.__new__(gc.Server)
    srv._h = ctypes.c_void_p(None)
    with pytest.raises(ValueError):
        srv.add_graph(np.array([0, 1, 2], np.int32), np.array([1, 2], np.int32), 3)
    with pytest.raises(ValueError):
        srv.add_graph(np.array([0, 1 << 31], np.int64), np.array([1, 2], np.int64), 3)
    with pytest.raises(TypeError):
        srv.add_graph(np.array([0.0, 1.0]), np.array([1.0, 2.0]), 3)
    with pytest.raises(ValueError):
        gc.build_graph(np.array([-(1 << 31) - 1], np.int64), np.array([0], np.int64), 1,
                       device="cpu")
    # in-range ids of any integer type arrive as int32, unchanged
    t = gc._host_ids(np.array([0, 5, (1 << 31) - 1], np.int64), "src")
    assert t.dtype == torch.int32 and t.tolist() == [0, 5, (1 << 31) - 1]
    a = np.array([3, 1], np.int32)
    assert np.shares_memory(gc._host_ids(a, "src").numpy(), a)


C_CONSUMER = r"""
#include <stdio.h>
#include <string.h>
#include "gc.h"

int main(int argc, char **argv) {
  /* host-only calls: no GPU is touched */
  if (argc != 2) return 4;
  int64_t n_pairs = 0, n_vertices = 0;
  gc_status st = gc_read_edges(argv[1], GC_FILE_AUTO, NULL, NULL, 0, &n_pairs, &n_vertices);
  if (st != GC_OK) { printf("size query failed: %s\n", gc_last_error()); return 1; }
  int32_t src[8], dst[8];
  st = gc_read_edges(argv[1], GC_FILE_TSV, src, dst, 8, &n_pairs, &n_vertices);
  if (st != GC_OK || n_pairs != 3 || n_vertices != 4) return 2;
  printf("pairs %lld n %lld first %d-%d\n", (long long)n_pairs, (long long)n_vertices,
         src[0], dst[0]);
  gc_graph *g = (gc_graph *)1;
  st = gc_build_csr(NULL, NULL, 5, 4, 0, NULL, &g);   /* NULL pairs with n_pairs > 0 */
  printf("build %d %s g=%p\n", (int)st, gc_status_str(st), (void *)g);
  printf("error '%s'\n", gc_last_error());
  gc_graph_free(NULL);
  return st == GC_EINVAL && g == NULL && strlen(gc_last_error()) > 0 ? 0 : 3;
}
"""


def test_header_is_plain_c_and_links(tmp_path):
    """include/gc.h compiles as C99 with warnings as errors, and a C program
    linked against libgc.so calls its host-only entry points."""
    import subprocess
    if not os.path.exists(LIB):
        from paper_1708_06866_amd import build
        build.build()
    c = tmp_path / "consumer.c"
    c.write_text(C_CONSUMER)
    exe = tmp_path / "consumer"
    libdir = os.path.dirname(LIB)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                           "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe),
                           LIB, "-Wl,-rpath," + libdir])
    tsv = tmp_path / "e.tsv"
    tsv.write_text("1\t2\t1\n2\t3\t1\n4\t1\t1\n")
    r = subprocess.run([str(exe), str(tsv)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert "pairs 3 n 4 first 0-1" in r.stdout
    assert "build -1 GC_EINVAL" in r.stdout and "g=(nil)" in r.stdout


def test_every_declaration_is_documented():
    """Each function of include/gc.h comes right after a comment of its own
    (meaning, layout, ownership, errors)."""
    text = open(HEADER).read()
    undocumented = []
    for name in declared_functions():
        decl = re.search(r"^[A-Za-z_][\w \*]*\b%s\s*\(" % name, text, re.M)
        assert decl is not None, name
        if not text[:decl.start()].rstrip().endswith("*/"):
            undocumented.append(name)
    assert not undocumented, undocumented
