"""Edge-file ingestion (gc_read_edges, host code): the TSV triples and Matrix
Market files the paper's data come in (Sec. II), read into 0-based pairs.
Runs on the CPU: no GPU call is made."""
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

gc = pytest.importorskip("paper_1708_06866_amd")


def write(tmp_path, name, text):
    p = os.path.join(tmp_path, name)
    with open(p, "w", newline="") as f:
        f.write(text)
    return p


def write_tsv(path, src, dst):
    """The paper's layout: u <TAB> v <TAB> 1, ids 1..n, one edge per line."""
    a = np.stack([src.astype(np.int64) + 1, dst.astype(np.int64) + 1,
                  np.ones(len(src), np.int64)], 1)
    np.savetxt(path, a, fmt="%d", delimiter="\t")


def test_tsv_layout_and_hygiene(tmp_path):
    p = write(tmp_path, "a.tsv",
              "# comment\n1\t2\t1\n2\t3\t1\n\n% another comment\n3 1 1\r\n  4\t1\n5\t5\t1")
    src, dst, n = gc.gc_read_edges(p)
    assert src.tolist() == [0, 1, 2, 3, 4]
    assert dst.tolist() == [1, 2, 0, 0, 4]
    assert n == 5
    assert src.dtype == np.int32 and dst.dtype == np.int32


def test_mmio_variants(tmp_path):
    body = "%%MatrixMarket matrix coordinate {f} {s}\n% made up\n%\n6 6 4\n1 2{v}\n2 3{v}\n6 1{v}\n4 5{v}\n"
    for field, val in (("pattern", ""), ("integer", " 7"), ("real", " 0.5")):
        for sym in ("general", "symmetric"):
            p = write(tmp_path, "m_%s_%s.mtx" % (field, sym), body.format(f=field, s=sym, v=val))
            for fmt in (gc.GC_FILE_AUTO, gc.GC_FILE_MMIO):
                src, dst, n = gc.gc_read_edges(p, fmt)
                assert n == 6
                assert src.tolist() == [0, 1, 5, 3] and dst.tolist() == [1, 2, 0, 4]


def test_empty_files(tmp_path):
    src, dst, n = gc.gc_read_edges(write(tmp_path, "e.tsv", ""))
    assert len(src) == 0 and n == 0
    src, dst, n = gc.gc_read_edges(write(tmp_path, "c.tsv", "# only a comment\n\n"))
    assert len(src) == 0
    p = write(tmp_path, "e.mtx", "%%MatrixMarket matrix coordinate pattern general\n7 7 0\n")
    src, dst, n = gc.gc_read_edges(p)
    assert len(src) == 0 and n == 7


@pytest.mark.parametrize("text,status", [
    ("1\t0\t1\n", "GC_ERANGE"),                 # ids start at 1
    ("1\tx\t1\n", "GC_EINVAL"),                 # malformed
    ("1\n", "GC_EINVAL"),                       # one field
    ("1\t2a\t1\n", "GC_EINVAL"),                # junk after an id
    ("1\t-2\t1\n", "GC_EINVAL"),                # negative
    ("1\t3000000000\t1\n", "GC_EOVERFLOW"),     # beyond int32
])
def test_tsv_errors(tmp_path, text, status):
    with pytest.raises(gc.GCError) as ei:
        gc.gc_read_edges(write(tmp_path, "bad.tsv", "1\t2\t1\n" + text))
    assert ei.value.status == getattr(gc, status)


@pytest.mark.parametrize("text,status", [
    ("%%MatrixMarket matrix coordinate pattern general\n3 3 2\n1 2\n", "GC_EINVAL"),  # nnz
    ("%%MatrixMarket matrix coordinate pattern general\n3 3 1\n1 4\n", "GC_ERANGE"),  # > n
    ("%%MatrixMarket matrix array real general\n3 3\n1.0\n", "GC_EINVAL"),           # dense
    ("%%MatrixMarket matrix coordinate complex general\n3 3 1\n1 2 1 1\n", "GC_EINVAL"),
    ("%%MatrixMarket matrix coordinate pattern general\n% no size line\n", "GC_EINVAL"),
    ("%%MatrixMarket matrix coordinate pattern general\n3000000000 3 0\n", "GC_EOVERFLOW"),
])
def test_mmio_errors(tmp_path, text, status):
    with pytest.raises(gc.GCError) as ei:
        gc.gc_read_edges(write(tmp_path, "bad.mtx", text))
    assert ei.value.status == getattr(gc, status)


def test_mmio_format_requires_banner(tmp_path):
    with pytest.raises(gc.GCError):
        gc.gc_read_edges(write(tmp_path, "x.tsv", "1\t2\t1\n"), gc.GC_FILE_MMIO)


def test_missing_file(tmp_path):
    with pytest.raises(gc.GCError) as ei:
        gc.gc_read_edges(os.path.join(tmp_path, "nope.tsv"))
    assert ei.value.status == gc.GC_EINVAL


def test_round_trip_large_file_parallel(tmp_path):
    """A file well above the single-thread threshold (many chunks) reads back
    exactly, in file order."""
    src, dst, n = gg.rmat(16, 16, seed=9)
    p = os.path.join(tmp_path, "r16.tsv")
    write_tsv(p, src, dst)
    assert os.path.getsize(p) > 4 << 20
    s2, d2, n2 = gc.gc_read_edges(p)
    assert np.array_equal(s2, src) and np.array_equal(d2, dst)
    assert n2 == int(max(src.max(), dst.max())) + 1


def test_table2_king_graph_from_tsv(tmp_path):
    """Table II, n = 8 written in the paper's TSV layout: read back, the oracle
    finds its 65,536 vertices' 260,610 edges and 4(M-1)^2 triangles."""
    src, dst, n = gg.king(256)
    p = os.path.join(tmp_path, "king256.tsv")
    write_tsv(p, src, dst)
    s2, d2, n2 = gc.gc_read_edges(p)
    assert n2 == n == 65536
    u, v = oracle.normalise(s2, d2, n2)
    assert len(u) == 260610
    assert oracle.triangle_count(n2, u, v) == 4 * 255 ** 2


_NO_THREAD_CHILD = r"""
import ctypes, resource, sys
import numpy as np
import paper_1708_06866_amd as gc

path = sys.argv[1]
L = gc.lib()
src0, dst0, n0 = gc.gc_read_edges(path)        # unconstrained read
src = np.zeros_like(src0)
dst = np.zeros_like(dst0)
n_pairs, n_vertices = ctypes.c_int64(0), ctypes.c_int64(0)
vm = [int(l.split()[1]) * 1024 for l in open("/proc/self/status") if l.startswith("VmSize:")][0]
soft, hard = resource.getrlimit(resource.RLIMIT_AS)
# room for the file mapping, but not for the worker threads' 8 MiB stacks
resource.setrlimit(resource.RLIMIT_AS, (vm + (12 << 20), hard))
st = L.gc_read_edges(path.encode(), gc.GC_FILE_AUTO, src.ctypes.data_as(ctypes.c_void_p),
                     dst.ctypes.data_as(ctypes.c_void_p), len(src), ctypes.byref(n_pairs),
                     ctypes.byref(n_vertices))
resource.setrlimit(resource.RLIMIT_AS, (soft, hard))
assert st == gc.GC_OK, st
assert n_pairs.value == len(src0) and n_vertices.value == n0
assert np.array_equal(src, src0) and np.array_equal(dst, dst0)
print("ok", len(src0))
"""


def test_reader_survives_threads_that_cannot_start(tmp_path):
    """With no address space left for thread stacks, a multi-chunk read runs
    its chunks on the calling thread and returns every pair (no C++
    exception escapes the C ABI to abort the process)."""
    import subprocess
    import sys
    src, dst, n = gg.rmat(14, 16, seed=4)
    p = os.path.join(tmp_path, "r14.tsv")
    write_tsv(p, src, dst)
    assert os.path.getsize(p) > 2 << 20           # several chunks
    child = os.path.join(tmp_path, "child.py")
    with open(child, "w") as f:
        f.write(_NO_THREAD_CHILD)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, PYTHONPATH=root)
    r = subprocess.run([sys.executable, child, p], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
    assert r.stdout.split() == ["ok", str(len(src))]


def _reference_tsv(text: str):
    """Plain reading of the TSV rules: skip blank and '#'/'%' lines, take the
    first two fields of every other line as 1-based ids."""
    src, dst = [], []
    for line in text.split("\n"):
        f = line.replace("\r", " ").split()
        if not f or f[0][0] in "#%":
            continue
        src.append(int(f[0]) - 1)
        dst.append(int(f[1]) - 1)
    return np.array(src, np.int32), np.array(dst, np.int32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_chunked_read_matches_a_plain_parser(tmp_path, seed):
    """Files a little above the multi-chunk threshold, with comments, blank
    lines, CRLF ends, runs of blanks and long lines falling on chunk cuts,
    read exactly as a line-by-line parser reads them."""
    rng = np.random.default_rng(seed)
    lines, size = [], 0
    while size < (1 << 20) + 300_000:
        r = rng.random()
        if r < 0.05:
            s = "# " + "c" * int(rng.integers(0, 3000))       # long comment
        elif r < 0.08:
            s = "% note"
        elif r < 0.11:
            s = " " * int(rng.integers(0, 4))                  # blank
        else:
            u, v = rng.integers(1, 1 << 20, 2)
            sep = [" ", "\t", "  ", " \t "][int(rng.integers(0, 4))]
            tail = ["", "\t1", " 7", "\t1.5"][int(rng.integers(0, 4))]
            s = " " * int(rng.integers(0, 2)) + "%d%s%d%s" % (u, sep, v, tail)
        end = "\r\n" if rng.random() < 0.3 else "\n"
        lines.append(s + end)
        size += len(s) + len(end)
    if rng.random() < 0.5:
        lines[-1] = lines[-1].rstrip("\r\n")                   # no final newline
    text = "".join(lines)
    p = write(tmp_path, "mixed.tsv", text)
    s_ref, d_ref = _reference_tsv(text)
    s2, d2, n2 = gc.gc_read_edges(p)
    assert np.array_equal(s2, s_ref) and np.array_equal(d2, d_ref)
    assert n2 == int(max(s_ref.max(), d_ref.max())) + 1


def test_bad_line_in_a_later_chunk_is_named(tmp_path):
    """A malformed line far into a multi-chunk file fails the read, and the
    error text quotes that line (not the first chunk's)."""
    good = "".join("%d\t%d\t1\n" % (i % 1000 + 1, (i * 7) % 1000 + 1) for i in range(200_000))
    p = write(tmp_path, "late.tsv", good + "17\tbroken-here\t1\n" + good[:5000])
    assert os.path.getsize(p) > 1 << 20              # above the multi-chunk threshold
    with pytest.raises(gc.GCError) as ei:
        gc.gc_read_edges(p)
    assert ei.value.status == gc.GC_EINVAL
    assert "17\tbroken-here" in str(ei.value)
