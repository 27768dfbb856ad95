"""bench.py's host-side accounting, on the CPU: the algorithmic byte counts
behind the roofline figure, checked against brute-force definitions on small
graphs, and the one-GPU contract of the command line."""
import itertools
import os
import subprocess
import sys

import numpy as np

import graphgen as gg
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def oriented(n, u, v):
    """Degree-ordered orientation, rank = position in (deg, id) order."""
    deg = np.bincount(u, minlength=n) + np.bincount(v, minlength=n)
    order = np.lexsort((np.arange(n), deg))
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    a = np.minimum(rank[u], rank[v])
    b = np.maximum(rank[u], rank[v])
    o = np.lexsort((b, a))
    a, b = a[o], b[o]
    row_ptr = np.concatenate([[0], np.cumsum(np.bincount(a, minlength=n))]).astype(np.int32)
    return row_ptr, b.astype(np.int32)


def brute(n, row_ptr, col, chunk, limits, stage_grid=None):
    out = {a: list(col[row_ptr[a]:row_ptr[a + 1]]) for a in range(n)}
    dout = {a: len(out[a]) for a in range(n)}
    din = {x: 0 for x in range(n)}
    for a in range(n):
        for b in out[a]:
            din[b] += 1
    s_src = sum(d * d for d in dout.values())
    s_dst = sum(dout[b] for a in range(n) for b in out[a])
    # tail elements streamed: for every in-edge a -> b whose head has out-edges,
    # the entries of N+(a) after b
    probes = sum(1 for a in range(n) for i, b in enumerate(out[a]) if dout[b] > 0
                 for _ in out[a][i + 1:])
    in_edges = sum(1 for a in range(n) for b in out[a] if dout[b] > 0)
    m = len(col)
    # the same bytes by the bin of the middle vertex b (limits inclusive)
    def bin_of(d):
        return sum(1 for lim in limits if d > lim)

    def ch(b):  # the unit size of b's bin
        return chunk[bin_of(dout[b])] if isinstance(chunk, (list, tuple)) else chunk
    units = sum(-(-din[b] // ch(b)) for b in range(n) if dout[b] > 0 and din[b] > 0)
    # times N+(b) is staged: once per unit, or, where a bin's blocks take
    # contiguous stretches of its units (listed vertex by vertex in rank
    # order), once per block holding a unit of b
    stagings = {b: -(-din[b] // ch(b)) for b in range(n) if dout[b] > 0 and din[b] > 0}
    for bb, grid in enumerate(stage_grid or []):
        if grid is None:
            continue
        unit_vertex = [b for b in range(n) if b in stagings and bin_of(dout[b]) == bb
                       for _ in range(-(-din[b] // ch(b)))]
        if not unit_vertex:
            continue
        g = min(grid, len(unit_vertex))
        per = -(-len(unit_vertex) // g)
        blocks = {}
        for i, b in enumerate(unit_vertex):
            blocks.setdefault(b, set()).add(i // per)
        for b, bl in blocks.items():
            stagings[b] = len(bl)
    staged = sum(stagings[b] * dout[b] for b in stagings)
    by_bin = [0] * (len(limits) + 1)
    for a in range(n):
        for i, b in enumerate(out[a]):
            if dout[b] > 0:
                by_bin[bin_of(dout[b])] += 8 + 4 * len(out[a][i + 1:])
    for b in range(n):
        if dout[b] > 0 and din[b] > 0:
            c = -(-din[b] // ch(b))
            by_bin[bin_of(dout[b])] += 24 * c + 4 * stagings[b] * dout[b]
    return {"S_src": s_src, "S_dst": s_dst, "probes": probes, "in_edges": in_edges,
            "units": units, "staged": staged, "bytes_by_bin": by_bin,
            "B_model_min": min(16 * n + 20 * m + 4 * s_dst, 16 * n + 24 * m + 4 * s_src),
            "bytes": 4 * probes + 8 * in_edges + 4 * staged + 24 * units}


def test_algorithmic_bytes_match_brute_force():
    for (src, dst, n), chunk in ((gg.rmat(8, 16, seed=3), 128), (gg.rmat(9, 8, seed=4), 4),
                                 (gg.complete(40), 8), (gg.king(12), 128), (gg.star(50), 16),
                                 (gg.rmat(9, 16, seed=5), [4, 8, 2, 16, 32]),
                                 (gg.complete(40), [3, 5, 7, 2, 1])):
        u, v = oracle.normalise(src, dst, n)
        row_ptr, col = oriented(n, u, v)
        for limits in (bench.COUNT_BIN_LIMITS, (2, 5, 9, 20)):
            for grid in (None, [None, None, 3, 1, None], [5, 2, 7, 4, 100]):
                got = bench.algorithmic_bytes(row_ptr, col, chunk=chunk, bin_limits=limits,
                                              stage_grid=grid)
                want = brute(n, row_ptr, col, chunk, limits, grid)
                for k, w in want.items():
                    assert got[k] == w, (k, grid, got[k], w)
                assert sum(got["bytes_by_bin"]) == got["bytes"]


def test_stage_grid_matches_the_kernel_source():
    """count_stage_grid's blocks per CU and stretch rule are the ones the
    count kernels launch with (read from gc_count.hip)."""
    import re
    src = open(os.path.join(ROOT, "paper_1708_06866_amd", "csrc", "gc_count.hip")).read()
    m = re.search(r"constexpr int tc_lds_per_cu\(int bytes\) \{.*?return (.*?);", src, re.S)
    assert m, "tc_lds_per_cu not found"
    steps = [(int(x), int(y)) for x, y in re.findall(r"bytes <= (\d+) \? (\d+)", m.group(1))]
    last = int(re.search(r": (\d+)\s*$", m.group(1)).group(1))

    def per_cu(nbytes):  # the chain bytes <= x1 ? y1 : bytes <= x2 ? y2 : ... : last
        for lim, val in steps:
            if nbytes <= lim:
                return val
        return last
    assert len(steps) >= 3
    c = re.search(r"constexpr bool tc_lds_contig\(int bytes\) \{ return bytes >= (\d+); \}", src)
    assert c, "tc_lds_contig not found"
    contig_min = int(c.group(1))
    for b in range(4):
        for st in (0, 1, 3, 4):
            slots = (1 << (6, 9, 12, 14)[b]) if st in (0, 1) else (4 << (4, 7, 10, 12)[b])
            tbytes = 4 * slots * (2 if st in (1, 4) else 1)
            want = 256 * per_cu(tbytes) if tbytes >= contig_min else None
            assert bench.count_stage_grid(b, st) == want, (b, st, tbytes)


def test_stage_grid_mirrors_the_launch_configuration():
    """Bins 2 and 3 with the LDS-table strategies take contiguous stretches
    (tables of 16 KB and up), bins 0 and 1 and the search and group
    strategies do not."""
    assert bench.count_stage_grid(2, 3) == 256 * 512 and bench.count_stage_grid(2, 0) == 256 * 512
    assert bench.count_stage_grid(2, 4) == 256 * 64 and bench.count_stage_grid(3, 1) == 256 * 16
    assert bench.count_stage_grid(3, 0) == 256 * 32
    for b, st in ((0, 0), (1, 3), (1, 4), (2, 2), (0, 5), (1, 6), (4, 2)):
        assert bench.count_stage_grid(b, st) is None, (b, st)


def test_tail_probes_count_the_wedges_once():
    """Every wedge a -> b, a -> c with b < c (both out of a) is one streamed
    element when b has out-edges: on K_n that is C(n, 3) minus the wedges
    whose middle is the last vertex."""
    n = 30
    u, v = oracle.normalise(*gg.complete(n)[:2], n)
    row_ptr, col = oriented(n, u, v)
    got = bench.algorithmic_bytes(row_ptr, col)
    wedges = sum(1 for _ in itertools.combinations(range(n), 3))
    assert got["probes"] == wedges  # every middle b < c has an out-edge to c


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_count_kernel_names_follow_the_dispatch_table():
    """The roofline names the kernel a degree bin runs under its strategy, as
    the library's dispatch does (include/gc.h lists the strategies)."""
    k = bench.count_kernel_name
    assert k(2, 3) == "gc::k_tc_lds<gc::BucketTable<10> >"
    assert k(1, 4) == "gc::k_tc_lds<gc::BucketTable<8> >"
    assert k(0, 5) == "gc::k_tc_group<6, 16>" and k(1, 5) == "gc::k_tc_group<9, 64>"
    assert k(2, 0) == "gc::k_tc_lds<gc::LinTable<12> >"
    assert k(3, 1) == "gc::k_tc_lds<gc::LinTable<15> >"
    assert k(4, 2) == "gc::k_tc_search" and k(2, 2) == "gc::k_tc_search"
