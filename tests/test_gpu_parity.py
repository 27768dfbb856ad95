"""GPU parity: libgc (through its C ABI) against the CPU oracle, bit-exact.

Every input is seeded and synthetic.  Small and medium graphs are checked
against the oracle run in the test; the larger seeded workloads against the
oracle digests in tests/golden/digests.json (written by make_digests.py from
oracle/ alone).  All results are integers: tolerance 0.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1708_06866_amd as gc  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "digests.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def check_all(src, dst, n, label, ks=None, decomposition=True, one_based=False):
    """Build on the GPU and compare edges, T, support, k-truss and truss numbers
    with the oracle."""
    say("case", label, "pairs", len(src), "n", n)
    g = gc.build_graph(src, dst, n, one_based=one_based)
    u, v = oracle.normalise(src, dst, n, one_based=one_based)
    gu, gv = g.edges()
    assert np.array_equal(gu.cpu().numpy(), u), label
    assert np.array_equal(gv.cpu().numpy(), v), label
    assert g.m == len(u)
    T = g.triangle_count()
    assert T == oracle.triangle_count(n, u, v), label
    sup = g.edge_support().cpu().numpy()
    sup_ref = oracle.support(n, u, v, "listing")
    assert np.array_equal(sup, sup_ref), label
    assert int(sup.astype(np.int64).sum()) == 3 * T
    if decomposition:
        tau, kmax = g.truss_decomposition()
        tau_ref, kmax_ref = oracle.truss_decomposition(n, u, v, "peel")
        assert kmax == kmax_ref, (label, kmax, kmax_ref)
        assert np.array_equal(tau.cpu().numpy(), tau_ref), label
        if ks is None:
            ks = sorted(set([2, 3, 4, kmax, kmax + 1]) - {0, 1})
        for k in ks:
            mask, mk = g.ktruss(k)
            ref = (tau_ref >= k).astype(np.uint8) if k >= 2 else None
            assert np.array_equal(mask.cpu().numpy(), ref), (label, k)
            assert mk == int(ref.sum())
    g.free()
    return T


# ----------------------------------------------------------------------------
# closed forms and the paper's examples
# ----------------------------------------------------------------------------

CLOSED = {
    "diamond_fig1": gg.diamond(),
    "K1": gg.complete(1), "K2": gg.complete(2), "K3": gg.complete(3), "K5": gg.complete(5),
    "K40": gg.complete(40),
    "tripartite_2_3_5": gg.complete_tripartite(2, 3, 5),
    "tripartite_6_7_9": gg.complete_tripartite(6, 7, 9),
    "king_2": gg.king(2), "king_16": gg.king(16), "king_64": gg.king(64),
    "wheel_9": gg.wheel(9), "windmill_50": gg.windmill(50), "book_7": gg.book(7),
    "star_300": gg.star(300), "path_50": gg.path(50), "cycle_17": gg.cycle(17),
    "tree_500": gg.random_tree(500, seed=3), "bipartite_20_30": gg.complete_bipartite(20, 30),
    "union": gg.disjoint_union(gg.complete(12), gg.king(8), gg.wheel(6), gg.book(4)),
}


@pytest.mark.parametrize("name", sorted(CLOSED))
def test_closed_forms(name):
    src, dst, n = CLOSED[name]
    check_all(src, dst, n, name)


def test_table2_king_256_closed_form():
    """Table II, n = 8: 65,536 vertices, 260,610 edges, 4(M-1)^2 triangles
    (the printed column is twice that); the whole graph is a 4-truss."""
    src, dst, n = gg.king(256)
    g = gc.build_graph(src, dst, n)
    assert g.m == 260610
    assert g.triangle_count() == 4 * 255 ** 2 == 520200 // 2
    tau, kmax = g.truss_decomposition()
    assert kmax == 4 and bool((tau == 4).all())
    g.free()


# ----------------------------------------------------------------------------
# R-MAT scale 10 (the CPU-fast configuration), seeds 1..8
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(1, 9))
def test_rmat_scale10(seed):
    src, dst, n = gg.rmat(10, 16, seed=seed)
    check_all(src, dst, n, "rmat10 seed %d" % seed, ks=list(range(2, 40)))


def test_rmat_presentation_invariance():
    src, dst, n = gg.rmat(11, 16, seed=5)
    s2, d2, _ = gg.scramble(src, dst, n, seed=6)
    T1 = check_all(src, dst, n, "rmat11")
    T2 = check_all(s2, d2, n, "rmat11 scrambled")
    s3, d3, _, _ = gg.relabel(src, dst, n, seed=7)
    T3 = check_all(s3, d3, n, "rmat11 relabelled")
    T4 = check_all(src + 1, dst + 1, n, "rmat11 one-based", one_based=True)
    assert T1 == T2 == T3 == T4


@pytest.mark.parametrize("scale", [12, 14, 16])
def test_rmat_medium(scale):
    src, dst, n = gg.rmat(scale, 16, seed=1)
    check_all(src, dst, n, "rmat%d" % scale, ks=[3, 4, 5, 6])


def test_er_and_rgg():
    check_all(*gg.er(1 << 14, 16 << 14, seed=2), "er14")
    check_all(*gg.rgg(1 << 13, 20.0, seed=3), "rgg13")


def test_edge_files_to_gpu(tmp_path):
    """The paper's input formats (Sec. II) end to end: the same R-MAT graph as
    TSV triples (both directions, duplicates, 1-based) and as a symmetric
    Matrix Market file (each edge once) gives, on the GPU, the oracle's
    results on the generated pairs."""
    src, dst, n = gg.rmat(12, 16, seed=11)
    u, v = oracle.normalise(src, dst, n)
    T = oracle.triangle_count(n, u, v)
    sup = oracle.support(n, u, v, "listing")
    tau_ref, kmax_ref = oracle.truss_decomposition(n, u, v, "peel")
    tsv = str(tmp_path / "g.tsv")
    np.savetxt(tsv, np.stack([src.astype(np.int64) + 1, dst.astype(np.int64) + 1,
                              np.ones(len(src), np.int64)], 1), fmt="%d", delimiter="\t")
    mtx = str(tmp_path / "g.mtx")
    with open(mtx, "w") as f:
        f.write("%%%%MatrixMarket matrix coordinate pattern symmetric\n%%\n%d %d %d\n" % (n, n, len(u)))
        np.savetxt(f, np.stack([v.astype(np.int64) + 1, u.astype(np.int64) + 1], 1), fmt="%d")
    for path in (tsv, mtx):
        say("case edge file", os.path.basename(path))
        s2, d2, n2 = gc.gc_read_edges(path)
        g = gc.build_graph(s2, d2, n2)
        gu, gv = g.edges()
        assert np.array_equal(gu.cpu().numpy(), u) and np.array_equal(gv.cpu().numpy(), v)
        assert g.triangle_count() == T
        assert np.array_equal(g.edge_support().cpu().numpy(), sup)
        tau, kmax = g.truss_decomposition()
        assert kmax == kmax_ref and np.array_equal(tau.cpu().numpy(), tau_ref)
        g.free()


# ----------------------------------------------------------------------------
# degree-bin boundaries, long in-lists, skew
# ----------------------------------------------------------------------------

def _complete_checks(nk):
    src, dst, n = gg.complete(nk)
    say("case complete", nk)
    g = gc.build_graph(src, dst, n)
    assert g.m == nk * (nk - 1) // 2
    assert g.triangle_count() == nk * (nk - 1) * (nk - 2) // 6
    sup = g.edge_support()
    assert bool((sup == nk - 2).all())
    mask, mk = g.ktruss(nk)
    assert mk == g.m
    mask, mk = g.ktruss(nk + 1)
    assert mk == 0
    tau, kmax = g.truss_decomposition()
    assert kmax == nk and bool((tau == nk).all())
    g.free()


@pytest.mark.parametrize("nk", [33, 34, 257, 258, 2049, 2050, 4098])
def test_complete_graph_bins(nk):
    """K_n has out-degrees 0..n-1 in any orientation, so it reaches every bin
    up to n-1, including the edges of each bin's limit."""
    _complete_checks(nk)


def test_complete_graph_global_search_bin():
    """Out-lists longer than the largest LDS table (binary search in HBM)."""
    _complete_checks(8200)


@pytest.mark.parametrize("p", [127, 128, 129, 5000])
def test_book_long_in_lists(p):
    """Hub vertices with in-lists around and far above one work unit."""
    src, dst, n = gg.book(p)
    check_all(src, dst, n, "book %d" % p)


def test_star_of_cliques_skew():
    parts = [gg.complete(30)] * 20 + [gg.star(3000)]
    src, dst, n = gg.disjoint_union(*parts)
    # join every clique's vertex 0 to the star centre (heavy hub)
    extra_s = np.arange(20, dtype=np.int32) * 30
    extra_d = np.full(20, 20 * 30, dtype=np.int32)
    check_all(np.concatenate([src, extra_s]), np.concatenate([dst, extra_d]), n, "skew")


# ----------------------------------------------------------------------------
# empty and degenerate inputs, errors
# ----------------------------------------------------------------------------

def test_empty_inputs():
    e = np.zeros(0, np.int32)
    for n in (0, 1, 10):
        g = gc.build_graph(e, e, n)
        assert g.m == 0 and g.triangle_count() == 0
        assert g.edge_support().numel() == 0
        mask, mk = g.ktruss(3)
        assert mk == 0
        tau, kmax = g.truss_decomposition()
        assert kmax == 0 and tau.numel() == 0
        g.free()
    loops = np.array([3, 3, 5], np.int32)
    g = gc.build_graph(loops, loops, 10)
    assert g.m == 0 and g.truss_decomposition()[1] == 0
    g.free()
    g = gc.build_graph(np.array([1, 0, 1], np.int32), np.array([0, 1, 0], np.int32), 2)
    assert g.m == 1 and g.triangle_count() == 0
    tau, kmax = g.truss_decomposition()
    assert kmax == 2 and tau.tolist() == [2]
    assert g.ktruss(2)[1] == 1 and g.ktruss(3)[1] == 0
    g.free()


def test_errors_are_reported():
    with pytest.raises(gc.GCError) as ei:
        gc.build_graph(np.array([0, 5], np.int32), np.array([1, 2], np.int32), 5)
    assert ei.value.status == gc.GC_ERANGE
    with pytest.raises(gc.GCError) as ei:
        gc.build_graph(np.array([0, 1], np.int32), np.array([1, 2], np.int32), 5, one_based=True)
    assert ei.value.status == gc.GC_ERANGE
    g = gc.build_graph(*gg.complete(5)[:2], 5)
    with pytest.raises(gc.GCError) as ei:
        g.ktruss(1)
    assert ei.value.status == gc.GC_EINVAL
    small = torch.empty(3, dtype=torch.int32, device="cuda")
    with pytest.raises(gc.GCError) as ei:
        g.edge_support(out=small)
    assert ei.value.status == gc.GC_ECAPACITY
    assert g.triangle_count() == 10   # handle still usable after errors
    g.free()


def test_repeat_runs_identical():
    src, dst, n = gg.rmat(13, 16, seed=9)
    g = gc.build_graph(src, dst, n)
    a = (g.triangle_count(), g.edge_support().cpu().numpy(), g.truss_decomposition()[0].cpu().numpy())
    for _ in range(2):
        b = (g.triangle_count(), g.edge_support().cpu().numpy(),
             g.truss_decomposition()[0].cpu().numpy())
        assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    g.free()
    g2 = gc.build_graph(src, dst, n)
    assert g2.triangle_count() == a[0]
    g2.free()


# ----------------------------------------------------------------------------
# larger seeded workloads against stored oracle digests
# ----------------------------------------------------------------------------

def _golden():
    if not os.path.exists(GOLDEN):
        return {}
    with open(GOLDEN) as f:
        return json.load(f)


DIGEST_GENS = {
    "rmat_s16_ef16_seed1": lambda: gg.rmat(16, 16, seed=1),
    "rmat_s18_ef16_seed1": lambda: gg.rmat(18, 16, seed=1),
    "rmat_s20_ef16_seed1": lambda: gg.rmat(20, 16, seed=1),
    "er_n20_m16n_seed2": lambda: gg.er(1 << 20, 16 << 20, seed=2),
    "rmat_s22_ef16_seed1": lambda: gg.rmat(22, 16, seed=1),
    # the full-size workloads: their truss numbers come from the oracle's
    # index-free peeling route (the triangle index does not fit in memory)
    "rmat_s24_ef16_seed1": lambda: _rmat24(),
    "er_n24_m16n_seed2": lambda: gg.er(1 << 24, 16 << 24, seed=2),
}


_RMAT24 = []


def _rmat24():
    if not _RMAT24:
        _RMAT24.append(gg.rmat(24, 16, seed=1))
    return _RMAT24[0]


@pytest.mark.parametrize("name", sorted(DIGEST_GENS))
def test_against_oracle_digest(name):
    gold = _golden().get(name)
    if gold is None:
        pytest.skip("no stored oracle digest for %s" % name)
    say("case digest", name)
    src, dst, n = DIGEST_GENS[name]()
    g = gc.build_graph(src, dst, n)
    assert g.m == gold["m"]
    u, v = g.edges()
    assert sha(torch.stack([u, v], 1).cpu().numpy()) == gold["edges_sha256"]
    assert g.triangle_count() == gold["triangles"]
    assert sha(g.edge_support().cpu().numpy().astype("<i4")) == gold["support_sha256"]
    if "kmax" in gold:
        tau, kmax = g.truss_decomposition()
        assert kmax == gold["kmax"]
        assert sha(tau.cpu().numpy().astype("<i4")) == gold["truss_sha256"]
        for k, rec in gold["ktruss"].items():
            mask, mk = g.ktruss(int(k))
            assert mk == rec["m_k"]
            assert sha(mask.cpu().numpy()) == rec["mask_sha256"]
    g.free()


def test_scale24_decomposition_properties():
    """Full decomposition of the scale-24 R-MAT graph, checked by properties
    beside the oracle's digest: every triangle is destroyed exactly once and every
    edge removed once; no truss number exceeds support + 2; and the top level
    (edges with truss number kmax) is a kmax-truss whose minimum support, counted
    here by the masked product (A A) .* A on that subgraph, is exactly kmax - 2
    (larger would make it a (kmax+1)-truss)."""
    gold = _golden().get("rmat_s24_ef16_seed1")
    if gold is None:
        pytest.skip("no stored oracle digest for the scale-24 graph")
    src, dst, n = _rmat24()
    say("case scale-24 decomposition")
    g = gc.build_graph(src, dst, n)
    tau, kmax = g.truss_decomposition()
    st = g.truss_stats()
    say("stats", {k: v for k, v in st.items() if k != "rounds_by_log2_size"})
    assert st["triangles_destroyed"] == gold["triangles"]
    assert st["removed"] == gold["m"]
    sup = g.edge_support()
    assert bool((tau >= 2).all()) and bool((tau <= sup + 2).all())
    assert int(tau.max()) == kmax
    top = (tau == kmax).nonzero().flatten()
    u, v = g.edges()
    tu, tv = u[top].cpu().numpy(), v[top].cpu().numpy()
    say("top level", kmax, len(tu))
    g.free()
    import scipy.sparse as sp
    ids, inv = np.unique(np.concatenate([tu, tv]), return_inverse=True)
    a, b = inv[:len(tu)], inv[len(tu):]
    k = len(ids)
    A = sp.coo_matrix((np.ones(2 * len(a), np.int64), (np.r_[a, b], np.r_[b, a])),
                      shape=(k, k)).tocsr()
    S = (A @ A).multiply(A).tocsr()
    tsup = np.asarray(S[a, b]).ravel()
    assert int(tsup.min()) == kmax - 2


def test_decomposition_peel_equals_rounds(monkeypatch):
    """Incremental peeling and recompute-per-round give the same truss numbers."""
    for label, (src, dst, n) in (("rmat14", gg.rmat(14, 16, seed=3)),
                                 ("rgg12", gg.rgg(1 << 12, 20.0, seed=4)),
                                 ("K60", gg.complete(60))):
        say("case decomposition methods", label)
        g = gc.build_graph(src, dst, n)
        monkeypatch.setenv("GC_TRUSS_METHOD", "rounds")
        t_rounds, k_rounds = g.truss_decomposition()
        t_rounds = t_rounds.cpu().numpy()
        monkeypatch.setenv("GC_TRUSS_METHOD", "peel")
        t_peel, k_peel = g.truss_decomposition()
        assert k_rounds == k_peel
        assert np.array_equal(t_rounds, t_peel.cpu().numpy())
        g.free()


@pytest.mark.parametrize("lb_min,sort_min", [("1", "0"), ("64", "0"), ("2147483647", "0"),
                                             ("1", "1"), ("2147483647", "1")])
def test_peel_lane_batches(monkeypatch, lb_min, sort_min):
    """The peel kernel's two schedules (lane-balanced batches of up to 64
    frontier edges, or whole waves per edge) give the oracle's truss numbers:
    GC_PEEL_LB_MIN = 1 takes batches in every round, 2^31 - 1 never; with
    GC_PEEL_SORT_MIN = 1 every level's first frontier is sorted by higher
    endpoint."""
    monkeypatch.setenv("GC_PEEL_LB_MIN", lb_min)
    monkeypatch.setenv("GC_PEEL_SORT_MIN", sort_min)
    for label, (src, dst, n) in (("rmat13", gg.rmat(13, 16, seed=11)),
                                 ("rgg11", gg.rgg(1 << 11, 24.0, seed=12)),
                                 ("K45", gg.complete(45)), ("king", gg.king(30)),
                                 ("tripartite", gg.complete_tripartite(5, 9, 20))):
        say("case lane batches", lb_min, sort_min, label)
        g = gc.build_graph(src, dst, n)
        u, v = oracle.normalise(src, dst, n)
        tau_ref, kmax_ref = oracle.truss_decomposition(n, u, v, "peel")
        tau, kmax = g.truss_decomposition()
        assert kmax == kmax_ref, (label, kmax, kmax_ref)
        assert np.array_equal(tau.cpu().numpy(), tau_ref), label
        st = g.truss_stats()
        assert st["triangles_destroyed"] == oracle.triangle_count(n, u, v), label
        g.free()


def test_ktruss_peel_equals_rounds(monkeypatch):
    """k-truss by peeling the levels 3 .. k and by Alg. 4's recount rounds give
    the same edge set and size, and both match the oracle's truss numbers."""
    for label, (src, dst, n) in (("rmat14", gg.rmat(14, 16, seed=7)),
                                 ("rgg12", gg.rgg(1 << 12, 20.0, seed=8)),
                                 ("K30", gg.complete(30)), ("star", gg.star(40))):
        say("case ktruss methods", label)
        g = gc.build_graph(src, dst, n)
        u, v = oracle.normalise(src, dst, n)
        tau_ref, kmax = oracle.truss_decomposition(n, u, v, "peel")
        for k in sorted(set([2, 3, 4, 5, kmax - 1, kmax, kmax + 1, kmax + 5]) - {0, 1}):
            ref = (tau_ref >= k).astype(np.uint8)
            for method in ("rounds", "peel"):
                monkeypatch.setenv("GC_TRUSS_METHOD", method)
                mask, mk = g.ktruss(k)
                assert np.array_equal(mask.cpu().numpy(), ref), (label, k, method)
                assert mk == int(ref.sum()), (label, k, method)
        g.free()


@pytest.mark.parametrize("strategy", [[0, 0, 0, 0, 2], [1, 1, 1, 1, 2], [2, 2, 2, 2, 2],
                                      [3, 3, 3, 3, 2], [4, 4, 4, 4, 2], [5, 5, 0, 0, 2],
                                      [6, 6, 3, 3, 2], [6, 5, 0, 0, 2]])
def test_count_strategies_agree(strategy):
    """Every count strategy gives the oracle's count (bins 0-3 exercised by the
    R-MAT graph and a complete graph reaching d+ > 2048)."""
    for src, dst, n in (gg.rmat(14, 16, seed=2), gg.complete(2300),
                        gg.er(1 << 15, 16 << 15, seed=5)):
        g = gc.build_graph(src, dst, n)
        g.set_strategy(strategy)
        u, v = oracle.normalise(src, dst, n)
        want = n * (n - 1) * (n - 2) // 6 if len(u) == n * (n - 1) // 2 else \
            oracle.triangle_count(n, u, v)
        assert g.triangle_count() == want, strategy
        g.free()


@pytest.mark.parametrize("tile", [[32] * 5, [64] * 5, [32, 64, 128, 32, 64]])
@pytest.mark.parametrize("strategy", [[0, 0, 0, 0, 2], [3, 5, 2, 4, 2], [6, 6, 3, 3, 2],
                                      [5, 1, 4, 3, 2]])
def test_count_tiles_agree(tile, strategy):
    """Work units of 32 or 64 in-edges give the oracle's count with every
    strategy (the complete graph puts up to 2299 in-edges on one vertex, so
    one middle vertex spans up to 72 units)."""
    for src, dst, n in (gg.rmat(14, 16, seed=2), gg.complete(2300)):
        g = gc.build_graph(src, dst, n)
        u, v = oracle.normalise(src, dst, n)
        want = n * (n - 1) * (n - 2) // 6 if len(u) == n * (n - 1) // 2 else \
            oracle.triangle_count(n, u, v)
        g.set_strategy(strategy)
        assert g.triangle_count() == want
        g.set_tile(tile)
        st, t = g.count_config()
        assert t.tolist() == tile and st.tolist() == strategy
        assert g.triangle_count() == want, (tile, strategy)
        g.set_tile([128] * 5)
        assert g.triangle_count() == want
        g.free()


def test_autotune_keeps_counts():
    src, dst, n = gg.rmat(15, 16, seed=3)
    g = gc.build_graph(src, dst, n)
    T = g.triangle_count()
    st, ms = g.autotune()
    st2, tile = g.count_config()
    say("graph autotune", st.tolist(), tile.tolist(), np.round(ms, 3).tolist())
    assert st[4] == 2 and g.triangle_count() == T
    assert st2.tolist() == st.tolist() and set(tile.tolist()) <= {32, 64, 128}
    with pytest.raises(gc.GCError):
        g.set_tile([128, 128, 16, 128, 128])
    with pytest.raises(gc.GCError):
        g.set_tile([256] * 5)
    assert g.count_config()[1].tolist() == tile.tolist()
    with pytest.raises(gc.GCError):
        g.set_strategy([0, 0, 0, 0, 1])
    with pytest.raises(gc.GCError):
        g.set_strategy([0, 0, 5, 0, 2])   # one wave per unit only for bins 0 and 1
    with pytest.raises(gc.GCError):
        g.set_strategy([0, 0, 6, 0, 2])   # merge only for bins 0 and 1
    g.free()


def test_autotune_cache_round_trip(tmp_path, monkeypatch):
    """The autotuner writes one line per bin (arch, bin, strategy, tile) to
    GC_AUTOTUNE_CACHE; a new handle takes them; a line without a tile keeps
    the default tile, and invalid lines are ignored."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("GC_AUTOTUNE_CACHE", str(path))
    src, dst, n = gg.rmat(13, 16, seed=5)
    u, v = oracle.normalise(src, dst, n)
    T = oracle.triangle_count(n, u, v)
    g = gc.build_graph(src, dst, n)
    st, _ = g.autotune()
    st_g, tile_g = g.count_config()
    lines = [ln.split() for ln in path.read_text().splitlines()]
    assert [int(f[1]) for f in lines] == list(range(5)) and all(len(f) == 4 for f in lines)
    assert [int(f[2]) for f in lines] == st.tolist() == st_g.tolist()
    assert [int(f[3]) for f in lines] == tile_g.tolist()
    h = gc.build_graph(src, dst, n)
    assert [x.tolist() for x in h.count_config()] == [st_g.tolist(), tile_g.tolist()]
    arch = lines[0][0]
    path.write_text("%s 2 3\n%s 1 4 64\n%s 0 6 48\n%s 3 9 32\nother 0 1 32\n"
                    % (arch, arch, arch, arch))
    k = gc.build_graph(src, dst, n)
    st_k, tile_k = k.count_config()
    assert st_k[2] == 3 and tile_k[2] == 128     # no tile on the line: default kept
    assert st_k[1] == 4 and tile_k[1] == 64
    assert st_k[0] == 6 and tile_k[0] == 128     # 48 is not a tile: strategy only
    assert st_k[3] == 0                          # 9 is not a strategy: line ignored
    assert k.triangle_count() == T
    for x in (g, h, k):
        x.free()


@pytest.mark.parametrize("label", ["rmat16", "er16", "K300", "king64"])
def test_peeling_destroys_each_triangle_once(label):
    """Incremental peeling subtracts every triangle exactly once over the whole
    decomposition, and removes every edge exactly once."""
    src, dst, n = {"rmat16": gg.rmat(16, 16, seed=4), "er16": gg.er(1 << 16, 16 << 16, seed=4),
                   "K300": gg.complete(300), "king64": gg.king(64)}[label]
    g = gc.build_graph(src, dst, n)
    T = g.triangle_count()
    for rep in range(2):  # the handle is reused: counters restart per call
        g.truss_decomposition()
        st = g.truss_stats()
        say(label, {k: v for k, v in st.items() if k != "rounds_by_log2_size"})
        assert st["triangles_destroyed"] == T
        assert st["removed"] == g.m
        assert sum(st["rounds_by_log2_size"]) == st["rounds"]
        assert st["largest_round"] <= g.m and st["levels"] <= st["rounds"]
    g.free()
