"""Pins of the CPU oracle against things other than itself: brute force,
exhaustive enumeration, the paper's own array formulations (Alg. 2, 3, 4),
closed forms, the paper's printed examples and invariants.  CPU only."""
import itertools
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def canon(s, d, n):
    u, v = oracle.normalise(s, d, n)
    return n, u, v


# --------------------------------------------------------------------------
# normalisation (Sec. II)
# --------------------------------------------------------------------------

def test_normalise_set_semantics():
    rng = np.random.default_rng(0)
    for trial in range(50):
        n = int(rng.integers(1, 30))
        P = int(rng.integers(0, 80))
        s = rng.integers(0, n, P).astype(np.int32)
        d = rng.integers(0, n, P).astype(np.int32)
        u, v = oracle.normalise(s, d, n)
        want = sorted({(min(a, b), max(a, b)) for a, b in zip(s.tolist(), d.tolist()) if a != b})
        assert list(zip(u.tolist(), v.tolist())) == want


def test_normalise_one_based_and_range():
    u, v = oracle.normalise([1, 2, 3], [2, 3, 1], 3, one_based=True)
    assert u.tolist() == [0, 0, 1] and v.tolist() == [1, 2, 2]
    with pytest.raises(ValueError):
        oracle.normalise([0], [3], 3)
    with pytest.raises(ValueError):
        oracle.normalise([0], [1], 3, one_based=True)  # id 0 invalid when 1-based


def test_normalise_invariant_to_presentation():
    s, d, n = gg.rmat(8, 8, seed=3)
    u0, v0 = oracle.normalise(s, d, n)
    s2, d2, _ = gg.scramble(s, d, n, seed=4)
    u1, v1 = oracle.normalise(s2, d2, n)
    assert np.array_equal(u0, u1) and np.array_equal(v0, v1)


# --------------------------------------------------------------------------
# Fig. 1 and Table II (values the paper prints)
# --------------------------------------------------------------------------

def _read_fig1():
    edges, exp = [], {}
    with open(os.path.join(GOLDEN, "fig1_two_triangles.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "edge":
                edges.append((int(tok[1]), int(tok[2])))
            else:
                exp[tok[0]] = [int(t) for t in tok[1:]]
    return edges, exp


def test_fig1_two_triangles():
    edges, exp = _read_fig1()
    s = np.array([e[0] for e in edges], np.int32)
    d = np.array([e[1] for e in edges], np.int32)
    n, u, v = canon(s, d, 4)
    assert oracle.triangle_count(n, u, v) == exp["triangles"][0]
    assert oracle.support(n, u, v).tolist() == exp["support"]
    assert oracle.truss_decomposition(n, u, v)[1] == exp["kmax"][0]


def _table2():
    rows = []
    with open(os.path.join(GOLDEN, "table2_image_graphs.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(t) for t in line.split()])
    return rows


def test_table2_closed_forms_match_printed_columns():
    # node column = M^2, edge column = 2(M-1)(2M-1), triangle column = 8(M-1)^2
    for n_, nodes, edges, tri_printed in _table2():
        M = 2 ** n_
        assert nodes == M * M
        assert edges == 2 * (M - 1) * (2 * M - 1)
        assert tri_printed == 2 * 4 * (M - 1) ** 2


@pytest.mark.parametrize("row", [0, 1])
def test_table2_oracle_on_printed_sizes(row):
    n_, nodes, edges, tri_printed = _table2()[row]
    M = 2 ** n_
    s, d, n = gg.king(M)
    n, u, v = canon(s, d, n)
    assert n == nodes and len(u) == edges
    T = oracle.triangle_count(n, u, v)
    assert 2 * T == tri_printed          # printed column is twice the count


def test_king_small_brute_force():
    for M in [1, 2, 3, 4, 5]:
        s, d, n = gg.king(M)
        n, u, v = canon(s, d, n)
        assert len(u) == 2 * (M - 1) * (2 * M - 1)
        T = oracle.triangle_count(n, u, v)
        assert T == dense.brute_triangles(n, u, v) == 4 * (M - 1) ** 2


# --------------------------------------------------------------------------
# triangle count vs brute force and the paper's Alg. 2 / Alg. 3
# --------------------------------------------------------------------------

def _random_graph(rng, n, p):
    iu = np.triu_indices(n, 1)
    keep = rng.random(len(iu[0])) < p
    return iu[0][keep].astype(np.int32), iu[1][keep].astype(np.int32)


def test_tc_random_vs_brute_and_dense():
    rng = np.random.default_rng(1)
    for trial in range(60):
        n = int(rng.integers(1, 40))
        p = float(rng.choice([0.05, 0.2, 0.5, 0.9]))
        u, v = _random_graph(rng, n, p)
        T = oracle.triangle_count(n, u, v)
        assert T == dense.brute_triangles(n, u, v)
        assert T == dense.triangle_count_alg2(n, u, v)
        assert T == dense.triangle_count_alg3(n, u, v)


def _all_graphs_on(nv):
    pairs = list(itertools.combinations(range(nv), 2))
    return pairs


def test_exhaustive_six_vertices_tc_and_support():
    """All 2^15 labelled graphs on 6 vertices."""
    nv = 6
    pairs = _all_graphs_on(nv)
    E = len(pairs)
    idx = {p: i for i, p in enumerate(pairs)}
    masks = np.arange(1 << E, dtype=np.int64)
    bits = ((masks[:, None] >> np.arange(E)) & 1).astype(np.int64)  # [G, E]
    # brute-force triangle count and per-edge support, vectorised over graphs
    T = np.zeros(len(masks), np.int64)
    sup = np.zeros((len(masks), E), np.int64)
    for a, b, c in itertools.combinations(range(nv), 3):
        ab, ac, bc = idx[(a, b)], idx[(a, c)], idx[(b, c)]
        t = bits[:, ab] & bits[:, ac] & bits[:, bc]
        T += t
        sup[:, ab] += t
        sup[:, ac] += t
        sup[:, bc] += t
    all_u = np.array([p[0] for p in pairs], np.int32)
    all_v = np.array([p[1] for p in pairs], np.int32)
    for g in range(len(masks)):
        sel = bits[g].astype(bool)
        u, v = all_u[sel], all_v[sel]
        assert oracle.triangle_count(nv, u, v) == T[g]
        assert np.array_equal(oracle.support(nv, u, v), sup[g][sel])


def test_exhaustive_five_vertices_ktruss_vs_subset_enumeration():
    """k-truss on all 2^10 graphs on 5 vertices vs the definition (union of
    every edge subset in which each edge has >= k-2 triangles)."""
    nv = 5
    pairs = _all_graphs_on(nv)
    all_u = np.array([p[0] for p in pairs], np.int32)
    all_v = np.array([p[1] for p in pairs], np.int32)
    rng = np.random.default_rng(5)
    graphs = rng.choice(1 << len(pairs), 160, replace=False)
    for g in graphs:
        sel = ((int(g) >> np.arange(len(pairs))) & 1).astype(bool)
        u, v = all_u[sel], all_v[sel]
        for k in (3, 4, 5):
            want = dense.brute_ktruss(nv, u, v, k)
            bulk, _ = oracle.ktruss(nv, u, v, k, "bulk")
            peel = oracle.ktruss(nv, u, v, k, "peel")
            search = oracle.ktruss(nv, u, v, k, "search")
            assert np.array_equal(bulk, want) and np.array_equal(peel, want)
            assert np.array_equal(search, want)


def test_five_vertices_decomposition_vs_subset_enumeration():
    """Truss numbers (Sec. III-B, last paragraph: the k-truss for growing k
    until it is empty) against the definition: tau(e) is the largest k whose
    maximal k-truss, enumerated over every edge subset, holds e; kmax is the
    largest tau (0 without edges, reading R2).  160 graphs on 5 vertices and
    K_5 itself, by the three oracle methods."""
    nv = 5
    pairs = _all_graphs_on(nv)
    all_u = np.array([p[0] for p in pairs], np.int32)
    all_v = np.array([p[1] for p in pairs], np.int32)
    rng = np.random.default_rng(11)
    graphs = list(rng.choice(1 << len(pairs), 160, replace=False)) + [(1 << len(pairs)) - 1, 0]
    for g in graphs:
        sel = ((int(g) >> np.arange(len(pairs))) & 1).astype(bool)
        u, v = all_u[sel], all_v[sel]
        want = np.full(len(u), 2, np.int32)
        for k in (3, 4, 5, 6):
            want[dense.brute_ktruss(nv, u, v, k).astype(bool)] = k
        want_kmax = int(want.max()) if len(u) else 0
        if sel.all():                                   # K_5: every edge in 3 triangles
            assert want_kmax == 5 and (want == 5).all()
        for method in ("peel", "bulk", "search"):
            tau, kmax = oracle.truss_decomposition(nv, u, v, method)
            assert np.array_equal(tau, want), (int(g), method)
            assert kmax == want_kmax, (int(g), method)


# --------------------------------------------------------------------------
# support vs Alg. 2's C(u,v) and Alg. 4's (EA == 2) 1
# --------------------------------------------------------------------------

def test_support_vs_dense_forms():
    rng = np.random.default_rng(2)
    for trial in range(40):
        n = int(rng.integers(2, 35))
        u, v = _random_graph(rng, n, float(rng.choice([0.1, 0.3, 0.7])))
        s = oracle.support(n, u, v)
        assert np.array_equal(s, dense.support_alg2(n, u, v))
        assert np.array_equal(s, dense.support_alg4(n, u, v))
        assert np.array_equal(s, dense.brute_support(n, u, v))
        assert int(s.sum()) == 3 * oracle.triangle_count(n, u, v)


# --------------------------------------------------------------------------
# k-truss: bulk rounds vs peeling vs literal Alg. 4 (with incremental R)
# --------------------------------------------------------------------------

def test_ktruss_vs_literal_alg4():
    rng = np.random.default_rng(3)
    for trial in range(30):
        n = int(rng.integers(3, 30))
        u, v = _random_graph(rng, n, float(rng.choice([0.2, 0.4, 0.7])))
        for k in (2, 3, 4, 5, 6):
            want, want_rounds = dense.ktruss_alg4(n, u, v, k)
            bulk, rounds = oracle.ktruss(n, u, v, k, "bulk")
            peel = oracle.ktruss(n, u, v, k, "peel")
            search = oracle.ktruss(n, u, v, k, "search")
            assert np.array_equal(bulk, want)
            assert np.array_equal(peel, want)
            assert np.array_equal(search, want)
            assert rounds == want_rounds


def test_truss_certificate_and_nesting_rmat():
    s, d, n = gg.rmat(9, 16, seed=7)
    n, u, v = canon(s, d, n)
    tau, kmax = oracle.truss_decomposition(n, u, v, "peel")
    tau_b, kmax_b = oracle.truss_decomposition(n, u, v, "bulk")
    assert kmax == kmax_b and np.array_equal(tau, tau_b)
    tau_s, kmax_s = oracle.truss_decomposition(n, u, v, "search")
    assert kmax == kmax_s and np.array_equal(tau, tau_s)
    sup = oracle.support(n, u, v)
    assert (tau <= sup + 2).all() and (tau >= 2).all()
    prev = np.ones(len(u), bool)
    for k in range(3, kmax + 2):
        Fk = tau >= k
        assert (Fk <= prev).all()                         # nesting
        mask = oracle.ktruss(n, u, v, k, "peel")
        assert np.array_equal(mask.astype(bool), Fk)      # decomposition = per-k truss
        if Fk.any():                                      # certificate
            uk, vk = u[Fk], v[Fk]
            assert (oracle.support(n, uk, vk) >= k - 2).all()
        prev = Fk
    assert not (tau >= kmax + 1).any() and (tau >= kmax).any()


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nk", [1, 2, 3, 4, 5, 8, 13, 30])
def test_complete_graph(nk):
    n, u, v = canon(*gg.complete(nk))
    T = oracle.triangle_count(n, u, v)
    assert T == nk * (nk - 1) * (nk - 2) // 6
    s = oracle.support(n, u, v)
    assert (s == nk - 2).all()
    for method in ("peel", "bulk", "search"):
        tau, kmax = oracle.truss_decomposition(n, u, v, method)
        if nk >= 2:
            assert kmax == nk and (tau == nk).all()  # K_n is an n-truss
        else:
            assert kmax == 0


# graph -> kmax of the whole graph in closed form (K_{a,b,c}: min + 2; king
# graphs: 4; wheels, windmills, books: 3; triangle-free: 2; a disjoint union:
# the largest of its parts)
CLOSED_KMAX = [
    ("tripartite 2,3,5", lambda: gg.complete_tripartite(2, 3, 5), 4),
    ("tripartite 4,4,6", lambda: gg.complete_tripartite(4, 4, 6), 6),
    ("king 8", lambda: gg.king(8), 4),
    ("wheel 9", lambda: gg.wheel(9), 3),
    ("windmill 7", lambda: gg.windmill(7), 3),
    ("book 10", lambda: gg.book(10), 3),
    ("cycle 9", lambda: gg.cycle(9), 2),
    ("union", lambda: gg.disjoint_union(gg.complete(6), gg.king(4), gg.wheel(7), gg.book(3)), 6),
]


@pytest.mark.parametrize("name,make,kmax", CLOSED_KMAX, ids=[c[0] for c in CLOSED_KMAX])
def test_closed_form_kmax_every_route(name, make, kmax):
    """The three decomposition routes reach the closed-form kmax, and the
    same truss numbers."""
    n, u, v = canon(*make())
    taus = []
    for method in ("peel", "bulk", "search"):
        tau, km = oracle.truss_decomposition(n, u, v, method)
        assert km == kmax, (name, method)
        taus.append(tau)
    assert np.array_equal(taus[0], taus[1]) and np.array_equal(taus[0], taus[2])


@pytest.mark.parametrize("threads", [1, 2, 3, 8])
def test_threaded_count_equals_closed_forms_and_serial(threads):
    """The count with its outer loop dealt over threads (the all-cores CPU
    baseline) gives C(n, 3) on K_n, 4(M-1)^2 on king graphs, 0 without
    triangles, and the serial count on R-MAT."""
    for nk in (1, 3, 30):
        n, u, v = canon(*gg.complete(nk))
        assert oracle.triangle_count_threads(n, u, v, threads) == nk * (nk - 1) * (nk - 2) // 6
    n, u, v = canon(*gg.king(16))
    assert oracle.triangle_count_threads(n, u, v, threads) == 4 * 15 * 15
    n, u, v = canon(*gg.complete_bipartite(5, 7))
    assert oracle.triangle_count_threads(n, u, v, threads) == 0
    n, u, v = canon(*gg.rmat(12, 16, seed=5))
    assert oracle.triangle_count_threads(n, u, v, threads) == oracle.triangle_count(n, u, v)


@pytest.mark.parametrize("abc", [(1, 1, 1), (1, 2, 3), (2, 2, 2), (2, 3, 5), (4, 4, 6)])
def test_complete_tripartite(abc):
    a, b, c = abc
    n, u, v = canon(*gg.complete_tripartite(a, b, c))
    assert oracle.triangle_count(n, u, v) == a * b * c
    s = oracle.support(n, u, v)
    part = np.array([0] * a + [1] * b + [2] * c)
    size = {0: a, 1: b, 2: c}
    for e in range(len(u)):
        other = 3 - part[u[e]] - part[v[e]]
        assert s[e] == size[other]
    assert oracle.truss_decomposition(n, u, v)[1] == min(a, b, c) + 2


@pytest.mark.parametrize("M", [2, 3, 4, 8, 16])
def test_king_support_and_truss(M):
    n, u, v = canon(*gg.king(M))
    s = oracle.support(n, u, v)
    diag = (np.abs(u // M - v // M) == 1) & (np.abs(u % M - v % M) == 1)
    axis = ~diag
    ur, uc, vr, vc = u // M, u % M, v // M, v % M
    horiz = ur == vr
    boundary = np.where(horiz, (ur == 0) | (ur == M - 1), (uc == 0) | (uc == M - 1))
    assert (s[diag] == 2).all()
    assert (s[axis & boundary] == 2).all()
    assert (s[axis & ~boundary] == 4).all()
    assert int((s == 4).sum()) == 2 * (M - 1) * (M - 2)
    tau, kmax = oracle.truss_decomposition(n, u, v)
    assert kmax == 4 and (tau == 4).all()


@pytest.mark.parametrize("r", [4, 5, 9])
def test_wheel(r):
    n, u, v = canon(*gg.wheel(r))
    assert oracle.triangle_count(n, u, v) == r
    assert oracle.truss_decomposition(n, u, v)[1] == 3


@pytest.mark.parametrize("t", [1, 2, 7])
def test_windmill(t):
    n, u, v = canon(*gg.windmill(t))
    assert oracle.triangle_count(n, u, v) == t
    assert oracle.truss_decomposition(n, u, v)[1] == 3


@pytest.mark.parametrize("p", [1, 2, 10])
def test_book(p):
    n, u, v = canon(*gg.book(p))
    assert oracle.triangle_count(n, u, v) == p
    s = oracle.support(n, u, v)
    spine = (u == 0) & (v == 1)
    assert s[spine].tolist() == [p] and (s[~spine] == 1).all()
    assert oracle.truss_decomposition(n, u, v)[1] == 3


@pytest.mark.parametrize("fam", ["star", "path", "cycle", "tree", "bipartite"])
def test_triangle_free(fam):
    g = {"star": gg.star(12), "path": gg.path(20), "cycle": gg.cycle(9),
         "tree": gg.random_tree(40, seed=1), "bipartite": gg.complete_bipartite(4, 6)}[fam]
    n, u, v = canon(*g)
    assert oracle.triangle_count(n, u, v) == 0
    assert (oracle.support(n, u, v) == 0).all()
    tau, kmax = oracle.truss_decomposition(n, u, v)
    assert kmax == 2 and (tau == 2).all()


def test_empty_graph():
    n, u, v = canon(np.zeros(0, np.int32), np.zeros(0, np.int32), 5)
    assert len(u) == 0
    assert oracle.triangle_count(n, u, v) == 0
    assert oracle.truss_decomposition(n, u, v)[1] == 0
    n, u, v = canon(np.array([2, 3], np.int32), np.array([2, 3], np.int32), 5)  # loops only
    assert len(u) == 0


def test_disjoint_union_adds():
    parts = [gg.complete(6), gg.king(4), gg.wheel(7), gg.book(3)]
    n, u, v = canon(*gg.disjoint_union(*parts))
    total = sum(oracle.triangle_count(*canon(*p)) for p in parts)
    assert oracle.triangle_count(n, u, v) == total
    assert oracle.truss_decomposition(n, u, v)[1] == 6


# --------------------------------------------------------------------------
# invariants on R-MAT
# --------------------------------------------------------------------------

def test_relabel_invariance_rmat():
    s, d, n = gg.rmat(10, 16, seed=11)
    n, u, v = canon(s, d, n)
    T = oracle.triangle_count(n, u, v)
    s2, d2, _, perm = gg.relabel(s, d, n, seed=12)
    n2, u2, v2 = canon(s2, d2, n)
    assert oracle.triangle_count(n2, u2, v2) == T
    # per-edge support follows the edges under relabelling
    sup = oracle.support(n, u, v)
    sup2 = oracle.support(n2, u2, v2)
    pu, pv = perm[u], perm[v]
    key = np.minimum(pu, pv) * n + np.maximum(pu, pv)
    key2 = u2.astype(np.int64) * n + v2
    pos = np.searchsorted(key2, key)
    assert np.array_equal(sup2[pos], sup)
    tau, kmax = oracle.truss_decomposition(n, u, v)
    tau2, kmax2 = oracle.truss_decomposition(n2, u2, v2)
    assert kmax == kmax2 and np.array_equal(tau2[pos], tau)


def test_sum_support_three_t_rmat():
    for seed in (1, 2, 3):
        n, u, v = canon(*gg.rmat(10, 16, seed=seed))
        assert int(oracle.support(n, u, v).astype(np.int64).sum()) == \
            3 * oracle.triangle_count(n, u, v)


def test_mutation_would_be_caught():
    """A plausible mistake (counting each triangle from every out-edge pair
    without the third edge) must break the pins: K_4 minus nothing vs C_4."""
    n, u, v = canon(*gg.cycle(4))
    assert oracle.triangle_count(n, u, v) == 0
    n, u, v = canon(*gg.complete_bipartite(3, 3))
    assert oracle.triangle_count(n, u, v) == 0


# --------------------------------------------------------------------------
# the two support routes and the two truss routes agree
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [1, 2])
def test_support_listing_equals_definition(seed):
    for g in (gg.rmat(11, 16, seed=seed), gg.er(2000, 40000, seed=seed),
              gg.rgg(1500, 20.0, seed=seed), gg.complete(25), gg.king(9)):
        n, u, v = canon(*g)
        assert np.array_equal(oracle.support(n, u, v, "listing"),
                              oracle.support(n, u, v, "definition"))


def test_ktruss_bulk_equals_peel_rmat():
    n, u, v = canon(*gg.rmat(10, 16, seed=4))
    for k in (3, 4, 6, 9, 15):
        bulk, _ = oracle.ktruss(n, u, v, k, "bulk")
        assert np.array_equal(bulk, oracle.ktruss(n, u, v, k, "peel"))
        assert np.array_equal(bulk, oracle.ktruss(n, u, v, k, "search"))


def test_stored_digest_is_reproduced_by_the_oracle():
    """tests/golden/digests.json holds values written by make_digests.py from
    the oracle alone: recomputing the R-MAT scale-16 entry (edges, T, support,
    truss numbers, k-truss masks) gives it back exactly.  Only the oracle's
    own run time may differ."""
    import importlib.util
    import json
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_digests",
                                                  os.path.join(here, "make_digests.py"))
    md = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(md)
    name = "rmat_s16_ef16_seed1"
    rec = md.digest(name)
    gold = json.load(open(os.path.join(here, "digests.json")))[name]
    rec.pop("oracle_seconds", None)
    gold = {k: v for k, v in gold.items() if k != "oracle_seconds"}
    assert rec == gold
