"""Serving path: results of every request are identical alone and in a mix
(continuous batching, k-truss overlapping counts), match the oracle, and the
server never charges more device memory than its budget."""
import sys
import threading
import time

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1708_06866_amd as gc  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pool(seed=0, count=24):
    rng = np.random.default_rng(seed)
    graphs = [gg.complete(9), gg.king(12), gg.book(40)]
    while len(graphs) < count:
        scale = int(rng.integers(8, 13))
        graphs.append(gg.rmat(scale, 16, seed=int(rng.integers(1, 1 << 30))))
    return graphs


def expected(graphs, k=4):
    out = []
    for s, d, n in graphs:
        u, v = oracle.normalise(s, d, n)
        T = oracle.triangle_count(n, u, v)
        mk = int(oracle.ktruss(n, u, v, k, "peel").sum()) if len(u) else 0
        out.append((T, mk))
    return out


def queries(ngraphs, seed=1, count=120):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(0, ngraphs)), int(rng.random() < 0.3)) for _ in range(count)]


def run_alone(srv, qs):
    res = []
    for g, kind in qs:
        t = srv.submit(g, kind, 4 if kind else 0)
        res.append(srv.wait(t))
    return res


def run_mix(srv, qs):
    tickets = [srv.submit(g, kind, 4 if kind else 0) for g, kind in qs]
    return [srv.wait(t) for t in tickets]


def test_alone_equals_mix_equals_oracle():
    graphs = pool(1)
    exp = expected(graphs)
    srv = gc.Server(8 << 30)
    ids = [srv.add_graph(*g) for g in graphs]
    assert ids == list(range(len(graphs)))
    qs = queries(len(graphs))
    say("case serve alone")
    alone = run_alone(srv, qs)
    say("case serve mix")
    mix = run_mix(srv, qs)
    for (g, kind), a, b in zip(qs, alone, mix):
        assert a["status"] == 0 and b["status"] == 0
        assert a["value"] == b["value"] == exp[g][kind], (g, kind)
        assert b["t_submit"] <= b["t_start"] <= b["t_done"]
    st = srv.stats()
    say("stats", st)
    assert st["completed"] == 2 * len(qs)
    assert st["max_batch"] > 1               # the counts of the mix were batched
    assert st["max_truss_batch"] > 1         # and so were its k-truss queries
    srv.close()


def test_ktruss_batches_mix_k_and_repeat_graphs():
    """k-truss queries with k = 3..6 on graphs that repeat within a batch:
    each batch groups one k, every graph appears once in its union, and every
    answer is the oracle's k-truss size of that graph alone."""
    graphs = pool(6, count=14)
    rng = np.random.default_rng(9)
    qs = [(int(rng.integers(0, len(graphs))), int(rng.integers(3, 7))) for _ in range(90)]
    want = {}
    for g, k in set(qs):
        s_, d_, n_ = graphs[g]
        u, v = oracle.normalise(s_, d_, n_)
        want[(g, k)] = int(oracle.ktruss(n_, u, v, k, "peel").sum()) if len(u) else 0
    srv = gc.Server(4 << 30)
    for g in graphs:
        srv.add_graph(*g)
    say("case serve k-truss mix")
    tickets = [srv.submit(g, gc.KTRUSS_EDGES, k) for g, k in qs]
    res = [srv.wait(t) for t in tickets]
    for (g, k), r in zip(qs, res):
        assert r["status"] == 0 and r["value"] == want[(g, k)], (g, k, r["value"])
    st = srv.stats()
    say("stats", st)
    assert st["max_truss_batch"] > 1
    srv.close()


def test_device_memory_stays_within_the_charge():
    """hipMemGetInfo during a mixed trace under a budget that forces
    eviction: the device memory the server holds never exceeds the most it
    charged to its budget (builds, resident graphs, k-truss unions), and once
    idle it holds at most what it charges for its resident graphs, and at
    least half of it."""
    rng = np.random.default_rng(12)
    graphs = [gg.rmat(int(rng.integers(13, 17)), 16, seed=int(rng.integers(1, 1 << 30)))
              for _ in range(12)]
    exp = expected(graphs)
    warm = gc.build_graph(*gg.complete(6))     # code objects and library arrays loaded
    warm.triangle_count()
    warm.free()
    torch.cuda.synchronize()
    budget = 512 << 20
    srv = gc.Server(budget)
    for g in graphs:
        srv.add_graph(*g)
    # first use of the server's streams (their queues, kernel arguments and
    # scratch are the runtime's, not the server's), then the baseline
    extra = srv.add_graph(*gg.complete(12))
    for kind in (gc.TRIANGLE_COUNT, gc.KTRUSS_EDGES):
        assert srv.wait(srv.submit(extra, kind, 4 if kind else 0))["status"] == 0
    torch.cuda.synchronize()
    charged0 = srv.stats()["bytes_charged"]
    base_free = torch.cuda.mem_get_info()[0]
    samples = []
    stop = threading.Event()

    def watch():
        while not stop.is_set():
            samples.append(base_free - torch.cuda.mem_get_info()[0])
            time.sleep(2e-4)
    th = threading.Thread(target=watch)
    th.start()
    qs = queries(len(graphs), seed=6, count=150)
    say("case serve memory watch")
    try:
        mix = run_mix(srv, qs)
    finally:
        stop.set()
        th.join()
    for (g, kind), r in zip(qs, mix):
        assert r["status"] == 0 and r["value"] == exp[g][kind]
    st = srv.stats()
    held = max(samples)
    say("device bytes held at most %d (%d samples), peak charged %d, budget %d, evictions %d"
        % (held, len(samples), st["peak_bytes_charged"], budget, st["evictions"]))
    assert st["peak_bytes_charged"] <= budget
    assert st["evictions"] > 0
    # the batch descriptors and counters (a few KB, outside the charge) are
    # the only device memory not charged
    assert charged0 + held <= st["peak_bytes_charged"] + (4 << 20)
    idle = base_free - torch.cuda.mem_get_info()[0]
    charged = st["bytes_charged"] - charged0
    say("idle: device bytes held %d beyond the baseline, charged %d beyond it (%d resident graphs)"
        % (idle, charged, st["resident_graphs"]))
    assert idle <= charged + (4 << 20)
    # the charge is no wild over-estimate either (the stream-ordered pool packs
    # small buffers more tightly than the charge assumes)
    assert idle >= 0.5 * charged
    srv.close()


def test_budget_forces_eviction_and_is_respected():
    rng = np.random.default_rng(2)
    graphs = [gg.rmat(int(rng.integers(13, 15)), 16, seed=int(rng.integers(1, 1 << 30)))
              for _ in range(16)]
    exp = expected(graphs)
    # a scale-14 build reserves ~99 MB and the graph then holds ~13 MB: the
    # 16 graphs (~150 MB resident) do not fit beside a build
    budget = 200 << 20
    srv = gc.Server(budget)
    for g in graphs:
        srv.add_graph(*g)
    qs = queries(len(graphs), seed=3, count=80)
    say("case serve small budget")
    mix = run_mix(srv, qs)
    for (g, kind), r in zip(qs, mix):
        assert r["status"] == 0 and r["value"] == exp[g][kind]
    st = srv.stats()
    say("stats", st)
    assert st["peak_bytes_charged"] <= budget
    assert st["evictions"] > 0
    srv.close()


def test_per_call_mode_same_results():
    graphs = pool(3, count=10)
    exp = expected(graphs)
    srv = gc.Server(4 << 30, mode=1)
    for g in graphs:
        srv.add_graph(*g)
    qs = queries(len(graphs), seed=4, count=40)
    res = run_mix(srv, qs)
    for (g, kind), r in zip(qs, res):
        assert r["value"] == exp[g][kind]
    assert srv.stats()["max_batch"] == 1
    srv.close()


def test_concurrent_submitters():
    graphs = pool(4, count=12)
    exp = expected(graphs)
    srv = gc.Server(4 << 30)
    for g in graphs:
        srv.add_graph(*g)
    errors = []

    def client(seed):
        try:
            rng = np.random.default_rng(seed)
            for _ in range(30):
                g = int(rng.integers(0, len(graphs)))
                kind = int(rng.random() < 0.25)
                r = srv.wait(srv.submit(g, kind, 4 if kind else 0))
                if r["value"] != exp[g][kind]:
                    errors.append((g, kind, r["value"]))
                time.sleep(float(rng.random()) * 1e-3)
        except Exception as e:  # pragma: no cover
            errors.append(repr(e))

    th = [threading.Thread(target=client, args=(s,)) for s in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join(120)
    assert not errors, errors[:5]
    srv.close()


def test_server_errors():
    srv = gc.Server(1 << 30)
    gid = srv.add_graph(*gg.complete(5))
    with pytest.raises(gc.GCError):
        srv.submit(gid + 5)
    with pytest.raises(gc.GCError):
        srv.submit(gid, gc.KTRUSS_EDGES, 1)
    with pytest.raises(gc.GCError):
        srv.add_graph(np.array([0, 9], np.int32), np.array([1, 2], np.int32), 5)
    r = srv.wait(srv.submit(gid))
    assert r["value"] == 10
    with pytest.raises(gc.GCError):
        srv.poll(123456)
    srv.close()
