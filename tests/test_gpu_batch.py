"""Batched path: many graphs in one device structure and one launch per bin.
Every graph's batched result must equal the oracle on that graph alone (and
the one-graph-per-call GPU path); strategies chosen by the autotuner must not
change any result; the captured HIP graph must give the eager result on every
replay."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_graphs(seed=0, count=40):
    rng = np.random.default_rng(seed)
    graphs = [gg.complete(7), gg.king(5), (np.zeros(0, np.int32), np.zeros(0, np.int32), 4),
              gg.book(300), gg.star(50), gg.complete(1), gg.wheel(12)]
    while len(graphs) < count:
        if rng.random() < 0.5:
            graphs.append(gg.rmat(int(rng.integers(5, 11)), int(rng.integers(8, 33)),
                                  seed=int(rng.integers(1, 1 << 30))))
        else:
            graphs.append(gg.rgg(int(rng.integers(64, 2048)), 20.0,
                                 seed=int(rng.integers(1, 1 << 30))))
    return graphs


def oracle_per_graph(graphs, k=4):
    out = []
    for s, d, n in graphs:
        u, v = oracle.normalise(s, d, n)
        T = oracle.triangle_count(n, u, v)
        sup = oracle.support(n, u, v, "listing")
        mask = oracle.ktruss(n, u, v, k, "peel") if len(u) else np.zeros(0, np.uint8)
        out.append((T, sup, mask))
    return out


def test_batch_matches_oracle_per_graph():
    graphs = mixed_graphs(1)
    say("case batch mixed", len(graphs))
    ref = oracle_per_graph(graphs)
    b = gc.build_batch(graphs)
    off = b.edge_offsets
    assert len(off) == len(graphs) + 1
    T = b.triangle_count().cpu().numpy()
    sup = b.edge_support().cpu().numpy()
    mask, mk = b.ktruss(4)
    mask = mask.cpu().numpy()
    mk = mk.cpu().numpy()
    for i, (Tr, sr, mr) in enumerate(ref):
        assert T[i] == Tr, i
        assert off[i + 1] - off[i] == len(sr), i
        assert np.array_equal(sup[off[i]:off[i + 1]], sr), i
        assert np.array_equal(mask[off[i]:off[i + 1]], mr), i
        assert mk[i] == int(mr.sum()), i
    b.free()


def test_batch_equals_per_call_path():
    graphs = mixed_graphs(2, count=24)
    say("case batch vs per-call")
    b = gc.build_batch(graphs)
    T = b.triangle_count().cpu().numpy()
    for i, (s, d, n) in enumerate(graphs):
        g = gc.build_graph(s, d, n)
        assert g.triangle_count() == T[i]
        g.free()
    b.free()


def test_every_strategy_same_counts():
    graphs = mixed_graphs(3, count=30) + [gg.complete(300), gg.complete(2100)]
    say("case batch strategies")
    b = gc.build_batch(graphs)
    base = b.triangle_count().cpu().numpy().copy()
    for st in ([0, 0, 0, 0, 2], [1, 1, 1, 1, 2], [2, 2, 2, 2, 2], [3, 3, 3, 3, 2],
               [4, 4, 4, 4, 2], [0, 1, 2, 3, 2], [4, 3, 1, 0, 2], [5, 5, 3, 4, 2],
               [6, 6, 3, 4, 2]):
        b.set_strategy(st)
        assert np.array_equal(b.triangle_count().cpu().numpy(), base), st
    chosen, ms = b.autotune()
    say("autotune", chosen.tolist(), np.round(ms, 3).tolist())
    assert chosen[4] == 2
    assert np.array_equal(b.triangle_count().cpu().numpy(), base)
    with pytest.raises(gc.GCError):
        b.set_strategy([0, 0, 0, 0, 0])   # the unbounded bin admits only search
    b.free()


def test_graph_replay_with_eager_work_between():
    graphs = mixed_graphs(4, count=16)
    say("case batch replay")
    b = gc.build_batch(graphs)
    first = b.triangle_count().cpu().numpy().copy()
    x = torch.arange(1 << 20, device="cuda")
    for rep in range(5):
        y = (x * 3 + rep).sum()          # eager work on the same stream
        torch.cuda.synchronize()
        out = torch.full((len(graphs),), -7, dtype=torch.int64, device="cuda")
        b.triangle_count(out=out)
        assert np.array_equal(out.cpu().numpy(), first), rep
        assert int(y) >= 0
    # on a side stream too
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = b.triangle_count()
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), first)
    b.free()


def per_graph_check(b, graphs, ref, mask, mk, label):
    off = b.edge_offsets
    mask = mask.cpu().numpy()
    mk = mk.cpu().numpy()
    for i, (_, _, mr) in enumerate(ref):
        assert np.array_equal(mask[off[i]:off[i + 1]], mr), (label, i)
        assert mk[i] == int(mr.sum()), (label, i)


def test_ktruss_replay_with_eager_work_between():
    """The batched k-truss is recorded into a HIP graph on its first call for
    a k and replayed afterwards: every replay, with eager work on the stream
    between them, and on a side stream, gives the oracle's k-truss of every
    graph."""
    graphs = mixed_graphs(5, count=20)
    x = torch.arange(1 << 20, device="cuda")
    for k in (3, 4, 5):
        ref = oracle_per_graph(graphs, k)
        say("case batch k-truss replay k=%d" % k)
        b = gc.build_batch(graphs)
        for rep in range(4):
            y = (x * 5 + rep).sum()
            torch.cuda.synchronize()
            mask, mk = b.ktruss(k)
            per_graph_check(b, graphs, ref, mask, mk, (k, rep))
            assert int(y) >= 0
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            mask, mk = b.ktruss(k, stream=s)
        s.synchronize()
        per_graph_check(b, graphs, ref, mask, mk, (k, "side stream"))
        b.free()


def test_ktruss_replay_needs_more_rounds_than_recorded(monkeypatch):
    """With one round recorded per level (GC_BATCH_KTRUSS_ROUNDS=1), the
    4-truss levels of R-MAT graphs need more: the call peels eagerly (same
    result) and the next call records twice the rounds, until a replay
    converges; every call gives the oracle's k-truss."""
    monkeypatch.setenv("GC_BATCH_KTRUSS_ROUNDS", "1")
    graphs = [gg.rmat(12, 16, seed=21), gg.complete(9), gg.king(6)] + mixed_graphs(6, count=8)
    ref = oracle_per_graph(graphs, 4)
    say("case batch k-truss re-recorded")
    b = gc.build_batch(graphs)
    for rep in range(6):
        mask, mk = b.ktruss(4)
        per_graph_check(b, graphs, ref, mask, mk, rep)
    b.free()


def test_batch_edge_cases_and_errors():
    b = gc.build_batch([])
    assert b.n_graphs == 0
    b.free()
    e = np.zeros(0, np.int32)
    b = gc.build_batch([(e, e, 0), (e, e, 3)])
    assert b.triangle_count().cpu().tolist() == [0, 0]
    b.free()
    bad = [gg.complete(4), (np.array([0, 7], np.int32), np.array([1, 2], np.int32), 5)]
    with pytest.raises(gc.GCError) as ei:
        gc.build_batch(bad)
    assert ei.value.status == gc.GC_ERANGE
