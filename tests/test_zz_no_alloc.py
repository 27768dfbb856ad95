"""gc_edge_support_noalloc (the allocation-free support entry point, for
callers that cannot allocate device memory) against gc_edge_support, through
the C ABI: bit-exact on two calls in a row, the second on a smaller graph;
at the size limit; refused beyond it.  All results are integers: tolerance 0."""
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

MAX_EDGES = 1 << 24  # GC_NOALLOC_MAX_EDGES in include/gc.h


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def noalloc_support(g):
    """Support by the allocation-free call into a buffer filled with -1, and
    the device memory free before and after it (the call allocates nothing)."""
    out = torch.full((max(g.m, 1),), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    g.edge_support_noalloc(out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return out[:g.m].cpu().numpy(), free0, free1


def test_noalloc_equals_edge_support_on_two_calls_second_smaller():
    big = gg.rmat(16, 16, seed=3)
    small = gg.rmat(11, 16, seed=4)
    results = []
    for label, (src, dst, n) in (("rmat16", big), ("rmat11", small)):
        say("case", label, "pairs", len(src))
        g = gc.build_graph(src, dst, n)
        ref = g.edge_support().cpu().numpy()
        got, free0, free1 = noalloc_support(g)
        assert np.array_equal(got, ref), label
        if label == "rmat16":   # the first call on the device has set up its scratch
            got, free0, free1 = noalloc_support(g)
            assert np.array_equal(got, ref), label
        assert free0 == free1, (label, free0, free1)
        results.append((label, g.m))
        g.free()
    assert results[1][1] < results[0][1]
    # the smaller graph's result also equals the oracle's support
    src, dst, n = small
    u, v = oracle.normalise(src, dst, n)
    g = gc.build_graph(src, dst, n)
    got, _, _ = noalloc_support(g)
    assert np.array_equal(got, oracle.support(n, u, v, "listing"))
    g.free()


def test_noalloc_at_the_size_limit():
    """K_5793 has 16,776,528 edges, just under the limit; every edge has
    support 5791 (K_n: n - 2)."""
    nk = 5793
    assert nk * (nk - 1) // 2 <= MAX_EDGES
    say("case K_%d" % nk)
    src, dst, n = gg.complete(nk)
    g = gc.build_graph(src, dst, n)
    got, _, _ = noalloc_support(g)
    assert len(got) == nk * (nk - 1) // 2
    assert (got == nk - 2).all()
    assert np.array_equal(got, g.edge_support().cpu().numpy())
    g.free()


def test_noalloc_refuses_beyond_the_limit_and_short_outputs():
    nk = 5794                      # 16,782,321 edges > 2^24
    assert nk * (nk - 1) // 2 > MAX_EDGES
    say("case K_%d (refused)" % nk)
    src, dst, n = gg.complete(nk)
    g = gc.build_graph(src, dst, n)
    out = torch.empty(g.m, dtype=torch.int32, device="cuda")
    with pytest.raises(gc.GCError) as ei:
        g.edge_support_noalloc(out)
    assert ei.value.status == gc.GC_ECAPACITY
    assert "GC_NOALLOC_MAX_EDGES" in str(ei.value)
    g.free()
    say("case short output (refused)")
    src, dst, n = gg.complete(10)
    g = gc.build_graph(src, dst, n)
    with pytest.raises(gc.GCError) as ei:
        g.edge_support_noalloc(torch.empty(g.m - 1, dtype=torch.int32, device="cuda"))
    assert ei.value.status == gc.GC_ECAPACITY
    g.free()
    say("case empty graph")
    g = gc.build_graph(np.zeros(0, np.int32), np.zeros(0, np.int32), 4)
    out = torch.empty(1, dtype=torch.int32, device="cuda")
    assert g.edge_support_noalloc(out).numel() == 0
    g.free()
