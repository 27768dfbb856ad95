"""Count and support on a graph dense enough to fill the unbounded degree bin
(middle vertices with more than 8,192 higher-ranked neighbours): the complete
graph K_n with n = 8,300.  Its triangle count C(n, 3) and its supports (n - 2
for every edge) are closed forms, so no oracle run is needed at this size
(34.4 M edges, 9.5e10 triangles)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1708_06866_amd as gc  # noqa: E402


def test_complete_graph_fills_the_unbounded_bin():
    n = 8300
    # in K_n every vertex has degree n - 1, so ranks follow ids and vertex b
    # has n - 1 - b higher-ranked neighbours: b = 1 .. 106 are middle vertices
    # of the unbounded bin (> 8,192)
    u, v = np.triu_indices(n, 1)
    src = torch.from_numpy(u.astype(np.int32)).cuda()
    dst = torch.from_numpy(v.astype(np.int32)).cuda()
    del u, v
    print("case K_%d" % n, flush=True)
    g = gc.build_graph(src, dst, n)
    del src, dst
    assert g.m == n * (n - 1) // 2
    assert g.triangle_count() == n * (n - 1) * (n - 2) // 6
    sup = g.edge_support()
    assert int(sup.min().item()) == n - 2 and int(sup.max().item()) == n - 2
    g.free()
