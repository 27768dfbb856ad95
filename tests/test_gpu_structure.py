"""Degrees, degree order and the oriented CSR (the first steps of the path)
against their definitions, element by element.  The vertex of rank r is the
r-th in the strict order (degree, id); every canonical edge is stored once,
in the row of its lower-ranked endpoint, as the rank of the other endpoint,
rows sorted; eid names its canonical edge (the row of the incidence matrix E,
Sec. III-B).  This is Alg. 3's strictly lower-triangular L taken in degree
order."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1708_06866_amd as gc  # noqa: E402


def oriented_reference(n, u, v):
    deg = np.bincount(u, minlength=n) + np.bincount(v, minlength=n)
    order = np.lexsort((np.arange(n), deg))          # by degree, then id
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    lo = np.minimum(rank[u], rank[v])
    hi = np.maximum(rank[u], rank[v])
    slots = np.lexsort((hi, lo))                     # rows by lower rank, sorted
    row_ptr = np.concatenate([[0], np.cumsum(np.bincount(lo, minlength=n))])
    return rank, row_ptr, hi[slots], slots


CASES = {
    "rmat12": lambda: gg.rmat(12, 16, seed=3),
    "rmat12 with isolated ids above": lambda: (lambda s, d, n: (s, d, n + 37))(*gg.rmat(12, 16, seed=3)),
    "king_16 (many equal degrees)": lambda: gg.king(16),
    "star_300 (one hub)": lambda: gg.star(300),
    "K40 (all degrees equal)": lambda: gg.complete(40),
    "book_50": lambda: gg.book(50),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_oriented_csr_matches_its_definition(name):
    src, dst, n = CASES[name]()
    print("case oriented", name, "pairs", len(src), "n", n, flush=True)
    g = gc.build_graph(src, dst, n)
    u, v = oracle.normalise(src, dst, n)
    rank_ref, row_ref, col_ref, eid_ref = oriented_reference(n, u, v)
    rank, row_ptr, col, eid = g.oriented()
    assert np.array_equal(rank.cpu().numpy(), rank_ref), name
    assert np.array_equal(row_ptr.cpu().numpy(), row_ref), name
    assert np.array_equal(col.cpu().numpy(), col_ref), name
    assert np.array_equal(eid.cpu().numpy(), eid_ref), name
    g.free()
