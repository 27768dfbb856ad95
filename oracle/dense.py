"""The paper's array formulations, written out with dense numpy matrices.

TEST INFRASTRUCTURE ONLY (tiny graphs).  These are independent of the C
oracle: they follow the matrix algebra of the paper rather than adjacency
lists, so agreement between the two pins both.

  triangle_count_alg2   Alg. 2: C = A^2 .* A,  n_T = sum(C) / 6
  triangle_count_alg3   Alg. 3: (L, U) <- A,  B = L U,  C = A .* B,
                        n_T = sum(C) / 2
  support_alg2          C(u, v) of Alg. 2 = number of common neighbours
  support_alg4          Alg. 4's R = E A and s = (R == 2) 1
  ktruss_alg4           Alg. 4 with its incremental update of R
  brute_triangles       direct enumeration of vertex triples (Sec. III-A)
"""
from __future__ import annotations

import itertools

import numpy as np


def adjacency(n: int, u, v) -> np.ndarray:
    """Symmetric 0/1 adjacency with zero diagonal (int64)."""
    A = np.zeros((n, n), dtype=np.int64)
    A[np.asarray(u), np.asarray(v)] = 1
    A[np.asarray(v), np.asarray(u)] = 1
    return A


def incidence(n: int, u, v) -> np.ndarray:
    """Unoriented incidence matrix E (m x n): row e has 1 at u(e) and v(e)."""
    m = len(u)
    E = np.zeros((m, n), dtype=np.int64)
    E[np.arange(m), np.asarray(u)] = 1
    E[np.arange(m), np.asarray(v)] = 1
    return E


def triangle_count_alg2(n: int, u, v) -> int:
    A = adjacency(n, u, v)
    C = (A @ A) * A
    total = int(C.sum())
    assert total % 6 == 0
    return total // 6


def triangle_count_alg3(n: int, u, v) -> int:
    A = adjacency(n, u, v)
    L = np.tril(A, -1)
    U = np.triu(A, 1)
    B = L @ U
    C = A * B
    total = int(C.sum())
    assert total % 2 == 0
    return total // 2


def support_alg2(n: int, u, v) -> np.ndarray:
    A = adjacency(n, u, v)
    C = (A @ A) * A
    return C[np.asarray(u), np.asarray(v)].astype(np.int32)


def support_alg4(n: int, u, v) -> np.ndarray:
    E = incidence(n, u, v)
    d = E.sum(axis=0)
    A = E.T @ E - np.diag(d)
    R = E @ A
    return (R == 2).sum(axis=1).astype(np.int32)


def ktruss_alg4(n: int, u, v, k: int):
    """Alg. 4 literally: returns (mask over the input edges, rounds).

    Rows of E are removed in bulk each round and R is updated incrementally
    with R <- R - E [E_x^T E_x - diag(d_x)]."""
    E = incidence(n, u, v)
    keep = np.arange(E.shape[0])              # original ids of remaining rows
    d = E.sum(axis=0)
    A = E.T @ E - np.diag(d)
    R = E @ A
    s = (R == 2).sum(axis=1)
    x = np.nonzero(s < k - 2)[0]
    rounds = 0
    while len(x):
        rounds += 1
        xc = np.setdiff1d(np.arange(E.shape[0]), x)
        Ex = E[x, :]
        E = E[xc, :]
        keep = keep[xc]
        dx = Ex.sum(axis=0)
        R = R[xc, :]
        R = R - E @ (Ex.T @ Ex - np.diag(dx))
        s = (R == 2).sum(axis=1)
        x = np.nonzero(s < k - 2)[0]
    mask = np.zeros(len(u), dtype=np.uint8)
    mask[keep] = 1
    return mask, rounds


def brute_triangles(n: int, u, v) -> int:
    adj = set(zip(np.asarray(u).tolist(), np.asarray(v).tolist()))
    adj |= {(b, a) for a, b in adj}
    t = 0
    for a, b, c in itertools.combinations(range(n), 3):
        if (a, b) in adj and (b, c) in adj and (a, c) in adj:
            t += 1
    return t


def brute_support(n: int, u, v) -> np.ndarray:
    nb = [set() for _ in range(n)]
    for a, b in zip(np.asarray(u).tolist(), np.asarray(v).tolist()):
        nb[a].add(b)
        nb[b].add(a)
    return np.array([len(nb[a] & nb[b]) for a, b in zip(np.asarray(u).tolist(),
                                                        np.asarray(v).tolist())],
                    dtype=np.int32)


def brute_ktruss(n: int, u, v, k: int) -> np.ndarray:
    """Maximal k-truss as the union of all edge subsets satisfying the
    definition -- enumerated over every subset (only for m <= ~14)."""
    u = np.asarray(u).tolist()
    v = np.asarray(v).tolist()
    m = len(u)
    best = np.zeros(m, dtype=np.uint8)
    for bits in range(1 << m):
        sel = [e for e in range(m) if bits >> e & 1]
        nb = [set() for _ in range(n)]
        for e in sel:
            nb[u[e]].add(v[e])
            nb[v[e]].add(u[e])
        if all(len(nb[u[e]] & nb[v[e]]) >= k - 2 for e in sel):
            for e in sel:
                best[e] = 1
    return best
