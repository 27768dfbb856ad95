"""Seeded input generators: determinism, the C code against its independent
numpy transcription, and distributional sanity.  CPU only."""
import math

import numpy as np
import pytest

import graphgen as gg


@pytest.mark.parametrize("scale", [0, 1, 5, 9])
@pytest.mark.parametrize("permute", [False, True])
def test_rmat_c_matches_numpy(scale, permute):
    s, d, n = gg.rmat(scale, 8, seed=21, permute=permute)
    s2, d2, n2 = gg.rmat_numpy(scale, 8, seed=21, permute=permute)
    assert n == n2 == 1 << scale
    assert np.array_equal(s, s2) and np.array_equal(d, d2)


def test_rmat_deterministic_and_seeded():
    a = gg.rmat(10, 16, seed=1)
    b = gg.rmat(10, 16, seed=1)
    c = gg.rmat(10, 16, seed=2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[0], c[0])


def test_rmat_range_and_quadrants():
    s, d, n = gg.rmat(12, 16, seed=3, permute=False)
    assert s.min() >= 0 and s.max() < n and d.min() >= 0 and d.max() < n
    # top-level quadrant frequencies follow the initiator (a, b, c, d)
    top_u = s >> 11
    top_v = d >> 11
    freq = [np.mean((top_u == i) & (top_v == j)) for i, j in ((0, 0), (0, 1), (1, 0), (1, 1))]
    for f, p in zip(freq, gg.RMAT_ABCD):
        assert abs(f - p) < 0.01


def test_permutation_is_bijection():
    for scale in (1, 4, 10):
        x = np.arange(1 << scale, dtype=np.int64)
        y = gg.permute_numpy(x, scale, seed=9)
        assert len(np.unique(y)) == 1 << scale


def test_er_mean_degree():
    n = 1 << 14
    s, d, _ = gg.er(n, 16 * n, seed=5)
    assert s.min() >= 0 and s.max() < n
    deg = np.bincount(s, minlength=n) + np.bincount(d, minlength=n)
    assert abs(deg.mean() - 32.0) < 1e-9
    assert deg.std() < 10


def test_rgg_mean_degree_and_brute_force():
    n = 300
    s, d, _ = gg.rgg(n, 20.0, seed=4)
    x, y = gg.rgg_points(n, seed=4)
    r2 = gg.rgg_radius2(n, 20.0)
    dx = np.abs(x[:, None] - x[None, :])
    dy = np.abs(y[:, None] - y[None, :])
    dx = np.where(dx > 0.5, 1.0 - dx, dx)
    dy = np.where(dy > 0.5, 1.0 - dy, dy)
    close = (dx * dx + dy * dy) < r2
    iu = np.triu_indices(n, 1)
    want = set(zip(iu[0][close[iu]].tolist(), iu[1][close[iu]].tolist()))
    got = set(zip(s.tolist(), d.tolist()))
    assert got == want
    s, d, _ = gg.rgg(1 << 12, 20.0, seed=5)
    assert abs(2 * len(s) / (1 << 12) - 20.0) < 1.0


def test_closed_form_sizes():
    assert len(gg.complete(7)[0]) == 21
    assert len(gg.king(8)[0]) == 2 * 7 * 15
    assert len(gg.wheel(6)[0]) == 12
    assert len(gg.book(4)[0]) == 9
    assert gg.disjoint_union(gg.complete(3), gg.complete(4))[2] == 7
