"""Pins for the oracle's lattice sampler, the paper's own per-triangle subdivision
(Sec. 3.1.1 Eqs. 1-3, Sec. 3.1.2 Eq. 4)."""
import math
from fractions import Fraction

import numpy as np

import oracle
import workloads


def test_point_count_is_the_lattice_size():
    """Eq. (1): (r+1)(r+2)/2 equals the number of (i, j, l) >= 0 with i + j + l = r."""
    for r in range(0, 60):
        brute = sum(1 for i in range(r + 1) for j in range(r + 1 - i))
        assert oracle.lattice_points(r) == brute


def test_row_col_matches_enumeration():
    """Eq. (2) (with the integer correction) against walking the rows one by one."""
    idx = 0
    for row in range(0, 700):
        for col in range(row + 1):
            if idx % 7 == 0 or row < 40:
                assert oracle.lattice_row_col(idx) == (row, col), idx
            idx += 1
    # large indices: the defining inequality f(row - 1) <= idx < f(row), 0 <= col <= row
    rng = np.random.default_rng(0)
    big = list(rng.integers(0, 2 ** 44, 2000)) + [oracle.lattice_points(n) - d for n in (10 ** 6, 3 * 10 ** 6)
                                                   for d in (-1, 0, 1, 2)]
    for i in big:
        i = int(i)
        row, col = oracle.lattice_row_col(i)
        below = oracle.lattice_points(row - 1) if row > 0 else 0
        assert below <= i < oracle.lattice_points(row)
        assert 0 <= col <= row and col == i - below


def _exact_resolution(k, A):
    """Eq. (4) in exact rationals: the largest whole r with f(r) <= k A, at least 1."""
    kA = Fraction(k) * Fraction(A)
    r = 1
    while Fraction((r + 2) * (r + 3), 2) <= kA:
        r += 1
    return r


def test_resolution_rule():
    # the clamp: Delta = 8 k A + 1 < 25, i.e. k A < 3, gives r = 1 (three vertices)
    assert oracle.lattice_resolution(1.0, 2.999) == 1
    assert oracle.lattice_resolution(1e-3, 1e-6) == 1
    assert oracle.lattice_resolution(5.0, 0.0) == 1
    # exact discriminants: k A = f(r) gives Delta = (2r + 3)^2 and the root r itself
    for r in range(1, 40):
        assert oracle.lattice_resolution(float(oracle.lattice_points(r)), 1.0) == r
        assert oracle.lattice_resolution(float(oracle.lattice_points(r)) - 0.25, 1.0) == max(1, r - 1)
    rng = np.random.default_rng(1)
    for _ in range(3000):
        k = float(10 ** rng.uniform(2, 6)); A = float(10 ** rng.uniform(-7, -1))
        r = oracle.lattice_resolution(k, A)
        kA = k * A
        # away from the boundaries FP64 and exact arithmetic agree
        near = any(abs(kA - oracle.lattice_points(q)) < 1e-9 * kA for q in (r, r + 1))
        if not near:
            assert r == _exact_resolution(k, A), (k, A)
        # the density bound: never more than k A points beyond the r = 1 floor
        assert oracle.lattice_points(r) <= kA or r == 1
        assert oracle.lattice_points(r + 1) > kA * (1 - 1e-12)


def test_barycentrics_enumerate_the_lattice_and_vertices_are_exact():
    V = np.array([[0.1, -0.3, 0.7], [1.9, 0.2, -0.4], [0.4, 1.3, 0.25]], np.float32)
    I = np.array([[0, 1, 2]], np.int32)
    A = oracle.triangle_areas(V, I)[0]
    for r_want in (1, 2, 5, 17):
        k = oracle.lattice_points(r_want) / A * (1 + 1e-9)
        r, cnt = oracle.lattice_counts(V, I, k)
        assert r[0] == r_want and cnt[0] == oracle.lattice_points(r_want)
        L = oracle.lattice_scene([(V, I)], k)
        assert len(L.pos32) == cnt[0]
        w2, w3 = L.bary32[:, 0].astype(np.float64), L.bary32[:, 1].astype(np.float64)
        ijl = set()
        for a, b in zip(w2, w3):
            j, l = round(a * r_want), round(b * r_want)
            assert abs(a * r_want - j) < 1e-5 and abs(b * r_want - l) < 1e-5
            ijl.add((r_want - j - l, j, l))
        lattice = {(i, j, r_want - i - j) for i in range(r_want + 1) for j in range(r_want + 1 - i)}
        assert ijl == lattice
        # the three corners land exactly on the vertices
        for v in V:
            assert np.any(np.all(L.pos32 == v, axis=1))
        # every point lies in the triangle's plane and inside it (FP64 positions)
        n = np.cross(V[1].astype(np.float64) - V[0], V[2].astype(np.float64) - V[0])
        assert np.max(np.abs((L.pos64 - V[0]) @ n)) < 1e-12


def test_positions_follow_the_completed_eq3():
    """P = w1 v0 + w2 v1 + w3 v2 with (w1, w2, w3) = (col, r - row, row - col) / r."""
    V = np.array([[0, 0, 0], [2, 0, 0], [0, 2, 0]], np.float32)
    I = np.array([[0, 1, 2]], np.int32)
    k = oracle.lattice_points(4) / 2.0 * (1 + 1e-9)   # area 2, r = 4
    L = oracle.lattice_scene([(V, I)], k)
    assert len(L.pos32) == 15
    for idx in range(15):
        row, col = oracle.lattice_row_col(idx)
        w1, w2, w3 = Fraction(col, 4), Fraction(4 - row, 4), Fraction(row - col, 4)
        want = [float(w1 * int(V[0][c]) + w2 * int(V[1][c]) + w3 * int(V[2][c])) for c in range(3)]
        assert list(L.pos64[idx]) == want


def test_icosphere_counts_and_adaptive_uniformity():
    """The tiny icosphere at 2,000 points/m^2: every face has k A in [3, 6), so r = 1 and
    the map holds 3 points per face.  On a mesh with a 16x density seam, the adaptive
    resolution keeps the points per square metre within the Eq. (4) bracket on both sides
    (Fig. 3's claim as a statistic), where one fixed resolution would not."""
    V, F = workloads.icosphere_unit(3)
    V = (0.5 * V).astype(np.float32); F = F.astype(np.int32)
    A = oracle.triangle_areas(V, F)
    assert np.all((2000 * A >= 3) & (2000 * A < 6))
    r, cnt = oracle.lattice_counts(V, F, 2000.0)
    assert np.all(r == 1) and cnt.sum() == 3 * len(F) == 3840

    hf = workloads.heightfield_mesh(size=2.0, fine=(32, 64), coarse=(8, 16), seed=3)
    Vh, Ih = hf.V.astype(np.float32), hf.I.astype(np.int32)
    Ah = oracle.triangle_areas(Vh, Ih)
    k = 40.0 / np.median(Ah)
    r, cnt = oracle.lattice_counts(Vh, Ih, k)
    fine = Ah < np.median(Ah) * 4
    coarse = ~fine
    assert fine.any() and coarse.any() and r[coarse].min() > r[fine].max()
    for sel in (fine, coarse):
        dens = cnt[sel].sum() / Ah[sel].sum()
        assert 0.5 * k < dens <= 1.05 * k
    # a single resolution for every triangle puts 16x more points per m^2 on the fine side
    fixed = oracle.lattice_points(int(np.median(r)))
    ratio = (fixed / Ah[fine].mean()) / (fixed / Ah[coarse].mean())
    assert ratio > 8


def test_scene_order_and_global_triangle_index():
    m0 = (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32), np.array([[0, 1, 2]], np.int32))
    m1 = (np.array([[0, 0, 1], [2, 0, 1], [0, 2, 1], [2, 2, 1]], np.float32), np.array([[0, 1, 2], [1, 3, 2]], np.int32))
    k = 30.0
    L = oracle.lattice_scene([m0, m1], k)
    c0 = oracle.lattice_counts(*m0, k)[1].sum(); c1 = oracle.lattice_counts(*m1, k)[1].sum()
    assert list(L.counts) == [c0, c1] and len(L.tri) == c0 + c1
    assert np.all(L.mesh[:c0] == 0) and np.all(L.mesh[c0:] == 1)
    assert np.all(L.tri[:c0] == 0) and set(L.tri[c0:]) == {1, 2}
    assert np.all(np.diff(L.tri) >= 0)
