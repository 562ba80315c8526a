"""Pins for the oracle's surface sampler (Sec. 3.1: samples proportional to area,
independent of triangulation), areas (Sec. 3.1.2) and the per-mesh counts."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads


def heron_kahan(a, b, c):
    """Heron's formula (Sec. 3.1.2) in Kahan's cancellation-free ordering a >= b >= c."""
    a, b, c = sorted([a, b, c], reverse=True)
    return 0.25 * math.sqrt((a + (b + c)) * (c - (a - b)) * (c + (a - b)) * (a + (b - c)))


def test_area_matches_heron():
    rng = np.random.default_rng(1)
    V = rng.normal(size=(300, 3)).astype(np.float32)
    I = np.arange(300, dtype=np.int32).reshape(-1, 3)
    A = oracle.triangle_areas(V, I)
    for t, (i, j, k) in enumerate(I):
        p = [V[i].astype(np.float64), V[j].astype(np.float64), V[k].astype(np.float64)]
        a = np.linalg.norm(p[1] - p[0]); b = np.linalg.norm(p[2] - p[1]); c = np.linalg.norm(p[2] - p[0])
        h = heron_kahan(a, b, c)
        assert abs(A[t] - h) <= 1e-12 * h


def test_area_closed_forms():
    V = np.array([[0, 0, 0], [3, 0, 0], [0, 4, 0], [1, 1, 1]], np.float32)
    I = np.array([[0, 1, 2], [0, 0, 3], [0, 1, 1]], np.int32)
    A = oracle.triangle_areas(V, I)
    assert A[0] == 6.0
    assert A[1] == 0.0 and A[2] == 0.0
    # regular icosahedron with circumradius 1: 20 faces of edge a, a = 1/sin(2 pi/5)
    Vi, Fi = workloads.icosphere_unit(0)
    A = oracle.triangle_areas(Vi.astype(np.float32), Fi.astype(np.int32))
    a = 1.0 / math.sin(2 * math.pi / 5)
    assert abs(A.sum() - 5 * math.sqrt(3) * a * a) < 2e-6


def test_weights_exact_integer_brute_force():
    rng = np.random.default_rng(2)
    A = rng.uniform(1e-6, 3e-3, 777)
    A[5] = 0.0
    W, C, S, tot = oracle.mesh_weights(A)
    M = max(A)
    _, e = math.frexp(len(A) * M)
    assert S == 52 - e
    run = 0
    for i, a in enumerate(A):
        w = int(math.floor(math.ldexp(a, S)))
        assert int(W[i]) == w
        run += w
        assert int(C[i]) == run
    assert tot == run < 2 ** 52
    assert W[5] == 0


def test_weights_literal_examples():
    """The integer weights written out: with n areas and the largest M, the scale is
    S = 52 - e where n M = f 2^e, f in [0.5, 1), and W_i = floor(A_i 2^S).  Binary fractions
    0.5, 0.25, 0.125 (n M = 2 = 0.5 * 2^2, S = 50) give 2^49, 2^48, 2^47; the doubles nearest
    0.3 and 0.1 (n M = 0.6, S = 52) give floor(0.29999999999999998889... * 2^52) and
    floor(0.10000000000000000555... * 2^52)."""
    W, C, S, tot = oracle.mesh_weights(np.array([0.5, 0.25, 0.125, 0.0]))
    assert S == 50
    assert [int(x) for x in W] == [562949953421312, 281474976710656, 140737488355328, 0]
    assert [int(x) for x in C] == [562949953421312, 844424930131968, 985162418487296, 985162418487296]
    assert tot == 985162418487296
    W, C, S, tot = oracle.mesh_weights(np.array([0.3, 0.1]))
    assert S == 52
    assert [int(x) for x in W] == [1351079888211148, 450359962737049]
    assert tot == 1351079888211148 + 450359962737049


def test_count_config1_is_k_times_area():
    w = workloads.tiny_icosphere_scene()
    m = w.meshes[0]
    A = oracle.triangle_areas(m.V, m.I)
    W, C, S, tot = oracle.mesh_weights(A)
    n = oracle.sample_count(tot, S, w.k)
    assert n == round(w.k * A.sum()) == 6253


def test_selection_and_placement_brute_force():
    """Linear-scan selection with exact 128-bit integers and the warp in Python floats."""
    rng = np.random.default_rng(3)
    V = rng.normal(size=(40, 3)).astype(np.float32)
    I = rng.integers(0, 40, (50, 3)).astype(np.int32)
    I[7] = [1, 1, 2]                      # zero-area triangle: never chosen
    A = oracle.triangle_areas(V, I)
    W, C, S, tot = oracle.mesh_weights(A)
    seed = 0xDEADBEEF12345678
    s = oracle.sample_scene([(V, I)], k=4000.0 / (tot * 2.0 ** -S), seed=seed)
    n = len(s.tri)
    assert n == 4000
    key = [seed & 0xFFFFFFFF, seed >> 32]
    Cl = [int(c) for c in C]
    for j in range(n):
        x = oracle.philox_py([j & 0xFFFFFFFF, j >> 32, 0, 0], key)
        U = (x[0] << 32) | x[1]
        target = (U * tot) >> 64
        t = next(i for i, c in enumerate(Cl) if c > target)
        assert s.tri[j] == t
        su = math.sqrt(x[2] / 2.0 ** 32)
        v = x[3] / 2.0 ** 32
        b1, b2, b0 = su * (1.0 - v), su * v, 1.0 - su
        assert s.bary64[j, 0] == b1 and s.bary64[j, 1] == b2
        p = [b0 * float(V[I[t, 0], c]) + b1 * float(V[I[t, 1], c]) + b2 * float(V[I[t, 2], c]) for c in range(3)]
        assert list(s.pos64[j]) == p
        assert list(s.pos32[j]) == [np.float32(q) for q in p]
    assert not np.any(s.tri == 7)


def test_two_triangle_area_ratio():
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [3, 0, 0], [3, 3, 0], [0, 0, 0]], np.float32)
    I = np.array([[0, 1, 2], [0, 1, 4]], np.int32)   # areas 0.5 and 1.5 -> ratio 1:3
    A = oracle.triangle_areas(V, I)
    assert abs(A[1] / A[0] - 3.0) < 1e-12
    n = 40000
    s = oracle.sample_scene([(V, I)], k=n / A.sum(), seed=11)
    assert len(s.tri) == n
    p = np.mean(s.tri == 0)
    assert abs(p - 0.25) < 3 * math.sqrt(0.25 * 0.75 / n)


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_per_triangle_counts_chi_square(seed):
    """Per-triangle counts are multinomial(N, A_i / A); the icosphere has unequal areas."""
    m = workloads.sphere_mesh(level=3, radius=0.5)
    A = oracle.triangle_areas(m.V, m.I)
    n_target = 150000
    s = oracle.sample_scene([(m.V, m.I)], k=n_target / A.sum(), seed=seed)
    cnt = np.bincount(s.tri, minlength=len(A))
    exp = len(s.tri) * A / A.sum()
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    p = stats.chi2.sf(chi2, len(A) - 1)
    assert p > 1e-3


def test_in_triangle_uniformity():
    V = np.array([[0, 0, 0], [2, 0, 0], [0.5, 1.5, 0]], np.float32)
    I = np.array([[0, 1, 2]], np.int32)
    A = oracle.triangle_areas(V, I)
    n = 20000
    s = oracle.sample_scene([(V, I)], k=n / A[0], seed=5)
    b1, b2 = s.bary64[:, 0], s.bary64[:, 1]
    b0 = 1.0 - (b1 + b2)
    assert np.all(b1 >= 0) and np.all(b2 >= 0) and np.all(b0 >= -1e-15)
    # uniform in a triangle: s = b1 + b2 has CDF s^2, b2 / (b1 + b2) is uniform
    ssum = b1 + b2
    assert stats.kstest(ssum, lambda x: np.clip(x, 0, 1) ** 2).pvalue > 1e-3
    assert stats.kstest(b2 / ssum, "uniform").pvalue > 1e-3
    # four midpoint sub-triangles get a quarter each
    sub = np.where(b0 >= 0.5, 0, np.where(b1 >= 0.5, 1, np.where(b2 >= 0.5, 2, 3)))
    cnt = np.bincount(sub, minlength=4)
    assert stats.chisquare(cnt).pvalue > 1e-3
    # positions are the barycentric combination
    P = (b0[:, None] * V[0].astype(np.float64) + b1[:, None] * V[1].astype(np.float64)
         + b2[:, None] * V[2].astype(np.float64))
    assert np.abs(P - s.pos64).max() < 1e-14


def test_density_independent_of_triangulation():
    """Same square surface cut into 2 or into 200 triangles: same sample count and a
    uniform spatial histogram (the paper's motivation, Sec. 3.1)."""
    def square(n):
        xs = np.linspace(0, 1, n + 1)
        X, Y = np.meshgrid(xs, xs, indexing="ij")
        V = np.stack([X, Y, np.zeros_like(X)], -1).reshape(-1, 3).astype(np.float32)
        i = np.arange(n)[:, None]; j = np.arange(n)[None, :]
        a = i * (n + 1) + j; b = (i + 1) * (n + 1) + j
        F = np.concatenate([np.stack([a, b, b + 1], -1).reshape(-1, 3), np.stack([a, b + 1, a + 1], -1).reshape(-1, 3)])
        return V, F.astype(np.int32)
    for n in (1, 10):
        V, F = square(n)
        s = oracle.sample_scene([(V, F)], k=30000.0, seed=9)
        assert len(s.tri) == 30000
        h, _, _ = np.histogram2d(s.pos64[:, 0], s.pos64[:, 1], bins=6, range=[[0, 1], [0, 1]])
        assert stats.chisquare(h.reshape(-1)).pvalue > 1e-3


def test_multi_mesh_order_and_counts():
    m1 = workloads.cube_mesh(1.0)
    m2 = workloads.sphere_mesh(level=2, radius=0.3)
    s = oracle.sample_scene([(m1.V, m1.I), (m2.V, m2.I)], k=500.0, seed=1)
    assert s.counts[0] == 3000
    assert np.all(s.mesh[:3000] == 0) and np.all(s.mesh[3000:] == 1)
    assert np.all(s.tri[3000:] >= len(m1.I))


def test_sample_at_is_one_entry_of_sample_scene():
    """sample_at draws the sample of a global index alone: the same position, scene-global
    triangle and mesh as sample_scene's entry, across the mesh boundary and at both ends."""
    m1 = workloads.cube_mesh(1.0)
    m2 = workloads.sphere_mesh(level=2, radius=0.3)
    meshes = [(m1.V, m1.I), (m2.V, m2.I)]
    s = oracle.sample_scene(meshes, k=500.0, seed=9)
    for i in (0, 1, 2999, 3000, 3001, len(s.tri) - 1):
        p, t, m = oracle.sample_at(meshes, 500.0, 9, i)
        assert np.array_equal(p, s.pos32[i]) and t == s.tri[i] and m == s.mesh[i], i
    with pytest.raises(IndexError):
        oracle.sample_at(meshes, 500.0, 9, len(s.tri))
