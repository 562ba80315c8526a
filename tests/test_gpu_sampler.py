"""GPU sampler (a1-a3) against the oracle: counts, triangles, meshes, barycentrics and
FP32 positions must be bit-exact."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gm():
    import torch
    import paper_2601_07571_amd as gm
    assert torch.cuda.is_available()
    gm.load_library()
    return gm


def _compare(gm, meshes, k, seed):
    scene = gm.Scene(meshes)
    counts = scene.count_samples(k)
    s = scene.build_samples(k, seed)
    ref = oracle.sample_scene(meshes, k, seed)
    assert np.array_equal(counts, ref.counts)
    assert np.array_equal(s.tri.cpu().numpy(), ref.tri)
    assert np.array_equal(s.mesh.cpu().numpy(), ref.mesh)
    assert np.array_equal(s.bary.cpu().numpy().view(np.uint32), ref.bary32.view(np.uint32))
    assert np.array_equal(s.pos.cpu().numpy().view(np.uint32), ref.pos32.view(np.uint32))
    return s, ref


def test_tiny_icosphere_bit_exact(gm):
    w = workloads.tiny_icosphere_scene()
    s, ref = _compare(gm, [(m.V, m.I) for m in w.meshes], w.k, w.seed)
    assert len(ref.tri) == 6253


@pytest.mark.parametrize("seed", [1, 0xFFFFFFFF00000001])
def test_multi_mesh_ragged_bit_exact(gm, seed):
    meshes = [(workloads.cube_mesh(0.5).V, workloads.cube_mesh(0.5).I),
              (lambda m: (m.V, m.I))(workloads.sphere_mesh(level=2, radius=0.3, displace=0.1, seed=3)),
              (lambda m: (m.V, m.I))(workloads.torus_knot_mesh(seg=37, ring=11))]
    _compare(gm, meshes, 12345.6, seed)


def test_paper_shaped_scene_two_million_bit_exact(gm):
    """Full size of the paper-shaped scene: ~806k triangles, ~2M samples."""
    meshes = [(m.V, m.I) for m in workloads.paper_shaped_meshes()]
    s, ref = _compare(gm, meshes, 204240.0, 0)
    assert abs(len(ref.tri) - 2_000_000) < 100


def test_single_triangle_and_zero_area_triangles(gm):
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.5, 0, 0]], np.float32)
    I = np.array([[0, 1, 2], [0, 3, 1], [1, 1, 1]], np.int32)   # two degenerate triangles
    s, ref = _compare(gm, [(V, I)], 1000.0, 7)
    assert np.all(ref.tri == 0)


def test_uneven_areas_and_an_all_degenerate_mesh(gm):
    """The triangle search starts from a per-mesh guide table of equal-width target buckets:
    one huge triangle spanning most buckets beside thousands of tiny ones packed into a few,
    and a mesh whose triangles are all degenerate (no targets, no samples)."""
    rng = np.random.default_rng(5)
    n = 5000
    base = rng.uniform(-1, 1, (n, 3)).astype(np.float32)
    tiny = np.concatenate([base, base + np.float32(1e-2) * rng.uniform(0, 1, (n, 3)).astype(np.float32),
                           base + np.float32(1e-2) * rng.uniform(0, 1, (n, 3)).astype(np.float32)])
    big = np.array([[-3, -3, 0], [3, -3, 0], [0, 3, 0]], np.float32)
    V = np.concatenate([big, tiny]).astype(np.float32)
    I = np.concatenate([np.array([[0, 1, 2]]),
                        np.stack([3 + np.arange(n), 3 + n + np.arange(n), 3 + 2 * n + np.arange(n)], 1)]).astype(np.int32)
    Vd = np.array([[0, 0, 0], [1, 1, 1], [2, 2, 2]], np.float32)   # collinear: zero area
    Id = np.array([[0, 1, 2], [2, 1, 0]], np.int32)
    s, ref = _compare(gm, [(V, I), (Vd, Id)], 3000.0, 11)
    assert ref.counts[1] == 0 and (ref.tri > 0).any() and (ref.tri == 0).any()


def test_capacity_and_argument_errors(gm):
    w = workloads.tiny_icosphere_scene()
    scene = gm.Scene([(m.V, m.I) for m in w.meshes])
    with pytest.raises(gm.GazemapError) as e:
        scene.build_samples(w.k, 0, capacity=100)
    assert e.value.status == -4
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(gm.GazemapError):
            scene.count_samples(bad)
    with pytest.raises(gm.GazemapError):
        gm.Scene([(w.meshes[0].V, w.meshes[0].I + 10_000)])


def test_fp64_sqrt_is_correctly_rounded(gm):
    """The canonical area and the square-root warp need the device's FP64 square root
    correctly rounded for bit-exact positions.  1e8 inputs against the host's IEEE sqrt:
    the warp's own inputs k * 2^-32 for random 32-bit k, positive doubles over the whole
    exponent range (subnormals included), squares and their neighbours (where a faithful
    but not correctly rounded root would show), and the special values."""
    import torch
    rng = np.random.default_rng(7)
    per = 25_000_000
    special = np.array([0.0, -0.0, 5e-324, 2.2250738585072014e-308, 1.0, 4.0, 2.0, 0.5, 1.7976931348623157e308,
                        np.inf, 2.0 ** -1074 * 3, 1.0 - 2.0 ** -53], np.float64)
    for part in range(4):
        if part == 0:
            x = rng.integers(0, 2 ** 32, per, dtype=np.uint64).astype(np.float64) * 2.0 ** -32
        elif part == 1:
            bits = rng.integers(1, 0x7FF0000000000000, per, dtype=np.uint64)
            x = bits.view(np.float64)
        elif part == 2:
            r = rng.uniform(1.0, 2.0 ** 26, per)
            sq = r * r
            x = (sq.view(np.uint64) + rng.integers(-2, 3, per).astype(np.int64).view(np.uint64)).view(np.float64)
        else:
            x = np.concatenate([special, rng.uniform(0.0, 1e-3, per - len(special)) ** 2])
        got = gm.sqrt_f64(torch.from_numpy(x)).cpu().numpy()
        want = np.sqrt(x)
        bad = got.view(np.uint64) != want.view(np.uint64)
        assert not bad.any(), (part, int(bad.sum()), x[bad][:5], got[bad][:5], want[bad][:5])
