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
