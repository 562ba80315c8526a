"""GPU lattice sampler (the paper's own per-triangle subdivision, Eqs. 1-4) against the
oracle: counts, triangles, meshes, barycentrics and FP32 positions bit-exact; the density
path on lattice points within the density tolerance."""
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


def _compare(gm, meshes, k):
    scene = gm.Scene(meshes)
    counts = scene.count_lattice(k)
    s = scene.build_lattice(k)
    ref = oracle.lattice_scene(meshes, k)
    assert np.array_equal(counts, ref.counts)
    assert np.array_equal(s.tri.cpu().numpy(), ref.tri)
    assert np.array_equal(s.mesh.cpu().numpy(), ref.mesh)
    assert np.array_equal(s.bary.cpu().numpy().view(np.uint32), ref.bary32.view(np.uint32))
    assert np.array_equal(s.pos.cpu().numpy().view(np.uint32), ref.pos32.view(np.uint32))
    return scene, s, ref


def test_tiny_icosphere_bit_exact(gm):
    w = workloads.tiny_icosphere_scene()
    _, s, ref = _compare(gm, [(m.V, m.I) for m in w.meshes], w.k)
    assert len(ref.tri) == 3840


def test_ragged_meshes_and_high_resolution_bit_exact(gm):
    """Uneven triangles (cube faces at r in the hundreds, a two-density heightfield, a
    torus knot), several tiles of points and a ragged tail."""
    hf = workloads.heightfield_mesh(size=2.0, fine=(32, 64), coarse=(8, 16), seed=3)
    meshes = [(workloads.cube_mesh(0.5).V, workloads.cube_mesh(0.5).I), (hf.V, hf.I),
              (lambda m: (m.V, m.I))(workloads.torus_knot_mesh(seg=37, ring=11))]
    _, s, ref = _compare(gm, meshes, 20011.5)
    assert len(ref.tri) > 100_000


def test_paper_shaped_scene_bit_exact(gm):
    """Full paper-shaped scene (~806k triangles) at its sampling rate: most faces are at
    the r = 1 floor (three points), the cube faces are subdivided hundreds of times."""
    meshes = [(m.V, m.I) for m in workloads.paper_shaped_meshes()]
    _, s, ref = _compare(gm, meshes, 204240.0)
    assert len(ref.tri) > 2_000_000


def test_capacity_and_argument_errors(gm):
    w = workloads.tiny_icosphere_scene()
    scene = gm.Scene([(m.V, m.I) for m in w.meshes])
    with pytest.raises(gm.GazemapError):
        scene.build_lattice(w.k, capacity=100)
    with pytest.raises(gm.GazemapError):
        scene.count_lattice(0.0)
    with pytest.raises(gm.GazemapError):
        scene.count_lattice(float("nan"))
    # degenerate triangles keep the r = 1 floor: three points each, all on the segment
    V = np.array([[0, 0, 0], [1, 0, 0], [0.5, 0, 0]], np.float32)
    I = np.array([[0, 1, 2], [1, 1, 1]], np.int32)
    _, s, ref = _compare(gm, [(V, I)], 1000.0)
    assert len(ref.tri) == 6


def test_density_on_lattice_points(gm):
    """accumulate_density does not care which sampler made the points: on the tiny
    scene's lattice it matches the oracle within the density tolerance."""
    import torch
    w = workloads.tiny_icosphere_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    scene, s, ref = _compare(gm, meshes, 6000.0)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    out = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    d = out.density.cpu().numpy().astype(np.float64)
    sc = oracle.Scene(meshes)
    r = oracle.density(sc, ref.pos32, ref.tri, ref.mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg,
                       mode=oracle.OCC_SELF)
    assert np.all(np.abs(d - r.rho) <= 1e-5 * r.rho + r.budget + 1e-30)
    assert (r.rho > 0).mean() > 0.05
