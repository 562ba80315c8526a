"""The back-face rule of the visibility test on the GPU: a point seen from behind on a
closed mesh, from an eye outside the mesh's box, is occluded by that mesh, and the
density kernel skips the BVH walk for it unless a triangle of the mesh near the point
could hold the entry within the visibility tolerance.  Each case against the FP64
oracle (which knows no such rule): thin and thick closed slabs (the guard), an eye
inside a closed box (the box test), the flag cleared, and the closed-mesh flags of the
workloads."""
import numpy as np
import pytest

import oracle
import parity_util
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gm():
    import torch
    import paper_2601_07571_amd as gm
    assert torch.cuda.is_available()
    gm.load_library()
    return gm


def _box(lo, hi, cells=4):
    """A closed axis-aligned box, each face split into cells x cells quads (outward
    winding), vertices shared along edges."""
    lo = np.asarray(lo, np.float64); hi = np.asarray(hi, np.float64)
    V, F, index = [], [], {}

    def vid(p):
        key = tuple(np.round(p, 12))
        if key not in index:
            index[key] = len(V)
            V.append(p)
        return index[key]
    for axis in range(3):
        u, v = [a for a in range(3) if a != axis]
        for side in (0, 1):
            for i in range(cells):
                for j in range(cells):
                    q = []
                    for di, dj in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = np.zeros(3)
                        p[axis] = hi[axis] if side else lo[axis]
                        p[u] = lo[u] + (hi[u] - lo[u]) * (i + di) / cells
                        p[v] = lo[v] + (hi[v] - lo[v]) * (j + dj) / cells
                        q.append(vid(p))
                    a, b, c, d = q
                    # outward: counter-clockwise seen from outside
                    flip = (side == 0) != ((axis % 2) == 1)
                    tris = [(a, c, b), (a, d, c)] if flip else [(a, b, c), (a, c, d)]
                    F += tris
    V = np.array(V, np.float32); F = np.array(F, np.int32)
    n = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]).astype(np.float64)
    vol = np.einsum("ij,ij->i", V[F[:, 0]].astype(np.float64), n).sum()
    if vol < 0:
        F = F[:, [0, 2, 1]]
    return V, F


def _fixations_above(rng, F, target_lo, target_hi, height):
    eye = np.zeros((F, 3)); tgt = np.zeros((F, 3))
    eye[:, :2] = rng.uniform(-0.3, 0.3, (F, 2)); eye[:, 2] = height + rng.uniform(-0.2, 0.2, F)
    tgt[:, :2] = rng.uniform(target_lo, target_hi, (F, 2))
    return eye.astype(np.float32), (tgt - eye).astype(np.float32), rng.uniform(0.1, 0.5, F).astype(np.float32)


def _map_vs_oracle(gm, meshes, k, eye, gaze, dur, theta=2.0, occlusion="full"):
    import torch
    scene = gm.Scene(meshes)
    s = scene.build_samples(k, 3)
    fix = gm.Fixations(eye, gaze, dur)
    out = scene.accumulate(s.pos, fix, theta, occlusion=occlusion, tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    st = scene.density_stats()
    pos = s.pos.cpu().numpy(); tri = s.tri.cpu().numpy(); mesh = s.mesh.cpu().numpy()
    mode = {"self": oracle.OCC_SELF, "full": oracle.OCC_FULL}[occlusion]
    ref = oracle.density(oracle.Scene(meshes), pos, tri, mesh, eye, gaze, dur, theta, mode=mode)
    d = out.density.cpu().numpy().astype(np.float64)
    parity_util.check(gm, scene, meshes, pos, tri, mesh, eye, gaze, dur, theta, mode, d, ref)
    firm, fragile, pairs = parity_util.count_flips(scene, meshes, pos, tri, mesh, eye, gaze, dur, theta, mode)
    assert firm == 0, (firm, pairs)
    return scene, st, ref, d


def test_closed_flags_of_the_workloads(gm):
    w = workloads.paper_shaped_scene()
    scene = gm.Scene([(m.V, m.I) for m in w.meshes])
    assert scene.mesh_closed().tolist() == [True, True, True, False]     # the heightfield is open
    scene.set_mesh_closed(1, False)
    assert scene.mesh_closed().tolist() == [True, False, True, False]
    scene.set_mesh_closed(1, True)
    with pytest.raises(gm.GazemapError):
        scene.set_mesh_closed(3, True)                                   # an open mesh cannot be declared closed
    V, F = _box((-0.2, -0.2, 0.0), (0.2, 0.2, 0.1))
    assert gm.Scene([(V, F)]).mesh_closed().tolist() == [True]


@pytest.mark.parametrize("thickness,rule_fires", [(5e-5, False), (5e-3, True)])
def test_slab_seen_from_above(gm, thickness, rule_fires):
    """Samples on the underside of a closed slab, eyes 1.5-2 m above it.  5 mm thick: the
    top face occludes (tau ~ 1 - 2.5e-3) and the rule settles the pairs.  0.05 mm thick:
    the top face lies inside the visibility tolerance (tau ~ 1 - 2.5e-5, visible), it is
    listed near every underside point, and the rule leaves the pairs to the walk."""
    V, F = _box((-0.2, -0.2, 0.0), (0.2, 0.2, thickness), cells=4)
    rng = np.random.default_rng(5)
    eye, gaze, dur = _fixations_above(rng, 24, -0.15, 0.15, 1.75)
    scene, st, ref, d = _map_vs_oracle(gm, [(V, F)], 4000.0, eye, gaze, dur)
    if rule_fires:
        assert st["backface"] > 0.2 * st["in_cone"], st
    else:
        assert st["backface"] < 0.01 * st["in_cone"], st
        # every underside point is seen through the top face (within the tolerance)
        assert st["visible"] > 0.9 * st["in_cone"], st


def test_eye_inside_a_closed_box(gm):
    """Eyes inside a closed box see its walls from behind and unoccluded: the rule's box
    test keeps it out, the walk answers."""
    V, F = _box((-1.0, -1.0, -1.0), (1.0, 1.0, 1.0), cells=6)
    rng = np.random.default_rng(8)
    n = 16
    eye = rng.uniform(-0.3, 0.3, (n, 3)).astype(np.float32)
    tgt = np.concatenate([rng.uniform(-0.6, 0.6, (n, 2)), np.full((n, 1), -1.0)], 1)
    gaze = (tgt - eye).astype(np.float32)
    dur = np.ones(n, np.float32)
    scene, st, ref, d = _map_vs_oracle(gm, [(V, F)], 3000.0, eye, gaze, dur)
    assert st["backface"] == 0 and st["visible"] == st["in_cone"] > 1000, st


def test_rule_off_by_flag_gives_the_oracle_map_too(gm):
    """The tiny workload with the sphere's flag cleared: no pair settled by the rule, the
    same oracle parity."""
    import torch
    w = workloads.tiny_icosphere_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    scene = gm.Scene(meshes)
    s = scene.build_samples(w.k, w.seed)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    on = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    st_on = scene.density_stats()
    scene.set_mesh_closed(0, False)
    off = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    st_off = scene.density_stats()
    assert st_on["backface"] > 0 and st_off["backface"] == 0
    assert st_off["traversals"] > st_on["traversals"]
    assert st_on["visible"] == st_off["visible"]
    pos = s.pos.cpu().numpy(); tri = s.tri.cpu().numpy(); mesh = s.mesh.cpu().numpy()
    ref = oracle.density(oracle.Scene(meshes), pos, tri, mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg,
                         mode=oracle.OCC_SELF)
    for o in (on, off):
        parity_util.check(gm, scene, meshes, pos, tri, mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg,
                          oracle.OCC_SELF, o.density.cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("lg", range(7))
def test_preparation_at_every_points_per_wave(gm, lg):
    """The back-face preparation packs 2^lg sorted points per wave, lg the largest (at most 6)
    that still leaves 4,096 waves.  Sample counts are chosen here so that every lg occurs: the
    sphere's map with its closed flag set (the rule settles pairs) against the same map with
    the flag cleared (every pair walked), which the other tests pin to the oracle.  A point
    given another point's data would settle pairs the walk finds visible."""
    import torch
    w = workloads.tiny_icosphere_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    scene = gm.Scene(meshes)
    want = int(4096 * (1 << lg) * (1.5 if lg < 6 else 2.0))
    s = scene.build_samples(want / 3.1266231, 7)
    n = int(s.pos.shape[0])
    got = 6
    while got > 0 and (n >> got) < 4096:
        got -= 1
    assert got == lg, (n, got)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    on = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    st_on = scene.density_stats()
    scene.set_mesh_closed(0, False)
    off = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    st_off = scene.density_stats()
    assert st_on["backface"] > 0.05 * st_on["in_cone"], st_on
    assert st_off["backface"] == 0
    assert st_on["in_cone"] == st_off["in_cone"]
    assert abs(st_on["visible"] - st_off["visible"]) <= 1e-4 * st_on["in_cone"], (st_on, st_off)
    a = on.density.cpu().numpy().astype(np.float64); b = off.density.cpu().numpy().astype(np.float64)
    differ = int(np.count_nonzero(a != b))
    assert differ <= max(1, int(1e-4 * n)), differ
