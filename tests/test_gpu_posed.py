"""Moving objects (posed maps) and the export format on the GPU, against the oracle:
each fixation sees the meshes where their poses put them; values stay bound to each
object's own frame."""
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


@pytest.fixture(scope="module")
def posed(gm):
    w = workloads.posed_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    scene = gm.Scene(meshes)
    s = scene.build_samples(w.k, seed=w.seed)
    ref_s = oracle.sample_scene(meshes, w.k, w.seed)
    return w, meshes, scene, s, ref_s


def _check(got, ref):
    d = got.density.cpu().numpy().astype(np.float64)
    ok = np.abs(d - ref.rho) <= 1e-5 * ref.rho + ref.budget + 1e-30
    assert ok.all(), f"{(~ok).sum()} samples off; worst {np.max(np.abs(d - ref.rho) / np.maximum(ref.rho, 1e-30))}"
    return d


@pytest.mark.parametrize("mode", ["none", "self", "full"])
def test_posed_recording_matches_the_oracle(gm, posed, mode):
    import torch
    w, meshes, scene, s, ref_s = posed
    pose = w.extra["pose"]
    m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion=mode, tri=s.tri, mesh=s.mesh, posed=True)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    got = m.add_posed(fix, pose).read()
    torch.cuda.synchronize()
    assert np.array_equal(s.pos.cpu().numpy(), ref_s.pos32)
    occ = {"none": oracle.OCC_NONE, "self": oracle.OCC_SELF, "full": oracle.OCC_FULL}[mode]
    ref = oracle.posed_density(meshes, ref_s.pos32, ref_s.tri, ref_s.mesh, w.fix.eye, w.fix.gaze, w.fix.dur, pose,
                               w.theta_deg, mode=occ)
    d = _check(got, ref)
    assert (d > 0).mean() > 0.05
    assert m.info()["added"] == len(w.fix.eye)
    if mode == "full":
        # the moving plate hides part of what the other objects show on their own
        own = oracle.posed_density(meshes, ref_s.pos32, ref_s.tri, ref_s.mesh, w.fix.eye, w.fix.gaze, w.fix.dur,
                                   pose, w.theta_deg, mode=oracle.OCC_SELF)
        hidden = (ref_s.mesh != 2) & (own.rho > ref.rho + own.budget + ref.budget)
        assert hidden.sum() > 100


def test_blocks_windows_and_identity(gm, posed):
    """Blocks and time windows on a posed map hold the bits of one add; identity poses
    give the static map of the scene coordinates."""
    import torch
    w, meshes, scene, s, ref_s = posed
    pose = torch.as_tensor(w.extra["pose"], device="cuda")
    t = torch.as_tensor(w.extra["time"], dtype=torch.float64, device="cuda")
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    one = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="full", tri=s.tri, mesh=s.mesh, posed=True)
    a = one.add_posed(fix, pose).read().density.cpu().numpy().view(np.uint32)
    parts = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="full", tri=s.tri, mesh=s.mesh, posed=True)
    cut = float(w.extra["time"][17])
    parts.add_posed(fix, pose, time=t, window=(cut, np.inf))
    parts.add_posed(fix.subset(0, 17), pose[:17].contiguous())
    assert np.array_equal(parts.read().density.cpu().numpy().view(np.uint32), a)
    # identity poses: the static map of the scene as given
    eye = np.zeros((len(w.fix.eye), len(meshes), 12), np.float32)
    eye[:, :, 0] = eye[:, :, 5] = eye[:, :, 10] = 1.0
    idm = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="full", tri=s.tri, mesh=s.mesh, posed=True)
    got = idm.add_posed(fix, eye).read()
    torch.cuda.synchronize()
    ref = oracle.density(oracle.Scene(meshes), ref_s.pos32, ref_s.tri, ref_s.mesh, w.fix.eye, w.fix.gaze, w.fix.dur,
                         w.theta_deg, mode=oracle.OCC_FULL)
    _check(got, ref)


def test_invalid_poses_and_arguments(gm, posed):
    w, meshes, scene, s, ref_s = posed
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    pose = w.extra["pose"].copy()
    pose[4, 1, 1] += 0.05            # a shear on the cube at fixation 4
    pose[9, 2, 0] = np.nan           # a broken pose at fixation 9
    m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh, posed=True)
    m.add_posed(fix, pose)
    info = m.info()
    assert info["invalid"] == 2 and info["added"] == len(w.fix.eye) - 2
    keep = np.ones(len(w.fix.eye), bool); keep[[4, 9]] = False
    ok = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh, posed=True)
    ok.add_posed(gm.Fixations(w.fix.eye[keep], w.fix.gaze[keep], w.fix.dur[keep]), w.extra["pose"][keep])
    assert np.array_equal(m.read().density.cpu().numpy().view(np.uint32),
                          ok.read().density.cpu().numpy().view(np.uint32))
    with pytest.raises(gm.GazemapError):
        m.add(fix)                   # a posed map needs poses
    plain = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    with pytest.raises(gm.GazemapError):
        plain.add_posed(fix, w.extra["pose"])
    with pytest.raises(gm.GazemapError):
        gm.DensityMap(scene, s.pos, w.theta_deg, posed=True)          # no mesh ids
    with pytest.raises(gm.GazemapError):
        gm.DensityMap(scene, s.pos.flip(0), w.theta_deg, mesh=s.mesh.flip(0), posed=True)  # not grouped


def test_export_records(gm, posed):
    import torch
    w, meshes, scene, s, ref_s = posed
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="full", tri=s.tri, mesh=s.mesh, posed=True)
    dens = m.add_posed(fix, w.extra["pose"]).read()
    last = w.extra["pose"][-1]
    rec = gm.records_to_numpy(gm.export_samples(scene, s, dens, pose=last))
    torch.cuda.synchronize()
    n = int(s.pos.shape[0])
    assert rec.shape == (n,)
    assert np.array_equal(rec["value"], dens.density.cpu().numpy())
    assert np.array_equal(rec["value_norm"], dens.density_norm.cpu().numpy())
    assert np.array_equal(rec["mesh"], ref_s.mesh)
    off = np.concatenate([[0], np.cumsum([len(I) for _, I in meshes])])
    assert np.array_equal(rec["triangle"], ref_s.tri - off[ref_s.mesh])
    assert np.array_equal(rec["bary"], s.bary.cpu().numpy())
    assert np.array_equal(rec["local"], ref_s.pos32)
    for k in range(len(meshes)):
        sel = ref_s.mesh == k
        assert np.array_equal(rec["world"][sel], oracle.posed_world(ref_s.pos32[sel], last[k]))
    # each point is where its barycentrics put it on its mesh-local triangle
    V, I = meshes[1]
    sel = np.nonzero(ref_s.mesh == 1)[0][:50]
    tri = I[rec["triangle"][sel]]
    b1, b2 = rec["bary"][sel, 0], rec["bary"][sel, 1]
    P = (1 - b1 - b2)[:, None] * V[tri[:, 0]] + b1[:, None] * V[tri[:, 1]] + b2[:, None] * V[tri[:, 2]]
    assert np.allclose(P, rec["local"][sel], atol=1e-6)
    # without a pose the world is the scene's frame
    rec0 = gm.records_to_numpy(gm.export_samples(scene, s, dens))
    assert np.array_equal(rec0["world"], rec0["local"])
