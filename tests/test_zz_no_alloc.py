"""accumulate_density_noalloc (no device allocation inside the call; its intermediate
buffers are one fixed per-device array) against accumulate_density: the same maps bit
for bit, on two calls in a row where the second is smaller (the shared array keeps the
first call's contents), and its capacity limits refused before anything is queued."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gm():
    import torch
    import paper_2601_07571_amd as gm
    assert torch.cuda.is_available()
    gm.load_library()
    return gm


def _same(a, b):
    assert np.array_equal(a.density.cpu().numpy(), b.density.cpu().numpy())
    assert np.array_equal(a.density_norm.cpu().numpy(), b.density_norm.cpu().numpy())
    assert np.array_equal(a.max.cpu().numpy(), b.max.cpu().numpy())


def test_noalloc_equals_accumulate_density_on_two_calls(gm):
    import torch
    w = workloads.batched_sessions(n_sessions=1, seed=3, t_range=(30_000, 60_000), f_range=(1500, 3000),
                                   k_range=(6000.0, 8000.0))[0]
    scene = gm.Scene([(m.V, m.I) for m in w.meshes])
    s = scene.build_samples(w.k, w.seed)
    n = int(s.pos.shape[0])
    assert n > 5000
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    print(f"noalloc: {n} samples, {len(w.fix.eye)} fixations, scratch "
          f"{gm.load_library().gm_noalloc_scratch_bytes() / 2**20:.1f} MiB", flush=True)
    for occ in ("full", "self", "none"):
        ref = scene.accumulate(s.pos, fix, w.theta_deg, occlusion=occ, tri=s.tri, mesh=s.mesh)
        got = scene.accumulate_noalloc(s.pos, fix, w.theta_deg, occlusion=occ, tri=s.tri, mesh=s.mesh)
        torch.cuda.synchronize()
        assert float(ref.max.cpu()[0]) > 0
        _same(got, ref)
        # second call, smaller: a ragged prefix of the points and of the fixations
        m = n // 3 + 77
        sub = fix.subset(0, len(w.fix.eye) // 2 + 3)
        ref2 = scene.accumulate(s.pos[:m], sub, w.theta_deg, occlusion=occ, tri=s.tri[:m], mesh=s.mesh[:m])
        got2 = scene.accumulate_noalloc(s.pos[:m], sub, w.theta_deg, occlusion=occ, tri=s.tri[:m], mesh=s.mesh[:m])
        torch.cuda.synchronize()
        _same(got2, ref2)


def test_noalloc_limits_and_empty_inputs(gm):
    import torch
    w = workloads.tiny_icosphere_scene()
    scene = gm.Scene([(m.V, m.I) for m in w.meshes])
    s = scene.build_samples(w.k, w.seed)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    # no points, no fixations
    e = scene.accumulate_noalloc(s.pos[:0], fix, 1.0, tri=s.tri[:0])
    z = scene.accumulate_noalloc(s.pos, fix.subset(0, 0), 1.0, tri=s.tri)
    torch.cuda.synchronize()
    assert e.density.numel() == 0 and float(e.max.cpu()[0]) == 0.0
    assert float(z.density.abs().max().cpu()) == 0.0 and float(z.max.cpu()[0]) == 0.0
    # limits: refused with GM_ERR_CAPACITY, outputs untouched
    big = torch.zeros((gm.NOALLOC_MAX_POINTS + 1, 3), dtype=torch.float32, device="cuda")
    out = gm.Density(torch.full((big.shape[0],), 7.0, device="cuda"), torch.full((big.shape[0],), 7.0, device="cuda"),
                     torch.full((1,), 7.0, device="cuda"))
    with pytest.raises(gm.GazemapError) as ex:
        scene.accumulate_noalloc(big, fix, 1.0, out=out)
    assert ex.value.status == gm.GM_ERR_CAPACITY
    many = np.repeat(w.fix.eye[:1], gm.NOALLOC_MAX_FIXATIONS + 1, 0)
    fbig = gm.Fixations(many, np.repeat(w.fix.gaze[:1], len(many), 0), np.ones(len(many), np.float32))
    with pytest.raises(gm.GazemapError) as ex:
        scene.accumulate_noalloc(s.pos, fbig, 1.0, tri=s.tri)
    assert ex.value.status == gm.GM_ERR_CAPACITY
    torch.cuda.synchronize()
    assert float(out.density[:5].min().cpu()) == 7.0 and float(out.max.cpu()[0]) == 7.0
    # and the largest accepted sizes in one call agree with the plain entry point
    k = gm.NOALLOC_MAX_POINTS / 3.1266
    s2 = scene.build_samples(k, 1, capacity=gm.NOALLOC_MAX_POINTS + 100000)
    m = min(int(s2.pos.shape[0]), gm.NOALLOC_MAX_POINTS)
    ref = scene.accumulate(s2.pos[:m], fix, 1.0, occlusion="self", tri=s2.tri[:m], mesh=s2.mesh[:m])
    got = scene.accumulate_noalloc(s2.pos[:m], fix, 1.0, occlusion="self", tri=s2.tri[:m], mesh=s2.mesh[:m])
    torch.cuda.synchronize()
    assert m == gm.NOALLOC_MAX_POINTS
    _same(got, ref)
