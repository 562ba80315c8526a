"""Incremental maps and time windows on the GPU (gm_map_*): blocks of fixations added
one after the other hold exactly the bits of one add of their union; a time window
takes the fixations that start inside it; both match the oracle over the same
fixations within the density tolerance."""
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
def tiny(gm):
    w = workloads.tiny_icosphere_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    scene = gm.Scene(meshes)
    s = scene.build_samples(w.k, seed=w.seed)
    ref_s = oracle.sample_scene(meshes, w.k, w.seed)
    return w, meshes, scene, s, ref_s


def _fix(gm, w, sel):
    return gm.Fixations(w.fix.eye[sel], w.fix.gaze[sel], w.fix.dur[sel])


def _bits(d):
    return d.density.cpu().numpy().view(np.uint32)


def test_one_block_matches_the_oracle_and_the_plain_call(gm, tiny):
    import torch
    w, meshes, scene, s, ref_s = tiny
    m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    got = m.add(fix).read()
    plain = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    ref = oracle.density(oracle.Scene(meshes), ref_s.pos32, ref_s.tri, ref_s.mesh, w.fix.eye, w.fix.gaze,
                         w.fix.dur, w.theta_deg, mode=oracle.OCC_SELF)
    d = got.density.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(d - ref.rho) <= 1e-5 * ref.rho + ref.budget + 1e-30)
    # the same kernels at another fixed-point scale: equal to the quantum of either
    p = plain.density.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(d - p) <= 1e-6 * p + 1e-9)
    assert (d > 0).sum() == (p > 0).sum()
    nm = got.density_norm.cpu().numpy()
    assert nm.max() == 1.0 and nm.min() >= 0.0
    assert m.info()["added"] == w.fix.eye.shape[0]


def test_blocks_in_any_order_hold_the_bits_of_one_add(gm, tiny):
    w, meshes, scene, s, ref_s = tiny
    F = w.fix.eye.shape[0]
    one = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    one.add(_fix(gm, w, slice(0, F)))
    a = _bits(one.read())
    inc = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    for lo, hi in ((70, 100), (0, 1), (1, 33), (33, 70)):
        inc.add(_fix(gm, w, slice(lo, hi)))
    assert np.array_equal(_bits(inc.read()), a)
    # an empty block changes nothing; a reset map fed again gives the same bits
    inc.add(_fix(gm, w, slice(0, 0)))
    assert np.array_equal(_bits(inc.read()), a)
    inc.reset()
    assert not inc.read().density.cpu().numpy().any()
    inc.add(_fix(gm, w, slice(0, F)))
    assert np.array_equal(_bits(inc.read()), a)
    assert inc.info()["added"] == F


def test_time_window_takes_the_fixations_that_start_inside(gm, tiny):
    import torch
    w, meshes, scene, s, ref_s = tiny
    t = workloads.start_times(w.fix.dur)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    tt = torch.as_tensor(t, dtype=torch.float64, device="cuda")
    win = (float(t[25]), float(t[61]))
    m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    got = m.add(fix, time=tt, window=win).read()
    torch.cuda.synchronize()
    ref = oracle.density_window(oracle.Scene(meshes), ref_s.pos32, ref_s.tri, ref_s.mesh, w.fix.eye, w.fix.gaze,
                                w.fix.dur, t, win, w.theta_deg, mode=oracle.OCC_SELF)
    d = got.density.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(d - ref.rho) <= 1e-5 * ref.rho + ref.budget + 1e-30)
    assert m.info()["added"] == 36 == oracle.in_window(t, *win).sum()
    # back-to-back windows over the recording hold the bits of the whole recording
    parts = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    edges = [-np.inf, float(t[25]), float(t[61]), float(t[62]), np.inf]
    for a, b in zip(edges[:-1], edges[1:]):
        parts.add(fix, time=tt, window=(a, b))
    whole = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    whole.add(fix)
    assert np.array_equal(_bits(parts.read()), _bits(whole.read()))
    # NaN start times are in no window
    tn = tt.clone(); tn[::2] = float("nan")
    nan_map = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    nan_map.add(fix, time=tn, window=(-np.inf, np.inf))
    assert nan_map.info()["added"] == w.fix.eye.shape[0] // 2


def test_budget_and_invalid_fixations(gm, tiny):
    import torch
    w, meshes, scene, s, ref_s = tiny
    F = w.fix.eye.shape[0]
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)   # t = 1 s each
    # a budget below one fixation takes nothing
    m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh,
                      max_total_duration=0.5)
    m.add(fix)
    info = m.info()
    assert info["added"] == 0 and info["over_budget"] == F and info["budget_used_s"] == 0.0
    assert not m.read().density.cpu().numpy().any()
    # a budget of exactly 40 fixations takes 40 of them (which ones is unspecified)
    m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh,
                      max_total_duration=40.0)
    m.add(fix)
    info = m.info()
    assert info["added"] == 40 and info["over_budget"] == F - 40 and info["budget_used_s"] == 40.0
    full = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    full.add(fix)
    part_d = m.read().density.cpu().numpy(); full_d = full.read().density.cpu().numpy()
    assert np.all(part_d <= full_d) and part_d.sum() > 0
    # invalid fixations are counted and contribute nothing
    eye = w.fix.eye.copy(); gaze = w.fix.gaze.copy(); dur = w.fix.dur.copy()
    gaze[3] = 0.0; eye[5, 1] = np.nan; dur[7] = -1.0; dur[9] = np.inf
    bad = gm.Fixations(eye, gaze, dur)
    keep = np.ones(F, bool); keep[[3, 5, 7, 9]] = False
    m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    m.add(bad)
    assert m.info()["invalid"] == 4 and m.info()["added"] == F - 4
    ok = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    ok.add(_fix(gm, w, keep))
    assert np.array_equal(_bits(m.read()), _bits(ok.read()))
    torch.cuda.synchronize()


def test_argument_errors(gm, tiny):
    w, meshes, scene, s, ref_s = tiny
    with pytest.raises(gm.GazemapError):
        gm.DensityMap(scene, s.pos, 0.0)
    with pytest.raises(gm.GazemapError):
        gm.DensityMap(scene, s.pos, 1.0, max_total_duration=0.0)
    with pytest.raises(gm.GazemapError):
        gm.DensityMap(scene, s.pos, 1.0, max_total_duration=2e9)
    m = gm.DensityMap(scene, s.pos, 1.0)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    import torch
    tt = torch.zeros(w.fix.eye.shape[0], dtype=torch.float64, device="cuda")
    with pytest.raises(gm.GazemapError):
        m.add(fix, time=tt, window=(float("nan"), 1.0))
    # an empty map reads as empty
    e = gm.DensityMap(scene, s.pos[:0], 1.0)
    e.add(fix)
    assert e.read().density.numel() == 0


def test_paper_shaped_blocks_match_the_plain_map(gm):
    """The paper-shaped workload (806k triangles, 2M samples, 6,000 fixations, full
    occlusion) fed as four uneven blocks: the same visible pairs as the plain call, values
    equal to the fixed-point quantum."""
    import torch
    w = workloads.paper_shaped_scene()
    scene = gm.Scene([(m.V, m.I) for m in w.meshes])
    s = scene.build_samples(w.k, seed=w.seed)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    plain = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="full", tri=s.tri, mesh=s.mesh)
    m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="full", tri=s.tri, mesh=s.mesh)
    F = fix.n
    for lo, hi in ((0, 1000), (1000, 1001), (1001, 4500), (4500, F)):
        m.add(fix.subset(lo, hi))
    got = m.read()
    torch.cuda.synchronize()
    d = got.density.cpu().numpy().astype(np.float64)
    p = plain.density.cpu().numpy().astype(np.float64)
    assert (d > 0).sum() == (p > 0).sum()
    assert np.all(np.abs(d - p) <= 1e-6 * p + 1e-8)
    assert m.info()["added"] == F


def test_gathered_blocks_overflow_and_large_blocks(gm, tiny):
    """Blocks wait in a buffer of 65,536 fixation records and run in one launch at the
    next read; a block that would overflow the buffer first runs what is pending, a block
    larger than the buffer runs alone.  Every split of 140,000 fixations gives the bits of
    one add of all of them, with the same counts; a reset drops pending blocks."""
    import torch
    w, meshes, scene, s, ref_s = tiny
    rng = np.random.default_rng(11)
    F = 140_000
    k = rng.integers(0, len(w.fix.eye), F)
    eye = (w.fix.eye[k] + rng.normal(0, 0.05, (F, 3))).astype(np.float32)
    gaze = (w.fix.gaze[k] + rng.normal(0, 0.05, (F, 3))).astype(np.float32)
    dur = rng.uniform(0.1, 0.5, F).astype(np.float32)
    fix = gm.Fixations(eye, gaze, dur)

    def run(sizes):
        m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh,
                          max_total_duration=1e5)
        lo = 0
        for n in sizes:
            m.add(fix.subset(lo, lo + n))
            lo += n
        assert lo == F
        return _bits(m.read()), m.info()

    one, info = run([F])                                   # larger than the buffer: alone
    assert info["added"] == F
    for sizes in ([30_000, 30_000, 30_000, 50_000],        # overflow flushes twice
                  [10_000, 70_000, 60_000],                # pending, then a large block, then pending
                  [65_536, 1, 74_463]):                    # exactly full, then overflow by one
        got, inf = run(sizes)
        assert np.array_equal(got, one), sizes
        assert inf == info, sizes
    # pending blocks are dropped by a reset; the map then holds only what follows
    m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh, max_total_duration=1e5)
    m.add(fix.subset(0, 40_000))
    m.reset()
    m.add(fix.subset(40_000, 45_000))
    a = _bits(m.read())
    m2 = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh, max_total_duration=1e5)
    b = _bits(m2.add(fix.subset(40_000, 45_000)).read())
    torch.cuda.synchronize()
    assert np.array_equal(a, b) and a.any()


def test_adds_and_read_on_different_streams(gm):
    """Blocks added on two streams and read on a third give the map of one add: each add
    records an event that the next add and the gathered launch wait for."""
    import torch
    w = workloads.tiny_icosphere_scene()
    scene = gm.Scene([(m.V, m.I) for m in w.meshes])
    s = scene.build_samples(w.k, w.seed)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    one = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    one.add(fix)
    ref = one.read()
    torch.cuda.synchronize()
    m = gm.DensityMap(scene, s.pos, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(3)]
    for k, lo in enumerate(range(0, fix.n, 25)):
        with torch.cuda.stream(streams[k % 2]):
            m.add(fix.subset(lo, min(fix.n, lo + 25)))
    with torch.cuda.stream(streams[2]):
        got = m.read()
    torch.cuda.synchronize()
    assert np.array_equal(got.density.cpu().numpy(), ref.density.cpu().numpy())
