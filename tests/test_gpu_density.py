"""GPU density path (a4-a7) against the FP64 oracle.

Tolerance (from the FP32 arithmetic of the exact path): per sample
|rho_gpu - rho_oracle| <= 1e-5 * rho_oracle + B_s, where B_s is the oracle's sum of g
over the sample's pairs whose cone decision sits within 1e-5 of the 4-sigma boundary
or whose visibility decision is within the bookkeeping tolerances of flipping.
Visibility disagreements must stay <= 1e-4 of the in-cone pairs."""
import numpy as np
import pytest

import oracle
import parity_util
import workloads

pytestmark = pytest.mark.gpu

REL = 1e-5


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
    s = scene.build_samples(w.k, w.seed)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    ref_s = oracle.sample_scene(meshes, w.k, w.seed)
    return w, meshes, scene, s, fix, ref_s


def _parity(got, ref, rel=REL):
    got = np.asarray(got, np.float64)
    err = np.abs(got - ref.rho)
    ok = err <= rel * ref.rho + ref.budget + 1e-30
    clean = (ref.budget == 0) & (ref.rho > 0)
    worst = float(np.max(err[clean] / ref.rho[clean])) if clean.any() else 0.0
    return ok, worst


@pytest.mark.parametrize("occ", ["none", "self", "full"])
def test_tiny_density_parity(gm, tiny, occ):
    import torch
    w, meshes, scene, s, fix, ref_s = tiny
    out = scene.accumulate(s.pos, fix, w.theta_deg, occlusion=occ, tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    sc = oracle.Scene(meshes)
    ref = oracle.density(sc, ref_s.pos32, ref_s.tri, ref_s.mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg,
                         mode={"none": oracle.OCC_NONE, "self": oracle.OCC_SELF, "full": oracle.OCC_FULL}[occ])
    ok, worst = _parity(out.density.cpu().numpy(), ref)
    assert ok.all(), f"{(~ok).sum()} samples outside tolerance, worst clean rel err {worst:.2e}"
    assert worst <= REL
    # normalisation: max = max rho, rho_hat = rho / max
    d = out.density.cpu().numpy().astype(np.float64)
    mx = float(out.max.cpu().numpy()[0])
    assert mx == np.float32(d.max())
    dn = out.density_norm.cpu().numpy()
    assert dn.max() == 1.0 and dn.min() >= 0.0
    assert np.allclose(dn, d / d.max(), rtol=1e-6, atol=1e-7)
    ref_n, ref_max = oracle.normalize(ref.rho)
    assert abs(mx - ref_max) <= REL * ref_max + ref.budget.max()


def test_pair_values_stage(gm, tiny):
    """Every (sample, fixation) pair of the tiny scene: the exact-path value."""
    import torch
    w, meshes, scene, s, fix, ref_s = tiny
    N, F = len(ref_s.tri), len(w.fix.eye)
    ps = np.repeat(np.arange(N), F); pf = np.tile(np.arange(F), N)
    g = gm.pair_values(s.pos, fix, w.theta_deg, ps, pf).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    rg, margin, inside = oracle.pair_values(ref_s.pos32, w.fix.eye, w.fix.gaze, w.fix.dur, ps, pf, w.theta_deg)
    amb = np.abs(margin) < 1e-5
    firm = ~amb
    assert np.all((g[firm] > 0) == inside[firm])
    rel = np.abs(g[firm & inside] - rg[firm & inside]) / rg[firm & inside]
    assert rel.max() <= REL, rel.max()
    assert inside.sum() > 10000


def test_visibility_stage(gm, tiny):
    w, meshes, scene, s, fix, ref_s = tiny
    N, F = len(ref_s.tri), len(w.fix.eye)
    ps = np.repeat(np.arange(N), F); pf = np.tile(np.arange(F), N)
    _, _, inside = oracle.pair_values(ref_s.pos32, w.fix.eye, w.fix.gaze, w.fix.dur, ps, pf, w.theta_deg)
    ps, pf = ps[inside], pf[inside]
    sc = oracle.Scene(meshes)
    for (occ, mode), gaze in [(m, g) for m in (("self", 1), ("full", 2)) for g in (None, fix.gaze)]:
        vis = scene.pair_visibility(s.pos, fix.eye, ps, pf, occlusion=occ, tri=s.tri, mesh=s.mesh,
                                    gaze=gaze).cpu().numpy()
        rv, frag = sc.pair_visibility(ref_s.pos32, ref_s.tri, ref_s.mesh, w.fix.eye, ps, pf, mode=mode)
        dis = (vis.astype(bool) != rv)
        assert dis.sum() <= 1e-4 * len(ps) + (dis & frag).sum()
        assert (dis & ~frag).sum() == 0
        assert 0.2 < rv.mean() < 0.9


def test_paper_shaped_sampled_parity(gm):
    """Full paper-shaped workload (806k triangles, ~2M samples, 6,000 fixations, full occlusion)
    in the launch configuration the benchmark times; the oracle recomputes 30,000 seeded samples."""
    import torch
    w = workloads.paper_shaped_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    scene = gm.Scene(meshes)
    s = scene.build_samples(204240.0, w.seed)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    out = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="full", tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    d = out.density.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(123)
    pick = rng.choice(len(d), 30000, replace=False)
    hot = np.argsort(d)[-20:]                # the densest samples set the normalisation
    pick = np.unique(np.concatenate([pick, hot]))
    pos = s.pos.cpu().numpy()[pick]; tri = s.tri.cpu().numpy()[pick]; mesh = s.mesh.cpu().numpy()[pick]
    sc = oracle.Scene(meshes)
    ref = oracle.density(sc, pos, tri, mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg, mode=oracle.OCC_FULL)
    ok, worst = _parity(d[pick], ref)
    parity_util.check(gm, scene, meshes, pos, tri, mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg,
                      oracle.OCC_FULL, d[pick], ref)
    firm, fragile, pairs = parity_util.count_flips(scene, meshes, pos, tri, mesh, w.fix.eye, w.fix.gaze, w.fix.dur,
                                                   w.theta_deg, oracle.OCC_FULL)
    print(f"visibility of all {pairs} in-cone pairs: {firm} disagreements outside the oracle's fragile set, "
          f"{fragile} inside it")
    assert firm == 0
    assert worst <= REL
    assert (ref.rho > 0).mean() > 0.2
    dn = out.density_norm.cpu().numpy()
    assert dn.max() == 1.0
    assert float(out.max.cpu()[0]) == np.float32(d.max())


def test_edge_cases(gm, tiny):
    import torch
    w, meshes, scene, s, fix, ref_s = tiny
    # no samples
    e = scene.accumulate(s.pos[:0], fix, 1.0, tri=s.tri[:0])
    torch.cuda.synchronize()
    assert e.density.numel() == 0 and float(e.max.cpu()[0]) == 0.0
    # no fixations: all zero
    z = scene.accumulate(s.pos, fix.subset(0, 0), 1.0, tri=s.tri)
    assert float(z.density.abs().max().cpu()) == 0.0 and float(z.density_norm.abs().max().cpu()) == 0.0
    # ragged sizes equal the prefix of the full run
    full = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="self", tri=s.tri).density.cpu().numpy()
    for n in (1, 63, 1025, 4097):
        part = scene.accumulate(s.pos[:n], fix, w.theta_deg, occlusion="self", tri=s.tri[:n]).density.cpu().numpy()
        assert np.array_equal(part, full[:n])
    # invalid fixations (zero gaze, NaN eye, negative duration) add nothing
    eye = np.concatenate([w.fix.eye, [[0, 0, 2], [np.nan, 0, 2], [0, 0, 2]]]).astype(np.float32)
    gaze = np.concatenate([w.fix.gaze, [[0, 0, 0], [0, 0, -1], [0, 0, -1]]]).astype(np.float32)
    dur = np.concatenate([w.fix.dur, [1, 1, -1]]).astype(np.float32)
    bad = scene.accumulate(s.pos, gm.Fixations(eye, gaze, dur), w.theta_deg, occlusion="self", tri=s.tri)
    assert np.array_equal(bad.density.cpu().numpy(), full)
    # theta outside (0, 45) is rejected
    with pytest.raises(gm.GazemapError):
        scene.accumulate(s.pos, fix, 0.0, tri=s.tri)


def test_bitwise_repeatable_and_order_independent(gm, tiny):
    w, meshes, scene, s, fix, ref_s = tiny
    a = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="self", tri=s.tri).density.cpu().numpy()
    b = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="self", tri=s.tri).density.cpu().numpy()
    assert np.array_equal(a, b)
    perm = np.random.default_rng(0).permutation(len(w.fix.eye))
    fp = gm.Fixations(w.fix.eye[perm], w.fix.gaze[perm], w.fix.dur[perm])
    c = scene.accumulate(s.pos, fp, w.theta_deg, occlusion="self", tri=s.tri).density.cpu().numpy()
    assert np.array_equal(a, c)
    # samples in a different order: same values, permuted
    sp = np.random.default_rng(1).permutation(len(ref_s.tri))
    d = scene.accumulate(s.pos.cpu().numpy()[sp], fix, w.theta_deg, occlusion="self",
                         tri=s.tri.cpu().numpy()[sp]).density.cpu().numpy()
    assert np.array_equal(d, a[sp])


def test_eyes_close_to_surface(gm):
    """Eyes a few centimetres from a dense plane, oblique gazes: the tile-local cheap gate
    must hand every in-cone pair to the exact path (near-eye tiles are forced)."""
    import torch
    xs = np.linspace(-0.3, 0.3, 121)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    V = np.stack([X, Y, np.zeros_like(X)], -1).reshape(-1, 3).astype(np.float32)
    i = np.arange(120)[:, None]; j = np.arange(120)[None, :]
    a = i * 121 + j; b = (i + 1) * 121 + j
    I = np.concatenate([np.stack([a, b, b + 1], -1).reshape(-1, 3), np.stack([a, b + 1, a + 1], -1).reshape(-1, 3)])
    meshes = [(V, I.astype(np.int32))]
    scene = gm.Scene(meshes)
    s = scene.build_samples(300000.0, 5)
    rng = np.random.default_rng(9)
    F = 64
    eye = np.stack([rng.uniform(-0.2, 0.2, F), rng.uniform(-0.2, 0.2, F), rng.uniform(0.005, 0.05, F)], -1)
    tgt = np.stack([rng.uniform(-0.25, 0.25, F), rng.uniform(-0.25, 0.25, F), np.zeros(F)], -1)
    eye, gaze = eye.astype(np.float32), (tgt - eye).astype(np.float32)
    dur = rng.uniform(0.1, 0.5, F).astype(np.float32)
    for theta in (0.5, 2.0):
        out = scene.accumulate(s.pos, gm.Fixations(eye, gaze, dur), theta, occlusion="none", tri=s.tri)
        torch.cuda.synchronize()
        ref = oracle.density(None, s.pos.cpu().numpy(), None, None, eye, gaze, dur, theta, mode=oracle.OCC_NONE)
        ok, worst = _parity(out.density.cpu().numpy(), ref)
        assert ok.all(), f"theta {theta}: {(~ok).sum()} samples off"
        assert worst <= REL
        assert (ref.rho > 0).sum() > 1000


@pytest.mark.parametrize("spl", [2, 4])
def test_several_samples_per_lane(gm, tiny, spl, monkeypatch):
    """Packets of 2 or 4 sample slots per lane: parity on the tiny scene with every
    occlusion mode, and on the paper-shaped scene the same in-cone and visible pair
    counts as one slot per lane (the visibility decision of a pair must not depend on
    which slots share its packet)."""
    import torch
    w, meshes, _, s, fix, ref_s = tiny
    monkeypatch.setenv("GM_SAMPLES_PER_LANE", str(spl))
    scene = gm.Scene(meshes)
    sc = oracle.Scene(meshes)
    for occ, mode in (("none", oracle.OCC_NONE), ("self", oracle.OCC_SELF), ("full", oracle.OCC_FULL)):
        out = scene.accumulate(s.pos, fix, w.theta_deg, occlusion=occ, tri=s.tri, mesh=s.mesh)
        torch.cuda.synchronize()
        ref = oracle.density(sc, ref_s.pos32, ref_s.tri, ref_s.mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg,
                             mode=mode)
        ok, worst = _parity(out.density.cpu().numpy(), ref)
        assert ok.all() and worst <= REL, (occ, int((~ok).sum()))

    wp = workloads.paper_shaped_scene()
    big = [(m.V, m.I) for m in wp.meshes]
    fixp = gm.Fixations(wp.fix.eye, wp.fix.gaze, wp.fix.dur)
    counts = []
    for n in (1, spl):
        monkeypatch.setenv("GM_SAMPLES_PER_LANE", str(n))
        sp = gm.Scene(big)
        smp = sp.build_samples(204240.0, wp.seed)
        sp.accumulate(smp.pos, fixp, wp.theta_deg, occlusion="full", tri=smp.tri, mesh=smp.mesh)
        torch.cuda.synchronize()
        counts.append(sp.density_stats())
    assert counts[0]["in_cone"] == counts[1]["in_cone"]
    assert abs(counts[0]["visible"] - counts[1]["visible"]) <= 1e-5 * counts[0]["in_cone"]


def test_counters(gm):
    """gm_density_stats and gm_density_counters agree; visible <= in-cone; no traversal
    work without occlusion; a packet tests at most kLeafMax triangles per node visit
    and both children's leaves."""
    import ctypes
    import torch
    w = workloads.tiny_icosphere_scene()
    scene = gm.Scene([(m.V, m.I) for m in w.meshes])
    s = scene.build_samples(w.k, seed=w.seed)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    scene.accumulate(s.pos, fix, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    c = scene.density_stats()
    four = (ctypes.c_int64 * 4)()
    assert gm._lib.gm_density_stats(scene._h, four) == 0
    eight = (ctypes.c_int64 * 8)()
    assert gm._lib.gm_density_counters(scene._h, eight, 8) == 0
    assert list(four) == [c["in_cone"], c["visible"], c["traversals"], c["node_visits"]]
    assert list(eight)[:7] == list(c.values()) and eight[7] == 0
    # the tile cone test keeps some but not all (tile, fixation) pairs of the 100 fixations
    tiles = -(-int(s.pos.shape[0]) // 256)
    assert 0 < c["gate_fixations"] < tiles * fix.n
    assert 0 < c["visible"] < c["in_cone"] and c["traversals"] > 0
    assert 0 < c["backface"] < c["in_cone"] - c["visible"]      # the closed sphere's far side
    assert 0 < c["triangle_tests"] <= 2 * 4 * c["node_visits"]
    scene.accumulate(s.pos, fix, w.theta_deg, occlusion="none", tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    c0 = scene.density_stats()
    assert c0["in_cone"] == c["in_cone"] and c0["visible"] == c0["in_cone"]
    assert c0["traversals"] == c0["node_visits"] == c0["triangle_tests"] == c0["backface"] == 0


def _grid_occluder(n=8, h=0.125, z=1.0):
    """An n x n grid of quads at height z (vertices on multiples of h, exact in FP32), each
    quad split along alternating diagonals."""
    ks = np.arange(-n // 2, n // 2 + 1)
    V = np.array([[i * h, j * h, z] for j in ks for i in ks], np.float32)
    m = n + 1
    I = []
    for j in range(n):
        for i in range(n):
            a, b, c, d = j * m + i, j * m + i + 1, (j + 1) * m + i + 1, (j + 1) * m + i
            I += [[a, b, c], [a, c, d]] if (i + j) % 2 == 0 else [[a, b, d], [b, c, d]]
    return V, np.array(I, np.int32)


@pytest.mark.parametrize("eye", [(-0.875, -0.875, 0.0), (0.0625, 0.0625, 0.0)])
def test_watertight_through_vertices_and_edges(gm, eye):
    """Segments that pass exactly through a grid occluder's vertices and edge midpoints
    (sample = 2 v - e, so the segment meets v at tau = 1/2 in exact arithmetic) must be
    occluded: the watertight test leaves no gap between triangles sharing a vertex or an
    edge.  The first eye puts every segment in one direction octant (the shared-axis
    walk), the second mixes signs (per-lane axis order).  Points beside the occluder's
    shadow stay visible and match the oracle."""
    import torch
    e = np.array(eye, np.float64)
    h = 0.125
    wall = (np.array([[-3, -3, 2], [4, -3, 2], [4, 4, 2], [-3, 4, 2]], np.float32), np.array([[0, 1, 2], [0, 2, 3]], np.int32))
    meshes = [wall, _grid_occluder(h=h)]
    through = np.array([2 * np.array([(i + di) * h, (j + dj) * h, 1.0]) - e
                        for j in range(-3, 4) for i in range(-3, 4)
                        for di, dj in ((0, 0), (0.5, 0), (0, 0.5), (0.5, 0.5))], np.float32)
    assert np.array_equal(((through.astype(np.float64) + e) / 2)[:, 2], np.ones(len(through)))
    ctrl = (np.array([[-0.5, 0.875, 2], [0.875, -0.5, 2], [-0.375, -0.375, 2]], np.float32) if eye[0] < 0 else
            np.array([[1.1, 0.0, 2], [0.0, 1.1, 2], [-1.2, 0.0, 2]], np.float32))
    pos = np.concatenate([through, ctrl])
    tri = np.where(pos[:, 0] >= pos[:, 1], 0, 1).astype(np.int32)
    mesh = np.zeros(len(pos), np.int32)
    gaze = (-e + np.array([0, 0, 1.0]))[None].astype(np.float32)
    eye32 = e[None].astype(np.float32)
    scene = gm.Scene(meshes)
    fix = gm.Fixations(eye32, gaze, np.ones(1, np.float32))
    got = scene.accumulate(pos, fix, 10.0, occlusion="full", tri=tri, mesh=mesh).density.cpu().numpy()
    torch.cuda.synchronize()
    ref = oracle.density(oracle.Scene(meshes), pos, tri, mesh, eye32, gaze, np.ones(1, np.float32), 10.0,
                         mode=oracle.OCC_FULL)
    nt = len(through)
    assert np.all(ref.stats[:, 0] == 1)                  # every pair in the cone
    assert np.all(ref.rho[:nt] == 0) and np.all(got[:nt] == 0), np.nonzero(got[:nt])[0]
    assert np.all(ref.rho[nt:] > 0)
    ok, _ = _parity(got[nt:], oracle.OracleDensity(ref.rho[nt:], ref.budget[nt:], ref.stats[nt:]))
    assert ok.all()


def test_grazing_segments_match_the_oracle(gm):
    """The three edge-on pairs of golden/grazing_pairs.json (scale-up workload; an FP32
    test from the eye gave the other answer on each, see test_grazing_segments.py): on
    their 2 cm patch, the kernel's own pair test and the fused density kernel (one point,
    its fixation, full occlusion) give the oracle's verdict."""
    import torch
    from test_grazing_segments import load_cases
    d, cases = load_cases()
    for c in cases:
        V = c["tris"].reshape(-1, 3)
        I = np.arange(len(V), dtype=np.int32).reshape(-1, 3)
        scene = gm.Scene([(V, I)])
        pos = c["point"][None].astype(np.float32)
        tri = np.array([c["own"]], np.int32)
        vis = scene.pair_visibility(pos, c["eye"][None], np.zeros(1, np.int32), np.zeros(1, np.int32),
                                    occlusion="full", tri=tri, gaze=c["gaze"][None]).cpu().numpy()
        assert bool(vis[0]) == c["oracle_visible"], c["sample"]
        fix = gm.Fixations(c["eye"][None], c["gaze"][None], np.ones(1, np.float32))
        out = scene.accumulate(pos, fix, d["theta_deg"], occlusion="full", tri=tri)
        torch.cuda.synchronize()
        g, _, inside = oracle.pair_values(pos, c["eye"][None], c["gaze"][None], np.ones(1, np.float32),
                                          np.array([0]), np.array([0]), d["theta_deg"])
        assert inside[0]
        got = float(out.density.cpu()[0])
        want = float(g[0]) if c["oracle_visible"] else 0.0
        assert abs(got - want) <= 1e-5 * want, (c["sample"], got, want)
        scene.close()


def test_tuning_overrides_keep_maps_bit_identical(gm, monkeypatch):
    """The overrides read at scene creation (BVH leaf size, sample slots per lane, fixations
    per work item) change the launch, not the result: the paper-shaped geometry with fewer
    samples and fixations gives the same map bits and the same in-cone and visible counts
    under each."""
    import torch
    w = workloads.paper_shaped_scene(n_samples=100_000, F=300)
    meshes = [(m.V, m.I) for m in w.meshes]

    def run(env):
        for k in ("GM_BVH_LEAF", "GM_SAMPLES_PER_LANE", "GM_FIX_PER_CHUNK"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        scene = gm.Scene(meshes)
        s = scene.build_samples(w.k, w.seed)
        fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
        out = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="full", tri=s.tri, mesh=s.mesh)
        torch.cuda.synchronize()
        st = scene.density_stats()
        d = out.density.cpu().numpy().copy()
        scene.close()
        return d, st

    base, st0 = run({})
    assert st0["in_cone"] > 0 and 0 < st0["visible"] < st0["in_cone"] and st0["backface"] > 0
    for env in ({"GM_BVH_LEAF": "1"}, {"GM_BVH_LEAF": "2"}, {"GM_SAMPLES_PER_LANE": "2"},
                {"GM_SAMPLES_PER_LANE": "4"}, {"GM_FIX_PER_CHUNK": "37"}):
        d, st = run(env)
        assert np.array_equal(d, base), env
        assert (st["in_cone"], st["visible"]) == (st0["in_cone"], st0["visible"]), (env, st, st0)


def test_zero_direction_component_finds_the_occluder(gm):
    """Points sharing the eye's x coordinate exactly (every segment has a zero x component),
    all on one side of the eye so that their packets take the shared-octant walk, under an
    occluding plate: every in-cone pair is occluded (the oracle's answer; the walk once read
    the node copy of the other x direction for such segments and missed the plate)."""
    import torch
    quad = np.array([[-1, -1, 0], [1, -1, 0], [1, 1, 0], [-1, 1, 0]], np.float32)
    idx = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    lid = quad * np.array([0.5, 0.5, 1.0], np.float32) + np.array([0.0, 0.0, 0.5], np.float32)
    meshes = [(quad, idx), (lid, idx)]
    scene = gm.Scene(meshes)
    s = scene.build_samples(4000.0, 11)
    pos = s.pos.cpu().numpy().copy(); tri = s.tri.cpu().numpy(); mesh = s.mesh.cpu().numpy()
    sel = np.nonzero((mesh == 0) & (pos[:, 1] > 0.05) & (pos[:, 1] < 0.3))[0]
    assert len(sel) > 200
    pos = pos[sel]; pos[:, 0] = 0.25; pos[:, 2] = 0.0
    eye = np.array([[0.25, 0.0, 2.0]], np.float32)
    gaze = np.array([[0.0, 0.1, -1.0]], np.float32)
    dur = np.array([0.3], np.float32)
    fix = gm.Fixations(eye, gaze, dur)
    out = scene.accumulate(torch.from_numpy(pos).cuda(), fix, 5.0, occlusion="full",
                           tri=torch.from_numpy(tri[sel]).cuda(), mesh=torch.from_numpy(mesh[sel]).cuda())
    torch.cuda.synchronize()
    st = scene.density_stats()
    assert st["in_cone"] == len(sel) and st["traversals"] > 0, st
    assert st["visible"] == 0, st
    assert float(out.density.abs().max().cpu()) == 0.0
    ref = oracle.density(oracle.Scene(meshes), pos, tri[sel], mesh[sel], eye, gaze, dur, 5.0, mode=oracle.OCC_FULL)
    assert float(np.abs(ref.rho).max()) == 0.0
