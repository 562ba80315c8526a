"""Neural density field on the GPU against its FP64 oracle (BF16 emulated at the same
points), its training, the per-mesh gate and the plain fallback of query_density."""
import time

import numpy as np
import pytest

import oracle
from oracle import field as fo
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
    return w, meshes, scene


def _geom(scene):
    info = scene.info()
    lo = np.array(info["bbox"][:3], np.float64)
    ext = float(np.max(np.array(info["bbox"][3:], np.float32) - np.array(info["bbox"][:3], np.float32)))
    return lo, ext


def test_forward_matches_oracle(gm, tiny):
    w, meshes, scene = tiny
    f = gm.Field(scene, seed=1)
    params = fo.init_params(11).astype(np.float32)
    params[fo.N_PARAMS - 1] = 0.1
    f.set_params(params)
    rng = np.random.default_rng(0)
    lo, ext = _geom(scene)
    x = (lo + rng.uniform(0, ext, (4099, 3))).astype(np.float32)      # ragged: not a multiple of 32
    y = f.predict(x).cpu().numpy().astype(np.float64)
    ref, _ = fo.forward(params.astype(np.float64), x, lo, ext, bf=True)
    rel = np.abs(y - ref) / np.maximum(np.abs(ref), 1e-3)
    assert np.median(rel) < 2e-3 and rel.max() < 5e-2, (np.median(rel), rel.max())


def test_gradient_matches_oracle(gm, tiny):
    """Gradients of the hand-written backward kernel against the oracle (BF16 emulated):
    cosine > 0.999 overall, relative norm difference <= 1e-2, per parameter block too."""
    w, meshes, scene = tiny
    f = gm.Field(scene, seed=2)
    rng = np.random.default_rng(1)
    params = (fo.init_params(12) + rng.normal(scale=0.02, size=fo.N_PARAMS)).astype(np.float32)
    f.set_params(params)
    lo, ext = _geom(scene)
    x = (lo + rng.uniform(0, ext, (2048, 3))).astype(np.float32)
    t = rng.uniform(0, 1, 2048).astype(np.float32)
    g, loss = f.gradient(x, t)
    rl, rg, _ = fo.loss_and_grad(params.astype(np.float64), x, t, lo, ext, bf=True)
    assert abs(loss - rl) <= 2e-3 * rl
    cos = g @ rg / (np.linalg.norm(g) * np.linalg.norm(rg))
    assert cos > 0.999, cos
    assert abs(np.linalg.norm(g) - np.linalg.norm(rg)) <= 1e-2 * np.linalg.norm(rg)
    o = 0
    for name, shape in fo.SHAPES:
        k = int(np.prod(shape))
        a, b = g[o:o + k].astype(np.float64), rg[o:o + k]
        if np.linalg.norm(b) > 0:
            c = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
            assert c > 0.995, (name, c)
        o += k


def test_adam_step_matches_oracle(gm, tiny):
    """One training step with a batch drawn on the device is checked against the oracle's
    Adam update of the same gradient (one step: the signed learning rate)."""
    w, meshes, scene = tiny
    f = gm.Field(scene, seed=3)
    params = fo.init_params(13).astype(np.float32)
    f.set_params(params)
    rng = np.random.default_rng(2)
    lo, ext = _geom(scene)
    x = (lo + rng.uniform(0, ext, (1000, 3))).astype(np.float32)
    t = rng.uniform(0, 1, 1000).astype(np.float32)
    f.train(x, np.zeros(1000, np.int32), t, steps=1, batch=256, lr=1e-3, lr_final=1e-3, holdout=0.5)
    p1 = f.get_params().astype(np.float64)
    step = p1 - params.astype(np.float64)
    moved = np.abs(step) > 0
    # Adam's first step moves every parameter by lr |g| / (|g| + eps): never more than lr,
    # and lr to within FP32 rounding wherever |g| >> eps
    assert moved.mean() > 0.5
    assert np.all(np.abs(step) <= 1e-3 * (1 + 1e-4) + 1e-7)
    assert np.mean(np.abs(np.abs(step[moved]) - 1e-3) < 2e-6) > 0.98


def test_adam_steps_match_oracle_step_for_step(gm):
    """Six Adam updates with the training loop's kernel on given, changing gradients
    (ragged count, zero and tiny gradients included), each compared with the oracle's
    update iterated from the same start: moments carried over and bias corrections
    taken at each step's number, to FP32 rounding."""
    import torch
    rng = np.random.default_rng(7)
    n = 18753 + 5
    b1, b2, eps = np.float32(0.9), np.float32(0.999), np.float32(1e-8)
    p0 = rng.normal(0, 0.1, n).astype(np.float32)
    grads = rng.normal(0, 1, (6, n)).astype(np.float32) * rng.choice([1e-4, 1.0, 30.0], (6, n)).astype(np.float32)
    grads[:, :7] = 0.0
    grads[2, 7:20] = 1e-9
    lrs = np.array([3e-3, 2e-3, 1e-3, 5e-4, 1e-3, 2e-3], np.float32)
    p = torch.tensor(p0, device="cuda")
    m = torch.zeros(n, device="cuda")
    v = torch.zeros(n, device="cuda")
    rp, rm, rv = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    am = np.zeros(n)           # the first moment's running magnitude (sum of |terms|): its rounding scale
    for k in range(6):
        g = torch.tensor(grads[k], device="cuda")
        gm.adam_step(p, m, v, g, k + 1, float(lrs[k]), float(b1), float(b2), float(eps))
        g64 = grads[k].astype(np.float64)
        rp, rm, rv = fo.adam_step(rp, rm, rv, g64, k + 1, lr=float(lrs[k]), b1=float(b1), b2=float(b2),
                                  eps=float(eps))
        am = float(b1) * am + (1 - float(b1)) * np.abs(g64)
        torch.cuda.synchronize()
        assert float(g.abs().max()) == 0.0          # the gradient is cleared after the update
        gp, gmm, gv = (t.cpu().numpy().astype(np.float64) for t in (p, m, v))
        assert np.all(np.abs(gmm - rm) <= 1e-6 * am), k
        assert np.allclose(gv, rv, rtol=3e-6, atol=1e-30), k
        # an update is at most ~3.2 lr (beta1, beta2 as here), rounded to ~1e-5 of that; the
        # running parameter adds its own rounding each step.  A bias correction taken at
        # another step, or moments not carried over, moves parameters by a good part of lr.
        tol = 4e-7 * (k + 1) * np.abs(rp) + 3e-5 * float(lrs[:k + 1].sum())
        assert np.all(np.abs(gp - rp) <= tol), (k, float(np.max(np.abs(gp - rp) - tol)))


def test_training_reaches_gate_and_query_paths(gm, tiny):
    """Train on the tiny scene's map at ~300k samples; the held-out error gates the
    field; query_density answers by the field where the gate is open and by the plain
    accumulation (exactly) where it is closed."""
    import torch
    w, meshes, scene = tiny
    k = 300000 / 3.1266
    s = scene.build_samples(k, 0)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    d = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    tmax = float(d.max.cpu()[0])
    f = gm.Field(scene, seed=4)
    t0 = time.time()
    info = f.train(s.pos, s.mesh, d.density_norm, steps=1500, batch=16384, lr=3e-3, lr_final=1e-4,
                   max_rel_l2=0.05, target_max=tmax, seed=5)
    torch.cuda.synchronize()
    dt = time.time() - t0
    print(f"training: {dt:.2f} s, loss {info['loss']:.3e}, held-out rel L2 {info['rel_l2']}")
    assert np.isfinite(info["loss"]) and info["rel_l2"][0] < 0.2
    q = s.pos[:50000]
    plain, used = gm.query_density(None, scene, fix, w.theta_deg, q, tri=s.tri[:50000], mesh=s.mesh[:50000],
                                   occlusion="self", ref_max=tmax)
    assert bool(used.all())
    assert np.array_equal(plain.cpu().numpy(), (d.density[:50000] / tmax).cpu().numpy()) or \
        np.allclose(plain.cpu().numpy(), (d.density[:50000] / tmax).cpu().numpy(), rtol=1e-6, atol=0)
    fv, used = gm.query_density(f, scene, fix, w.theta_deg, q, tri=s.tri[:50000], mesh=s.mesh[:50000],
                                occlusion="self")
    if info["gate"][0]:
        assert not bool(used.any())
        assert np.allclose(fv.cpu().numpy(), f.predict(q).cpu().numpy())
    else:
        assert bool(used.all())
        assert np.allclose(fv.cpu().numpy(), plain.cpu().numpy(), rtol=1e-6)
    # a threshold of 0 closes every gate: the plain path answers everything
    f2 = gm.Field(scene, seed=6)
    info2 = f2.train(s.pos, s.mesh, d.density_norm, steps=10, batch=1024, max_rel_l2=0.0, target_max=tmax)
    assert not info2["gate"].any()
    fb, used = gm.query_density(f2, scene, fix, w.theta_deg, q, tri=s.tri[:50000], mesh=s.mesh[:50000],
                                occlusion="self")
    assert bool(used.all()) and np.allclose(fb.cpu().numpy(), plain.cpu().numpy(), rtol=1e-6)


def test_one_network_per_mesh(gm):
    """Two meshes, two networks: each point is answered by its mesh's network over that
    mesh's bounding cube, through predict (mesh ids) and query_density (triangle ids)."""
    import torch
    sph = workloads.sphere_mesh(level=2, radius=0.3, displace=0.05, seed=2)
    cube = workloads.cube_mesh(0.5)
    Vc = (cube.V + np.array([1.5, 0.2, -0.4], np.float32)).astype(np.float32)
    meshes = [(sph.V, sph.I), (Vc, cube.I)]
    scene = gm.Scene(meshes)
    f = gm.Field(scene, seed=7)
    rng = np.random.default_rng(3)
    params = np.stack([fo.init_params(21), fo.init_params(22) + rng.normal(scale=0.02, size=fo.N_PARAMS)])
    params[:, fo.N_PARAMS - 1] = [0.1, -0.2]
    params = params.astype(np.float32)
    f.set_params(params)
    assert np.array_equal(f.get_params(), params)
    xs, ids, refs = [], [], []
    for m, (V, _) in enumerate(meshes):
        lo32 = V.min(axis=0).astype(np.float32)
        ext = float(np.max(V.max(axis=0).astype(np.float32) - lo32))
        x = (lo32 + rng.uniform(0, ext, (2051 + m, 3))).astype(np.float32)
        ref, _ = fo.forward(params[m].astype(np.float64), x, lo32.astype(np.float64), ext, bf=True)
        xs.append(x); ids.append(np.full(len(x), m, np.int32)); refs.append(ref)
    x = np.concatenate(xs); ids = np.concatenate(ids); ref = np.concatenate(refs)
    perm = rng.permutation(len(x))
    x, ids, ref = x[perm], ids[perm], ref[perm]
    y = f.predict(x, mesh=ids).cpu().numpy().astype(np.float64)
    rel = np.abs(y - ref) / np.maximum(np.abs(ref), 1e-3)
    assert np.median(rel) < 2e-3 and rel.max() < 5e-2, (np.median(rel), rel.max())
    with pytest.raises(gm.GazemapError):
        f.predict(x)          # two meshes: mesh ids are required
    # query_density routes by triangle when no mesh ids are given: train so both gates open
    s = scene.build_samples(20000.0, 1)
    tgt = torch.full((s.pos.shape[0],), 0.5, device="cuda")
    info = f.train(s.pos, s.mesh, tgt, steps=800, batch=4096, lr=3e-3, lr_final=1e-4, max_rel_l2=0.1,
                   target_max=1.0, seed=9)
    assert info["gate"].all(), info
    fix = gm.Fixations(np.array([[0, 0, 3.0]], np.float32), np.array([[0, 0, -1.0]], np.float32),
                       np.array([1.0], np.float32))
    out, used = gm.query_density(f, scene, fix, 1.0, s.pos, tri=s.tri, occlusion="full")
    assert not bool(used.any())
    assert np.allclose(out.cpu().numpy(), f.predict(s.pos, mesh=s.mesh).cpu().numpy())


def test_routed_inference_in_place_and_listed(gm):
    """Routed inference reads a mesh's points in place when they are contiguous in the
    input and through an index list otherwise: every arrangement of the same points (mesh
    blocks in order, shuffled, one block beside interleaved points of no mesh, a mesh split
    in two blocks) gives every point the same bits, and those match the oracle."""
    import torch
    sph = workloads.sphere_mesh(level=2, radius=0.3, displace=0.05, seed=4)
    cube = workloads.cube_mesh(0.5)
    Vc = (cube.V + np.array([1.5, 0.2, -0.4], np.float32)).astype(np.float32)
    meshes = [(sph.V, sph.I), (Vc, cube.I)]
    scene = gm.Scene(meshes)
    f = gm.Field(scene, seed=5)
    params = np.stack([fo.init_params(31), fo.init_params(32)]).astype(np.float32)
    f.set_params(params)
    rng = np.random.default_rng(6)
    xs, refs = [], []
    for m, (V, _) in enumerate(meshes):
        lo32 = V.min(axis=0).astype(np.float32)
        ext = float(np.max(V.max(axis=0).astype(np.float32) - lo32))
        x = (lo32 + rng.uniform(0, ext, (5000 + 3000 * m, 3))).astype(np.float32)  # several route chunks
        ref, _ = fo.forward(params[m].astype(np.float64), x, lo32.astype(np.float64), ext, bf=True)
        xs.append(x); refs.append(ref)
    n0, n1 = len(xs[0]), len(xs[1])
    x = np.concatenate(xs); ids = np.concatenate([np.zeros(n0, np.int32), np.ones(n1, np.int32)])
    ref = np.concatenate(refs)
    base = f.predict(x, mesh=ids).cpu().numpy()
    rel = np.abs(base.astype(np.float64) - ref) / np.maximum(np.abs(ref), 1e-3)
    assert np.median(rel) < 2e-3 and rel.max() < 5e-2, (np.median(rel), rel.max())
    arrangements = {"shuffled": rng.permutation(n0 + n1)}
    # mesh 1's points spread over a block twice its size; the gaps hold points of no mesh
    gap = np.full(n0 + 2 * n1, -1, np.int64)
    gap[np.arange(n0)] = np.arange(n0)
    gap[n0 + 2 * np.arange(n1)] = n0 + np.arange(n1)
    arrangements["block_and_interleaved"] = gap
    # mesh 0 in two blocks with mesh 1 between them
    h = n0 // 2
    arrangements["split"] = np.concatenate([np.arange(h), n0 + np.arange(n1), np.arange(h, n0)])
    for name, order in arrangements.items():
        src = order.copy()
        xa = x[np.maximum(src, 0)]
        ia = np.where(src >= 0, ids[np.maximum(src, 0)], -1).astype(np.int32)
        out = torch.full((len(src),), -5.0, device="cuda")
        f.predict(xa, mesh=ia, out=out)
        y = out.cpu().numpy()
        assert np.array_equal(y[src >= 0], base[src[src >= 0]]), name
        assert bool((y[src < 0] == -5.0).all()), name


def test_training_and_gradient_are_bit_reproducible(gm):
    """Gradients are summed in a fixed order (per-wave slots, then slot order): two
    trainings from the same start give the same weights, errors and gates bit for bit,
    and two gradient calls the same gradient; routed inference leaves points of no mesh
    untouched."""
    import torch
    sph = workloads.sphere_mesh(level=3, radius=0.4, displace=0.05, seed=3)
    cube = workloads.cube_mesh(0.4)
    Vc = (cube.V + np.array([1.2, 0.0, 0.3], np.float32)).astype(np.float32)
    scene = gm.Scene([(sph.V, sph.I), (Vc, cube.I)])
    s = scene.build_samples(30000.0, 2)
    n = int(s.pos.shape[0])
    tgt = torch.linspace(0.0, 1.0, n, device="cuda")
    runs = []
    for _ in range(2):
        f = gm.Field(scene, seed=11)
        info = f.train(s.pos, s.mesh, tgt, steps=120, batch=3000, lr=3e-3, lr_final=1e-4, max_rel_l2=0.5,
                       target_max=1.0, seed=12)
        runs.append((f.get_params(), np.asarray(info["rel_l2"]), np.asarray(info["gate"]), info["loss"]))
        f.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][2], runs[1][2])
    assert runs[0][3] == runs[1][3]
    f = gm.Field(scene, seed=13)
    x = s.pos[:5000].cpu().numpy()
    t = tgt[:5000].cpu().numpy()
    g1, l1 = f.gradient(x, t, net=0)
    g2, l2 = f.gradient(x, t, net=0)
    assert np.array_equal(g1, g2) and l1 == l2
    # points whose mesh id is outside [0, M) are not written
    ids = s.mesh[:4096].clone()
    ids[::7] = -1
    ids[3::11] = 2
    out = torch.full((4096,), 7.0, device="cuda")
    f.predict(s.pos[:4096], mesh=ids, out=out)
    keep = (ids < 0) | (ids > 1)
    assert bool((out[keep] == 7.0).all()) and not bool((out[~keep] == 7.0).any())


def test_tiny_scene_field_meets_two_percent(gm):
    """The tiny scene's map at 2M samples (100 fixations, self occlusion), learned by the
    fixed 4 x 64 network with the benchmark's schedule (150k steps, batch 16,384, learning
    rate 5e-3 cosine to 1e-5, top band 24 cycles): held-out relative L2 at most 2 %, so the
    gate opens and query_density answers from the field.  Training is deterministic (fixed-
    order gradient and error sums), so this is the same run every time."""
    import torch
    t = workloads.tiny_icosphere_scene()
    sc = gm.Scene([(m.V, m.I) for m in t.meshes])
    s = sc.build_samples(2_000_000 / 3.1266231, 0)
    fx = gm.Fixations(t.fix.eye, t.fix.gaze, t.fix.dur)
    d = sc.accumulate(s.pos, fx, t.theta_deg, occlusion="self", tri=s.tri, mesh=s.mesh)
    f = gm.Field(sc, seed=1, max_cycles=24.0)
    info = f.train(s.pos, s.mesh, d.density_norm, steps=150000, batch=16384, lr=5e-3, lr_final=1e-5,
                   max_rel_l2=0.02, target_max=float(d.max.cpu()[0]), seed=3)
    torch.cuda.synchronize()
    assert info["rel_l2"][0] <= 0.02 and bool(info["gate"][0]), info
    out, used = gm.query_density(f, sc, fx, t.theta_deg, s.pos[:100000], tri=s.tri[:100000], occlusion="self")
    assert not bool(used.any())
    f.close()
