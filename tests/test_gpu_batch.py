"""Batched sessions in one persistent, graph-captured launch: every map equals its
plain accumulate_density call bit for bit (exact fixed-point sums), on every replay of
the graph, with eager work between replays; the autotuner's choice is cached."""
import os

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


def _sessions(gm, n=6):
    ws = workloads.batched_sessions(n_sessions=n, seed=7, t_range=(2000, 40000), f_range=(50, 2000),
                                    k_range=(2000.0, 6000.0))
    out = []
    for w in ws:
        scene = gm.Scene([(m.V, m.I) for m in w.meshes])
        s = scene.build_samples(w.k, w.seed)
        out.append({"scene": scene, "pos": s.pos, "tri": s.tri, "mesh": s.mesh,
                    "fix": gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur), "theta_deg": w.theta_deg,
                    "occlusion": "full"})
    return out


def test_batch_equals_plain_calls_on_every_replay(gm, tmp_path):
    import torch
    ss = _sessions(gm)
    plain = []
    for x in ss:
        d = x["scene"].accumulate(x["pos"], x["fix"], x["theta_deg"], occlusion="full", tri=x["tri"], mesh=x["mesh"])
        plain.append((d.density.cpu().numpy(), d.density_norm.cpu().numpy(), float(d.max.cpu()[0])))
    cache = str(tmp_path / "tune.json")
    b = gm.Batch(ss, tune_cache=cache, tune=True)
    info = b.info()
    assert info["work_items"] > 0 and info["tuned_ms"] > 0 and not info["from_cache"]
    assert os.path.exists(cache)
    for rep in range(3):
        outs = b.run()
        torch.cuda.synchronize()
        for (pd, pn, pm), o in zip(plain, outs):
            assert np.array_equal(o.density.cpu().numpy(), pd)
            assert np.array_equal(o.density_norm.cpu().numpy(), pn)
            assert float(o.max.cpu()[0]) == pm
        # eager work between replays overwrites the scenes' own scratch
        x = ss[rep % len(ss)]
        x["scene"].accumulate(x["pos"], x["fix"], x["theta_deg"], occlusion="full", tri=x["tri"])
        for o in outs:
            o.density.zero_()
        torch.cuda.synchronize()
    b2 = gm.Batch(ss, tune_cache=cache, tune=False)
    assert b2.info()["from_cache"]
    assert {k: b2.info()[k] for k in ("samples_per_lane", "fix_block", "fix_per_chunk")} == \
        {k: info[k] for k in ("samples_per_lane", "fix_block", "fix_per_chunk")}
    outs = b2.run()
    torch.cuda.synchronize()
    for (pd, pn, pm), o in zip(plain, outs):
        assert np.array_equal(o.density.cpu().numpy(), pd)


def _oracle_sessions(gm):
    """Batch-shaped sessions with theta at both ends of the 0.5-2 degree range and one
    session of >= 100k triangles and >= 5k fixations, plus uneven ones from the batch
    generator."""
    import math
    rng = np.random.default_rng(31)
    ws = []
    big = workloads.sphere_mesh(freq=72, radius=0.5, displace=0.04, seed=901, name="big")      # 103,680 tris
    ws.append(workloads.Workload("big", [big], workloads.shell_fixations(rng, [big], 5000, r_in=1.5, r_out=2.5,
                                                                         dur=(0.1, 0.5)), 1.2, 3000.0, 17, "full"))
    for th, s in ((0.5, 3), (2.0, 5)):
        w = workloads.batched_sessions(n_sessions=1, seed=s, t_range=(10_000, 60_000), f_range=(500, 3000),
                                       k_range=(4000.0, 8000.0))[0]
        w.theta_deg = th
        ws.append(w)
    ws += workloads.batched_sessions(n_sessions=3, seed=9, t_range=(10_000, 80_000), f_range=(500, 4000),
                                     k_range=(1000.0, 8000.0))
    assert min(w.theta_deg for w in ws) == 0.5 and max(w.theta_deg for w in ws) == 2.0
    out = []
    for w in ws:
        meshes = [(m.V, m.I) for m in w.meshes]
        scene = gm.Scene(meshes)
        s = scene.build_samples(w.k, w.seed)
        out.append({"scene": scene, "pos": s.pos, "tri": s.tri, "mesh": s.mesh,
                    "fix": gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur), "theta_deg": w.theta_deg,
                    "occlusion": "full", "w": w, "meshes": meshes})
    assert sum(len(m[1]) for m in out[0]["meshes"]) >= 100_000 and len(out[0]["w"].fix.eye) >= 5000
    return out


def test_batch_matches_oracle_and_every_tile_configuration(gm, tmp_path):
    """A tuned batch against the FP64 oracle: every session's seeded samples plus its
    densest ones, within the density tolerance with visibility flips accounted for.  Then
    every tile configuration the tuner can return (samples per lane x fixation block, and
    the chunk lengths), forced through the cache, gives those same maps bit for bit."""
    import json
    import torch
    import oracle
    import parity_util
    ss = _oracle_sessions(gm)
    cache = str(tmp_path / "tune.json")
    b = gm.Batch(ss, tune_cache=cache, tune=True)
    outs = b.run()
    torch.cuda.synchronize()
    ref_maps = [(o.density.cpu().numpy().copy(), o.density_norm.cpu().numpy().copy(), float(o.max.cpu()[0]))
                for o in outs]
    rng = np.random.default_rng(5)
    checked = 0
    for x, (d, dn, mx) in zip(ss, ref_maps):
        w = x["w"]
        n = len(d)
        pick = np.unique(np.concatenate([rng.choice(n, min(n, 600), replace=False), np.argsort(d)[-8:]]))
        pos = x["pos"].cpu().numpy()[pick]; tri = x["tri"].cpu().numpy()[pick]; mesh = x["mesh"].cpu().numpy()[pick]
        sc = oracle.Scene(x["meshes"])
        ref = oracle.density(sc, pos, tri, mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg, mode=oracle.OCC_FULL)
        flips, in_cone, _ = parity_util.check(gm, x["scene"], x["meshes"], pos, tri, mesh, w.fix.eye, w.fix.gaze,
                                              w.fix.dur, w.theta_deg, oracle.OCC_FULL, d[pick].astype(np.float64), ref)
        assert (ref.rho > 0).mean() > 0.05, w.name
        assert mx == np.float32(d.max()) and dn.max() == (1.0 if mx > 0 else 0.0)
        checked += len(pick)
    print(f"batch vs oracle: {len(ss)} sessions, {checked} samples checked")
    # every configuration through the cache
    key = next(iter(json.load(open(cache))))
    configs = [(spl, fb, 0) for spl in (1, 2, 4) for fb in (64, 128, 256)] + [(1, 128, 256), (2, 256, 4096)]
    for spl, fb, chunk in configs:
        with open(cache, "w") as fp:
            json.dump({key: {"spl": spl, "fb": fb, "chunk": chunk, "ms": 1.0}}, fp)
        bc = gm.Batch(ss, tune_cache=cache, tune=False)
        info = bc.info()
        assert info["from_cache"] and (info["samples_per_lane"], info["fix_block"], info["fix_per_chunk"]) == \
            (spl, fb, chunk)
        outs = bc.run()
        torch.cuda.synchronize()
        for (d, dn, mx), o in zip(ref_maps, outs):
            assert np.array_equal(o.density.cpu().numpy(), d), (spl, fb, chunk)
            assert np.array_equal(o.density_norm.cpu().numpy(), dn), (spl, fb, chunk)
        bc.close()
