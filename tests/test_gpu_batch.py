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
