"""Benchmark of the density-map hot path on one MI355X.

One step = build_surface_samples (area weights, weight scan, Philox sampler) +
accumulate_density (fixation records, spatial sort, cone gate / exact value /
BVH visibility, fixed-point accumulation, maximum and normalisation) on the
paper-shaped synthetic scene: 4 meshes, 806,220 triangles, ~2M samples,
6,000 fixations, theta = 1 degree, full inter-mesh occlusion.  Inputs (scene,
BVH, fixations) are resident in HBM before the timed region.

Prints one JSON line.  `value` is fixation-sample pairs per second of the whole
step; `roofline` is for the dominant kernel (the density kernel), timed with HIP
events that the library records on its launch stream; `cpu_baseline` is the FP64
oracle timed on this host on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VALU = 157.3e12      # MI355X FP32 vector peak, FLOP/s
GATE_FLOP_PER_PAIR = 16        # 8 FMA per (sample, fixation) pair in the cone gate
K_PAPER_SHAPED = 204240.0      # samples/m^2 giving ~2,000,000 samples on the paper-shaped scene


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target wall time of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs the path on a single MI355X "
              "(the multi-GPU design is described, not launched)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2601_07571_amd as gm
    import workloads

    torch.cuda.set_device(0)
    w = workloads.paper_shaped_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    scene = gm.Scene(meshes)
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    k = K_PAPER_SHAPED
    N = int(scene.count_samples(k).sum())
    F = fix.n
    T = sum(len(I) for _, I in meshes)
    samples = scene.build_samples(k, w.seed)
    dens = gm.Density(torch.empty(N, device="cuda"), torch.empty(N, device="cuda"), torch.empty(1, device="cuda"))

    def step(occ="full"):
        scene.build_samples(k, w.seed, out=samples)
        scene.accumulate(samples.pos, fix, w.theta_deg, occlusion=occ, tri=samples.tri, mesh=samples.mesh, out=dens)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    scene.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage = {s: scene.profile_read(s) for s in ("sample", "prep", "density", "finalize")}
    scene.profile(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    pairs = float(N) * F
    dens_ms = stage["density"][0] / max(1, stage["density"][1])

    # the same step with occlusion off isolates the cone gate + exact value
    for _ in range(args.warmup):
        step("none")
    torch.cuda.synchronize()
    scene.profile(True)
    for _ in range(args.steps):
        step("none")
    torch.cuda.synchronize()
    g_ms, g_n = scene.profile_read("density")
    scene.profile(False)
    gate_ms = g_ms / max(1, g_n)
    step()
    torch.cuda.synchronize()

    achieved = GATE_FLOP_PER_PAIR * pairs / (dens_ms * 1e-3)
    out = {
        "metric": "fixation-sample pairs/s (map of 2M samples x 6k fixations)",
        "value": pairs / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper-shaped scene: displaced icosphere + cube + torus knot + two-density "
                               "heightfield, 806,220 triangles, ~2M samples, 6,000 fixations, theta 1 deg, "
                               "full occlusion",
                   "triangles": T, "samples": N, "fixations": F, "samples_per_m2": k},
        "map_time_ms": ms_step,
        "stage_ms": {s: v[0] / args.steps for s, v in stage.items()},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU, "traffic": None,
                     "kernel": "k_density (gate + exact value + visibility)", "kernel_ms": dens_ms,
                     "flop_per_pair": GATE_FLOP_PER_PAIR},
        "gate_only": {"kernel_ms": gate_ms, "pairs_per_s": pairs / (gate_ms * 1e-3),
                      "frac_fp32_peak": GATE_FLOP_PER_PAIR * pairs / (gate_ms * 1e-3) / PEAK_FP32_VALU},
        "paper_context": {"map_time_s": 6.9, "hardware": "NVIDIA GeForce GTX 1060",
                          "workload": "the paper's 800k-triangle scene, 2M samples, 6,000 fixations"},
    }

    if not args.no_cpu_baseline:
        import oracle
        d = dens.density.cpu().numpy()
        pos = samples.pos.cpu().numpy(); tri = samples.tri.cpu().numpy(); mesh = samples.mesh.cpu().numpy()
        sc = oracle.Scene(meshes)
        threads = os.cpu_count() or 1
        rng = np.random.default_rng(0)
        n_s = 64
        while True:
            pick = rng.choice(N, n_s, replace=False)
            c0 = time.perf_counter()
            oracle.density(sc, pos[pick], tri[pick], mesh[pick], w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg,
                           mode=oracle.OCC_FULL, nthreads=threads)
            dt = time.perf_counter() - c0
            if dt >= args.cpu_seconds * 0.5 or n_s >= N:
                break
            n_s = min(N, int(n_s * max(2.0, min(16.0, args.cpu_seconds / max(dt, 1e-3)))))
        out["cpu_baseline"] = {"value": n_s * float(F) / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
                               "sample": f"{n_s} random samples of {N} x all {F} fixations, full occlusion, "
                                         f"FP64, {dt:.1f} s wall"}
        del d
    print(json.dumps(out))


if __name__ == "__main__":
    main()
