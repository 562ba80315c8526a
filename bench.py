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
import math
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VALU = 157.3e12      # MI355X FP32 vector peak, FLOP/s
PEAK_HBM = 8.0e12              # MI355X HBM3E peak, bytes/s
NODE_BYTES, TRI_BYTES = 64, 48 # BVH node and triangle record sizes
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_density_traffic_paper_shaped.md")
VALU_SUMMARY = os.path.join(ROOT, "profiles", "k_density_valu_paper_shaped.md")
SIMDS = 256 * 4                # compute units x SIMDs
CLOCK_HZ = 2.4e9
VALU_CYCLES = 4                # a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles
COPY_PROBE_BYTES = 256 << 20   # the calibration copy of --traffic-probe (read and written once each)
GATE_FLOP_PER_PAIR = 16        # 8 FMA per (sample, fixation) pair in the cone gate
FIELD_FLOP_PER_POINT = 2 * (96 * 64 + 3 * 64 * 64 + 64)   # the field's four layer products and output
PEAK_BF16_MFMA = 2.5e15        # MI355X dense BF16 matrix peak, FLOP/s
K_PAPER_SHAPED = 204240.0      # samples/m^2 giving ~2,000,000 samples on the paper-shaped scene


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target wall time of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-session batched comparison")
    ap.add_argument("--no-field", action="store_true", help="skip the neural-field comparison")
    ap.add_argument("--field-steps", type=int, default=150000)
    ap.add_argument("--no-incremental", action="store_true", help="skip the incremental-map and time-window timing")
    ap.add_argument("--no-posed", action="store_true", help="skip the moving-objects timing")
    ap.add_argument("--no-zbuffer", action="store_true", help="skip the paper's z-buffer approximation")
    ap.add_argument("--no-scale-up", action="store_true",
                    help="skip the scale-up workload (5M triangles, 20M samples, 50,000 fixations)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run one plain copy of known size, then one full-occlusion step, and exit (for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path runs on a single MI355X; sharding over "
              "several GPUs is a design, not an implemented launch", file=sys.stderr)
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

    if args.traffic_probe:
        src = torch.ones(COPY_PROBE_BYTES // 4, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)   # one elementwise kernel: reads and writes COPY_PROBE_BYTES
        torch.cuda.synchronize()
        step()
        torch.cuda.synchronize()
        print("traffic probe done", file=sys.stderr)
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    scene.profile(True)
    torch.cuda.synchronize()
    # per-step HIP events on the launch stream (no host synchronisation inside the timed
    # region), for the spread of the step time
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage = {s: scene.profile_read(s) for s in ("sample", "prep", "density", "finalize")}
    scene.profile(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    per_step = np.array([a.elapsed_time(b) for a, b in evs])
    sd = float(per_step.std(ddof=1)) if len(per_step) > 1 else 0.0
    spread = {"mean_ms": float(per_step.mean()), "std_ms": sd,
              "ci95_ms": [float(per_step.mean() - 1.96 * sd / math.sqrt(len(per_step))),
                          float(per_step.mean() + 1.96 * sd / math.sqrt(len(per_step)))]}
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
    # the tile cone test skips, per tile, the fixations whose cone cannot reach it: the
    # per-sample gate runs for the (tile, fixation) pairs it keeps, on 512 samples each
    # (two per lane, the library's choice with occlusion off)
    gate_kept = scene.density_stats()["gate_fixations"]
    gate_tiles = -(-N // 512)
    gate_evaluated = float(gate_kept) * 512
    gate_frac = GATE_FLOP_PER_PAIR * gate_evaluated / (gate_ms * 1e-3) / PEAK_FP32_VALU
    step()
    torch.cuda.synchronize()
    counters = scene.density_stats()

    achieved = GATE_FLOP_PER_PAIR * pairs / (dens_ms * 1e-3)
    valu_n = measured_valu()
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
        "step_spread": spread,
        "stage_ms": {s: v[0] / args.steps for s, v in stage.items()},
        # the HBM-bound stages priced by their algorithmic bytes: sampling (a1-a3) ~72 B per
        # triangle and ~60 B per sample, finalisation (a7) 8 B read + 8 B for the maximum +
        # 8 B written per sample
        "stage_GBps": {"sample": (72.0 * T + 60.0 * N) / (stage["sample"][0] / args.steps * 1e-3) / 1e9,
                       "finalize": 24.0 * N / (stage["finalize"][0] / args.steps * 1e-3) / 1e9},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU, "traffic": measured_traffic(),
                     "kernel": "k_density (gate + exact value + visibility)", "kernel_ms": dens_ms,
                     "flop_per_pair": GATE_FLOP_PER_PAIR,
                     # the kernel's time is the BVH traversal of the in-cone segments (instruction
                     # issue of divergent packet tests), which the FLOP count above does not price:
                     # the two parts separately
                     "limiter": "BVH traversal of the in-cone segments (VALU issue of divergent packet tests)",
                     "parts": {"gate": {"kernel_ms": gate_ms, "frac_fp32_peak_evaluated": gate_frac},
                               # the instruction-issue roof the kernel actually meets: its VALU
                               # wave instructions (counted by rocprofv3 on this kernel) at 4 cycles
                               # each, against every SIMD's cycles over the kernel's time
                               "valu_issue": {"instructions": valu_n,
                                              "frac": (valu_n * VALU_CYCLES / (SIMDS * CLOCK_HZ * dens_ms * 1e-3)
                                                       if valu_n else None)},
                               "visibility": {"ms": dens_ms - gate_ms,
                                              "share_of_kernel": (dens_ms - gate_ms) / dens_ms,
                                              "rays_per_s": counters["in_cone"] / ((dens_ms - gate_ms) * 1e-3),
                                              "traversal_frac_hbm_peak":
                                                  (NODE_BYTES * counters["node_visits"] +
                                                   TRI_BYTES * counters["triangle_tests"]) /
                                                  ((dens_ms - gate_ms) * 1e-3) / PEAK_HBM}}},
        "gate_only": {"kernel_ms": gate_ms, "pairs_per_s": pairs / (gate_ms * 1e-3),
                      "tile_fixations_kept": gate_kept, "tile_fixations_total": gate_tiles * F,
                      "evaluated_pairs": gate_evaluated,
                      # 16 FLOP per pair over the pairs the per-sample gate actually evaluated
                      "frac_fp32_peak_evaluated": gate_frac},
        "visibility": {"in_cone_pairs": counters["in_cone"], "visible_pairs": counters["visible"],
                       "backface_rule_pairs": counters["backface"],
                       "rays_per_s": counters["in_cone"] / (dens_ms * 1e-3),
                       "packet_traversals": counters["traversals"], "bvh_node_visits": counters["node_visits"],
                       "triangle_tests": counters["triangle_tests"],
                       # the traversal's own memory work: one 64-byte node and one 48-byte record
                       # per wave-level visit / test, against the HBM peak
                       "traversal_bytes": NODE_BYTES * counters["node_visits"] + TRI_BYTES * counters["triangle_tests"],
                       "traversal_GBps": (NODE_BYTES * counters["node_visits"] + TRI_BYTES * counters["triangle_tests"])
                       / (dens_ms * 1e-3) / 1e9,
                       "traversal_frac_hbm_peak": (NODE_BYTES * counters["node_visits"] +
                                                   TRI_BYTES * counters["triangle_tests"]) / (dens_ms * 1e-3) / PEAK_HBM},
        "paper_context": {"map_time_s": 6.9, "hardware": "NVIDIA GeForce GTX 1060",
                          "workload": "the paper's 800k-triangle scene, 2M samples, 6,000 fixations"},
    }

    # a1 + a2 (areas, weights, their scan) do not depend on k: a scene computes them once,
    # at its first sampling call, so the step above runs only the counts and the sampler;
    # their one-time cost on a fresh scene object
    sc_w = gm.Scene(meshes)
    sc_w.profile(True)
    sc_w.count_samples(k)
    torch.cuda.synchronize()
    out["stage_ms"]["sample_weights_once_per_scene"] = sc_w.profile_read("sample")[0]
    sc_w.close()

    out["lattice"] = bench_lattice(gm, torch, args, scene, k)
    if not args.no_scale_up:
        out["scale_up"] = bench_scale_up(gm, workloads, torch, args)
    if not args.no_incremental:
        out["incremental"] = bench_incremental(gm, workloads, torch, np, args, scene, samples, fix, w, ms_step)
    if not args.no_posed:
        out["posed"] = bench_posed(gm, workloads, torch, np, args, scene, samples, fix, w, ms_step)
    if not args.no_zbuffer:
        out["zbuffer"] = bench_zbuffer(gm, torch, np, args, scene, samples, fix, w, dens, ms_step)
    if not args.no_batched:
        out["batched"] = bench_batched(gm, workloads, torch, args)
    if not args.no_field:
        out["field"] = bench_field(gm, workloads, torch, np, args, scene, samples, fix, dens, w, k)

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
        # the same oracle on one thread, on a smaller sample (~a third of the time)
        n1 = max(8, int(n_s * (args.cpu_seconds / 3.0) / (dt * threads)))
        pick = rng.choice(N, n1, replace=False)
        c0 = time.perf_counter()
        oracle.density(sc, pos[pick], tri[pick], mesh[pick], w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg,
                       mode=oracle.OCC_FULL, nthreads=1)
        dt1 = time.perf_counter() - c0
        out["cpu_baseline"]["one_thread"] = {"value": n1 * float(F) / dt1, "unit": "pairs/s", "cores": 1,
                                             "sample": f"{n1} random samples x all {F} fixations, {dt1:.1f} s wall"}
        del d
    print(json.dumps(out))


TRAFFIC_SOURCES = ("k_density.hip", "capi.cpp")   # the kernel and its launch configuration


def traffic_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2601_07571_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def summary_field(path, key):
    """A number recorded in a committed rocprofv3 summary ("- key: `value`" lines), or None
    when the density kernel or its launch configuration changed since it was taken (the
    summary's "k_density.hip + capi.cpp sha256" no longer matches)."""
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, val = line[2:].split(":", 1)
            fields[k.strip()] = val.strip().strip("`")
    if fields.get("k_density.hip + capi.cpp sha256") != traffic_sources_digest():
        return None
    try:
        return float(fields[key])
    except (KeyError, ValueError):
        return None


def measured_traffic():
    """HBM bytes per launch of the full-occlusion density kernel (FETCH_SIZE + WRITE_SIZE,
    calibrated), from the committed counter summary."""
    return summary_field(TRAFFIC_SUMMARY, "traffic bytes per launch")


def measured_valu():
    """VALU wave instructions per launch of the full-occlusion density kernel
    (SQ_INSTS_VALU), from the committed counter summary."""
    return summary_field(VALU_SUMMARY, "full-occlusion VALU instructions per launch")


def _time(fn, torch, reps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def bench_lattice(gm, torch, args, scene, k):
    """The paper's own lattice sampler on the same scene and rate: whole call (counts,
    blocking read-back, points) and its kernels alone (library stage timer)."""
    lat = scene.build_lattice(k)
    n = int(lat.pos.shape[0])
    call_ms = _time(lambda: scene.build_lattice(k, out=lat), torch, args.steps)
    scene.profile(True)
    for _ in range(args.steps):
        scene.build_lattice(k, out=lat)
    torch.cuda.synchronize()
    ms, cnt = scene.profile_read("sample")
    scene.profile(False)
    kern_ms = ms / max(1, cnt) * 2   # two timed regions per call: counts, then points
    written = n * (4 + 4 + 8 + 12)
    return {"points": n, "call_ms": call_ms, "kernels_ms": kern_ms,
            "points_per_s": n / (kern_ms * 1e-3), "output_GBps": written / (kern_ms * 1e-3) / 1e9}


def bench_scale_up(gm, workloads, torch, args):
    """The scale-up workload (25 displaced geodesic spheres of 200k triangles on a 5 x 5 grid,
    5M triangles; 50,000 fixations from 10 head walks; theta 1 degree; full occlusion): the
    map at 20M samples (pair throughput, and the in-cone segments per second of the density
    kernel as BVH rays/s), and the literal 10,000 samples/m^2 of the same scene."""
    w = workloads.scale_up_scene()
    scene = gm.Scene([(m.V, m.I) for m in w.meshes])
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    res = {"triangles": w.n_triangles, "fixations": fix.n}
    for name, k in (("n20M", w.k), ("k10000", 10000.0)):
        s = scene.build_samples(k, w.seed)
        n = int(s.pos.shape[0])
        dens = gm.Density(torch.empty(n, device="cuda"), torch.empty(n, device="cuda"), torch.empty(1, device="cuda"))

        def step():
            scene.build_samples(k, w.seed, out=s)
            scene.accumulate(s.pos, fix, w.theta_deg, occlusion="full", tri=s.tri, mesh=s.mesh, out=dens)
        step()
        torch.cuda.synchronize()
        reps = 2
        scene.profile(True)
        ms = _time(step, torch, reps)
        d_ms = scene.profile_read("density")[0] / reps
        scene.profile(False)
        st = scene.density_stats()
        res[name] = {"samples": n, "samples_per_m2": k, "map_ms": ms, "pairs_per_s": n * float(fix.n) / (ms * 1e-3),
                     "density_kernel_ms": d_ms, "in_cone_pairs": st["in_cone"], "visible_pairs": st["visible"],
                     "backface_rule_pairs": st["backface"],
                     "rays_per_s": st["in_cone"] / (d_ms * 1e-3)}
        del s, dens
    scene.close()
    return res


def bench_incremental(gm, workloads, torch, np, args, scene, samples, fix, w, plain_ms):
    """The same map fed as a growing recording (blocks of 500 fixations, each added as it
    arrives, then read), and one 300 s analysis window of the recording (start times of the
    fixations played back to back, 30 ms saccades), on an incremental map."""
    t = workloads.start_times(w.fix.dur)
    tt = torch.as_tensor(t, dtype=torch.float64, device="cuda")
    m = gm.DensityMap(scene, samples.pos, w.theta_deg, occlusion="full", tri=samples.tri, mesh=samples.mesh)
    blocks = [fix.subset(lo, min(fix.n, lo + 500)) for lo in range(0, fix.n, 500)]
    res = m.read()

    def feed():
        m.reset()
        for b in blocks:
            m.add(b)
        m.read(out=res)

    feed()
    feed_ms = _time(feed, torch, max(1, args.steps // 2))
    mid = float(t[len(t) // 2])
    win = (mid, mid + 300.0)

    def window():
        m.reset()
        m.add(fix, time=tt, window=win)
        m.read(out=res)

    window()
    win_ms = _time(window, torch, max(1, args.steps // 2))
    return {"blocks": len(blocks), "fixations_per_block": 500, "feed_ms": feed_ms, "plain_call_ms": plain_ms,
            "window_s": 300.0, "window_fixations": int(((t >= win[0]) & (t < win[1])).sum()),
            "recording_s": float(t[-1] + w.fix.dur[-1]), "window_ms": win_ms}


def bench_posed(gm, workloads, torch, np, args, scene, samples, fix, w, plain_ms):
    """The same recording with moving objects: each object of the paper-shaped scene turns
    about the vertical axis through its centre (0.05, 0.10, 0.15 rad/s; the heightfield
    stays), one pose per mesh per fixation at its start time; full occlusion between the
    moving objects.  Also the same map with identity poses (the static scene through the
    posed path) and the number of samples where it differs from the plain map."""
    t = workloads.start_times(w.fix.dur)
    M = len(w.meshes)
    pose = np.zeros((fix.n, M, 3, 4))
    for m, mesh in enumerate(w.meshes):
        c = 0.5 * (mesh.V.min(0).astype(np.float64) + mesh.V.max(0))
        rate = 0.05 * (m + 1) if m < M - 1 else 0.0
        for f in range(fix.n):
            a = rate * t[f]
            R = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])
            pose[f, m, :, :3] = R
            pose[f, m, :, 3] = c - R @ c
    pose_d = torch.as_tensor(pose.reshape(fix.n, M, 12).astype(np.float32), device="cuda")
    ident = torch.zeros_like(pose_d)
    ident[:, :, 0] = ident[:, :, 5] = ident[:, :, 10] = 1.0
    m = gm.DensityMap(scene, samples.pos, w.theta_deg, occlusion="full", tri=samples.tri, mesh=samples.mesh,
                      posed=True)
    res = m.read()

    def run(p):
        m.reset()
        m.add_posed(fix, p)
        m.read(out=res)

    run(pose_d)
    moving_ms = _time(lambda: run(pose_d), torch, max(1, args.steps // 2))
    moving = res.density.clone()
    run(ident)
    ident_ms = _time(lambda: run(ident), torch, max(1, args.steps // 2))
    plain = scene.accumulate(samples.pos, fix, w.theta_deg, occlusion="full", tri=samples.tri, mesh=samples.mesh)
    torch.cuda.synchronize()
    d, p = res.density, plain.density
    differ = int(((d - p).abs() > 1e-6 * p + 1e-8).sum())
    return {"map_ms_moving": moving_ms, "map_ms_identity_poses": ident_ms, "plain_map_ms": plain_ms,
            "samples_moved_by_motion": int(((moving - p).abs() > 1e-6 * p + 1e-8).sum()),
            "identity_vs_plain_samples_differing": differ, "samples": int(samples.pos.shape[0]),
            "meshes": M, "fixations": fix.n}


def bench_zbuffer(gm, torch, np, args, scene, samples, fix, w, dens, plain_ms):
    """The paper's own approximation on the same map (camera along the gaze, cropped to
    the 4-sigma cone, per-fixation z-buffer, depth tolerance 1 %): map time, and how far
    its normalised map lies from the exact one (relative L2, samples off by more than 10 %
    of the maximum)."""
    exact = dens.density.double().clone()
    emax = float(exact.max())
    res = {}
    for R, eps in ((64, 1e-2), (128, 1e-2), (256, 1e-2), (256, 1e-3)):
        out = scene.accumulate_zbuffer(samples.pos, fix, w.theta_deg, resolution=R, depth_eps=eps)
        ms = _time(lambda: scene.accumulate_zbuffer(samples.pos, fix, w.theta_deg, resolution=R, depth_eps=eps,
                                                    out=out), torch, max(1, args.steps // 2))
        scene.profile(True)
        scene.accumulate_zbuffer(samples.pos, fix, w.theta_deg, resolution=R, depth_eps=eps, out=out)
        torch.cuda.synchronize()
        prep_ms = scene.profile_read("prep")[0]
        dens_ms = scene.profile_read("density")[0]
        scene.profile(False)
        diff = out.density.double() - exact
        res[f"R{R}_eps{eps:g}"] = {"map_ms": ms, "zbuffer_render_ms": prep_ms, "density_ms": dens_ms,
                                   "rel_l2_vs_exact": float(diff.norm() / exact.norm()),
                                   "samples_off_by_10pct_of_max": int((diff.abs() > 0.1 * emax).sum()),
                                   "samples_gaining": int((diff > 1e-3 * emax).sum()),
                                   "samples_losing": int((diff < -1e-3 * emax).sum())}
    return {"near_m": 0.05, "far_m": 1000.0, "exact_map_ms": plain_ms, "runs": res}


def bench_batched(gm, workloads, torch, args):
    """64 independent sessions of uneven size: one persistent graph-captured launch against
    64 sequential accumulate_density calls on the same inputs (outputs are bit-equal)."""
    sessions = []
    pairs = 0.0
    for w in workloads.batched_sessions(64):
        sc = gm.Scene([(m.V, m.I) for m in w.meshes])
        sm = sc.build_samples(w.k, w.seed)
        fx = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
        sessions.append({"scene": sc, "pos": sm.pos, "tri": sm.tri, "mesh": sm.mesh, "fix": fx,
                         "theta_deg": w.theta_deg, "occlusion": "full"})
        pairs += float(sm.pos.shape[0]) * fx.n
    outs = []
    for x in sessions:
        n = int(x["pos"].shape[0])
        outs.append(gm.Density(torch.empty(n, device="cuda"), torch.empty(n, device="cuda"),
                               torch.empty(1, device="cuda")))

    def plain():
        for x, o in zip(sessions, outs):
            x["scene"].accumulate(x["pos"], x["fix"], x["theta_deg"], occlusion="full", tri=x["tri"], mesh=x["mesh"],
                                  out=o)
    plain()
    torch.cuda.synchronize()
    st = [x["scene"].density_stats() for x in sessions]   # counters of each session's call
    in_cone = float(sum(s["in_cone"] for s in st))
    plain_ms = _time(plain, torch, max(1, args.steps // 2))
    cache = os.environ.get("GM_TUNE_CACHE") or "/tmp/gazemap_tune.json"
    t0 = time.perf_counter()
    batch = gm.Batch(sessions, tune_cache=cache, tune=True)
    tune_s = time.perf_counter() - t0
    batch.run()
    batched_ms = _time(batch.run, torch, max(1, args.steps // 2))
    same = all(bool(torch.equal(a.density, b.density)) for a, b in zip(outs, batch.outputs))
    tot = {k: float(sum(s[k] for s in st)) for k in ("backface", "traversals", "node_visits", "triangle_tests")}
    walk = {"backface_rule_pairs": tot["backface"], "packet_traversals": tot["traversals"],
            "bvh_node_visits": tot["node_visits"], "triangle_tests": tot["triangle_tests"],
            "walked_pairs_per_traversal": (in_cone - tot["backface"]) / max(tot["traversals"], 1.0),
            "node_visits_per_traversal": tot["node_visits"] / max(tot["traversals"], 1.0),
            "triangle_tests_per_traversal": tot["triangle_tests"] / max(tot["traversals"], 1.0)}
    return {"sessions": 64, "pairs": pairs, "in_cone_pairs": in_cone, "visibility": walk,
            "in_cone_fraction": in_cone / pairs, "plain_sequential_ms": plain_ms, "batched_graph_ms": batched_ms,
            "speedup": plain_ms / batched_ms, "pairs_per_s": pairs / (batched_ms * 1e-3),
            "rays_per_s": in_cone / (batched_ms * 1e-3), "bit_equal_to_plain": same, "plan_and_tune_s": tune_s,
            "tile_config": batch.info()}


def bench_field(gm, workloads, torch, np, args, scene, samples, fix, dens, w, k):
    """Neural density field trained on the map of the paper-shaped scene (per-mesh gates)
    and on the tiny scene's geometry resampled to 2M points; time per frame of 2M queries
    by the field, by the plain accumulation and by query_density (field where the gate is
    open, plain elsewhere)."""
    res = {}
    tmax = float(dens.max.cpu()[0])
    field = gm.Field(scene, seed=1, max_cycles=128.0)
    t0 = time.perf_counter()
    info = field.train(samples.pos, samples.mesh, dens.density_norm, steps=args.field_steps, batch=16384, lr=3e-3,
                       lr_final=1e-5, max_rel_l2=0.02, target_max=tmax, seed=3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    q = samples.pos
    pred = torch.empty(q.shape[0], device="cuda")
    field.predict(q, mesh=samples.mesh, out=pred)
    field_ms = _time(lambda: field.predict(q, mesh=samples.mesh, out=pred), torch, args.steps)
    tmp = gm.Density(torch.empty(q.shape[0], device="cuda"), None, torch.empty(1, device="cuda"))
    plain_ms = _time(lambda: scene.accumulate(q, fix, w.theta_deg, occlusion="full", tri=samples.tri,
                                              mesh=samples.mesh, out=tmp), torch, max(1, args.steps // 2))
    qout = torch.empty(q.shape[0], device="cuda"); used = torch.empty(q.shape[0], dtype=torch.uint8, device="cuda")
    query_ms = _time(lambda: gm.query_density(field, scene, fix, w.theta_deg, q, tri=samples.tri, mesh=samples.mesh,
                                              occlusion="full", out=qout, used=used), torch, max(1, args.steps // 2))
    res["paper_shaped"] = {"points": int(q.shape[0]), "rel_l2_per_mesh": [float(x) for x in info["rel_l2"]],
                           "gate_open": [bool(x) for x in info["gate"]], "train_steps": info["steps"],
                           "train_s": train_s, "field_ms_per_frame": field_ms, "plain_ms_per_frame": plain_ms,
                           "query_density_ms_per_frame": query_ms,
                           "fallback_fraction": float(used.float().mean().cpu()),
                           "bf16_mfma_frac": FIELD_FLOP_PER_POINT * int(q.shape[0]) / (field_ms * 1e-3) / PEAK_BF16_MFMA}
    # the tiny scene's geometry and fixations at ~2M samples
    t = workloads.tiny_icosphere_scene()
    sc1 = gm.Scene([(m.V, m.I) for m in t.meshes])
    s1 = sc1.build_samples(2_000_000 / 3.1266231, 0)
    f1 = gm.Fixations(t.fix.eye, t.fix.gaze, t.fix.dur)
    d1 = sc1.accumulate(s1.pos, f1, t.theta_deg, occlusion="self", tri=s1.tri, mesh=s1.mesh)
    fl1 = gm.Field(sc1, seed=1, max_cycles=24.0)
    t0 = time.perf_counter()
    i1 = fl1.train(s1.pos, s1.mesh, d1.density_norm, steps=args.field_steps, batch=16384, lr=5e-3, lr_final=1e-5,
                   max_rel_l2=0.02, target_max=float(d1.max.cpu()[0]), seed=3)
    torch.cuda.synchronize()
    train1_s = time.perf_counter() - t0
    p1 = torch.empty(s1.pos.shape[0], device="cuda")
    fms = _time(lambda: fl1.predict(s1.pos, out=p1), torch, args.steps)
    tmp1 = gm.Density(torch.empty(s1.pos.shape[0], device="cuda"), None, torch.empty(1, device="cuda"))
    pms = _time(lambda: sc1.accumulate(s1.pos, f1, t.theta_deg, occlusion="self", tri=s1.tri, mesh=s1.mesh,
                                       out=tmp1), torch, args.steps)
    res["tiny_scene_2M"] = {"points": int(s1.pos.shape[0]), "rel_l2": float(i1["rel_l2"][0]),
                            "gate_open": bool(i1["gate"][0]), "train_steps": i1["steps"], "train_s": train1_s,
                            "field_ms_per_frame": fms, "plain_ms_per_frame": pms,
                            "bf16_mfma_frac": FIELD_FLOP_PER_POINT * int(s1.pos.shape[0]) / (fms * 1e-3) /
                            PEAK_BF16_MFMA}
    res["network"] = ("one network per mesh: 96 Fourier features (16 bands to 32 cycles per mesh-box edge; 24 on "
                      "the tiny scene) -> 4 x 64 ReLU -> softplus, bf16 MFMA")
    return res


if __name__ == "__main__":
    main()
