#!/usr/bin/env python3
"""Benchmark of the tracking-and-fusion hot path on one MI355X.

Workload (paper scale): a synthetic 6x5x3 m room with 20 objects, 640x480 depth frames
(fx = fy = 525), a 512^3 FP32 TSDF at 1 cm with 4 cm truncation, and per frame the randomized
optimization with 3072 particles x 20 iterations at point sub-sampling rates 1/8, 1/16, 1/32
(Sec. III-B; schedule of Sec. IV-A), followed by fusion of the frame at the tracked pose.
Frame 0 is fused at the identity; each later frame starts from the previous estimate composed
with the pose-regression stand-in (ground-truth relative pose times a seeded 3 deg / 3 cm
perturbation). One step = one frame (track + fuse). All depth frames are resident in HBM before
the timed region starts.

Prints one JSON line: value = particle-point fitness evaluations per second over the whole
timed job (scoring launches' (K+1) x |S_i| samples / wall time), ms_per_step = ms per frame,
plus the roofline of the particle launch (timed live with HIP events on its stream, around the
launches of the last timed frame) and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle·point fitness evals/s + ms/frame (track+fuse) at 640×480, 3072 particles"
HBM_PEAK_GBS = 8000.0
BYTES_PER_EVAL = 32  # 8 stencil corners x 4 B (validity is carried by T, W is not read)
FUSE_BYTES_PER_VOXEL = 16   # T and W (FP32) read and written for each voxel a fusion updates
# Vector-ALU peak in lane operations per second: 256 compute units x 4 SIMDs x 16 lanes x 2.4 GHz (a
# wave of 64 lanes issues one instruction per 4 cycles on a SIMD); an FMA counts as one operation.
# The 157.3 TFLOP/s FP32 figure counts an FMA as two flops and doubles again for packed FP32.
CUS, SIMDS_PER_CU, LANES_PER_SIMD, CLOCK_HZ = 256, 4, 16, 2.4e9
VALU_CYCLES_PER_INST = 4
VALU_PEAK_TOPS = CUS * SIMDS_PER_CU * LANES_PER_SIMD * CLOCK_HZ / 1e12
# The method's vector arithmetic per sample (pose k, point x): the transform into grid coordinates
# (9 multiply-adds, the voxel size and origin folded into the pose), floor and fraction on 3 axes (6),
# the in-grid test (3), the cell index (2), the trilinear interpolation (7 lerps of a subtraction and a
# multiply-add: 14), and the absolute value converted and added to the pose's sum and count (4).
OPS_PER_EVAL = 9 + 6 + 3 + 2 + 14 + 4


def rot_err(Ra, Rb):
    """Angle of Ra^T Rb (radians)."""
    import numpy as np
    c = (np.trace(np.asarray(Ra).T @ np.asarray(Rb)) - 1.0) / 2.0
    return math.acos(max(-1.0, min(1.0, float(c))))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(frames, vol_spec, intr, n_frames, seconds, schedule="fixed"):
    """Times the FP64 oracle on a bounded sample of the same workload: it fuses frame 0, then
    tracks (3072 particles x 20 iterations, rates 1/8, 1/16, 1/32) and fuses frames 1, 2, ...
    until `seconds` have elapsed. Throughput counts the same (K+1) x |S_i| samples per iteration
    as the GPU figure."""
    import numpy as np
    import oracle
    ov = oracle.Volume(vol_spec)
    t0 = time.perf_counter()
    ov.integrate(frames["depth"](0), intr, np.eye(3), np.zeros(3))
    est = [(np.eye(3), np.zeros(3))]
    evals, done = 0, 0
    track_s = 0.0
    for t in range(1, n_frames):
        Rp, tp = est[-1]
        Rr, tr = frames["rel"][t]
        if schedule == "paper":
            prm = oracle.make_params(seed=14, frame_index=t, n_iters=20, Ks=(1024, 3072, 10240), rates=(8, 16, 32),
                                     pixel_stride=1, s1_deg=10.0, s1_m=0.10, stop_deg=0.05, stop_m=0.0005)
        else:
            prm = oracle.make_params(seed=14, frame_index=t, n_iters=20, K=3072, rates=(8, 16, 32), pixel_stride=1,
                                     s1_deg=10.0, s1_m=0.10)
        depth = frames["depth"](t)
        t1 = time.perf_counter()
        R, tt, recs = ov.track_frame(depth, intr, Rp @ Rr, Rp @ tr + tp, prm)
        ov.integrate(depth, intr, R, tt)
        track_s += time.perf_counter() - t1
        est.append((R, tt))
        evals += sum((r.n_particles + 1) * r.n_pts for r in recs)
        done += 1
        log(f"[bench] oracle frame {t}: {track_s:.1f} s so far")
        if time.perf_counter() - t0 >= seconds:
            break
    # one core: the oracle's fitness of 256 poses around the last estimate on the 1/8 view
    cores = oracle.num_threads()
    X, _ = oracle.backproject(frames["depth"](1), intr, 1)
    S8 = oracle.subsample(X, 8)
    rng = np.random.default_rng(1)
    Rp, tp = est[-1]
    poses = [oracle.compose(rng.uniform(-1, 1, 3) * math.radians(10.0), rng.uniform(-1, 1, 3) * 0.1, Rp, tp)
             for _ in range(256)]
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    ov.fitness_many(S8, poses)
    one = 256 * S8.shape[0] / (time.perf_counter() - t1)
    oracle.set_num_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": evals / track_s, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "host_logical_cpus": os.cpu_count(),
            "one_core": {"value": one, "unit": "evals/s",
                         "sample": f"FP64 fitness of 256 poses (10 deg / 10 cm box) on the 1/8 view of frame 1, "
                                   f"{S8.shape[0]} points, one thread"},
            "ms_per_frame": 1e3 * track_s / done,
            "sample": f"FP64 oracle, same sequence and schedule: fusion of frame 0, then track + fuse of frames "
                      f"1..{done} on a 512^3 volume ({track_s:.1f} s timed)"}


def adjoint_timing(vol, depth_dev, intr, R, t, n_poses=256, reps=5):
    """The adjoint (particles_score_grad: E and dE/dxi of each pose in one gather pass) beside the
    scoring kernel on the same poses: n_poses poses within +-1 deg / +-1 cm of (R, t) on the rate-1/8
    subsample of the frame's points, each timed with HIP events on the current stream (median of
    reps calls after one warm-up call)."""
    import numpy as np
    import torch
    from scipy.spatial.transform import Rotation
    import paper_2509_24236_amd as pf
    px, py, pz, n = pf.backproject(depth_dev, intr, 1)
    m = int(n[0].item())
    x, y, z = (a[:m:8].contiguous() for a in (px, py, pz))
    rng = np.random.default_rng(5)
    poses = []
    for _ in range(n_poses):
        dR = Rotation.from_rotvec(rng.uniform(-1, 1, 3) * math.radians(1.0)).as_matrix()
        poses.append((dR @ R, t + rng.uniform(-1, 1, 3) * 0.01))
    base = torch.as_tensor(np.stack([np.concatenate([Rk, tk.reshape(3, 1)], 1).reshape(12) for Rk, tk in poses]),
                           dtype=torch.float64, device=depth_dev.device)
    P32 = torch.as_tensor(pf.poses_to_f32(poses)).to(depth_dev.device)

    def timed(fn):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    g_ms = timed(lambda: pf.particles_score_grad(vol, x, y, z, base))
    s_ms = timed(lambda: pf.particles_score(vol, x, y, z, P32))
    E_g = pf.particles_score_grad(vol, x, y, z, base)[0]
    E_s = pf.particles_score(vol, x, y, z, P32)[0]
    samples = n_poses * x.numel()
    return {"poses": n_poses, "points": int(x.numel()), "adjoint_ms": g_ms, "scoring_ms": s_ms,
            "adjoint_samples_per_s": samples / (g_ms * 1e-3), "scoring_samples_per_s": samples / (s_ms * 1e-3),
            "E_bitwise_equal_to_scoring": bool(torch.equal(E_g.view(torch.int32), E_s.view(torch.int32))),
            "note": "particles_score_grad (one 256-thread workgroup per pose and point chunk, E exact as the "
                    "scoring kernel forms it, FP32 gradient sums in a fixed order) against particles_score on the "
                    "same FP32 poses, poses within 1 deg / 1 cm of the last tracked pose, rate-1/8 points"}


COUNTERS = os.path.join(ROOT, "profiles", "k_draw_score_sequence_counters.txt")
SCORE_SOURCES = ("pf_sample.hpp", "pf_score_steps.hpp", "pf_steps.hpp", "pf_draw_score.hip", "pf_internal.hpp")


def score_source_hash():
    """SHA-256 over the code (comments and blank space removed) of the sources the scoring kernel is
    compiled from, so that an edit of a comment does not invalidate the counter summary."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in SCORE_SOURCES:
        with open(os.path.join(ROOT, "paper_2509_24236_amd", "csrc", name)) as f:
            code = f.read()
        code = re.sub(r"/\*.*?\*/", " ", code, flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()


def read_counters():
    """The committed counter summary of the scoring launch, as a dict of numbers, or None when there is
    none or the scoring kernel's sources changed since it was taken."""
    if not os.path.exists(COUNTERS):
        return None
    vals = {}
    with open(COUNTERS) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("score_source_sha256") != score_source_hash():
        return None
    return {k: float(v) for k, v in vals.items() if k != "score_source_sha256"}


def roofline(avg_launch_ms, evals_per_launch):
    """Roofline of the particle-scoring launch. The launch is bound by vector-ALU issue (the counters
    show HBM traffic far below peak and the VALU busy), so `achieved` is the method's own vector
    arithmetic per sample (OPS_PER_EVAL lane operations) times the samples per launch over the
    launch's measured time, against the chip's lane-operation rate. The committed counter summary, when
    it matches the kernel's sources, adds the measured instruction issue, HBM traffic (FETCH_SIZE +
    WRITE_SIZE scaled by a plain copy's reading) and L2 figures, scaled to this run's samples per
    launch."""
    t = avg_launch_ms * 1e-3
    achieved = OPS_PER_EVAL * evals_per_launch / t / 1e12
    out = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
           "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
           "kernel": "particle launch per iteration (k_draw_score<f32, cells>: draws its K particles, then scores "
                     "them at 4 poses x 256 threads; through the cell-validity mask with compaction while the "
                     "particles are spread over more than a quarter voxel), timed with HIP events on its stream "
                     "around each of the 20 launches of the last timed frame",
           "ops_per_eval": OPS_PER_EVAL, "avg_launch_ms": avg_launch_ms, "evals_per_launch": evals_per_launch,
           "algorithmic_stencil_GBps": BYTES_PER_EVAL * evals_per_launch / t / 1e9,
           "counters": None}
    c = read_counters()
    if c:
        scale = evals_per_launch / c["evals_per_dispatch"]
        traffic_bytes = (c["fetch_kib_per_dispatch"] * c["fetch_scale"] +
                         c["write_kib_per_dispatch"] * c["write_scale"]) * 1024.0 * scale
        out["traffic"] = traffic_bytes / t / 1e9
        out["traffic_bytes_per_launch"] = traffic_bytes
        l1l2 = c["tcp_tcc_read_req_per_dispatch"] * 64.0 * scale
        hit, miss = c["tcc_hit_per_dispatch"], c["tcc_miss_per_dispatch"]
        valu = c["valu_insts_per_dispatch"] * scale
        out["counters"] = {
            "valu_issue_frac": valu * VALU_CYCLES_PER_INST / (CUS * SIMDS_PER_CU * CLOCK_HZ) / t,
            "valu_lane_insts_per_eval": c["valu_insts_per_dispatch"] * 64.0 / c["evals_per_dispatch"],
            "hbm_GBps": out["traffic"], "hbm_frac": out["traffic"] / HBM_PEAK_GBS,
            "l2_hit_rate": hit / max(1.0, hit + miss),
            "l1_to_l2_GBps": l1l2 / t / 1e9,
            "gather_efficiency": BYTES_PER_EVAL * evals_per_launch / max(1.0, l1l2),
            "source": os.path.relpath(COUNTERS, ROOT),
        }
    return out


def copy_calibration():
    """A plain device copy of known size, to scale the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 1 << 28                       # 2^28 float32 = 1 GiB read + 1 GiB written per copy
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}))


def bench_batch(args):
    """Batching workload: 64 independent problems (own rooms, resolutions 160x120 .. 640x480,
    K in [256, 4096], own 256^3 FP32 volumes at 1 cm, 10 iterations, every 2nd pixel), each with
    frame 1 fused; frame 2 tracked as (a) 64 sequential track_frame calls, (b) one batch, (c) one
    replay of the batch captured in a HIP graph. Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2509_24236_amd as pf
    import synth
    from paper_2509_24236_amd import autotune
    dev = torch.device("cuda:0")
    n = args.problems
    log(f"[bench] building {n} batching problems")
    probs, evals = [], 0
    for p in range(n):
        d = synth.random_depth_for_batch(p)
        vol = pf.Tsdf(d["vol"], device=dev)
        vol.integrate(torch.as_tensor(d["depth1"]).to(dev), d["intr"], np.eye(3), np.zeros(3))
        prm = pf.TrackParams(seed=40 + p, frame_index=1, n_iters=10, K=d["K"], rates=(1,), pixel_stride=2,
                             s1_deg=10.0, s1_m=0.10)
        probs.append((vol, torch.as_tensor(d["depth2"]).to(dev), d["intr"], *d["init2"], prm))
    torch.cuda.synchronize()
    plan = autotune.plan_for(probs) if not args.tune else autotune.tune(probs, log=log)
    trackers = [pf.Tracker(p[2], p[5], device=dev) for p in probs]

    def sequential():
        out = []
        for trk, (vol, depth, intr, R0, t0, prm) in zip(trackers, probs):
            out.append(trk.track(vol, depth, R0, t0))
        return out

    seq = sequential()           # warm-up, and the per-problem reference
    evals = sum((p[5].K + 1) * st.n_sub[i] for p, (_, _, st) in zip(probs, seq) for i in range(st.n_iters))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sequential()
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / args.steps
    b = pf.Batch(probs, plan, device=dev)
    b.run()
    res = b.results()
    same = all(np.array_equal(r[0], q[0]) and np.array_equal(r[1], q[1]) for r, q in zip(res, seq))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.run(stream=s)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / args.steps
    res_g = b.results()
    same_g = all(np.array_equal(r[0], q[0]) and np.array_equal(r[1], q[1]) for r, q in zip(res_g, seq))
    b.close()
    out = {"metric": "batched particle-point fitness evals/s (64 heterogeneous problems, one frame each)",
           "value": evals / t_graph, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "ms_per_step": 1e3 * t_graph, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{n} problems: 160x120..640x480, K 256..4096, 256^3 f32 at 1 cm, 10 iterations, "
                                  "every 2nd pixel", "plan": dataclasses_asdict(plan)},
           "sequential_ms": 1e3 * t_seq, "batch_eager_ms": 1e3 * t_batch, "batch_graph_ms": 1e3 * t_graph,
           "speedup_vs_sequential": t_seq / t_graph, "bitwise_equal_to_plain": bool(same and same_g),
           "evals_per_batch": evals}
    print(json.dumps(out), flush=True)


def bench_regimes(args):
    """Scoring kernel alone across the spread regimes of one frame's optimization: 3073 poses drawn
    in a box of +-s around the true pose of frame 1 (s = 10, 1, 0.1, 0.001 deg with s/100 m), scored
    on the rate-1/8 view (in track_frame's tiled order) against the 512^3 FP32 volume holding frame
    0, with the launch track_frame's automatic mode uses for that spread (4 poses x 256 threads,
    through the cell-validity mask with compaction at the three spreads above a quarter voxel).
    Prints one JSON line; for counter runs
    (rocprofv3 --pmc), every regime is launched 1 + args.steps times in order."""
    import numpy as np
    import torch
    import paper_2509_24236_amd as pf
    import synth
    dev = torch.device("cuda:0")
    f = synth.cfg2_frames(2)
    intr, spec = f["intr"], f["vol"]
    vol = pf.Tsdf(spec, device=dev)
    vol.integrate(torch.as_tensor(f["depth"](0)).to(dev), intr, np.eye(3), np.zeros(3))
    px, py, pz, n = pf.backproject(torch.as_tensor(f["depth"](1)).to(dev), intr, 1)
    N = int(n[0].item())
    # the rate-1/8 view in the order track_frame builds it: tiles of 32 image rows by 16 columns,
    # row by row inside a tile (the pixel of each point recovered from its coordinates)
    S = torch.stack([px[:N:8], py[:N:8], pz[:N:8]], 1).cpu().numpy().astype(np.float64)
    u = np.rint(intr.fx * S[:, 0] / S[:, 2] + intr.cx).astype(np.int64)
    v = np.rint(intr.fy * S[:, 1] / S[:, 2] + intr.cy).astype(np.int64)
    tile = (v // 32) * ((intr.width + 15) // 16) + u // 16
    order = torch.as_tensor(np.lexsort((u, v % 32, tile))).to(dev)
    x, y, z = px[:N:8][order].contiguous(), py[:N:8][order].contiguous(), pz[:N:8][order].contiguous()
    Rg, tg = f["gt"][1]
    rng = np.random.default_rng(0)
    out = {"workload": "particles_score, 3073 poses x rate-1/8 view of frame 1 (%d points), 512^3 f32 cells"
                       % x.numel(), "regimes": []}
    for s_deg, shape, mask in [(10.0, (4, 256), True), (1.0, (4, 256), True), (0.1, (4, 256), True),
                               (0.001, (4, 256), False)]:
        poses = [(Rg, tg)]
        for _ in range(3072):
            r = rng.uniform(-1, 1, 3) * math.radians(s_deg)
            poses.append((synth.rot(r) @ Rg, tg + rng.uniform(-1, 1, 3) * s_deg / 100.0))
        P = torch.as_tensor(pf.poses_to_f32(poses)).to(dev)
        pf.score_config(*shape)
        pf.score_mask(pf.MASK_ALWAYS if mask else pf.MASK_NEVER)
        E, nv = pf.particles_score(vol, x, y, z, P)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pf.particles_score(vol, x, y, z, P, E, nv)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = sorted(ts)[len(ts) // 2]
        ev = 3073 * x.numel()
        out["regimes"].append({"spread_deg": s_deg, "shape": list(shape), "mask": mask, "ms": ms,
                               "evals_per_s": ev / ms * 1e3, "algorithmic_GBps": BYTES_PER_EVAL * ev / ms / 1e6,
                               "valid_fraction": float(nv.sum().item()) / ev})
        log(f"[regimes] spread {s_deg} deg, shape {shape}, mask {mask}: {ms:.4f} ms, {ev / ms / 1e6:.1f} Gevals/s")
    pf.score_config(0, 0)
    pf.score_mask(pf.MASK_BY_SPREAD)
    print(json.dumps(out), flush=True)


def bench_combined(args):
    """Batched + adjoint form against the plain per-frame path at equal accuracy, on the batching
    workload (64 problems as in --workload batch). Plain: 64 sequential track_frame calls with 10
    iterations, the configured method. Combined: one batched launch sequence (a replayed HIP graph)
    with fewer iterations followed by 5 gradient-polish steps, for I = 3 .. 9. Accuracy is the error
    against the ground-truth pose: the reported configuration is the fewest iterations whose median
    rotation and translation errors are both no larger than the plain path's. The polish moves the
    pose to a different point than further particle iterations would, so the combined poses are not
    close to the plain ones (the sweep lists the largest deviation); both are compared to the truth.
    Prints one JSON line."""
    import dataclasses
    import numpy as np
    import torch
    import paper_2509_24236_amd as pf
    from paper_2509_24236_amd import autotune
    import synth
    dev = torch.device("cuda:0")
    n = args.problems
    log(f"[combined] building {n} problems")
    probs, gts = [], []
    for p in range(n):
        d = synth.random_depth_for_batch(p)
        vol = pf.Tsdf(d["vol"], device=dev)
        vol.integrate(torch.as_tensor(d["depth1"]).to(dev), d["intr"], np.eye(3), np.zeros(3))
        prm = pf.TrackParams(seed=40 + p, frame_index=1, n_iters=10, K=d["K"], rates=(1,), pixel_stride=2,
                             s1_deg=10.0, s1_m=0.10)
        probs.append((vol, torch.as_tensor(d["depth2"]).to(dev), d["intr"], *d["init2"], prm))
        gts.append(d["gt2"])
    torch.cuda.synchronize()
    trackers = [pf.Tracker(p[2], p[5], device=dev) for p in probs]

    def plain():
        return [trk.track(vol, depth, R0, t0) for trk, (vol, depth, intr, R0, t0, prm) in zip(trackers, probs)]

    ref = plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / args.steps

    def rot_deg(Ra, Rb):
        c = (np.trace(Ra.T @ Rb) - 1.0) / 2.0
        return math.degrees(math.acos(max(-1.0, min(1.0, c))))

    def gt_err(res):
        return (float(np.median([rot_deg(R, g[0]) for (R, t, _), g in zip(res, gts)])),
                float(np.median([1e3 * np.linalg.norm(t - g[1]) for (R, t, _), g in zip(res, gts)])))

    plain_err = gt_err(ref)

    rows, chosen = [], None
    for iters in range(3, 10):
        cp = [(v, d, k, R, t, dataclasses.replace(prm, n_iters=iters, polish_steps=5)) for v, d, k, R, t, prm in probs]
        b = pf.Batch(cp, autotune.plan_for(cp), device=dev)
        b.run()
        res = b.results()
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            b.run(stream=s)
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        t_comb = (time.perf_counter() - t0) / args.steps
        b.close()
        dr = max(rot_deg(R, Rr) for (R, _, _), (Rr, _, _) in zip(res, ref))
        dt = max(1e3 * float(np.linalg.norm(t - tr)) for (_, t, _), (_, tr, _) in zip(res, ref))
        err = gt_err(res)
        row = {"iterations": iters, "polish_steps": 5, "ms": 1e3 * t_comb, "gt_median_deg": err[0],
               "gt_median_mm": err[1], "max_dev_from_plain_deg": dr, "max_dev_from_plain_mm": dt,
               "polish_accepted_mean": float(np.mean([st.polish_accepted for *_, st in res]))}
        rows.append(row)
        log(f"[combined] I = {iters} + 5 polish: {1e3 * t_comb:.1f} ms, median error vs truth {err[0]:.3f} deg / "
            f"{err[1]:.2f} mm (plain {plain_err[0]:.3f} deg / {plain_err[1]:.2f} mm)")
        if chosen is None and err[0] <= plain_err[0] and err[1] <= plain_err[1]:
            chosen = row
    out = {"metric": "time to the plain path's accuracy, 64 heterogeneous problems (batched + polish vs plain)",
           "value": (1e3 * t_plain / chosen["ms"]) if chosen else None, "unit": "x (plain ms / combined ms)",
           "n_gpus": 1, "steps": args.steps, "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{n} problems: 160x120..640x480, K 256..4096, 256^3 f32 at 1 cm, every 2nd pixel; "
                                  "plain = 10 iterations per problem, sequential track_frame calls; combined = one "
                                  "batched graph with I iterations + 5 polish steps",
                      "accuracy": "median rotation and translation error against the ground-truth pose, no larger "
                                  "than the plain path's"},
           "plain_ms": 1e3 * t_plain, "plain_gt_median_deg": plain_err[0], "plain_gt_median_mm": plain_err[1],
           "chosen": chosen, "sweep": rows}
    print(json.dumps(out), flush=True)


_RENDER = {}


def bench_precision(args):
    """Precision workload (form 1) on the first frames of the paper-scale sequence: the room in a 1024^3
    grid at 0.5 cm (tau 2 cm), 640x480 depth, 4096 particles x 20 iterations at rates 1/8, 1/16, 1/32,
    then fusion at the tracked pose, in each storage format (FP32 T + FP32 W, FP16 T + uint8 W, int16
    T + uint8 W; sums exact, pose math FP64). Frame 0 is fused at the true pose; frame t starts from
    the previous estimate composed with the stand-in. Per frame (t = 1 .. args.frames) and format:
    - the pose against the FP64 oracle tracking from the same initial pose with the same random
      stream on this format's own volume as it stood (dequantized): the kernels' arithmetic;
    - the fitness of the tracked pose on the densest view against its FP64 value on that same
      volume, and against the FP64 fusion of the same frames at the same poses (no storage rounding):
      the error of the form itself;
    - the oracle's count of particle/pose near-ties (|E_k - E_0| <= 1e-4 E_0) over the iterations, the
      decisions FP32 rounding can flip.
    GPU time per frame (track + fuse) excludes the oracle's work. Prints one JSON line."""
    import numpy as np
    import torch
    import oracle
    import paper_2509_24236_amd as pf
    import synth
    dev = torch.device("cuda:0")
    n_frames = args.frames + 1
    log(f"[precision] rendering {n_frames} frames")
    f = synth.cfg2_frames(n_frames)
    intr, rel = f["intr"], f["rel"]
    spec = synth.VolumeSpec.centred(1024, 0.005, 0.02, synth.room_centre_world(f["scene"]))
    depth = [torch.as_tensor(f["depth"](t)).to(dev) for t in range(n_frames)]
    K, I, rates = 4096, 20, (8, 16, 32)
    names = {pf.F32_W_F32: "f32", pf.F16_W_U8: "f16+u8", pf.I16_W_U8: "i16+u8"}
    fmts = {"f32": pf.F32_W_F32, "f16": pf.F16_W_U8, "i16": pf.I16_W_U8}
    res = {}
    for key in args.formats.split(","):
        fmt = fmts[key]
        vol = pf.Tsdf(spec, fmt=fmt, device=dev)
        trk = pf.Tracker(intr, pf.TrackParams(seed=15, frame_index=1, n_iters=I, K=K, rates=rates, pixel_stride=1,
                                              s1_deg=10.0, s1_m=0.10), device=dev)
        vol.integrate(depth[0], intr, *f["gt"][0])
        ov = oracle.Volume(spec)                  # FP64 fusion of the same frames at the same poses
        ov.integrate(f["depth"](0), intr, *f["gt"][0])
        est = [f["gt"][0]]
        rows, gpu_s, evals = [], 0.0, 0
        for t in range(1, n_frames):
            Rp, tp = est[-1]
            R0, t0 = Rp @ rel[t][0], Rp @ rel[t][1] + tp
            # the oracle on this format's volume as it stands (dequantized), same init and stream
            Tq, Wq = vol.export_linear()
            oq = oracle.Volume(spec, T=Tq.cpu().numpy(), W=Wq.cpu().numpy())
            del Tq, Wq
            oprm = oracle.make_params(seed=15, frame_index=t, n_iters=I, K=K, rates=rates, pixel_stride=1,
                                      s1_deg=10.0, s1_m=0.10)
            Rq, tq, recs = oq.track_frame(f["depth"](t), intr, R0, t0, oprm)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            trk.set_frame(t)
            R, tt, st = trk.track(vol, depth[t], R0, t0)
            vol.integrate(depth[t], intr, R, tt)
            torch.cuda.synchronize()
            gpu_s += time.perf_counter() - t1
            evals += sum((st.n_particles[i] + 1) * st.n_sub[i] for i in range(st.n_iters))
            X, _ = oracle.backproject(f["depth"](t), intr, 1)
            S8 = oracle.subsample(X, min(rates)).astype(np.float32).astype(np.float64)
            Eq, _ = oq.fitness(S8, R, tt)           # FP64, same pose, this format's volume
            E64, _ = ov.fitness(S8, R, tt)          # FP64, same pose, unrounded FP64 fusion
            del oq
            ov.integrate(f["depth"](t), intr, R, tt)
            est.append((R, tt))
            row = {"frame": t, "vs_oracle_same_volume_deg": math.degrees(oracle.rot_err(R, Rq)),
                   "vs_oracle_same_volume_mm": 1e3 * float(np.linalg.norm(tt - tq)),
                   "E_final": float(st.E_final), "E_fp64_same_volume": Eq, "E_fp64_unrounded": E64,
                   "E_rel_err_same_volume": abs(float(st.E_final) - Eq) / Eq,
                   "E_rel_err_vs_fp64": abs(float(st.E_final) - E64) / E64,
                   "near_ties": int(sum(r.n_near for r in recs)), "near_ties_iter1": int(recs[0].n_near),
                   "vs_truth_mm": 1e3 * float(np.linalg.norm(tt - f["gt"][t][1]))}
            rows.append(row)
            log(f"[precision] {names[fmt]} frame {t}: pose vs oracle {row['vs_oracle_same_volume_deg']:.3f} deg "
                f"{row['vs_oracle_same_volume_mm']:.3f} mm, E err {row['E_rel_err_same_volume']:.1e} (same volume) "
                f"{row['E_rel_err_vs_fp64']:.1e} (vs FP64), near-ties {row['near_ties']}")
        dd = np.array([r["vs_oracle_same_volume_deg"] for r in rows])
        dm = np.array([r["vs_oracle_same_volume_mm"] for r in rows])
        res[names[fmt]] = {
            "ms_per_frame": 1e3 * gpu_s / len(rows), "evals_per_s": evals / gpu_s,
            "frames": rows,
            "frames_within_1mm_0.05deg": int(np.sum((dd <= 0.05) & (dm <= 1.0))),
            "median_vs_oracle_deg": float(np.median(dd)), "median_vs_oracle_mm": float(np.median(dm)),
            "max_E_rel_err_same_volume": max(r["E_rel_err_same_volume"] for r in rows),
            "max_E_rel_err_vs_fp64": max(r["E_rel_err_vs_fp64"] for r in rows),
            "volume_bytes": vol.T.numel() * vol.T.element_size() + vol.W.numel() * vol.W.element_size()}
        del vol, trk, ov
        torch.cuda.empty_cache()
    if "f32" in res:
        for v in res.values():
            v["speedup_vs_f32"] = res["f32"]["ms_per_frame"] / v["ms_per_frame"]
    main_key = "i16+u8" if "i16+u8" in res else next(iter(res))
    out = {"metric": "particle-point fitness evals/s + ms/frame (track+fuse) at 640x480, 4096 particles, by TSDF format",
           "value": res[main_key]["evals_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": args.frames, "warmup": 0,
           "ms_per_step": res[main_key]["ms_per_frame"], "higher_is_better": True,
           "dtype": main_key.split("+")[0], "data": "synthetic",
           "config": {"workload": f"paper-scale room, frames 1..{args.frames}, 1024^3 TSDF at 0.5 cm (tau 2 cm), "
                                  "640x480, 4096 particles x 20 iterations at rates 1/8, 1/16, 1/32, then fusion; "
                                  f"value = the {main_key} form", "formats": res}}
    print(json.dumps(out), flush=True)


def _render_init(n_frames):
    import synth
    _RENDER["frames"] = synth.cfg2_frames(n_frames)


def _render_noisy(t):
    return _RENDER["frames"]["depth"](t)


def _render_clean(t):
    import synth
    f = _RENDER["frames"]
    return synth.render_depth(f["scene"], f["intr"], *f["gt"][t])


def surface_points(T, W, origin, vs):
    """Zero crossings of a fused TSDF: between x-, y- or z-neighbouring voxels that are both observed
    (W > 0) and inside the band (|T| < 1) with opposite signs, the linearly interpolated point."""
    import numpy as np
    pts = []
    for axis in range(3):                      # arrays are (z, y, x)
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[2 - axis] = slice(0, -1)
        b[2 - axis] = slice(1, None)
        T0, T1 = T[tuple(a)], T[tuple(b)]
        ok = (W[tuple(a)] > 0) & (W[tuple(b)] > 0) & (np.abs(T0) < 1) & (np.abs(T1) < 1) & ((T0 > 0) != (T1 > 0))
        k, j, i = np.nonzero(ok)
        f = T0[k, j, i] / (T0[k, j, i] - T1[k, j, i])
        P = np.stack([i, j, k], 1).astype(np.float64)
        P[:, axis] += f
        pts.append(P * vs + np.asarray(origin, np.float64))
    return np.concatenate(pts, 0)


def bench_accuracy(args):
    """Tracking and reconstruction accuracy on the paper-scale sequence against its analytic ground
    truth (the synthetic stand-in for the paper's benchmarks): ATE-RMSE of the camera positions
    (same world frame, and after a rigid alignment), the median rotation error, and the
    reconstruction's accuracy (mean distance of the fused surface's zero crossings to the true
    surfaces) and completeness (share of true surface samples, from noise-free renders of every 10th
    frame, with a reconstructed point within 10 cm). Runs the fixed schedule, the paper's schedule,
    fusion at the true poses (tracking-free reference) and the stand-in chained without any
    optimization, each with the configured stand-in (3 deg / 3 cm per frame) and, suffix _pr0.3, with
    one at about the regression network's reported accuracy (0.3 deg / 0.3 cm), and the fixed
    schedule with no stand-in at all (each frame starts from the previous estimate). Prints one JSON
    line."""
    import multiprocessing as mp
    import numpy as np
    import torch
    from scipy.spatial import cKDTree
    import paper_2509_24236_amd as pf
    import synth
    n = args.frames
    dev = torch.device("cuda:0")
    f = synth.cfg2_frames(n)
    intr, spec, gt, rel, scene = f["intr"], f["vol"], f["gt"], f["rel"], f["scene"]
    bricks = args.volume == "bricks"
    if bricks:   # the whole room, walls included, as a sparse volume at the same voxel size
        spec = synth.room_spec(scene, spec.voxel_size, spec.trunc)
    # the configured stand-in (3 deg / 3 cm per frame) and one at about the regression network's own
    # accuracy (Table VIII: median 0.26 cm), same scene, depth and seeds
    rel_fine = synth.cfg2_frames(n, pr_sigma_deg=0.3, pr_sigma_m=0.003)["rel"]
    workers = max(1, min(16, os.cpu_count() or 1))
    log(f"[accuracy] rendering {n} frames with {workers} processes")
    with mp.get_context("fork").Pool(workers, initializer=_render_init, initargs=(n,)) as pool:
        depths = pool.map(_render_noisy, range(n))
        clean = pool.map(_render_clean, range(0, n, 10))
    gt_pts = np.concatenate([synth.backproject_world(d, intr, *gt[t], stride=4)
                             for d, t in zip(clean, range(0, n, 10))], 0)
    dev_depth = [torch.as_tensor(d).to(dev) for d in depths]

    def rot_deg(Ra, Rb):
        c = (np.trace(Ra.T @ Rb) - 1.0) / 2.0
        return math.degrees(math.acos(max(-1.0, min(1.0, c))))

    def traj_metrics(est):
        P = np.stack([t for _, t in est])
        G = np.stack([t for _, t in gt[:len(est)]])
        e = np.linalg.norm(P - G, axis=1)
        # rigid alignment (Umeyama, no scale) of the estimate onto the truth
        mp_, mg = P.mean(0), G.mean(0)
        U, _, Vt = np.linalg.svd((G - mg).T @ (P - mp_))
        D = np.diag([1.0, 1.0, np.sign(np.linalg.det(U @ Vt))])
        Ra = U @ D @ Vt
        ea = np.linalg.norm((P - mp_) @ Ra.T + mg - G, axis=1)
        rot = [rot_deg(R, g[0]) for (R, _), g in zip(est, gt)]
        return {"ate_rmse_cm": 100 * float(np.sqrt(np.mean(e ** 2))),
                "ate_rmse_aligned_cm": 100 * float(np.sqrt(np.mean(ea ** 2))),
                "median_rot_err_deg": float(np.median(rot)), "max_trans_err_cm": 100 * float(e.max())}

    def recon_metrics(vol):
        T, W = vol.export_linear()
        T, W = T.cpu().numpy(), W.cpu().numpy()
        S = surface_points(T, W, spec.origin, spec.voxel_size)
        del T, W
        acc = synth.scene_distance(scene, S)
        dist, _ = cKDTree(S).query(gt_pts, k=1, distance_upper_bound=0.10)
        return {"surface_points": int(S.shape[0]), "accuracy_cm": 100 * float(acc.mean()),
                "accuracy_median_cm": 100 * float(np.median(acc)),
                "completeness_10cm": float(np.mean(np.isfinite(dist)))}

    out = {"metric": "ATE-RMSE (cm) and reconstruction accuracy / completeness on the synthetic sequence",
           "frames": n, "gt_surface_samples": int(gt_pts.shape[0]), "runs": {},
           "volume": (f"bricks over the whole room, {spec.nx}x{spec.ny}x{spec.nz} at {spec.voxel_size * 100:g} cm"
                      if bricks else f"dense {spec.nx}x{spec.ny}x{spec.nz} at {spec.voxel_size * 100:g} cm")}
    identity = [None] + [(np.eye(3), np.zeros(3))] * (n - 1)
    for name in ("fixed", "paper", "gt_poses", "standin_only", "fixed_pr0.3", "paper_pr0.3", "standin_only_pr0.3",
                 "ro_only"):
        # ro_only: no pose regression at all, each frame starts from the previous estimate (the
        # analogue of running the optimization alone)
        rel_run = rel_fine if name.endswith("_pr0.3") else (identity if name == "ro_only" else rel)
        vol = (pf.Tsdf(spec, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=args.max_bricks) if bricks
               else pf.Tsdf(spec, device=dev))
        vol.integrate(dev_depth[0], intr, np.eye(3), np.zeros(3))
        est = [(np.eye(3), np.zeros(3))]
        trk = None
        if name.startswith("fixed") or name == "ro_only":
            trk = pf.Tracker(intr, pf.TrackParams(seed=14, n_iters=20, K=3072, rates=(8, 16, 32), pixel_stride=1,
                                                  s1_deg=10.0, s1_m=0.10), device=dev)
        elif name.startswith("paper"):
            trk = pf.Tracker(intr, pf.TrackParams(seed=14, n_iters=20, K=10240, Ks=(1024, 3072, 10240),
                                                  rates=(8, 16, 32), pixel_stride=1, s1_deg=10.0, s1_m=0.10,
                                                  stop_deg=0.05, stop_m=0.0005), device=dev)
        iters = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(1, n):
            Rp, tp = est[-1]
            Rr, tr = rel_run[t]
            R0, t0_ = Rp @ Rr, Rp @ tr + tp
            if name == "gt_poses":
                R, tt = gt[t]
            elif name.startswith("standin_only"):
                R, tt = R0, t0_
            else:
                trk.set_frame(t)
                R, tt, st = trk.track(vol, dev_depth[t], R0, t0_)
                iters.append(st.n_iters)
            vol.integrate(dev_depth[t], intr, R, tt)
            est.append((R, tt))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        row = traj_metrics(est)
        row.update(recon_metrics(vol))
        if bricks:
            row["bricks_used"], row["brick_overflow"] = vol.bricks_used()
        row["ms_per_frame"] = 1e3 * wall / (n - 1)
        if iters:
            row["mean_iterations"] = float(np.mean(iters))
        out["runs"][name] = row
        log(f"[accuracy] {name}: {json.dumps(row)}")
        del vol
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def dataclasses_asdict(x):
    import dataclasses
    return dataclasses.asdict(x)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed frames")
    ap.add_argument("--warmup", type=int, default=3, help="untimed frames before the timed ones")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true", help="run only a plain 1 GiB device copy")
    ap.add_argument("--frames", type=int, default=None,
                    help="accuracy: frames of the sequence (200); precision: frames tracked (20)")
    ap.add_argument("--workload", default="sequence", choices=["sequence", "batch", "regimes", "combined", "accuracy", "precision"],
                    help="sequence: the paper-scale sequence (the headline); batch: 64 heterogeneous problems; "
                         "regimes: the scoring kernel alone at four particle spreads (diagnostic); combined: "
                         "batched + polish against plain at equal accuracy; accuracy: ATE and reconstruction "
                         "quality of the whole sequence against the analytic ground truth; precision: the "
                         "1024^3 grid in FP32, FP16 and int16 storage against each other and the FP64 oracle")
    ap.add_argument("--problems", type=int, default=64)
    ap.add_argument("--schedule", default="fixed", choices=["fixed", "paper"],
                    help="sequence: fixed = 3072 particles x 20 iterations (the headline configuration); paper = "
                         "the alternating particle counts and early exit of Sec. IV-A")
    ap.add_argument("--tune", action="store_true", help="batch: run the autotuner first and record the plan")
    ap.add_argument("--volume", default="dense", choices=["dense", "bricks"],
                    help="sequence, accuracy: dense = the 512^3 cell-replica grid centred on the room (the "
                         "headline); bricks = a sparse brick pool over the whole room at the same 1 cm voxels")
    ap.add_argument("--max-bricks", type=int, default=120000, help="bricks: pool slots")
    ap.add_argument("--formats", default="f32,f16,i16", help="precision: storage formats to run (f32, f16, i16)")
    ap.add_argument("--only-tracked", action="store_true",
                    help="sequence: skip the run fused at the ground-truth poses (counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures the single-GPU path only (--gpus {args.gpus} requested); the multi-GPU "
              "particle sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "regimes":
        bench_regimes(args)
        return
    if args.workload == "combined":
        bench_combined(args)
        return
    if args.workload == "accuracy":
        args.frames = args.frames or 200
        bench_accuracy(args)
        return
    if args.workload == "precision":
        args.frames = args.frames or 20
        bench_precision(args)
        return

    import numpy as np
    import torch

    import paper_2509_24236_amd as pf
    import synth

    pf.lib()
    dev = torch.device("cuda:0")
    n_frames = args.warmup + args.steps + 2
    log(f"[bench] rendering {n_frames} frames of the paper-scale sequence")
    frames = synth.cfg2_frames(n_frames)
    intr, spec = frames["intr"], frames["vol"]
    depth = [torch.as_tensor(frames["depth"](t)).to(dev) for t in range(n_frames)]
    rel = frames["rel"]
    K, I, rates = 3072, 20, (8, 16, 32)
    if args.schedule == "paper":
        # Sec. IV-A's own schedule: K alternates 1024 / 3072 / 10240 with the rates, early exit
        params = pf.TrackParams(seed=14, frame_index=1, n_iters=I, K=10240, Ks=(1024, 3072, 10240), rates=rates,
                                pixel_stride=1, s1_deg=10.0, s1_m=0.10, stop_deg=0.05, stop_m=0.0005)
    else:
        params = pf.TrackParams(seed=14, frame_index=1, n_iters=I, K=K, rates=rates, pixel_stride=1, s1_deg=10.0,
                                s1_m=0.10)
    if args.volume == "bricks":
        spec = synth.room_spec(frames["scene"], spec.voxel_size, spec.trunc)
        vol = pf.Tsdf(spec, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=args.max_bricks)
    else:
        vol = pf.Tsdf(spec, device=dev)
    vol_bytes = vol.T.numel() * vol.T.element_size() + vol.W.numel() * vol.W.element_size()
    trk = pf.Tracker(intr, params, device=dev)
    torch.cuda.synchronize()

    def run_sequence(fuse_at_gt):
        """Fuses frame 0 at the identity, then tracks and fuses frames 1.. (the warm-up ones untimed).
        Each frame starts from the previous estimate composed with the stand-in; the frame is fused at
        the tracked pose, or (fuse_at_gt) at the ground-truth pose."""
        vol.init()
        est = [(np.eye(3), np.zeros(3))]
        vol.integrate(depth[0], intr, *est[0])
        iters_run, fuse_events, method_evals = [], [], [0]

        def step(t, measured=False):
            Rp, tp = est[t - 1]
            Rr, tr = rel[t]
            R0, t0 = Rp @ Rr, Rp @ tr + tp            # P_t^(0) = P_{t-1} P_(t,t-1)
            trk.set_frame(t)
            if fuse_at_gt or measured:
                # (the measured frame fuses in a call of its own, between the events that time it)
                R, tt, st = trk.track(vol, depth[t], R0, t0)
                if measured:
                    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                    ev[0].record()
                vol.integrate(depth[t], intr, *(frames["gt"][t] if fuse_at_gt else (R, tt)))
                if measured:
                    ev[1].record()
                    fuse_events.append(ev)
            else:
                # track, then fuse at the tracked pose in the same call: the fusion is enqueued on the
                # device before the call waits for its result
                R, tt, st = trk.track_fuse(vol, depth[t], R0, t0)
            est.append((R, tt))
            iters_run.append(st.n_iters)
            # the method's samples: each iteration scores its particles and the current pose on S_i
            method_evals[0] += sum((st.n_particles[i] + 1) * st.n_sub[i] for i in range(st.n_iters))

        for t in range(1, args.warmup + 1):
            step(t)
        torch.cuda.synchronize()
        pf.timing_read(reset=True)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        del iters_run[:]
        del fuse_events[:]
        method_evals[0] = 0
        # The last timed frame is the measured one: HIP events bracket each of its particle launches
        # and its fusion (each event is a packet of its own on the stream, ~6 us, so events around
        # every launch of every frame would lengthen the frame they time by ~0.2 ms).
        last = args.warmup + args.steps
        for t in range(args.warmup + 1, last + 1):
            if t == last:
                pf.timing_enable(True)
            step(t, measured=t == last)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        score_ms, launches, evals = pf.timing_read(reset=True)
        pf.timing_enable(False)
        fuse_ms = sum(a.elapsed_time(b) for a, b in fuse_events) / max(1, len(fuse_events))
        t_err = [float(np.linalg.norm(est[t][1] - frames["gt"][t][1])) for t in range(1, len(est))]
        r_err = [math.degrees(rot_err(est[t][0], frames["gt"][t][0])) for t in range(1, len(est))]
        return {"elapsed": elapsed, "ms_per_frame": 1e3 * elapsed / args.steps, "method_evals": method_evals[0],
                "score_ms": score_ms, "launches": launches, "evals": evals, "fuse_ms": fuse_ms,
                "iters_run": iters_run, "est": est,
                "gt_error": {"translation_median_mm": 1e3 * float(np.median(t_err)),
                             "translation_max_mm": 1e3 * float(np.max(t_err)),
                             "rotation_median_deg": float(np.median(r_err)),
                             "frames": len(t_err)}}

    log(f"[bench] sequence fused at the tracked poses: warmup {args.warmup}, timing {args.steps} frames")
    run = run_sequence(False)
    run_gt = None
    if not args.only_tracked:
        log(f"[bench] sequence fused at the ground-truth poses (reported beside)")
        run_gt = run_sequence(True)
    elapsed, launches, evals, score_ms = run["elapsed"], run["launches"], run["evals"], run["score_ms"]
    ms_per_frame = run["ms_per_frame"]
    avg_launch_ms = score_ms / max(1, launches)
    evals_per_launch = evals / max(1, launches)
    fuse_ms = run["fuse_ms"]
    log(f"[bench] {ms_per_frame:.3f} ms/frame, scoring {avg_launch_ms:.4f} ms/launch avg, "
        f"{evals / max(score_ms, 1e-9) * 1e3:.3e} evals/s in-kernel; GT translation error median "
        f"{run['gt_error']['translation_median_mm']:.2f} mm" +
        (f" (fused at the truth: {run_gt['ms_per_frame']:.3f} ms/frame, "
         f"{run_gt['gt_error']['translation_median_mm']:.2f} mm)" if run_gt else ""))

    # fusion roofline: the voxels one fusion updates (W grows), from one more frame after the timing
    n_next = args.warmup + args.steps + 1
    W0 = vol.export_linear()[1]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    vol.integrate(depth[n_next], intr, *frames["gt"][n_next])
    e1.record()
    torch.cuda.synchronize()
    W1 = vol.export_linear()[1]
    n_upd = int((W1 != W0).sum().item())
    del W0, W1
    fuse1_ms = e0.elapsed_time(e1)
    fuse_bytes = FUSE_BYTES_PER_VOXEL * n_upd + 4 * intr.width * intr.height
    torch.cuda.empty_cache()
    adj = adjoint_timing(vol, depth[n_next], intr, *frames["gt"][n_next])
    log(f"[bench] adjoint {adj['adjoint_ms']:.3f} ms vs scoring {adj['scoring_ms']:.3f} ms for {adj['poses']} poses x "
        f"{adj['points']} points; E bitwise equal: {adj['E_bitwise_equal_to_scoring']}")

    roof = roofline(avg_launch_ms, evals_per_launch)
    out = {
        "metric": METRIC,
        "value": run["method_evals"] / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_frame,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "paper-scale sequence: 640x480 depth, 512^3 FP32 TSDF at 1 cm (tau 4 cm), 3072 particles x "
                        "20 iterations at point rates 1/8, 1/16, 1/32, then fusion at the tracked pose; one step = "
                        "one frame"
                        if args.schedule == "fixed" else
                        "paper-scale sequence: 640x480 depth, 512^3 FP32 TSDF at 1 cm (tau 4 cm), particles "
                        "alternating 1024 / 3072 / 10240 with point rates 1/8, 1/16, 1/32, at most 20 iterations, "
                        "stop once the search size is below (0.05 deg, 0.5 mm), then fusion at the tracked pose; "
                        "one step = one frame",
            "frames_timed": args.steps,
            "particles": K if args.schedule == "fixed" else [1024, 3072, 10240],
            "iterations": I,
            "mean_iterations_run": sum(run["iters_run"]) / max(1, len(run["iters_run"])),
            "tsdf": "512^3 f32 T + f32 W, cell-major f32 replica and cell-validity mask for scoring",
            "fusion_ms_per_frame": fuse_ms,
            "volume_bytes": vol_bytes,
        },
        "accuracy": {"vs_ground_truth": run["gt_error"],
                     "note": "the tracked trajectory drifts (the method as read does not track this sequence); the "
                             "same sequence fused at the ground-truth poses is timed beside it"},
        "fused_at_ground_truth": None if run_gt is None else {
            "value": run_gt["method_evals"] / run_gt["elapsed"], "unit": "evals/s",
            "ms_per_step": run_gt["ms_per_frame"], "fusion_ms_per_frame": run_gt["fuse_ms"],
            "scoring_ms_per_launch": run_gt["score_ms"] / max(1, run_gt["launches"]),
            "vs_ground_truth": run_gt["gt_error"]},
        "roofline": roof,
        "fusion_roofline": {"bound": "hbm", "achieved": fuse_bytes / (fuse1_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": fuse_bytes / (fuse1_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                            "updated_voxels": n_upd, "bytes": fuse_bytes, "ms": fuse1_ms,
                            "note": f"{FUSE_BYTES_PER_VOXEL} B per updated voxel (T and W read and written) plus the "
                                    "depth image, over one fusion of the frame after the timed ones"},
        "adjoint": adj,
    }
    if args.volume == "bricks":
        used, overflow = vol.bricks_used()
        if overflow:
            raise SystemExit(f"the brick pool of {args.max_bricks} slots overflowed: raise --max-bricks")
        c = out["config"]
        c["workload"] = c["workload"].replace("512^3 FP32 TSDF at 1 cm", f"sparse FP32 TSDF over the whole room "
                                              f"({spec.nx}x{spec.ny}x{spec.nz} at 1 cm, 8^3 bricks)")
        c["tsdf"] = (f"brick pool: {used} of {args.max_bricks} slots in use after the last frame, f32 T + f32 W + "
                     f"per-brick cell blocks; {spec.nx}x{spec.ny}x{spec.nz} grid ({spec.nx * spec.ny * spec.nz / 1e6:.1f}M "
                     f"voxels), {used * 512 / (spec.nx * spec.ny * spec.nz):.1%} of them stored")
        c["bricks_used"] = used
        out["roofline"]["kernel"] = ("particle launch per iteration: k_draw_score<f32, bricks>, 4 poses x 256 threads")
        out["roofline"]["counters"] = out["roofline"]["traffic"] = None
        log(f"[bench] bricks {used}, fusion {fuse_ms:.3f} ms/frame, volume {vol_bytes / 2**30:.2f} GiB")
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(frames, spec, intr, n_frames, args.cpu_seconds, args.schedule)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
