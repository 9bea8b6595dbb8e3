"""Parity of the HIP path (through the C ABI) with the FP64 oracle on identical seeded inputs.

Bars: bit-exact for integer/index work (compaction order and counts, fusion weights, RNG
deltas, advantage-set size); FP32 fitness inside the oracle's near-face interval widened by
1e-4 relative; fused T within FP32 rounding of the FP64 value; tracked poses within 1 mm and
0.05 degrees of the oracle's with the same random stream."""
import math
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pf():
    import paper_2509_24236_amd as pf
    pf.lib()
    assert torch.cuda.is_available()
    return pf


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def cfg1():
    return synth.cfg1_inputs()


@pytest.fixture(scope="module")
def cfg1_vol(orc, cfg1):
    """Oracle TSDF after fusing frame 1, and its float32 rounding (the shared scoring input)."""
    v = orc.Volume(cfg1["vol"])
    v.integrate(cfg1["depth1"], cfg1["intr"], np.eye(3), np.zeros(3))
    T32 = v.T.astype(np.float32)
    v32 = orc.Volume(cfg1["vol"], T=T32.astype(np.float64), W=v.W)
    return v, v32, T32


def upload(pf, spec, T32, W, dev, fmt=0, layout=1):
    vol = pf.Tsdf(spec, fmt=fmt, device=dev, init=False, layout=layout)
    vol.import_linear(T32, W.astype(np.float32))
    return vol


def check_fitness(E_gpu, nv_gpu, lo, hi, rel=1e-4):
    E_gpu = np.asarray(E_gpu, np.float64)
    lo_w = lo - rel * np.abs(lo) - 1e-7
    hi_w = hi + rel * np.abs(hi) + 1e-7
    bad = np.flatnonzero((E_gpu < lo_w) | (E_gpu > hi_w))
    assert bad.size == 0, f"{bad.size} poses outside the oracle interval, e.g. k={bad[:5]}: " \
                          f"gpu {E_gpu[bad[:5]]} lo {lo[bad[:5]]} hi {hi[bad[:5]]}"


# ----------------------------------------------------------------------------- back-projection
@pytest.mark.parametrize("case", ["cfg1_stride2", "ragged_invalid", "cfg2_full"])
def test_backproject_parity(pf, orc, dev, cfg1, case):
    say(f"[backproject] {case}")
    if case == "cfg1_stride2":
        depth, intr, stride = cfg1["depth2"], cfg1["intr"], 2
    elif case == "ragged_invalid":
        rng = np.random.default_rng(7)
        intr = synth.Intrinsics(30.0, 31.0, 18.3, 11.7, 37, 23)
        depth = rng.uniform(0.2, 4.0, (23, 37)).astype(np.float32)
        depth[rng.random(depth.shape) < 0.2] = 0.0
        depth[1, 2], depth[3, 4], depth[5, 6], depth[7, 8] = np.nan, -1.0, np.inf, -np.inf
        stride = 3
    else:
        f = synth.cfg2_frames(2)
        depth, intr, stride = f["depth"](1), f["intr"], 1
    xyz, pix = orc.backproject(depth, intr, stride)
    px, py, pz, n = pf.backproject(torch.as_tensor(depth).to(dev), intr, stride)
    n = int(n[0].item())
    assert n == xyz.shape[0]
    g = np.stack([px[:n].cpu().numpy(), py[:n].cpu().numpy(), pz[:n].cpu().numpy()], 1).astype(np.float64)
    assert np.array_equal(g[:, 2], xyz[:, 2])                 # z is the depth value itself: order and bits
    # float32 x = ((u - cx) z) / fx: the rounding of cx itself bounds the error by |cx| z / fx
    # times 2^-24, plus a few roundings of |x|
    z = xyz[:, 2]
    bx = 1.2e-7 * (abs(intr.cx) * z / intr.fx + 5 * np.abs(xyz[:, 0])) + 1e-12
    by = 1.2e-7 * (abs(intr.cy) * z / intr.fy + 5 * np.abs(xyz[:, 1])) + 1e-12
    assert np.all(np.abs(g[:, 0] - xyz[:, 0]) <= bx) and np.all(np.abs(g[:, 1] - xyz[:, 1]) <= by)


# ----------------------------------------------------------------------------- fusion
@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_integrate_parity_cfg1(pf, orc, dev, cfg1, fmt):
    say(f"[integrate] cfg1 two frames, format {fmt}")
    spec, intr = cfg1["vol"], cfg1["intr"]
    ov = orc.Volume(spec)
    gv = pf.Tsdf(spec, fmt=fmt, device=dev, layout=pf.LAYOUT_CELLS)
    frames = [(cfg1["depth1"], cfg1["gt1"]), (cfg1["depth2"], cfg1["gt2"])]
    for depth, (R, t) in frames:
        ov.integrate(depth, intr, R, t)
        gv.integrate(torch.as_tensor(depth).to(dev), intr, R, t)
        T, W = gv.export_linear()
        T, W = T.cpu().numpy().astype(np.float64), W.cpu().numpy()
        assert np.array_equal(W, ov.W.astype(np.float32)), "weights must match exactly"
        upd = ov.W > 0
        err = np.abs(T - ov.T)
        tol = {0: 2e-6, 1: 1.5e-3, 2: 1e-4}[fmt]
        assert err[upd].max() <= tol, (fmt, err[upd].max())
        assert np.all(T[~upd] == 1.0)
    assert (ov.W == 2).sum() > 100000


def test_integrate_parity_ragged_and_behind(pf, orc, dev):
    say("[integrate] ragged volume, camera inside, rotated pose")
    spec = synth.VolumeSpec(37, 29, 23, 0.05, 0.12, (-0.9, -0.7, -0.5))
    rng = np.random.default_rng(11)
    intr = synth.Intrinsics(40.0, 41.0, 20.5, 15.5, 41, 31)
    depth = rng.uniform(0.3, 1.5, (31, 41)).astype(np.float32)
    depth[rng.random(depth.shape) < 0.1] = 0.0
    from scipy.spatial.transform import Rotation
    R = Rotation.from_rotvec([0.3, -0.2, 0.1]).as_matrix()
    t = np.array([0.05, -0.02, 0.1])
    ov = orc.Volume(spec)
    ov.integrate(depth, intr, R, t)
    gv = pf.Tsdf(spec, device=dev)
    gv.integrate(torch.as_tensor(depth).to(dev), intr, R, t)
    T, W = gv.export_linear()
    assert np.array_equal(W.cpu().numpy(), ov.W.astype(np.float32))
    assert np.abs(T.cpu().numpy() - ov.T).max() <= 2e-6


# ----------------------------------------------------------------------------- scoring
def _poses_around(orc, R, t, n, rot, trans, seed):
    rng = np.random.default_rng(seed)
    out = [(R, t)]
    for _ in range(n - 1):
        out.append(orc.compose(rng.uniform(-rot, rot, 3), rng.uniform(-trans, trans, 3), R, t))
    return out


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("K", [1, 5, 64, 65, 257])
def test_score_parity_cfg1(pf, orc, dev, cfg1, cfg1_vol, K, layout):
    say(f"[score] cfg1 K={K} layout={layout}")
    v, v32, T32 = cfg1_vol
    xyz, _ = orc.backproject(cfg1["depth2"], cfg1["intr"], 2)
    x32 = xyz.astype(np.float32)
    R, t = cfg1["init2"]
    poses = _poses_around(orc, R, t, K, math.radians(5), 0.03, K)
    P32 = pf.poses_to_f32(poses)
    poses64 = [(P32[k].reshape(3, 4)[:, :3].astype(np.float64), P32[k].reshape(3, 4)[:, 3].astype(np.float64))
               for k in range(K)]
    lo, hi, na = v32.fitness_interval_many(x32.astype(np.float64), poses64, eps=1e-3)
    gv = upload(pf, cfg1["vol"], T32, v.W, dev, layout=layout)
    xt = torch.as_tensor(x32).to(dev)
    E, nv = pf.particles_score(gv, xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous(),
                               torch.as_tensor(P32).to(dev))
    check_fitness(E.cpu().numpy(), nv.cpu().numpy(), lo, hi)
    assert np.all(nv.cpu().numpy() > 0)
    # bitwise reproducible
    E2, nv2 = pf.particles_score(gv, xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous(),
                                 torch.as_tensor(P32).to(dev))
    assert torch.equal(E, E2) and torch.equal(nv, nv2)


@pytest.mark.parametrize("n_pts", [1, 3, 1000])
def test_score_edge_cases(pf, orc, dev, cfg1, cfg1_vol, n_pts):
    say(f"[score] edge n_pts={n_pts}")
    v, v32, T32 = cfg1_vol
    xyz, _ = orc.backproject(cfg1["depth1"], cfg1["intr"], 1)
    x32 = xyz[:n_pts].astype(np.float32)
    far = np.array([[50.0, 0.0, 1.0]], np.float32)     # outside the grid for every pose
    pts = np.concatenate([x32, far]) if n_pts > 1 else x32
    poses = [(np.eye(3), np.zeros(3)), (np.eye(3), np.array([100.0, 0.0, 0.0]))]
    P32 = pf.poses_to_f32(poses)
    lo, hi, _ = v32.fitness_interval_many(pts.astype(np.float64), poses, eps=1e-3)
    gv = upload(pf, cfg1["vol"], T32, v.W, dev)
    pt = torch.as_tensor(np.ascontiguousarray(pts)).to(dev)
    E, nv = pf.particles_score(gv, pt[:, 0].contiguous(), pt[:, 1].contiguous(), pt[:, 2].contiguous(),
                               torch.as_tensor(P32).to(dev))
    check_fitness(E.cpu().numpy(), nv.cpu().numpy(), lo, hi)
    assert E[1].item() == 1.0 and nv[1].item() == 0          # every sample outside: E = 1


def test_score_affine_field_is_zero(pf, orc, dev):
    say("[score] plane field")
    spec = synth.VolumeSpec.centred(96, 0.02, 0.08, (0.0, 0.0, 1.2))
    n = np.array([0.1, -0.2, -1.0])
    n /= np.linalg.norm(n)
    c = np.array([0.0, 0.0, 1.2])
    T = synth.fill_plane_volume(spec, n, float(n @ c)).astype(np.float32)
    u = np.cross(n, [1.0, 0, 0])
    u /= np.linalg.norm(u)
    w = np.cross(n, u)
    ab = np.random.default_rng(0).uniform(-0.4, 0.4, (5000, 2))
    P = (c + ab[:, :1] * u + ab[:, 1:] * w).astype(np.float32)
    gv = upload(pf, spec, T, np.ones(T.shape), dev)
    pt = torch.as_tensor(P).to(dev)
    E, nv = pf.particles_score(gv, pt[:, 0].contiguous(), pt[:, 1].contiguous(), pt[:, 2].contiguous(),
                               torch.as_tensor(pf.poses_to_f32([(np.eye(3), np.zeros(3))])).to(dev))
    assert nv.item() == 5000 and E.item() <= 2e-6


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_cells_replica_tracks_fusion(pf, orc, dev, cfg1, fmt):
    """After GPU fusion of two frames, scoring through the cell replica is bitwise identical to
    scoring through the x-fastest storage (the replica holds exactly the stored values)."""
    say(f"[score] cell replica vs linear after fusion, format {fmt}")
    spec, intr = cfg1["vol"], cfg1["intr"]
    gv = pf.Tsdf(spec, fmt=fmt, device=dev, layout=pf.LAYOUT_CELLS)
    for depth, (R, t) in [(cfg1["depth1"], cfg1["gt1"]), (cfg1["depth2"], cfg1["gt2"])]:
        gv.integrate(torch.as_tensor(depth).to(dev), intr, R, t)
    lin = pf.Tsdf(spec, fmt=fmt, device=dev, layout=pf.LAYOUT_LINEAR, init=False)
    n = spec.nx * spec.ny * spec.nz
    lin.T[:n].copy_(gv.T[:n])
    lin.W.copy_(gv.W)
    xyz, _ = orc.backproject(cfg1["depth2"], intr, 1)
    xt = torch.as_tensor(xyz.astype(np.float32)).to(dev)
    poses = _poses_around(orc, *cfg1["init2"], 300, math.radians(5), 0.03, 1)
    P = torch.as_tensor(pf.poses_to_f32(poses)).to(dev)
    a = pf.particles_score(gv, xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous(), P)
    b = pf.particles_score(lin, xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous(), P)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert int((a[1] > 0).sum()) > 250


# ----------------------------------------------------------------------------- update
def test_update_parity(pf, orc, dev, cfg1, cfg1_vol):
    say("[update] state init, draw, advantage set on identical fitness")
    v, v32, T32 = cfg1_vol
    K = 1000
    prm = pf.TrackParams(seed=12345, frame_index=7, n_iters=3, K=K, rates=(1,), s1_deg=10.0, s1_m=0.1)
    R0, t0 = cfg1["init2"]
    state = torch.zeros(pf.state_bytes(K), dtype=torch.uint8, device=dev)
    poses = torch.zeros((K + 1, 12), dtype=torch.float32, device=dev)
    pf.particles_state_init(state, R0, t0, prm, poses)
    D = pf.read_deltas(state, K)
    s_rad = math.radians(10.0)
    for k in range(1, K + 1):
        r, tau = orc.draw_delta(12345, 7, 1, k, s_rad, 0.1)
        assert np.array_equal(D[k, :3], r) and np.array_equal(D[k, 3:], tau), k
    Pg = poses.cpu().numpy()
    for k in (0, 1, 500, K):
        Ro, to = orc.compose(D[k, :3], D[k, 3:], R0, t0) if k else (R0, t0)
        ref = pf.poses_to_f32([(Ro, to)])[0]
        assert np.abs(Pg[k] - ref).max() <= 2 * np.abs(ref).max() * 2 ** -24
    # identical fitness input on both sides, with exact ties to E_0 that must be excluded
    rng = np.random.default_rng(5)
    fit = rng.uniform(0.1, 0.5, K + 1).astype(np.float32)
    fit[0] = 0.3
    fit[rng.choice(np.arange(1, K + 1), 20, replace=False)] = 0.3
    xyz, _ = orc.backproject(cfg1["depth2"], cfg1["intr"], 2)
    x32 = xyz.astype(np.float32)
    gv = upload(pf, cfg1["vol"], T32, v.W, dev)
    xt = torch.as_tensor(x32).to(dev)
    nvz = torch.zeros(K + 1, dtype=torch.int32, device=dev)
    pf.particles_update(gv, xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous(),
                        torch.as_tensor(fit).to(dev), nvz, state, K, poses)
    st = pf.read_state(state)
    na, Ro, to, mean = orc.advantage_update(fit.astype(np.float64), D, R0, t0)
    assert st.n_adv == na == int((fit[1:] < fit[0]).sum())
    assert np.abs(np.array(st.mean[:]) - mean).max() <= 1e-15 * max(1.0, np.abs(mean).max()) * 50
    Rg, tg = np.array(st.R[:]).reshape(3, 3), np.array(st.t[:])
    assert np.abs(Rg - Ro).max() <= 1e-13 and np.abs(tg - to).max() <= 1e-13
    # E* of the new pose on the same points, and the search-size update
    P32 = pf.poses_to_f32([(Rg, tg)])[0].reshape(3, 4).astype(np.float64)
    lo, hi, _ = v32.fitness_interval_many(x32.astype(np.float64), [(P32[:, :3], P32[:, 3])], eps=1e-3)
    check_fitness([st.Estar], None, lo, hi)
    f_lo, f_hi = 0.1 + 0.9 * lo[0], 0.1 + 0.9 * hi[0]
    assert s_rad * f_lo * (1 - 1e-4) <= st.s_rad <= s_rad * f_hi * (1 + 1e-4)
    assert st.iter == 2 and st.E0 == np.float32(0.3)


# ----------------------------------------------------------------------------- whole frame
@pytest.mark.parametrize("mode", [0, 1])
def test_track_frame_parity_cfg1(pf, orc, dev, cfg1, cfg1_vol, mode):
    say(f"[track] cfg1 compose mode {mode}")
    v, v32, T32 = cfg1_vol
    gv = upload(pf, cfg1["vol"], T32, v.W, dev)
    R0, t0 = cfg1["init2"]
    prm = pf.TrackParams(seed=3, frame_index=1, n_iters=10, K=256, rates=(1,), pixel_stride=2, s1_deg=5.0, s1_m=0.03,
                         compose_mode=mode)
    trk = pf.Tracker(cfg1["intr"], prm, device=dev)
    depth = torch.as_tensor(cfg1["depth2"]).to(dev)
    R, t, st = trk.track(gv, depth, R0, t0)
    oprm = orc.make_params(seed=3, frame_index=1, n_iters=10, K=256, rates=(1,), pixel_stride=2, s1_deg=5.0,
                           s1_m=0.03, compose_mode=mode)
    Ro, to, recs = v32.track_frame(cfg1["depth2"], cfg1["intr"], R0, t0, oprm)
    dr, dt = math.degrees(orc.rot_err(R, Ro)), float(np.linalg.norm(t - to))
    say(f"    pose vs oracle: {dr:.3e} deg, {dt * 1e3:.3e} mm; |A| gpu {list(st.n_adv[:10])} "
        f"oracle {[r.n_adv for r in recs]}")
    assert dr <= 0.05 and dt <= 1e-3
    assert st.n_points == 4800 - int((cfg1["depth2"][::2, ::2] <= 0).sum())
    for i in range(10):
        assert abs(st.E0[i] - recs[i].E0) <= 1e-3 and abs(st.Estar[i] - recs[i].Estar) <= 1e-3
    # determinism
    R2, t2, st2 = trk.track(gv, depth, R0, t0)
    assert np.array_equal(R, R2) and np.array_equal(t, t2)
    assert list(st.n_adv[:10]) == list(st2.n_adv[:10])


def test_track_frame_rates_and_stats(pf, orc, dev, cfg1, cfg1_vol):
    say("[track] cfg1 rate cycle 1,2,3")
    v, v32, T32 = cfg1_vol
    gv = upload(pf, cfg1["vol"], T32, v.W, dev)
    R0, t0 = cfg1["init2"]
    prm = pf.TrackParams(seed=9, frame_index=2, n_iters=6, K=300, rates=(1, 2, 3), pixel_stride=1, s1_deg=5.0,
                         s1_m=0.03)
    trk = pf.Tracker(cfg1["intr"], prm, device=dev)
    R, t, st = trk.track(gv, torch.as_tensor(cfg1["depth2"]).to(dev), R0, t0)
    oprm = orc.make_params(seed=9, frame_index=2, n_iters=6, K=300, rates=(1, 2, 3), pixel_stride=1, s1_deg=5.0,
                           s1_m=0.03)
    Ro, to, recs = v32.track_frame(cfg1["depth2"], cfg1["intr"], R0, t0, oprm)
    n = st.n_points
    assert [st.n_sub[i] for i in range(6)] == [r.n_pts for r in recs] == [n, (n + 1) // 2, (n + 2) // 3] * 2
    assert math.degrees(orc.rot_err(R, Ro)) <= 0.05 and np.linalg.norm(t - to) <= 1e-3


def test_track_frame_paper_schedule_cfg1(pf, orc, dev, cfg1, cfg1_vol):
    """Sec. IV-A's own schedule: the particle count alternates with the rate, and the optimization
    stops once the updated search size is below (0.05 deg, 0.5 mm)."""
    say("[schedule] cfg1, K 64/128/256 with rates 1/2/3, stop rule")
    v, v32, T32 = cfg1_vol
    gv = upload(pf, cfg1["vol"], T32, v.W, dev)
    R0, t0 = cfg1["init2"]
    kw = dict(seed=9, frame_index=2, n_iters=16, rates=(1, 2, 3), pixel_stride=2, s1_deg=5.0, s1_m=0.03,
              stop_deg=0.05, stop_m=0.0005)
    R, t, st = pf.Tracker(cfg1["intr"], pf.TrackParams(K=256, Ks=(64, 128, 256), **kw), device=dev).track(
        gv, torch.as_tensor(cfg1["depth2"]).to(dev), R0, t0)
    Ro, to, recs = v32.track_frame(cfg1["depth2"], cfg1["intr"], R0, t0, orc.make_params(Ks=(64, 128, 256), **kw))
    dr, dt = math.degrees(orc.rot_err(R, Ro)), float(np.linalg.norm(t - to))
    say(f"    iterations gpu {st.n_iters} oracle {len(recs)}; pose vs oracle {dr:.2e} deg {dt * 1e3:.3e} mm")
    assert st.n_iters == len(recs) < 16
    assert [st.n_particles[i] for i in range(st.n_iters)] == [r.n_particles for r in recs]
    assert [st.n_sub[i] for i in range(st.n_iters)] == [r.n_pts for r in recs]
    assert dr <= 0.05 and dt <= 1e-3


SHAPES = [(1, 256), (2, 256), (4, 256), (8, 256), (1, 512), (2, 512), (4, 512), (8, 512), (2, 128), (4, 128),
          (8, 128), (2, 64), (4, 64), (8, 64)]


@pytest.mark.parametrize("spread_deg", [5.0, 0.01])
def test_score_shapes_bitwise_identical(pf, orc, dev, cfg1, cfg1_vol, spread_deg):
    """Fitness sums are exact, so every launch shape (and the few-pose path) gives the same bits."""
    say(f"[shapes] 257 poses, spread {spread_deg} deg, {len(SHAPES)} launch shapes")
    v, v32, T32 = cfg1_vol
    gv = upload(pf, cfg1["vol"], T32, v.W, dev)
    X, _ = orc.backproject(cfg1["depth2"], cfg1["intr"], 2)
    xt = torch.as_tensor(X.astype(np.float32)).to(dev)
    pts = (xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous())
    R, t = cfg1["gt2"]
    poses = _poses_around(orc, R, t, 257, math.radians(spread_deg), spread_deg * 0.006, seed=77)
    P = torch.as_tensor(pf.poses_to_f32(poses)).to(dev)
    ref = None
    try:
        for tk, blk in SHAPES:
            pf.score_config(tk, blk)
            E, nv = pf.particles_score(gv, *pts, P)
            got = (E.cpu().numpy().view(np.uint32), nv.cpu().numpy())
            if ref is None:
                ref = got
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (tk, blk)
    finally:
        pf.score_config(0, 0)
    E64, nv64 = pf.particles_score(gv, *pts, P[:64].contiguous())
    assert np.array_equal(E64.cpu().numpy().view(np.uint32), ref[0][:64])
    assert np.array_equal(nv64.cpu().numpy(), ref[1][:64])


def test_track_frame_automatic_shape_matches_fixed(pf, orc, dev, cfg1, cfg1_vol):
    """track_frame picks the scoring shape per iteration from the spread on the device; the
    result is bitwise that of any fixed shape."""
    say("[shapes] track_frame automatic vs fixed launch shapes")
    v, v32, T32 = cfg1_vol
    gv = upload(pf, cfg1["vol"], T32, v.W, dev)
    R0, t0 = cfg1["init2"]
    prm = pf.TrackParams(seed=3, frame_index=1, n_iters=10, K=256, rates=(1,), pixel_stride=2, s1_deg=5.0, s1_m=0.03)
    depth = torch.as_tensor(cfg1["depth2"]).to(dev)
    R, t, st = pf.Tracker(cfg1["intr"], prm, device=dev).track(gv, depth, R0, t0)
    try:
        for tk, blk in [(4, 256), (2, 64), (8, 512)]:
            pf.score_config(tk, blk)
            Rf, tf, stf = pf.Tracker(cfg1["intr"], prm, device=dev).track(gv, depth, R0, t0)
            assert np.array_equal(R, Rf) and np.array_equal(t, tf), (tk, blk)
            assert list(st.n_adv[:10]) == list(stf.n_adv[:10])
            assert list(st.Estar[:10]) == list(stf.Estar[:10])
    finally:
        pf.score_config(0, 0)


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_track_frame_narrow_form_matches_generic(pf, orc, dev, cfg1, cfg1_vol, fmt):
    """With K >= 1024 on a cubic volume whose replica 32-bit offsets address (cfg1: 128^3), the
    automatic launches take their narrow form (max3 in-grid test, 32-bit gather offsets, per-wave
    counts) and the spread regime its compacting masked form; a configured launch shape takes the
    generic per-lane form without the mask. Both track bitwise alike, on the first call (the
    regime-gated scoring launches) and on the second (the particle launch that draws)."""
    say(f"[narrow] format {fmt}: track_frame K=1024 automatic (narrow, masked) vs configured 4x256 (generic)")
    v, v32, T32 = cfg1_vol
    gv = upload(pf, cfg1["vol"], T32, v.W, dev, fmt=fmt)
    R0, t0 = cfg1["init2"]
    prm = pf.TrackParams(seed=5, frame_index=1, n_iters=8, K=1024, rates=(1,), pixel_stride=2, s1_deg=5.0, s1_m=0.03)
    depth = torch.as_tensor(cfg1["depth2"]).to(dev)
    trk = pf.Tracker(cfg1["intr"], prm, device=dev)
    auto = [trk.track(gv, depth, R0, t0) for _ in range(2)]
    assert np.array_equal(auto[0][0], auto[1][0]) and np.array_equal(auto[0][1], auto[1][1])
    try:
        pf.score_config(4, 256)
        R, t, st = pf.Tracker(cfg1["intr"], prm, device=dev).track(gv, depth, R0, t0)
    finally:
        pf.score_config(0, 0)
    for Ra, ta, sta in auto:
        assert np.array_equal(R, Ra) and np.array_equal(t, ta)
        assert list(st.n_adv[:8]) == list(sta.n_adv[:8])
        assert list(st.Estar[:8]) == list(sta.Estar[:8])


# ----------------------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def cfg2_full(orc):
    f = synth.cfg2_frames(2)
    ov = orc.Volume(f["vol"])
    ov.integrate(f["depth"](0), f["intr"], np.eye(3), np.zeros(3))
    return f, ov


def test_fullsize_fusion_weights_exact(pf, dev, cfg2_full):
    say("[fullsize] 512^3 fusion of frame 0: weights exact, values within FP32 rounding")
    f, ov = cfg2_full
    gv = pf.Tsdf(f["vol"], device=dev)
    gv.integrate(torch.as_tensor(f["depth"](0)).to(dev), f["intr"], np.eye(3), np.zeros(3))
    T, W = gv.export_linear()
    W = W.cpu().numpy()
    assert np.array_equal(W, ov.W.astype(np.float32))
    T = T.cpu().numpy()
    upd = ov.W > 0
    assert np.abs(T[upd].astype(np.float64) - ov.T[upd]).max() <= 1e-6
    assert upd.sum() > 10_000_000


def test_fullsize_scoring_sampled(pf, orc, dev, cfg2_full):
    """The bench launch configuration (3073 poses, rate-1/8 view, cell replica, 4 poses per
    workgroup): 48 sampled poses against the oracle's intervals."""
    say("[fullsize] 3073 poses on the rate-1/8 view, 48 sampled against the oracle")
    f, ov = cfg2_full
    T32 = ov.T.astype(np.float32)
    gv = upload(pf, f["vol"], T32, ov.W, dev)
    X, _ = orc.backproject(f["depth"](1), f["intr"], 1)
    S = orc.subsample(X, 8).astype(np.float32)
    R0, t0 = f["gt"][1]
    poses = _poses_around(orc, R0, t0, 3073, math.radians(10), 0.10, 5)
    P32 = pf.poses_to_f32(poses)
    st = torch.as_tensor(S).to(dev)
    E, nv = pf.particles_score(gv, st[:, 0].contiguous(), st[:, 1].contiguous(), st[:, 2].contiguous(),
                               torch.as_tensor(P32).to(dev))
    E = E.cpu().numpy()
    idx = np.unique(np.concatenate([[0, 1, 2, 3072], np.random.default_rng(6).choice(3073, 44, replace=False)]))
    v32 = orc.Volume(f["vol"], T=T32.astype(np.float64), W=ov.W)
    p64 = [(P32[k].reshape(3, 4)[:, :3].astype(np.float64), P32[k].reshape(3, 4)[:, 3].astype(np.float64)) for k in idx]
    lo, hi, _ = v32.fitness_interval_many(S.astype(np.float64), p64, eps=1e-3)
    check_fitness(E[idx], None, lo, hi)
    del v32


def test_fullsize_track_frame(pf, orc, dev, cfg2_full):
    say("[fullsize] track frame 1: 3072 particles x 20 iterations, rates 8/16/32")
    f, ov = cfg2_full
    T32 = ov.T.astype(np.float32)
    gv = upload(pf, f["vol"], T32, ov.W, dev)
    v32 = orc.Volume(f["vol"], T=T32.astype(np.float64), W=ov.W)
    R0, t0 = f["rel"][1]                    # P_1^(0) = I * P_(1,0)
    prm = pf.TrackParams(seed=14, frame_index=1, n_iters=20, K=3072, rates=(8, 16, 32), pixel_stride=1)
    R, t, st = pf.Tracker(f["intr"], prm, device=dev).track(gv, torch.as_tensor(f["depth"](1)).to(dev), R0, t0)
    oprm = orc.make_params(seed=14, frame_index=1, n_iters=20, K=3072, rates=(8, 16, 32), pixel_stride=1,
                           s1_deg=10.0, s1_m=0.10)
    Ro, to, recs = v32.track_frame(f["depth"](1), f["intr"], R0, t0, oprm)
    dr, dt = math.degrees(orc.rot_err(R, Ro)), float(np.linalg.norm(t - to))
    say(f"    pose vs oracle {dr:.2e} deg {dt * 1e3:.3e} mm; |A| gpu {list(st.n_adv[:6])} oracle "
        f"{[r.n_adv for r in recs[:6]]}")
    assert dr <= 0.05 and dt <= 1e-3
    assert [st.n_sub[i] for i in range(20)] == [r.n_pts for r in recs]
    del v32


def test_fullsize_regime_forecast_changes_nothing(pf, dev, cfg2_full):
    """track_frame launches, per iteration, only the scoring launch of the spread regime the same
    iteration had in the previous call with the same parameters (the masked, compacting launch or
    the per-lane one). Whether that forecast is right
    (same frame again), wrong (forecast from a run started far away) or absent (other parameters
    in between) changes nothing in the result."""
    say("[fullsize] regime forecast: right, wrong and absent give the same frame")
    f, ov = cfg2_full
    gv = upload(pf, f["vol"], ov.T.astype(np.float32), ov.W, dev)
    depth = torch.as_tensor(f["depth"](1)).to(dev)
    R0, t0 = f["rel"][1]
    prm = pf.TrackParams(seed=14, frame_index=1, n_iters=20, K=3072, rates=(8, 16, 32), pixel_stride=1)
    other = pf.TrackParams(seed=14, frame_index=1, n_iters=19, K=3072, rates=(8, 16, 32), pixel_stride=1)
    trk = pf.Tracker(f["intr"], prm, device=dev)
    pf.Tracker(f["intr"], other, device=dev).track(gv, depth, R0, t0)             # no forecast for prm
    ref = trk.track(gv, depth, R0, t0)
    same = trk.track(gv, depth, R0, t0)                                            # right forecast
    far = synth.rot(np.array([0.02, -0.03, 0.01])) @ R0
    trk.track(gv, depth, far, t0 + 0.04)                                           # forecast from elsewhere
    wrong = trk.track(gv, depth, R0, t0)
    for R, t, st in (same, wrong):
        assert np.array_equal(R, ref[0]) and np.array_equal(t, ref[1])
        assert list(st.Estar) == list(ref[2].Estar) and list(st.n_adv) == list(ref[2].n_adv)
        assert st.E_final == ref[2].E_final
    # the paper's schedule with the early exit: iterations after the stop take the last regime
    paper = pf.TrackParams(seed=14, frame_index=1, n_iters=20, K=10240, Ks=(1024, 3072, 10240), rates=(8, 16, 32),
                           pixel_stride=1, stop_deg=0.05, stop_m=0.0005)
    tp = pf.Tracker(f["intr"], paper, device=dev)
    pf.Tracker(f["intr"], other, device=dev).track(gv, depth, R0, t0)
    ref = tp.track(gv, depth, R0, t0)
    again = tp.track(gv, depth, R0, t0)
    assert ref[2].n_iters < 20 and again[2].n_iters == ref[2].n_iters
    assert np.array_equal(again[0], ref[0]) and np.array_equal(again[1], ref[1])


def test_fullsize_track_frame_paper_schedule(pf, orc, dev, cfg2_full):
    say("[fullsize] track frame 1 with K 1024/3072/10240 at rates 8/16/32 and the stop rule")
    f, ov = cfg2_full
    T32 = ov.T.astype(np.float32)
    gv = upload(pf, f["vol"], T32, ov.W, dev)
    v32 = orc.Volume(f["vol"], T=T32.astype(np.float64), W=ov.W)
    R0, t0 = f["rel"][1]
    kw = dict(seed=14, frame_index=1, n_iters=20, rates=(8, 16, 32), pixel_stride=1, s1_deg=10.0, s1_m=0.10,
              stop_deg=0.05, stop_m=0.0005)
    R, t, st = pf.Tracker(f["intr"], pf.TrackParams(K=10240, Ks=(1024, 3072, 10240), **kw), device=dev).track(
        gv, torch.as_tensor(f["depth"](1)).to(dev), R0, t0)
    Ro, to, recs = v32.track_frame(f["depth"](1), f["intr"], R0, t0, orc.make_params(Ks=(1024, 3072, 10240), **kw))
    dr, dt = math.degrees(orc.rot_err(R, Ro)), float(np.linalg.norm(t - to))
    say(f"    iterations gpu {st.n_iters} oracle {len(recs)}; pose vs oracle {dr:.2e} deg {dt * 1e3:.3e} mm")
    assert st.n_iters == len(recs)
    assert [st.n_particles[i] for i in range(st.n_iters)] == [r.n_particles for r in recs]
    assert dr <= 0.05 and dt <= 1e-3
    del v32
