"""Two end-to-end checks of the HIP path against the FP64 oracle.

1. Brute force (the oracle's exhaustive pose grid): on a tiny exact scene (a box room whose banded
   distance field is affine on every cell away from its edges), all 5^6 poses of a grid around the
   true pose are scored through particles_score. Every fitness lies in the oracle's near-face
   interval, the GPU's argmin index equals the oracle's (which is the true pose's node) once the
   oracle shows that minimum separated from every other node by more than the intervals' width, and
   track_frame from the grid centre lands within one grid step of the truth on every axis, matching
   the oracle's own track_frame with the same random stream.

2. The track-then-fuse cycle (Sec. III "Method overview", Fig. 2) on the paper-scale sequence: frame
   0 fused at the identity, then frames 1..10 each tracked from the previous estimate composed with
   the pose-regression stand-in and fused at the tracked pose. The oracle tracks every frame from
   the same initial pose on its own FP64 fusion and fuses at the same pose as the GPU; per frame the
   poses agree within 1 mm / 0.05 deg and the fusion weights are bit-exact."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def pf():
    import paper_2509_24236_amd as pf
    pf.lib()
    return pf


def _rotvec_matrix(r):
    from scipy.spatial.transform import Rotation
    return Rotation.from_rotvec(r).as_matrix()


def _box_room_scene():
    """A 2 m box room seen from inside, 64^3 at 4 cm (tau 16 cm), 40x30 depth."""
    from scipy.spatial.transform import Rotation
    lo, hi = np.array([-1.0, -1.0, -1.0]), np.array([1.0, 1.0, 1.0])
    R_rc1 = Rotation.from_euler("YXZ", [0.5, -0.3, 0.1]).as_matrix()
    scene = synth.make_room_scene(lo, hi, [], [], R_rc1, np.array([-0.2, -0.1, -0.3]))
    spec = synth.VolumeSpec.centred(64, 0.04, 0.16, synth.room_centre_world(scene))
    T = synth.fill_room_volume(spec, scene)
    K = synth.Intrinsics(30.0, 30.0, 19.5, 14.5, 40, 30)
    return scene, spec, T, K


def test_exhaustive_grid_argmin_and_track_on_gpu(pf, orc):
    say("[grid] 5^6 poses around the truth on the exact box room, 40x30 depth, 64^3 at 4 cm")
    dev = torch.device("cuda:0")
    scene, spec, T, K = _box_room_scene()
    vol = orc.Volume(spec, T=T)
    R_gt = _rotvec_matrix([0.03, -0.05, 0.02])
    t_gt = np.array([0.04, -0.03, 0.05])
    depth = synth.render_depth(scene, K, R_gt, t_gt)
    X, _ = orc.backproject(depth, K, 1)
    rot_step, trans_step, m = math.radians(2.0), 0.03, 5
    # grid centred one step off on every axis, so the truth is node (1, 3, 1, 3, 1, 1)
    Rc, tc = orc.compose(np.array([rot_step, -rot_step, rot_step]), np.array([-trans_step, trans_step, trans_step]),
                         R_gt, t_gt)
    best, E64 = vol.grid_search(X, Rc, tc, m, rot_step, trans_step)
    assert list(np.unravel_index(best, (m,) * 6)) == [1, 3, 1, 3, 1, 1]
    # the same nodes as FP32 poses (node q: index digits, rotation digits first, x fastest last)
    poses = []
    for q in range(m ** 6):
        idx = np.unravel_index(q, (m,) * 6)
        r = (np.array(idx[:3]) - 0.5 * (m - 1)) * rot_step
        tau = (np.array(idx[3:]) - 0.5 * (m - 1)) * trans_step
        poses.append(orc.compose(r, tau, Rc, tc))
    P32 = pf.poses_to_f32(poses)
    p64 = [(P[:, :3].astype(np.float64), P[:, 3].astype(np.float64)) for P in P32.reshape(-1, 3, 4)]
    W = (np.abs(T) < 1).astype(np.float32)
    gv = pf.Tsdf(spec, device=dev, init=False)
    gv.import_linear(T.astype(np.float32), W)
    X32 = X.astype(np.float32)
    xt = torch.as_tensor(X32).to(dev)
    E, nv = pf.particles_score(gv, xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous(),
                               torch.as_tensor(P32).to(dev))
    E = E.cpu().numpy().astype(np.float64)
    v32 = orc.Volume(spec, T=T.astype(np.float32).astype(np.float64))
    lo, hi, _ = v32.fitness_interval_many(X32.astype(np.float64), p64, eps=1e-3)
    # Next to the 1e-4 relative margin, an absolute one for fitness values near 0 (the truth's node
    # on an exact field): an FP32 sample position is off by a few ulps of its grid coordinate (at
    # most 64 here, ulp 2^-17 voxel), and |T| changes by at most vs / tau per voxel, so each sample's
    # value, and hence the mean, is within 8 * 2^-17 * vs / tau of the FP64 one.
    abs_m = 8 * 2.0 ** -17 * spec.voxel_size / spec.trunc
    lo_w, hi_w = lo - 1e-4 * lo - abs_m, hi + 1e-4 * hi + abs_m
    bad = np.flatnonzero((E < lo_w) | (E > hi_w))
    assert bad.size == 0, f"{bad.size} of {m ** 6} grid poses outside the oracle interval, e.g. {bad[:5]}: " \
                          f"{E[bad[:5]]} vs [{lo[bad[:5]]}, {hi[bad[:5]]}]"
    # margin rule: the oracle's minimum (on the FP32 poses) is separated from every other node
    others = np.delete(np.arange(m ** 6), best)
    assert hi_w[best] < lo_w[others].min(), "grid minimum not separated from the other nodes"
    g_best = int(np.argmin(E))
    say(f"    argmin gpu {g_best} oracle {best}; E {E[g_best]:.3e}, next {np.sort(E)[1]:.3e}")
    assert g_best == best
    # track_frame from the grid centre with the paper's initial search size
    prm = pf.TrackParams(seed=3, frame_index=1, n_iters=20, K=1024, rates=(1,), pixel_stride=1, s1_deg=10.0,
                         s1_m=0.10)
    R, t, st = pf.Tracker(K, prm, device=dev).track(gv, torch.as_tensor(depth).to(dev), Rc, tc)
    oprm = orc.make_params(seed=3, frame_index=1, n_iters=20, K=1024, rates=(1,), pixel_stride=1, s1_deg=10.0,
                           s1_m=0.10)
    Ro, to, _ = v32.track_frame(depth, K, Rc, tc, oprm)
    dr, dt = math.degrees(orc.rot_err(R, Ro)), float(np.linalg.norm(t - to))
    rot_axes = np.abs(orc.so3_log(R @ R_gt.T))
    say(f"    track: vs oracle {dr:.2e} deg {dt * 1e3:.2e} mm; vs truth per axis "
        f"{np.degrees(rot_axes).round(3)} deg, {np.abs(t - t_gt).round(4)} m")
    assert dr <= 0.05 and dt <= 1e-3
    assert np.all(rot_axes <= rot_step) and np.all(np.abs(t - t_gt) <= trans_step)


def test_track_and_fuse_sequence_frames_1_to_10(pf, orc):
    n = 11
    say(f"[sequence] paper-scale room, frames 0..{n - 1}: track (3072 x 20, rates 8/16/32) then fuse")
    dev = torch.device("cuda:0")
    f = synth.cfg2_frames(n)
    spec, intr = f["vol"], f["intr"]
    gv = pf.Tsdf(spec, device=dev)
    ov = orc.Volume(spec)
    est = (np.eye(3), np.zeros(3))
    gv.integrate(torch.as_tensor(f["depth"](0)).to(dev), intr, *est)
    ov.integrate(f["depth"](0), intr, *est)
    trk = pf.Tracker(intr, pf.TrackParams(seed=14, frame_index=1, n_iters=20, K=3072, rates=(8, 16, 32),
                                          pixel_stride=1, s1_deg=10.0, s1_m=0.10), device=dev)
    worst = (0.0, 0.0)
    for t in range(1, n):
        Rr, tr = f["rel"][t]
        R0, t0 = est[0] @ Rr, est[0] @ tr + est[1]
        depth = f["depth"](t)
        trk.set_frame(t)
        R, tt, st = trk.track(gv, torch.as_tensor(depth).to(dev), R0, t0)
        oprm = orc.make_params(seed=14, frame_index=t, n_iters=20, K=3072, rates=(8, 16, 32), pixel_stride=1,
                               s1_deg=10.0, s1_m=0.10)
        Ro, to, recs = ov.track_frame(depth, intr, R0, t0, oprm)
        dr, dt = math.degrees(orc.rot_err(R, Ro)), float(np.linalg.norm(tt - to))
        worst = (max(worst[0], dr), max(worst[1], dt))
        adv_g, adv_o = list(st.n_adv[:20]), [r.n_adv for r in recs]
        say(f"    frame {t}: vs oracle {dr:.2e} deg {dt * 1e3:.2e} mm; |A| equal in "
            f"{sum(a == b for a, b in zip(adv_g, adv_o))}/20 iterations")
        assert dr <= 0.05 and dt <= 1e-3, f"frame {t}: {dr} deg, {dt * 1e3} mm"
        # fuse both at the GPU's pose: the update decisions are FP64 on both sides
        gv.integrate(torch.as_tensor(depth).to(dev), intr, R, tt)
        ov.integrate(depth, intr, R, tt)
        if t % 5 == 0 or t == n - 1:
            Tg, Wg = gv.export_linear()
            Wg = Wg.cpu().numpy()
            assert np.array_equal(Wg, ov.W.astype(np.float32)), f"frame {t}: fusion weights differ"
            upd = ov.W > 0
            assert np.abs(Tg.cpu().numpy()[upd].astype(np.float64) - ov.T[upd]).max() <= 1e-5
            del Tg, Wg
        est = (R, tt)
    say(f"    worst frame vs oracle: {worst[0]:.2e} deg, {worst[1] * 1e3:.2e} mm")
