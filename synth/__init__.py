"""Seeded synthetic inputs for the tracking-and-fusion hot path.

This module only builds inputs: analytic indoor scenes, ray-cast depth maps, camera
trajectories, the stand-in for the pose-regression network, and analytic signed-distance
volumes used as test fixtures. It holds none of the tracking or fusion arithmetic (no
back-projection, integration, fitness, sampling of delta poses or pose update), so the FP64
oracle and the HIP library consume identical arrays without sharing any code.

Conventions (stated once, used everywhere):
  * A pose is a pair (R, t) of float64 arrays, camera -> world: x_world = R @ x_cam + t.
  * The camera frame is x right, y down, z forward; pixel (u, v) sees the ray
    ((u - cx)/fx, (v - cy)/fy, 1). Depth is the z coordinate of the hit point in the
    camera frame, float32, 0 where invalid.
  * The world frame is the first frame's camera frame (the paper fixes frame 1 at the
    identity pose, Sec. III "Method overview").
  * Scenes are described in a room frame (y down, floor at +y); `scene["T_wr"]` maps room
    coordinates to world coordinates.

Rotations here use scipy's Rotation, an independent library routine: the input generator
must not borrow the SO(3) exponential that the method itself implements on each side.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np
from scipy.spatial.transform import Rotation

__all__ = [
    "Intrinsics", "VolumeSpec", "rot", "pose_inv", "pose_mul", "make_room_scene",
    "render_depth", "add_noise_additive", "add_noise_axial", "cfg1_inputs", "cfg2_scene",
    "cfg2_trajectory", "pr_standin", "cfg2_frames", "fill_plane_volume",
    "fill_sphere_volume", "fill_room_volume", "random_depth_for_batch",
]


# ----------------------------------------------------------------------------- basic types
@dataclasses.dataclass(frozen=True)
class Intrinsics:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int


@dataclasses.dataclass(frozen=True)
class VolumeSpec:
    """Dense grid: voxel (i, j, k) has its centre at origin + voxel_size * (i, j, k)."""
    nx: int
    ny: int
    nz: int
    voxel_size: float
    trunc: float
    origin: Tuple[float, float, float]

    @staticmethod
    def centred(n: int, voxel_size: float, trunc: float, centre) -> "VolumeSpec":
        half = 0.5 * n * voxel_size
        o = tuple(float(c) - half + 0.5 * voxel_size for c in centre)
        return VolumeSpec(n, n, n, float(voxel_size), float(trunc), o)


def rot(rotvec) -> np.ndarray:
    """Rotation matrix for a rotation vector (radians), via scipy."""
    return Rotation.from_rotvec(np.asarray(rotvec, dtype=np.float64)).as_matrix()


def pose_inv(R, t):
    R = np.asarray(R, np.float64)
    return R.T.copy(), -(R.T @ np.asarray(t, np.float64))


def pose_mul(Ra, ta, Rb, tb):
    """(Ra, ta) o (Rb, tb): apply b first, then a."""
    return Ra @ Rb, Ra @ tb + ta


def _euler_yxz(yaw, pitch, roll) -> np.ndarray:
    """Camera orientation in the room frame: yaw about -y (up), then pitch about x, then roll about z."""
    return Rotation.from_euler("YXZ", [yaw, pitch, roll]).as_matrix()


# ----------------------------------------------------------------------------- scenes
def make_room_scene(room_lo, room_hi, spheres, boxes, R_rc1, c_r1) -> Dict:
    """A room interior (axis-aligned in the room frame) with solid spheres and boxes.

    R_rc1, c_r1: orientation and position of the frame-1 camera in the room frame. The world
    frame is that camera's frame, so world = inverse(frame-1 pose) applied to room points.
    """
    R_rc1 = np.asarray(R_rc1, np.float64)
    c_r1 = np.asarray(c_r1, np.float64)
    R_wr, t_wr = pose_inv(R_rc1, c_r1)
    return {
        "room_lo": np.asarray(room_lo, np.float64),
        "room_hi": np.asarray(room_hi, np.float64),
        "spheres": [(np.asarray(c, np.float64), float(r)) for c, r in spheres],
        "boxes": [(np.asarray(lo, np.float64), np.asarray(hi, np.float64)) for lo, hi in boxes],
        "R_wr": R_wr, "t_wr": t_wr,          # room -> world
        "R_rw": R_rc1, "t_rw": c_r1,          # world -> room
    }


def room_centre_world(scene) -> np.ndarray:
    c_r = 0.5 * (scene["room_lo"] + scene["room_hi"])
    return scene["R_wr"] @ c_r + scene["t_wr"]


def render_depth(scene: Dict, K: Intrinsics, R_wc, t_wc) -> np.ndarray:
    """Exact FP64 ray casting of the analytic scene; returns float32 H x W z-depth.

    The ray for pixel (u, v) is d = ((u-cx)/fx, (v-cy)/fy, 1) in the camera frame, so the ray
    parameter of the first hit equals the camera-frame depth z.
    """
    H, W = K.height, K.width
    u = np.arange(W, dtype=np.float64)
    v = np.arange(H, dtype=np.float64)
    uu, vv = np.meshgrid(u, v)
    d_cam = np.stack([(uu - K.cx) / K.fx, (vv - K.cy) / K.fy, np.ones_like(uu)], -1).reshape(-1, 3)
    # camera -> room
    R_rc = scene["R_rw"] @ np.asarray(R_wc, np.float64)
    o_r = scene["R_rw"] @ np.asarray(t_wc, np.float64) + scene["t_rw"]
    d = d_cam @ R_rc.T
    lam = np.full(d.shape[0], np.inf)
    # room interior: exit distance
    with np.errstate(divide="ignore", invalid="ignore"):
        lo, hi = scene["room_lo"], scene["room_hi"]
        tx = np.where(d > 0, (hi - o_r) / d, np.where(d < 0, (lo - o_r) / d, np.inf))
        lam = np.minimum(lam, tx.min(axis=1))
        for c, r in scene["spheres"]:
            oc = o_r - c
            b = d @ oc
            a = np.einsum("ij,ij->i", d, d)
            cc = oc @ oc - r * r
            disc = b * b - a * cc
            ok = disc >= 0
            sq = np.sqrt(np.where(ok, disc, 0.0))
            l1 = (-b - sq) / a
            l2 = (-b + sq) / a
            hit = np.where(l1 > 1e-9, l1, np.where(l2 > 1e-9, l2, np.inf))
            lam = np.where(ok, np.minimum(lam, hit), lam)
        for blo, bhi in scene["boxes"]:
            t1 = (blo - o_r) / d
            t2 = (bhi - o_r) / d
            tmin = np.nanmax(np.minimum(t1, t2), axis=1)
            tmax = np.nanmin(np.maximum(t1, t2), axis=1)
            hit = (tmax >= tmin) & (tmax > 1e-9)
            ent = np.where(tmin > 1e-9, tmin, np.inf)   # camera never starts inside a box
            lam = np.where(hit, np.minimum(lam, ent), lam)
    lam = np.where(np.isfinite(lam), lam, 0.0)
    return lam.reshape(H, W).astype(np.float32)


def add_noise_additive(depth: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    out = depth.astype(np.float64) + rng.normal(0.0, sigma, depth.shape)
    out = np.where(depth > 0, out, 0.0)
    return out.astype(np.float32)


def add_noise_axial(depth: np.ndarray, k: float, dropout: float, seed: int) -> np.ndarray:
    """Axial noise N(0, (k z^2)^2) (z in metres) plus i.i.d. dropout to 0."""
    rng = np.random.default_rng(seed)
    z = depth.astype(np.float64)
    out = z + rng.normal(0.0, 1.0, z.shape) * (k * z * z)
    drop = rng.random(z.shape) < dropout
    out = np.where((z > 0) & ~drop, out, 0.0)
    return out.astype(np.float32)


# ----------------------------------------------------------------------------- config 1 (tiny)
CFG1_INTR = Intrinsics(120.0, 120.0, 80.0, 60.0, 160, 120)


def cfg1_inputs(scene_seed=0, noise_seed=1, init_seed=2, gt_seed=None):
    """Tiny analytic room: a 2x2x2 m box interior plus 3 spheres, 160x120 depth, 128^3 at 2 cm.

    Frame 2 is frame 1 rotated 10 degrees about a seeded unit axis and translated 5 cm along
    a seeded direction. The initial pose is GT2 o Exp(delta), delta uniform within half the
    +-5 deg / +-3 cm search box, so the optimum is reachable from the init.
    """
    rng = np.random.default_rng(scene_seed)
    lo, hi = np.array([-1.0, -1.0, -1.0]), np.array([1.0, 1.0, 1.0])
    # frame-1 camera in the room: off-centre, yawed and pitched so it sees two walls and the floor
    c_r1 = np.array([-0.25, -0.15, -0.35])
    R_rc1 = _euler_yxz(math.radians(22.0), math.radians(-14.0), math.radians(3.0))
    spheres = []
    while len(spheres) < 3:
        r = rng.uniform(0.2, 0.4)
        c = rng.uniform(lo + r + 0.3, hi - r - 0.3)
        if np.linalg.norm(c - c_r1) < r + 0.45:
            continue
        if any(np.linalg.norm(c - c2) < r + r2 + 0.05 for c2, r2 in spheres):
            continue
        spheres.append((c, r))
    scene = make_room_scene(lo, hi, spheres, [], R_rc1, c_r1)
    vol = VolumeSpec.centred(128, 0.02, 0.08, room_centre_world(scene))
    g = np.random.default_rng(scene_seed + 1000 if gt_seed is None else gt_seed)
    axis = g.normal(size=3)
    axis /= np.linalg.norm(axis)
    tdir = g.normal(size=3)
    tdir /= np.linalg.norm(tdir)
    R2 = rot(math.radians(10.0) * axis)
    t2 = 0.05 * tdir
    I3 = np.eye(3)
    d1 = add_noise_additive(render_depth(scene, CFG1_INTR, I3, np.zeros(3)), 0.002, noise_seed)
    d2 = add_noise_additive(render_depth(scene, CFG1_INTR, R2, t2), 0.002, noise_seed + 100)
    ri = np.random.default_rng(init_seed)
    dr = ri.uniform(-1, 1, 3) * math.radians(2.5)
    dt = ri.uniform(-1, 1, 3) * 0.015
    Ri, ti = pose_mul(R2, t2, rot(dr), dt)
    return {
        "scene": scene, "intr": CFG1_INTR, "vol": vol,
        "depth1": d1, "depth2": d2,
        "gt1": (I3, np.zeros(3)), "gt2": (R2, t2), "init2": (Ri, ti),
    }


# ----------------------------------------------------------------------------- config 2 (paper scale)
CFG2_INTR = Intrinsics(525.0, 525.0, 319.5, 239.5, 640, 480)


def cfg2_trajectory(n_frames=200, seed=11):
    """Camera path mixing slow motion, fast translation and in-place yaw bursts.

    Positions stay in a safe region of the 6x5x3 m room; pitch is kept within +-20 degrees.
    Returns room-frame (R_rc, c_r) per frame, and frame 0 has yaw = pitch = roll = 0.
    """
    rng = np.random.default_rng(seed)
    pos = np.array([0.0, 0.0, -0.6])
    yaw = pitch = roll = 0.0
    lo_b, hi_b = np.array([-1.6, -0.5, -1.5]), np.array([1.6, 0.5, 1.2])
    out = [(_euler_yxz(yaw, pitch, roll), pos.copy())]
    f = 1
    while f < n_frames:
        kind = rng.choice(["slow", "fast", "yaw"], p=[0.45, 0.3, 0.25])
        seg = int(rng.integers(6, 16)) if kind != "yaw" else int(rng.integers(3, 8))
        vdir = rng.normal(size=3)
        vdir[1] *= 0.3
        vdir /= np.linalg.norm(vdir)
        speed = rng.uniform(0.06, 0.15)
        ysign = rng.choice([-1.0, 1.0])
        yrate = math.radians(rng.uniform(12.0, 25.0))
        for _ in range(seg):
            if f >= n_frames:
                break
            if kind == "slow":
                dp = rng.uniform(-1, 1, 3) * 0.02 / math.sqrt(3)
                dyaw = math.radians(rng.uniform(-2, 2))
                dpitch = math.radians(rng.uniform(-1, 1))
            elif kind == "fast":
                dp = vdir * speed
                dyaw = math.radians(rng.uniform(-2, 2))
                dpitch = math.radians(rng.uniform(-1, 1))
            else:
                dp = rng.uniform(-1, 1, 3) * 0.01 / math.sqrt(3)
                dyaw = ysign * yrate
                dpitch = math.radians(rng.uniform(-2, 2))
            npos = pos + dp
            # bounce off the safe region
            for a in range(3):
                if npos[a] < lo_b[a] or npos[a] > hi_b[a]:
                    dp[a] = -dp[a]
                    vdir[a] = -vdir[a]
            pos = np.clip(pos + dp, lo_b, hi_b)
            yaw += dyaw
            pitch = float(np.clip(pitch + dpitch, math.radians(-20), math.radians(20)))
            roll = float(np.clip(roll + math.radians(rng.uniform(-0.5, 0.5)), math.radians(-5), math.radians(5)))
            out.append((_euler_yxz(yaw, pitch, roll), pos.copy()))
            f += 1
    return out


def cfg2_scene(traj_room, seed=10, n_objects=20):
    """6x5x3 m room plus seeded spheres (r in [0.15, 0.5] m) and axis-aligned boxes (sides
    0.2-0.8 m), each at least 0.5 m from every camera position of the trajectory."""
    rng = np.random.default_rng(seed)
    lo, hi = np.array([-3.0, -1.5, -2.5]), np.array([3.0, 1.5, 2.5])
    cams = np.array([c for _, c in traj_room])
    spheres, boxes = [], []
    tries = 0
    while len(spheres) + len(boxes) < n_objects and tries < 10000:
        tries += 1
        if rng.random() < 0.5:
            r = rng.uniform(0.15, 0.5)
            c = rng.uniform(lo + r, hi - r)
            c[1] = rng.uniform(lo[1] + r, hi[1] - r)
            if np.min(np.linalg.norm(cams - c, axis=1)) < r + 0.5:
                continue
            spheres.append((c, r))
        else:
            s = rng.uniform(0.2, 0.8, 3)
            c = rng.uniform(lo + s / 2, hi - s / 2)
            c[1] = hi[1] - s[1] / 2 if rng.random() < 0.6 else c[1]   # most boxes stand on the floor
            blo, bhi = c - s / 2, c + s / 2
            dist = np.linalg.norm(np.maximum(np.maximum(blo - cams, cams - bhi), 0.0), axis=1)
            if np.min(dist) < 0.5:
                continue
            boxes.append((blo, bhi))
    R_rc1, c_r1 = traj_room[0]
    return make_room_scene(lo, hi, spheres, boxes, R_rc1, c_r1)


def world_trajectory(scene, traj_room):
    """Room-frame camera poses -> world-frame (camera -> world) poses."""
    out = []
    for R_rc, c_r in traj_room:
        out.append(pose_mul(scene["R_wr"], scene["t_wr"], R_rc, c_r))
    return out


def pr_standin(gt_prev, gt_cur, rng, sigma_rot_deg=3.0, sigma_t=0.03):
    """Stand-in for the pose-regression output P_(t,t-1): the ground-truth relative pose
    composed on the right with a seeded perturbation Exp(delta), delta ~ N(0, sigma^2)."""
    Rp, tp = gt_prev
    Rc, tc = gt_cur
    Ri, ti = pose_inv(Rp, tp)
    Rrel, trel = pose_mul(Ri, ti, Rc, tc)
    dr = rng.normal(0.0, math.radians(sigma_rot_deg), 3)
    dt = rng.normal(0.0, sigma_t, 3)
    return pose_mul(Rrel, trel, rot(dr), dt)


CFG2_LENGTH = 200


def cfg2_frames(n_frames=CFG2_LENGTH, traj_seed=11, scene_seed=10, noise_seed=12, pr_seed=13, pr_sigma_deg=3.0,
                pr_sigma_m=0.03):
    """The paper-scale sequence: scene, world GT poses, noisy depth maps (lazy) and PR stand-ins.

    The scene is always placed against the full 200-frame trajectory, so the first n_frames of
    any call are the same frames. Depth maps are rendered on demand by `depth(t)` so callers can
    bound host memory.
    """
    traj_full = cfg2_trajectory(max(n_frames, CFG2_LENGTH), traj_seed)
    scene = cfg2_scene(traj_full, scene_seed)
    traj_room = traj_full[:n_frames]
    gt = world_trajectory(scene, traj_room)
    vol = VolumeSpec.centred(512, 0.01, 0.04, room_centre_world(scene))
    rng = np.random.default_rng(pr_seed)
    rel = [None] + [pr_standin(gt[t - 1], gt[t], rng, pr_sigma_deg, pr_sigma_m) for t in range(1, n_frames)]

    def depth(t):
        d = render_depth(scene, CFG2_INTR, *gt[t])
        return add_noise_axial(d, 0.0015, 0.02, noise_seed * 100003 + t)

    return {"scene": scene, "intr": CFG2_INTR, "vol": vol, "gt": gt, "rel": rel, "depth": depth}


def room_spec(scene, voxel_size: float, trunc: float, edge: int = 8) -> VolumeSpec:
    """A grid over the whole room of a scene whose room frame is axis-aligned with the world (as
    cfg2's is: its frame-0 camera has no rotation), with one truncation distance of margin beyond
    every wall, each dimension rounded up to a multiple of `edge` (the brick edge)."""
    assert np.allclose(scene["R_wr"], np.eye(3)), "the room must be axis-aligned with the world"
    ext = scene["room_hi"] - scene["room_lo"] + 2.0 * trunc
    n = [int(math.ceil(e / voxel_size / edge - 1e-9)) * edge for e in ext]
    c = room_centre_world(scene)
    o = tuple(float(c[a]) - 0.5 * n[a] * voxel_size + 0.5 * voxel_size for a in range(3))
    return VolumeSpec(n[0], n[1], n[2], float(voxel_size), float(trunc), o)


# ----------------------------------------------------------------------------- batched problems
def random_depth_for_batch(p: int, base_seed=40):
    """One of the 64 heterogeneous tracking problems: its own small room, resolution drawn
    from {160x120, 320x240, 480x360, 640x480} with fx = fy = 0.75 W, its own 256^3 volume at
    1 cm (tau 4 cm), K drawn from [256, 4096] and its own init perturbation (3 deg, 3 cm)."""
    rng = np.random.default_rng(base_seed + p)
    W, H = [(160, 120), (320, 240), (480, 360), (640, 480)][int(rng.integers(0, 4))]
    intr = Intrinsics(0.75 * W, 0.75 * W, W / 2.0, H / 2.0, W, H)
    K = int(rng.integers(256, 4097))
    lo, hi = np.array([-1.2, -1.0, -1.2]), np.array([1.2, 1.0, 1.2])
    c_r1 = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.2, 0.2), rng.uniform(-0.5, -0.2)])
    R_rc1 = _euler_yxz(rng.uniform(-0.6, 0.6), rng.uniform(-0.3, 0.1), 0.0)
    spheres = []
    while len(spheres) < 3:
        r = rng.uniform(0.15, 0.35)
        c = rng.uniform(lo + r + 0.2, hi - r - 0.2)
        if np.linalg.norm(c - c_r1) < r + 0.5:
            continue
        spheres.append((c, r))
    scene = make_room_scene(lo, hi, spheres, [], R_rc1, c_r1)
    vol = VolumeSpec.centred(256, 0.01, 0.04, room_centre_world(scene))
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    R2 = rot(math.radians(rng.uniform(2, 8)) * axis)
    t2 = rng.normal(size=3)
    t2 *= rng.uniform(0.01, 0.05) / np.linalg.norm(t2)
    I3 = np.eye(3)
    d1 = add_noise_additive(render_depth(scene, intr, I3, np.zeros(3)), 0.002, base_seed + 1000 + p)
    d2 = add_noise_additive(render_depth(scene, intr, R2, t2), 0.002, base_seed + 2000 + p)
    dr = rng.normal(0, math.radians(3.0), 3)
    dt = rng.normal(0, 0.03, 3)
    Ri, ti = pose_mul(R2, t2, rot(dr), dt)
    return {"intr": intr, "K": K, "vol": vol, "depth1": d1, "depth2": d2,
            "gt2": (R2, t2), "init2": (Ri, ti), "scene": scene}


# ----------------------------------------------------------------------------- analytic volumes
def _centres(vol: VolumeSpec):
    i = np.arange(vol.nx) * vol.voxel_size + vol.origin[0]
    j = np.arange(vol.ny) * vol.voxel_size + vol.origin[1]
    k = np.arange(vol.nz) * vol.voxel_size + vol.origin[2]
    Z, Y, X = np.meshgrid(k, j, i, indexing="ij")
    return X, Y, Z


def _band(sdf: np.ndarray, tau: float) -> np.ndarray:
    """Normalised TSDF fixture: sdf/tau inside the band |sdf| < tau, +1 (unobserved) outside."""
    t = sdf / tau
    return np.where(np.abs(t) < 1.0, t, 1.0)


def fill_plane_volume(vol: VolumeSpec, n, d) -> np.ndarray:
    """Signed distance to the plane n.x = d (n unit), positive on the side n.x < d, as an
    x-fastest (nz, ny, nx) float64 array, normalised and banded."""
    X, Y, Z = _centres(vol)
    n = np.asarray(n, np.float64)
    sdf = d - (n[0] * X + n[1] * Y + n[2] * Z)
    return _band(sdf, vol.trunc)


def fill_sphere_volume(vol: VolumeSpec, c, r, inside_positive=False) -> np.ndarray:
    X, Y, Z = _centres(vol)
    dist = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) - r
    return _band(-dist if inside_positive else dist, vol.trunc)


def fill_room_volume(vol: VolumeSpec, scene) -> np.ndarray:
    """Signed distance to the interior walls of the room (positive inside)."""
    X, Y, Z = _centres(vol)
    P = np.stack([X, Y, Z], -1) @ scene["R_rw"].T + scene["t_rw"]
    lo, hi = scene["room_lo"], scene["room_hi"]
    dist = np.minimum(P - lo, hi - P).min(axis=-1)
    return _band(dist, vol.trunc)


# ----------------------------------------------------------------------------- evaluation helpers
def _box_distance(P, lo, hi):
    """Unsigned distance from points P (N, 3) to the surface of the axis-aligned box [lo, hi]."""
    q = np.maximum(lo - P, P - hi)                       # > 0 outside along an axis
    outside = np.linalg.norm(np.maximum(q, 0.0), axis=1)
    inside = -np.max(q, axis=1)                          # distance to the nearest face from inside
    return np.where(np.max(q, axis=1) > 0.0, outside, inside)


def scene_distance(scene, P_world) -> np.ndarray:
    """Unsigned distance from world points (N, 3) to the nearest surface of the analytic scene
    (room walls, spheres, boxes), for reconstruction accuracy against the true geometry."""
    P = np.asarray(P_world, np.float64) @ scene["R_rw"].T + scene["t_rw"]
    d = _box_distance(P, scene["room_lo"], scene["room_hi"])
    for c, r in scene["spheres"]:
        d = np.minimum(d, np.abs(np.linalg.norm(P - c, axis=1) - r))
    for lo, hi in scene["boxes"]:
        d = np.minimum(d, _box_distance(P, lo, hi))
    return d


def backproject_world(depth, K: Intrinsics, R_wc, t_wc, stride: int = 1) -> np.ndarray:
    """World points of the valid pixels of a depth map (every `stride`-th pixel in u and v)."""
    d = np.asarray(depth, np.float64)[::stride, ::stride]
    v, u = np.nonzero(d > 0)
    z = d[v, u]
    u = u * stride
    v = v * stride
    X = np.stack([(u - K.cx) * z / K.fx, (v - K.cy) * z / K.fy, z], 1)
    return X @ np.asarray(R_wc, np.float64).T + np.asarray(t_wc, np.float64)
