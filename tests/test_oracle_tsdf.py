"""Pins of the oracle's fusion, TSDF query and fitness against closed forms: a fronto-parallel
plane (projective distance known exactly), affine fields (trilinear interpolation is exact),
a sphere (trilinear error bound), and the stated validity and empty-set rules. CPU only."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth

TAU = 0.08
VS = 0.02


def small_spec(n=48, vs=VS, tau=TAU, centre=(0.0, 0.0, 1.0)):
    return synth.VolumeSpec.centred(n, vs, tau, centre)


def centres(spec):
    i = np.arange(spec.nx) * spec.voxel_size + spec.origin[0]
    j = np.arange(spec.ny) * spec.voxel_size + spec.origin[1]
    k = np.arange(spec.nz) * spec.voxel_size + spec.origin[2]
    Z, Y, X = np.meshgrid(k, j, i, indexing="ij")
    return np.stack([X, Y, Z], -1)


# ----------------------------------------------------------------------------- fusion
@pytest.mark.parametrize("rotated", [False, True])
def test_integrate_fronto_parallel_plane_closed_form(orc, rotated):
    """A plane perpendicular to the optical axis at camera depth d: the projective distance of
    every voxel equals d - n.(p - t) with n the optical axis in world coordinates."""
    K = synth.Intrinsics(40.0, 40.0, 15.5, 11.5, 32, 24)
    R = Rotation.from_rotvec([0.05, -0.12, 0.03]).as_matrix() if rotated else np.eye(3)
    t = np.array([0.013, -0.021, 0.007]) if rotated else np.zeros(3)
    d = 1.0
    depth = np.full((24, 32), d, np.float32)
    spec = small_spec(48, 0.02, 0.08, centre=t + R @ np.array([0.0, 0.0, 1.0]))
    vol = orc.Volume(spec)
    vol.integrate(depth, K, R, t)
    P = centres(spec)
    q = (P - t) @ R                                # rows: R^T (p - t)
    eta = d - q[..., 2]
    # voxels well inside the viewing cone (2 pixels from the border) and in front of the camera
    inside = (q[..., 2] > 0.05) & (np.abs(q[..., 0] / q[..., 2]) < (16 - 2) / 40.0) & \
             (np.abs(q[..., 1] / q[..., 2]) < (12 - 2) / 40.0)
    upd = inside & (eta >= -0.08 + 1e-9)
    exp_T = np.minimum(1.0, eta / 0.08)
    assert upd.sum() > 1000
    assert np.abs(vol.T[upd] - exp_T[upd]).max() <= 1e-12
    assert np.all(vol.W[upd] == 1.0)
    behind_surface = inside & (eta < -0.08 - 1e-9)
    assert behind_surface.sum() > 100
    assert np.all(vol.W[behind_surface] == 0.0) and np.all(vol.T[behind_surface] == 1.0)
    behind_camera = q[..., 2] < -1e-9
    assert np.all(vol.W[behind_camera] == 0.0)
    # the same frame again: W counts frames, T is a fixed point of the running average
    T1 = vol.T.copy()
    for n in (2, 3):
        vol.integrate(depth, K, R, t)
        assert np.all(vol.W[upd] == n)
        assert np.abs(vol.T[upd] - T1[upd]).max() <= 1e-15 * 4


def test_integrate_running_average_and_cap(orc):
    K = synth.Intrinsics(40.0, 40.0, 15.5, 11.5, 32, 24)
    spec = small_spec(32, 0.02, 0.08)
    vol = orc.Volume(spec)
    d1, d2 = 1.0, 1.03
    vol.integrate(np.full((24, 32), d1, np.float32), K, np.eye(3), np.zeros(3))
    vol.integrate(np.full((24, 32), d2, np.float32), K, np.eye(3), np.zeros(3))
    P = centres(spec)
    z = P[..., 2]
    inside = (z > 0.3) & (np.abs(P[..., 0] / z) < 14 / 40) & (np.abs(P[..., 1] / z) < 10 / 40)
    both = inside & (d1 - z >= -0.08 + 1e-9)
    phi1 = np.minimum(1, (d1 - z) / 0.08)
    phi2 = np.minimum(1, (np.float32(d2) - z) / 0.08)
    assert np.abs(vol.T[both] - 0.5 * (phi1[both] + phi2[both])).max() <= 1e-12
    assert np.all(vol.W[both] == 2)
    # the weight cap: W stays at W_max and the update still averages with weight W_max
    vol2 = orc.Volume(spec, w_max=255, T=np.full(vol.T.shape, 0.25), W=np.full(vol.T.shape, 254.0))
    vol2.integrate(np.full((24, 32), d1, np.float32), K, np.eye(3), np.zeros(3))
    m = inside & (d1 - z >= -0.08 + 1e-9)
    assert np.all(vol2.W[m] == 255)
    assert np.abs(vol2.T[m] - (0.25 * 254 + phi1[m]) / 255).max() <= 1e-14
    vol2.integrate(np.full((24, 32), d1, np.float32), K, np.eye(3), np.zeros(3))
    assert np.all(vol2.W[m] == 255)
    exp2 = ((0.25 * 254 + phi1[m]) / 255 * 255 + phi1[m]) / 256
    assert np.abs(vol2.T[m] - exp2).max() <= 1e-14


def test_integrate_weights_integer_monotone(orc):
    d = synth.cfg1_inputs()
    spec = synth.VolumeSpec.centred(48, 0.05, 0.15, synth.room_centre_world(d["scene"]))
    vol = orc.Volume(spec)
    prev = vol.W.copy()
    rng = np.random.default_rng(5)
    for f in range(4):
        R = Rotation.from_rotvec(rng.normal(size=3) * 0.1).as_matrix()
        t = rng.normal(size=3) * 0.05
        depth = synth.render_depth(d["scene"], d["intr"], R, t)
        n = vol.integrate(depth, d["intr"], R, t)
        assert n == int((vol.W - prev).sum())
        assert np.all(vol.W >= prev) and np.all(vol.W - prev <= 1)
        assert np.all(vol.W == np.round(vol.W))
        assert np.all(np.abs(vol.T) <= 1.0)
        prev = vol.W.copy()


def test_integrate_ambiguity_flags(orc):
    K = synth.Intrinsics(40.0, 40.0, 15.5, 11.5, 32, 24)
    spec = small_spec(32, 0.02, 0.08)
    vol = orc.Volume(spec)
    depth = np.full((24, 32), 1.0, np.float32)
    n, flags = vol.integrate(depth, K, np.eye(3), np.zeros(3), pix_margin=1e-3, eta_margin=1e-6, want_flags=True)
    assert flags.dtype == np.uint8 and flags.mean() < 0.05


# ----------------------------------------------------------------------------- query and fitness
def test_sample_validity_rules(orc):
    spec = synth.VolumeSpec(6, 5, 4, 0.1, 0.3, (0.0, 0.0, 0.0))
    rng = np.random.default_rng(0)
    T = rng.uniform(-0.9, 0.9, (4, 5, 6))
    vol = orc.Volume(spec, T=T)
    # voxel centres return the stored value; the last cell index on each axis is n - 2
    ok, v = vol.sample([0.2, 0.1, 0.2])
    assert ok and v == T[2, 1, 2]
    ok, v = vol.sample([0.4 + 1e-12, 0.3 + 1e-12, 0.2 + 1e-12])
    assert ok
    assert not vol.sample([0.5 + 1e-9, 0.1, 0.1])[0]       # x cell would be n - 1
    assert not vol.sample([-1e-9, 0.1, 0.1])[0]             # below the grid
    # a +1 or -1 corner anywhere in the stencil invalidates the sample
    for corner in [(1, 1, 1), (2, 2, 2), (1, 2, 1)]:
        T2 = T.copy()
        T2[corner[2], corner[1], corner[0]] = 1.0
        assert not orc.Volume(spec, T=T2).sample([0.15, 0.15, 0.15])[0]
    T3 = T.copy()
    T3[1, 1, 1] = -1.0
    assert not orc.Volume(spec, T=T3).sample([0.15, 0.15, 0.15])[0]


def test_sample_is_multilinear(orc):
    spec = synth.VolumeSpec(6, 5, 4, 0.1, 0.3, (0.2, -0.1, 0.3))
    rng = np.random.default_rng(1)
    T = rng.uniform(-0.9, 0.9, (4, 5, 6))
    vol = orc.Volume(spec, T=T)
    for _ in range(300):
        g = rng.uniform(0, [4.999, 3.999, 2.999])
        y = np.array(spec.origin) + 0.1 * g
        ok, v = vol.sample(y)
        c = np.floor(g).astype(int)
        f = g - c
        ref = 0.0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    w = (f[0] if dx else 1 - f[0]) * (f[1] if dy else 1 - f[1]) * (f[2] if dz else 1 - f[2])
                    ref += w * T[c[2] + dz, c[1] + dy, c[0] + dx]
        assert ok and abs(v - ref) <= 1e-14


def _plane_setup(seed=0, n_pts=2000):
    rng = np.random.default_rng(seed)
    spec = small_spec(64, VS, TAU, centre=(0.0, 0.0, 1.2))
    n = rng.normal(size=3)
    n[2] = -abs(n[2]) - 1.0       # facing the camera
    n /= np.linalg.norm(n)
    c = np.array([0.0, 0.0, 1.2])
    dpl = float(n @ c)
    T = synth.fill_plane_volume(spec, n, dpl)
    u = np.cross(n, [1.0, 0, 0])
    u /= np.linalg.norm(u)
    w = np.cross(n, u)
    ab = rng.uniform(-0.35, 0.35, (n_pts, 2))
    P = c + ab[:, :1] * u + ab[:, 1:] * w            # world points on the plane
    R = Rotation.from_rotvec(rng.normal(size=3) * 0.2).as_matrix()
    t = rng.normal(size=3) * 0.05
    X = (P - t) @ R                                   # camera coordinates under pose (R, t)
    return spec, T, n, dpl, P, R, t, X


def test_fitness_zero_on_affine_field(orc):
    spec, T, n, dpl, P, R, t, X = _plane_setup()
    vol = orc.Volume(spec, T=T)
    E, nv = vol.fitness(X, R, t)
    assert nv == X.shape[0]
    assert E <= 1e-14


@pytest.mark.parametrize("delta", [0.004, -0.011, 0.023])
def test_fitness_normal_offset(orc, delta):
    spec, T, n, dpl, P, R, t, X = _plane_setup(1)
    vol = orc.Volume(spec, T=T)
    Xo = (P - delta * n - t) @ R
    E, nv = vol.fitness(Xo, R, t)
    assert nv == X.shape[0]
    assert abs(E - abs(delta) / TAU) <= 1e-13


def test_fitness_small_rotation_closed_form(orc):
    spec, T, n, dpl, P, R, t, X = _plane_setup(2)
    vol = orc.Volume(spec, T=T)
    r = np.array([0.004, -0.007, 0.002])
    Rn, tn = orc.compose(r, np.zeros(3), R, t, orc.COMPOSE_DECOUPLED)
    E, nv = vol.fitness(X, Rn, tn)
    RD = Rotation.from_rotvec(r).as_matrix()
    ref = np.mean(np.abs((P - t) @ (RD - np.eye(3)).T @ n)) / TAU
    assert nv == X.shape[0]
    assert abs(E - ref) <= 1e-12


def test_fitness_sphere_trilinear_bound(orc):
    spec = small_spec(128, VS, TAU, centre=(0.0, 0.0, 1.3))
    c, r = np.array([0.05, -0.03, 1.3]), 0.3
    vol = orc.Volume(spec, T=synth.fill_sphere_volume(spec, c, r))
    rng = np.random.default_rng(3)
    dirs = rng.normal(size=(3000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    P = c + r * dirs
    E, nv = vol.fitness(P, np.eye(3), np.zeros(3))
    bound = VS ** 2 / (4 * TAU * (r - math.sqrt(3) * VS))
    assert nv == P.shape[0]
    assert 0 < E <= bound


def test_fitness_empty_set_is_one(orc):
    spec = small_spec(16)
    vol = orc.Volume(spec)                    # all unobserved
    E, nv = vol.fitness(np.array([[0.0, 0.0, 1.0], [0.01, 0.0, 1.0]]), np.eye(3), np.zeros(3))
    assert E == 1.0 and nv == 0
    E, nv = vol.fitness(np.array([[50.0, 0.0, 1.0]]), np.eye(3), np.zeros(3))
    assert E == 1.0 and nv == 0


def test_fitness_interval_contains_value(orc):
    spec, T, n, dpl, P, R, t, X = _plane_setup(4)
    rng = np.random.default_rng(4)
    T = np.where(rng.random(T.shape) < 0.02, 1.0, T)     # holes make validity discontinuous
    vol = orc.Volume(spec, T=T)
    poses = [orc.compose(rng.normal(size=3) * 0.01, rng.normal(size=3) * 0.01, R, t) for _ in range(16)]
    E, nv = vol.fitness_many(X, poses)
    lo, hi, na = vol.fitness_interval_many(X, poses, eps=1e-3)
    assert np.all(lo <= E + 1e-15) and np.all(E <= hi + 1e-15)
    lo0, hi0, na0 = vol.fitness_interval_many(X, poses, eps=0.0)
    assert np.all(na0 == 0) and np.array_equal(lo0, hi0)
    assert np.abs(lo0 - E).max() <= 1e-15


# ----------------------------------------------------------------------------- sparse bricks
def test_integrate_bricks_matches_dense_per_brick(orc):
    """The bricked reading, rebuilt from the dense fusion: a brick is recorded at the first frame
    whose dense fusion into an empty volume leaves one of its voxels below +1 (phi < 1: in the
    band), and from then on its voxels hold the dense fusion of exactly the frames since then;
    every other voxel stays (+1, 0)."""
    d = synth.cfg1_inputs()
    E = 8
    spec = synth.VolumeSpec.centred(48, 0.05, 0.15, synth.room_centre_world(d["scene"]))
    rng = np.random.default_rng(21)
    frames = []
    for f in range(4):
        R = Rotation.from_rotvec(rng.normal(size=3) * 0.15).as_matrix()
        t = rng.normal(size=3) * 0.1
        frames.append((synth.render_depth(d["scene"], d["intr"], R, t), R, t))
    sparse = orc.Volume(spec)
    nb = (spec.nz // E, spec.ny // E, spec.nx // E)

    def per_brick(mask_vox):
        return mask_vox.reshape(nb[0], E, nb[1], E, nb[2], E).any(axis=(1, 3, 5))

    first = np.full(nb, -1)
    for f, (depth, R, t) in enumerate(frames):
        fresh = orc.Volume(spec)
        fresh.integrate(depth, d["intr"], R, t)
        band = per_brick(fresh.T < 1.0)
        new = band & (first < 0)
        first[new] = f
        assert sparse.integrate_bricks(depth, d["intr"], R, t, edge=E) == int(new.sum())
        assert np.array_equal(sparse.bricks.astype(bool), first >= 0)
    assert 0 < (first >= 0).sum() < first.size            # some bricks stay free space
    assert len(set(first[first >= 0].tolist())) > 1        # and some are recorded late
    # expected volume: per brick, the dense fusion of the frames from its first one on
    exp_T, exp_W = np.ones(sparse.T.shape), np.zeros(sparse.T.shape)
    for f0 in sorted(set(first[first >= 0].tolist())):
        dense = orc.Volume(spec)
        for depth, R, t in frames[f0:]:
            dense.integrate(depth, d["intr"], R, t)
        m = np.repeat(np.repeat(np.repeat(first == f0, E, 0), E, 1), E, 2)
        exp_T[m], exp_W[m] = dense.T[m], dense.W[m]
    assert np.array_equal(sparse.T, exp_T) and np.array_equal(sparse.W, exp_W)
    # the dense fusion also updates free space in front of surfaces, which the bricks leave out
    dense_all = orc.Volume(spec)
    for depth, R, t in frames:
        dense_all.integrate(depth, d["intr"], R, t)
    assert ((dense_all.W > 0) & (sparse.W == 0)).sum() > 100


def test_integrate_bricks_plane_records_only_the_band(orc):
    """A fronto-parallel plane filling the image: the recorded bricks are exactly those that hold
    a voxel with -tau <= eta < tau inside the view, from the closed-form projective distance
    (bricks whose only such voxels sit within 1e-6 of a decision boundary are not judged)."""
    K = synth.Intrinsics(40.0, 40.0, 15.5, 11.5, 32, 24)
    spec = synth.VolumeSpec(48, 40, 32, 0.02, 0.08, (-0.47, -0.39, 0.61))
    dpl = 0.9
    vol = orc.Volume(spec)
    assert vol.integrate_bricks(np.full((24, 32), dpl, np.float32), K, np.eye(3), np.zeros(3), edge=8) > 0
    P = centres(spec)
    z = P[..., 2]
    u = 40.0 * P[..., 0] / z + 15.5
    v = 40.0 * P[..., 1] / z + 11.5
    eta = dpl - z
    margin = 1e-6
    sure_in = (u > -0.5 + margin) & (u < 31.5 - margin) & (v > -0.5 + margin) & (v < 23.5 - margin)
    maybe_in = (u > -0.5 - margin) & (u < 31.5 + margin) & (v > -0.5 - margin) & (v < 23.5 + margin)
    sure_band = (eta >= -0.08 + margin) & (eta < 0.08 - margin)
    maybe_band = (eta >= -0.08 - margin) & (eta < 0.08 + margin)
    nb = (spec.nz // 8, spec.ny // 8, spec.nx // 8)
    red = lambda m: m.reshape(nb[0], 8, nb[1], 8, nb[2], 8).any(axis=(1, 3, 5))
    must = red(sure_in & sure_band)
    may = red(maybe_in & maybe_band)
    got = vol.bricks.astype(bool)
    assert must.sum() > 4 and np.all(got[must]) and not np.any(got[~may])
    # in recorded bricks every viewed voxel in front of the plane is updated, beyond the band too
    rec = np.repeat(np.repeat(np.repeat(got, 8, 0), 8, 1), 8, 2)
    front = rec & sure_in & (eta >= 0.08 + margin)
    assert front.sum() > 0 and np.all(vol.W[front] == 1) and np.all(vol.T[front] == 1.0)
    assert np.all(vol.W[~rec] == 0) and np.all(vol.T[~rec] == 1.0)
