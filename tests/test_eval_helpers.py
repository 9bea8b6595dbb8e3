"""CPU pins of the evaluation helpers used by `bench.py --workload accuracy`: the analytic scene
distance and the TSDF zero-crossing extraction."""
import math
import os
import sys

import numpy as np

import synth

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_scene_distance_on_and_off_the_surfaces():
    f = synth.cfg2_frames(2)
    sc = f["scene"]
    R, t = f["gt"][1]
    d = synth.render_depth(sc, f["intr"], R, t)
    P = synth.backproject_world(d, f["intr"], R, t, stride=16)
    assert synth.scene_distance(sc, P).max() < 1e-6          # rendered points lie on a surface
    # a point at the room centre is as far from the walls as the nearest wall (no object there
    # closer than that is guaranteed only for the walls, so compare against the wall term alone)
    c_r = 0.5 * (sc["room_lo"] + sc["room_hi"])
    half = 0.5 * (sc["room_hi"] - sc["room_lo"])
    Pw = (c_r - sc["t_rw"]) @ sc["R_rw"]                       # room -> world
    assert synth.scene_distance(sc, Pw[None])[0] <= half.min() + 1e-12
    # sphere: a point at distance r + 0.1 from a lone sphere's centre
    lone = synth.make_room_scene([-50, -50, -50], [50, 50, 50], [(np.zeros(3), 0.3)], [], np.eye(3), np.zeros(3))
    assert abs(synth.scene_distance(lone, np.array([[0.4, 0.0, 0.0]]))[0] - 0.1) < 1e-12
    box = synth.make_room_scene([-50, -50, -50], [50, 50, 50], [], [(np.array([-1.0, -1, -1]), np.array([1.0, 1, 1]))],
                                np.eye(3), np.zeros(3))
    assert abs(synth.scene_distance(box, np.array([[2.0, 2.0, 0.0]]))[0] - math.sqrt(2)) < 1e-12
    assert abs(synth.scene_distance(box, np.array([[0.5, 0.0, 0.0]]))[0] - 0.5) < 1e-12


def test_surface_points_plane_exact_sphere_close():
    vol = synth.VolumeSpec.centred(48, 0.02, 0.08, np.zeros(3))
    n = np.array([0.3, -0.5, 0.81])
    n = n / np.linalg.norm(n)
    T = synth.fill_plane_volume(vol, n, 0.05).astype(np.float32)
    W = np.ones_like(T)
    S = bench.surface_points(T, W, vol.origin, vol.voxel_size)
    assert S.shape[0] > 1000
    assert np.abs(S @ n - 0.05).max() < 1e-5                  # a plane's TSDF is linear: exact
    Ts = synth.fill_sphere_volume(vol, np.zeros(3), 0.3).astype(np.float32)
    S2 = bench.surface_points(Ts, W, vol.origin, vol.voxel_size)
    r = np.linalg.norm(S2, axis=1)
    assert np.abs(r - 0.3).max() < 0.02 ** 2 / 0.3             # chord error of linear interpolation
    # unobserved voxels (W = 0) contribute nothing
    W0 = W.copy()
    W0[:, :, :24] = 0
    S3 = bench.surface_points(T, W0, vol.origin, vol.voxel_size)
    assert S3.shape[0] < S.shape[0] and (S3[:, 0] >= vol.origin[0] + 23 * vol.voxel_size - 1e-9).all()
