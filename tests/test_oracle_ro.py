"""Pins of the oracle's randomized optimization (Sec. III-B), its gradient and polish, against
special cases with known answers, brute force over a pose grid, and convergence on a scene
whose TSDF is exact (piecewise affine). CPU only."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth


def _deltas(rng, K):
    d = np.zeros((K + 1, 6))
    d[1:, :3] = rng.uniform(-0.05, 0.05, (K, 3))
    d[1:, 3:] = rng.uniform(-0.03, 0.03, (K, 3))
    return d


def test_advantage_single_member_returns_that_delta(orc):
    rng = np.random.default_rng(0)
    R = Rotation.from_rotvec([0.1, 0.2, -0.1]).as_matrix()
    t = np.array([0.3, -0.2, 0.1])
    d = _deltas(rng, 5)
    E = np.array([0.5, 0.6, 0.5, 0.49999, 0.7, 0.9])          # equal fitness is not an advantage
    na, R2, t2, mean = orc.advantage_update(E, d, R, t)
    assert na == 1 and np.array_equal(mean, d[3])
    Rr, tr = orc.compose(d[3, :3], d[3, 3:], R, t)
    assert np.array_equal(R2, Rr) and np.array_equal(t2, tr)


def test_advantage_symmetric_pair_and_empty(orc):
    R, t = np.eye(3), np.array([0.1, 0.0, 0.0])
    d = np.zeros((3, 6))
    d[1] = [0.02, -0.01, 0.03, 0.01, 0.02, -0.004]
    d[2] = [-0.02, 0.01, -0.03, 0.03, -0.01, 0.006]
    na, R2, t2, mean = orc.advantage_update(np.array([1.0, 0.2, 0.3]), d, R, t)
    assert na == 2
    assert np.array_equal(mean[:3], [0.0, 0.0, 0.0])
    assert np.array_equal(R2, R)
    assert np.abs(t2 - (t + 0.5 * (d[1, 3:] + d[2, 3:]))).max() <= 1e-17
    na, R3, t3, _ = orc.advantage_update(np.array([0.1, 0.2, 0.3]), d, R, t)
    assert na == 0 and np.array_equal(R3, R) and np.array_equal(t3, t)


def test_draw_delta_in_box(orc):
    for k in range(1, 200):
        r, tau = orc.draw_delta(9, 4, 2, k, math.radians(10), 0.1)
        assert np.all(np.abs(r) <= math.radians(10)) and np.all(np.abs(tau) <= 0.1)
        assert r[0] == math.radians(10) * orc.uniform_pm1(9, 4, 2, k, 0)
        assert tau[2] == 0.1 * orc.uniform_pm1(9, 4, 2, k, 5)


def _plane_problem(seed=0):
    rng = np.random.default_rng(seed)
    spec = synth.VolumeSpec.centred(64, 0.02, 0.08, (0.0, 0.0, 1.2))
    n = np.array([0.1, -0.2, -1.0])
    n /= np.linalg.norm(n)
    c = np.array([0.0, 0.0, 1.2])
    T = synth.fill_plane_volume(spec, n, float(n @ c))
    u = np.cross(n, [1.0, 0, 0])
    u /= np.linalg.norm(u)
    w = np.cross(n, u)
    ab = rng.uniform(-0.3, 0.3, (800, 2))
    P = c + ab[:, :1] * u + ab[:, 1:] * w
    return spec, T, P


def test_search_size_special_cases(orc):
    # E* = 1 (nothing observed): A is empty, the pose is unchanged and s keeps its value
    spec = synth.VolumeSpec.centred(32, 0.02, 0.08, (0, 0, 1))
    vol = orc.Volume(spec)
    prm = orc.make_params(K=32, n_iters=1)
    S = np.array([[0.0, 0.0, 1.0], [0.05, 0.0, 1.0]])
    R, t, sr, sm, E, nv, rec = vol.ro_iteration(S, prm, 1, np.eye(3), np.zeros(3), 0.1, 0.05)
    assert rec.n_adv == 0 and np.all(E == 1.0) and rec.Estar == 1.0
    assert sr == 0.1 and sm == 0.05
    assert np.array_equal(R, np.eye(3)) and np.array_equal(t, np.zeros(3))
    # E* = 0 (points exactly on an affine field at the optimum): every particle is worse, the
    # pose stays, and s shrinks by exactly beta
    spec, T, P = _plane_problem()
    vol = orc.Volume(spec, T=T)
    R, t, sr, sm, E, nv, rec = vol.ro_iteration(P, prm, 1, np.eye(3), np.zeros(3), 0.1, 0.05)
    assert E[0] <= 1e-14 and rec.n_adv == 0 and rec.Estar == E[0]
    assert sr == 0.1 * (0.1 + 0.9 * rec.Estar) and sm == 0.05 * (0.1 + 0.9 * rec.Estar)
    assert abs(sr - 0.01) <= 1e-15


def test_near_tie_count(orc):
    """The record counts the particles whose fitness is within 1e-4 relative of E_0: all of them when
    nothing is observed (every E_k = E_0 = 1), and otherwise exactly those the returned values show."""
    spec = synth.VolumeSpec.centred(32, 0.02, 0.08, (0, 0, 1))
    prm = orc.make_params(K=32, n_iters=1)
    S = np.array([[0.0, 0.0, 1.0], [0.05, 0.0, 1.0]])
    *_, E, nv, rec = orc.Volume(spec).ro_iteration(S, prm, 1, np.eye(3), np.zeros(3), 0.1, 0.05)
    assert rec.n_near == 32
    d = synth.cfg1_inputs()
    vol = orc.Volume(d["vol"])
    vol.integrate(d["depth1"], d["intr"], np.eye(3), np.zeros(3))
    X, _ = orc.backproject(d["depth2"], d["intr"], 2)
    prm = orc.make_params(K=512, n_iters=1)
    for s_deg in (5.0, 0.001):
        *_, E, nv, rec = vol.ro_iteration(X, prm, 1, *d["init2"], np.radians(s_deg), s_deg / 100.0)
        near = int(np.sum(np.abs(E[1:] - E[0]) <= 1e-4 * E[0]))
        assert rec.n_near == near
    assert near > 100   # at a tiny spread most particles tie with the current pose


def test_search_size_lower_bound_over_iterations(orc):
    d = synth.cfg1_inputs()
    vol = orc.Volume(d["vol"])
    vol.integrate(d["depth1"], d["intr"], np.eye(3), np.zeros(3))
    prm = orc.make_params(K=64, n_iters=6)
    Ri, ti = d["init2"]
    R, t, recs = vol.track_frame(d["depth2"], d["intr"], Ri, ti, prm)
    s1 = math.radians(5.0)
    for i, rec in enumerate(recs):
        assert rec.s_rad >= 0.1 ** i * s1 * (1 - 1e-15)
        assert 0 <= rec.Estar <= 1
        if i + 1 < len(recs):
            assert recs[i + 1].s_rad == rec.s_rad * (0.1 + 0.9 * rec.Estar)
            assert recs[i + 1].s_rad <= rec.s_rad


def _piecewise_affine_room():
    """A 2 m box room seen from inside: its TSDF (distance to the nearest wall, banded) is
    affine on every cell away from the room's edges, so the fitness vanishes at the true pose."""
    lo, hi = np.array([-1.0, -1.0, -1.0]), np.array([1.0, 1.0, 1.0])
    R_rc1 = Rotation.from_euler("YXZ", [0.5, -0.3, 0.1]).as_matrix()
    scene = synth.make_room_scene(lo, hi, [], [], R_rc1, np.array([-0.2, -0.1, -0.3]))
    spec = synth.VolumeSpec.centred(64, 0.04, 0.16, synth.room_centre_world(scene))
    T = synth.fill_room_volume(spec, scene)
    K = synth.Intrinsics(30.0, 30.0, 19.5, 14.5, 40, 30)
    return scene, spec, T, K


def test_exhaustive_grid_argmin_is_ground_truth(orc):
    scene, spec, T, K = _piecewise_affine_room()
    vol = orc.Volume(spec, T=T)
    R_gt = Rotation.from_rotvec([0.03, -0.05, 0.02]).as_matrix()
    t_gt = np.array([0.04, -0.03, 0.05])
    depth = synth.render_depth(scene, K, R_gt, t_gt)
    X, _ = orc.backproject(depth, K, 1)
    rot_step, trans_step = math.radians(2.0), 0.03
    # the grid is centred one step away from GT on every axis; GT is then a grid node
    r_off = np.array([rot_step, -rot_step, rot_step])
    t_off = np.array([-trans_step, trans_step, trans_step])
    Rc, tc = orc.compose(r_off, t_off, R_gt, t_gt)
    best, E = vol.grid_search(X, Rc, tc, 5, rot_step, trans_step)
    idx = np.unravel_index(best, (5,) * 6)
    assert list(idx) == [1, 3, 1, 3, 1, 1]
    assert E[best] == E.min() and np.sum(E == E.min()) == 1
    # the randomized optimization from the grid centre (paper defaults s1 = (10 deg, 10 cm)) moves
    # toward GT on both components; the search size contracts by beta + (1 - beta) E* per
    # iteration, so a start this far off is not expected to reach GT exactly
    prm = orc.make_params(K=1024, n_iters=20, rates=(1,), pixel_stride=1, s1_deg=10.0, s1_m=0.10)
    vol2 = orc.Volume(spec, T=T)
    R, t, recs = vol2.track_frame(depth, K, Rc, tc, prm)
    assert orc.rot_err(R, R_gt) < 0.6 * orc.rot_err(Rc, R_gt)
    assert np.linalg.norm(t - t_gt) < 0.8 * np.linalg.norm(tc - t_gt)
    assert recs[-1].Estar < 0.25 * E[np.ravel_multi_index((2,) * 6, (5,) * 6)]


def test_ro_improves_on_exact_field(orc):
    """On an exact (piecewise affine) TSDF the iteration moves toward the true pose on both
    components and lowers the fitness; the contraction of s by beta + (1 - beta) E* per
    iteration makes the method a local refiner, so only a fraction of the offset is removed."""
    scene, spec, T, K = _piecewise_affine_room()
    K = synth.Intrinsics(60.0, 60.0, 39.5, 29.5, 80, 60)
    vol = orc.Volume(spec, T=T)
    R_gt = Rotation.from_rotvec([-0.02, 0.04, 0.01]).as_matrix()
    t_gt = np.array([0.02, 0.01, -0.03])
    depth = synth.render_depth(scene, K, R_gt, t_gt)
    Ri, ti = orc.compose([0.03, -0.02, 0.025], [0.02, -0.015, 0.01], R_gt, t_gt)
    prm = orc.make_params(K=1024, n_iters=20, rates=(1,), pixel_stride=1, s1_deg=5.0, s1_m=0.05)
    R, t, recs = vol.track_frame(depth, K, Ri, ti, prm)
    e0 = (orc.rot_err(Ri, R_gt), np.linalg.norm(ti - t_gt))
    e1 = (orc.rot_err(R, R_gt), np.linalg.norm(t - t_gt))
    assert e1[0] < 0.5 * e0[0] and e1[1] < 0.75 * e0[1]
    assert recs[-1].Estar < 0.25 * recs[0].E0


@pytest.mark.parametrize("mode", [0, 1])
def test_gradient_matches_frozen_central_differences(orc, mode):
    d = synth.cfg1_inputs()
    vol = orc.Volume(d["vol"])
    vol.integrate(d["depth1"], d["intr"], np.eye(3), np.zeros(3))
    X, _ = orc.backproject(d["depth2"], d["intr"], 2)
    R, t = d["init2"]
    E, g, nv = vol.fitness_grad(X, R, t, mode)
    assert nv > 1000
    # at xi = 0 the frozen objective is sum s_j T_j / |X| = mean |T| = E
    assert abs(vol.fitness_frozen(X, R, t, np.zeros(6), mode) - E) <= 1e-15
    h = 1e-4
    fd = np.zeros(6)
    for a in range(6):
        e = np.zeros(6)
        e[a] = h
        fd[a] = (vol.fitness_frozen(X, R, t, e, mode) - vol.fitness_frozen(X, R, t, -e, mode)) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-6 * np.abs(g).max()


def test_gradient_plane_closed_form(orc):
    spec, T, P = _plane_problem(1)
    vol = orc.Volume(spec, T=T)
    n = np.array([0.1, -0.2, -1.0])
    n /= np.linalg.norm(n)
    for delta in (0.01, -0.02):
        Y = P - delta * n             # sdf = delta at every point
        R, t = np.eye(3), np.array([0.01, 0.02, -0.01])
        X = Y - t
        E, g, nv = vol.fitness_grad(X, R, t, 0)
        s = np.sign(delta)
        assert abs(E - abs(delta) / 0.08) <= 1e-13
        assert np.abs(g[:3] - (-s * n / 0.08)).max() <= 1e-12
        ref_phi = np.mean(np.cross(Y - t, -s * n / 0.08), axis=0)
        assert np.abs(g[3:] - ref_phi).max() <= 1e-12


def test_polish_decreases_fitness(orc):
    spec, T, P = _plane_problem(2)
    vol = orc.Volume(spec, T=T)
    n = np.array([0.1, -0.2, -1.0])
    n /= np.linalg.norm(n)
    t0 = np.array([0.0, 0.0, 0.0])
    R0 = Rotation.from_rotvec([0.01, -0.005, 0.0]).as_matrix()
    X = (P + 0.012 * n - t0) @ Rotation.from_rotvec([0.0, 0.0, 0.0]).as_matrix()
    E0, _ = vol.fitness(X, R0, t0)
    R1, t1, acc, E1 = vol.polish(X, R0, t0, steps=5)
    assert acc >= 1 and E1 < E0
    E1b, _ = vol.fitness(X, R1, t1)
    assert abs(E1b - E1) <= 1e-15


def _left_jacobian(phi):
    """Left Jacobian of SO(3) (textbook closed form): exp(phi + d) = exp(J_l(phi) d) exp(phi) + O(d^2)."""
    th = np.linalg.norm(phi)
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    return np.eye(3) + (1 - np.cos(th)) / th ** 2 * K + (th - np.sin(th)) / th ** 3 * K @ K


@pytest.mark.parametrize("mode", [0, 1])
def test_grad_xi_fd_chain_rule(orc, mode):
    """The oracle's xi-space finite differences agree with the closed-form chain rule through the
    SO(3) left Jacobian applied to the analytic gradient at the composed pose."""
    d = synth.cfg1_inputs()
    vol = orc.Volume(d["vol"])
    vol.integrate(d["depth1"], d["intr"], np.eye(3), np.zeros(3))
    X, _ = orc.backproject(d["depth2"], d["intr"], 2)
    R, t = d["init2"]
    xi0 = np.array([0.004, -0.003, 0.002, 0.03, -0.02, 0.015])       # (rho, phi)
    g_fd = vol.grad_xi_fd(X, R, t, xi0, mode)
    R0, t0 = orc.compose(xi0[3:], xi0[:3], R, t, mode)
    _, g, nv = vol.fitness_grad(X, R0, t0, mode)
    g_rho, g_phi = g[:3], g[3:]
    J = _left_jacobian(xi0[3:])
    if mode == 0:
        ref = np.concatenate([g_rho, J.T @ g_phi])
    else:
        ref = np.concatenate([g_rho, J.T @ (g_phi - np.cross(xi0[:3], g_rho))])
    assert np.abs(g_fd - ref).max() <= 1e-6 * np.abs(ref).max()
    # at xi0 = 0 the xi-space derivative is the analytic gradient itself
    assert np.abs(vol.grad_xi_fd(X, R, t, np.zeros(6), mode) - vol.fitness_grad(X, R, t, mode)[1]).max() \
        <= 1e-6 * np.abs(g).max()


@pytest.mark.parametrize("mode", [0, 1])
def test_grad_interval_contains_exact(orc, mode):
    d = synth.cfg1_inputs()
    vol = orc.Volume(d["vol"])
    vol.integrate(d["depth1"], d["intr"], np.eye(3), np.zeros(3))
    X, _ = orc.backproject(d["depth2"], d["intr"], 2)
    rng = np.random.default_rng(8)
    R0, t0 = d["init2"]
    poses = [orc.compose(rng.uniform(-0.05, 0.05, 3), rng.uniform(-0.02, 0.02, 3), R0, t0) for _ in range(12)]
    E, g, nv = vol.fitness_grad_many(X, poses, mode)
    lo, hi = vol.fitness_grad_interval_many(X, poses, mode, eps=1e-3)
    exact = np.concatenate([E[:, None], g], 1)
    assert np.all(lo <= exact + 1e-15) and np.all(exact <= hi + 1e-15)
    lo0, hi0 = vol.fitness_grad_interval_many(X, poses, mode, eps=0.0)
    assert np.abs(lo0 - exact).max() <= 1e-15 * np.abs(exact).max() * 10 and np.abs(hi0 - exact).max() <= 1e-13
    # the sign band only widens the interval
    lo1, hi1 = vol.fitness_grad_interval_many(X, poses, mode, eps=1e-3, sign_eps=1e-3)
    assert np.all(lo1 <= lo + 1e-15) and np.all(hi1 >= hi - 1e-15)
    assert np.any(lo1 < lo) or np.any(hi1 > hi)


# ----------------------------------------------------------------------------- the paper's schedule
@pytest.fixture(scope="module")
def cfg1_fused(orc):
    d = synth.cfg1_inputs()
    vol = orc.Volume(d["vol"])
    vol.integrate(d["depth1"], d["intr"], np.eye(3), np.zeros(3))
    return d, vol


def _same_pose(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_alternating_K_reduces_to_fixed_K(orc, cfg1_fused):
    """Sec. IV-A alternates the particle count with the sampling rate. With every entry equal to
    K the run is the fixed-K run bit for bit, and each iteration draws Ks[(i-1) mod 3]."""
    d, vol = cfg1_fused
    Ri, ti = d["init2"]
    base = dict(seed=5, n_iters=6, rates=(1, 2, 3), pixel_stride=2)
    fixed = vol.track_frame(d["depth2"], d["intr"], Ri, ti, orc.make_params(K=48, **base))
    alt = vol.track_frame(d["depth2"], d["intr"], Ri, ti, orc.make_params(Ks=(48, 48, 48), **base))
    assert _same_pose(fixed, alt)
    assert [r.n_adv for r in fixed[2]] == [r.n_adv for r in alt[2]]
    R, t, recs = vol.track_frame(d["depth2"], d["intr"], Ri, ti, orc.make_params(Ks=(16, 48, 80), **base))
    assert [r.n_particles for r in recs] == [16, 48, 80, 16, 48, 80]
    assert all(r.n_adv <= r.n_particles for r in recs)


def test_alternating_K_first_iteration_is_the_fixed_run(orc, cfg1_fused):
    """Iteration 1 only sees Ks[0]: the pose after it equals a one-iteration run with K = Ks[0]."""
    d, vol = cfg1_fused
    Ri, ti = d["init2"]
    a = vol.track_frame(d["depth2"], d["intr"], Ri, ti,
                        orc.make_params(seed=6, n_iters=3, Ks=(32, 64, 96), rates=(1, 1, 1)))
    b = vol.track_frame(d["depth2"], d["intr"], Ri, ti, orc.make_params(seed=6, n_iters=3, K=32, rates=(1, 1, 1)))
    assert a[2][0].n_adv == b[2][0].n_adv
    assert np.array_equal(a[2][0].pose.rt()[0], b[2][0].pose.rt()[0])
    assert a[2][0].Estar == b[2][0].Estar


def test_early_exit_rule(orc, cfg1_fused):
    """Stop once s^(i+1) = s^(i) (beta + (1 - beta) E*) is below the stop size in both parts: the run
    ends at the first such i, and its pose is the fixed-I run with I = that i (same stream)."""
    d, vol = cfg1_fused
    Ri, ti = d["init2"]
    base = dict(seed=7, K=64, rates=(1,), pixel_stride=2, s1_deg=5.0, s1_m=0.03)
    full = vol.track_frame(d["depth2"], d["intr"], Ri, ti, orc.make_params(n_iters=12, **base))
    assert len(full[2]) == 12                              # no stop size: all iterations run
    stop_deg, stop_m = 0.05, 0.0005
    R, t, recs = vol.track_frame(d["depth2"], d["intr"], Ri, ti,
                                 orc.make_params(n_iters=12, stop_deg=stop_deg, stop_m=stop_m, **base))
    n = len(recs)
    nxt = [(r.s_rad * (0.1 + 0.9 * r.Estar), r.s_m * (0.1 + 0.9 * r.Estar)) for r in full[2]]
    below = [sr < math.radians(stop_deg) and sm < stop_m for sr, sm in nxt]
    assert n == below.index(True) + 1 and 1 < n < 12
    ref = vol.track_frame(d["depth2"], d["intr"], Ri, ti, orc.make_params(n_iters=n, **base))
    assert _same_pose((R, t), ref)
    # a stop size above s^(2) ends the run after the first iteration
    one = vol.track_frame(d["depth2"], d["intr"], Ri, ti, orc.make_params(n_iters=12, stop_deg=90.0, stop_m=1.0, **base))
    assert len(one[2]) == 1
    assert _same_pose(one[:2], vol.track_frame(d["depth2"], d["intr"], Ri, ti, orc.make_params(n_iters=1, **base))[:2])
