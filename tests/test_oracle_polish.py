"""Pins of the oracle's gradient polish and of the candidate it starts from, against closed forms.

The polish is not in the paper (which optimizes with particles only); its rule is stated in the
oracle: steps xi = -alpha grad E with the first alpha of each step making the point-displacement
bound alpha (|g_rho| + |g_phi| Rmax) half a voxel, Armijo acceptance E_new <= E - c alpha |g|^2
with c = 1e-4, up to 5 halvings, stop when none is accepted. On an affine (plane) field every
quantity of that rule has a closed form, computed here with numpy and scipy only:
  T(y) = (d - n.y) / tau  =>  grad T = -n / tau,
  g_rho = -s n / tau,  g_phi = mean_j (y_j - c) x g_rho  (s = sign of the common offset, c the
  camera centre), and E = mean_j |d - n.y_j| / tau while no point crosses the plane.
A point offset delta from the plane moved by D along s n ends at |delta - D|, so with no rotation
(g_phi = 0) a trial of displacement D is accepted iff D (1 + c) <= 2 delta (for D > delta). Those
thresholds pin the first alpha, the halving factor, the number of halvings and c. CPU only."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth

TAU, VS = 0.08, 0.02
N = np.array([0.1, -0.2, -1.0]) / np.linalg.norm([0.1, -0.2, -1.0])
C0 = np.array([0.0, 0.0, 1.2])
D_PLANE = float(N @ C0)


def _plane_vol(orc):
    spec = synth.VolumeSpec.centred(64, VS, TAU, tuple(C0))
    return orc.Volume(spec, T=synth.fill_plane_volume(spec, N, D_PLANE))


def _plane_points(seed=0, n=400):
    """Points on the plane, symmetric about C0 (each (a, b) with its negative), so their mean is C0."""
    u = np.cross(N, [1.0, 0.0, 0.0])
    u /= np.linalg.norm(u)
    w = np.cross(N, u)
    ab = np.random.default_rng(seed).uniform(-0.3, 0.3, (n // 2, 2))
    ab = np.concatenate([ab, -ab])
    return C0 + ab[:, :1] * u + ab[:, 1:] * w


def _closed_form_step(Y, t, delta_sign):
    """g_rho, g_phi, Rmax and the first alpha of a polish step at world points Y, camera centre t
    (decoupled composition: the rotation acts about t)."""
    g_rho = -delta_sign * N / TAU
    U = Y - t
    g_phi = np.mean(np.cross(U, g_rho), axis=0)
    rmax = np.max(np.linalg.norm(U, axis=1))
    alpha = 0.5 * VS / (np.linalg.norm(g_rho) + np.linalg.norm(g_phi) * rmax)
    return g_rho, g_phi, rmax, alpha


def _apply(Y, R, t, xi):
    """Pose after xi = (rho, phi) with the decoupled composition (exp(phi) R, t + rho), and the
    moved world points."""
    E = Rotation.from_rotvec(xi[3:]).as_matrix()
    R2, t2 = E @ R, t + xi[:3]
    return R2, t2, (Y - t) @ E.T + t2


def _E(Y):
    return float(np.mean(np.abs(D_PLANE - Y @ N)) / TAU)


def _setup(delta, t_off):
    Y = _plane_points() - delta * N            # every point at signed distance delta
    t = C0 - (delta + 1.0) * N + np.asarray(t_off)  # on the normal through the mean when t_off = 0
    R = np.eye(3)
    X = Y - t                                  # camera coordinates (R = I)
    return Y, X, R, t


@pytest.mark.parametrize("t_off", [(0.0, 0.0, 0.0), (0.25, 0.1, 0.05)])
def test_polish_first_steps_closed_form(orc, t_off):
    """The first step (and the second) equal the closed-form alpha and compose(-alpha g)."""
    vol = _plane_vol(orc)
    delta = 0.03
    Y, X, R, t = _setup(delta, t_off)
    E0 = _E(Y)
    Eo, go, nv = vol.fitness_grad(X, R, t, 0)
    assert nv == X.shape[0] and abs(Eo - E0) <= 1e-13
    R_ref, t_ref, Y_ref = R, t, Y
    for steps in (1, 2):
        g_rho, g_phi, rmax, alpha = _closed_form_step(Y_ref, t_ref, 1.0)
        if steps == 1:
            assert np.abs(go[:3] - g_rho).max() <= 1e-12 and np.abs(go[3:] - g_phi).max() <= 1e-12
            if t_off == (0.0, 0.0, 0.0):
                assert np.abs(g_phi).max() <= 1e-12          # lever arms' mean lies along n
            else:
                assert np.abs(g_phi).max() > 1e-2             # the rotation part is exercised
        xi = -alpha * np.concatenate([g_rho, g_phi])
        R_new, t_new, Y_new = _apply(Y_ref, R_ref, t_ref, xi)
        gg = float(g_rho @ g_rho + g_phi @ g_phi)
        assert _E(Y_new) <= _E(Y_ref) - 1e-4 * alpha * gg       # the first trial is accepted
        R_ref, t_ref, Y_ref = R_new, t_new, Y_new
        R_o, t_o, acc, E_o = vol.polish(X, R, t, steps=steps)
        assert acc == steps
        assert np.abs(R_o - R_ref).max() <= 1e-12 and np.abs(t_o - t_ref).max() <= 1e-12
        assert abs(E_o - _E(Y_ref)) <= 1e-12
    # half a voxel bounds the first step's largest point displacement
    g_rho, g_phi, rmax, alpha = _closed_form_step(Y, t, 1.0)
    _, _, Y1 = _apply(Y, R, t, -alpha * np.concatenate([g_rho, g_phi]))
    assert np.max(np.linalg.norm(Y1 - Y, axis=1)) <= 0.5 * VS * (1 + 1e-6)


# displacement of trial h is D_h = (VS / 2) / 2^h along n (no rotation); acceptance iff
# D_h (1 + 1e-4) <= 2 delta once D_h > delta
D5 = 0.5 * VS / 32


@pytest.mark.parametrize("delta,accepted_at", [
    (0.03, 0),                    # D_0 = 1 cm < delta: the first trial
    (0.004, 1),                   # D_0 = 10 mm > 8 mm, D_1 = 5 mm <= 8 mm
    (0.0002, 5),                  # D_4 = 0.625 mm > 0.4 mm >= D_5 = 0.3125 mm: the fifth halving
    (0.5 * D5 * (1 + 2e-4), 5),   # D_5 (1 + 1e-4) <= 2 delta: accepted (c < 2e-4)
    (0.5 * D5 * (1 + 0.5e-4), None),  # D_5 (1 + 1e-4) > 2 delta: rejected (c > 0.5e-4); no sixth halving
    (0.0001, None),               # 2 delta = 0.2 mm < D_5: every trial overshoots
])
def test_polish_halvings_and_armijo_constant(orc, delta, accepted_at):
    vol = _plane_vol(orc)
    Y, X, R, t = _setup(delta, (0.0, 0.0, 0.0))
    E0 = _E(Y)
    R_o, t_o, acc, E_o = vol.polish(X, R, t, steps=1)
    if accepted_at is None:
        assert acc == 0
        assert np.array_equal(R_o, R) and np.array_equal(t_o, t)
        assert abs(E_o - E0) <= 1e-13
        return
    assert acc == 1
    g_rho, g_phi, _, alpha = _closed_form_step(Y, t, 1.0)
    a = alpha / 2 ** accepted_at
    R_ref, t_ref, Y_ref = _apply(Y, R, t, -a * np.concatenate([g_rho, g_phi]))
    assert np.abs(t_o - t_ref).max() <= 1e-13 and np.abs(R_o - R_ref).max() <= 1e-13
    D = 0.5 * VS / 2 ** accepted_at
    assert abs(E_o - abs(delta - D) / TAU) <= 1e-10
    assert abs(E_o - _E(Y_ref)) <= 1e-12


def test_polish_stops_when_nothing_is_accepted(orc):
    """With several steps requested, the first step that accepts nothing ends the polish."""
    vol = _plane_vol(orc)
    Y, X, R, t = _setup(0.0002, (0.0, 0.0, 0.0))
    _, _, acc, E = vol.polish(X, R, t, steps=5)
    # step 1 lands 0.1125 mm past the plane (delta - D_5); step 2 starts from the same first alpha
    # (the gradient norm is unchanged) and needs D <= 0.225 mm: D_5 = 0.3125 mm overshoots
    assert acc == 1
    assert abs(E - (D5 - 0.0002) / TAU) <= 1e-10


@pytest.mark.parametrize("seed", range(6))
def test_best_candidate_rule(orc, seed):
    """Lowest fitness among P^(I) (Estar) and the last iteration's particles; ties to P^(I), then to
    the lowest index: the first minimum of the list [Estar, E_1 .. E_K]."""
    rng = np.random.default_rng(seed)
    K = int(rng.integers(0, 40))
    E = np.concatenate([[np.nan], rng.choice([0.1, 0.2, 0.3], K)])   # slot 0 (E_0) is not a candidate
    Estar = float(rng.choice([0.1, 0.2, 0.3]))
    cand = np.concatenate([[Estar], E[1:]])
    assert orc.best_candidate(Estar, E) == int(np.argmin(cand))


def test_best_candidate_hand_built(orc):
    nan = np.nan
    assert orc.best_candidate(0.3, np.array([nan, 0.4, 0.3, 0.5])) == 0          # a tie with P^(I)
    assert orc.best_candidate(0.3, np.array([nan, 0.4, 0.2, 0.25, 0.2])) == 2    # tie between particles
    assert orc.best_candidate(0.3, np.array([nan, 0.29999999999999993])) == 1
    assert orc.best_candidate(0.3, np.array([nan])) == 0                        # no particles
    assert orc.best_candidate(1.0, np.array([nan, 1.0, 1.0])) == 0              # nothing observed
