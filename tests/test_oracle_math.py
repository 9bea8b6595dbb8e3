"""Pins of the FP64 oracle's building blocks against mathematics it does not itself compute:
published generator outputs, textbook rotations, an independent rotation library, exact
round trips and closed forms. CPU only."""
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- RNG
def test_splitmix64_published_vectors(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_vectors.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) >= 6
    for seed, n, out in rows:
        assert orc.splitmix64(int(seed), int(n)) == int(out)


def test_uniform_mapping_exact_and_in_range(orc):
    for k in range(2000):
        x = orc.splitmix64(77, orc.counter(5, 3, k, k % 6))
        a = orc.uniform_pm1(77, 5, 3, k, k % 6)
        assert -1.0 <= a < 1.0
        # a = 2 (x >> 11) 2^-53 - 1 exactly: recover the integer
        assert (a + 1.0) * 2.0 ** 52 == float(x >> 11)


def test_counter_packing_distinct(orc):
    seen = set()
    for t in (0, 1, 199):
        for i in (1, 2, 20):
            for k in (0, 1, 3072, 10240):
                for d in range(6):
                    seen.add(orc.counter(t, i, k, d))
    assert len(seen) == 3 * 3 * 4 * 6


def test_uniform_chi_square(orc):
    n, bins = 60000, 20
    a = np.array([orc.uniform_pm1(3, 1, 1 + (j // 6000), j % 6000, j % 6) for j in range(n)])
    h, _ = np.histogram(a, bins=bins, range=(-1, 1))
    chi2 = ((h - n / bins) ** 2 / (n / bins)).sum()
    # 19 degrees of freedom: the 0.999 quantile is about 43.8
    assert chi2 < 43.8


# ----------------------------------------------------------------------------- SO(3)
def test_exp_properties(orc):
    rng = np.random.default_rng(0)
    assert np.array_equal(orc.so3_exp([0, 0, 0]), np.eye(3))
    for _ in range(200):
        r = rng.normal(size=3) * rng.choice([1e-8, 1e-3, 0.2, 1.0, 3.0])
        R = orc.so3_exp(r)
        assert np.abs(R.T @ R - np.eye(3)).max() <= 1e-15 * 8
        assert abs(np.linalg.det(R) - 1.0) <= 1e-14
        assert np.abs(orc.so3_exp(-r) - R.T).max() <= 1e-15 * 4
        # an independent implementation of the same map
        assert np.abs(R - Rotation.from_rotvec(r).as_matrix()).max() <= 5e-15


def test_exp_planar_textbook(orc):
    for th in (0.1, 1.0, 2.5):
        c, s = math.cos(th), math.sin(th)
        Rz = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
        assert np.abs(orc.so3_exp([0, 0, th]) - Rz).max() <= 1e-15 * 4
        Rx = np.array([[1.0, 0, 0], [0, c, -s], [0, s, c]])
        assert np.abs(orc.so3_exp([th, 0, 0]) - Rx).max() <= 1e-15 * 4


def test_exp_taylor_branch_continuity(orc):
    ax = np.array([0.6, -0.48, 0.64])
    lo = orc.so3_exp(ax * (1e-6 * (1 - 1e-12)))   # Taylor branch
    hi = orc.so3_exp(ax * (1e-6 * (1 + 1e-12)))   # Rodrigues branch
    assert np.abs(lo - hi).max() <= 1e-15


def test_log_inverts_exp(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        r = rng.normal(size=3)
        r *= rng.uniform(1e-9, 3.1) / np.linalg.norm(r)
        assert np.abs(orc.so3_log(orc.so3_exp(r)) - r).max() <= 1e-9 * max(1.0, np.linalg.norm(r))


def test_rot_err_metric(orc):
    for th in (1e-7, 1e-4, 0.01, 0.5, 2.0):
        R = orc.so3_exp([0, th, 0])
        assert abs(orc.rot_err(np.eye(3), R) - th) <= 1e-12 * max(1.0, th) + 1e-15


# ----------------------------------------------------------------------------- composition
def test_compose_modes(orc):
    rng = np.random.default_rng(2)
    R = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    t = rng.normal(size=3)
    r, tau = rng.normal(size=3) * 0.1, rng.normal(size=3) * 0.05
    E = Rotation.from_rotvec(r).as_matrix()
    Rd, td = orc.compose(r, tau, R, t, orc.COMPOSE_DECOUPLED)
    Rl, tl = orc.compose(r, tau, R, t, orc.COMPOSE_LITERAL)
    assert np.abs(Rd - E @ R).max() < 1e-14 and np.abs(Rl - E @ R).max() < 1e-14
    assert np.abs(td - (t + tau)).max() < 1e-15
    assert np.abs(tl - (E @ t + tau)).max() < 1e-14
    # the two readings agree when the camera sits at the origin
    R0, t0 = orc.compose(r, tau, R, np.zeros(3), orc.COMPOSE_DECOUPLED)
    R1, t1 = orc.compose(r, tau, R, np.zeros(3), orc.COMPOSE_LITERAL)
    assert np.abs(R0 - R1).max() == 0 and np.abs(t0 - t1).max() == 0
    # decoupled: a pure delta rotation keeps the camera centre fixed
    Rz, tz = orc.compose(r, np.zeros(3), R, t, orc.COMPOSE_DECOUPLED)
    assert np.array_equal(tz, t)


# ----------------------------------------------------------------------------- back-projection
def test_backprojection_round_trip(orc):
    K = synth.Intrinsics(525.0, 520.0, 319.5, 239.5, 64, 48)
    rng = np.random.default_rng(3)
    d = rng.uniform(0.3, 6.0, (48, 64)).astype(np.float32)
    d[rng.random(d.shape) < 0.1] = 0.0
    d[0, 5] = np.nan
    d[1, 7] = -1.0
    d[2, 9] = np.inf
    xyz, pix = orc.backproject(d, K, 1)
    valid = np.isfinite(d) & (d > 0)
    assert xyz.shape[0] == valid.sum()
    assert np.array_equal(pix, np.flatnonzero(valid.reshape(-1)))   # raster order
    u = K.fx * xyz[:, 0] / xyz[:, 2] + K.cx
    v = K.fy * xyz[:, 1] / xyz[:, 2] + K.cy
    assert np.abs(u - pix % 64).max() <= 1e-12 and np.abs(v - pix // 64).max() <= 1e-12
    assert np.array_equal(xyz[:, 2], d.reshape(-1)[pix].astype(np.float64))
    xyz2, pix2 = orc.backproject(d, K, 2)
    keep = (pix % 64 % 2 == 0) & (pix // 64 % 2 == 0)
    assert np.array_equal(pix2, pix[keep]) and np.array_equal(xyz2, xyz[keep])


def test_subsample_view(orc):
    x = np.arange(30.0).reshape(10, 3)
    s = orc.subsample(x, 4)
    assert np.array_equal(s[:, 0], [0.0, 12.0, 24.0])
