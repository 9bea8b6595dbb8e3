"""Pins of the oracle's storage-rounding fitness interval (the per-pose bound used for the
int16 / FP16 forms), against things other than itself: with no rounding it is the near-face
interval; brute force over randomly rounded copies of a fused volume (every value moved within
its bound, and values at the band edge pushed out of the band at random) never leaves it; and the
actual int16 and FP16 roundings of the volume land inside it."""
import math

import numpy as np
import pytest

import synth

I16_Q = (0.0, 0.5 / 32767.0)          # (qrel, qabs): half a step of 1/32767
F16_Q = (2.0 ** -11, 2.0 ** -25)      # half an ulp of FP16 is at most 2^-11 |x| (subnormals: 2^-25)


@pytest.fixture(scope="module")
def setup(orc):
    d = synth.cfg1_inputs()
    v = orc.Volume(d["vol"])
    v.integrate(d["depth1"], d["intr"], np.eye(3), np.zeros(3))
    X, _ = orc.backproject(d["depth2"], d["intr"], 2)
    rng = np.random.default_rng(11)
    R0, t0 = d["init2"]
    poses = [(R0, t0)] + [orc.compose(rng.uniform(-1, 1, 3) * math.radians(3.0), rng.uniform(-1, 1, 3) * 0.02, R0, t0)
                          for _ in range(7)]
    return d, v, X, poses


def test_no_rounding_is_the_near_face_interval(orc, setup):
    d, v, X, poses = setup
    for eps in (0.0, 1e-3):
        lo, hi, _ = v.fitness_interval_many(X, poses, eps=eps)
        lo2, hi2 = v.fitness_interval_rounded_many(X, poses, eps=eps)
        assert np.array_equal(lo, lo2) and np.array_equal(hi, hi2)


@pytest.mark.parametrize("q", [I16_Q, F16_Q, (1e-3, 1e-4)])
def test_randomly_rounded_volumes_stay_inside(orc, setup, q):
    d, v, X, poses = setup
    qrel, qabs = q
    rng = np.random.default_rng(3)
    # one fusion leaves few values within a rounding of the band edge: move 3% of the band there
    T = v.T.copy()
    band = np.abs(T) < 1.0
    pick = band & (rng.random(T.shape) < 0.03)
    dpk = qrel + qabs
    T[pick] = np.sign(T[pick] + 1e-300) * (1.0 - rng.uniform(0.0, 1.0, int(pick.sum())) * dpk)
    v = orc.Volume(d["vol"], T=T, W=v.W)
    lo, hi = v.fitness_interval_rounded_many(X, poses, eps=0.0, qrel=qrel, qabs=qabs)
    dd = qrel * np.abs(T) + qabs
    edge = band & (np.abs(T) >= 1.0 - dd)
    assert edge.sum() > 200
    for rep in range(6):
        Tp = T.copy()
        Tp[band] += rng.uniform(-1.0, 1.0, int(band.sum())) * dd[band]
        Tp[edge] = np.where(rng.random(int(edge.sum())) < 0.5, np.sign(T[edge]), np.clip(T[edge], -1 + 1e-12, 1 - 1e-12))
        # the extreme choices: every value at the end of its range that raises (or lowers) |T|
        if rep == 4:
            Tp[band] = T[band] + np.sign(T[band]) * dd[band]
            Tp[edge] = np.sign(T[edge])
        if rep == 5:
            Tp[band] = T[band] - np.sign(T[band]) * dd[band]
        Tp[band & ~edge] = np.clip(Tp[band & ~edge], -1 + 1e-15, 1 - 1e-15)
        vp = orc.Volume(d["vol"], T=Tp, W=v.W)
        E, _ = vp.fitness_many(X, poses)
        assert np.all(E >= lo) and np.all(E <= hi), (rep, E, lo, hi)


def test_actual_roundings_stay_inside(orc, setup):
    d, v, X, poses = setup
    T = v.T
    q16 = np.clip(np.rint(T * 32767.0), -32767, 32767) / 32767.0
    h16 = T.astype(np.float16).astype(np.float64)
    for Tq, (qrel, qabs) in ((q16, I16_Q), (h16, F16_Q)):
        lo, hi = v.fitness_interval_rounded_many(X, poses, eps=0.0, qrel=qrel, qabs=qabs)
        E, _ = orc.Volume(d["vol"], T=Tq, W=v.W).fitness_many(X, poses)
        assert np.all(E >= lo) and np.all(E <= hi)
        E64, _ = v.fitness_many(X, poses)
        # the bound is informative: int16 within 3e-4 relative, FP16 within 1e-2
        width = (hi - lo) / E64
        assert width.max() < (3e-4 if qrel == 0 else 1e-2), width


def test_value_rounding_alone_is_bounded(orc, setup):
    """A freshly fused volume has no int16 value within half a step of the band edge, so only the
    values move: raising (lowering) every |T| by the full bound stays inside, and the interval is
    then no wider than twice the bound on either side."""
    d, v, X, poses = setup
    qrel, qabs = I16_Q
    T = v.T
    band = np.abs(T) < 1.0
    assert not np.any(band & (np.abs(T) >= 1.0 - qabs))
    lo, hi = v.fitness_interval_rounded_many(X, poses, eps=0.0, qrel=qrel, qabs=qabs)
    E64, _ = v.fitness_many(X, poses)
    assert np.all(hi - E64 <= qabs * (1 + 1e-9)) and np.all(E64 - lo <= qabs * (1 + 1e-9))
    for sgn in (1.0, -1.0):
        Tp = T.copy()
        Tp[band] = T[band] + sgn * np.sign(T[band]) * qabs
        E, _ = orc.Volume(d["vol"], T=Tp, W=v.W).fitness_many(X, poses)
        assert np.all(E >= lo) and np.all(E <= hi)
        assert np.all(sgn * (E - E64) > 0.5 * qabs)      # the perturbation really moves the fitness
