"""Form (3): the hand-written adjoint (particles_score_grad), its torch.autograd wrapper and the
gradient polish inside track_frame, against the FP64 oracle on the differentiation workload
(the tiny room, 1000 seeded poses in the +-5 deg / +-3 cm box around the true pose, seed 30)."""
import math
import sys

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


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def setup(orc, pf, dev):
    d = synth.cfg1_inputs()
    v = orc.Volume(d["vol"])
    v.integrate(d["depth1"], d["intr"], np.eye(3), np.zeros(3))
    T32 = v.T.astype(np.float32)
    v32 = orc.Volume(d["vol"], T=T32.astype(np.float64), W=v.W)
    gv = pf.Tsdf(d["vol"], device=dev, init=False)
    gv.import_linear(T32, v.W.astype(np.float32))
    X, _ = orc.backproject(d["depth2"], d["intr"], 2)
    X32 = X.astype(np.float32)
    xt = torch.as_tensor(X32).to(dev)
    pts = (xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous())
    return d, v32, gv, X32, pts


def cfg3_poses(orc, d, n, seed=30):
    rng = np.random.default_rng(seed)
    R, t = d["gt2"]
    return [orc.compose(rng.uniform(-1, 1, 3) * math.radians(5), rng.uniform(-1, 1, 3) * 0.03, R, t) for _ in range(n)]


def rows(poses):
    return np.stack([np.concatenate([R, t.reshape(3, 1)], 1).reshape(12) for R, t in poses])


@pytest.mark.parametrize("mode", [0, 1])
def test_adjoint_parity_1000_poses(pf, orc, dev, setup, mode):
    say(f"[grad] 1000 poses, mode {mode}")
    d, v32, gv, X32, pts = setup
    poses = cfg3_poses(orc, d, 1000)
    base = torch.as_tensor(rows(poses)).to(dev)
    E, g, nv = pf.particles_score_grad(gv, *pts, base, None, mode)
    # the GPU rounds each pose to FP32 before sampling; give the oracle the same pose
    P32 = pf.poses_to_f32(poses).astype(np.float64).reshape(-1, 3, 4)
    # a value near 0 may take the other sign in FP32: the sample position carries ~1e-5 voxel of
    # rounding (grid coordinates up to 128), and the field changes by vs / tau = 0.25 per voxel,
    # so |T| < 1e-5 is not sign-stable; the band is 1e-4
    lo, hi = v32.fitness_grad_interval_many(X32.astype(np.float64), [(P[:, :3], P[:, 3]) for P in P32], mode,
                                            eps=1e-3, sign_eps=1e-4)
    got = np.concatenate([E.cpu().numpy()[:, None], g.cpu().numpy()], 1).astype(np.float64)
    scale = np.maximum(np.abs(lo), np.abs(hi))
    tol = np.concatenate([1e-4 * scale[:, :1], 2e-4 * scale[:, 1:].max(1, keepdims=True).repeat(6, 1)], 1) + 1e-6
    bad = (got < lo - tol) | (got > hi + tol)
    if bad.any():
        b = np.flatnonzero(bad.any(1))[:5]
        say(f"    outside: poses {b}\n    got {got[b]}\n    lo {lo[b]}\n    hi {hi[b]}")
    assert not bad.any(), f"{bad.any(1).sum()} poses outside the oracle interval; first {np.flatnonzero(bad.any(1))[:5]}"
    assert (nv.cpu().numpy() > 100).all()
    # the adjoint's E and valid count are the scoring kernel's, bit for bit (same sample steps,
    # exact fixed-point sum)
    Es, nvs = pf.particles_score(gv, *pts, torch.as_tensor(pf.poses_to_f32(poses)).to(dev))
    assert np.array_equal(E.cpu().numpy().view(np.uint32), Es.cpu().numpy().view(np.uint32))
    assert np.array_equal(nv.cpu().numpy(), nvs.cpu().numpy())


@pytest.mark.parametrize("mode", [0, 1])
def test_adjoint_chain_vs_central_differences(pf, orc, dev, setup, mode):
    """dE/dxi at xi != 0 vs central differences (h = 1e-4) of the oracle's frozen objective."""
    say(f"[grad] chain rule vs central differences, 1000 poses, mode {mode}")
    d, v32, gv, X32, pts = setup
    B = 1000
    rng = np.random.default_rng(31)
    poses = cfg3_poses(orc, d, B, seed=32)
    xi = np.concatenate([rng.uniform(-0.02, 0.02, (B, 3)), rng.uniform(-0.06, 0.06, (B, 3))], 1)
    base = torch.as_tensor(rows(poses)).to(dev)
    E, g, nv = pf.particles_score_grad(gv, *pts, base, torch.as_tensor(xi).to(dev), mode)
    g = g.cpu().numpy().astype(np.float64)
    X64 = X32.astype(np.float64)
    # Bound per pose and component. The frozen set (cells and signs) can differ between the GPU's
    # FP32 pose and the oracle's FP64 one only for samples within rounding of a cell face or of a
    # zero of T; the oracle's interval [lo, hi] at the FP32 pose takes every such choice for the
    # gradient with respect to a delta applied there, and the gradient with respect to xi is that
    # one through J(phi)^T (and, LITERAL, a rho x term): with |phi| <= 0.11 and |rho| <= 0.035 m its
    # rows sum to less than 1.25, so |gpu - fd| <= 1.25 max(hi - lo) + arithmetic. The
    # arithmetic is a fixed-order FP32 sum of ~4800 terms, ~(log2 4800 + 2) 2^-24 = 9e-7 of the
    # terms' magnitudes, times the cancellation of the sum (below 20 here), plus O(h^2) = 1e-8 of
    # the central differences: 2e-5 of the gradient's largest component.
    comp = [orc.compose(xi[b, 3:], xi[b, :3], R, t, mode) for b, (R, t) in enumerate(poses)]
    P32 = pf.poses_to_f32(comp).astype(np.float64).reshape(-1, 3, 4)
    lo, hi = v32.fitness_grad_interval_many(X64, [(P[:, :3], P[:, 3]) for P in P32], mode, eps=1e-3, sign_eps=1e-4)
    width = np.repeat((hi - lo)[:, 1:].max(1, keepdims=True), 6, 1)
    dev_abs = np.zeros((B, 6))
    scale = np.zeros(B)
    for b, (R, t) in enumerate(poses):
        ref = v32.grad_xi_fd(X64, R, t, xi[b], mode, h=1e-4)
        dev_abs[b] = np.abs(g[b] - ref)
        scale[b] = np.abs(ref).max()
    err = dev_abs.max(1) / scale
    bound = 1.25 * width + 2e-5 * scale[:, None]
    q = np.percentile(err, [50, 90, 99, 100])
    say(f"    relative deviation: median {q[0]:.2e}, 90% {q[1]:.2e}, 99% {q[2]:.2e}, max {q[3]:.2e}; largest "
        f"deviation over its bound {np.max(dev_abs / bound):.2f}; interval width / gradient median "
        f"{np.median(width.max(1) / scale):.2e}")
    bad = np.flatnonzero((dev_abs > bound).any(1))
    assert bad.size == 0, f"{bad.size} poses beyond the bound, e.g. {bad[:5]}"


def test_autograd_function(pf, orc, dev, setup):
    say("[grad] autograd.Function")
    d, v32, gv, X32, pts = setup
    poses = cfg3_poses(orc, d, 8, seed=33)
    base = torch.as_tensor(rows(poses)).to(dev)
    xi = torch.zeros((8, 6), dtype=torch.float64, device=dev, requires_grad=True)
    E = pf.fitness(xi, base, gv, *pts)
    w = torch.linspace(0.5, 2.0, 8, dtype=torch.float64, device=dev)
    (E * w).sum().backward()
    E2, g2, _ = pf.particles_score_grad(gv, *pts, base, None, 0)
    assert torch.equal(E, E2.double())
    assert torch.allclose(xi.grad, w[:, None] * g2.double(), rtol=0, atol=0)


def test_unfrozen_finite_difference_agreement(pf, orc, dev, setup):
    """Report only: central differences (h = 1e-4) of the FP32, unfrozen fitness jump where samples
    enter or leave the valid set, so agreement with the adjoint is a fraction, not a bound."""
    d, v32, gv, X32, pts = setup
    poses = cfg3_poses(orc, d, 64, seed=34)
    base = torch.as_tensor(rows(poses)).to(dev)
    E, g, _ = pf.particles_score_grad(gv, *pts, base, None, 0)
    h = 1e-4
    fd = np.zeros((64, 6))
    for a in range(6):
        e = torch.zeros((64, 6), dtype=torch.float64, device=dev)
        e[:, a] = h
        Ep, _, _ = pf.particles_score_grad(gv, *pts, base, e, 0)
        Em, _, _ = pf.particles_score_grad(gv, *pts, base, -e, 0)
        fd[:, a] = (Ep.double() - Em.double()).cpu().numpy() / (2 * h)
    g = g.cpu().numpy()
    rel = np.abs(fd - g) / (np.abs(g).max(1, keepdims=True) + 1e-12)
    frac = float((rel < 0.1).mean())
    say(f"    unfrozen FD within 10% of the adjoint for {100 * frac:.1f}% of components")
    assert frac > 0.3


@pytest.mark.parametrize("mode", [0, 1])
def test_polish_parity(pf, orc, dev, setup, mode):
    say(f"[polish] track_frame with 5 polish steps, mode {mode}")
    d, v32, gv, X32, pts = setup
    R0, t0 = d["init2"]
    prm = pf.TrackParams(seed=3, frame_index=1, n_iters=10, K=256, rates=(1,), pixel_stride=2, s1_deg=5.0,
                         s1_m=0.03, compose_mode=mode, polish_steps=5)
    trk = pf.Tracker(d["intr"], prm, device=dev)
    R, t, st = trk.track(gv, torch.as_tensor(d["depth2"]).to(dev), R0, t0)
    oprm = orc.make_params(seed=3, frame_index=1, n_iters=10, K=256, rates=(1,), pixel_stride=2, s1_deg=5.0,
                           s1_m=0.03, compose_mode=mode, polish_steps=5)
    Ro, to, recs = v32.track_frame(d["depth2"], d["intr"], R0, t0, oprm)
    dr, dt = math.degrees(orc.rot_err(R, Ro)), float(np.linalg.norm(t - to))
    say(f"    pose vs oracle {dr:.2e} deg {dt * 1e3:.3e} mm; accepted {st.polish_accepted}; E_final {st.E_final:.5f}")
    assert dr <= 0.05 and dt <= 1e-3
    # the polish lowered the fitness on the densest view relative to the unpolished pose
    prm0 = pf.TrackParams(seed=3, frame_index=1, n_iters=10, K=256, rates=(1,), pixel_stride=2, s1_deg=5.0,
                          s1_m=0.03, compose_mode=mode, polish_steps=0)
    _, _, st0 = pf.Tracker(d["intr"], prm0, device=dev).track(gv, torch.as_tensor(d["depth2"]).to(dev), R0, t0)
    assert st.E_final <= st0.E_final
