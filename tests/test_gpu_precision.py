"""Form (1): TSDF stored as scaled int16 or FP16 with uint8 weights, FP32 sums, FP64 pose math.

Parity: the low-precision kernels against the oracle on the same quantized values (the oracle's
FP64 volume quantized on the host), inside the near-face interval. Error against FP64: the
low-precision path (its own fusion) against the unquantized FP64 oracle, within 1e-3 relative on
the fitness, at the tiny scale and at 1024^3 / 0.5 cm on sampled poses."""
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


def quantize(T, fmt):
    if fmt == 2:
        return (np.clip(np.rint(T * 32767.0), -32767, 32767) / 32767.0)
    return T.astype(np.float16).astype(np.float64)


def poses_around(orc, R, t, n, rot, trans, seed):
    rng = np.random.default_rng(seed)
    return [(R, t)] + [orc.compose(rng.uniform(-rot, rot, 3), rng.uniform(-trans, trans, 3), R, t)
                       for _ in range(n - 1)]


@pytest.mark.parametrize("fmt", [1, 2])
def test_low_precision_kernel_parity_and_error(pf, orc, fmt):
    say(f"[precision] tiny scale, format {fmt}")
    dev = torch.device("cuda:0")
    d = synth.cfg1_inputs()
    v = orc.Volume(d["vol"])
    v.integrate(d["depth1"], d["intr"], np.eye(3), np.zeros(3))
    Tq = quantize(v.T, fmt)
    vq = orc.Volume(d["vol"], T=Tq, W=v.W)
    gv = pf.Tsdf(d["vol"], fmt=fmt, device=dev, init=False)
    gv.import_linear(Tq.astype(np.float32), v.W.astype(np.float32))
    X, _ = orc.backproject(d["depth2"], d["intr"], 2)
    X32 = X.astype(np.float32)
    poses = poses_around(orc, *d["init2"], 129, math.radians(5), 0.03, 7)
    P32 = pf.poses_to_f32(poses)
    p64 = [(P[:, :3].astype(np.float64), P[:, 3].astype(np.float64)) for P in P32.reshape(-1, 3, 4)]
    xt = torch.as_tensor(X32).to(dev)
    E, nv = pf.particles_score(gv, xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous(),
                               torch.as_tensor(P32).to(dev))
    E = E.cpu().numpy().astype(np.float64)
    lo, hi, _ = vq.fitness_interval_many(X32.astype(np.float64), p64, eps=1e-3)
    assert np.all(E >= lo - 1e-4 * lo - 1e-7) and np.all(E <= hi + 1e-4 * hi + 1e-7)
    # error of the low-precision form against FP64 (unquantized volume)
    E64, _ = v.fitness_many(X32.astype(np.float64), p64)
    rel = np.abs(E - E64) / E64
    say(f"    vs FP64: median {np.median(rel):.2e}, max {rel.max():.2e} relative")
    assert np.median(rel) <= 1e-3


@pytest.mark.parametrize("fmt", [2, 1])
def test_low_precision_fused_vs_fp64_at_scale(pf, orc, fmt):
    """1024^3 at 0.5 cm (tau 2 cm) on the paper-scale room: GPU fusion of frame 0 into int16 / FP16,
    then the fitness of 17 poses around frame 1 on the rate-1/8 view, against the FP64 oracle's
    own fusion and fitness."""
    say(f"[precision] 1024^3 / 0.5 cm, format {fmt}")
    dev = torch.device("cuda:0")
    f = synth.cfg2_frames(2)
    c = synth.room_centre_world(f["scene"])
    spec = synth.VolumeSpec.centred(1024, 0.005, 0.02, c)
    depth0, depth1 = f["depth"](0), f["depth"](1)
    ov = orc.Volume(spec)
    ov.integrate(depth0, f["intr"], np.eye(3), np.zeros(3))
    gv = pf.Tsdf(spec, fmt=fmt, device=dev)
    gv.integrate(torch.as_tensor(depth0).to(dev), f["intr"], np.eye(3), np.zeros(3))
    X, _ = orc.backproject(depth1, f["intr"], 1)
    S = orc.subsample(X, 8).astype(np.float32)
    Rg, tg = f["gt"][1]
    poses = poses_around(orc, Rg, tg, 17, math.radians(1.0), 0.01, 9)
    P32 = pf.poses_to_f32(poses)
    p64 = [(P[:, :3].astype(np.float64), P[:, 3].astype(np.float64)) for P in P32.reshape(-1, 3, 4)]
    xt = torch.as_tensor(S).to(dev)
    E, nv = pf.particles_score(gv, xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous(),
                               torch.as_tensor(P32).to(dev))
    E = E.cpu().numpy().astype(np.float64)
    E64, n64 = ov.fitness_many(S.astype(np.float64), p64)
    rel = np.abs(E - E64) / E64
    say(f"    vs FP64: median {np.median(rel):.2e}, max {rel.max():.2e}; valid {nv.cpu().numpy()[:3]} vs {n64[:3]}")
    assert np.median(rel) <= 1e-3
    del ov
