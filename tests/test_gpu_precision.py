"""Form (1): TSDF stored as scaled int16 or FP16 with uint8 weights, FP32 sums, FP64 pose math.

Parity: the low-precision kernels against the oracle on the same quantized values (the oracle's
FP64 volume quantized on the host), inside the near-face interval. Error against FP64, per pose:
the low-precision path (on its own fusion) lies inside the oracle's storage-rounding interval of
the unquantized FP64 volume (every stored value within half a step of int16, half an ulp of FP16,
plus the FP32 fusion arithmetic), and within 1e-3 relative of the FP64 fitness wherever the
rounding moved no sample across the band edge (same valid count); the largest error is printed.
At 1024^3 / 0.5 cm the paper-scale frame 1 also runs in lockstep with the oracle for 20 iterations
in each storage format (FP32, FP16, int16): every particle's fitness in the oracle's interval, the
advantage set equal except where a particle and the current pose are tied within that interval
(counted and printed), and each update equal to the oracle's on identical fitness."""
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


# storage rounding of each format: (qrel, qabs), a stored value within qrel |T| + qabs of T
ROUNDING = {0: (0.0, 0.0), 1: (2.0 ** -11, 2.0 ** -25), 2: (0.0, 0.5 / 32767.0)}


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
    # error of the low-precision form against FP64 (unquantized volume), per pose
    check_against_fp64(v, X32, p64, E, nv.cpu().numpy(), fmt, fusion_abs=0.0)


def check_against_fp64(v64, X32, p64, E, nv, fmt, fusion_abs):
    """Per pose: E inside the storage-rounding interval of the FP64 volume v64 (widened by 1e-4
    relative for the FP32 sums), and within 1e-3 relative of the FP64 fitness where the valid count
    is the FP64 one."""
    qrel, qabs = ROUNDING[fmt]
    x64 = X32.astype(np.float64)
    lo, hi = v64.fitness_interval_rounded_many(x64, p64, eps=1e-3, qrel=qrel, qabs=qabs + fusion_abs)
    bad = np.flatnonzero((E < lo - 1e-4 * lo - 1e-7) | (E > hi + 1e-4 * hi + 1e-7))
    assert bad.size == 0, f"{bad.size} poses outside the rounding interval, e.g. {bad[:4]}: {E[bad[:4]]} " \
                          f"[{lo[bad[:4]]}, {hi[bad[:4]]}]"
    E64, n64 = v64.fitness_many(x64, p64)
    rel = np.abs(E - E64) / E64
    same = nv == n64
    say(f"    vs FP64: max {rel.max():.2e}, median {np.median(rel):.2e} relative; valid count equal for "
        f"{same.sum()}/{len(E)} poses (max {rel[same].max() if same.any() else 0:.2e} there), the others "
        f"inside the rounding interval (max {rel[~same].max() if (~same).any() else 0:.2e})")
    assert np.all(rel[same] <= 1e-3)


@pytest.mark.parametrize("fmt", [2, 1])
def test_low_precision_fused_vs_fp64_at_scale(pf, orc, fmt):
    """1024^3 at 0.5 cm (tau 2 cm) on the paper-scale room: GPU fusion of frame 0 into int16 / FP16,
    then the fitness of 129 poses around frame 1 on the rate-1/8 view, against the FP64 oracle's
    own fusion and fitness, per pose."""
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
    poses = poses_around(orc, Rg, tg, 129, math.radians(1.0), 0.01, 9)
    P32 = pf.poses_to_f32(poses)
    p64 = [(P[:, :3].astype(np.float64), P[:, 3].astype(np.float64)) for P in P32.reshape(-1, 3, 4)]
    xt = torch.as_tensor(S).to(dev)
    E, nv = pf.particles_score(gv, xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous(),
                               torch.as_tensor(P32).to(dev))
    E = E.cpu().numpy().astype(np.float64)
    # the GPU fuses in FP32 (values within 1e-6 of the FP64 fusion), then stores in the format
    check_against_fp64(ov, S, p64, E, nv.cpu().numpy(), fmt, fusion_abs=1e-6)
    del ov


@pytest.fixture(scope="module")
def cfg5_frames():
    f = synth.cfg2_frames(2)
    spec = synth.VolumeSpec.centred(1024, 0.005, 0.02, synth.room_centre_world(f["scene"]))
    return f, spec


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_lockstep_frame1_at_1024(pf, orc, cfg5_frames, fmt):
    """Frame 1 of the paper-scale sequence at 1024^3 / 0.5 cm (tau 2 cm), 4096 particles x 20
    iterations at rates 8/16/32, each iteration checked against the oracle on the same inputs: the
    volume the GPU fused from frame 0 (dequantized), the same FP32 points and the GPU's own poses."""
    import time
    f, spec = cfg5_frames
    say(f"[lockstep] 1024^3, format {fmt}: fuse frame 0, then 20 iterations of frame 1 against the oracle")
    dev = torch.device("cuda:0")
    t_start = time.time()
    gv = pf.Tsdf(spec, fmt=fmt, device=dev)
    gv.integrate(torch.as_tensor(f["depth"](0)).to(dev), f["intr"], np.eye(3), np.zeros(3))
    T, W = gv.export_linear()
    oq = orc.Volume(spec, T=T.cpu().numpy(), W=W.cpu().numpy())
    del T, W
    X, _ = orc.backproject(f["depth"](1), f["intr"], 1)
    views = {}
    for r in (8, 16, 32):
        S = orc.subsample(X, r).astype(np.float32)
        st_ = torch.as_tensor(S).to(dev)
        views[r] = (S.astype(np.float64), st_[:, 0].contiguous(), st_[:, 1].contiguous(), st_[:, 2].contiguous())
    K = 4096
    prm = pf.TrackParams(seed=15, frame_index=1, n_iters=20, K=K, rates=(8, 16, 32), pixel_stride=1, s1_deg=10.0,
                         s1_m=0.10)
    Rr, tr = f["rel"][1]
    state = torch.zeros(pf.state_bytes(K), dtype=torch.uint8, device=dev)
    poses = torch.zeros((K + 1, 12), dtype=torch.float32, device=dev)
    pf.particles_state_init(state, Rr, tr, prm, poses)
    near_total, differ_total, amb_total = 0, 0, 0
    for i in range(1, 21):
        r = (8, 16, 32)[(i - 1) % 3]
        S64, px, py, pz = views[r]
        E, nv = pf.particles_score(gv, px, py, pz, poses)
        E = E.cpu().numpy().astype(np.float64)
        P32 = poses.cpu().numpy()
        p64 = [(P[:, :3].astype(np.float64), P[:, 3].astype(np.float64)) for P in P32.reshape(-1, 3, 4)]
        lo, hi, namb = oq.fitness_interval_many(S64, p64, eps=1e-3)
        lo_w, hi_w = lo - 1e-4 * lo - 1e-7, hi + 1e-4 * hi + 1e-7
        bad = np.flatnonzero((E < lo_w) | (E > hi_w))
        assert bad.size == 0, f"iteration {i}: {bad.size} particles outside the oracle interval, e.g. {bad[:5]}"
        # advantage membership against the FP64 values; a difference must be a near-tie: the
        # particle's interval and the current pose's overlap
        E64, _ = oq.fitness_many(S64, p64)
        a_gpu, a_64 = E[1:] < E[0], E64[1:] < E64[0]
        near = (lo_w[1:] <= hi_w[0]) & (hi_w[1:] >= lo_w[0])
        differ = np.flatnonzero(a_gpu != a_64)
        assert np.all(near[differ]), f"iteration {i}: membership differs at non-tied particles {differ[~near[differ]][:5] + 1}"
        near_total += int(near.sum())
        differ_total += differ.size
        amb_total += int(namb.sum())
        # the update on identical fitness: the oracle's advantage step with the GPU's fitness and deltas
        before = pf.read_state(state)
        D = pf.read_deltas(state, K)
        Rp, tp = np.array(before.R[:]).reshape(3, 3), np.array(before.t[:])
        pf.particles_update(gv, px, py, pz, torch.as_tensor(E.astype(np.float32)).to(dev), nv, state, K, poses)
        st = pf.read_state(state)
        na, Ro, to, mean = orc.advantage_update(E.astype(np.float32).astype(np.float64), D, Rp, tp)
        assert st.n_adv == na
        Rg, tg = np.array(st.R_new[:]).reshape(3, 3), np.array(st.t_new[:])
        assert np.abs(Rg - Ro).max() <= 1e-13 and np.abs(tg - to).max() <= 1e-13
        if i in (1, 2, 3, 10, 20):
            say(f"    iteration {i} (rate 1/{r}): |A| {na}, near-ties {int(near.sum())}, membership differs at "
                f"{differ.size} (all tied), samples near a face {int(namb.sum())}")
    say(f"    20 iterations: {near_total} particle/pose near-ties, {differ_total} membership differences (all "
        f"near-ties), {amb_total} near-face samples; {time.time() - t_start:.0f} s")
    del oq, gv
    torch.cuda.empty_cache()
