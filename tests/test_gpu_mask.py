"""The cell-validity mask of the CELLS layout: its words against the band cells of the stored volume,
and scoring through it against scoring without it and against the FP64 oracle.

Bars: the mask bit-exact against a host evaluation of the definition (a cell's bit is set iff all 8
of its corners are in the band) after init, fusion and import, with every flag byte back at 0;
fitness and valid counts bitwise identical with and without the mask in every launch; FP32 fitness
inside the oracle's near-face interval, as for the unmasked path."""
import math
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pf():
    import paper_2509_24236_amd as pf
    pf.lib()
    assert torch.cuda.is_available()
    return pf


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def cfg1():
    return synth.cfg1_inputs()


def host_mask(T, fmt):
    """Mask words of an exported (nz, ny, nx) volume, from the definition."""
    lim = 0.99999 if fmt == 2 else 1.0    # int16: the band ends at 32766 / 32767
    B = np.abs(T) < lim                   # NaN is not in the band
    V = (B[:-1, :-1, :-1] & B[:-1, :-1, 1:] & B[:-1, 1:, :-1] & B[:-1, 1:, 1:]
         & B[1:, :-1, :-1] & B[1:, :-1, 1:] & B[1:, 1:, :-1] & B[1:, 1:, 1:])
    cz, cy, cx = V.shape
    mz, my, mx = (cz + 3) // 4, (cy + 3) // 4, (cx + 3) // 4
    P = np.zeros((mz * 4, my * 4, mx * 4), bool)
    P[:cz, :cy, :cx] = V
    bits = P.reshape(mz, 4, my, 4, mx, 4).transpose(0, 2, 4, 1, 3, 5).reshape(mz, my, mx, 64)
    return np.packbits(bits, axis=-1, bitorder="little").view("<u8")[..., 0], int(V.sum())


def check_mask(vol, fmt, what):
    T, _ = vol.export_linear(with_weight=False)
    want, n_valid = host_mask(T.cpu().numpy(), fmt)
    words, flags = vol.cell_mask()
    got = words.cpu().numpy().view(np.uint64)
    bad = np.argwhere(got != want)
    assert bad.size == 0, f"{what}: {len(bad)} mask words differ, first at {bad[:3].tolist()}"
    assert int(flags.sum()) == 0, f"{what}: flag bytes left set"
    return n_valid


def _poses_around(orc, R, t, K, s_rad, s_m, seed):
    return [orc.compose(*orc.draw_delta(seed, 1, 1, k, s_rad, s_m), R, t) for k in range(K)]


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_mask_follows_init_and_fusion(pf, dev, cfg1, fmt):
    say(f"[mask] init + 3 fusions, format {fmt}")
    vol = pf.Tsdf(cfg1["vol"], fmt=fmt, device=dev, layout=pf.LAYOUT_CELLS)
    assert check_mask(vol, fmt, "after init") == 0
    frames = [(cfg1["depth1"], cfg1["gt1"]), (cfg1["depth2"], cfg1["gt2"]), (cfg1["depth1"], cfg1["gt1"])]
    counts = []
    for f, (depth, (R, t)) in enumerate(frames):
        vol.integrate(torch.as_tensor(depth).to(dev), cfg1["intr"], R, t)
        counts.append(check_mask(vol, fmt, f"after fusion {f}"))
    assert counts[0] > 1000 and counts[1] != counts[0]
    # a re-init clears every word
    vol.init()
    assert check_mask(vol, fmt, "after re-init") == 0


@pytest.mark.parametrize("fmt", [0, 2])
def test_mask_follows_fusion_ragged_grid(pf, dev, cfg1, fmt):
    """Fusion into a grid whose dimensions are not multiples of 4 (partial words at the far faces,
    voxels on word boundaries flagging up to 8 words)."""
    say(f"[mask] fusion into a 101 x 67 x 93 grid, format {fmt}")
    s0 = cfg1["vol"]
    centre = np.array(s0.origin) + 0.5 * (np.array([s0.nx, s0.ny, s0.nz]) - 1) * s0.voxel_size
    n = np.array([101, 67, 93])
    spec = synth.VolumeSpec(101, 67, 93, 0.025, 0.1, tuple(centre - 0.5 * (n - 1) * 0.025 + 0.0031))
    vol = pf.Tsdf(spec, fmt=fmt, device=dev, layout=pf.LAYOUT_CELLS)
    counts = []
    for depth, (R, t) in [(cfg1["depth1"], cfg1["gt1"]), (cfg1["depth2"], cfg1["gt2"])]:
        vol.integrate(torch.as_tensor(depth).to(dev), cfg1["intr"], R, t)
        counts.append(check_mask(vol, fmt, "after fusion"))
    assert counts[0] > 1000 and counts[1] != counts[0]


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_mask_after_import_ragged(pf, dev, fmt):
    """Dimensions that are not multiples of 4 (partial words at the far faces) and values on both
    sides of the band edge."""
    say(f"[mask] import into a 23 x 14 x 9 grid, format {fmt}")
    spec = synth.VolumeSpec(23, 14, 9, 0.05, 0.2, (0.0, 0.0, 0.0))
    rng = np.random.default_rng(31 + fmt)
    T = rng.uniform(-0.9, 0.9, (9, 14, 23)).astype(np.float32)
    out = rng.random(T.shape) < 0.03
    T[out] = rng.choice(np.array([1.0, -1.0, 1.5, -3.0, np.nan], np.float32), int(out.sum()))
    T[0, 0, :] = 0.999     # in the band in every format after rounding
    vol = pf.Tsdf(spec, fmt=fmt, device=dev, layout=pf.LAYOUT_CELLS, init=False)
    vol.import_linear(T, np.ones(T.shape, np.float32))
    n = check_mask(vol, fmt, "after import")
    assert 0 < n < 22 * 13 * 8


@pytest.mark.parametrize("spread_deg", [5.0, 0.01])
@pytest.mark.parametrize("K", [5, 65, 257])
def test_masked_scoring_bitwise_and_parity(pf, orc, dev, cfg1, K, spread_deg):
    say(f"[mask] scoring with and without the mask, K={K}, spread {spread_deg} deg")
    v = orc.Volume(cfg1["vol"])
    v.integrate(cfg1["depth1"], cfg1["intr"], np.eye(3), np.zeros(3))
    T32 = v.T.astype(np.float32)
    v32 = orc.Volume(cfg1["vol"], T=T32.astype(np.float64), W=v.W)
    gv = pf.Tsdf(cfg1["vol"], device=dev, init=False, layout=pf.LAYOUT_CELLS)
    gv.import_linear(T32, v.W.astype(np.float32))
    X, _ = orc.backproject(cfg1["depth2"], cfg1["intr"], 2)
    x32 = X.astype(np.float32)
    xt = torch.as_tensor(x32).to(dev)
    pts = (xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous())
    poses = _poses_around(orc, *cfg1["gt2"], K, math.radians(spread_deg), spread_deg * 0.006, 91)
    P32 = pf.poses_to_f32(poses)
    P = torch.as_tensor(P32).to(dev)
    try:
        res = {}
        for mode in (pf.MASK_NEVER, pf.MASK_ALWAYS, pf.MASK_BY_SPREAD):
            pf.score_mask(mode)
            E, nv = pf.particles_score(gv, *pts, P)
            res[mode] = (E.cpu().numpy().view(np.uint32), nv.cpu().numpy())
    finally:
        pf.score_mask(pf.MASK_BY_SPREAD)
    for mode in (pf.MASK_ALWAYS, pf.MASK_BY_SPREAD):
        assert np.array_equal(res[mode][0], res[pf.MASK_NEVER][0]), mode
        assert np.array_equal(res[mode][1], res[pf.MASK_NEVER][1]), mode
    poses64 = [(P32[k].reshape(3, 4)[:, :3].astype(np.float64), P32[k].reshape(3, 4)[:, 3].astype(np.float64))
               for k in range(K)]
    lo, hi, _ = v32.fitness_interval_many(x32.astype(np.float64), poses64, eps=1e-3)
    E = res[pf.MASK_ALWAYS][0].view(np.float32).astype(np.float64)
    lo_w, hi_w = lo - 1e-4 * np.abs(lo) - 1e-7, hi + 1e-4 * np.abs(hi) + 1e-7
    assert np.all((E >= lo_w) & (E <= hi_w))
    assert np.all(res[pf.MASK_ALWAYS][1] > 0)


def test_masked_configured_shapes_bitwise(pf, orc, dev, cfg1):
    """PF_MASK_ALWAYS with configured shapes: those whose queues fit in LDS compact the valid
    samples, the larger ones (8x256, 4x512, 8x512) take the per-lane masked path; all equal the
    unmasked result bit for bit, over a ragged point count."""
    say("[mask] configured shapes through the mask")
    gv = pf.Tsdf(cfg1["vol"], device=dev, layout=pf.LAYOUT_CELLS)
    gv.integrate(torch.as_tensor(cfg1["depth1"]).to(dev), cfg1["intr"], np.eye(3), np.zeros(3))
    X, _ = orc.backproject(cfg1["depth2"], cfg1["intr"], 2)
    X = X[:4093]
    xt = torch.as_tensor(X.astype(np.float32)).to(dev)
    pts = (xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous())
    poses = _poses_around(orc, *cfg1["gt2"], 203, math.radians(3.0), 0.02, 17)
    P = torch.as_tensor(pf.poses_to_f32(poses)).to(dev)
    try:
        pf.score_mask(pf.MASK_NEVER)
        E0, n0 = pf.particles_score(gv, *pts, P)
        ref = (E0.cpu().numpy().view(np.uint32), n0.cpu().numpy())
        pf.score_mask(pf.MASK_ALWAYS)
        for tk, blk in [(2, 64), (4, 128), (2, 512), (8, 256), (4, 512), (8, 512)]:
            pf.score_config(tk, blk)
            E, nv = pf.particles_score(gv, *pts, P)
            assert np.array_equal(E.cpu().numpy().view(np.uint32), ref[0]), (tk, blk)
            assert np.array_equal(nv.cpu().numpy(), ref[1]), (tk, blk)
    finally:
        pf.score_config(0, 0)
        pf.score_mask(pf.MASK_BY_SPREAD)
    assert int((ref[1] > 0).sum()) > 150


def test_track_frame_mask_modes_bitwise(pf, orc, dev, cfg1):
    say("[mask] track_frame in the three mask modes")
    gv = pf.Tsdf(cfg1["vol"], device=dev, layout=pf.LAYOUT_CELLS)
    gv.integrate(torch.as_tensor(cfg1["depth1"]).to(dev), cfg1["intr"], np.eye(3), np.zeros(3))
    prm = pf.TrackParams(seed=5, frame_index=1, n_iters=12, K=512, rates=(1, 2), pixel_stride=2, s1_deg=10.0,
                         s1_m=0.1)
    depth = torch.as_tensor(cfg1["depth2"]).to(dev)
    out = {}
    try:
        for mode in (pf.MASK_BY_SPREAD, pf.MASK_NEVER, pf.MASK_ALWAYS):
            pf.score_mask(mode)
            R, t, st = pf.Tracker(cfg1["intr"], prm, device=dev).track(gv, depth, *cfg1["init2"])
            out[mode] = (R, t, list(st.n_adv[:12]), list(st.Estar[:12]))
    finally:
        pf.score_mask(pf.MASK_BY_SPREAD)
    ref = out[pf.MASK_NEVER]
    for mode in (pf.MASK_BY_SPREAD, pf.MASK_ALWAYS):
        R, t, n_adv, Estar = out[mode]
        assert np.array_equal(R, ref[0]) and np.array_equal(t, ref[1]), mode
        assert n_adv == ref[2] and Estar == ref[3], mode


def test_score_mask_rejects_unknown_mode(pf):
    with pytest.raises(pf.PFError):
        pf.score_mask(3)
    pf.score_mask(pf.MASK_BY_SPREAD)


def test_fullsize_mask_follows_fusion(pf, dev):
    """The 512^3 volume of the headline sequence after fusing three of its frames."""
    say("[mask] 512^3 after three fusions")
    f = synth.cfg2_frames(3)
    vol = pf.Tsdf(f["vol"], device=dev, layout=pf.LAYOUT_CELLS)
    R0, t0 = f["gt"][0]
    for k in range(3):
        Rk, tk = f["gt"][k]
        R, t = R0.T @ Rk, R0.T @ (tk - t0)
        vol.integrate(torch.as_tensor(f["depth"](k)).to(dev), f["intr"], R, t)
    n = check_mask(vol, 0, "512^3 after three fusions")
    assert n > 100000
