"""The sparse brick pool (PF_LAYOUT_BRICKS) against the oracle's bricked fusion, and the brick
gather against the dense cell replica holding the same values.

Bars: the set of bricks with a slot and every weight bit-exact; T within the rounding of the
storage format of the FP64 value (the dense fusion's bars); every cell block of every slot equal
to the 8 stored corners it stands for; scoring, gradients and whole tracked frames bitwise equal
to the dense CELLS layout loaded with the exported values."""
import ctypes
import math
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

E = 8
T_TOL = {0: 2e-6, 1: 1.5e-3, 2: 1e-4}


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


def frames_cfg1(cfg1):
    """Frames 1 and 2 of the small room, then a third view turned 25 degrees away, so that the
    last fusion gives slots to new bricks beside bricks that already hold values."""
    R3 = synth.rot(math.radians(25.0) * np.array([0.0, 1.0, 0.0]))
    t3 = np.array([0.1, 0.0, -0.05])
    d3 = synth.render_depth(cfg1["scene"], cfg1["intr"], R3, t3)
    return [(cfg1["depth1"], *cfg1["gt1"]), (cfg1["depth2"], *cfg1["gt2"]), (d3, R3, t3)]


def raw_pool(pf, vol):
    """Host copies of the index grid, slot coordinates, slots' T and cells (storage dtype)."""
    s = vol.spec
    index_off, coords_off, t_off, c_off = vol.brick_offsets()
    n_used, overflow = vol.bricks_used()
    raw = vol.T.view(torch.uint8)
    nb = (s.nz // E) * (s.ny // E) * (s.nx // E)
    index = raw[index_off:index_off + 4 * nb].view(torch.int32).cpu().numpy().reshape(s.nz // E, s.ny // E, s.nx // E)
    coords = raw[coords_off:coords_off + 16 * n_used].view(torch.int32).cpu().numpy().reshape(n_used, 4)
    el = vol.T.element_size()
    Tp = raw[t_off:t_off + el * 512 * n_used].view(vol.T.dtype).cpu().numpy().reshape(n_used, 512)
    Cp = raw[c_off:c_off + el * 4096 * n_used].view(vol.T.dtype).cpu().numpy().reshape(n_used, 512, 8)
    return index, coords, Tp, Cp, n_used, overflow


def check_pool_consistent(pf, vol):
    """Index and coordinates agree, and every cell block holds the stored values of its corners
    (+1 for corners in bricks without a slot or outside the grid), with corners outside the band
    (|T| >= 1) marked NaN in the FP32 and FP16 formats."""
    s = vol.spec
    index, coords, Tp, Cp, n, _ = raw_pool(pf, vol)
    slots = np.flatnonzero(index.reshape(-1) >= 0)
    assert slots.size == n and np.array_equal(np.sort(index.reshape(-1)[slots]), np.arange(n))
    for q in range(n):
        bx, by, bz, _ = coords[q]
        assert index[bz, by, bx] == q
    one = {np.dtype(np.float32): np.float32(1), np.dtype(np.float16): np.float16(1),
           np.dtype(np.int16): np.int16(32767)}[Tp.dtype]
    # dense grid of stored values, padded by one voxel of +1 along +x/+y/+z
    G = np.full((s.nz + 1, s.ny + 1, s.nx + 1), one, Tp.dtype)
    for q in range(n):
        bx, by, bz, _ = coords[q]
        G[8 * bz:8 * bz + 8, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8] = Tp[q].reshape(8, 8, 8)
    lz, ly, lx = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    for q in range(n):
        bx, by, bz, _ = coords[q]
        k, j, i = 8 * bz + lz.reshape(-1), 8 * by + ly.reshape(-1), 8 * bx + lx.reshape(-1)
        for c in range(8):
            dx, dy, dz = c & 1, (c >> 1) & 1, c >> 2
            exp = G[k + dz, j + dy, i + dx]
            # cells of the last voxel row of the grid are never read; their corners sit outside
            valid = (i + 1 < s.nx) & (j + 1 < s.ny) & (k + 1 < s.nz)
            got = np.ascontiguousarray(Cp[q, :, c])
            exp = np.ascontiguousarray(exp)
            if got.dtype != np.int16:
                out = ~(np.abs(exp.astype(np.float32)) < 1.0)
                assert np.all(np.isnan(got[valid & out])), (q, c)
                keep = valid & ~out
            else:
                keep = valid
            bits = f"u{got.itemsize}"
            assert np.array_equal(got.view(bits)[keep], exp.view(bits)[keep]), (q, c)
    return index, n


# ----------------------------------------------------------------------------- fusion
@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_bricks_fusion_parity_cfg1(pf, orc, dev, cfg1, fmt):
    say(f"[bricks] cfg1 three frames, format {fmt}")
    spec, intr = cfg1["vol"], cfg1["intr"]
    ov = orc.Volume(spec)
    gv = pf.Tsdf(spec, fmt=fmt, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=4096)
    for depth, R, t in frames_cfg1(cfg1):
        new = ov.integrate_bricks(depth, intr, R, t, edge=E)
        gv.integrate(torch.as_tensor(depth).to(dev), intr, R, t)
        n, overflow = gv.bricks_used()
        assert overflow == 0 and n == int(ov.bricks.sum()), (n, int(ov.bricks.sum()), new)
        T, W = gv.export_linear()
        T, W = T.cpu().numpy().astype(np.float64), W.cpu().numpy()
        assert np.array_equal(W, ov.W.astype(np.float32)), "weights must match exactly"
        upd = ov.W > 0
        assert np.abs(T - ov.T)[upd].max() <= T_TOL[fmt]
        assert np.all(T[~upd] == 1.0)
        index, _ = check_pool_consistent(pf, gv)
        assert np.array_equal(index >= 0, ov.bricks.astype(bool))
        say(f"    {n} bricks ({new} new) of {index.size}")
    assert 0 < int(ov.bricks.sum()) < ov.bricks.size


def test_bricks_fusion_extreme_depths(pf, orc, dev, cfg1):
    """Depth pixels far beyond the grid (up to 1e30 m), invalid values and a camera inside the grid:
    the candidate search stays bounded and the bricks match the oracle's."""
    say("[bricks] extreme depth values")
    spec, intr = cfg1["vol"], cfg1["intr"]
    rng = np.random.default_rng(17)
    depth = cfg1["depth1"].copy()
    m = rng.random(depth.shape)
    depth[m < 0.02] = 1e30
    depth[(m >= 0.02) & (m < 0.04)] = 1e6
    depth[(m >= 0.04) & (m < 0.05)] = np.nan
    depth[(m >= 0.05) & (m < 0.06)] = -1.0
    depth[(m >= 0.06) & (m < 0.07)] = np.inf
    R, t = cfg1["gt1"]
    ov = orc.Volume(spec)
    ov.integrate_bricks(depth, intr, R, t, edge=E)
    gv = pf.Tsdf(spec, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=4096)
    gv.integrate(torch.as_tensor(depth).to(dev), intr, R, t)
    n, overflow = gv.bricks_used()
    assert overflow == 0 and n == int(ov.bricks.sum()) > 0
    T, W = gv.export_linear()
    assert np.array_equal(W.cpu().numpy(), ov.W.astype(np.float32))
    assert np.abs(T.cpu().numpy().astype(np.float64) - ov.T)[ov.W > 0].max() <= T_TOL[0]


def test_bricks_overflow(pf, orc, dev, cfg1):
    say("[bricks] pool smaller than the band")
    spec, intr = cfg1["vol"], cfg1["intr"]
    ov = orc.Volume(spec)
    fr = frames_cfg1(cfg1)
    ov.integrate_bricks(fr[0][0], intr, fr[0][1], fr[0][2], edge=E)
    need = int(ov.bricks.sum())
    cap = need // 3
    gv = pf.Tsdf(spec, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=cap)
    gv.integrate(torch.as_tensor(fr[0][0]).to(dev), intr, fr[0][1], fr[0][2])
    assert gv.bricks_used() == (cap, 1)
    index, _ = check_pool_consistent(pf, gv)
    got = index >= 0
    assert got.sum() == cap and np.all(ov.bricks.astype(bool)[got])
    # the bricks that got a slot hold the oracle's values; the rest read (+1, 0)
    T, W = gv.export_linear()
    T, W = T.cpu().numpy().astype(np.float64), W.cpu().numpy()
    m = np.repeat(np.repeat(np.repeat(got, E, 0), E, 1), E, 2)
    assert np.array_equal(W[m], ov.W[m].astype(np.float32)) and np.abs(T - ov.T)[m].max() <= T_TOL[0]
    assert np.all(W[~m] == 0) and np.all(T[~m] == 1.0)
    # a full pool stays full and keeps its flag; the allocated bricks keep fusing
    gv.integrate(torch.as_tensor(fr[1][0]).to(dev), intr, fr[1][1], fr[1][2])
    assert gv.bricks_used() == (cap, 1)
    check_pool_consistent(pf, gv)
    gv.init()
    assert gv.bricks_used() == (0, 0)


@pytest.mark.parametrize("fmt", [0, 2])
def test_bricks_import_export_roundtrip(pf, dev, fmt):
    say(f"[bricks] import/export round trip, format {fmt}")
    spec = synth.VolumeSpec(40, 24, 32, 0.02, 0.08, (-0.4, -0.24, 0.7))
    rng = np.random.default_rng(3)
    T = np.ones((32, 24, 40), np.float32)
    W = np.zeros_like(T)
    nbz, nby, nbx = 4, 3, 5
    keep = rng.random((nbz, nby, nbx)) < 0.4
    keep[0, 0, 0] = keep[-1, -1, -1] = True
    for bz, by, bx in zip(*np.nonzero(keep)):
        sl = np.s_[8 * bz:8 * bz + 8, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
        T[sl] = rng.uniform(-1, 1, (8, 8, 8)).astype(np.float32)
        W[sl] = rng.integers(0, 6, (8, 8, 8))
    T[0, 0, 8] = -1.0                      # a lone -1 with weight 0 still needs its brick
    keep[0, 0, 1] = True
    if fmt == 2:   # values the int16 storage holds exactly: q / 32767 as the export computes it
        T = np.round(T.astype(np.float64) * 32767).astype(np.float32) * np.float32(1.0 / 32767.0)
    gv = pf.Tsdf(spec, fmt=fmt, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=64)
    gv.import_linear(T, W)
    assert gv.bricks_used() == (int(keep.sum()), 0)
    index, _ = check_pool_consistent(pf, gv)
    assert np.array_equal(index >= 0, keep)
    T2, W2 = gv.export_linear()
    assert np.array_equal(T2.cpu().numpy(), T) and np.array_equal(W2.cpu().numpy(), W)


# ----------------------------------------------------------------------------- brick gather
def fused_pair(pf, dev, cfg1, fmt):
    """The bricked volume after three fusions, and a dense CELLS volume loaded with its values."""
    spec, intr = cfg1["vol"], cfg1["intr"]
    gb = pf.Tsdf(spec, fmt=fmt, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=4096)
    for depth, R, t in frames_cfg1(cfg1):
        gb.integrate(torch.as_tensor(depth).to(dev), intr, R, t)
    T, W = gb.export_linear()
    gc = pf.Tsdf(spec, fmt=fmt, device=dev, layout=pf.LAYOUT_CELLS, init=False)
    gc.import_linear(T, W)
    return gb, gc


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_bricks_scoring_equals_cells(pf, orc, dev, cfg1, fmt):
    say(f"[bricks] scoring and gradients vs the dense replica, format {fmt}")
    gb, gc = fused_pair(pf, dev, cfg1, fmt)
    xyz, _ = orc.backproject(cfg1["depth2"], cfg1["intr"], 1)
    far = np.array([[50.0, 0.0, 1.0], [-3.0, 2.0, 0.5]])
    xt = torch.as_tensor(np.concatenate([xyz, far]).astype(np.float32)).to(dev)
    px, py, pz = xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous()
    for K, rot, trans in ((3073, 10.0, 0.1), (300, 1.0, 0.01), (64, 30.0, 0.5), (5, 5.0, 0.03)):
        rng = np.random.default_rng(K)
        R0, t0 = cfg1["init2"]
        poses = [(R0, t0)] + [orc.compose(rng.uniform(-1, 1, 3) * math.radians(rot), rng.uniform(-1, 1, 3) * trans,
                                          R0, t0) for _ in range(K - 1)]
        P = torch.as_tensor(pf.poses_to_f32(poses)).to(dev)
        a = pf.particles_score(gb, px, py, pz, P)
        b = pf.particles_score(gc, px, py, pz, P)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), K
        assert int((a[1] > 0).sum()) > K // 2
    base = torch.as_tensor(np.stack([np.concatenate([np.asarray(R).reshape(3, 3), np.asarray(t).reshape(3, 1)], 1)
                                     .reshape(-1) for R, t in poses[:5]]), dtype=torch.float64).to(dev)
    ga = pf.particles_score_grad(gb, px, py, pz, base)
    gcc = pf.particles_score_grad(gc, px, py, pz, base)
    for x, y in zip(ga, gcc):
        assert torch.equal(x, y)


def check_brick_mask(pf, vol):
    """Every slot's 8 cell-validity words against its cell blocks: bit l % 64 of word l / 64 is set
    iff all 8 corners of the cell at local index l are in the band."""
    _, _, _, Cp, n, _ = raw_pool(pf, vol)
    off = pf.lib().tsdf_mask_offset(ctypes.byref(vol.desc))
    words = vol.T.view(torch.uint8)[off:off + 64 * n].view(torch.int64).cpu().numpy().view(np.uint64).reshape(n, 8)
    if Cp.dtype == np.int16:
        ok = np.abs(Cp.astype(np.int32)) < 32767
    else:
        ok = np.abs(Cp.astype(np.float32)) < 1.0           # NaN-marked corners fail
    valid = ok.all(axis=2).reshape(n, 8, 64)
    want = np.packbits(valid, axis=-1, bitorder="little").view("<u8")[..., 0]
    bad = np.argwhere(words != want)
    assert bad.size == 0, f"{len(bad)} slot words differ, first (slot, word) {bad[:3].tolist()}"
    return int(valid.sum())


@pytest.mark.parametrize("fmt", [0, 1, 2])
def test_bricks_mask_and_masked_scoring(pf, orc, dev, cfg1, fmt):
    """The slots' cell-validity words follow fusion and import, and scoring through them (with the
    compaction, over spreads that reach unallocated bricks and outside the grid) equals scoring
    without them bit for bit."""
    say(f"[bricks] cell-validity words and masked scoring, format {fmt}")
    gb, gc = fused_pair(pf, dev, cfg1, fmt)
    assert check_brick_mask(pf, gb) > 1000
    T, W = gb.export_linear()
    gi = pf.Tsdf(cfg1["vol"], fmt=fmt, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=4096, init=False)
    gi.import_linear(T, W)
    check_brick_mask(pf, gi)
    xyz, _ = orc.backproject(cfg1["depth2"], cfg1["intr"], 1)
    far = np.array([[50.0, 0.0, 1.0], [-3.0, 2.0, 0.5]])
    xt = torch.as_tensor(np.concatenate([xyz, far]).astype(np.float32)).to(dev)
    pts = (xt[:, 0].contiguous(), xt[:, 1].contiguous(), xt[:, 2].contiguous())
    try:
        for K, rot, trans in ((3073, 10.0, 0.1), (257, 1.0, 0.01), (5, 30.0, 0.5)):
            rng = np.random.default_rng(K + fmt)
            R0, t0 = cfg1["init2"]
            poses = [(R0, t0)] + [orc.compose(rng.uniform(-1, 1, 3) * math.radians(rot),
                                              rng.uniform(-1, 1, 3) * trans, R0, t0) for _ in range(K - 1)]
            P = torch.as_tensor(pf.poses_to_f32(poses)).to(dev)
            pf.score_mask(pf.MASK_NEVER)
            a = pf.particles_score(gb, *pts, P)
            pf.score_mask(pf.MASK_ALWAYS)
            b = pf.particles_score(gb, *pts, P)
            c = pf.particles_score(gc, *pts, P)
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), K
            assert torch.equal(b[0], c[0]) and torch.equal(b[1], c[1]), K
    finally:
        pf.score_mask(pf.MASK_BY_SPREAD)


@pytest.mark.parametrize("schedule", ["fixed", "paper_polish"])
def test_bricks_track_frame_equals_cells(pf, dev, cfg1, schedule):
    say(f"[bricks] track_frame vs the dense replica, {schedule}")
    gb, gc = fused_pair(pf, dev, cfg1, 0)
    if schedule == "fixed":
        prm = pf.TrackParams(seed=5, frame_index=2, n_iters=10, K=1024, rates=(1,), pixel_stride=2, s1_deg=5.0,
                             s1_m=0.03)
    else:
        prm = pf.TrackParams(seed=5, frame_index=2, n_iters=12, K=1024, rates=(8, 16, 32), pixel_stride=1,
                             s1_deg=5.0, s1_m=0.03, Ks=(1024, 3072, 10240), polish_steps=5, stop_deg=0.05,
                             stop_m=0.0005)
    depth = torch.as_tensor(cfg1["depth2"]).to(dev)
    R0, t0 = cfg1["init2"]
    Ra, ta, sa = pf.Tracker(cfg1["intr"], prm).track(gb, depth, R0, t0)
    Rb, tb, sb = pf.Tracker(cfg1["intr"], prm).track(gc, depth, R0, t0)
    assert np.array_equal(Ra, Rb) and np.array_equal(ta, tb)
    n = sa.n_iters
    assert n == sb.n_iters and list(sa.Estar[:n]) == list(sb.Estar[:n]) and list(sa.n_adv[:n]) == list(sb.n_adv[:n])
    assert sa.E_final == sb.E_final and sa.polish_accepted == sb.polish_accepted
    R2, t2 = cfg1["gt2"]
    say(f"    {n} iterations, rot err {math.degrees(np.arccos(np.clip((np.trace(R2.T @ Ra) - 1) / 2, -1, 1))):.3f} deg")


def test_bricks_batch_equals_cells(pf, dev, cfg1):
    say("[bricks] batched tracking on bricked volumes vs dense")
    gb, gc = fused_pair(pf, dev, cfg1, 0)
    depth = torch.as_tensor(cfg1["depth2"]).to(dev)
    R0, t0 = cfg1["init2"]
    out = []
    for vol in (gb, gc):
        probs = [(vol, depth, cfg1["intr"], R0, t0,
                  pf.TrackParams(seed=40 + p, frame_index=2, n_iters=6, K=512 * (p + 1), rates=(1,), pixel_stride=2,
                                 s1_deg=5.0, s1_m=0.03)) for p in range(3)]
        b = pf.Batch(probs, pf.BatchPlan(4, 1024, 1))
        b.run()
        out.append(b.results())
        b.close()
    for (R1, t1, s1), (R2, t2, s2) in zip(*out):
        assert np.array_equal(R1, R2) and np.array_equal(t1, t2) and s1.E_final == s2.E_final


def test_bricks_sequence_room_2cm(pf, orc, dev):
    """Sixteen frames of the paper-scale sequence (every 12th, so the camera sweeps the room, with
    fast rotations between them) fused at the true poses into the whole room at 2 cm: after every
    fourth frame the bricks, weights and values match the oracle's bricked fusion, and at the end
    every cell block of every slot equals its stored corners."""
    f = synth.cfg2_frames(181)
    spec = synth.room_spec(f["scene"], 0.02, 0.08)
    say(f"[bricks] sequence into the room at 2 cm: {spec.nx}x{spec.ny}x{spec.nz}")
    intr = f["intr"]
    ov = orc.Volume(spec)
    gv = pf.Tsdf(spec, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=40000)
    for q, t in enumerate(range(0, 181, 12)):
        depth = f["depth"](t)
        ov.integrate_bricks(depth, intr, *f["gt"][t], edge=E)
        gv.integrate(torch.as_tensor(depth).to(dev), intr, *f["gt"][t])
        if q % 4 == 3 or t == 180:
            n, overflow = gv.bricks_used()
            assert overflow == 0 and n == int(ov.bricks.sum())
            T, W = gv.export_linear()
            assert np.array_equal(W.cpu().numpy(), ov.W.astype(np.float32)), t
            upd = ov.W > 0
            # the FP32 running average rounds once per update
            assert np.abs(T.cpu().numpy().astype(np.float64) - ov.T)[upd].max() <= 2e-6 * (1 + q), t
            say(f"    frame {t}: {n} bricks")
    index, _ = check_pool_consistent(pf, gv)
    assert np.array_equal(index >= 0, ov.bricks.astype(bool))


# ----------------------------------------------------------------------------- full size
def test_fullsize_bricks_whole_room(pf, orc, dev):
    """The paper-scale sequence's room as one bricked grid at 1 cm (608 x 312 x 512 voxels, the
    walls the dense 512^3 cube leaves out included): three fusions at the true poses against the
    oracle's bricked fusion over the whole grid, then scoring 3073 poses on a full 640x480 frame
    bitwise equal to the dense replica loaded with the same values."""
    f = synth.cfg2_frames(3)
    spec = synth.room_spec(f["scene"], 0.01, 0.04)
    say(f"[bricks] whole room {spec.nx}x{spec.ny}x{spec.nz}, three fusions")
    intr = f["intr"]
    ov = orc.Volume(spec)
    gv = pf.Tsdf(spec, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=120000)
    for t in range(3):
        depth = f["depth"](t)
        ov.integrate_bricks(depth, intr, *f["gt"][t], edge=E)
        gv.integrate(torch.as_tensor(depth).to(dev), intr, *f["gt"][t])
    n, overflow = gv.bricks_used()
    assert overflow == 0 and n == int(ov.bricks.sum())
    T, W = gv.export_linear()
    W = W.cpu().numpy()
    assert np.array_equal(W, ov.W.astype(np.float32))
    T = T.cpu().numpy()
    upd = ov.W > 0
    assert np.abs(T.astype(np.float64) - ov.T)[upd].max() <= T_TOL[0]
    assert np.all(T[~upd] == 1.0)
    say(f"    {n} bricks of {ov.bricks.size}, {int(upd.sum())} voxels observed")
    del ov
    gc = pf.Tsdf(spec, device=dev, layout=pf.LAYOUT_CELLS, init=False)
    gc.import_linear(torch.as_tensor(T).to(dev), torch.as_tensor(W).to(dev))
    del T, W
    px, py, pz, nd = pf.backproject(torch.as_tensor(f["depth"](2)).to(dev), intr, 1)
    npts = int(nd[0].item())
    rng = np.random.default_rng(9)
    R0, t0 = f["gt"][2]
    poses = [(R0, t0)] + [orc.compose(rng.uniform(-1, 1, 3) * math.radians(5), rng.uniform(-1, 1, 3) * 0.05, R0, t0)
                          for _ in range(3072)]
    P = torch.as_tensor(pf.poses_to_f32(poses)).to(dev)
    a = pf.particles_score(gv, px, py, pz, P, n_pts=npts)
    b = pf.particles_score(gc, px, py, pz, P, n_pts=npts)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert int(a[1][0].item()) > npts // 2


def test_bricks_grid_beyond_dense_limit(pf, dev):
    """A 2048 x 1024 x 2048 grid at 0.5 cm (4.3e9 voxels: more than the dense layouts address)
    around the paper-scale room, against a bricked grid that covers only the room plus two bricks
    of margin on the same lattice: after two fusions both hold the same bricks with identical
    weights and T within FP32 rounding (the voxel centres, origin + vs i, round differently in FP64
    from the two origins), and score 512 poses alike (sample positions round differently in FP32)."""
    f = synth.cfg2_frames(2)
    intr, sc = f["intr"], f["scene"]
    vs, tau = 0.005, 0.02
    c = synth.room_centre_world(sc)
    big = synth.VolumeSpec(2048, 1024, 2048, vs, tau, tuple(float(c[a]) - 0.5 * n * vs + 0.5 * vs
                                                              for a, n in enumerate((2048, 1024, 2048))))
    lo_w = sc["R_wr"] @ sc["room_lo"] + sc["t_wr"] - 2 * E * vs
    hi_w = sc["R_wr"] @ sc["room_hi"] + sc["t_wr"] + 2 * E * vs
    o = np.array(big.origin)
    start = (np.floor((lo_w - o) / vs / E) * E).astype(int)
    end = (np.ceil((hi_w - o) / vs / E) * E).astype(int)
    n = end - start
    small = synth.VolumeSpec(int(n[0]), int(n[1]), int(n[2]), vs, tau, tuple(float(x) for x in o + start * vs))
    say(f"[bricks] {big.nx}x{big.ny}x{big.nz} grid vs {small.nx}x{small.ny}x{small.nz} at offset {start.tolist()}")
    gb = pf.Tsdf(big, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=300000)
    gs = pf.Tsdf(small, device=dev, layout=pf.LAYOUT_BRICKS, max_bricks=300000)
    with pytest.raises(pf.PFError):
        gb.export_linear()
    # Frame 0 sits at the identity and this lattice is axis-aligned with it, so many voxel centres
    # project exactly onto pixel borders; the two grids compute those centres from different
    # origins (origin + vs i rounds differently in FP64) and would break such ties differently.
    # A small generic rotation and shift of both fusion poses removes the exact ties.
    Rp, tp = synth.rot(np.array([0.0031, -0.0047, 0.0023])), np.array([0.00123, -0.00077, 0.00051])
    ms = {}
    for t in range(2):
        d = torch.as_tensor(f["depth"](t)).to(dev)
        Rt, tt = f["gt"][t]
        for name, vol in (("big", gb), ("small", gs)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            vol.integrate(d, intr, Rp @ Rt, Rp @ tt + tp)
            e1.record()
            torch.cuda.synchronize()
            ms[name] = e0.elapsed_time(e1)
    say(f"    second fusion: {ms['big']:.2f} ms on the big grid, {ms['small']:.2f} ms on the room grid")
    ib, cb, Tb, Cb, nb_, ob = raw_pool(pf, gb)
    is_, cs, Ts, Cs, ns_, os_ = raw_pool(pf, gs)
    assert ob == 0 and os_ == 0 and nb_ == ns_ > 1000
    say(f"    {ns_} bricks in both")
    Wb = gb.W[:512 * nb_].cpu().numpy().reshape(nb_, 512)
    Ws = gs.W[:512 * ns_].cpu().numpy().reshape(ns_, 512)
    off = start // E
    qb = ib[cs[:, 2] + off[2], cs[:, 1] + off[1], cs[:, 0] + off[0]]      # big slot of every small slot
    assert np.all(qb >= 0) and np.unique(qb).size == ns_
    assert np.array_equal(Ws, Wb[qb])
    assert np.abs(Ts - Tb[qb]).max() <= 2e-6
    # cells of the room grid's last voxel row along an axis have corners outside it; they are never
    # read (sample cells are clamped one voxel inside) and are left out
    lz, ly, lx = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    gi = cs[:, :1] * 8 + lx.reshape(1, -1)
    gj = cs[:, 1:2] * 8 + ly.reshape(1, -1)
    gk = cs[:, 2:3] * 8 + lz.reshape(1, -1)
    inner = (gi < small.nx - 1) & (gj < small.ny - 1) & (gk < small.nz - 1)
    a, b = Cs[inner], Cb[qb][inner]
    assert np.array_equal(np.isnan(a), np.isnan(b))       # corners outside the band are NaN in both
    fin = ~np.isnan(a)
    assert np.abs(a[fin] - b[fin]).max() <= 2e-6
    # scoring reads the same cells through either index grid
    px, py, pz, nd = pf.backproject(torch.as_tensor(f["depth"](1)).to(dev), intr, 1)
    npts = int(nd[0].item())
    rng = np.random.default_rng(4)
    R0, t0 = Rp @ f["gt"][1][0], Rp @ f["gt"][1][1] + tp      # the pose frame 1 was fused at
    poses = [(R0, t0)] + [(synth.rot(rng.uniform(-1, 1, 3) * math.radians(2.0)) @ R0, t0 + rng.uniform(-1, 1, 3) * 0.02)
                          for _ in range(511)]
    P = torch.as_tensor(pf.poses_to_f32(poses)).to(dev)
    a = pf.particles_score(gb, px, py, pz, P, n_pts=npts)
    b = pf.particles_score(gs, px, py, pz, P, n_pts=npts)
    Ea, Eb = a[0].cpu().numpy().astype(np.float64), b[0].cpu().numpy().astype(np.float64)
    na, nb2 = a[1].cpu().numpy(), b[1].cpu().numpy()
    assert int(na[0]) > npts // 2
    assert np.all(np.abs(na - nb2) <= 1 + na // 2000)
    assert np.all(np.abs(Ea - Eb) <= 1e-4 * Eb)
