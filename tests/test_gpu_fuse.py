"""track_frame_fuse: one frame of the method's cycle (Sec. III "Method overview", Fig. 2), tracking
then fusion at the tracked pose, against track_frame followed by tsdf_integrate at the returned
pose. Bars: the poses and the per-iteration records bitwise equal, and after every frame the stored
volume (T, W and, for the replica, the cell-validity mask) bitwise equal, in the three layouts and in
FP16 storage; then the same over three frames of the paper-scale sequence."""
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


def _same_volume(a, b, layout, what):
    Ta, Wa = a.export_linear()
    Tb, Wb = b.export_linear()
    assert torch.equal(Wa, Wb), f"{what}: W differs"
    assert torch.equal(Ta.view(torch.int32), Tb.view(torch.int32)), f"{what}: T differs"
    if layout == 1:
        assert torch.equal(a.cell_mask()[0], b.cell_mask()[0]), f"{what}: mask differs"


def _run(pf, spec, intr, depths, poses0, prm, layout, fmt=0, max_bricks=0):
    dev = torch.device("cuda:0")
    kw = dict(device=dev, layout=layout, fmt=fmt, max_bricks=max_bricks)
    va, vb = pf.Tsdf(spec, **kw), pf.Tsdf(spec, **kw)
    for v in (va, vb):
        v.integrate(depths[0], intr, np.eye(3), np.zeros(3))
    ta, tb = pf.Tracker(intr, prm, device=dev), pf.Tracker(intr, prm, device=dev)
    for t in range(1, len(depths)):
        R0, t0 = poses0[t]
        ta.set_frame(t)
        tb.set_frame(t)
        Ra, tra, sa = ta.track(va, depths[t], R0, t0)
        va.integrate(depths[t], intr, Ra, tra)
        Rb, trb, sb = tb.track_fuse(vb, depths[t], R0, t0)
        assert np.array_equal(Ra, Rb) and np.array_equal(tra, trb), f"frame {t}: poses differ"
        n = sa.n_iters
        assert n == sb.n_iters and list(sa.n_adv[:n]) == list(sb.n_adv[:n]) and list(sa.Estar[:n]) == list(sb.Estar[:n])
        assert sa.E_final == sb.E_final
        _same_volume(va, vb, layout, f"layout {layout} format {fmt}, frame {t}")
    return va, vb


@pytest.mark.parametrize("layout,fmt", [(1, 0), (0, 0), (2, 0), (1, 1)])
def test_track_fuse_equals_track_then_integrate(pf, layout, fmt):
    say(f"[fuse] track_frame_fuse vs track_frame + tsdf_integrate, layout {layout}, format {fmt}")
    d = synth.cfg1_inputs()
    dev = torch.device("cuda:0")
    depths = [torch.as_tensor(d["depth1"]).to(dev), torch.as_tensor(d["depth2"]).to(dev),
              torch.as_tensor(d["depth1"]).to(dev)]
    poses0 = [None, d["init2"], d["init2"]]
    prm = pf.TrackParams(seed=9, frame_index=1, n_iters=12, K=768, rates=(1, 2), pixel_stride=2, s1_deg=8.0,
                         s1_m=0.08)
    _run(pf, d["vol"], d["intr"], depths, poses0, prm, layout, fmt, max_bricks=4096 if layout == 2 else 0)


def test_track_fuse_paper_scale_three_frames(pf):
    say("[fuse] paper-scale sequence, frames 1..3: track_frame_fuse vs track_frame + tsdf_integrate")
    f = synth.cfg2_frames(4)
    dev = torch.device("cuda:0")
    depths = [torch.as_tensor(f["depth"](t)).to(dev) for t in range(4)]
    # each frame starts from the previous frame's true pose composed with the stand-in
    R0, t0 = f["gt"][0]
    gt = [(R0.T @ f["gt"][k][0], R0.T @ (f["gt"][k][1] - t0)) for k in range(4)]
    poses0 = [None] + [(gt[t - 1][0] @ f["rel"][t][0], gt[t - 1][0] @ f["rel"][t][1] + gt[t - 1][1]) for t in range(1, 4)]
    prm = pf.TrackParams(seed=14, frame_index=1, n_iters=20, K=3072, rates=(8, 16, 32), pixel_stride=1, s1_deg=10.0,
                         s1_m=0.10)
    _run(pf, f["vol"], f["intr"], depths, poses0, prm, 1)
