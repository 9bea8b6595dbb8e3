"""track_frame_noalloc (the entry point whose workspace is the library's own per-GPU array, for
callers that cannot allocate) against track_frame with a caller workspace: two calls in a row, the
second on a smaller frame, each bit for bit equal to track_frame on the same input."""
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


def _problem(pf, p, dev):
    d = synth.random_depth_for_batch(p)
    vol = pf.Tsdf(d["vol"], device=dev)
    vol.integrate(torch.as_tensor(d["depth1"]).to(dev), d["intr"], np.eye(3), np.zeros(3))
    return d, vol, torch.as_tensor(d["depth2"]).to(dev)


def _same(a, b):
    (R1, t1, s1), (R2, t2, s2) = a, b
    assert np.array_equal(R1, R2) and np.array_equal(t1, t2)
    assert s1.n_iters == s2.n_iters and s1.n_points == s2.n_points
    n = s1.n_iters
    for f in ("E0", "Estar", "n_adv", "n_sub", "n_valid", "s_rad", "s_m", "n_particles"):
        assert list(getattr(s1, f)[:n]) == list(getattr(s2, f)[:n]), f
    assert s1.E_final == s2.E_final and s1.n_valid_final == s2.n_valid_final
    assert s1.polish_accepted == s2.polish_accepted


def test_noalloc_equals_track_frame_on_two_calls(pf):
    dev = torch.device("cuda:0")
    # a 640x480 problem, then a 160x120 one, of the batching workload's shape
    sizes = {}
    for p in range(64):
        w = synth.random_depth_for_batch(p)["intr"].width
        sizes.setdefault(w, p)
        if 640 in sizes and 160 in sizes:
            break
    cases = [(sizes[640], dict(K=3072, n_iters=20, rates=(8, 16, 32), pixel_stride=1, polish_steps=5)),
             (sizes[160], dict(K=256, n_iters=10, rates=(1,), pixel_stride=2, polish_steps=0))]
    prev_need = None
    for p, kw in cases:
        d, vol, depth = _problem(pf, p, dev)
        prm = pf.TrackParams(seed=40 + p, frame_index=1, s1_deg=10.0, s1_m=0.10, **kw)
        need = pf.track_workspace_bytes(d["intr"], prm)
        say(f"[noalloc] problem {p}: {d['intr'].width}x{d['intr'].height}, K {kw['K']}, workspace {need} bytes")
        assert need <= pf.NOALLOC_WORKSPACE_BYTES
        if prev_need is not None:
            assert need < prev_need    # the second call is the smaller one
        prev_need = need
        R0, t0 = d["init2"]
        ref = pf.Tracker(d["intr"], prm, device=dev).track(vol, depth, R0, t0)
        got = pf.track_frame_noalloc(vol, depth, d["intr"], R0, t0, prm)
        _same(ref, got)
        # and again, now that the array holds this call's own contents
        _same(ref, pf.track_frame_noalloc(vol, depth, d["intr"], R0, t0, prm))
