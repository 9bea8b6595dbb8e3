"""Form (2): batched tracking of heterogeneous problems in one fixed kernel sequence, against the
plain per-problem path (bitwise: the batching does not change any reduction order), under
several launch plans, and replayed from a captured HIP graph."""
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
def problems(pf):
    """Six problems of the batching workload shape (own rooms, resolutions 160x120 .. 640x480,
    K in [256, 4096], own 256^3 volumes at 1 cm), each with frame 1 fused on the GPU."""
    dev = torch.device("cuda:0")
    out = []
    for p in range(6):
        d = synth.random_depth_for_batch(p)
        vol = pf.Tsdf(d["vol"], device=dev)
        vol.integrate(torch.as_tensor(d["depth1"]).to(dev), d["intr"], np.eye(3), np.zeros(3))
        prm = pf.TrackParams(seed=40 + p, frame_index=1, n_iters=6, K=d["K"], rates=(1,), pixel_stride=2,
                             s1_deg=10.0, s1_m=0.10)
        out.append((vol, torch.as_tensor(d["depth2"]).to(dev), d["intr"], *d["init2"], prm))
    torch.cuda.synchronize()
    return out


def plain(pf, problems):
    res = []
    for vol, depth, intr, R0, t0, prm in problems:
        R, t, st = pf.Tracker(intr, prm).track(vol, depth, R0, t0)
        res.append((R, t, st))
    return res


def same(a, b):
    for (R1, t1, s1), (R2, t2, s2) in zip(a, b):
        assert np.array_equal(R1, R2) and np.array_equal(t1, t2)
        n = s1.n_iters
        assert list(s1.n_adv[:n]) == list(s2.n_adv[:n])
        assert list(s1.Estar[:n]) == list(s2.Estar[:n])
        assert s1.E_final == s2.E_final and s1.n_valid_final == s2.n_valid_final and s1.n_points == s2.n_points


@pytest.mark.parametrize("tk,grid,order", [(0, 1024, 1), (4, 1024, 1), (1, 512, 0), (8, 4096, 1), (2, 2048, 0)])
def test_batch_equals_plain(pf, problems, tk, grid, order):
    say(f"[batch] plan tk={tk} grid={grid} order={order}")
    ref = plain(pf, problems)
    b = pf.Batch(problems, pf.BatchPlan(tk, grid, order))
    b.run()
    got = b.results()
    b.close()
    same(got, ref)


def test_batch_polish_equals_plain(pf, problems):
    """The batched gradient polish (form 3 inside form 2) reproduces track_frame's polish bit for bit."""
    import dataclasses
    say("[batch] 4 RO iterations + 5 polish steps, batched vs plain")
    probs = [(v, d, k, R, t, dataclasses.replace(prm, n_iters=4, polish_steps=5)) for v, d, k, R, t, prm in problems]
    ref = plain(pf, probs)
    b = pf.Batch(probs, pf.BatchPlan(4, 1024, 1))
    b.run()
    got = b.results()
    b.close()
    same(got, ref)
    assert [s.polish_accepted for _, _, s in got] == [s.polish_accepted for _, _, s in ref]
    assert sum(s.polish_accepted for _, _, s in got) > 0
    say(f"    accepted steps per problem {[s.polish_accepted for _, _, s in got]}")


def test_batch_graph_replay(pf, problems):
    say("[batch] HIP graph capture and replay")
    b = pf.Batch(problems, pf.BatchPlan(0, 1024, 1))
    b.run()
    eager = b.results()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        b.run(stream=s)
    for rep in range(3):
        # unrelated eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        same(b.results(), eager)
    b.close()


def test_autotuner_records_a_plan(pf, problems, tmp_path):
    from paper_2509_24236_amd import autotune
    path = str(tmp_path / "table.json")
    cands = [pf.BatchPlan(4, 1024, 1), pf.BatchPlan(8, 2048, 1)]
    best = autotune.tune(problems, cands, reps=2, path=path, log=say)
    assert best in cands
    assert autotune.plan_for(problems, path) == best


@pytest.fixture(scope="module")
def problems16(pf):
    """Sixteen problems of the batching workload (seeds 40..55): all four resolutions, K from 256 to
    4096 (the drawn counts, with the two ends of the range forced on problems 13 and 1)."""
    dev = torch.device("cuda:0")
    out = []
    for p in range(16):
        d = synth.random_depth_for_batch(p)
        K = {13: 256, 1: 4096}.get(p, d["K"])
        vol = pf.Tsdf(d["vol"], device=dev)
        vol.integrate(torch.as_tensor(d["depth1"]).to(dev), d["intr"], np.eye(3), np.zeros(3))
        prm = pf.TrackParams(seed=40 + p, frame_index=1, n_iters=10, K=K, rates=(1,), pixel_stride=2,
                             s1_deg=10.0, s1_m=0.10)
        out.append((vol, torch.as_tensor(d["depth2"]).to(dev), d["intr"], *d["init2"], prm))
    torch.cuda.synchronize()
    return out


def test_batch_matches_oracle(pf, orc, problems16):
    """Every problem of a 16-problem batch (the autotuner's plan) lands within 1 mm / 0.05 deg of the
    FP64 oracle's track_frame on that problem's own volume with the same random stream."""
    import math
    from paper_2509_24236_amd import autotune
    widths = sorted({p[2].width for p in problems16})
    Ks = [p[5].K for p in problems16]
    say(f"[batch] 16 problems, widths {widths}, K {min(Ks)}..{max(Ks)}, plan {autotune.plan_for(problems16)}")
    assert widths == [160, 320, 480, 640] and min(Ks) == 256 and max(Ks) == 4096
    b = pf.Batch(problems16, autotune.plan_for(problems16))
    b.run()
    got = b.results()
    b.close()
    worst = (0.0, 0.0)
    for q, ((vol, depth, intr, R0, t0, prm), (R, t, st)) in enumerate(zip(problems16, got)):
        T, W = vol.export_linear()
        ov = orc.Volume(vol.spec, T=T.cpu().numpy().astype(np.float64), W=W.cpu().numpy())
        del T, W
        oprm = orc.make_params(seed=prm.seed, frame_index=1, n_iters=10, K=prm.K, rates=(1,), pixel_stride=2,
                               s1_deg=10.0, s1_m=0.10)
        Ro, to, recs = ov.track_frame(depth.cpu().numpy(), intr, R0, t0, oprm)
        dr, dt = math.degrees(orc.rot_err(R, Ro)), float(np.linalg.norm(t - to))
        worst = (max(worst[0], dr), max(worst[1], dt))
        say(f"    problem {q}: {intr.width}x{intr.height}, K {prm.K}: vs oracle {dr:.2e} deg {dt * 1e3:.2e} mm")
        assert dr <= 0.05 and dt <= 1e-3, f"problem {q}"
        assert [st.n_sub[i] for i in range(10)] == [r.n_pts for r in recs]
        del ov
    say(f"    worst {worst[0]:.2e} deg, {worst[1] * 1e3:.2e} mm")


def test_batch_rate_cycle_equals_plain(pf, problems):
    """The batched sub-sampled views (rates 8, 16, 32 over every pixel) and the per-rate partial sums
    of E* reproduce track_frame bit for bit, under two plans."""
    import dataclasses
    say("[batch] rates 8/16/32 at pixel stride 1, 9 iterations, batched vs plain")
    probs = [(v, d, k, R, t, dataclasses.replace(prm, n_iters=9, rates=(8, 16, 32), pixel_stride=1))
             for v, d, k, R, t, prm in problems]
    ref = plain(pf, probs)
    for plan in (pf.BatchPlan(0, 1024, 1), pf.BatchPlan(2, 512, 0)):
        b = pf.Batch(probs, plan)
        b.run()
        got = b.results()
        b.close()
        same(got, ref)
        assert [list(s.n_sub[:9]) for _, _, s in got] == [list(s.n_sub[:9]) for _, _, s in ref]
