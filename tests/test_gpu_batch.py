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
