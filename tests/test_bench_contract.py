"""CPU checks of bench.py's command-line contract (no GPU): the single-GPU path refuses other
GPU counts before touching a device, and the counter summary it reads belongs to the current
scoring kernel."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_gpus_other_than_one_exit_with_a_message():
    for n in ("2", "8"):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", n], capture_output=True,
                           text=True, timeout=120)
        assert r.returncode == 2, r
        assert "single-GPU" in r.stderr and r.stdout == ""


def test_counter_summary_matches_the_scoring_sources():
    import bench
    vals = {}
    for line in open(bench.COUNTERS):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    assert vals["score_source_sha256"] == bench.score_source_hash(), \
        "the scoring kernel changed since profiles/k_draw_score_sequence_counters.txt was taken"
    for k in ("evals_per_dispatch", "fetch_kib_per_dispatch", "write_kib_per_dispatch", "fetch_scale", "write_scale",
              "valu_insts_per_dispatch", "tcp_tcc_read_req_per_dispatch", "tcc_hit_per_dispatch",
              "tcc_miss_per_dispatch"):
        assert float(vals[k]) > 0, k
    c = bench.read_counters()
    r = bench.roofline(0.15, c["evals_per_dispatch"])
    assert 0 < r["frac"] <= 1 and 0 < r["counters"]["valu_issue_frac"] <= 1 and r["counters"]["hbm_frac"] < 1


def test_roofline_bound_is_a_rate_below_peak():
    """The scoring roofline counts the method's own vector operations per sample against the chip's
    lane-operation rate: 38 operations per sample, 256 x 4 x 16 lanes at 2.4 GHz."""
    import bench
    assert bench.OPS_PER_EVAL == 38
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9
    r = bench.roofline(1.0, 1e9)   # 1e9 samples in 1 ms
    assert r["bound"] == "alu" and abs(r["achieved"] - 38.0) < 1e-9 and r["frac"] < 1
