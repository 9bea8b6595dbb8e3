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
        "the scoring kernel changed since profiles/k_score_sequence_counters.txt was taken"
    assert float(vals["fetch_scale"]) > 0 and float(vals["write_scale"]) > 0
