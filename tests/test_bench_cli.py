"""bench.py's contract on the CPU: one GPU only, and HBM traffic attached only
to the kernel it was measured on."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_kernel_id_tracks_options_and_traffic_records_are_keyed():
    a = bench.kernel_id({"precision": "mixed", "schedule": "batched", "ssa_k": 8})
    b = bench.kernel_id({"precision": "mixed", "schedule": "batched", "ssa_k": 4})
    assert a != b and len(a) == 16
    assert bench.recorded_traffic("0000000000000000") is None
    # every traffic record in the profile summaries is well formed
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if not name.endswith(".md"):
            continue
        for ln in open(os.path.join(ROOT, "profiles", name)):
            if ln.startswith("<!-- traffic "):
                rec = json.loads(ln.strip()[len("<!-- traffic "):-len("-->")])
                assert rec["fetch_bytes"] > 0 and rec["write_bytes"] > 0
                assert bench.recorded_traffic(rec["kernel_id"])[0] == (rec["fetch_bytes"]
                                                                       + rec["write_bytes"])


def test_repeat_timed_runs_until_the_time_has_passed():
    import time
    import bench
    calls = []
    first, reps, secs = bench.repeat_timed(lambda: calls.append(1) or len(calls), 0.2)
    assert first == 1 and reps == len(calls) and reps >= 2 and secs >= 0.2
    first, reps, _ = bench.repeat_timed(lambda: time.sleep(0.05) or "x", 0.0)
    assert first == "x" and reps == 1
