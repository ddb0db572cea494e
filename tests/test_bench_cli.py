"""bench.py's command line on the CPU: more than one GPU is refused with a
message before anything touches a device, and the counter record it reads
for roofline.traffic is well formed."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counter_record_is_well_formed():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert len(rec["source_hash"]) == 64
    cal = rec["calibration"]
    assert 1.9 < cal["fetch_factor"] < 2.1 and 0.9 < cal["write_factor"] < 1.1
    for e in rec["entries"]:
        assert e["read_bytes"] > 0 and e["write_bytes"] > 0
        assert {"poles", "width", "n", "m", "points_per_lane", "variant"} <= set(e)
