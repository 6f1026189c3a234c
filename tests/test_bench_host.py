"""The benchmark's contract on the host: the one-GPU refusal and the CPU
baseline record (the oracle timed on a small scene)."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_cpu_baseline_record():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2503_16424_amd import scenes
    sc = scenes.tiny_128(0)
    tgt = scenes.tiny_128_target(0).astype(np.float64)
    rec = bench.cpu_baseline(sc, tgt, rows=32)
    assert rec["kind"] == "oracle" and rec["unit"] == "steps/s"
    assert rec["value"] > 0 and rec["cores"] >= 1
    assert "rows 48..79 (32 of 128" in rec["sample"]
    full = bench.cpu_baseline(sc, tgt, rows=10 ** 6)           # clamped to the frame
    assert "(128 of 128" in full["sample"]
