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
    assert full["oracle_pairs"] > 0 and "oracle_pairs_band" in rec
    assert full["one_core"]["value"] > 0 and set(full["configs"]) == {"tiny_128", "open_512"}
    assert full["cpu_model"] and "_gauss" in full


def test_stage_rooflines_take_the_larger_bound():
    sys.path.insert(0, ROOT)
    import bench
    ms = {"sample_bin": 1.0, "fwd_l2": 1.0, "bwd_gauss": 1.0, "bwd_curves": 1.0}
    st = bench.stage_rooflines(ms, n_gauss=10 ** 6, pairs=10 ** 7, n_alg=10 ** 9, n_tiles=10 ** 4,
                               hw=10 ** 6, trans_slots=2.0, bw_gbs=8000.0, lane_ops=4e13)
    # sample_bin: 48e6 + 4e7 + 8e4 bytes at 8 TB/s
    assert abs(st["sample_bin"]["roof_ms"] - (48e6 + 4e7 + 8e4) / 8e12 * 1e3) < 1e-12
    assert st["sample_bin"]["bound"] == "hbm" and st["bwd_curves"]["bound"] == "hbm"
    # forward: 1e9 pairs x (13 + 2) slots at 4e13 slots/s
    assert st["fwd_l2"]["bound"] == "alu"
    assert abs(st["fwd_l2"]["roof_ms"] - 1e9 * 15 / 4e13 * 1e3) < 1e-9
    assert abs(st["bwd_gauss"]["roof_ms"] - 1e9 * 34 / 4e13 * 1e3) < 1e-9
