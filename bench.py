"""Throughput of the differentiable rasterizer on one MI355X.

One step = bz_sample + bz_bin + bz_render_fwd + L2 gradient + bz_render_bwd
(both stages) over a fixed synthetic scene already resident in HBM.  Default
workload: 2048x2048 canvas, 20,000 curves (12,000 closed with R = 20 interior
rows and 8,000 open 3-segment strokes, 24 samples per row), 6,528,000
Gaussians, seeded draw order, uniform-noise target.

Prints one JSON line (see the README for the fields).  Other workloads:
--workload batched_64 (64 canvases in one batch, against the canvases one
after the other), --workload curvenet (the learned initialiser's training
step), --workload open_512 / tiny_128; --blend-state recompute and
--persistent select the other launch forms of the 2048x2048 step.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd steps/s at 2048², 20k curves; steps-to-PSNR learned vs plain init"

# Algorithmic work per contributing (pixel, Gaussian) pair, in FP32 flops with
# an FMA counted as 2, derived from the blending recurrence:
#   forward : offset d (4), p = 1/2 d^T Q d (7), exp (1), support test (1),
#             alpha = min(alpha_max, o'(G - g_min)) (3), w = alpha T (1),
#             C += w c (6), T *= 1 - alpha (2)                            = 25
#   backward: offset (4), p (7), exp (1), test (1), alpha + clamp (4),
#             T before = T / (1 - alpha) (3), w (1), colour grads (3),
#             alpha grad T sum (c - A) g (9), A update (9), opacity grad (3),
#             p grad (3), d and d d^T moments (5)                          = 53
FLOPS_FWD_PAIR = 25
FLOPS_BWD_PAIR = 53
# The same work as VALU issue slots (one lane operation each, an FMA one
# slot): 13 plain operations + 1 transcendental (exp2) per pair forward, 30 +
# 2 (exp2, reciprocal) backward.  A transcendental's slot cost is measured by
# the rate probes (bz_peak.h); the default below is what they measured on
# MI355X (exp2 and rcp issue at half the FMA rate).
VALU_FWD_PAIR, TRANS_FWD_PAIR = 13, 1
VALU_BWD_PAIR, TRANS_BWD_PAIR = 30, 2
TRANS_SLOTS_DEFAULT = 2.0
# MI355X published peaks: HBM3E 8 TB/s; FP32 vector 157.3 TFLOP/s
# (256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed FP32) x 2.4 GHz).  The
# build leaves packed FP32 off, so its attainable vector rate is half that:
# 78.6 TFLOP/s, 39.3 T lane operations/s.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 256 * 4 * 16 * 2 * 2 * 2.4e9 / 1e12
PEAK_FP32_VALU_TFLOPS = PEAK_FP32_TFLOPS / 2
BYTES_REC = 48


def stage_rooflines(ms, n_gauss, pairs, n_alg, n_tiles, hw, trans_slots, bw_gbs, lane_ops):
    """Per-stage roofline times (ms) of one step at HBM bandwidth bw_gbs and
    lane_ops VALU slots per second: max(algorithmic bytes / bandwidth,
    algorithmic slots / issue rate), with the byte and slot counts of the
    method's work (not of the kernels' tiling):
      sample_bin: records written (48 B per Gaussian), tile lists (4 B per
                  pair) and ranges (8 B per tile);
      fwd_l2:     per pair 13 slots + 1 transcendental; per pixel the image,
                  t_final, n_last written and target read, d_image written
                  (44 B);
      bwd_gauss:  per pair 30 slots + 2 transcendentals; per pixel d_image and
                  state read (20 B); per Gaussian its nine gradient planes
                  read and written (72 B);
      bwd_curves: per Gaussian its nine planes read (36 B)."""
    work = {
        "sample_bin": (BYTES_REC * n_gauss + 4 * pairs + 8 * n_tiles, 0.0),
        "fwd_l2": (44 * hw, n_alg * (VALU_FWD_PAIR + TRANS_FWD_PAIR * trans_slots)),
        "bwd_gauss": (20 * hw + 72 * n_gauss, n_alg * (VALU_BWD_PAIR + TRANS_BWD_PAIR * trans_slots)),
        "bwd_curves": (36 * n_gauss, 0.0),
    }
    out = {}
    for k, (byts, slots) in work.items():
        t_mem = byts / (bw_gbs * 1e9) * 1e3
        t_alu = slots / lane_ops * 1e3
        out[k] = {"roof_ms": max(t_mem, t_alu), "bound": "alu" if t_alu > t_mem else "hbm",
                  "ms": ms[k], "bytes": byts, "slots": slots}
    return out


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper_2048",
                    choices=["paper_2048", "paper_2048_e400", "paper_analog_open",
                             "paper_analog_closed", "open_512", "tiny_128", "batched_64",
                             "curvenet"])
    ap.add_argument("--batch", type=int, default=256, help="curvenet: patches per step")
    ap.add_argument("--persistent", action="store_true",
                    help="persistent blend launches (tiles from a counter)")
    ap.add_argument("--autotune", action="store_true",
                    help="batched_64: pick tile shape and launch form by measurement first")
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--blend-state", default="stored", choices=["stored", "recompute"],
                    help="keep the forward's per-pixel blend state for the backward, or "
                         "recompute it per tile inside the backward")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the rate probes (roofline fractions then use the published "
                         "peaks and a transcendental cost of 2 slots)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before the timed steps, copy a MIB-sized buffer once (a known-size "
                         "kernel to scale hardware byte counters against)")
    ap.add_argument("--no-learned-init", action="store_true",
                    help="skip the steps-to-PSNR measurement of the learned initialiser")
    ap.add_argument("--cpu-rows", type=int, default=2048,
                    help="rows of the frame the CPU oracle renders for its baseline "
                         "(default: the whole 2048-row frame)")
    return ap.parse_args()


def measured_traffic(kernel, workload, tw, th):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE x its copy-calibrated factor + WRITE_SIZE x its factor),
    or None when there is none or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{tw}x{th}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = dict(line.split(":", 1) for line in open(path) if ":" in line and not line.startswith("#"))
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    src = os.path.join(ROOT, "paper_2503_16424_amd", "csrc", kv.get("source", ""))
    if not os.path.exists(src):
        return None
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if digest != kv.get("source_sha256"):
        return None
    return float(kv["traffic_bytes_per_launch"])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def _oracle_step(sc, target, rows):
    """One step of the FP64 oracle on sc: sampling, forward + backward of
    `rows` (with the mean-L2 gradient against target), chain to the curves.
    Returns (seconds of the step scaled to the whole frame, details)."""
    import numpy as np

    import oracle
    H, W = sc.height, sc.width
    rows = min(rows, H)
    y0 = H // 2 - rows // 2
    y1 = y0 + rows
    t0 = time.perf_counter()
    g = oracle.sample(sc)
    t1 = time.perf_counter()
    fw = oracle.render(g, W, H, sc.bg, rows=(y0, y1))
    d = np.zeros((3, H, W))
    d[:, y0:y1] = 2.0 * (fw["image"][:, y0:y1] - target[:, y0:y1]) / (3.0 * H * W)
    t2 = time.perf_counter()
    bw = oracle.render(g, W, H, sc.bg, rows=(y0, y1), d_image=d)
    t3 = time.perf_counter()
    oracle.chain(sc, bw["d_gauss"])
    t4 = time.perf_counter()
    # the backward call re-runs the band's forward itself
    step = (t1 - t0) + (t3 - t2) * (H / rows) + (t4 - t3)
    return step, dict(sample_s=t1 - t0, band_s=t3 - t2, chain_s=t4 - t3, rows=(y0, y1),
                      pairs=bw["pairs"], g=g)


def cpu_baseline(sc, target, rows, one_core_rows=64):
    """The FP64 oracle timed on the host: one step of the same workload on all
    cores (by default the whole frame; with rows < height a band whose time is
    scaled to the frame), the same on one core over a band of one_core_rows
    rows, and one step of the 128x128 and 512x512 workloads on all cores."""
    import numpy as np

    import oracle
    from paper_2503_16424_amd import scenes
    oracle.build()
    cores = oracle.num_threads()
    H = sc.height
    step, det = _oracle_step(sc, target, rows)
    y0, y1 = det["rows"]
    out = dict(value=1.0 / step, unit="steps/s", cores=cores, kind="oracle",
               sample=(f"FP64 oracle on {cores} threads: full sampling ({det['sample_s']:.2f} s) "
                       f"and per-curve chain ({det['chain_s']:.2f} s); forward+backward of rows "
                       f"{y0}..{y1 - 1} ({y1 - y0} of {H}, {det['band_s']:.2f} s) scaled by "
                       f"{H / (y1 - y0):.0f}; host CPU {cpu_model()}"),
               seconds=step, cpu_model=cpu_model(), oracle_pairs=det["pairs"])
    if y1 - y0 < H:
        out["oracle_pairs_band"] = out.pop("oracle_pairs")
    oracle.set_threads(1)
    try:
        s1, d1 = _oracle_step(sc, target, one_core_rows)
    finally:
        oracle.set_threads(cores)
    out["one_core"] = {"value": 1.0 / s1, "seconds": s1,
                       "sample": (f"1 thread: full sampling ({d1['sample_s']:.2f} s), chain "
                                  f"({d1['chain_s']:.2f} s), forward+backward of "
                                  f"{one_core_rows} rows ({d1['band_s']:.2f} s) scaled by "
                                  f"{H / one_core_rows:.0f}")}
    small = {}
    for name, scn, tgt in (("tiny_128", scenes.tiny_128(0), scenes.tiny_128_target(0)),
                           ("open_512", scenes.open_512(0), scenes.target_noise(1, 512, 512))):
        st, _ = _oracle_step(scn, tgt.astype(np.float64), scn.height)
        small[name] = {"steps_per_s": 1.0 / st, "seconds": st}
    out["configs"] = small
    out["_gauss"] = det["g"]
    return out


def tile_depth(sc, g):
    """Distinct curves per 16x16 tile (the workload's depth complexity), from
    the oracle: curves contributing to a pixel of the tile, and curves whose
    support box reaches it."""
    import numpy as np

    import oracle
    d = oracle.tile_depth(g, sc.n_curves, sc.width, sc.height, (16, 16))
    return {k: {"mean": float(np.mean(v)), "p99": float(np.percentile(v, 99)),
                "max": int(np.max(v))} for k, v in d.items()}


def learned_init_figure(size=1024, steps=1000, seed=77):
    """Second half of the metric: steps the learned start needs to reach the
    PSNR the uniform random start has after `steps` Adam steps, on one
    synthetic 1024x1024 target, under the learning rates of Sec. 4.1 and under
    the 512x512 workload's (control points 1e-2)."""
    import numpy as np

    from paper_2503_16424_amd import cnn, learned_init
    if not os.path.exists(learned_init.WEIGHTS):
        return None
    print("# learned initialiser: steps-to-PSNR at 1024x1024", file=sys.stderr, flush=True)
    net = cnn.CurveNet()
    with np.load(learned_init.WEIGHTS, allow_pickle=False) as f:
        net.load_state_dict({k: f[k] for k in f.files})
    o = learned_init.evaluate(net, size, steps, seed)
    labels = {"paper_lr": "Sec. 4.1 (control points 2e-4)",
              "ctrl_lr_1e-2": "512x512 workload (control points 1e-2)"}
    out = {"metric": "steps to the random start's PSNR after 1000 steps", "size": size,
           "steps": steps, "target_seed": seed, "propose_ms": o["propose_ms"], "sets": {}}
    for key, lab in labels.items():
        e = o[key]
        out["sets"][key] = {"lr": lab, "random_psnr_1000": e["random"]["psnr_final"],
                            "learned_psnr_initial": e["learned"]["psnr_initial"],
                            "learned_psnr_1000": e["learned"]["psnr_final"],
                            "learned_steps": e["learned"]["steps_to_random_final"],
                            "fraction_of_steps": e["learned"]["fraction_of_steps"]}
    fr = [v["fraction_of_steps"] for v in out["sets"].values()]
    out["fraction_of_steps_worst"] = None if None in fr else max(fr)
    return out


PEAK_BF16_MFMA_TFLOPS = 2500.0


def bench_curvenet(a):
    """One training step of the curve-proposal network (forward, filter and
    input gradients of every layer) on a batch of 32x32 patches, per kernel,
    against the dense BF16 matrix-core peak."""
    import numpy as np
    import torch

    from paper_2503_16424_amd import cnn
    net = cnn.CurveNet(seed=0)
    net.sync_weights()
    rng = np.random.default_rng(0)
    x = torch.as_tensor(rng.uniform(0, 1, (a.batch, 32, 32, 3)).astype(np.float32),
                        device="cuda").to(torch.bfloat16).view(torch.int16)
    dz = torch.as_tensor(rng.standard_normal((a.batch, cnn.OUT)).astype(np.float32),
                         device="cuda")
    for _ in range(a.warmup):
        net.forward(x)
        net.backward(dz)
    torch.cuda.synchronize()
    ds = net._shapes(a.batch)
    rows = []
    for i, d in enumerate(ds):
        M = d.n * d.ho * d.wo
        flops = 2.0 * M * d.k * d.r * d.r * d.c
        acts = net._acts
        y = torch.empty((d.n, d.ho, d.wo, d.k), dtype=torch.int16, device="cuda")
        dy = torch.randn((d.n, d.ho, d.wo, d.k), device="cuda")
        dw = torch.empty(net.params[i][0].shape, device="cuda")
        db = torch.empty(net.params[i][1].shape, device="cuda")
        dx = torch.empty(acts[i].shape, device="cuda")
        w = net._bf[i]
        # layer 0's forward reads the zero-padded input (net._x8) with its own descriptor
        df, xf = net._dsf[i], (net._x8 if i == 0 else acts[i])
        calls = {"fwd": lambda: cnn.conv_fwd(df, xf, w, net.params[i][1], True, y_bf16=y),
                 "bwd_weight": lambda: cnn.conv_bwd_weight(d, dy, acts[i], dw, db),
                 "bwd_data": lambda: cnn.conv_bwd_data(d, dy, w, dx, x_mask=acts[i])}
        for name, fn in calls.items():
            if name == "bwd_data" and i == 0:
                continue
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            fn()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(a.steps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / a.steps
            rows.append({"layer": i, "pass": name, "gemm_mnk": [M, d.k, d.r * d.r * d.c]
                         if name == "fwd" else None, "ms": ms, "tflops": flops / ms / 1e9})
    t0 = time.perf_counter()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.steps):
        net.forward(x)
        net.backward(dz)
    e1.record()
    torch.cuda.synchronize()
    step_ms_eager = e0.elapsed_time(e1) / a.steps
    # the same step recorded once as a graph and replayed: no host gaps
    tg = cnn.TrainGraph(net, x, dz)
    tg.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(a.steps):
        tg.replay()
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / a.steps
    dom = max(rows, key=lambda r: r["ms"])
    out = {"metric": "curve-proposal network training steps/s (forward + backward)",
           "value": 1000.0 / step_ms, "unit": "steps/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": step_ms, "higher_is_better": True,
           "dtype": "bf16 (fp32 accumulate)", "data": "synthetic",
           "config": {"workload": "curvenet-32x32-patches", "batch": a.batch,
                      "launch": "one HIP graph replay per step"},
           "ms_per_step_eager": step_ms_eager,
           "roofline": {"kernel": f"k_igemm layer {dom['layer']} {dom['pass']}", "bound": "mfma",
                        "achieved": dom["tflops"], "peak": PEAK_BF16_MFMA_TFLOPS,
                        "unit": "TFLOP/s", "frac": dom["tflops"] / PEAK_BF16_MFMA_TFLOPS,
                        "traffic": None},
           "kernels": rows}
    print(json.dumps(out), flush=True)
    return 0


def bench_batched(a):
    """64 canvases of uneven size (sides log-uniform 128..1024 px, 256..8192
    open curves, K 16..32): the batched step (one tile space, every stage one
    launch, the whole step one graph replay) against the same 64 canvases run
    one after the other, each with its own launches."""
    import torch

    from paper_2503_16424_amd import bz, scenes
    from paper_2503_16424_amd.autotune import autotune, time_graph
    from paper_2503_16424_amd.graph import StepGraph
    parts = scenes.batched(0)
    ng = sum(p.n_gauss for p in parts)
    npx = sum(p.width * p.height for p in parts)
    print(f"# batched: {len(parts)} canvases, {ng} Gaussians, {npx} px", file=sys.stderr,
          flush=True)
    tgt_np = [scenes.target_noise(1000 + c, p.width, p.height) for c, p in enumerate(parts)]
    import numpy as np
    flat = torch.as_tensor(np.concatenate([t.reshape(-1) for t in tgt_np]), device="cuda")
    tw, th = (int(v) for v in a.tile.split("x"))
    ro = bz.RenderOptions(tile_w=tw, tile_h=th, persistent=a.persistent)
    table = None
    if a.autotune:
        print("# autotuning tile shape and launch form", file=sys.stderr, flush=True)
        ro, table = autotune(parts, flat, reps=5,
                             log=lambda m: print("#" + m, file=sys.stderr, flush=True))
    r = bz.Rasterizer(parts, ro)
    g = StepGraph(r, flat, warmup=a.warmup)
    for _ in range(a.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_graph_events = time_graph(g, a.steps)
    wall_batched = (time.perf_counter() - t0) * 1000.0 / (a.steps + 1)
    if g.replay(check=True):
        raise RuntimeError("pair buffer overflowed during the timed steps")
    del g, r
    torch.cuda.empty_cache()
    # the same canvases, one after the other, eager launches
    seq_ro = bz.RenderOptions(tile_w=16, tile_h=16)
    rs = [bz.Rasterizer(p, seq_ro) for p in parts]
    ts = [torch.as_tensor(t, device="cuda") for t in tgt_np]
    for rr in rs:
        rr.render()
        need = rr.pairs_required()
        if need * 1.25 > rr.cap_pairs:
            rr._alloc_pairs(int(need * 1.25) + 1024)
    for _ in range(a.warmup):
        for rr, t in zip(rs, ts):
            rr.step(t)
    torch.cuda.synchronize()
    seq_steps = max(1, a.steps // 2)
    t0 = time.perf_counter()
    for _ in range(seq_steps):
        for rr, t in zip(rs, ts):
            rr.step(t)
    torch.cuda.synchronize()
    wall_seq = (time.perf_counter() - t0) * 1000.0 / seq_steps
    out = {
        "metric": "fwd+bwd steps/s, 64 canvases in one batch (step = every canvas once)",
        "value": 1000.0 / wall_batched,
        "unit": "steps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": wall_batched,
        "ms_per_step_events": ms_graph_events,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched-64-canvases", "canvases": len(parts), "gaussians": ng,
                   "pixels": npx, "tile": [ro.tile_w, ro.tile_h],
                   "persistent": bool(ro.persistent), "graph": True,
                   "parallelism": "single GPU"},
        "sequential": {"ms_per_step": wall_seq, "steps_per_s": 1000.0 / wall_seq,
                       "launch": "64 canvases one after the other, 16x16 tiles, eager"},
        "speedup_vs_sequential": wall_seq / wall_batched,
    }
    if table:
        out["autotune"] = [dict(c, ms=round(ms, 4)) for c, ms in table]
    print(json.dumps(out), flush=True)
    return 0


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        return 2
    if a.workload == "batched_64":
        return bench_batched(a)
    if a.workload == "curvenet":
        return bench_curvenet(a)
    import numpy as np
    import torch

    from paper_2503_16424_amd import bz, scenes
    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tw, th = (int(v) for v in a.tile.split("x"))
    if a.workload == "paper_2048":
        sc, target = scenes.paper_2048(0), scenes.target_noise(1, 2048, 2048)
    elif a.workload == "paper_2048_e400":
        sc, target = scenes.paper_2048_e400(0), scenes.target_noise(1, 2048, 2048)
    elif a.workload.startswith("paper_analog"):
        # the frame and curve count of the paper's speed comparison (2040x1344,
        # 2,048 open or closed curves): context beside its published timings
        sc = scenes.paper_analog(0, closed=a.workload.endswith("closed"))
        target = scenes.target_noise(1, sc.width, sc.height)
    elif a.workload == "open_512":
        sc, target = scenes.open_512(0), scenes.target_noise(1, 512, 512)
    else:
        sc, target = scenes.tiny_128(0), scenes.tiny_128_target(0)
    print(f"# workload {sc.name}: {sc.n_curves} curves, {sc.n_gauss} Gaussians", file=sys.stderr,
          flush=True)
    ro = bz.RenderOptions(tile_w=tw, tile_h=th, persistent=a.persistent)
    r = bz.Rasterizer(sc, ro, device="cuda:0")
    tgt = torch.as_tensor(target, device=dev)
    r.render()                                    # sizes the pair buffer (synchronises)
    need = r.pairs_required()
    # contributing (pixel, Gaussian) pairs, from the stored state's counters
    n_alg = int(r.n_contrib.to(torch.int64).sum().item())
    if a.blend_state == "recompute":
        del r
        torch.cuda.empty_cache()
        r = bz.Rasterizer(sc, ro, device="cuda:0", blend_state="recompute")
    if need * 1.1 > r.cap_pairs:
        r._alloc_pairs(int(need * 1.1) + 1024)
    for _ in range(a.warmup):
        r.step(tgt)
    if a.copy_calibration > 0:
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# calibration copy: {a.copy_calibration} MiB read + {a.copy_calibration} MiB "
              "written", file=sys.stderr, flush=True)
        del src, dst
    torch.cuda.synchronize()
    print(f"# warmup done, {need} pairs", file=sys.stderr, flush=True)

    # the sampler does the binning's counting pass (bz_sample_bin) and the
    # forward writes the L2 loss gradient with the image (bz_render_fwd_l2)
    stages = ["sample_bin", "fwd_l2", "bwd_gauss", "bwd_curves"]
    calls = [r.sample_bin, lambda: r.forward_l2(tgt), r.backward_gauss, r.backward_curves]
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)]
          for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        e = ev[i]
        e[0].record()
        for j, call in enumerate(calls):
            call()
            e[j + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = sum(ev[i][0].elapsed_time(ev[i][-1]) for i in range(a.steps)) / a.steps
    stage_ms = {s: sum(ev[i][j].elapsed_time(ev[i][j + 1]) for i in range(a.steps)) / a.steps
                for j, s in enumerate(stages)}
    ms_per_step = wall * 1000.0 / a.steps
    flags = r.flags()
    if flags & bz.STATUS_OVERFLOW:
        raise RuntimeError("pair buffer overflowed during the timed steps")
    loss = float(r.loss.item()) / (3 * sc.width * sc.height)
    print(f"# {a.steps} steps: {ms_per_step:.3f} ms/step wall, {gpu_ms:.3f} ms/step events; "
          f"stages {json.dumps({k: round(v, 4) for k, v in stage_ms.items()})}; "
          f"contributing pairs {n_alg}; mse {loss:.5f}", file=sys.stderr, flush=True)

    # Rate probes: the sustained HBM copy rate, FP32 FMA rate and the issue
    # cost of the transcendentals, measured on this device.
    peaks = None
    if not a.no_peaks:
        from paper_2503_16424_amd import peaks as peak_probes
        peaks = peak_probes.measure()
        print(f"# rate probes: {json.dumps({k: round(v, 4) for k, v in peaks.items()})}",
              file=sys.stderr, flush=True)
    trans = peaks["exp2_fma_slots"] if peaks else TRANS_SLOTS_DEFAULT
    hw = sc.width * sc.height
    bases = {"published": (PEAK_HBM_GBS, PEAK_FP32_TFLOPS * 1e12 / 2),
             "nonpacked": (PEAK_HBM_GBS, PEAK_FP32_VALU_TFLOPS * 1e12 / 2)}
    if peaks:
        bases["measured"] = (peaks["copy_GBs"], peaks["fma_TFLOPs"] * 1e12 / 2)
    step_roof = {}
    for basis, (bw, lanes) in bases.items():
        st = stage_rooflines(stage_ms, sc.n_gauss, need, n_alg, r.n_tiles, hw, trans, bw, lanes)
        step_roof[basis] = {"step_frac": sum(v["roof_ms"] for v in st.values()) / ms_per_step,
                            "stages": {k: {"roof_ms": round(v["roof_ms"], 4), "bound": v["bound"],
                                           "frac": v["roof_ms"] / v["ms"]}
                                       for k, v in st.items()}}

    # Roofline of the dominant stage's kernel, against the published FP32
    # vector peak (and, beside it, the non-packed and measured rates).
    dom = max(("fwd_l2", "bwd_gauss", "bwd_curves", "sample_bin"), key=lambda s: stage_ms[s])
    if dom in ("fwd_l2", "bwd_gauss"):
        flops = FLOPS_FWD_PAIR if dom == "fwd_l2" else FLOPS_BWD_PAIR
        ach = n_alg * flops / (stage_ms[dom] * 1e-3) / 1e12
        kern = ("k_fwd_l2 (bz_render_fwd_l2)" if dom == "fwd_l2" else
                "k_bwd_tiles (bz_render_bwd_gauss, with its d_gauss clear)")
        roof = dict(kernel=kern, bound="alu", achieved=ach, peak=PEAK_FP32_TFLOPS, unit="TFLOP/s")
        roof["frac_nonpacked"] = ach / PEAK_FP32_VALU_TFLOPS
        if peaks:
            roof["frac_measured"] = ach / peaks["fma_TFLOPs"]
    elif dom == "bwd_curves":
        byts = sc.n_gauss * 36
        ach = byts / (stage_ms["bwd_curves"] * 1e-3) / 1e9
        roof = dict(kernel="k_bwd_curves", bound="hbm", achieved=ach, peak=PEAK_HBM_GBS,
                    unit="GB/s")
    else:
        byts = sc.n_gauss * BYTES_REC + need * 4 + r.n_tiles * 8
        ach = byts / (stage_ms["sample_bin"] * 1e-3) / 1e9
        roof = dict(kernel="bz_sample_bin", bound="hbm", achieved=ach, peak=PEAK_HBM_GBS,
                    unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(roof["kernel"].split()[0], a.workload, tw, th)
    roof["step_frac"] = step_roof["published"]["step_frac"]
    roof["step"] = step_roof
    roof["transcendental_slots"] = trans

    out = {
        "metric": METRIC,
        "value": 1000.0 / ms_per_step,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": sc.name, "canvas": [sc.width, sc.height],
                   "curves": sc.n_curves, "gaussians": sc.n_gauss, "seed": 0,
                   "tile": [tw, th], "blend_state": a.blend_state,
                   "persistent": bool(a.persistent),
                   "parallelism": "single GPU"},
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "pairs": {"tile_pairs": need, "contributing": n_alg},
        "roofline": roof,
    }
    if peaks:
        out["peaks_measured"] = peaks
    if not a.no_learned_init and a.workload == "paper_2048":
        out["learned_init"] = learned_init_figure()
    if not a.no_cpu_baseline:
        print("# timing the CPU oracle baseline", file=sys.stderr, flush=True)
        cb = cpu_baseline(sc, target.astype(np.float64), a.cpu_rows)
        g = cb.pop("_gauss")
        if "oracle_pairs" in cb:
            out["pairs"]["contributing_oracle"] = cb["oracle_pairs"]
        out["cpu_baseline"] = cb
        print("# per-tile depth (oracle)", file=sys.stderr, flush=True)
        out["config"]["tile_depth"] = tile_depth(sc, g)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
