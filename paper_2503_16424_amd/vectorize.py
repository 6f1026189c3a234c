"""Image vectorisation with the libbz rasterizer (Sec. 3.5, Sec. 4.1).

``python -m paper_2503_16424_amd.vectorize [--steps 500] [--out result.json]``

The 512x512 workload: 2,048 open single-segment cubic curves x 32 samples
(65,536 Gaussians, seed 0) fitted by Adam to a target made of a hidden
4,096-curve scene (seed 1), rendered by libbz and overlaid with N(0, 0.02^2)
noise (seed 2), clipped to [0, 1].  Prints one JSON line per logged step
(PSNR, per-step forward / backward / optimiser milliseconds) and a summary
line; ``--out`` also writes the summary with the whole trajectory.
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--log-every", type=int, default=25)
    ap.add_argument("--optimizer", default="adam", choices=["adam", "sgd"])
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--hidden-seed", type=int, default=1)
    ap.add_argument("--noise-seed", type=int, default=2)
    ap.add_argument("--sigma", type=float, default=0.02)
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    import torch
    from . import bz, scenes
    from .optim import FitConfig, fit, noisy_target, psnr_from_mse

    tw, th = (int(v) for v in a.tile.split("x"))
    ro = bz.RenderOptions(tile_w=tw, tile_h=th)
    hidden = scenes.hidden_512(a.hidden_seed)
    clean = bz.Rasterizer(hidden, ro).render().cpu().numpy()
    tgt_np = noisy_target(clean, a.noise_seed, a.sigma)
    noise_floor = psnr_from_mse(float(np.mean((tgt_np.astype(np.float64) - clean) ** 2)))
    target = torch.as_tensor(tgt_np, device="cuda")

    init = scenes.open_512(a.init_seed)
    rast = bz.Rasterizer(init, ro)
    cfg = FitConfig(steps=a.steps, optimizer=a.optimizer, log_every=a.log_every)

    def log(step, p):
        print(json.dumps({"step": step, "psnr": round(p, 4)}), flush=True)

    res = fit(rast, target, cfg, callback=log)
    med = lambda xs: statistics.median(xs) if xs else None
    summary = {
        "workload": "open-512x512-2048c-K32 fitted to hidden-512x512-4096c-K32 + noise",
        "n_gauss": int(rast.n_gauss), "steps": a.steps, "optimizer": a.optimizer,
        "lr": {"ctrl_normalised": cfg.lr_ctrl, "color": cfg.lr_color,
               "opacity": cfg.lr_opacity, "width_px": cfg.lr_width},
        "psnr_initial": res.psnr[0][1] if res.psnr else None,
        "psnr_final": res.final_psnr,
        "psnr_clean_vs_target": noise_floor,
        "fwd_ms_median": med(res.fwd_ms), "bwd_ms_median": med(res.bwd_ms),
        "opt_ms_median": med(res.opt_ms), "step_ms_wall": res.step_ms,
        "pair_buffer_regrown": res.regrown, "tile": a.tile,
    }
    print(json.dumps(summary), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(dict(summary, trajectory=res.psnr, fwd_ms=res.fwd_ms, bwd_ms=res.bwd_ms,
                           opt_ms=res.opt_ms), fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
