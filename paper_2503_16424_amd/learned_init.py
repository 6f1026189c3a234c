"""Learned curve initialiser: training data from the plain optimiser, training
of the curve-proposal network on the GPU, and steps-to-PSNR evaluation.

The plain method starts from random curves and optimises them (Sec. 3.5).
Here a network proposes the initial curves instead, patch by patch:

1. data:  seeded synthetic 512x512 targets (hidden scenes of 4,096 open
   strokes rendered by libbz, plus N(0, 0.02^2) noise).  Each is fitted by the
   plain optimiser from the deterministic per-patch initialisation
   (:func:`scenes.grid_init`: 8 curves in fixed slots of every 32x32 patch),
   and every patch gives one pair (target patch, its 8 optimised curves in
   slot order): 256 pairs per target.
2. train: :class:`cnn.CurveNet` regresses the normalised curve parameters of
   the pairs (mean squared error on control points in patch sides, widths,
   colours and opacities), Adam on FP32 weights, forward and backward in
   libbz's BF16 matrix-core kernels.
3. eval:  on seeded 1024x1024 targets, the plain optimiser runs from the
   uniform random initialisation and from the network's proposal; the
   figure of merit is the number of steps the learned start needs to reach
   the PSNR the random start has after ``steps`` steps.

``python -m paper_2503_16424_amd.learned_init all --out DIR`` runs the three.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "curvenet.npz")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def synthetic_target(seed: int, W: int, H: int, density: float = 4096 / (512 * 512),
                     sigma: float = 0.02):
    """A hidden scene of open strokes (K = 32) at the given density, rendered by
    libbz, plus N(0, sigma^2) noise, clipped: float32 [3, H, W] (host)."""
    from . import bz, scenes
    from .optim import noisy_target
    n = max(1, int(round(density * W * H)))
    hidden = scenes.uniform_open(seed, W, H, n, 32)
    clean = bz.Rasterizer(hidden).render().cpu().numpy()
    return noisy_target(clean, seed + 7919, sigma)


def make_pairs(n_canvas: int = 40, fit_steps: int = 600, seed0: int = 1000, size: int = 512,
               side: int = 32, lr_ctrl: float = 2e-3):
    """(patches [N, side, side, 3] float32, labels [N, 8, 13] normalised)."""
    import torch
    from . import bz, cnn, scenes
    from .optim import FitConfig, fit
    xs, ys = [], []
    for t in range(n_canvas):
        t0 = time.perf_counter()
        tgt = synthetic_target(seed0 + t, size, size)
        r = bz.Rasterizer(scenes.grid_init(size, size, side, cnn.CURVES))
        res = fit(r, torch.as_tensor(tgt, device="cuda"), FitConfig(steps=fit_steps, log_every=fit_steps,
                                                                   lr_ctrl=lr_ctrl))
        org = scenes.patch_origins(size, size, side)
        lab = cnn.normalise(r.ctrl.cpu().numpy(), r.stroke_w.cpu().numpy(), r.color.cpu().numpy(),
                            r.opacity.cpu().numpy(), org.astype(np.float64), side)
        hw = tgt.transpose(1, 2, 0)
        for (x0, y0) in org:
            xs.append(hw[y0: y0 + side, x0: x0 + side])
        ys.append(lab)
        _log(f"  target {t}: fitted {fit_steps} steps to {res.final_psnr:.2f} dB "
             f"({time.perf_counter() - t0:.1f} s)")
    return np.stack(xs).astype(np.float32), np.concatenate(ys).astype(np.float32)


LOSS_W = np.array([1.0] * 8 + [0.5] + [1.0] * 3 + [0.5], np.float32)


def train(patches, labels, epochs: int = 40, batch: int = 256, lr: float = 1e-3, seed: int = 0,
          log_every: int = 5, render_epochs: int = 0, param_weight: float = 0.5):
    """Train a CurveNet on (patch, curves) pairs; returns (net, loss history).

    Phase 1 (``epochs``): regression of the normalised curve parameters.
    Phase 2 (``render_epochs``): the proposed curves of every patch of a batch
    are rendered by libbz (the batch's patches as one batch of 32x32
    canvases) and compared with the patch itself; the image error's gradient
    reaches the network through the rasterizer's backward, plus
    ``param_weight`` times the regression term."""
    import torch
    from . import cnn
    dev = torch.device("cuda")
    net = cnn.CurveNet(seed=seed)
    opt = torch.optim.Adam(net.tensors(), lr=lr)
    n = patches.shape[0]
    xb = torch.as_tensor(patches, device=dev).to(torch.bfloat16).view(torch.int16)
    yt = torch.as_tensor(labels, device=dev)
    lw = torch.as_tensor(LOSS_W, device=dev)
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    steps = epochs * math.ceil(n / batch)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, steps)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(dev)
        tot, cnt = 0.0, 0
        for i in range(0, n, batch):
            idx = perm[i: i + batch]
            net.sync_weights()
            z = net.forward(xb[idx].contiguous())
            z.requires_grad_(True)
            u = cnn.decode(z)
            loss = (((u - yt[idx]) ** 2) * lw).mean()
            loss.backward()
            net.backward(z.grad)
            opt.step()
            sched.step()
            tot += float(loss.detach()) * idx.numel()
            cnt += idx.numel()
        hist.append(tot / cnt)
        if ep % log_every == 0 or ep == epochs - 1:
            _log(f"  epoch {ep}: loss {hist[-1]:.5f}")
    if render_epochs > 0:
        hist += _train_render(net, patches, labels, render_epochs, batch, lr * 0.5, g,
                              param_weight, log_every)
    net.sync_weights()
    return net, hist


def _train_render(net, patches, labels, epochs, batch, lr, g, param_weight, log_every):
    import torch
    from . import bz, cnn, scenes
    from .optim import BzRender
    dev = torch.device("cuda")
    side = patches.shape[1]
    n = (patches.shape[0] // batch) * batch
    canvases = [scenes.open_curves(side, side, np.zeros((cnn.CURVES, 4, 2)),
                                   np.ones(cnn.CURVES), np.zeros((cnn.CURVES, 3)),
                                   np.ones(cnn.CURVES), 16) for _ in range(batch)]
    rast = bz.Rasterizer(canvases)
    xb = torch.as_tensor(patches, device=dev).to(torch.bfloat16).view(torch.int16)
    # the rasterizer's flat layout: canvas after canvas, planar [3][side][side]
    tgt = torch.as_tensor(patches.transpose(0, 3, 1, 2).copy(), device=dev)
    yt = torch.as_tensor(labels, device=dev)
    lw = torch.as_tensor(LOSS_W, device=dev)
    zero = torch.zeros((batch, 2), device=dev)
    opt = torch.optim.Adam(net.tensors(), lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, epochs * (n // batch))
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(patches.shape[0], generator=g)[:n].to(dev)
        tot = 0.0
        for i in range(0, n, batch):
            idx = perm[i: i + batch]
            net.sync_weights()
            z = net.forward(xb[idx].contiguous())
            z.requires_grad_(True)
            u = cnn.decode(z)
            ctrl, w, col, opa = cnn.to_curves(u, zero, side)
            img = BzRender.apply(rast, ctrl.reshape(-1, 2), w, col, opa)
            loss = ((img - tgt[idx].reshape(-1)) ** 2).mean()
            if param_weight > 0:
                loss = loss + param_weight * (((u - yt[idx]) ** 2) * lw).mean()
            loss.backward()
            net.backward(z.grad)
            opt.step()
            sched.step()
            tot += float(loss.detach())
        hist.append(tot / (n // batch))
        if ep % log_every == 0 or ep == epochs - 1:
            _log(f"  render epoch {ep}: loss {hist[-1]:.5f}")
    return hist


def propose(net, target, side: int = 32):
    """The network's curves for every patch of ``target`` ([3, H, W] float32 on
    the device): a scene of open curves (8 per patch, K = 16)."""
    import torch
    from . import cnn, scenes
    H, W = target.shape[1], target.shape[2]
    org = scenes.patch_origins(W, H, side)
    xy = torch.as_tensor(org, device=target.device)
    pt = torch.empty((org.shape[0], side, side, 3), dtype=torch.int16, device=target.device)
    cnn.extract_patches(target, xy, side, 1.0, pt)
    with torch.no_grad():
        z = net.forward(pt)
        u = cnn.decode(z)
        ctrl, w, col, opa = cnn.to_curves(u, torch.as_tensor(org, dtype=torch.float32,
                                                             device=target.device), side)
    return scenes.open_curves(W, H, ctrl.cpu().numpy(), w.cpu().numpy(), col.cpu().numpy(),
                              opa.cpu().numpy(), 16, name=f"learned-init-{W}x{H}")


def run_fit(scene, target, steps: int, log_every: int = 10, lrs=None):
    from . import bz
    from .optim import FitConfig, fit
    r = bz.Rasterizer(scene)
    res = fit(r, target, FitConfig(steps=steps, log_every=log_every, **(lrs or {})))
    return res


def steps_to_reach(traj, final_psnr, steps, level):
    """First step whose render reaches ``level`` (the trajectory holds the PSNR
    of the render each logged step optimises; after the last step the final
    render counts as ``steps``)."""
    for s, p in traj:
        if p >= level:
            return s
    return steps if final_psnr >= level else None


def lr_sets():
    """Optimiser settings the evaluation runs under: the learning rates of
    Sec. 4.1 (control points 2e-4), and those of the 512x512 workload
    (control points 1e-2)."""
    from .optim import PAPER_LR
    return {"paper_lr": dict(PAPER_LR), "ctrl_lr_1e-2": {}}


def evaluate(net, size: int = 1024, steps: int = 1000, seed: int = 77, log_every: int = 10,
             sets=None):
    """Steps-to-PSNR of the learned start against the uniform random one (and
    the deterministic grid start) on one synthetic target, under each
    optimiser setting of ``sets`` (default :func:`lr_sets`)."""
    import torch
    from . import scenes
    tgt = torch.as_tensor(synthetic_target(seed, size, size), device="cuda")
    out = {"size": size, "steps": steps, "target_seed": seed}
    t0 = time.perf_counter()
    learned = propose(net, tgt)
    torch.cuda.synchronize()
    out["propose_ms"] = (time.perf_counter() - t0) * 1000.0
    runs = {"random": scenes.random_init(seed + 1, size, size), "grid": scenes.grid_init(size, size),
            "learned": learned}
    for sname, lrs in (sets or lr_sets()).items():
        o = {}
        for name, sc in runs.items():
            res = run_fit(sc, tgt, steps, log_every, lrs)
            o[name] = {"psnr_initial": res.psnr[0][1], "psnr_final": res.final_psnr,
                       "trajectory": res.psnr, "step_ms": res.step_ms}
            _log(f"  [{sname}] {name}: {res.psnr[0][1]:.2f} -> {res.final_psnr:.2f} dB in "
                 f"{steps} steps")
        level = o["random"]["psnr_final"]
        for name in ("learned", "grid"):
            k = steps_to_reach(o[name]["trajectory"], o[name]["psnr_final"], steps, level)
            o[name]["steps_to_random_final"] = k
            o[name]["fraction_of_steps"] = None if k is None else k / steps
        out[sname] = o
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="learned curve initialiser")
    ap.add_argument("cmd", choices=["all", "eval"])
    ap.add_argument("--canvases", type=int, default=320)
    ap.add_argument("--fit-steps", type=int, default=600)
    ap.add_argument("--epochs", type=int, default=80)
    ap.add_argument("--render-epochs", type=int, default=60)
    ap.add_argument("--eval-size", type=int, default=1024)
    ap.add_argument("--eval-steps", type=int, default=1000)
    ap.add_argument("--eval-seeds", default="77,78,79")
    ap.add_argument("--weights", default=WEIGHTS)
    ap.add_argument("--out", default=None, help="directory for the result JSON (and weights)")
    a = ap.parse_args(argv)
    from . import cnn
    res = {}
    if a.cmd == "all":
        t0 = time.perf_counter()
        _log(f"# data: {a.canvases} targets x 256 patches, {a.fit_steps} fit steps each")
        X, Y = make_pairs(a.canvases, a.fit_steps)
        res["data_s"] = time.perf_counter() - t0
        res["pairs"] = int(X.shape[0])
        t0 = time.perf_counter()
        _log(f"# train: {a.epochs} epochs")
        net, hist = train(X, Y, a.epochs, render_epochs=a.render_epochs)
        res["train_s"] = time.perf_counter() - t0
        res["loss_history"] = hist
        wpath = os.path.join(a.out, "curvenet.npz") if a.out else a.weights
        os.makedirs(os.path.dirname(wpath), exist_ok=True)
        np.savez(wpath, **net.state_dict())
        res["weights"] = wpath
    else:
        net = cnn.CurveNet()
        with np.load(a.weights, allow_pickle=False) as f:
            net.load_state_dict({k: f[k] for k in f.files})
    res["eval"] = []
    for s in [int(v) for v in a.eval_seeds.split(",")]:
        _log(f"# eval at {a.eval_size}x{a.eval_size}, target seed {s}")
        res["eval"].append(evaluate(net, a.eval_size, a.eval_steps, s))
    summary = {k: v for k, v in res.items() if k not in ("eval", "loss_history")}
    def strip(v):
        if isinstance(v, dict):
            return {kk: strip(vv) for kk, vv in v.items() if kk != "trajectory"}
        return v
    summary["eval"] = [strip(e) for e in res["eval"]]
    print(json.dumps(summary), flush=True)
    if a.out:
        os.makedirs(a.out, exist_ok=True)
        with open(os.path.join(a.out, "learned_init.json"), "w") as fh:
            json.dump(res, fh)
    return 0


if __name__ == "__main__":
    sys.exit(main())
