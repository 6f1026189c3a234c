"""Differentiation and optimisation on top of libbz (Sec. 3.5).

* :class:`BzRender` -- a ``torch.autograd.Function``: curve parameters in,
  image out; its backward runs ``bz_render_bwd`` on the incoming image
  gradient, so any torch loss can sit on top of the rasterizer.
* :func:`fit` -- the image-vectorisation loop of Sec. 3.5 / Sec. 4.1: a
  gradient optimiser (Adam by default) on control points, colours, opacities
  and stroke widths against the mean squared error.  Each step is sample + bin
  + forward + L2 gradient + backward in libbz; torch supplies the optimiser
  update and device memory.

Control points are optimised in the normalised coordinates [-1, 1]^2 of the
canvas (x_n = 2 x / W - 1, the coordinates of the paper's SVG export), to
which the control-point learning rate refers; the chain factor W/2 (H/2) is
applied to the pixel-space gradient.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import bz


class BzRender(torch.autograd.Function):
    """image [3, H, W] = render(ctrl, stroke_w, color, opacity) through ``rast``.

    ``BzRender.apply(rast, ctrl, stroke_w, color, opacity)``: the four tensors
    (shapes of ``rast.ctrl`` etc.) are copied into the rasterizer's curve
    buffers, the scene is sampled, binned (growing the pair buffer when it
    overflows) and blended.  The backward returns the gradients of all four;
    the draw order, kinds, segment and sample counts stay those of ``rast``.
    The returned image is a fresh tensor; one rasterizer serves one graph at a
    time (its blend state is kept for the backward).
    """

    @staticmethod
    def forward(ctx, rast, ctrl, stroke_w, color, opacity):
        rast.set_params(ctrl=ctrl, stroke_w=stroke_w, color=color, opacity=opacity)
        img = rast.render()
        ctx.rast = rast
        return img.clone()

    @staticmethod
    def backward(ctx, grad_img):
        rast = ctx.rast
        rast.backward(grad_img.contiguous())
        return (None, rast.d_ctrl.clone(), rast.d_width.clone(), rast.d_color.clone(),
                rast.d_opacity.clone())


def psnr_from_mse(mse: float) -> float:
    """Peak signal-to-noise ratio of images in [0, 1]."""
    return float("inf") if mse <= 0 else 10.0 * math.log10(1.0 / mse)


@dataclass
class FitConfig:
    steps: int = 500
    optimizer: str = "adam"     # "adam" or "sgd"
    momentum: float = 0.0       # sgd only
    lr_ctrl: float = 1e-2       # normalised coordinates
    lr_color: float = 1e-2      # Sec. 4.1
    lr_opacity: float = 1e-1    # Sec. 4.1
    lr_width: float = 1e-2      # px (the paper states none)
    min_width: float = 0.5      # px
    log_every: int = 50         # PSNR / timing samples
    check_every: int = 10       # pair-buffer overflow checks (each one synchronises)
    xing_weight: float = 0.0    # weight of the Xing loss (Sec. 3.5) on closed curves


# Learning rates of Sec. 4.1 (control points 2e-4 in the normalised
# coordinates, colours 1e-2, opacities 1e-1; the width's is not stated).
PAPER_LR = dict(lr_ctrl=2e-4, lr_color=1e-2, lr_opacity=1e-1, lr_width=1e-2)


@dataclass
class FitResult:
    psnr: list = field(default_factory=list)        # (step, PSNR of that step's render)
    fwd_ms: list = field(default_factory=list)      # sample + bin + forward with the L2 gradient
    bwd_ms: list = field(default_factory=list)      # backward (and Xing loss), per logged step
    opt_ms: list = field(default_factory=list)      # optimiser update, per logged step
    step_ms: float = 0.0                            # wall clock per step over the loop
    final_psnr: float = 0.0
    regrown: int = 0                                # pair-buffer growths during the loop


class Fitter:
    """Parameters, optimiser and rasterizer of one optimisation."""

    def __init__(self, rast: "bz.Rasterizer", cfg: FitConfig | None = None):
        self.rast, self.cfg = rast, cfg or FitConfig()
        self.half = torch.tensor([rast.W / 2.0, rast.H / 2.0], device=rast.dev)
        self.ctrl_n = torch.nn.Parameter(rast.ctrl / self.half - 1.0)
        self.color = torch.nn.Parameter(rast.color.clone())
        self.opacity = torch.nn.Parameter(rast.opacity.clone())
        self.width = torch.nn.Parameter(rast.stroke_w.clone())
        c = self.cfg
        groups = [{"params": [self.ctrl_n], "lr": c.lr_ctrl},
                  {"params": [self.color], "lr": c.lr_color},
                  {"params": [self.opacity], "lr": c.lr_opacity},
                  {"params": [self.width], "lr": c.lr_width}]
        if c.optimizer == "adam":
            self.opt = torch.optim.Adam(groups)
        elif c.optimizer == "sgd":
            self.opt = torch.optim.SGD(groups, momentum=c.momentum)
        else:
            raise ValueError(f"unknown optimizer {c.optimizer!r}")

    def push(self):
        """Parameters -> the rasterizer's curve buffers."""
        with torch.no_grad():
            self.rast.set_params(ctrl=(self.ctrl_n + 1.0) * self.half, color=self.color,
                                 opacity=self.opacity, stroke_w=self.width)

    def update(self):
        """One optimiser step from the rasterizer's last backward, then the
        box constraints (colours and opacities in [0, 1], widths >= min)."""
        r = self.rast
        self.ctrl_n.grad = r.d_ctrl * self.half
        self.color.grad = r.d_color.clone()
        self.opacity.grad = r.d_opacity.clone()
        self.width.grad = r.d_width.clone()
        self.opt.step()
        with torch.no_grad():
            self.color.clamp_(0.0, 1.0)
            self.opacity.clamp_(0.0, 1.0)
            self.width.clamp_(min=self.cfg.min_width)

    def state_arrays(self, step: int) -> dict:
        """Everything a resumed run needs, as host arrays: the step reached,
        the parameters (control points in normalised coordinates), the
        optimiser's per-parameter state (Adam moments and step counts) and the
        torch random generators' states."""
        out = {"step": np.array(step, np.int64),
               "ctrl_n": self.ctrl_n.detach().cpu().numpy(),
               "color": self.color.detach().cpu().numpy(),
               "opacity": self.opacity.detach().cpu().numpy(),
               "width": self.width.detach().cpu().numpy(),
               "rng_cpu": torch.get_rng_state().numpy()}
        if torch.cuda.is_available():
            out["rng_cuda"] = torch.cuda.get_rng_state().numpy()
        out.update(optimizer_state_arrays(self.opt))
        return out

    def load_state_arrays(self, a: dict) -> int:
        """Restore what state_arrays saved (shapes must match); returns its step."""
        with torch.no_grad():
            for name in ("ctrl_n", "color", "opacity", "width"):
                p = getattr(self, name)
                src = torch.as_tensor(np.asarray(a[name]), device=p.device)
                if src.shape != p.shape:
                    raise ValueError(f"checkpoint {name} has shape {tuple(src.shape)}, "
                                     f"the optimisation {tuple(p.shape)}")
                p.copy_(src)
        load_optimizer_state(self.opt, a)
        torch.set_rng_state(torch.as_tensor(np.asarray(a["rng_cpu"]), dtype=torch.uint8))
        if "rng_cuda" in a and torch.cuda.is_available():
            torch.cuda.set_rng_state(torch.as_tensor(np.asarray(a["rng_cuda"]), dtype=torch.uint8))
        return int(a["step"])

    def params_host(self) -> dict:
        """Current parameters in the rasterizer's units (px for points)."""
        with torch.no_grad():
            return dict(ctrl=((self.ctrl_n + 1.0) * self.half).cpu().numpy(),
                        color=self.color.cpu().numpy(), opacity=self.opacity.cpu().numpy(),
                        stroke_w=self.width.cpu().numpy())


def optimizer_state_arrays(opt) -> dict:
    """A torch optimiser's per-parameter state as host arrays keyed
    ``opt_<group>_<param>_<name>`` (tensors only; Adam: step, exp_avg,
    exp_avg_sq)."""
    out = {}
    for gi, group in enumerate(opt.param_groups):
        for pi, p in enumerate(group["params"]):
            for k, v in opt.state.get(p, {}).items():
                if torch.is_tensor(v):
                    out[f"opt_{gi}_{pi}_{k}"] = v.detach().cpu().numpy()
    return out


def load_optimizer_state(opt, a: dict) -> None:
    """Inverse of optimizer_state_arrays for the same parameter layout (state
    tensors go back to the device and dtype torch keeps them on: a step count
    stays where the optimiser creates it, on the host)."""
    for gi, group in enumerate(opt.param_groups):
        for pi, p in enumerate(group["params"]):
            pre = f"opt_{gi}_{pi}_"
            keys = [k for k in a if k.startswith(pre)]
            if not keys:
                opt.state.pop(p, None)
                continue
            st = {}
            for k in keys:
                name = k[len(pre):]
                v = torch.as_tensor(np.asarray(a[k]))
                st[name] = v if name == "step" else v.to(p.device)
            opt.state[p] = st


def save_checkpoint(path: str, fitter: "Fitter", step: int) -> None:
    """Write fitter.state_arrays(step) to ``path`` (.npz, plain arrays only)."""
    np.savez(path, **fitter.state_arrays(step))


def load_checkpoint(path: str) -> dict:
    """Read a checkpoint written by save_checkpoint (no pickled objects)."""
    with np.load(path, allow_pickle=False) as f:
        return {k: f[k] for k in f.files}


def fit(rast: "bz.Rasterizer", target, cfg: FitConfig | None = None, callback=None,
        checkpoint_path: str | None = None, checkpoint_every: int = 0,
        resume_from: str | None = None) -> FitResult:
    """Optimise the curve parameters of ``rast`` against ``target`` ([3, H, W]
    float32 on the device) for ``cfg.steps`` steps; the rasterizer ends up
    holding the optimised parameters.

    The pair buffer is checked for overflow every ``check_every`` steps (and
    on logged steps); a step whose binning overflowed is binned again with the
    grown buffer before its gradient is used.  A step that overflows between
    checks yields zero gradients (libbz skips blending on overflow).

    Checkpoints: with ``checkpoint_path`` and ``checkpoint_every`` > 0 the
    parameters, optimiser moments and random-generator states are written
    there (.npz) after every ``checkpoint_every``-th step; ``resume_from``
    restores such a file and continues from the step it reached, so a run
    interrupted and resumed takes the same steps as an uninterrupted one."""
    f = Fitter(rast, cfg)
    cfg = f.cfg
    start = 0
    if resume_from is not None:
        start = f.load_state_arrays(load_checkpoint(resume_from))
    res = FitResult()
    n = 3 * rast.W * rast.H
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(start, cfg.steps):
        f.push()
        logged = step % cfg.log_every == 0 or step == cfg.steps - 1
        if logged:
            ev[0].record()
        rast.sample_bin()
        if (logged or step % cfg.check_every == 0) and rast.ensure_capacity():
            res.regrown += 1
            rast.bin()
        rast.forward_l2(target)
        if logged:
            ev[1].record()
        rast.backward()
        if cfg.xing_weight > 0.0:
            rast.xing(cfg.xing_weight)          # L = mean squared error + weight * Xing
        if logged:
            ev[2].record()
        f.update()
        if logged:
            ev[3].record()
            res.psnr.append((step, psnr_from_mse(float(rast.loss.item()) / n)))
            res.fwd_ms.append(ev[0].elapsed_time(ev[1]))
            res.bwd_ms.append(ev[1].elapsed_time(ev[2]))
            res.opt_ms.append(ev[2].elapsed_time(ev[3]))
            if callback:
                callback(step, res.psnr[-1][1])
        if checkpoint_path and checkpoint_every > 0 and (step + 1) % checkpoint_every == 0:
            save_checkpoint(checkpoint_path, f, step + 1)
    torch.cuda.synchronize()
    res.step_ms = (time.perf_counter() - t0) * 1000.0 / max(cfg.steps - start, 1)
    f.push()
    rast.render()
    rast.l2_grad(target)
    res.final_psnr = psnr_from_mse(float(rast.loss.item()) / n)
    return res


def noisy_target(clean, seed_noise: int = 2, sigma: float = 0.02):
    """Optimisation target of the 512x512 workload: a clean render of the hidden
    curve set plus N(0, sigma^2) noise, clipped to [0, 1] ([3, H, W] float32)."""
    from . import scenes
    c = np.asarray(clean, np.float64)
    return np.clip(c + scenes.gaussian_noise(seed_noise, c.shape, sigma), 0.0, 1.0).astype(np.float32)
