"""The rasterizer behind torch autograd and inside the optimisation loop.

* BzRender's gradients equal the oracle's for an arbitrary torch loss;
* they match central finite differences of the HIP forward itself;
* a short gradient-descent run through the loop follows the trajectory that
  the oracle's gradients give, step by step;
* Adam raises the PSNR, also when the pair buffer has to grow in the loop.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2503_16424_amd import scenes
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3


def _note(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return torch


def _params(torch, r):
    return [r.ctrl.clone().requires_grad_(), r.stroke_w.clone().requires_grad_(),
            r.color.clone().requires_grad_(), r.opacity.clone().requires_grad_()]


SCENES = {
    "tiny_128": lambda: scenes.tiny_128(0),
    "mixed_small_b": lambda: scenes.small_mixed(2, W=131, H=77, n_closed=9, n_open=12, K=12,
                                                R=6, extent=(4.0, 60.0)),
}


@pytest.mark.parametrize("name", list(SCENES))
def test_autograd_function_matches_oracle_gradient(torch_cuda, name):
    """loss = sum(w * image) + mean((image - target)^2) through BzRender."""
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    from paper_2503_16424_amd.optim import BzRender
    sc = SCENES[name]()
    _note(f"autograd vs oracle {name}")
    r = bz.Rasterizer(sc)
    wt = np.random.default_rng(5).uniform(-1.0, 1.0, (3, sc.height, sc.width)).astype(np.float32)
    tgt = scenes.target_noise(6, sc.width, sc.height)
    p = _params(torch, r)
    img = BzRender.apply(r, *p)
    loss = (torch.as_tensor(wt, device="cuda") * img).sum() + \
        ((img - torch.as_tensor(tgt, device="cuda")) ** 2).mean()
    loss.backward()
    o0 = oracle.forward_backward(sc)
    d = wt.astype(np.float64) + 2.0 * (o0["image"] - tgt) / o0["image"].size
    o = oracle.forward_backward(sc, d)
    assert np.abs(img.detach().cpu().numpy() - o0["image"]).max() <= 1e-5
    for t, k in zip(p, ("d_ctrl", "d_width", "d_color", "d_opacity")):
        g = t.grad.cpu().numpy().reshape(o[k].shape)
        if k == "d_width" and not np.any(sc.kind == 0):
            continue
        e = rel_l2(g, o[k])
        _note(f"  {k}: rel L2 {e:.2e}")
        assert e <= GRAD_TOL, k


@pytest.mark.parametrize("name", list(SCENES))
def test_autograd_function_matches_finite_differences(torch_cuda, name):
    """Directional central differences of the HIP forward, L = sum(w * image),
    along random directions of each parameter group (and all together)."""
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    from paper_2503_16424_amd.optim import BzRender
    sc = SCENES[name]()
    r = bz.Rasterizer(sc)
    wt = np.random.default_rng(8).uniform(-1.0, 1.0, (3, sc.height, sc.width))
    w_dev = torch.as_tensor(wt.astype(np.float32), device="cuda")
    p = _params(torch, r)
    (w_dev * BzRender.apply(r, *p)).sum().backward()
    grads = [t.grad.double().cpu().numpy().ravel() for t in p]
    base = [t.detach().clone() for t in p]
    rng = np.random.default_rng(9)
    # 1e-3 px: the central difference of a mixed scene is already off by 12%
    # at 1e-2 px (the oracle's own differences agree), curvature of the small
    # closed curves' tangents; the termination threshold leaves a ~1e-3 floor.
    steps = (1e-3, 1e-3, 1e-3, 1e-3)        # px for points and widths; colours, opacities

    def L(vals):
        with torch.no_grad():
            img = BzRender.apply(r, *vals).double().cpu().numpy()
        return float((wt * img).sum())

    groups = [[0], [1], [2], [3], [0, 1, 2, 3]]
    if not np.any(sc.kind == 0):
        groups = [[0], [2], [3], [0, 2, 3]]
    for grp in groups:
        plus, minus, pred = list(base), list(base), 0.0
        for j in grp:
            v = rng.standard_normal(base[j].numel())
            dv = torch.as_tensor((steps[j] * v).reshape(base[j].shape), dtype=torch.float32,
                                 device="cuda")
            plus[j] = base[j] + dv
            minus[j] = base[j] - dv
            if j == 2 or j == 3:                  # stay inside [0, 1]
                plus[j] = plus[j].clamp(0.0, 1.0)
                minus[j] = minus[j].clamp(0.0, 1.0)
            delta = (plus[j].double() - minus[j].double()).cpu().numpy().ravel()
            pred += float(grads[j] @ delta)
        fd = L(plus) - L(minus)
        err = abs(fd - pred) / max(abs(pred), 1e-12)
        _note(f"  group {grp}: fd {fd:.6e} analytic {pred:.6e} rel {err:.2e}")
        assert err <= 2e-2, grp


def _oracle_sgd(sc, tgt, steps, lr, min_width):
    """Plain gradient descent with the oracle's gradients, in the loop's own
    parametrisation (control points in [-1, 1] canvas coordinates)."""
    half = np.array([sc.width / 2.0, sc.height / 2.0])
    s = scenes.Scene(**{k: getattr(sc, k) for k in sc.__dataclass_fields__})
    ctrl_n = sc.ctrl.astype(np.float64).reshape(-1, 2) / half - 1.0
    color = sc.color.astype(np.float64).reshape(-1, 3).copy()
    opac = sc.opacity.astype(np.float64).copy()
    width = sc.stroke_w.astype(np.float64).copy()
    n = 3 * sc.width * sc.height
    for _ in range(steps):
        s.ctrl, s.color, s.opacity, s.stroke_w = (ctrl_n + 1.0) * half, color, opac, width
        img = oracle.forward_backward(s)["image"]
        o = oracle.forward_backward(s, 2.0 * (img - tgt) / n)
        ctrl_n = ctrl_n - lr[0] * o["d_ctrl"] * half
        color = np.clip(color - lr[1] * o["d_color"], 0.0, 1.0)
        opac = np.clip(opac - lr[2] * o["d_opacity"], 0.0, 1.0)
        width = np.maximum(width - lr[3] * o["d_width"], min_width)
    return dict(ctrl=(ctrl_n + 1.0) * half, color=color, opacity=opac, stroke_w=width)


def test_gradient_descent_loop_follows_oracle_trajectory(torch_cuda):
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    from paper_2503_16424_amd.optim import FitConfig, fit
    sc = SCENES["mixed_small_b"]()
    tgt = scenes.target_noise(4, sc.width, sc.height)
    # learning rates that move points by about a pixel per step
    lr = (1.0, 3.0, 5.0, 100.0)
    cfg = FitConfig(steps=4, optimizer="sgd", lr_ctrl=lr[0], lr_color=lr[1], lr_opacity=lr[2],
                    lr_width=lr[3], log_every=1, check_every=1)
    r = bz.Rasterizer(sc)
    init = dict(ctrl=sc.ctrl.astype(np.float64).reshape(-1, 2), color=sc.color.reshape(-1, 3),
                opacity=sc.opacity, stroke_w=sc.stroke_w)
    fit(r, torch.as_tensor(tgt, device="cuda"), cfg)
    got = dict(ctrl=r.ctrl.cpu().numpy(), color=r.color.cpu().numpy(),
               opacity=r.opacity.cpu().numpy(), stroke_w=r.stroke_w.cpu().numpy())
    ref = _oracle_sgd(sc, tgt.astype(np.float64), 4, lr, cfg.min_width)
    moved = np.abs(ref["ctrl"] - init["ctrl"]).max()
    _note(f"  max control-point travel {moved:.3f} px")
    assert 0.2 < moved < 20.0
    for k in ("ctrl", "color", "opacity", "stroke_w"):
        dref = ref[k] - init[k].astype(np.float64).reshape(ref[k].shape)
        dgot = got[k].astype(np.float64).reshape(ref[k].shape) - \
            init[k].astype(np.float64).reshape(ref[k].shape)
        if not np.any(dref):
            assert np.abs(dgot).max() < 1e-6, k
            continue
        e = rel_l2(dgot, dref)
        _note(f"  {k}: rel L2 of the 4-step displacement {e:.2e}")
        assert e <= 3e-3, k


def test_adam_fit_raises_psnr_and_survives_buffer_growth(torch_cuda):
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    from paper_2503_16424_amd.optim import FitConfig, fit
    hidden = scenes.uniform_open(11, 128, 128, 512, 16)
    clean = bz.Rasterizer(hidden).render().cpu().numpy()
    sc = scenes.uniform_open(12, 128, 128, 256, 16)
    r = bz.Rasterizer(sc, cap_pairs=64)          # far too small: the loop must grow it
    res = fit(r, torch.as_tensor(clean, device="cuda"),
              FitConfig(steps=120, log_every=20, check_every=5))
    first = res.psnr[0][1]
    _note(f"  PSNR {first:.2f} -> {res.final_psnr:.2f} dB, buffer grown {res.regrown}x")
    assert res.regrown >= 1
    assert np.isfinite(res.final_psnr)
    assert res.final_psnr > first + 3.0
    assert all(np.isfinite(p) for _, p in res.psnr)


def test_gradient_at_the_512_workload_after_adam_steps(torch_cuda):
    """The 512x512 fit (2,048 strokes x K = 32) after 20 Adam steps on the GPU:
    the image and the four gradient groups at the reached parameters match
    the oracle evaluated at the same parameters."""
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    from paper_2503_16424_amd.optim import FitConfig, fit, noisy_target
    clean = bz.Rasterizer(scenes.hidden_512(1)).render().cpu().numpy()
    tgt = noisy_target(clean, 2, 0.02)
    sc = scenes.open_512(0)
    r = bz.Rasterizer(sc)
    fit(r, torch.as_tensor(tgt, device="cuda"), FitConfig(steps=20, log_every=20))
    s2 = sc.copy()
    s2.ctrl = r.ctrl.cpu().numpy().astype(np.float32)
    s2.color = r.color.cpu().numpy().astype(np.float32)
    s2.opacity = r.opacity.cpu().numpy().astype(np.float32)
    s2.stroke_w = r.stroke_w.cpu().numpy().astype(np.float32)
    img = r.render().cpu().numpy()
    o0 = oracle.forward_backward(s2)
    assert np.abs(img - o0["image"]).max() <= 1e-5
    d = 2.0 * (o0["image"] - tgt.astype(np.float64)) / o0["image"].size
    o = oracle.forward_backward(s2, d)
    r.backward(torch.as_tensor(d.astype(np.float32), device="cuda"))
    torch.cuda.synchronize()
    for k in ("d_ctrl", "d_width", "d_color", "d_opacity"):
        e = rel_l2(getattr(r, k).cpu().numpy(), o[k])
        _note(f"  512 workload {k}: rel L2 {e:.2e}")
        assert e <= GRAD_TOL, k


def test_fit_checkpoint_resume_matches_uninterrupted_run(torch_cuda, tmp_path):
    """60 optimiser steps straight against 30 steps, a checkpoint (.npz of the
    parameters, the optimiser's momentum buffers and the generator states), a
    fresh rasterizer and 30 resumed steps: the same parameters, up to the
    run-to-run spread of the backward's float atomics (measured here as the
    largest difference among three straight runs: one pair alone can land
    well below the spread a third run shows).  Momentum SGD keeps that spread at the rounding
    level (Adam's normalisation amplifies it chaotically; its moments' round
    trip is checked bit for bit on the host)."""
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    from paper_2503_16424_amd.optim import FitConfig, fit
    hidden = scenes.uniform_open(21, 96, 80, 300, 16)
    clean = torch.as_tensor(bz.Rasterizer(hidden).render().cpu().numpy(), device="cuda")
    sc = scenes.uniform_open(22, 96, 80, 120, 16)
    kw = dict(optimizer="sgd", momentum=0.9, lr_ctrl=2.0, lr_color=20.0, lr_opacity=20.0,
              lr_width=20.0, log_every=20)
    cfg = FitConfig(steps=60, **kw)

    def params(r):
        return np.concatenate([r.ctrl.cpu().numpy().ravel(), r.color.cpu().numpy().ravel(),
                               r.opacity.cpu().numpy().ravel(), r.stroke_w.cpu().numpy().ravel()])

    start = params(bz.Rasterizer(sc))
    straight = []
    for _ in range(3):
        r = bz.Rasterizer(sc)
        fit(r, clean, cfg)
        straight.append(params(r))
    path = str(tmp_path / "fit.npz")
    r = bz.Rasterizer(sc)
    fit(r, clean, FitConfig(steps=30, **kw), checkpoint_path=path, checkpoint_every=30)
    mid = params(r)
    r2 = bz.Rasterizer(sc)
    fit(r2, clean, cfg, resume_from=path)
    resumed = params(r2)
    moved = float(np.abs(straight[0] - mid).max())
    spread = max(float(np.abs(straight[i] - straight[j]).max())
                 for i in range(3) for j in range(i + 1, 3))
    err = float(np.abs(resumed - straight[0]).max())
    _note(f"  resumed vs straight {err:.2e}, straight vs straight {spread:.2e}, "
          f"second half moved {moved:.2e}, whole run {float(np.abs(straight[0] - start).max()):.2e}")
    assert moved > 1e-3                                   # the resumed half did work
    assert err <= max(10.0 * spread, 1e-4)
    # the checkpoint holds the step and the momentum buffers of all four groups
    with np.load(path, allow_pickle=False) as f:
        assert int(f["step"]) == 30
        assert all(f"opt_{g}_0_momentum_buffer" in f.files for g in range(4))
