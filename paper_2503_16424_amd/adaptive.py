"""Adaptive curve pruning and densification (Sec. 3.5 and the appendix
algorithm), around the optimisation loop.

Every ``interval`` steps (not in the last ``stop_before_end``), with the
curve budget held fixed:

* prune curves whose mean opacity is below a threshold that decreases
  linearly from ``opacity_start`` to ``opacity_end`` over the pruning phase;
* prune curves whose area (``bz_curve_area``) is below ``min_area``;
* prune a curve whose control-point bounding box overlaps the box of an
  earlier-drawn curve of nearly the same colour (Euclidean RGB distance below
  ``color_tol``) with intersection-over-union above ``iou_max``;
* split an open stroke whose middle segment's opacity is more than
  ``split_drop`` below both end segments: its first and last segments become
  strokes of their own (each subdivided back to the stroke's segment count),
  the faint middle is dropped;
* densify: the per-pixel error |render - target| summed over channels is
  thresholded at its ``error_quantile`` quantile; its connected regions
  (8-connected), largest first, each receive one new curve until the budget
  is back: a closed curve shaped as a circle (both boundaries as half
  circles) of the region's equivalent radius, or an open stroke across the
  region, with the region's mean target colour.

The decisions are host logic on a handful of per-curve numbers; the areas,
renders and errors come from libbz.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import scenes


@dataclass
class AdaptiveConfig:
    interval: int = 400             # steps between two passes (Sec. 4.1)
    stop_before_end: int = 1000     # no pass in the last steps (Sec. 4.1)
    opacity_start: float = 0.2
    opacity_end: float = 0.02       # Sec. 4.1
    min_area: float = 4.0           # px^2
    iou_max: float = 0.9            # Sec. 4.1
    color_tol: float = 0.03         # appendix
    split_drop: float = 0.5         # appendix
    error_quantile: float = 0.9
    circle_max_radius: float = 32.0


@dataclass
class PassReport:
    step: int
    pruned_opacity: int = 0
    pruned_area: int = 0
    pruned_overlap: int = 0
    split: int = 0
    added: int = 0
    regions: int = 0


def opacity_threshold(step: int, last_pass: int, cfg: AdaptiveConfig) -> float:
    f = 0.0 if last_pass <= 0 else min(max(step / last_pass, 0.0), 1.0)
    return cfg.opacity_start + (cfg.opacity_end - cfg.opacity_start) * f


def _mean_opacity(sc):
    return np.array([sc.opacity[sc.opa_off[i]: sc.opa_off[i + 1]].mean()
                     for i in range(sc.n_curves)])


def _boxes(sc):
    P = np.asarray(sc.ctrl, np.float64).reshape(-1, 2)
    lo = np.array([P[sc.ctrl_off[i]: sc.ctrl_off[i + 1]].min(0) for i in range(sc.n_curves)])
    hi = np.array([P[sc.ctrl_off[i]: sc.ctrl_off[i + 1]].max(0) for i in range(sc.n_curves)])
    return lo, hi


def prune_mask(sc, area, step, last_pass, cfg: AdaptiveConfig, rep: PassReport):
    """Keep-mask of the curves (by index)."""
    n = sc.n_curves
    keep = np.ones(n, bool)
    op = _mean_opacity(sc)
    low = op < opacity_threshold(step, last_pass, cfg)
    keep &= ~low
    rep.pruned_opacity = int(low.sum())
    small = (np.asarray(area) < cfg.min_area) & keep
    keep &= ~small
    rep.pruned_area = int(small.sum())
    lo, hi = _boxes(sc)
    col = np.asarray(sc.color, np.float64).reshape(-1, 3)
    pos = np.empty(n, np.int64)
    pos[np.argsort(sc.rank, kind="stable")] = np.arange(n)     # draw position of each curve
    areas = np.prod(hi - lo, axis=1)
    over = 0
    for i in np.argsort(pos):               # front to back: earlier survivors are final
        if not keep[i]:
            continue
        cand = keep & (pos < pos[i]) & (np.linalg.norm(col - col[i], axis=1) < cfg.color_tol)
        if not cand.any():
            continue
        a = np.maximum(lo[cand], lo[i])
        b = np.minimum(hi[cand], hi[i])
        inter = np.prod(np.maximum(b - a, 0.0), axis=1)
        union = areas[cand] + areas[i] - inter
        iou = np.where(union > 0, inter / np.where(union > 0, union, 1.0), 0.0)
        if np.any(iou > cfg.iou_max):
            keep[i] = False
            over += 1
    rep.pruned_overlap = over
    return keep


def _subdivide(P, S):
    """Cubic P0..P3 as S cubic segments (de Casteljau at u = s/S): 3S+1 points."""
    out = [P[0]]
    cur = np.asarray(P, np.float64)
    rem = 1.0
    for s in range(S - 1):
        t = (1.0 / S) / rem
        a = (1 - t) * cur[0] + t * cur[1]
        b = (1 - t) * cur[1] + t * cur[2]
        c = (1 - t) * cur[2] + t * cur[3]
        d = (1 - t) * a + t * b
        e = (1 - t) * b + t * c
        f = (1 - t) * d + t * e
        out += [a, d, f]
        cur = np.array([f, e, c, cur[3]])
        rem -= 1.0 / S
    out += [cur[1], cur[2], cur[3]]
    return np.asarray(out)


def split_candidates(sc, cfg: AdaptiveConfig):
    """Open strokes (3 or more segments, one opacity per segment) whose middle
    segment is more than split_drop fainter than both end segments."""
    out = []
    for i in range(sc.n_curves):
        S = int(sc.nseg[i])
        o = sc.opacity[sc.opa_off[i]: sc.opa_off[i + 1]]
        if sc.kind[i] != 0 or S < 3 or o.size != S:
            continue
        mid = o[S // 2]
        if mid < o[0] - cfg.split_drop and mid < o[-1] - cfg.split_drop:
            out.append(i)
    return out


def _circle(c, r, S=1):
    """A closed curve approximating the circle of centre c, radius r: A the
    upper half, B the lower half (cubic arcs, the 4/3 tan(pi/4) handles)."""
    k = 4.0 / 3.0 * np.tan(np.pi / 4.0)
    x0, y0 = c
    A = np.array([[x0 - r, y0], [x0 - r, y0 - k * r], [x0 + r, y0 - k * r], [x0 + r, y0]])
    B = np.array([[x0 - r, y0], [x0 - r, y0 + k * r], [x0 + r, y0 + k * r], [x0 + r, y0]])
    if S == 1:
        return np.concatenate([A, B[1:3]])
    Ad, Bd = _subdivide(A, S), _subdivide(B, S)
    return np.concatenate([Ad, Bd[1:-1]])


def error_regions(render, target, q):
    """Connected regions (8-connected) of the pixels whose error exceeds the
    q-quantile, largest first: [(pixel count, centroid x, centroid y, mean
    target colour, principal direction)]."""
    import scipy.ndimage as ndi
    err = np.abs(np.asarray(render, np.float64) - np.asarray(target, np.float64)).sum(0)
    thr = np.quantile(err, q)
    lab, n = ndi.label(err > thr, structure=np.ones((3, 3), int))
    regs = []
    for k in range(1, n + 1):
        ys, xs = np.nonzero(lab == k)
        if xs.size == 0:
            continue
        col = np.asarray(target)[:, ys, xs].mean(1)
        cov = np.cov(np.stack([xs, ys])) if xs.size > 2 else np.eye(2)
        w, v = np.linalg.eigh(np.atleast_2d(cov))
        regs.append((int(xs.size), xs.mean() + 0.5, ys.mean() + 0.5, col, v[:, -1]))
    regs.sort(key=lambda r: -r[0])
    return regs


def adapt(sc, area, render, target, step, last_pass, cfg: AdaptiveConfig):
    """One pruning + densification pass; returns (new scene, report).  The new
    scene keeps the curve count; new curves are drawn in front of the others."""
    rep = PassReport(step=step)
    n = sc.n_curves
    keep = prune_mask(sc, area, step, last_pass, cfg, rep)
    splits = [i for i in split_candidates(sc, cfg) if keep[i]]
    rep.split = len(splits)
    P = np.asarray(sc.ctrl, np.float64).reshape(-1, 2)
    parts = []                                          # (kind, S, K, R, ctrl, w, col, opa, tau)
    for i in range(n):
        if not keep[i]:
            continue
        c = P[sc.ctrl_off[i]: sc.ctrl_off[i + 1]]
        o = sc.opacity[sc.opa_off[i]: sc.opa_off[i + 1]]
        tau = sc.tau[sc.tau_off[i]: sc.tau_off[i + 1]]
        base = (int(sc.kind[i]), int(sc.nseg[i]), int(sc.k_samples[i]), int(sc.r_interior[i]))
        if i in splits:
            S = base[1]
            for seg, oo in ((0, o[0]), (S - 1, o[-1])):
                parts.append((0, S, base[2], 0, _subdivide(c[3 * seg: 3 * seg + 4], S),
                              sc.stroke_w[i], sc.color[i], np.full(S, oo), tau, int(sc.rank[i])))
        else:
            parts.append((*base, c, sc.stroke_w[i], sc.color[i], o, tau, int(sc.rank[i])))
    budget = n - len(parts)
    regs = error_regions(render, target, cfg.error_quantile) if budget > 0 else []
    rep.regions = len(regs)
    closed = bool(np.mean(sc.kind == 1) >= 0.5) if n else True
    ref = 0
    new = []
    for (cnt, cx, cy, col, d) in regs[:budget]:
        r = float(np.clip(np.sqrt(cnt / np.pi), 2.0, cfg.circle_max_radius))
        if closed:
            K = int(sc.k_samples[sc.kind == 1][0]) if np.any(sc.kind == 1) else 16
            R = int(sc.r_interior[sc.kind == 1][0]) if np.any(sc.kind == 1) else 4
            new.append((1, 1, K, R, _circle((cx, cy), r), 0.0, col, np.array([0.8]),
                        scenes.cdf_tau(R), -1))
        else:
            K = int(sc.k_samples[0])
            S = int(sc.nseg[0])
            seg = np.array([[cx, cy] - d * r, [cx, cy] - d * r / 3, [cx, cy] + d * r / 3,
                            [cx, cy] + d * r])
            opa = np.full(S if sc.opa_off[1] - sc.opa_off[0] == S else 1, 0.8)
            new.append((0, S, K, 0, _subdivide(seg, S), 2.0, col, opa, scenes.cdf_tau(0), -1))
        ref += 1
    rep.added = len(new)
    allp = new + parts
    # draw order: new curves in front (in region order), survivors keep their relative order
    old_rank = np.array([p[9] for p in parts], np.int64)
    rank = np.concatenate([np.arange(len(new)),
                           len(new) + np.argsort(np.argsort(old_rank, kind="stable"), kind="stable")])
    out = scenes._assemble(sc.width, sc.height, [p[0] for p in allp], [p[1] for p in allp],
                           [p[2] for p in allp], [p[3] for p in allp], [p[4] for p in allp],
                           np.array([p[5] for p in allp], np.float64),
                           np.array([p[6] for p in allp], np.float64).reshape(-1, 3),
                           [np.asarray(p[7]) for p in allp], rank, bg=sc.bg,
                           tau_list=[np.asarray(p[8]) for p in allp], name=sc.name, meta=sc.meta)
    return out, rep


def pull_params(sc, rast):
    """Copy the rasterizer's (optimised) parameters back into a scene."""
    s = sc.copy()
    s.ctrl = rast.ctrl.detach().cpu().numpy().astype(np.float32)
    s.stroke_w = rast.stroke_w.detach().cpu().numpy().astype(np.float32)
    s.color = rast.color.detach().cpu().numpy().reshape(-1, 3).astype(np.float32)
    s.opacity = rast.opacity.detach().cpu().numpy().astype(np.float32)
    return s


@dataclass
class AdaptiveResult:
    psnr: list = field(default_factory=list)
    reports: list = field(default_factory=list)
    final_psnr: float = 0.0
    scene: object = None


def fit_adaptive(sc, target, steps: int, fit_cfg=None, cfg: AdaptiveConfig | None = None,
                 draw_order: str = "rank", log=None) -> AdaptiveResult:
    """The optimisation loop with pruning and densification passes.  The
    optimiser restarts (fresh Adam moments) after every pass, since the curve
    set changes."""
    import dataclasses

    import torch

    from . import bz
    from .optim import FitConfig, fit
    cfg = cfg or AdaptiveConfig()
    fit_cfg = fit_cfg or FitConfig()
    last_pass = steps - cfg.stop_before_end
    res = AdaptiveResult()
    tgt_host = target.detach().cpu().numpy()
    done = 0
    while done < steps:
        chunk = cfg.interval if done + cfg.interval <= last_pass else steps - done
        r = bz.Rasterizer(sc, draw_order=draw_order)
        fr = fit(r, target, dataclasses.replace(fit_cfg, steps=chunk))
        res.psnr += [(done + s, p) for s, p in fr.psnr]
        done += chunk
        sc = pull_params(sc, r)
        if done < last_pass + 1 and done < steps:
            img = r.render().detach().cpu().numpy()
            area = r.curve_area().cpu().numpy()[: sc.n_curves]
            sc, rep = adapt(sc, area, img, tgt_host, done, last_pass, cfg)
            res.reports.append(rep)
            if log:
                log(f"  step {done}: {rep}")
        res.final_psnr = fr.final_psnr
        del r
        torch.cuda.empty_cache()
    res.scene = sc
    return res


def main(argv=None):
    """Closed-curve fit on a synthetic 512x512 target, with and without the
    paper's additions (area draw order, Xing loss, pruning + densification)."""
    import argparse
    import json
    import sys

    import torch

    from . import bz
    from .optim import PAPER_LR, FitConfig, fit, noisy_target
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--curves", type=int, default=400)
    ap.add_argument("--xing", type=float, default=1e-5)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    W = H = 512
    hidden = scenes.mixed(5, W, H, a.curves, 0, K=16, R=8, extent=(8.0, 160.0),
                          name="hidden-closed-512")
    clean = bz.Rasterizer(hidden).render().cpu().numpy()
    tgt = torch.as_tensor(noisy_target(clean, 6, 0.02), device="cuda")
    init = scenes.mixed(7, W, H, a.curves, 0, K=16, R=8, extent=(8.0, 80.0), name="init")
    out = {"steps": a.steps, "curves": a.curves, "xing_weight": a.xing, "lr": "Sec. 4.1"}
    runs = [("plain", "rank", 0.0, False), ("area_order+xing", "area", a.xing, False),
            ("area_order+xing+adaptive", "area", a.xing, True)]
    for name, order, xw, adaptive in runs:
        cfg = FitConfig(steps=a.steps, log_every=100, xing_weight=xw, **PAPER_LR)
        if adaptive:
            res = fit_adaptive(init, tgt, a.steps, cfg, draw_order=order, log=log)
            r = bz.Rasterizer(res.scene, draw_order=order)
            extra = {"passes": [vars(p) for p in res.reports]}
            final, traj = res.final_psnr, res.psnr
        else:
            r = bz.Rasterizer(init, draw_order=order)
            fr = fit(r, tgt, cfg)
            final, traj, extra = fr.final_psnr, fr.psnr, {}
        r.render()
        xv = float(r.xing(1.0).item())
        out[name] = dict(psnr_final=final, xing_final=xv,
                         trajectory=[(s, round(p, 3)) for s, p in traj], **extra)
        log(f"{name}: final PSNR {final:.2f} dB, Xing {xv:.3f}")
    print(json.dumps({k: (v if not isinstance(v, dict) else
                          {kk: vv for kk, vv in v.items() if kk != "trajectory"})
                      for k, v in out.items()}), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(out, fh)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
