"""Seeded synthetic curve scenes shared by the tests, the benchmark and the oracle runs.

This module only draws random inputs and lays them out in the flat
structure-of-arrays form that both the CPU oracle and the HIP library accept.
It holds none of the rendering method's arithmetic: no Bernstein evaluation, no
scales, no blending.  Everything is drawn with numpy's PCG64 generator
(``numpy.random.default_rng(seed)``) in a fixed, documented order so that a
scene is reproducible from its seed alone.

Curve model (Sec. 3.2 of the paper, "Primitives of Bezier Splatting"):

* an *open* curve (kind 0) is a stroke of ``S`` cubic segments sharing
  endpoints, i.e. ``3S+1`` control points, with a stroke width and one or
  ``S`` opacities (per-segment opacity, appendix on flexible attributes);
* a *closed* curve (kind 1) is the paired structure of Sec. 3.3: two boundary
  curves of ``S`` cubic segments that share their first and last control
  point.  It is stored as the ``3S+1`` points of boundary A followed by the
  ``3S-1`` interior points of boundary B (``6S`` points in total) and carries
  ``R`` interpolated interior rows with a per-curve table ``tau`` of ``R+2``
  interpolation weights (``tau[0]=0``, ``tau[R+1]=1``).

All coordinates are in pixels, pixel ``(x, y)`` has its centre at
``(x+0.5, y+0.5)``; colours and opacities are the activated values in [0, 1].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

OPEN = 0
CLOSED = 1


@dataclass
class Scene:
    width: int
    height: int
    bg: np.ndarray              # float32[3]
    kind: np.ndarray            # int32[n]
    nseg: np.ndarray            # int32[n]   S
    k_samples: np.ndarray       # int32[n]   K >= 2
    r_interior: np.ndarray      # int32[n]   R (0 for open curves)
    ctrl: np.ndarray            # float32[n_ctrl, 2]
    ctrl_off: np.ndarray        # int32[n+1]
    tau: np.ndarray             # float32[n_tau]
    tau_off: np.ndarray         # int32[n+1] (R+2 entries per curve)
    stroke_w: np.ndarray        # float32[n] (stroke width of open curves, px)
    color: np.ndarray           # float32[n, 3]
    opacity: np.ndarray         # float32[n_opa]
    opa_off: np.ndarray         # int32[n+1] (1 or S entries per curve)
    rank: np.ndarray            # int32[n] draw order, 0 = front
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_curves(self) -> int:
        return int(self.kind.shape[0])

    def rows(self) -> np.ndarray:
        """Rows of sample points per curve: 1 for open, R+2 for closed."""
        return np.where(self.kind == CLOSED, self.r_interior + 2, 1).astype(np.int64)

    def n_gauss_per_curve(self) -> np.ndarray:
        return self.rows() * self.k_samples.astype(np.int64)

    @property
    def n_gauss(self) -> int:
        return int(self.n_gauss_per_curve().sum())

    def arrays(self) -> dict:
        return {k: getattr(self, k) for k in (
            "bg", "kind", "nseg", "k_samples", "r_interior", "ctrl", "ctrl_off", "tau",
            "tau_off", "stroke_w", "color", "opacity", "opa_off", "rank")}

    def copy(self) -> "Scene":
        a = {k: np.array(v, copy=True) for k, v in self.arrays().items()}
        return Scene(width=self.width, height=self.height, name=self.name,
                     meta=dict(self.meta), **a)


def cdf_tau(R: int) -> np.ndarray:
    """Interpolation weights of the R interior rows of a closed curve.

    The paper draws them from an unnamed normalised CDF that must place rows
    more densely near the two boundaries (Sec. 3.3).  The reading used here is
    the standard normal CDF on [-2, 2], renormalised to [0, 1], evaluated at
    R+2 equally spaced abscissae; this is an *input* table, swappable by the
    caller.
    """
    z = -2.0 + 4.0 * np.arange(R + 2) / (R + 1)
    phi = lambda v: 0.5 * (1.0 + math.erf(v / math.sqrt(2.0)))
    lo, hi = phi(-2.0), phi(2.0)
    t = np.array([(phi(v) - lo) / (hi - lo) for v in z], dtype=np.float64)
    t[0], t[-1] = 0.0, 1.0
    return t.astype(np.float32)


def _assemble(width, height, kinds, nsegs, ks, rs, ctrl_list, widths, colors,
              opa_list, rank, bg=(1.0, 1.0, 1.0), tau_list=None, name="", meta=None) -> Scene:
    n = len(kinds)
    ctrl_off = np.zeros(n + 1, np.int32)
    opa_off = np.zeros(n + 1, np.int32)
    tau_off = np.zeros(n + 1, np.int32)
    taus = []
    for i in range(n):
        ctrl_off[i + 1] = ctrl_off[i] + len(ctrl_list[i])
        opa_off[i + 1] = opa_off[i] + len(opa_list[i])
        tb = tau_list[i] if tau_list is not None else cdf_tau(int(rs[i]))
        taus.append(np.asarray(tb, np.float32))
        tau_off[i + 1] = tau_off[i] + len(tb)
    ctrl = (np.concatenate([np.asarray(c, np.float32).reshape(-1, 2) for c in ctrl_list])
            if n else np.zeros((0, 2), np.float32))
    opacity = (np.concatenate([np.asarray(o, np.float32).reshape(-1) for o in opa_list])
               if n else np.zeros(0, np.float32))
    tau = np.concatenate(taus) if n else np.zeros(0, np.float32)
    return Scene(
        width=int(width), height=int(height), bg=np.asarray(bg, np.float32),
        kind=np.asarray(kinds, np.int32), nseg=np.asarray(nsegs, np.int32),
        k_samples=np.asarray(ks, np.int32), r_interior=np.asarray(rs, np.int32),
        ctrl=np.ascontiguousarray(ctrl, np.float32), ctrl_off=ctrl_off,
        tau=np.ascontiguousarray(tau, np.float32), tau_off=tau_off,
        stroke_w=np.asarray(widths, np.float32).reshape(n),
        color=np.asarray(colors, np.float32).reshape(n, 3),
        opacity=np.ascontiguousarray(opacity, np.float32), opa_off=opa_off,
        rank=np.asarray(rank, np.int32), name=name, meta=meta or {})


def uniform_open(seed: int, W: int, H: int, n: int, K: int, S: int = 1,
                 per_segment_opacity: bool = False, name: str = "") -> Scene:
    """Open strokes with every control point uniform over the canvas.

    Draw order of the generator: control points, widths, colours, opacities.
    Widths U[1,4] px, colours U[0,1]^3, opacities U[0.3,1]; identity draw order.
    """
    rng = np.random.default_rng(seed)
    npts = 3 * S + 1
    ctrl = rng.uniform(0.0, 1.0, (n, npts, 2)) * np.array([W, H], np.float64)
    widths = rng.uniform(1.0, 4.0, n)
    colors = rng.uniform(0.0, 1.0, (n, 3))
    n_opa = S if per_segment_opacity else 1
    opas = rng.uniform(0.3, 1.0, (n, n_opa))
    return _assemble(W, H, [OPEN] * n, [S] * n, [K] * n, [0] * n, list(ctrl), widths,
                     colors, list(opas), np.arange(n), name=name)


def mixed(seed: int, W: int, H: int, n_closed: int, n_open: int, K: int = 24, R: int = 20,
          S_open: int = 3, S_closed: int = 1, extent=(4.0, 400.0), per_segment_opacity=True,
          permute=True, name: str = "") -> Scene:
    """Closed lenses and open strokes scattered over the canvas.

    Per curve: centre U[0,W)xU[0,H), linear extent L log-uniform in ``extent``.
    Closed (drawn first, all closed curves): chord endpoints centre +- (L/2)(cos f, sin f)
    with f ~ U[0,pi); the inner control points of boundary A sit on the chord at
    equal spacing offset by +h_A along the chord normal, those of boundary B by
    -h_B, with h ~ U[0.15,0.5]*L each, giving convex lenses.  Open: every
    control point is centre + L*U[-1/2,1/2]^2.  Then widths U[1,4] (open),
    colours U[0,1]^3, opacities U[0.3,1] (one per curve, or one per segment for
    open curves when ``per_segment_opacity``), and finally a random draw-order
    permutation when ``permute``.
    """
    rng = np.random.default_rng(seed)
    n = n_closed + n_open
    lo, hi = math.log(extent[0]), math.log(extent[1])
    centre = rng.uniform(0.0, 1.0, (n, 2)) * np.array([W, H], np.float64)
    L = np.exp(rng.uniform(lo, hi, n))
    ctrl_list, kinds, nsegs, rs = [], [], [], []
    # closed lenses
    phi = rng.uniform(0.0, math.pi, n_closed)
    hA = rng.uniform(0.15, 0.5, n_closed) * L[:n_closed]
    hB = rng.uniform(0.15, 0.5, n_closed) * L[:n_closed]
    for i in range(n_closed):
        e = np.array([math.cos(phi[i]), math.sin(phi[i])])
        nrm = np.array([-e[1], e[0]])
        p0 = centre[i] - 0.5 * L[i] * e
        p3 = centre[i] + 0.5 * L[i] * e
        m = 3 * S_closed
        along = [p0 + (j / m) * (p3 - p0) for j in range(m + 1)]
        A = [along[0]] + [along[j] + hA[i] * nrm for j in range(1, m)] + [along[m]]
        B = [along[j] - hB[i] * nrm for j in range(1, m)]
        ctrl_list.append(np.array(A + B))
        kinds.append(CLOSED)
        nsegs.append(S_closed)
        rs.append(R)
    # open strokes
    m = 3 * S_open + 1
    off = rng.uniform(-0.5, 0.5, (n_open, m, 2))
    for j in range(n_open):
        i = n_closed + j
        ctrl_list.append(centre[i] + L[i] * off[j])
        kinds.append(OPEN)
        nsegs.append(S_open)
        rs.append(0)
    widths = rng.uniform(1.0, 4.0, n)
    widths[:n_closed] = 0.0
    colors = rng.uniform(0.0, 1.0, (n, 3))
    opa_list = []
    for i in range(n):
        k = nsegs[i] if (kinds[i] == OPEN and per_segment_opacity) else 1
        opa_list.append(rng.uniform(0.3, 1.0, k))
    rank = rng.permutation(n) if permute else np.arange(n)
    return _assemble(W, H, kinds, nsegs, [K] * n, rs, ctrl_list, widths, colors,
                     opa_list, rank, name=name)


def target_noise(seed: int, W: int, H: int) -> np.ndarray:
    """Uniform-noise target image, planar [3][H][W] float32."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, (3, H, W)).astype(np.float32)


# ---------------------------------------------------------------------------
# Named workloads.  Sizes follow the paper's experiments (2K frames, thousands
# of curves, K Gaussians per row, R = 20 interior rows for closed curves).
# ---------------------------------------------------------------------------

def tiny_128(seed: int = 0) -> Scene:
    """128x128 canvas, 256 open single-segment curves x 16 samples (4,096 Gaussians).

    Draw order: control points U[0,128)^2, widths, colours, opacities; the
    uniform-noise target is drawn afterwards from the same generator by
    :func:`tiny_128_target`.
    """
    return uniform_open(seed, 128, 128, 256, 16, S=1, name="open-128x128-256c-K16")


def tiny_128_target(seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    n, npts = 256, 4
    rng.uniform(0.0, 1.0, (n, npts, 2))
    rng.uniform(1.0, 4.0, n)
    rng.uniform(0.0, 1.0, (n, 3))
    rng.uniform(0.3, 1.0, (n, 1))
    return rng.uniform(0.0, 1.0, (3, 128, 128)).astype(np.float32)


def open_512(seed: int = 0) -> Scene:
    """512x512 canvas, 2,048 open single-segment curves x 32 samples (65,536 Gaussians)."""
    return uniform_open(seed, 512, 512, 2048, 32, S=1, name="open-512x512-2048c-K32")


def hidden_512(seed: int = 1) -> Scene:
    """The 4,096-curve hidden scene whose render is the 512x512 optimisation target."""
    return uniform_open(seed, 512, 512, 4096, 32, S=1, name="hidden-512x512-4096c-K32")


# Upper extent bound of the 2048x2048 workload.  Its definition asks for curve
# sizes from 4 to 400 px and for a per-tile depth complexity of up to about
# 300 (distinct curves per 16x16 tile).  Read as linear extents, 4..400 px
# gives at most 87 curves whose support reaches a tile (mean 58), so the
# upper bound is raised until the measured maximum is about 300: 1000 px
# gives 307 (mean 225; 289 at the 99th percentile).  The lower bound, the
# curve counts and every other draw are unchanged.
PAPER_EXTENT = (4.0, 1000.0)


def paper_2048(seed: int = 0) -> Scene:
    """2048x2048, 20,000 curves: 12,000 closed (R=20, K=24) + 8,000 open (S=3, K=24).

    6,528,000 Gaussians; extents log-uniform over PAPER_EXTENT (4..1000 px,
    per-tile depth up to ~300 curves); seeded draw order.
    """
    return mixed(seed, 2048, 2048, 12000, 8000, K=24, R=20, S_open=3, S_closed=1,
                 extent=PAPER_EXTENT, name="mixed-2048x2048-20k-R20-K24-depth300")


def paper_2048_e400(seed: int = 0) -> Scene:
    """The same 20,000-curve frame with extents over 4..400 px only (per-tile
    depth at most 87 curves): the lighter variant, kept for comparison."""
    return mixed(seed, 2048, 2048, 12000, 8000, K=24, R=20, S_open=3, S_closed=1,
                 extent=(4.0, 400.0), name="mixed-2048x2048-20k-R20-K24-L400")


def paper_analog(seed: int = 0, closed: bool = False) -> Scene:
    """2040x1344 frame with 2,048 curves (the size of the paper's speed comparison)."""
    if closed:
        return mixed(seed, 2040, 1344, 2048, 0, K=24, R=20, name="closed-2040x1344-2048c")
    return mixed(seed, 2040, 1344, 0, 2048, K=24, S_open=3, name="open-2040x1344-2048c")


def batched(seed: int = 0, n_canvas: int = 64, side=(128, 1024), curves=(256, 8192),
            k_range=(16, 32)) -> list:
    """Many canvases of uneven size and curve count (open single-segment curves).

    Per canvas: width and height independently log-uniform over ``side`` px,
    floor(log-uniform over ``curves``) curves, K per curve uniform over the
    integers of ``k_range``.  Draw order of the generator: all widths, all
    heights, all curve counts, one child seed per canvas; each canvas then
    draws control points (uniform over its area), widths U[1,4], colours
    U[0,1]^3, opacities U[0.3,1] and the K values from its child seed.
    """
    rng = np.random.default_rng(seed)
    lo, hi = math.log(side[0]), math.log(side[1])
    Ws = np.clip(np.floor(np.exp(rng.uniform(lo, hi, n_canvas))), side[0], side[1]).astype(int)
    Hs = np.clip(np.floor(np.exp(rng.uniform(lo, hi, n_canvas))), side[0], side[1]).astype(int)
    ncs = np.floor(np.exp(rng.uniform(math.log(curves[0]), math.log(curves[1]), n_canvas)))
    ncs = np.clip(ncs, curves[0], curves[1]).astype(int)
    child = rng.integers(0, 2 ** 31 - 1, n_canvas)
    out = []
    for c in range(n_canvas):
        W, H, n = int(Ws[c]), int(Hs[c]), int(ncs[c])
        r = np.random.default_rng(int(child[c]))
        ctrl = r.uniform(0.0, 1.0, (n, 4, 2)) * np.array([W, H], np.float64)
        widths = r.uniform(1.0, 4.0, n)
        colors = r.uniform(0.0, 1.0, (n, 3))
        opas = r.uniform(0.3, 1.0, (n, 1))
        ks = r.integers(k_range[0], k_range[1] + 1, n)
        out.append(_assemble(W, H, [OPEN] * n, [1] * n, ks, [0] * n, list(ctrl), widths, colors,
                             list(opas), np.arange(n), name=f"canvas{c}-{W}x{H}-{n}c"))
    return out


def patch_origins(W: int, H: int, side: int = 32) -> np.ndarray:
    """Top-left corners [n, 2] (px) of the side x side patches tiling a canvas, row-major."""
    ys, xs = np.mgrid[0:H:side, 0:W:side]
    return np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)


def open_curves(W: int, H: int, ctrl, widths, colors, opacities, K: int, name: str = "") -> Scene:
    """Open single-segment curves from arrays: ctrl [n, 4, 2] px, widths [n],
    colours [n, 3], opacities [n]; identity draw order."""
    ctrl = np.asarray(ctrl, np.float64).reshape(-1, 4, 2)
    n = ctrl.shape[0]
    return _assemble(W, H, [OPEN] * n, [1] * n, [K] * n, [0] * n, list(ctrl),
                     np.asarray(widths).reshape(n), np.asarray(colors).reshape(n, 3),
                     list(np.asarray(opacities).reshape(n, 1)), np.arange(n), name=name)


def grid_init(W: int, H: int, side: int = 32, per: int = 8, K: int = 16) -> Scene:
    """Deterministic per-patch initialisation: the patch is cut into per cells
    (4 columns x per/4 rows); slot j's curve is a straight horizontal stroke
    across cell j (control points at 1/8, 3/8, 5/8, 7/8 of its width, at its
    mid height), width 2 px, grey, opacity 0.5."""
    org = patch_origins(W, H, side).astype(np.float64)
    cols, rows = 4, per // 4
    cw, ch = side / cols, side / rows
    ctrl = []
    for j in range(per):
        cx0, cy = (j % cols) * cw, (j // cols) * ch + ch / 2
        ctrl.append([[cx0 + cw * f, cy] for f in (0.125, 0.375, 0.625, 0.875)])
    ctrl = np.asarray(ctrl)[None] + org[:, None, None, :]
    n = ctrl.shape[0] * per
    return open_curves(W, H, ctrl.reshape(n, 4, 2), np.full(n, 2.0), np.full((n, 3), 0.5),
                       np.full(n, 0.5), K, name=f"grid-init-{W}x{H}")


def random_init(seed: int, W: int, H: int, side: int = 32, per: int = 8, K: int = 16) -> Scene:
    """Uniform random initialisation, per curves per patch (the same count and
    density as the learned one): control points uniform over the curve's
    patch, widths U[1,4], colours U[0,1]^3, opacities U[0.3,1].  Drawn in that
    order for all curves at once."""
    rng = np.random.default_rng(seed)
    org = patch_origins(W, H, side).astype(np.float64)
    n = org.shape[0] * per
    ctrl = rng.uniform(0.0, side, (org.shape[0], per, 4, 2)) + org[:, None, None, :]
    widths = rng.uniform(1.0, 4.0, n)
    colors = rng.uniform(0.0, 1.0, (n, 3))
    opas = rng.uniform(0.3, 1.0, n)
    return open_curves(W, H, ctrl.reshape(n, 4, 2), widths, colors, opas, K,
                       name=f"random-init-{W}x{H}")


def small_mixed(seed: int, W: int = 48, H: int = 40, n_closed: int = 3, n_open: int = 4,
                K: int = 8, R: int = 3, extent=(6.0, 30.0)) -> Scene:
    """Small mixed scenes for finite-difference and parity tests."""
    return mixed(seed, W, H, n_closed, n_open, K=K, R=R, S_open=3, S_closed=1,
                 extent=extent, name=f"small-mixed-{W}x{H}-s{seed}")


WORKLOADS = {
    "tiny_128": tiny_128,
    "open_512": open_512,
    "paper_2048": paper_2048,
    "paper_2048_e400": paper_2048_e400,
}


def gaussian_noise(seed: int, shape, sigma: float) -> np.ndarray:
    """Additive N(0, sigma^2) noise of the given shape (float64), seeded."""
    return np.random.default_rng(seed).normal(0.0, sigma, shape)


def concat(parts) -> Scene:
    """One curve set holding the curves of several canvases, canvas by canvas:
    the draw order of canvas c follows every curve of canvases before it.
    Width and height are the largest of the parts (a batch's canvases keep
    their own sizes and backgrounds in the batch layout)."""
    kinds, nsegs, ks, rs, ctrl, taus, ws, cols, opas, ranks = ([] for _ in range(10))
    ctrl_off, tau_off, opa_off = [0], [0], [0]
    base = 0
    for sc in parts:
        n = sc.n_curves
        kinds.append(sc.kind); nsegs.append(sc.nseg); ks.append(sc.k_samples)
        rs.append(sc.r_interior); ctrl.append(np.asarray(sc.ctrl).reshape(-1, 2))
        taus.append(np.asarray(sc.tau).reshape(-1)); ws.append(sc.stroke_w)
        cols.append(np.asarray(sc.color).reshape(-1, 3)); opas.append(np.asarray(sc.opacity).reshape(-1))
        ranks.append(np.asarray(sc.rank) + base)
        ctrl_off.extend((np.asarray(sc.ctrl_off[1:]) + ctrl_off[-1]).tolist())
        tau_off.extend((np.asarray(sc.tau_off[1:]) + tau_off[-1]).tolist())
        opa_off.extend((np.asarray(sc.opa_off[1:]) + opa_off[-1]).tolist())
        base += n
    cat = lambda xs, dt: np.ascontiguousarray(np.concatenate(xs), dt)
    return Scene(width=max(sc.width for sc in parts), height=max(sc.height for sc in parts),
                 bg=np.asarray(parts[0].bg, np.float32), kind=cat(kinds, np.int32),
                 nseg=cat(nsegs, np.int32), k_samples=cat(ks, np.int32),
                 r_interior=cat(rs, np.int32), ctrl=cat(ctrl, np.float32),
                 ctrl_off=np.asarray(ctrl_off, np.int32), tau=cat(taus, np.float32),
                 tau_off=np.asarray(tau_off, np.int32), stroke_w=cat(ws, np.float32),
                 color=cat(cols, np.float32), opacity=cat(opas, np.float32),
                 opa_off=np.asarray(opa_off, np.int32), rank=cat(ranks, np.int32),
                 name=f"batch-{len(parts)}", meta={})
