"""Test helpers that are independent of both the oracle and the HIP library."""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from paper_2503_16424_amd import scenes


def de_casteljau(P, t):
    """Point on a Bezier curve by repeated linear interpolation (de Casteljau)."""
    pts = [np.asarray(p, dtype=np.float64) for p in P]
    while len(pts) > 1:
        pts = [(1.0 - t) * a + t * b for a, b in zip(pts[:-1], pts[1:])]
    return pts[0]


def composite_point(P, S, k, K):
    """Point at global parameter u = k/(K-1) on an S-segment composite cubic.

    The segment is chosen with exact rational arithmetic; a parameter that
    lands exactly on a joint belongs to the later segment (both give the same
    point by continuity)."""
    u = Fraction(k, K - 1)
    s = min(int(u * S), S - 1)
    t = float(u * S - s)
    return de_casteljau(P[3 * s:3 * s + 4], t), s


def closed_boundaries(ctrl, S):
    """Boundary A (3S+1 points) and B (A's endpoints around the 3S-1 stored
    interior points) of a closed curve's control points."""
    m = 3 * S
    A = np.asarray(ctrl[:m + 1], np.float64)
    B = np.concatenate([A[:1], np.asarray(ctrl[m + 1:], np.float64), A[m:]])
    return A, B


def gauss_set(mu, conic, opac, color):
    return dict(mu=np.asarray(mu, np.float64).reshape(-1, 2),
                conic=np.asarray(conic, np.float64).reshape(-1, 3),
                opac=np.asarray(opac, np.float64).reshape(-1),
                color=np.asarray(color, np.float64).reshape(-1, 3))


def scene_from_curves(W, H, curves, bg=(1.0, 1.0, 1.0), rank=None):
    """curves: list of dicts(kind, S, K, R, ctrl, width, color, opacity[, tau])."""
    n = len(curves)
    taus = [c.get("tau", scenes.cdf_tau(c.get("R", 0))) for c in curves]
    sc = scenes._assemble(W, H, [c["kind"] for c in curves], [c["S"] for c in curves],
                          [c["K"] for c in curves], [c.get("R", 0) for c in curves],
                          [np.asarray(c["ctrl"], np.float64) for c in curves],
                          [c.get("width", 0.0) for c in curves], [c["color"] for c in curves],
                          [np.atleast_1d(c["opacity"]) for c in curves],
                          np.arange(n) if rank is None else rank, bg=bg, tau_list=taus)
    sc = to_f64(sc)
    # keep the exact float64 inputs (the assembler stores float32)
    sc.ctrl = np.concatenate([np.asarray(c["ctrl"], np.float64).reshape(-1, 2) for c in curves])
    sc.tau = np.concatenate([np.asarray(t, np.float64) for t in taus])
    sc.stroke_w = np.array([c.get("width", 0.0) for c in curves], np.float64)
    sc.color = np.array([c["color"] for c in curves], np.float64).reshape(n, 3)
    sc.opacity = np.concatenate([np.atleast_1d(np.asarray(c["opacity"], np.float64))
                                 for c in curves])
    return sc


def to_f64(sc):
    """Float64 copies of the float inputs (so finite differences can perturb them)."""
    sc = sc.copy()
    for k in ("ctrl", "tau", "stroke_w", "color", "opacity", "bg"):
        setattr(sc, k, np.asarray(getattr(sc, k), np.float64))
    return sc


def rel_l2(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def _lens(S, c, L, h):
    """Control points of an S-segment closed curve: boundary A (3S+1 points)
    bowed down by h/2 around centre c, then B's 3S-1 interior points a
    height h above A's straight chord."""
    import numpy as np
    A = [c + np.array([(-0.5 + j / (3 * S)) * L, 0.0]) for j in range(3 * S + 1)]
    B = [c + np.array([(-0.5 + j / (3 * S)) * L, h]) for j in range(1, 3 * S)]
    A = [a + np.array([0.0, -0.5 * h * np.sin(np.pi * j / (3 * S))]) for j, a in enumerate(A)]
    return np.array(A + B)


def size_split_scene(W=120, H=96):
    """Curves on both sides of the per-curve kernels' split at 64 Gaussians,
    interleaved in draw order: open strokes of K = 63, 64, 65 and closed
    curves of K*(R+2) = 63 (21x3), 64 (16x4, 32x2, 2x32), 65 (13x5) and 96."""
    import numpy as np
    from paper_2503_16424_amd import scenes
    rng = np.random.default_rng(2024)
    # (kind, S, K, R): 0 open, 1 closed
    spec = [(0, 2, 63, 0), (1, 1, 16, 2), (0, 1, 64, 0), (1, 2, 13, 3), (0, 3, 65, 0),
            (1, 1, 21, 1), (1, 2, 32, 0), (1, 1, 2, 30), (0, 1, 24, 0), (1, 3, 24, 2)]
    kinds, nsegs, ks, rs, ctrl, widths, opa = [], [], [], [], [], [], []
    for kind, S, K, R in spec:
        kinds.append(kind); nsegs.append(S); ks.append(K); rs.append(R)
        if kind == 0:
            ctrl.append(rng.uniform([4, 4], [W - 4, H - 4], (3 * S + 1, 2)))
            widths.append(rng.uniform(1.0, 3.0))
        else:
            c = rng.uniform([25, 25], [W - 25, H - 25])
            ctrl.append(_lens(S, c, rng.uniform(16.0, 40.0), rng.uniform(6.0, 16.0)))
            widths.append(0.0)
        opa.append(rng.uniform(0.4, 0.95, S if S > 1 and rng.uniform() < 0.5 else 1))
    rank = rng.permutation(len(spec))
    return scenes._assemble(W, H, kinds, nsegs, ks, rs, ctrl, widths,
                            rng.uniform(0, 1, (len(spec), 3)), opa, rank, name="size-split")


def max_size_scene(W=96, H=80):
    """Curves at the per-curve limits: a 4-segment stroke of K = 1024 samples,
    a 4-segment closed curve of R = 254 interior rows (K = 8), and a closed
    curve of K = 60, R = 30 (together at the per-curve kernels' LDS budget:
    the widest curve and the curve with most Gaussians share it)."""
    import numpy as np
    from paper_2503_16424_amd import scenes
    rng = np.random.default_rng(99)
    stroke = rng.uniform([5, 5], [W - 5, H - 5], (13, 2))
    ctrl = [stroke, _lens(4, np.array([40.0, 40.0]), 60.0, 20.0),
            _lens(1, np.array([60.0, 30.0]), 30.0, 12.0)]
    return scenes._assemble(W, H, [0, 1, 1], [4, 4, 1], [1024, 8, 60], [0, 254, 30], ctrl,
                            [2.0, 0.0, 0.0], rng.uniform(0, 1, (3, 3)),
                            [[0.6, 0.9, 0.4, 0.8], [0.7], [0.5]], [2, 0, 1])


def fused_l2_matches_separate(torch, r, tgt, ref_of):
    """Render with bz_render_fwd then bz_l2_grad, then with bz_render_fwd_l2
    over sentinel-filled outputs: image, blend state and d_image bit for bit,
    the loss within float rounding of its sum (reference: ref_of(image)); the
    same without the contributor counts, which are then left untouched."""
    r.render()
    r.l2_grad(tgt)
    torch.cuda.synchronize()
    names = ["image", "d_image"] + (["t_final", "n_last", "n_contrib"] if r.state else [])
    want = {k: getattr(r, k).clone() for k in names}
    loss_sep = float(r.loss.item())
    for k in names:
        getattr(r, k).fill_(-7)
    r.loss.fill_(-7.0)
    r.forward_l2(tgt, count=True)
    torch.cuda.synchronize()
    for k in names:
        assert torch.equal(getattr(r, k).view(torch.int32), want[k].view(torch.int32)), k
    ref = ref_of(r.image)
    assert abs(float(r.loss.item()) - ref) <= 1e-5 * ref
    assert abs(loss_sep - ref) <= 1e-5 * ref
    # without the contributor counts (as the step runs it): the rest unchanged,
    # the counts left as they were
    if r.state:
        r.n_contrib.fill_(-5)
    for k in names:
        if k != "n_contrib":
            getattr(r, k).fill_(-7)
    r.forward_l2(tgt)
    torch.cuda.synchronize()
    for k in names:
        if k == "n_contrib":
            assert bool((r.n_contrib == -5).all())
        else:
            assert torch.equal(getattr(r, k).view(torch.int32), want[k].view(torch.int32)), k


def sample_bin_matches_separate(torch, r):
    """bz_sample then bz_bin, then bz_sample_bin over sentinel-filled outputs:
    records, the two status words, tile ranges and the tile lists bit for bit (the
    lists only without overflow: with it neither call writes them)."""
    r.sample()
    r.bin()
    torch.cuda.synchronize()
    n = r.pairs_required()
    want = dict(rec=r.rec[: 12 * r.n_gauss].clone(), status=r.status[:2].clone(),
                ranges=r.ranges.clone())
    if n <= r.cap_pairs:
        want["ids"] = r.ids[:n].clone()
    r.rec.fill_(-7.0)
    r.status.fill_(-7)
    r.ranges.fill_(-7)
    r.ids.fill_(-7)
    r.sample_bin()
    torch.cuda.synchronize()
    got = dict(rec=r.rec[: 12 * r.n_gauss], status=r.status[:2], ranges=r.ranges, ids=r.ids[:n])
    for k in want:
        assert torch.equal(got[k].view(torch.int32), want[k].view(torch.int32)), k
    return n
