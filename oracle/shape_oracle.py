"""Plain FP64 reference of the per-curve shape terms: area, draw order by area
(Sec. 3.3) and the Xing convexity loss (Sec. 3.5).

TEST INFRASTRUCTURE ONLY: imported by tests/ alone.

* ``curve_area``: closed curve: area of the polygon of its boundary samples
  A_0..A_{K-1}, B_{K-2}..B_1 (rows 0 and R+1 of the oracle's own sampling),
  by the shoelace formula; open stroke: polyline length of its samples times
  its width.
* ``area_order``: the curves sorted by area, smallest first, equal areas by
  index (a stable sort), and the first Gaussian of every position.
* ``xing_loss``: per cubic segment P0..P3 of each boundary of a closed curve,
  D1 = [cross(P1-P0, P2-P1) >= 0], D2 = sine from P1-P0 to P3-P2; the segment
  costs D1 max(0, -D2) + (1 - D1) max(0, D2).
"""
from __future__ import annotations

import numpy as np

from . import oracle as _o


def _cross(a, b):
    return a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]


def curve_area(sc, opts=None) -> np.ndarray:
    g = _o.sample(sc, opts)
    mu, curve = g["mu"], g["curve"]
    # a curve's Gaussians are consecutive, row-major: (r, k) at first + r K + k
    first = np.full(sc.n_curves, -1, np.int64)
    idx = np.flatnonzero(np.r_[True, curve[1:] != curve[:-1]]) if curve.size else np.zeros(0, int)
    first[curve[idx]] = idx
    out = np.zeros(sc.n_curves)
    for i in range(sc.n_curves):
        K, f = int(sc.k_samples[i]), int(first[i])
        A = mu[f: f + K]
        if sc.kind[i] == 1:
            R = int(sc.r_interior[i])
            B = mu[f + (R + 1) * K: f + (R + 2) * K]
            poly = np.concatenate([A, B[K - 2:0:-1]]) - A[0]
            out[i] = 0.5 * abs(np.sum(_cross(poly, np.roll(poly, -1, axis=0))))
        else:
            out[i] = np.sum(np.linalg.norm(np.diff(A, axis=0), axis=1)) * float(sc.stroke_w[i])
    return out


def area_order(sc, opts=None):
    # The order is an integer decision taken from the areas, so it is taken in
    # the precision the kernels sort in: the FP64 areas rounded to float32,
    # then a stable sort (equal keys keep curve index order).
    a = curve_area(sc, opts).astype(np.float32)
    order = np.argsort(a, kind="stable")
    per = np.where(sc.kind == 1, sc.r_interior + 2, 1) * sc.k_samples
    goff = np.concatenate([[0], np.cumsum(per[order])]).astype(np.int64)
    return a, order.astype(np.int32), goff


def _segments(sc, i):
    """(P0, P1, P2, P3) of every cubic segment of both boundaries of closed curve i."""
    P = np.asarray(sc.ctrl, np.float64).reshape(-1, 2)[sc.ctrl_off[i]: sc.ctrl_off[i + 1]]
    S = int(sc.nseg[i])
    m = 3 * S
    A = P[: m + 1]
    B = np.concatenate([A[:1], P[m + 1:], A[m:]])
    return [bnd[3 * s: 3 * s + 4] for bnd in (A, B) for s in range(S)]


def segment_cost(P) -> float:
    e1, e2, e3 = P[1] - P[0], P[2] - P[1], P[3] - P[2]
    n1, n3 = np.linalg.norm(e1), np.linalg.norm(e3)
    if n1 == 0 or n3 == 0:
        return 0.0
    d1 = _cross(e1, e2) >= 0
    d2 = _cross(e1, e3) / (n1 * n3)
    return float(max(0.0, -d2) if d1 else max(0.0, d2))


def xing_loss(sc, weight: float = 1.0) -> float:
    tot = 0.0
    for i in range(sc.n_curves):
        if sc.kind[i] == 1:
            tot += sum(segment_cost(P) for P in _segments(sc, i))
    return weight * tot
