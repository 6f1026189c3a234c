"""Pins of the shape-term reference (area, draw order, Xing loss) on the CPU.

* a straight stroke covers length x width exactly;
* the lens between a straight boundary and the cubic 3 h t (1 - t) has the
  trapezoid-rule area h L (1/2 - 1/(2 N^2)) on N = K - 1 intervals;
* areas are invariant under translation and scale as s^2 (closed) / s (open
  length, width fixed);
* the order is a stable sort (ties by index) and its offsets follow the
  per-curve Gaussian counts;
* Xing cost in closed form for a known S bend, zero for a convex lens,
  invariant under rotation, translation and mirroring.
"""
import math

import numpy as np
import pytest

from oracle import shape_oracle as so
from paper_2503_16424_amd import scenes


def _closed(ctrl6_list, K=12, R=3, W=256, H=256):
    n = len(ctrl6_list)
    return scenes._assemble(W, H, [1] * n, [1] * n, [K] * n, [R] * n,
                            [np.asarray(c, np.float64) for c in ctrl6_list], np.zeros(n),
                            np.full((n, 3), 0.5), [[0.8]] * n, np.arange(n))


def _open(ctrl4_list, widths, K=9, W=256, H=256):
    n = len(ctrl4_list)
    return scenes._assemble(W, H, [0] * n, [1] * n, [K] * n, [0] * n,
                            [np.asarray(c, np.float64) for c in ctrl4_list], np.asarray(widths),
                            np.full((n, 3), 0.5), [[0.8]] * n, np.arange(n))


def test_straight_stroke_area_is_length_times_width():
    sc = _open([[[10, 20], [40, 60], [70, 100], [100, 140]]], [2.5])
    assert abs(so.curve_area(sc)[0] - 150.0 * 2.5) < 1e-9


@pytest.mark.parametrize("K", [2, 5, 12, 33])
def test_lens_area_closed_form(K):
    L, h = 90.0, 30.0
    x0, y0 = 20.0, 50.0
    # A: straight from (x0, y0) to (x0 + L, y0); B: interior points lifted by h
    ctrl = [[x0, y0], [x0 + L / 3, y0], [x0 + 2 * L / 3, y0], [x0 + L, y0],
            [x0 + L / 3, y0 + h], [x0 + 2 * L / 3, y0 + h]]
    sc = _closed([ctrl], K=K)
    N = K - 1
    assert abs(so.curve_area(sc)[0] - h * L * (0.5 - 0.5 / N ** 2)) < 1e-9 * h * L


def test_area_invariances():
    rng = np.random.default_rng(3)
    sc = scenes.small_mixed(4, W=120, H=90, n_closed=4, n_open=5)
    a = so.curve_area(sc)
    t = sc.copy()
    t.ctrl = (t.ctrl + np.float32([17.0, -9.0])).astype(np.float32)
    assert np.allclose(so.curve_area(t), a, rtol=1e-6, atol=1e-6)
    s = sc.copy()
    s.ctrl = (s.ctrl * np.float32(2.0)).astype(np.float32)
    scale = np.where(sc.kind == 1, 4.0, 2.0)
    assert np.allclose(so.curve_area(s), a * scale, rtol=1e-9)
    assert rng is not None


def test_order_is_stable_and_offsets_follow_counts():
    base = [[10, 10], [20, 10], [30, 10], [40, 10], [20, 20], [30, 20]]
    big = [[10, 10], [50, 10], [90, 10], [130, 10], [50, 60], [90, 60]]
    sc = _closed([big, base, big, base], K=6, R=2)
    a, order, goff = so.area_order(sc)
    assert a[0] == a[2] and a[1] == a[3] and a[1] < a[0]
    assert list(order) == [1, 3, 0, 2]
    assert list(np.diff(goff)) == [6 * 4] * 4 and goff[0] == 0


def test_xing_closed_form_and_invariances():
    # e1 = (1, 0), e2 = (0, 1): left turn (D1 = 1); e3 = (1, -1): D2 = -1/sqrt(2)
    P = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [2.0, 0.0]])
    assert abs(so.segment_cost(P) - 1.0 / math.sqrt(2.0)) < 1e-12
    # convex arc: no cost
    Q = np.array([[0.0, 0.0], [1.0, 1.0], [2.0, 1.0], [3.0, 0.0]])
    assert so.segment_cost(Q) == 0.0
    rot = np.array([[math.cos(0.7), -math.sin(0.7)], [math.sin(0.7), math.cos(0.7)]])
    for M in (rot, np.diag([1.0, -1.0]), np.diag([-1.0, 1.0])):
        assert abs(so.segment_cost(P @ M.T + 5.0) - so.segment_cost(P)) < 1e-12
        assert so.segment_cost(Q @ M.T - 3.0) == 0.0
    # a convex lens costs nothing; bending one boundary into an S costs
    lens = [[10, 10], [30, 0], [60, 0], [80, 10], [30, 30], [60, 30]]
    assert so.xing_loss(_closed([lens])) == 0.0
    # boundary A turns left, then its last edge heads down-right: 1/sqrt(2)
    s_bend = [[10, 10], [40, 10], [40, 40], [70, 10], [30, 30], [50, 30]]
    assert abs(so.xing_loss(_closed([s_bend]), weight=2.0) - 2.0 / math.sqrt(2.0)) < 1e-12


def test_many_equal_areas_keep_index_order():
    small = [[10, 10], [20, 10], [30, 10], [40, 10], [20, 20], [30, 20]]
    big = [[10, 10], [40, 10], [70, 10], [100, 10], [40, 40], [70, 40]]
    sc = _closed([big, small] * 40, K=6, R=2)
    a, order, _ = so.area_order(sc)
    assert list(order) == list(range(1, 80, 2)) + list(range(0, 80, 2))


def test_xing_cost_on_boundary_b():
    # A is convex; B turns left then heads down-right: 1/sqrt(2) from B alone
    ctrl = [[10, 10], [30, 0], [60, 0], [70, 10], [40, 10], [40, 40]]
    assert abs(so.xing_loss(_closed([ctrl])) - 1.0 / math.sqrt(2.0)) < 1e-12
