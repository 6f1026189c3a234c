"""Per-curve shape terms on the GPU against the FP64 reference.

* areas within 2e-7 relative (FP64 sums rounded to float);
* the device draw order: a permutation, non-decreasing in the areas, ties by
  index, areas equal to the reference's float keys; offsets follow the counts;
* rendering and differentiating in that order matches the oracle run on the
  same order; a recorded step graph with the reordering inside replays it;
* Xing loss within 1e-6 relative; its gradient, added to d_ctrl, matches
  central differences of the reference loss.
"""
import numpy as np
import pytest

import oracle
from oracle import shape_oracle as so
from paper_2503_16424_amd import scenes
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return torch


SCENES = {
    "mixed_small": lambda: scenes.small_mixed(5, W=131, H=77, n_closed=9, n_open=12, K=12, R=6,
                                              extent=(4.0, 60.0)),
    "mixed_R20": lambda: scenes.mixed(3, 200, 168, 40, 30, K=24, R=20, S_open=3,
                                      extent=(4.0, 120.0)),
}


def _check_order(order, goff, area_gpu, sc):
    n = sc.n_curves
    assert sorted(order.tolist()) == list(range(n))
    keys = area_gpu[order]
    assert np.all(np.diff(keys) >= 0)
    same = np.diff(keys) == 0
    assert np.all(np.diff(order)[same] > 0)                       # ties by index
    per = np.where(sc.kind == 1, sc.r_interior + 2, 1) * sc.k_samples
    assert np.array_equal(goff, np.concatenate([[0], np.cumsum(per[order])]))


@pytest.mark.parametrize("name", list(SCENES) + ["paper_2048"])
def test_area_and_order_match_reference(torch_cuda, name):
    from paper_2503_16424_amd import bz
    sc = SCENES[name]() if name in SCENES else scenes.paper_2048(0)
    r = bz.Rasterizer(sc, draw_order="area")
    r.reorder()
    area = r.area.cpu().numpy()[: sc.n_curves]
    ref = so.curve_area(sc)
    assert np.all(np.abs(area - ref) <= 2e-7 * np.abs(ref) + 1e-30)
    ref_keys = ref.astype(np.float32)
    assert np.all(np.abs(area.view(np.int32) - ref_keys.view(np.int32)) <= 1)
    _check_order(r.order.cpu().numpy(), r.gauss_off.cpu().numpy(), area, sc)


def test_render_and_gradients_in_area_order(torch_cuda):
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    sc = SCENES["mixed_R20"]()
    r = bz.Rasterizer(sc, draw_order="area")
    img = r.render().cpu().numpy()
    order = r.order.cpu().numpy()
    s2 = sc.copy()
    s2.rank = np.empty(sc.n_curves, np.int32)
    s2.rank[order] = np.arange(sc.n_curves, dtype=np.int32)
    o0 = oracle.forward_backward(s2)
    assert np.abs(img - o0["image"]).max() <= 1e-5
    tgt = scenes.target_noise(3, sc.width, sc.height).astype(np.float64)
    d = 2.0 * (o0["image"] - tgt) / o0["image"].size
    o = oracle.forward_backward(s2, d)
    r.backward(torch.as_tensor(d.astype(np.float32), device="cuda"))
    torch.cuda.synchronize()
    for k in ("d_ctrl", "d_width", "d_color", "d_opacity"):
        assert rel_l2(getattr(r, k).cpu().numpy(), o[k]) <= 1e-3, k


def test_area_order_inside_a_step_graph(torch_cuda):
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    from paper_2503_16424_amd.graph import StepGraph
    sc = SCENES["mixed_small"]()
    r = bz.Rasterizer(sc, draw_order="area")
    tgt = torch.as_tensor(scenes.target_noise(8, sc.width, sc.height), device="cuda")
    r.step(tgt)
    torch.cuda.synchronize()
    ref_img, ref_order = r.image.clone(), r.order.clone()
    g = StepGraph(r, tgt)
    for rep in range(3):
        r.order.fill_(-1)
        r.image.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.order, ref_order), rep
        assert torch.equal(r.image.view(torch.int32), ref_img.view(torch.int32)), rep


def _xing_scene(seed):
    """Closed curves with random inner control points: many S bends."""
    rng = np.random.default_rng(seed)
    n = 40
    ctrl = []
    for _ in range(n):
        c = rng.uniform(20, 180, 2)
        pts = c + rng.normal(0, 25, (6, 2))
        ctrl.append(pts)
    return scenes._assemble(200, 200, [1] * n, [1] * n, [10] * n, [3] * n, ctrl, np.zeros(n),
                            rng.uniform(0, 1, (n, 3)), [[0.7]] * n, np.arange(n))


def test_xing_loss_and_gradient(torch_cuda):
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    sc = scenes.concat([_xing_scene(11), scenes.small_mixed(12, n_closed=3, n_open=4)])
    r = bz.Rasterizer(sc)
    base = np.random.default_rng(1).standard_normal(r.d_ctrl.shape).astype(np.float32)
    r.d_ctrl.copy_(torch.as_tensor(base))
    w = 0.37
    loss = float(r.xing(w).item())
    ref = so.xing_loss(sc, w)
    assert ref > 0 and abs(loss - ref) <= 1e-6 * ref
    grad = r.d_ctrl.cpu().numpy() - base
    # central differences of the reference loss, point by point
    fd = np.zeros_like(grad, dtype=np.float64)
    ctrl0 = sc.ctrl.astype(np.float64).reshape(-1, 2)
    h = 1e-5
    for j in range(ctrl0.shape[0]):
        for a in range(2):
            s = sc.copy()
            p = ctrl0.copy()
            p[j, a] += h
            s.ctrl = p
            lp = so.xing_loss(s, w)
            p[j, a] -= 2 * h
            s.ctrl = p
            fd[j, a] = (lp - so.xing_loss(s, w)) / (2 * h)
    assert rel_l2(grad, fd) <= 1e-5
    assert np.all(grad[np.repeat(sc.kind, np.diff(sc.ctrl_off)) == 0] == 0)   # open curves: none


def test_area_order_of_a_batch_is_per_canvas(torch_cuda):
    from paper_2503_16424_amd import bz
    parts = [SCENES["mixed_small"](), scenes.small_mixed(21, W=60, H=50, n_closed=5, n_open=6),
             scenes.uniform_open(22, 30, 30, 0, 8), SCENES["mixed_R20"]()]
    r = bz.Rasterizer(parts, draw_order="area")
    r.reorder()
    order = r.order.cpu().numpy()
    area = r.area.cpu().numpy()
    goff = r.gauss_off.cpu().numpy()
    c0 = 0
    for p in parts:
        seg = order[c0: c0 + p.n_curves]
        assert sorted(seg.tolist()) == list(range(c0, c0 + p.n_curves))     # canvas kept together
        local = p.copy()
        _check_order(seg - c0, goff[c0: c0 + p.n_curves + 1] - goff[c0], area[c0: c0 + p.n_curves],
                     local)
        ref = so.curve_area(p)
        assert np.all(np.abs(area[c0: c0 + p.n_curves] - ref) <= 2e-7 * np.abs(ref) + 1e-30)
        c0 += p.n_curves
    img = r.render()
    for c, p in enumerate(parts):
        s2 = p.copy()
        seg = order[sum(q.n_curves for q in parts[:c]):][: p.n_curves] - sum(q.n_curves for q in parts[:c])
        s2.rank = np.empty(p.n_curves, np.int32)
        s2.rank[seg] = np.arange(p.n_curves, dtype=np.int32)
        o = oracle.forward_backward(s2)
        assert np.abs(r.canvas_view(img, c).cpu().numpy() - o["image"]).max() <= 1e-5, c
