"""Batches of canvases in one tile space, persistent launches and step graphs.

* every canvas of a batch renders bit for bit as it does alone, and matches
  the oracle; its gradients match the oracle's;
* persistent and one-workgroup-per-tile launches give the same bits;
* a recorded step graph, replayed several times with eager work between the
  replays, reproduces the eager step every time;
* the 64-canvas workload (3,988,428 Gaussians over 14.8 Mpx) in the launch
  configuration the benchmark uses: sampled pixels of sampled canvases match
  the oracle, and canvases match their single-canvas renders bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2503_16424_amd import scenes
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5
GRAD_TOL = 1e-3


def _note(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return torch


def _small_batch():
    parts = [scenes.small_mixed(31, W=96, H=80, n_closed=6, n_open=8, K=10, R=4,
                                extent=(6.0, 40.0)),
             scenes.small_mixed(32, W=1, H=1, n_closed=1, n_open=1),
             scenes.tiny_128(0),
             scenes.small_mixed(33, W=131, H=77, n_closed=9, n_open=12, K=12, R=6,
                                extent=(4.0, 60.0)),
             scenes.small_mixed(34, W=17, H=203, n_closed=2, n_open=3, extent=(3.0, 30.0)),
             scenes.uniform_open(35, 40, 24, 0, 8)]                    # no curves at all
    parts[1].bg = np.array([0.2, 0.4, 0.6], np.float32)
    return parts


def _rast(parts, tile=(16, 16), persistent=False, **kw):
    from paper_2503_16424_amd import bz
    ro = bz.RenderOptions(tile_w=tile[0], tile_h=tile[1], persistent=persistent)
    return bz.Rasterizer(parts, ro, **kw)


@pytest.mark.parametrize("tile,persistent", [((16, 16), False), ((16, 16), True),
                                             ((32, 8), True), ((8, 8), False)])
def test_batch_canvases_render_as_alone_and_as_the_oracle(torch_cuda, tile, persistent):
    from paper_2503_16424_amd import bz
    parts = _small_batch()
    _note(f"batch of {len(parts)} canvases, tile {tile}, persistent {persistent}")
    r = _rast(parts, tile, persistent)
    img = r.render()
    for c, sc in enumerate(parts):
        got = r.canvas_view(img, c).cpu().numpy()
        alone = bz.Rasterizer(sc, bz.RenderOptions(tile_w=tile[0], tile_h=tile[1])).render()
        assert np.array_equal(got.view(np.uint32), alone.cpu().numpy().view(np.uint32)), c
        o = oracle.forward_backward(sc)
        assert np.abs(got - o["image"]).max() <= IMG_TOL, c


@pytest.mark.parametrize("state", ["stored", "recompute"])
@pytest.mark.parametrize("persistent", [False, True])
def test_batch_gradients_match_the_oracle_per_canvas(torch_cuda, state, persistent):
    torch = torch_cuda
    parts = _small_batch()
    r = _rast(parts, persistent=persistent, blend_state=state)
    r.render()
    ups, refs = [], []
    for c, sc in enumerate(parts):
        o0 = oracle.forward_backward(sc)
        tgt = scenes.target_noise(40 + c, sc.width, sc.height).astype(np.float64)
        d = 2.0 * (o0["image"] - tgt) / o0["image"].size
        ups.append(d.astype(np.float32))
        refs.append(oracle.forward_backward(sc, d))
    r.backward(torch.as_tensor(r.flat_images(ups), device="cuda"))
    torch.cuda.synchronize()
    c0 = p0 = o0_ = 0
    d_ctrl, d_col = r.d_ctrl.cpu().numpy(), r.d_color.cpu().numpy()
    d_opa, d_w = r.d_opacity.cpu().numpy(), r.d_width.cpu().numpy()
    for c, sc in enumerate(parts):
        n, npt, nop = sc.n_curves, sc.ctrl.reshape(-1, 2).shape[0], sc.opacity.size
        got = dict(d_ctrl=d_ctrl[p0:p0 + npt], d_color=d_col[c0:c0 + n],
                   d_opacity=d_opa[o0_:o0_ + nop], d_width=d_w[c0:c0 + n])
        for k, v in got.items():
            if n == 0 or not np.any(refs[c][k]):
                assert np.all(v == 0.0), (c, k)
                continue
            e = rel_l2(v, refs[c][k])
            assert e <= GRAD_TOL, (c, k, e)
        c0, p0, o0_ = c0 + n, p0 + npt, o0_ + nop


@pytest.mark.parametrize("persistent", [False, True])
def test_step_graph_replays_reproduce_the_eager_step(torch_cuda, persistent):
    torch = torch_cuda
    from paper_2503_16424_amd.graph import StepGraph
    parts = _small_batch()
    r = _rast(parts, persistent=persistent)
    tgt = torch.as_tensor(r.flat_images([scenes.target_noise(50 + c, sc.width, sc.height)
                                         for c, sc in enumerate(parts)]), device="cuda")
    r.render()
    r.step(tgt)
    torch.cuda.synchronize()
    ref_img, ref_ctrl = r.image.clone(), r.d_ctrl.clone()
    ref_loss = float(r.loss.item())
    g = StepGraph(r, tgt)
    for rep in range(4):
        r.image.fill_(-1.0)                        # eager work between the replays
        r.d_ctrl.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.image.view(torch.int32), ref_img.view(torch.int32)), rep
        assert rel_l2(r.d_ctrl.cpu().numpy(), ref_ctrl.cpu().numpy()) <= 1e-5, rep
        assert abs(float(r.loss.item()) - ref_loss) <= 1e-5 * abs(ref_loss), rep


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_forward_fused_with_l2_matches_separate_calls(torch_cuda, persistent):
    """bz_render_fwd_l2 over a batch (a 1x1 canvas and one without curves
    among them): image, blend state and d_image bit for bit as bz_render_fwd
    then bz_l2_grad, the loss within float rounding."""
    torch = torch_cuda
    from tests.helpers import fused_l2_matches_separate
    parts = _small_batch()
    r = _rast(parts, persistent=persistent)
    tgts = [scenes.target_noise(70 + c, sc.width, sc.height) for c, sc in enumerate(parts)]
    flat = r.flat_images(tgts)
    tgt = torch.as_tensor(flat, device="cuda")

    def ref_of(img):
        e = img.cpu().numpy().astype(np.float64) - np.asarray(flat, np.float64)
        return float(np.sum(e * e))
    fused_l2_matches_separate(torch, r, tgt, ref_of)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_batch_sample_bin_matches_separate_calls(torch_cuda, tile):
    """bz_sample_bin over a batch (each Gaussian bounded on its own canvas):
    records and tile lists bit for bit as bz_sample then bz_bin."""
    from tests.helpers import sample_bin_matches_separate
    r = _rast(_small_batch(), tile)
    r.render()
    assert sample_bin_matches_separate(torch_cuda, r) > 0


def test_step_graph_grows_the_pair_buffer_and_records_again(torch_cuda):
    torch = torch_cuda
    from paper_2503_16424_amd.graph import StepGraph
    parts = _small_batch()
    r = _rast(parts, cap_pairs=16)               # grown to ~1.25x the need before recording
    tgt = torch.zeros(3 * r.n_pixels, device="cuda")
    g = StepGraph(r, tgt, slack=1.0)
    cap = r.cap_pairs
    # wider strokes: more pairs than the recorded buffer holds
    r.stroke_w.mul_(3.0)
    assert g.replay(check=True)
    assert r.cap_pairs > cap and g.records == 2
    img = r.image.clone()
    r.render()
    assert torch.equal(img.view(torch.int32), r.image.view(torch.int32))


def test_batched_64_canvases_sampled_parity(torch_cuda):
    """The 64-canvas workload in the benchmark's launch configuration."""
    from paper_2503_16424_amd import bz
    parts = scenes.batched(0)
    _note(f"64 canvases: {sum(p.n_gauss for p in parts)} Gaussians")
    # (16, 32) persistent: the configuration the autotuner picks on this workload
    for tile, persistent in (((16, 16), False), ((16, 16), True), ((16, 32), True)):
        r = _rast(parts, tile, persistent=persistent)
        img = r.render()
        rng = np.random.default_rng(7)
        for c in rng.choice(len(parts), 6, replace=False):
            sc = parts[c]
            got = r.canvas_view(img, int(c)).cpu().numpy()
            if persistent:
                alone = bz.Rasterizer(sc).render().cpu().numpy()
                assert np.array_equal(got.view(np.uint32), alone.view(np.uint32)), c
            g = oracle.sample(sc)
            xs = rng.integers(0, sc.width, 200)
            ys = rng.integers(0, sc.height, 200)
            p = oracle.render_pixels(g, sc.width, sc.height, sc.bg, xs, ys)
            err = np.abs(got[:, ys, xs].T - p["rgb"]).max()
            assert err <= IMG_TOL, (c, err)
        del r


def test_many_tiny_canvases(torch_cuda):
    """300 canvases of 1..40 px sides (many with no curve): every one renders
    bit for bit as alone, with both launch forms."""
    from paper_2503_16424_amd import bz
    rng = np.random.default_rng(61)
    parts = []
    for c in range(300):
        W, H = int(rng.integers(1, 41)), int(rng.integers(1, 41))
        n = int(rng.integers(0, 4))
        parts.append(scenes.uniform_open(1000 + c, W, H, n, int(rng.integers(2, 12))))
    ref = [bz.Rasterizer(sc).render().cpu().numpy() for sc in parts]
    for persistent in (False, True):
        r = _rast(parts, (8, 8), persistent)
        img = r.render()
        for c in range(len(parts)):
            got = r.canvas_view(img, c).cpu().numpy()
            assert np.array_equal(got.view(np.uint32), ref[c].view(np.uint32)), (c, persistent)


def test_step_graph_with_every_option(torch_cuda):
    """Batch + persistent launches + recomputed blend state + area draw order,
    recorded as one graph: replays reproduce the eager step, and the
    gradients match the oracle run on the same draw order."""
    torch = torch_cuda
    from paper_2503_16424_amd.graph import StepGraph
    parts = _small_batch()[:5]
    r = _rast(parts, (16, 8), True, blend_state="recompute", draw_order="area")
    tgts = [scenes.target_noise(70 + c, sc.width, sc.height) for c, sc in enumerate(parts)]
    tgt = torch.as_tensor(r.flat_images(tgts), device="cuda")
    r.render()
    r.step(tgt)
    torch.cuda.synchronize()
    ref_img, ref_ctrl = r.image.clone(), r.d_ctrl.clone()
    g = StepGraph(r, tgt)
    for rep in range(3):
        r.image.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(r.image.view(torch.int32), ref_img.view(torch.int32)), rep
        assert rel_l2(r.d_ctrl.cpu().numpy(), ref_ctrl.cpu().numpy()) <= 1e-5, rep
    # oracle on the concatenated scene in the device's draw order
    order = r.order.cpu().numpy()
    sc = scenes.concat(parts)
    sc.rank = np.empty(sc.n_curves, np.int32)
    sc.rank[order] = np.arange(sc.n_curves, dtype=np.int32)
    # per canvas: each canvas's curves keep their relative area order
    n0 = 0
    d_ref = []
    for c, p in enumerate(parts):
        sub = p.copy()
        rk = sc.rank[n0: n0 + p.n_curves]
        sub.rank = np.argsort(np.argsort(rk)).astype(np.int32)
        o0 = oracle.forward_backward(sub)
        assert np.abs(r.canvas_view(r.image, c).cpu().numpy() - o0["image"]).max() <= IMG_TOL
        d = 2.0 * (o0["image"] - tgts[c].astype(np.float64)) / (3.0 * r.n_pixels)
        d_ref.append(oracle.forward_backward(sub, d)["d_ctrl"])
        n0 += p.n_curves
    assert rel_l2(r.d_ctrl.cpu().numpy(), np.concatenate(d_ref)) <= GRAD_TOL
