"""Parity of the HIP rasterizer (through the C ABI) with the FP64 CPU oracle.

Bars: images within 1e-5 max abs of the oracle; per-group gradients
(control points, widths, colours, opacities) within 1e-3 relative L2; tile
lists valid and complete; images bitwise identical across tile shapes and
runs.  Inputs come from the seeded scene generator only.
"""
import math
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


def _rast(scene, tile=(16, 16), radix=False, **kw):
    from paper_2503_16424_amd import bz
    ro = bz.RenderOptions(tile_w=tile[0], tile_h=tile[1], radix_bins=radix)
    return bz.Rasterizer(scene, ro, **kw)


def _upstream(scene, img_oracle, seed=7):
    tgt = scenes.target_noise(seed, scene.width, scene.height).astype(np.float64)
    return (2.0 * (img_oracle - tgt) / img_oracle.size).astype(np.float32)


SCENES = {
    "tiny_128": lambda: scenes.tiny_128(0),
    "mixed_small_a": lambda: scenes.small_mixed(1, W=96, H=80, n_closed=6, n_open=8, K=10, R=4,
                                                extent=(6.0, 40.0)),
    "mixed_small_b": lambda: scenes.small_mixed(2, W=131, H=77, n_closed=9, n_open=12, K=12,
                                                R=6, extent=(4.0, 60.0)),
    "mixed_R20": lambda: scenes.mixed(3, 200, 168, 40, 30, K=24, R=20, S_open=3,
                                      extent=(4.0, 120.0)),
}


@pytest.mark.parametrize("name", list(SCENES))
def test_sample_matches_oracle(torch_cuda, name):
    sc = SCENES[name]()
    _note(f"sample parity {name} n_gauss={sc.n_gauss}")
    r = _rast(sc)
    r.sample()
    g = r.gaussians_host()
    o = oracle.sample(sc)
    assert np.abs(g["mu"] - o["mu"]).max() < 1e-6
    # the low part carries what float32 cannot: hi is the rounded mean
    assert np.all(np.abs(g["hi"].astype(np.float64) - o["mu"]) <= np.spacing(np.abs(g["hi"])))
    scale = np.maximum(np.abs(o["conic"][:, 0]), np.abs(o["conic"][:, 2]))[:, None]
    assert (np.abs(g["conic"] - o["conic"]) / scale).max() < 1e-6
    assert np.array_equal(g["opac"], o["opac"].astype(np.float32).astype(np.float64))
    assert np.array_equal(g["color"], o["color"].astype(np.float32).astype(np.float64))
    assert np.array_equal(g["curve"], o["curve"])


def _aabb_tiles(mu, conic, W, H, tw, th, g_min, scale, pad):
    """Tile rectangles of the support bounding box (float64 reference)."""
    P = -math.log(g_min)
    det = conic[:, 0] * conic[:, 2] - conic[:, 1] ** 2
    hx = np.sqrt(2 * P * conic[:, 2] / det) * scale + pad
    hy = np.sqrt(2 * P * conic[:, 0] / det) * scale + pad
    x0 = np.maximum(np.ceil(mu[:, 0] - hx - 0.5), 0)
    x1 = np.minimum(np.floor(mu[:, 0] + hx - 0.5), W - 1)
    y0 = np.maximum(np.ceil(mu[:, 1] - hy - 0.5), 0)
    y1 = np.minimum(np.floor(mu[:, 1] + hy - 0.5), H - 1)
    ok = (x0 <= x1) & (y0 <= y1)
    return ok, (x0 // tw).astype(int), (x1 // tw).astype(int), (y0 // th).astype(int), (y1 // th).astype(int)


def _support_tiles(mu, conic, W, H, tw, th, g_min):
    """(Gaussian, tile) pairs whose tile holds a pixel centre inside the exact
    support ellipse (float64, a relative 1e-9 inside the boundary)."""
    lim = -2.0 * math.log(g_min) * (1.0 - 1e-9)
    ok, x0, x1, y0, y1 = _aabb_tiles(mu, conic, W, H, 1, 1, g_min, 1.0, 1.0)
    tx = -(-W // tw)
    out = set()
    for g in np.nonzero(ok)[0]:
        xs = np.arange(x0[g], x1[g] + 1)
        ys = np.arange(y0[g], y1[g] + 1)
        dx = xs[None, :] + 0.5 - mu[g, 0]
        dy = ys[:, None] + 0.5 - mu[g, 1]
        q = conic[g, 0] * dx * dx + 2 * conic[g, 1] * dx * dy + conic[g, 2] * dy * dy
        iy, ix = np.nonzero(q <= lim)
        for t in set(((ys[iy] // th) * tx + xs[ix] // tw).tolist()):
            out.add((int(g), int(t)))
    return out


@pytest.mark.parametrize("radix", [False, True])
@pytest.mark.parametrize("name", ["tiny_128", "mixed_small_b", "mixed_R20"])
@pytest.mark.parametrize("tile", [(16, 16), (32, 8)])
def test_tile_lists_valid_and_complete(torch_cuda, name, tile, radix):
    sc = SCENES[name]()
    _note(f"tile lists {name} tile={tile} radix={radix}")
    r = _rast(sc, tile, radix)
    r.sample()
    r.bin()
    assert not r.ensure_capacity()
    ranges, ids = r.tile_lists()
    o = oracle.sample(sc)
    tw, th = tile
    tx = -(-sc.width // tw)
    got = set()
    for t, (s, e) in enumerate(ranges):
        lst = ids[s:e]
        assert np.all(np.diff(lst) > 0), "tile list not in strictly increasing draw order"
        got.update((int(g), t) for g in lst)
    assert len(got) == r.pairs_required() == sum(e - s for s, e in ranges)
    gm = oracle.DEFAULTS["g_min"]
    may = _aabb_tiles(o["mu"], o["conic"], sc.width, sc.height, tw, th, gm, 1.0012, 0.02 + 1e-3)
    want_max = set()
    ok, x0, x1, y0, y1 = may
    for g in np.nonzero(ok)[0]:
        for ty in range(y0[g], y1[g] + 1):
            for txx in range(x0[g], x1[g] + 1):
                want_max.add((int(g), ty * tx + txx))
    # required: every tile holding a pixel centre inside the exact support
    # ellipse d^T Q d <= -2 ln g_min (brute force over the box's pixels)
    want_min = _support_tiles(o["mu"], o["conic"], sc.width, sc.height, tw, th, gm)
    assert want_min <= got, f"{len(want_min - got)} required pairs missing"
    assert got <= want_max, f"{len(got - want_max)} pairs outside the padded support box"
    # the lists stay close to the support: at most 10% more pairs than it needs
    assert len(got) <= 1.1 * len(want_min) + 16, (len(got), len(want_min))


@pytest.mark.parametrize("name", list(SCENES) + ["open_512"])
def test_forward_matches_oracle(torch_cuda, name):
    sc = scenes.open_512(0) if name == "open_512" else SCENES[name]()
    _note(f"forward parity {name} n_gauss={sc.n_gauss}")
    r = _rast(sc)
    img = r.render().cpu().numpy().astype(np.float64)
    T = r.t_final.cpu().numpy().astype(np.float64)
    nc = r.n_contrib.cpu().numpy()
    o = oracle.forward_backward(sc)
    err = np.abs(img - o["image"])
    _note(f"  max |img - oracle| = {err.max():.3e}")
    assert err.max() <= IMG_TOL
    assert np.abs(T - o["t_final"]).max() <= IMG_TOL
    # contributor counts: identical except where a float32/float64 decision
    # sits on the support boundary or the termination threshold
    mism = np.mean(nc != o["n_contrib"])
    assert mism < 2e-3
    assert abs(int(nc.sum()) - o["pairs"]) <= 2e-3 * max(o["pairs"], 1)


def test_forward_bitwise_across_tile_shapes_and_runs(torch_cuda):
    sc = SCENES["mixed_small_b"]()
    imgs = []
    for tile in [(16, 16), (8, 8), (32, 8), (8, 32), (16, 8), (32, 32)]:
        r = _rast(sc, tile)
        imgs.append((tile, r.render().cpu().numpy().copy(), r.t_final.cpu().numpy().copy()))
    imgs.append(("again", _rast(sc).render().cpu().numpy().copy(), None))
    ref = imgs[0][1]
    for tile, im, _ in imgs[1:]:
        assert np.array_equal(im.view(np.uint32), ref.view(np.uint32)), f"tile {tile} differs"


@pytest.mark.parametrize("state", ["stored", "recompute"])
@pytest.mark.parametrize("name", list(SCENES) + ["dense_tile", "size_split"])
def test_backward_matches_oracle(torch_cuda, name, state):
    import torch
    from tests.helpers import size_split_scene
    sc = (SCENES[name]() if name in SCENES else
          size_split_scene() if name == "size_split" else _dense_tile_scene())
    _note(f"backward parity {name} n_gauss={sc.n_gauss} blend state {state}")
    o0 = oracle.forward_backward(sc)
    dimg = _upstream(sc, o0["image"])
    o = oracle.forward_backward(sc, dimg.astype(np.float64))
    r = _rast(sc, blend_state=state)
    img = r.render().cpu().numpy()
    assert np.abs(img - o0["image"]).max() <= IMG_TOL
    r.backward(torch.as_tensor(dimg, device="cuda"))
    torch.cuda.synchronize()
    got = dict(d_ctrl=r.d_ctrl.cpu().numpy(), d_width=r.d_width.cpu().numpy(),
               d_color=r.d_color.cpu().numpy(), d_opacity=r.d_opacity.cpu().numpy())
    for k in ("d_ctrl", "d_color", "d_opacity"):
        e = rel_l2(got[k], o[k])
        _note(f"  {k}: rel L2 = {e:.3e}")
        assert e <= GRAD_TOL, k
    if np.any(sc.kind == 0):
        e = rel_l2(got["d_width"], o["d_width"])
        _note(f"  d_width: rel L2 = {e:.3e}")
        assert e <= GRAD_TOL
    assert np.all(got["d_width"][sc.kind == 1] == 0.0)
    dg = r.d_gauss_host()
    for j, label in enumerate(["mu_x", "mu_y", "Qxx", "Qxy", "Qyy", "o", "r", "g", "b"]):
        e = rel_l2(dg[:, j], o["d_gauss"][:, j])
        assert e <= GRAD_TOL, label


@pytest.mark.parametrize("state", ["stored", "recompute"])
def test_backward_across_tile_shapes(torch_cuda, state):
    """Tile shape is a tuning choice: every allowed shape gives the oracle's
    gradients (1 to 16 waves per workgroup)."""
    import torch
    sc = SCENES["mixed_small_b"]()
    o0 = oracle.forward_backward(sc)
    dimg = _upstream(sc, o0["image"])
    o = oracle.forward_backward(sc, dimg.astype(np.float64))
    for tile in [(8, 8), (32, 8), (8, 32), (16, 32), (32, 32)]:
        _note(f"  tile {tile} blend state {state}")
        r = _rast(sc, tile, blend_state=state)
        r.render()
        r.backward(torch.as_tensor(dimg, device="cuda"))
        torch.cuda.synchronize()
        for k in ("d_ctrl", "d_width", "d_color", "d_opacity"):
            assert rel_l2(getattr(r, k).cpu().numpy(), o[k]) <= GRAD_TOL, (tile, k)


def _dense_tile_scene():
    """12,800 faint Gaussians over a 32x32 canvas: every tile list is longer
    than the 8,192 entries whose contribution masks the recomputing backward
    keeps on chip, and no pixel terminates."""
    sc = scenes.uniform_open(21, 32, 32, 400, 32)
    sc.ctrl = (np.float32(10.0) + sc.ctrl * np.float32(12.0 / 32.0)).astype(np.float32)
    sc.opacity = np.random.default_rng(22).uniform(2e-4, 8e-4, sc.opacity.shape).astype(np.float32)
    return sc


def test_recomputed_blend_state_gives_the_stored_state_results(torch_cuda):
    """Same image bits, and per-Gaussian gradients equal up to the order of
    the float atomics, with and without stored blend state."""
    import torch
    for name in ("mixed_R20", "dense_tile"):
        sc = SCENES[name]() if name in SCENES else _dense_tile_scene()
        dimg = torch.as_tensor(_upstream(sc, oracle.forward_backward(sc)["image"]), device="cuda")
        out = {}
        for state in ("stored", "recompute"):
            r = _rast(sc, blend_state=state)
            img = r.render().clone()
            r.backward(dimg)
            torch.cuda.synchronize()
            out[state] = (img, r.d_gauss[: 9 * sc.n_gauss].clone(), r.d_ctrl.clone())
        a, b = out["stored"], out["recompute"]
        assert torch.equal(a[0].view(torch.int32), b[0].view(torch.int32)), name
        e = rel_l2(b[1].cpu().numpy(), a[1].cpu().numpy())
        _note(f"  {name}: per-Gaussian gradients rel L2 {e:.2e}")
        assert e <= 1e-5, name
        assert rel_l2(b[2].cpu().numpy(), a[2].cpu().numpy()) <= 1e-5, name


def test_step_with_l2_kernel_matches_oracle_gradient(torch_cuda):
    """The step (sample, bin, forward fused with the L2 gradient, backward)."""
    import torch
    sc = scenes.tiny_128(0)
    tgt = scenes.tiny_128_target(0)
    r = _rast(sc)
    r.render()
    t = torch.as_tensor(tgt, device="cuda")
    r.step(t)
    torch.cuda.synchronize()
    o0 = oracle.forward_backward(sc)
    d = 2.0 * (o0["image"] - tgt.astype(np.float64)) / o0["image"].size
    o = oracle.forward_backward(sc, d)
    assert np.abs(r.d_image.cpu().numpy() - d).max() < 1e-9
    mse = float(np.mean((o0["image"] - tgt) ** 2))
    assert abs(r.loss.item() / o0["image"].size - mse) < 1e-6
    for k in ("d_ctrl", "d_width", "d_color", "d_opacity"):
        assert rel_l2(getattr(r, k).cpu().numpy(), o[k]) <= GRAD_TOL, k


def test_overflow_is_flagged_and_recovers(torch_cuda):
    sc = SCENES["mixed_small_a"]()
    r = _rast(sc, cap_pairs=16)
    r.sample()
    r.bin()
    from paper_2503_16424_amd import bz
    assert r.flags() & bz.STATUS_OVERFLOW
    need = r.pairs_required()
    assert need > 16
    r.forward()
    assert np.all(np.isnan(r.image.cpu().numpy()))
    import torch
    r.forward_l2(torch.zeros_like(r.image))
    assert np.all(np.isnan(r.image.cpu().numpy()))
    assert np.all(np.isnan(r.d_image.cpu().numpy())) and np.isnan(r.loss.item())
    assert r.ensure_capacity()
    r.bin()
    assert not (r.flags() & bz.STATUS_OVERFLOW)
    img = r.forward().cpu().numpy()
    o = oracle.forward_backward(sc)
    assert np.abs(img - o["image"]).max() <= IMG_TOL


def test_degenerate_scenes(torch_cuda):
    # every curve far outside the canvas
    sc = scenes.small_mixed(9, W=64, H=48)
    sc.ctrl = sc.ctrl + np.float32(5000.0)
    r = _rast(sc)
    img = r.render().cpu().numpy()
    assert np.all(img == 1.0) and r.pairs_required() == 0
    # zero opacity: background exactly
    sc = scenes.small_mixed(10, W=64, H=48)
    sc.opacity[:] = 0.0
    sc.bg = np.array([0.25, 0.5, 0.75], np.float32)
    r = _rast(sc)
    img = r.render().cpu().numpy()
    assert np.all(img == sc.bg[:, None, None])
    assert np.all(r.t_final.cpu().numpy() == 1.0)
    # a one-pixel canvas and a ragged canvas
    for W, H in [(1, 1), (17, 9), (8, 200)]:
        sc = scenes.small_mixed(11, W=W, H=H, n_closed=2, n_open=2, extent=(3.0, 20.0))
        r = _rast(sc)
        img = r.render().cpu().numpy()
        o = oracle.forward_backward(sc)
        assert np.abs(img - o["image"]).max() <= IMG_TOL


def test_paper_scale_sampled_parity(torch_cuda):
    """2048x2048, 20,000 curves (6,528,000 Gaussians) in the benchmark's launch
    configuration: Gaussians sampled one by one, pixels checked one by one."""
    sc = scenes.paper_2048(0)
    _note(f"paper-scale n_gauss={sc.n_gauss}")
    r = _rast(sc)
    img = r.render().cpu().numpy()
    rng = np.random.default_rng(123)
    g = r.gaussians_host()
    o = oracle.sample(sc)
    assert g["mu"].shape == o["mu"].shape
    assert np.abs(g["mu"] - o["mu"]).max() < 1e-6
    scale = np.maximum(np.abs(o["conic"][:, 0]), np.abs(o["conic"][:, 2]))[:, None]
    assert (np.abs(g["conic"] - o["conic"]) / scale).max() < 1e-6
    xs = rng.integers(0, sc.width, 400)
    ys = rng.integers(0, sc.height, 400)
    p = oracle.render_pixels(o, sc.width, sc.height, sc.bg, xs, ys)
    err = np.abs(img[:, ys, xs].T - p["rgb"]).max()
    _note(f"  sampled pixels max err {err:.3e}")
    assert err <= IMG_TOL


def test_split_backward_stages_match_combined_call(torch_cuda):
    """bz_render_bwd_gauss followed by bz_render_bwd_curves gives the same
    gradients as bz_render_bwd; the per-curve stage is deterministic."""
    import torch
    sc = SCENES["mixed_small_b"]()
    o0 = oracle.forward_backward(sc)
    dimg = torch.as_tensor(_upstream(sc, o0["image"]), device="cuda")
    r = _rast(sc)
    r.render()
    r.backward(dimg)
    torch.cuda.synchronize()
    combined = {k: getattr(r, k).clone() for k in ("d_ctrl", "d_width", "d_color", "d_opacity")}
    r.backward_gauss(dimg)
    dg = r.d_gauss.clone()
    r.backward_curves()
    first = {k: getattr(r, k).clone() for k in combined}
    r.backward_curves()
    torch.cuda.synchronize()
    for k in combined:
        assert torch.equal(first[k], getattr(r, k)), f"{k}: stage 2 not deterministic"
        assert rel_l2(first[k].cpu().numpy(), combined[k].cpu().numpy()) <= 1e-6, k
    # stage 2 alone on the oracle's own per-Gaussian gradients
    o = oracle.forward_backward(sc, dimg.cpu().numpy().astype(np.float64))
    r.d_gauss[: 9 * sc.n_gauss].copy_(
        torch.as_tensor(o["d_gauss"].T.astype(np.float32).reshape(-1), device="cuda"))
    r.backward_curves()
    torch.cuda.synchronize()
    for k in ("d_ctrl", "d_width", "d_color", "d_opacity"):
        assert rel_l2(getattr(r, k).cpu().numpy(), o[k]) <= 1e-5, k
    assert rel_l2(dg[: 9 * sc.n_gauss].cpu().numpy(), o["d_gauss"].T.reshape(-1)) <= GRAD_TOL


def test_largest_curves_and_empty_scene(torch_cuda):
    """Per-curve limits (a 4-segment stroke of K = 1024, a closed curve of
    R = 254 rows, together at the per-curve LDS budget) and a scene with no
    curves at all."""
    import torch
    from tests.helpers import max_size_scene
    sc = max_size_scene()
    _note(f"largest curves: n_gauss={sc.n_gauss}")
    o0 = oracle.forward_backward(sc)
    dimg = _upstream(sc, o0["image"])
    o = oracle.forward_backward(sc, dimg.astype(np.float64))
    r = _rast(sc)
    r.sample()
    g = r.gaussians_host()
    assert np.abs(g["mu"] - o0["gauss"]["mu"]).max() < 1e-6
    img = r.render().cpu().numpy()
    assert np.abs(img - o0["image"]).max() <= IMG_TOL
    r.backward(torch.as_tensor(dimg, device="cuda"))
    torch.cuda.synchronize()
    for k in ("d_ctrl", "d_width", "d_color", "d_opacity"):
        assert rel_l2(getattr(r, k).cpu().numpy(), o[k]) <= GRAD_TOL, k
    empty = scenes.uniform_open(3, 40, 24, 0, 8)
    empty.bg = np.array([0.1, 0.2, 0.3], np.float32)
    r = _rast(empty)
    img = r.render().cpu().numpy()
    assert np.all(img == empty.bg[:, None, None]) and r.pairs_required() == 0
    r.backward(torch.zeros((3, 24, 40), device="cuda"))
    torch.cuda.synchronize()
    # the fused step on it: background image, the L2 gradient of the background
    tgt = np.full((3, 24, 40), 0.5, np.float32)
    r.step(torch.as_tensor(tgt, device="cuda"))
    torch.cuda.synchronize()
    assert np.all(r.image.cpu().numpy() == empty.bg[:, None, None]) and r.pairs_required() == 0
    want = np.float32(2.0 / tgt.size) * (np.broadcast_to(empty.bg[:, None, None], tgt.shape) - tgt)
    assert np.array_equal(r.d_image.cpu().numpy(), want)


def test_paper_scale_backward_on_a_band(torch_cuda):
    """2048x2048, 20,000 curves, the benchmark's launch configuration: with
    the image gradient zero outside rows 960..1087, the per-Gaussian and
    per-curve gradients are exactly those of the band, which the oracle
    computes in full."""
    import torch
    sc = scenes.paper_2048(0)
    H, W = sc.height, sc.width
    y0, y1 = 960, 1088
    d = np.zeros((3, H, W))
    d[:, y0:y1] = np.random.default_rng(5).uniform(-1e-6, 1e-6, (3, y1 - y0, W))
    _note("paper-scale backward on rows 960..1087")
    g = oracle.sample(sc)
    ob = oracle.render(g, W, H, sc.bg, rows=(y0, y1), d_image=d)
    oc = oracle.chain(sc, ob["d_gauss"])
    r = _rast(sc)
    r.render()
    r.backward(torch.as_tensor(d.astype(np.float32), device="cuda"))
    torch.cuda.synchronize()
    dg = r.d_gauss_host()
    for j, label in enumerate(["mu_x", "mu_y", "Qxx", "Qxy", "Qyy", "o", "r", "g", "b"]):
        e = rel_l2(dg[:, j], ob["d_gauss"][:, j])
        _note(f"  {label}: rel L2 {e:.2e}")
        assert e <= GRAD_TOL, label
    for k in ("d_ctrl", "d_width", "d_color", "d_opacity"):
        e = rel_l2(getattr(r, k).cpu().numpy(), oc[k])
        _note(f"  {k}: rel L2 {e:.2e}")
        assert e <= GRAD_TOL, k


def _opaque_scene():
    """Overlapping opaque lenses and strokes on a 96x80 canvas: the lens
    interiors are sampled densely, so most pixels stop (T below t_min) after a
    few contributors, many of them in the middle of their tile lists."""
    sc = scenes.mixed(31, 96, 80, 24, 10, K=16, R=8, extent=(30.0, 110.0))
    sc.opacity = np.random.default_rng(32).uniform(0.9, 1.0, sc.opacity.shape).astype(np.float32)
    return sc


@pytest.mark.parametrize("t_min", [1e-6, 1e-2])
@pytest.mark.parametrize("state", ["stored", "recompute"])
def test_stopping_pixels_match_oracle(torch_cuda, t_min, state):
    """Pixels whose blend stops part-way through the tile list: image and
    gradients against the oracle, for both blend-state modes."""
    import torch
    from paper_2503_16424_amd import bz
    sc = _opaque_scene()
    _note(f"stopping pixels t_min={t_min} state={state}")
    opts = dict(t_min=t_min)
    o0 = oracle.forward_backward(sc, opts=opts)
    stopped = float(np.mean(o0["t_final"] < t_min))
    _note(f"  stopped fraction {stopped:.2f}")
    assert stopped > 0.3
    dimg = _upstream(sc, o0["image"])
    o = oracle.forward_backward(sc, dimg.astype(np.float64), opts=opts)
    ro = bz.RenderOptions(t_min=t_min)
    r = bz.Rasterizer(sc, ro, blend_state=state)
    img = r.render().cpu().numpy()
    assert np.abs(img - o0["image"]).max() <= IMG_TOL
    r.backward(torch.as_tensor(dimg, device="cuda"))
    torch.cuda.synchronize()
    for k in ("d_ctrl", "d_width", "d_color", "d_opacity"):
        e = rel_l2(getattr(r, k).cpu().numpy(), o[k])
        _note(f"  {k}: rel L2 {e:.2e}")
        assert e <= GRAD_TOL, k
    if state == "stored":
        # the stored transmittance after each pixel's last contributor
        T = r.t_final.cpu().numpy()
        assert np.abs(T - o0["t_final"]).max() <= 1e-5


def test_l2_gradient_and_loss_on_an_odd_sized_canvas(torch_cuda):
    """131x77 canvas (30,261 values, not a multiple of the kernel's 4-wide
    loads): d_image and the summed squared error against numpy."""
    import torch
    sc = SCENES["mixed_small_b"]()
    r = _rast(sc)
    img = r.render().cpu().numpy().astype(np.float64)
    tgt = scenes.target_noise(4, sc.width, sc.height)
    r.l2_grad(torch.as_tensor(tgt, device="cuda"))
    torch.cuda.synchronize()
    e = img - tgt.astype(np.float64)
    assert img.size % 4 != 0
    assert np.abs(r.d_image.cpu().numpy() - 2.0 * e / img.size).max() <= 1e-9
    assert abs(r.loss.item() - float(np.sum(e * e))) <= 1e-5 * float(np.sum(e * e))


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("state", ["stored", "recompute"])
@pytest.mark.parametrize("name", ["tiny_128", "mixed_small_b", "size_split"])
def test_forward_fused_with_l2_matches_separate_calls(torch_cuda, name, state, persistent):
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    from tests.helpers import fused_l2_matches_separate, size_split_scene
    sc = size_split_scene() if name == "size_split" else SCENES[name]()
    _note(f"fused forward + L2 {name} state {state} persistent {persistent}")
    r = bz.Rasterizer(sc, bz.RenderOptions(persistent=persistent), blend_state=state)
    tgt_np = scenes.target_noise(5, sc.width, sc.height)
    tgt = torch.as_tensor(tgt_np, device="cuda")

    def ref_of(img):
        e = img.cpu().numpy().astype(np.float64) - tgt_np.astype(np.float64)
        return float(np.sum(e * e))
    fused_l2_matches_separate(torch, r, tgt, ref_of)
    # the fused step's gradients are the separate calls' gradients
    o0 = oracle.forward_backward(sc)
    d = 2.0 * (o0["image"] - tgt_np.astype(np.float64)) / o0["image"].size
    assert np.abs(r.d_image.cpu().numpy() - d).max() < 1e-9
    r.backward()
    torch.cuda.synchronize()
    o = oracle.forward_backward(sc, d)
    for k in ("d_ctrl", "d_color", "d_opacity"):
        assert rel_l2(getattr(r, k).cpu().numpy(), o[k]) <= GRAD_TOL, k


@pytest.mark.parametrize("radix", [False, True])
@pytest.mark.parametrize("tile", [(16, 16), (32, 8)])
@pytest.mark.parametrize("name", ["tiny_128", "mixed_small_b", "mixed_R20", "size_split"])
def test_sample_bin_matches_separate_calls(torch_cuda, name, tile, radix):
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    from tests.helpers import sample_bin_matches_separate, size_split_scene
    sc = size_split_scene() if name == "size_split" else SCENES[name]()
    _note(f"sample+bin {name} tile {tile} radix={radix}")
    r = _rast(sc, tile, radix)
    r.render()                                  # sizes the pair buffer
    assert sample_bin_matches_separate(torch, r) > 0
    assert not r.flags() & bz.STATUS_OVERFLOW


@pytest.mark.parametrize("radix", [False, True])
def test_sample_bin_overflow_and_non_finite_flags(torch_cuda, radix):
    """Too small a pair buffer and a NaN control point: bz_sample_bin raises
    the same status bits and counts the same pairs as the two calls."""
    torch = torch_cuda
    from paper_2503_16424_amd import bz
    from tests.helpers import sample_bin_matches_separate
    sc = SCENES["mixed_small_b"]()
    pts = np.array(sc.ctrl, copy=True)
    pts[int(sc.ctrl_off[3])] = np.nan
    sc.ctrl = pts
    r = _rast(sc, radix=radix, cap_pairs=64)
    need = sample_bin_matches_separate(torch, r)
    assert need > 64
    assert r.flags() & bz.STATUS_OVERFLOW and r.flags() & bz.STATUS_NONFINITE


def test_paper_scale_sample_bin_matches_separate_calls(torch_cuda):
    """2048x2048, 20,000 curves: the fused call's records and tile lists are
    those of the two calls, bit for bit."""
    torch = torch_cuda
    from tests.helpers import sample_bin_matches_separate
    sc = scenes.paper_2048(0)
    r = _rast(sc)
    r.render()
    assert sample_bin_matches_separate(torch, r) > 10 ** 7


def test_non_finite_curve_is_skipped_and_flagged(torch_cuda):
    """A NaN control point makes its curve's Gaussians non-finite: binning
    skips them and raises the status bit; the image and every other curve's
    gradients are those of the scene with that curve fully transparent."""
    import torch
    from paper_2503_16424_amd import bz
    sc = SCENES["mixed_small_b"]()
    bad = 3
    s_nan = sc.copy()
    pts = np.array(s_nan.ctrl, copy=True)
    pts[int(s_nan.ctrl_off[bad])] = np.nan
    s_nan.ctrl = pts
    s_ref = sc.copy()
    op = np.array(s_ref.opacity, copy=True)
    op[int(s_ref.opa_off[bad]):int(s_ref.opa_off[bad + 1])] = 0.0
    s_ref.opacity = op
    r = _rast(s_nan)
    img = r.render().cpu().numpy()
    assert r.flags() & bz.STATUS_NONFINITE
    o0 = oracle.forward_backward(s_ref)
    assert np.abs(img - o0["image"]).max() <= IMG_TOL
    dimg = _upstream(s_ref, o0["image"])
    o = oracle.forward_backward(s_ref, dimg.astype(np.float64))
    r.backward(torch.as_tensor(dimg, device="cuda"))
    torch.cuda.synchronize()
    keep = np.arange(sc.n_curves) != bad
    pts_keep = np.ones(sc.ctrl.shape[0], bool)
    pts_keep[int(sc.ctrl_off[bad]):int(sc.ctrl_off[bad + 1])] = False
    opa_keep = np.ones(sc.opacity.shape[0], bool)
    opa_keep[int(sc.opa_off[bad]):int(sc.opa_off[bad + 1])] = False
    for k, sel in (("d_ctrl", pts_keep), ("d_color", keep), ("d_width", keep),
                   ("d_opacity", opa_keep)):
        got = getattr(r, k).cpu().numpy()[sel]
        assert np.all(np.isfinite(got)), k
        assert rel_l2(got, o[k][sel]) <= GRAD_TOL, k
