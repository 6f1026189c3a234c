"""Tile lists (Sec. 3.4): the bucketed builder (pairs emitted into buckets of
256 tile keys, one radix pass inside each bucket) and the two-pass radix sort
of (tile, Gaussian) pairs give the same ranges and ids, bit for bit."""
import sys

import numpy as np
import pytest

from paper_2503_16424_amd import scenes

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return torch


def _lists(torch, sc, radix, tile=(16, 16)):
    from paper_2503_16424_amd import bz
    r = bz.Rasterizer(sc, bz.RenderOptions(tile_w=tile[0], tile_h=tile[1], radix_bins=radix))
    r.sample()
    r.bin()
    if r.ensure_capacity():
        r.bin()
    assert not r.ensure_capacity()
    n = r.pairs_required()
    torch.cuda.synchronize()
    return r.ranges.clone(), r.ids[:n].clone(), n


def _same(torch, sc, tile=(16, 16)):
    a = _lists(torch, sc, False, tile)
    b = _lists(torch, sc, True, tile)
    assert a[2] == b[2] > 0
    if not torch.equal(a[0], b[0]):
        ra, rb = a[0].view(-1, 2).cpu().numpy(), b[0].view(-1, 2).cpu().numpy()
        bad = np.nonzero((ra != rb).any(1))[0]
        raise AssertionError(f"ranges differ on {bad.size} tiles, first {bad[:5].tolist()}: "
                             f"bucketed {ra[bad[:5]].tolist()} radix {rb[bad[:5]].tolist()}")
    if not torch.equal(a[1], b[1]):
        ia, ib = a[1].cpu().numpy(), b[1].cpu().numpy()
        bad = np.nonzero(ia != ib)[0]
        raise AssertionError(f"ids differ at {bad.size} positions, first {bad[:5].tolist()}")
    return a[2]


def _odd_canvas():
    # 63 tiles a row: rows straddle the 256-key buckets
    return scenes.mixed(5, 1000, 600, 60, 80, K=24, R=10, S_open=3, extent=(4.0, 300.0))


@pytest.mark.parametrize("tile", [(16, 16), (32, 8), (8, 8)])
def test_bucketed_lists_equal_radix_lists(torch_cuda, tile):
    _note(f"bucketed vs radix lists, 1000x600, tile {tile}")
    assert _same(torch_cuda, _odd_canvas(), tile) > 1000


def test_bucketed_lists_equal_radix_lists_at_the_bucket_limit(torch_cuda):
    # 256 x 256 tiles of 8 x 8: 65,536 tile keys, the builder's 256 buckets
    _note("bucketed vs radix lists, 2048x2048, tile (8, 8), 256 buckets")
    sc = scenes.mixed(8, 2048, 2048, 150, 300, K=24, R=8, S_open=3, extent=(4.0, 600.0))
    assert _same(torch_cuda, sc, (8, 8)) > 10 ** 5


def test_bucketed_lists_equal_radix_lists_at_paper_scale(torch_cuda):
    _note("bucketed vs radix lists, 2048x2048 20k curves")
    assert _same(torch_cuda, scenes.paper_2048(0)) > 10 ** 7


def test_bucketed_lists_equal_radix_lists_for_a_batch(torch_cuda):
    _note("bucketed vs radix lists, batch of 12 canvases")
    cvs = scenes.batched(3, n_canvas=12, side=(96, 700), curves=(40, 400))
    assert _same(torch_cuda, cvs) > 1000


def test_more_than_65536_tiles_take_the_radix_sort(torch_cuda):
    """A canvas of 263 x 263 tiles is past the bucketed builder's limit: the
    automatic choice is the radix sort, and its lists are sound."""
    from paper_2503_16424_amd import bz
    torch = torch_cuda
    _note("radix fallback, 4200x4200")
    sc = scenes.mixed(6, 4200, 4200, 30, 60, K=24, R=6, S_open=3, extent=(8.0, 900.0))
    lib = bz.load_library()
    import ctypes as C
    o = bz.make_opts(sc.width, sc.height, sc.bg, bz.RenderOptions())
    auto, radix = C.c_int64(0), C.c_int64(0)
    assert lib.bz_workspace_size(C.byref(o), 10 ** 5, 10 ** 6, C.byref(auto)) == bz.BZ_OK
    o.bin_sort = 1
    assert lib.bz_workspace_size(C.byref(o), 10 ** 5, 10 ** 6, C.byref(radix)) == bz.BZ_OK
    assert auto.value == radix.value
    ranges, ids, n = _lists(torch, sc, False)
    assert n > 1000
    rg = ranges.view(-1, 2).cpu().numpy().astype(np.int64)
    assert (rg[:, 1] >= rg[:, 0]).all() and rg[:, 1].max() == n
    idn = ids.cpu().numpy().astype(np.int64)
    for s, e in rg[rg[:, 1] > rg[:, 0] + 1][:2000]:
        assert np.all(np.diff(idn[s:e]) > 0)
