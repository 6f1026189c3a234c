"""bz_sample_bin_static (the binning workspace in the library's fixed device
array, for callers that cannot allocate) against bz_sample_bin on the same
inputs: records, status words, tile ranges and tile lists bit for bit, on two
calls in a row, the second with a smaller input (the array then holds the
first call's contents), and a request beyond the array's size rejected on the
host before anything is launched."""
import sys

import numpy as np
import pytest

from paper_2503_16424_amd import scenes

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, file=sys.stderr, flush=True)


def _reference(torch, r):
    """bz_sample_bin's outputs (with its own workspace), then the outputs
    filled with sentinels."""
    r.sample_bin()
    torch.cuda.synchronize()
    if r.ensure_capacity():
        r.sample_bin()
        torch.cuda.synchronize()
    n = r.pairs_required()
    want = dict(rec=r.rec[: 12 * r.n_gauss].clone(), status=r.status[:2].clone(),
                ranges=r.ranges.clone(), ids=r.ids[:n].clone())
    r.rec.fill_(-7.0)
    r.status.fill_(-7)
    r.ranges.fill_(-7)
    r.ids.fill_(-7)
    torch.cuda.synchronize()
    return n, want


def _static_matches(torch, r, n, want):
    r.sample_bin_static()
    torch.cuda.synchronize()
    got = dict(rec=r.rec[: 12 * r.n_gauss], status=r.status[:2], ranges=r.ranges, ids=r.ids[:n])
    assert r.pairs_required() == n
    for k in want:
        assert torch.equal(got[k].view(torch.int32), want[k].view(torch.int32)), k


def test_static_sample_bin_matches_sample_bin_twice_then_smaller():
    import torch
    from paper_2503_16424_amd import bz
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    big = scenes.mixed(4, 512, 384, 60, 200, K=24, R=8, S_open=3, extent=(4.0, 200.0))
    small = scenes.tiny_128(0)
    rs = []
    for sc in (big, small):
        r = bz.Rasterizer(sc, bz.RenderOptions(tile_w=16, tile_h=16))
        n, want = _reference(torch, r)
        rs.append((r, n, want))
    need = bz.C.c_int64(0)
    for r, n, _ in rs:
        bz._check("bz_workspace_size", r.lib.bz_workspace_size(
            bz.C.byref(r.opts), r.n_gauss, r.cap_pairs, bz.C.byref(need)))
        _note(f"scene {r.scene.name}: {r.n_gauss} Gaussians, {n} pairs, workspace "
              f"{need.value} of {bz.STATIC_SCRATCH_BYTES} bytes")
        assert need.value <= bz.STATIC_SCRATCH_BYTES
    (rb, nb, wb), (rsm, ns, ws) = rs
    assert ns < nb and rsm.n_gauss < rb.n_gauss
    _static_matches(torch, rb, nb, wb)
    _static_matches(torch, rsm, ns, ws)
    # the same again: repeated calls keep matching
    _static_matches(torch, rb, nb, wb)
    # a renderer built on the static call's lists matches the plain one
    img_static = rb.forward().cpu().numpy()
    rb.sample_bin()
    img = rb.forward().cpu().numpy()
    assert np.array_equal(img, img_static)


def test_static_sample_bin_rejects_what_does_not_fit():
    import torch
    from paper_2503_16424_amd import bz
    sc = scenes.open_512(0)
    r = bz.Rasterizer(sc, bz.RenderOptions(tile_w=16, tile_h=16), cap_pairs=9 << 20)
    r.status.fill_(-7)
    torch.cuda.synchronize()
    with pytest.raises(bz.BzError) as e:
        r.sample_bin_static()
    assert e.value.code == bz.BZ_ERR_CAPACITY
    torch.cuda.synchronize()
    assert int(r.status[1].item()) == -7      # nothing was launched
