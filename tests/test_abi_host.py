"""The C ABI without a GPU: exports, host-side layout and argument validation."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2503_16424_amd import bz, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(bz_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_function():
    from paper_2503_16424_amd import cnn
    lib = bz.load_library()
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(bz.EXPORTS) | set(cnn.EXPORTS)


def test_status_strings():
    lib = bz.load_library()
    for code in (0, -1, -2, -3, -4):
        assert lib.bz_status_str(code)
    assert lib.bz_status_str(7) == b"unknown status"


def test_layout_matches_rank_order():
    sc = scenes.small_mixed(3, n_closed=4, n_open=5)
    order, goff, mg, mk = bz.layout_host(sc)
    assert sorted(order) == list(range(sc.n_curves))
    assert np.all(sc.rank[order] == np.arange(sc.n_curves))
    per = sc.n_gauss_per_curve()[order]
    assert np.array_equal(np.diff(goff), per)
    assert goff[-1] == sc.n_gauss
    assert mg == per.max() and mk == sc.k_samples.max()


@pytest.mark.parametrize("mutate", ["rank_dup", "k_one", "ctrl_count", "opa_count", "tau_short",
                                    "kind", "negative_r"])
def test_layout_rejects_inconsistent_curves(mutate):
    sc = scenes.small_mixed(5, n_closed=3, n_open=3)
    if mutate == "rank_dup":
        sc.rank[1] = sc.rank[0]
    elif mutate == "k_one":
        sc.k_samples[0] = 1
    elif mutate == "ctrl_count":
        sc.ctrl_off[1:] += 1
    elif mutate == "opa_count":
        i = int(np.nonzero(sc.kind == 0)[0][0])
        sc.opa_off[i + 1:] += 1                          # S + 1 opacities
    elif mutate == "tau_short":
        i = int(np.nonzero(sc.kind == 1)[0][0])
        sc.tau_off[i + 1:] -= 1
    elif mutate == "kind":
        sc.kind[0] = 7
    elif mutate == "negative_r":
        i = int(np.nonzero(sc.kind == 1)[0][0])
        sc.r_interior[i] = -1
    with pytest.raises(bz.BzError) as e:
        bz.layout_host(sc)
    assert e.value.code == bz.BZ_ERR_ARG


def test_layout_flags_unsupported_sizes():
    sc = scenes.uniform_open(0, 64, 64, 3, 8, S=1)
    sc.k_samples[1] = 2000
    with pytest.raises(bz.BzError) as e:
        bz.layout_host(sc)
    assert e.value.code == bz.BZ_ERR_UNSUPPORTED


def test_layout_accepts_the_largest_curves_and_rejects_beyond():
    # the largest K for a stroke and the largest R for a short closed curve fit the
    # per-curve kernels' LDS together; R = 254 rows at K = 64 does not
    ok = _max_size_scene()
    bz.layout_host(ok)
    big = _max_size_scene()
    big.k_samples[1] = 64
    with pytest.raises(bz.BzError) as e:
        bz.layout_host(big)
    assert e.value.code == bz.BZ_ERR_UNSUPPORTED


def _max_size_scene():
    from tests.helpers import max_size_scene
    return max_size_scene()


def _opts(**kw):
    ro = bz.RenderOptions(**{k: v for k, v in kw.items() if k in bz.RenderOptions.__dataclass_fields__})
    return bz.make_opts(kw.get("W", 128), kw.get("H", 96), (1, 1, 1), ro)


@pytest.mark.parametrize("tw,th,ok", [(16, 16, True), (8, 8, True), (32, 8, True), (32, 32, True),
                                      (12, 16, False), (4, 16, False), (64, 32, False),
                                      (8, 4, False)])
def test_tile_shape_validation(tw, th, ok):
    lib = bz.load_library()
    o = _opts(tile_w=tw, tile_h=th)
    n = C.c_int64(0)
    st = lib.bz_num_tiles(C.byref(o), C.byref(n))
    assert (st == bz.BZ_OK) == ok
    if ok:
        assert n.value == -(-128 // tw) * -(-96 // th)


@pytest.mark.parametrize("field,value", [("g_min", 0.0), ("g_min", 1.0), ("alpha_max", 0.0),
                                         ("alpha_max", 1.5), ("t_min", -1e-3), ("rho", 0.0),
                                         ("sigma0_sq", -0.1), ("width", 0)])
def test_option_validation(field, value):
    lib = bz.load_library()
    o = _opts()
    setattr(o, field, value)
    n = C.c_int64(0)
    assert lib.bz_num_tiles(C.byref(o), C.byref(n)) == bz.BZ_ERR_ARG


def test_workspace_size_monotone():
    lib = bz.load_library()
    o = _opts()
    sizes = []
    for cap in (0, 1000, 100000, 10 ** 7):
        b = C.c_int64(0)
        assert lib.bz_workspace_size(C.byref(o), 5000, cap, C.byref(b)) == bz.BZ_OK
        sizes.append(b.value)
    # bucketed lists: the packed pairs (4 bytes each) and their digit counts
    assert sizes == sorted(sizes) and 4 * 10 ** 7 < sizes[-1] < 5 * 10 ** 7
    b = C.c_int64(0)
    assert lib.bz_workspace_size(C.byref(o), 5000, 1 << 32, C.byref(b)) == bz.BZ_ERR_ARG
    # the two-pass radix sort keeps keys, a second key array and a second id array
    o.bin_sort = 1
    assert lib.bz_workspace_size(C.byref(o), 5000, 10 ** 7, C.byref(b)) == bz.BZ_OK
    assert b.value > 3 * 4 * 10 ** 7
    o.bin_sort = 2
    assert lib.bz_workspace_size(C.byref(o), 5000, 10 ** 7, C.byref(b)) == bz.BZ_ERR_ARG


def test_device_calls_reject_null_arguments_before_launch():
    """Argument errors are caught on the host, so these calls never touch HIP."""
    lib = bz.load_library()
    o = _opts()
    assert lib.bz_sample(None, C.byref(o), None, None) == bz.BZ_ERR_ARG
    assert lib.bz_sample_bin(None, C.byref(o), None, None, None) == bz.BZ_ERR_ARG
    assert lib.bz_bin(None, C.byref(o), None, None) == bz.BZ_ERR_ARG
    g = bz.Gaussians(10, 10, 0)
    assert lib.bz_bin(C.byref(g), C.byref(o), None, None) == bz.BZ_ERR_ARG
    assert lib.bz_render_fwd(None, None, C.byref(o), None, None, None) == bz.BZ_ERR_ARG
    assert lib.bz_render_bwd(None, None, None, C.byref(o), None, None, None, None) == bz.BZ_ERR_ARG
    assert lib.bz_l2_grad(None, None, 10, C.c_float(1.0), None, None, None) == bz.BZ_ERR_ARG
    assert lib.bz_render_fwd_l2(None, None, C.byref(o), None, None, None, C.c_float(1.0), None,
                                None, None) == bz.BZ_ERR_ARG
    bad = _opts(tile_w=12)
    assert lib.bz_sample(None, C.byref(bad), None, None) == bz.BZ_ERR_ARG


def test_sample_rejects_small_capacity_on_host():
    lib = bz.load_library()
    o = _opts()
    cv = bz.Curves()
    cv.n_curves, cv.n_gauss, cv.max_gauss_per_curve, cv.max_k = 1, 16, 16, 16
    for f in ("kind", "nseg", "k_samples", "r_interior", "ctrl", "ctrl_off", "tau", "tau_off",
              "stroke_w", "color", "opacity", "opa_off", "order", "gauss_off"):
        setattr(cv, f, 4096)                               # never dereferenced on the host
    g = bz.Gaussians(8, 0, 4096)
    assert lib.bz_sample(C.byref(cv), C.byref(o), C.byref(g), None) == bz.BZ_ERR_CAPACITY


def _fake_curves(n_gauss=16):
    cv = bz.Curves()
    cv.n_curves, cv.n_gauss, cv.max_gauss_per_curve, cv.max_k = 1, n_gauss, 16, 16
    for f in ("kind", "nseg", "k_samples", "r_interior", "ctrl", "ctrl_off", "tau", "tau_off",
              "stroke_w", "color", "opacity", "opa_off", "order", "gauss_off"):
        setattr(cv, f, 4096)                               # never dereferenced on the host
    return cv


def _fake_bins(workspace_bytes=1 << 40):
    return bz.Bins(1024, 4096, 4096, 4096, workspace_bytes, 4096)


def test_sample_bin_checks_both_calls_arguments_on_host():
    """bz_sample_bin refuses what bz_sample or bz_bin would, before any launch."""
    lib = bz.load_library()
    o = _opts()
    cv = _fake_curves()
    g = bz.Gaussians(8, 0, 4096)                           # capacity below n_gauss
    assert lib.bz_sample_bin(C.byref(cv), C.byref(o), C.byref(g), C.byref(_fake_bins()),
                             None) == bz.BZ_ERR_CAPACITY
    g = bz.Gaussians(16, 0, 4096)
    assert lib.bz_sample_bin(C.byref(cv), C.byref(o), C.byref(g), None, None) == bz.BZ_ERR_ARG
    assert lib.bz_sample_bin(C.byref(cv), C.byref(o), C.byref(g), C.byref(_fake_bins(256)),
                             None) == bz.BZ_ERR_CAPACITY       # workspace too small
    misaligned = bz.Gaussians(16, 0, 4104)
    assert lib.bz_sample_bin(C.byref(cv), C.byref(o), C.byref(misaligned),
                             C.byref(_fake_bins()), None) == bz.BZ_ERR_ARG


def test_fused_forward_checks_its_loss_arguments_on_host():
    """bz_render_fwd_l2: no target or gradient, d_image on the image itself or
    a non-finite scale are refused before any launch."""
    lib = bz.load_library()
    o = _opts()
    g = bz.Gaussians(16, 16, 4096)
    b = _fake_bins()
    img, tgt, dimg = 8192, 16384, 24576
    for args in ((img, None, 1.0, dimg), (img, tgt, 1.0, None), (img, tgt, 1.0, img),
                 (img, tgt, float("inf"), dimg), (img, tgt, float("nan"), dimg)):
        im, t, sc, d = args
        assert lib.bz_render_fwd_l2(C.byref(g), C.byref(b), C.byref(o), im, None, t, C.c_float(sc),
                                    d, None, None) == bz.BZ_ERR_ARG, args


def _batch_layout(sizes, goff, bg=None, tile=(16, 16)):
    lib = bz.load_library()
    o = bz.make_opts(1, 1, (1.0, 1.0, 1.0), bz.RenderOptions(tile_w=tile[0], tile_h=tile[1]))
    n = len(sizes)
    size = np.ascontiguousarray(sizes, np.int32)
    g = np.ascontiguousarray(goff, np.int64)
    bgp = None if bg is None else np.ascontiguousarray(bg, np.float32).ctypes.data_as(C.c_void_p)
    recs = (bz.Canvas * (n + 1))()
    batch = bz.Batch()
    coff = np.ascontiguousarray(np.arange(n + 1) * 3, np.int32)
    st = lib.bz_batch_layout(C.byref(o), n, size.ctypes.data_as(C.c_void_p), bgp,
                             g.ctypes.data_as(C.c_void_p), coff.ctypes.data_as(C.c_void_p),
                             C.addressof(recs), C.byref(batch))
    return st, recs, batch


def test_batch_records_have_the_c_layout():
    assert C.sizeof(bz.Canvas) == 56
    assert C.sizeof(bz.Batch) == 40
    assert bz.Opts.batch.offset == 56 and C.sizeof(bz.Opts) == 64
    assert bz.Canvas.bg.offset == 40 and bz.Canvas.curve_off.offset == 52


def test_batch_layout_numbers_tiles_and_pixels_canvas_by_canvas():
    sizes = [(17, 9), (1, 1), (128, 40), (33, 200)]
    goff = [0, 10, 10, 500, 777]
    st, recs, batch = _batch_layout(sizes, goff, bg=[[0.1, 0.2, 0.3]] * 4, tile=(32, 8))
    assert st == bz.BZ_OK
    tiles = [((W + 31) // 32) * ((H + 7) // 8) for W, H in sizes]
    pix = [W * H for W, H in sizes]
    for c, (W, H) in enumerate(sizes):
        r = recs[c]
        assert (r.width, r.height) == (W, H)
        assert (r.tiles_x, r.tiles_y) == ((W + 31) // 32, (H + 7) // 8)
        assert r.tile_off == sum(tiles[:c]) and r.pix_off == sum(pix[:c])
        assert r.gauss_off == goff[c] and r.curve_off == 3 * c
        assert abs(r.bg[2] - 0.3) < 1e-7
    end = recs[len(sizes)]
    assert (end.tile_off, end.pix_off, end.gauss_off, end.curve_off) == \
        (sum(tiles), sum(pix), 777, 12)
    assert (batch.n_canvas, batch.n_tiles, batch.n_pixels, batch.n_gauss) == \
        (4, sum(tiles), sum(pix), 777)


@pytest.mark.parametrize("sizes,goff", [
    ([], [0]),                                  # no canvas
    ([(0, 5)], [0, 3]),                         # empty canvas side
    ([(5, 40000)], [0, 3]),                     # side beyond the limit
    ([(5, 5), (5, 5)], [0, 4, 2]),              # Gaussian offsets decrease
    ([(5, 5)], [1, 4]),                         # offsets not from 0
])
def test_batch_layout_rejects_bad_batches(sizes, goff):
    if not sizes:
        lib = bz.load_library()
        o = bz.make_opts(1, 1, (1, 1, 1), bz.RenderOptions())
        assert lib.bz_batch_layout(C.byref(o), 0, None, None, None, None, None,
                                   C.byref(bz.Batch())) == bz.BZ_ERR_ARG
        return
    st, _, _ = _batch_layout(sizes, goff)
    assert st == bz.BZ_ERR_ARG


def test_concatenated_scene_keeps_each_canvas_in_draw_order():
    parts = [scenes.small_mixed(1, n_closed=2, n_open=3), scenes.uniform_open(2, 40, 30, 5, 8)]
    sc = scenes.concat(parts)
    assert sc.n_curves == 10 and sc.n_gauss == parts[0].n_gauss + parts[1].n_gauss
    order, goff, _, _ = bz.layout_host(sc)
    # every curve of the first canvas is drawn before every curve of the second
    assert set(order[:5]) == set(range(5)) and set(order[5:]) == set(range(5, 10))
    assert goff[5] == parts[0].n_gauss
    assert np.array_equal(sc.ctrl[sc.ctrl_off[5]:], parts[1].ctrl.reshape(-1, 2))


def test_conv_shape_validation():
    from paper_2503_16424_amd import cnn
    d = cnn.conv_desc(2, 32, 32, 3, 64, 3, 2, 1)
    assert (d.ho, d.wo) == (16, 16)
    lib = cnn.lib()
    for bad in [(0, 8, 8, 3, 4, 3, 1, 1), (1, 8, 8, 3, 4, 2, 1, 0), (1, 8, 8, 3, 4, 3, 1, 3),
                (1, 1, 1, 3, 4, 3, 1, 0), (1, 8, 8, 3, 4, 3, 0, 1)]:
        assert lib.bz_conv_shape(C.byref(cnn.ConvDesc(*bad, 0, 0))) == bz.BZ_ERR_ARG, bad
    big = cnn.ConvDesc(1 << 15, 256, 256, 64, 64, 3, 1, 1, 0, 0)
    assert lib.bz_conv_shape(C.byref(big)) == bz.BZ_ERR_UNSUPPORTED
    # tensors stay below 2^30 elements (32-bit index arithmetic in the kernels)
    edge = cnn.ConvDesc(1 << 14, 256, 256, 1, 1, 1, 1, 0, 0, 0)
    assert lib.bz_conv_shape(C.byref(edge)) == bz.BZ_ERR_UNSUPPORTED
    below = cnn.ConvDesc((1 << 14) - 1, 256, 256, 1, 1, 1, 1, 0, 0, 0)
    assert lib.bz_conv_shape(C.byref(below)) == bz.BZ_OK
    # a descriptor whose output size was not set by bz_conv_shape is rejected
    d2 = cnn.ConvDesc(2, 32, 32, 3, 64, 3, 2, 1, 15, 16)
    assert lib.bz_conv_fwd(C.byref(d2), 1, 1, None, 0, 1, None, None) == bz.BZ_ERR_ARG
    assert lib.bz_conv_fwd(C.byref(d), None, 1, None, 0, 1, None, None) == bz.BZ_ERR_ARG
    assert lib.bz_conv_fwd(C.byref(d), 1, 1, None, 2, 1, None, None) == bz.BZ_ERR_ARG


def test_peak_probe_arguments_and_work_counts():
    """Rate probes: argument checks happen on the host before any launch, and
    the work counts follow the documented units."""
    import ctypes as C
    lib = bz.load_library()
    w = C.c_double(0.0)
    assert lib.bz_peak_work(0, 1 << 20, 0, C.byref(w)) == bz.BZ_OK and w.value == 2.0 * (1 << 20)
    assert lib.bz_peak_work(1, 256, 10, C.byref(w)) == bz.BZ_OK and w.value == 2.0 * 8 * 10 * 256
    assert lib.bz_peak_work(5, 1024, 3, C.byref(w)) == bz.BZ_OK and w.value == 8 * 3 * 16
    assert lib.bz_peak_work(99, 256, 1, C.byref(w)) == bz.BZ_ERR_ARG
    # null buffer, ragged sizes, unknown kind: rejected without a launch
    assert lib.bz_peak_run(1, 256, 1, None, 1024, None) == bz.BZ_ERR_ARG
    fake = C.c_void_p(16)
    assert lib.bz_peak_run(1, 300, 1, fake, 1 << 20, None) == bz.BZ_ERR_ARG
    assert lib.bz_peak_run(0, 100, 0, fake, 1 << 20, None) == bz.BZ_ERR_ARG
    assert lib.bz_peak_run(0, 1 << 20, 0, fake, 1 << 20, None) == bz.BZ_ERR_ARG
    assert lib.bz_peak_run(42, 256, 1, fake, 1 << 20, None) == bz.BZ_ERR_ARG


def test_static_sample_bin_checks_arguments_and_size_on_host():
    """bz_sample_bin_static refuses bad arguments and workspaces beyond its
    fixed array on the host, before touching the device (none here)."""
    lib = bz.load_library()
    o = _opts()
    g = bz.Gaussians(16, 0, 4096)
    assert lib.bz_sample_bin_static(None, C.byref(o), C.byref(g), C.byref(_fake_bins()),
                                    None) == bz.BZ_ERR_ARG
    assert lib.bz_sample_bin_static(C.byref(_fake_curves()), C.byref(o), C.byref(g), None,
                                    None) == bz.BZ_ERR_ARG
    small_cap = bz.Gaussians(8, 0, 4096)
    assert lib.bz_sample_bin_static(C.byref(_fake_curves()), C.byref(o), C.byref(small_cap),
                                    C.byref(_fake_bins()), None) == bz.BZ_ERR_CAPACITY
    # a pair capacity whose workspace exceeds BZ_STATIC_SCRATCH_BYTES (about 4.3
    # bytes a pair on the bucketed path)
    big = bz.Bins(9 << 20, 4096, 4096, 0, 0, 4096)
    need = C.c_int64(0)
    assert lib.bz_workspace_size(C.byref(o), 16, 9 << 20, C.byref(need)) == bz.BZ_OK
    assert need.value > bz.STATIC_SCRATCH_BYTES
    assert lib.bz_sample_bin_static(C.byref(_fake_curves()), C.byref(o), C.byref(g), C.byref(big),
                                    None) == bz.BZ_ERR_CAPACITY
