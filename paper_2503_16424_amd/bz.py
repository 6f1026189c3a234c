"""Thin Python binding of libbz (include/bz.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream, every step of the rasterizer runs in libbz's HIP kernels.  The
binding raises if libbz.so is missing or if no GPU is present; there is no
CPU path.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbz.so")

BZ_OK, BZ_ERR_ARG, BZ_ERR_CAPACITY, BZ_ERR_HIP, BZ_ERR_UNSUPPORTED = 0, -1, -2, -3, -4
STATUS_OVERFLOW = 1
STATUS_NONFINITE = 2
STATUS_LIST_MISMATCH = 4


class Canvas(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("tiles_x", C.c_int32),
                ("tiles_y", C.c_int32), ("tile_off", C.c_int64), ("pix_off", C.c_int64),
                ("gauss_off", C.c_int64), ("bg", C.c_float * 3), ("curve_off", C.c_int32)]


class Batch(C.Structure):
    _fields_ = [("n_canvas", C.c_int32), ("n_tiles", C.c_int64), ("n_pixels", C.c_int64),
                ("n_gauss", C.c_int64), ("canvas", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("bg", C.c_float * 3),
                ("rho", C.c_float), ("sigma0_sq", C.c_float), ("g_min", C.c_float),
                ("alpha_max", C.c_float), ("t_min", C.c_float), ("tile_w", C.c_int32),
                ("tile_h", C.c_int32), ("persistent", C.c_int32), ("bin_sort", C.c_int32),
                ("batch", C.c_void_p)]


class Curves(C.Structure):
    _fields_ = [("n_curves", C.c_int32), ("n_gauss", C.c_int64),
                ("max_gauss_per_curve", C.c_int32), ("max_k", C.c_int32),
                ("kind", C.c_void_p), ("nseg", C.c_void_p), ("k_samples", C.c_void_p),
                ("r_interior", C.c_void_p), ("ctrl", C.c_void_p), ("ctrl_off", C.c_void_p),
                ("tau", C.c_void_p), ("tau_off", C.c_void_p), ("stroke_w", C.c_void_p),
                ("color", C.c_void_p), ("opacity", C.c_void_p), ("opa_off", C.c_void_p),
                ("order", C.c_void_p), ("gauss_off", C.c_void_p)]


class Gaussians(C.Structure):
    _fields_ = [("cap", C.c_int64), ("n", C.c_int64), ("rec", C.c_void_p)]


class Bins(C.Structure):
    _fields_ = [("cap_pairs", C.c_int64), ("ids", C.c_void_p), ("ranges", C.c_void_p),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_int64),
                ("status", C.c_void_p)]


class PixState(C.Structure):
    _fields_ = [("t_final", C.c_void_p), ("n_last", C.c_void_p), ("n_contrib", C.c_void_p),
                ("visit", C.c_void_p), ("visit_words", C.c_int64)]


class Grads(C.Structure):
    _fields_ = [("d_ctrl", C.c_void_p), ("d_width", C.c_void_p), ("d_color", C.c_void_p),
                ("d_opacity", C.c_void_p), ("d_gauss", C.c_void_p)]


EXPORTS = ("bz_layout_host", "bz_workspace_size", "bz_num_tiles", "bz_batch_layout",
           "bz_visit_words", "bz_sample", "bz_sample_bin", "bz_bin",
           "bz_render_fwd", "bz_render_fwd_l2", "bz_render_bwd", "bz_render_bwd_gauss", "bz_render_bwd_curves",
           "bz_curve_area", "bz_area_order_workspace", "bz_area_order", "bz_xing_loss",
           "bz_l2_grad", "bz_status_str", "bz_peak_run", "bz_peak_work",
           "bz_sample_bin_static")

STATIC_SCRATCH_BYTES = 32 * 1024 * 1024   # BZ_STATIC_SCRATCH_BYTES of bz.h

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libbz.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libbz.so not found at {path}; build it with "
                           "`python -m paper_2503_16424_amd.build`")
    lib = C.CDLL(path)
    P = C.POINTER
    lib.bz_status_str.restype = C.c_char_p
    lib.bz_status_str.argtypes = [C.c_int]
    lib.bz_layout_host.restype = C.c_int
    lib.bz_layout_host.argtypes = [C.c_int32] + [C.c_void_p] * 10 + [P(C.c_int32), P(C.c_int32)]
    lib.bz_workspace_size.restype = C.c_int
    lib.bz_workspace_size.argtypes = [P(Opts), C.c_int64, C.c_int64, P(C.c_int64)]
    lib.bz_num_tiles.restype = C.c_int
    lib.bz_num_tiles.argtypes = [P(Opts), P(C.c_int64)]
    lib.bz_batch_layout.restype = C.c_int
    lib.bz_batch_layout.argtypes = [P(Opts), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, P(Batch)]
    lib.bz_visit_words.restype = C.c_int
    lib.bz_visit_words.argtypes = [P(Opts), C.c_int64, P(C.c_int64)]
    lib.bz_sample.restype = C.c_int
    lib.bz_sample.argtypes = [P(Curves), P(Opts), P(Gaussians), C.c_void_p]
    lib.bz_sample_bin.restype = C.c_int
    lib.bz_sample_bin.argtypes = [P(Curves), P(Opts), P(Gaussians), P(Bins), C.c_void_p]
    lib.bz_sample_bin_static.restype = C.c_int
    lib.bz_sample_bin_static.argtypes = [P(Curves), P(Opts), P(Gaussians), P(Bins), C.c_void_p]
    lib.bz_bin.restype = C.c_int
    lib.bz_bin.argtypes = [P(Gaussians), P(Opts), P(Bins), C.c_void_p]
    lib.bz_render_fwd.restype = C.c_int
    lib.bz_render_fwd.argtypes = [P(Gaussians), P(Bins), P(Opts), C.c_void_p, P(PixState),
                                  C.c_void_p]
    lib.bz_render_fwd_l2.restype = C.c_int
    lib.bz_render_fwd_l2.argtypes = [P(Gaussians), P(Bins), P(Opts), C.c_void_p, P(PixState),
                                     C.c_void_p, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.bz_render_bwd.restype = C.c_int
    lib.bz_render_bwd.argtypes = [P(Curves), P(Gaussians), P(Bins), P(Opts), C.c_void_p,
                                  P(PixState), P(Grads), C.c_void_p]
    lib.bz_render_bwd_gauss.restype = C.c_int
    lib.bz_render_bwd_gauss.argtypes = [P(Gaussians), P(Bins), P(Opts), C.c_void_p, P(PixState),
                                        C.c_void_p, C.c_void_p]
    lib.bz_render_bwd_curves.restype = C.c_int
    lib.bz_render_bwd_curves.argtypes = [P(Curves), P(Opts), C.c_void_p, P(Grads), C.c_void_p]
    lib.bz_curve_area.restype = C.c_int
    lib.bz_curve_area.argtypes = [P(Curves), C.c_void_p, C.c_void_p]
    lib.bz_area_order_workspace.restype = C.c_int
    lib.bz_area_order_workspace.argtypes = [C.c_int32, P(C.c_int64)]
    lib.bz_area_order.restype = C.c_int
    lib.bz_area_order.argtypes = [P(Curves), P(Opts), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_int64, C.c_void_p]
    lib.bz_xing_loss.restype = C.c_int
    lib.bz_xing_loss.argtypes = [P(Curves), C.c_float, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.bz_l2_grad.restype = C.c_int
    lib.bz_l2_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p,
                               C.c_void_p, C.c_void_p]
    lib.bz_peak_run.restype = C.c_int
    lib.bz_peak_run.argtypes = [C.c_int32, C.c_int64, C.c_int32, C.c_void_p, C.c_int64,
                                C.c_void_p]
    lib.bz_peak_work.restype = C.c_int
    lib.bz_peak_work.argtypes = [C.c_int32, C.c_int64, C.c_int32, P(C.c_double)]
    _lib = lib
    return lib


class BzError(RuntimeError):
    def __init__(self, fn: str, code: int):
        msg = load_library().bz_status_str(code).decode()
        super().__init__(f"{fn} failed: {msg} ({code})")
        self.code = code


def _check(fn, code):
    if code != BZ_OK:
        raise BzError(fn, code)


@dataclass
class RenderOptions:
    rho: float = 2.0
    sigma0_sq: float = 0.3
    g_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-6
    tile_w: int = 16
    tile_h: int = 16
    persistent: bool = False
    # tile lists: False = automatic (bucketed emission when it applies), True =
    # always the two-pass radix sort; the lists are the same either way
    radix_bins: bool = False

    def as_dict(self):
        return dict(rho=self.rho, sigma0_sq=self.sigma0_sq, g_min=self.g_min,
                    alpha_max=self.alpha_max, t_min=self.t_min)


def make_opts(width, height, bg, ro: RenderOptions) -> Opts:
    o = Opts()
    o.width, o.height = int(width), int(height)
    for i in range(3):
        o.bg[i] = float(bg[i])
    o.rho, o.sigma0_sq, o.g_min = ro.rho, ro.sigma0_sq, ro.g_min
    o.alpha_max, o.t_min = ro.alpha_max, ro.t_min
    o.tile_w, o.tile_h = int(ro.tile_w), int(ro.tile_h)
    o.persistent = int(bool(ro.persistent))
    o.bin_sort = int(bool(ro.radix_bins))
    o.batch = None
    return o


def layout_host(scene):
    """order / gauss_off / max sizes of a scene (host call into libbz)."""
    lib = load_library()
    n = scene.n_curves
    a = {k: np.ascontiguousarray(getattr(scene, k), np.int32)
         for k in ("kind", "nseg", "k_samples", "r_interior", "ctrl_off", "tau_off", "opa_off",
                   "rank")}
    order = np.zeros(max(n, 1), np.int32)
    goff = np.zeros(n + 1, np.int64)
    mg, mk = C.c_int32(0), C.c_int32(0)
    p = lambda x: x.ctypes.data_as(C.c_void_p)
    st = lib.bz_layout_host(n, p(a["kind"]), p(a["nseg"]), p(a["k_samples"]),
                            p(a["r_interior"]), p(a["ctrl_off"]), p(a["tau_off"]),
                            p(a["opa_off"]), p(a["rank"]), p(order), p(goff), C.byref(mg),
                            C.byref(mk))
    _check("bz_layout_host", st)
    return order[:n], goff, int(mg.value), int(mk.value)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


class Rasterizer:
    """Device buffers of one scene and the four library calls on them.

    Curve parameters live in float32 device tensors (``ctrl``, ``stroke_w``,
    ``color``, ``opacity``) that an optimiser may update in place; gradients
    land in ``d_ctrl``, ``d_width``, ``d_color``, ``d_opacity`` after
    :meth:`backward`.

    ``blend_state="stored"`` keeps the forward pass's per-pixel state (T after
    the last contributor, a bound on its list position) and per-batch contribution masks
    for the backward; ``"recompute"`` keeps none of it and the backward
    recomputes it tile by tile (one more sweep of the tile lists).
    """

    def __init__(self, scene, opts: RenderOptions | None = None, device: str = "cuda",
                 cap_pairs: int | None = None, blend_state: str = "stored",
                 draw_order: str = "rank"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libbz needs a GPU; none is visible")
        self.lib = load_library()
        self.torch = torch
        self.dev = torch.device(device)
        self.ro = opts or RenderOptions()
        if blend_state not in ("stored", "recompute"):
            raise ValueError("blend_state is 'stored' or 'recompute'")
        if draw_order not in ("rank", "area"):
            raise ValueError("draw_order is 'rank' (the scene's) or 'area' (Sec. 3.3)")
        self.draw_order = draw_order
        self.recompute = blend_state == "recompute"
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=self.dev)
        self.canvases = None
        if isinstance(scene, (list, tuple)):             # a batch of canvases
            from .scenes import concat
            self.canvases = list(scene)
            scene = concat(self.canvases)
        self.scene = scene
        self.W, self.H = scene.width, scene.height
        self.opts = make_opts(self.W, self.H, scene.bg, self.ro)
        order, goff, mg, mk = layout_host(scene)
        self.n_gauss = int(goff[-1])
        self.n_pixels = self.W * self.H
        if self.canvases is not None:
            n = len(self.canvases)
            curve_off = np.concatenate([[0], np.cumsum([c.n_curves for c in self.canvases])])
            coff32 = np.ascontiguousarray(curve_off, np.int32)
            size = np.array([[c.width, c.height] for c in self.canvases], np.int32)
            bg = np.array([np.asarray(c.bg, np.float32) for c in self.canvases], np.float32)
            cgoff = np.ascontiguousarray(goff[curve_off], np.int64)
            recs = (Canvas * (n + 1))()
            self.batch = Batch()
            p = lambda x: x.ctypes.data_as(C.c_void_p)
            _check("bz_batch_layout", self.lib.bz_batch_layout(
                C.byref(self.opts), n, p(size), p(bg), p(cgoff), p(coff32), C.addressof(recs),
                C.byref(self.batch)))
            raw = np.frombuffer(bytes(recs), np.uint8).copy()
            self.canvas_table = t(raw, torch.uint8)
            self.batch.canvas = self.canvas_table.data_ptr()
            self.opts.batch = C.addressof(self.batch)
            self.canvas_host = [(r.width, r.height, r.pix_off) for r in recs[:n]]
            self.n_pixels = int(self.batch.n_pixels)
        i32, f32 = torch.int32, torch.float32
        self.kind = t(scene.kind, i32)
        self.nseg = t(scene.nseg, i32)
        self.k_samples = t(scene.k_samples, i32)
        self.r_interior = t(scene.r_interior, i32)
        self.ctrl = t(np.asarray(scene.ctrl, np.float32).reshape(-1, 2), f32)
        self.ctrl_off = t(scene.ctrl_off, i32)
        self.tau = t(np.asarray(scene.tau, np.float32), f32)
        self.tau_off = t(scene.tau_off, i32)
        self.stroke_w = t(np.asarray(scene.stroke_w, np.float32), f32)
        self.color = t(np.asarray(scene.color, np.float32).reshape(-1, 3), f32)
        self.opacity = t(np.asarray(scene.opacity, np.float32), f32)
        self.opa_off = t(scene.opa_off, i32)
        self.order = t(order, i32)
        self.gauss_off = t(goff, torch.int64)
        cv = Curves()
        cv.n_curves, cv.n_gauss = scene.n_curves, self.n_gauss
        cv.max_gauss_per_curve, cv.max_k = mg, mk
        for f in ("kind", "nseg", "k_samples", "r_interior", "ctrl", "ctrl_off", "tau", "tau_off",
                  "stroke_w", "color", "opacity", "opa_off", "order", "gauss_off"):
            setattr(cv, f, _ptr(getattr(self, f)).value)
        self.curves = cv
        # Gaussians
        self.rec = torch.empty(max(self.n_gauss, 1) * 12, dtype=f32, device=self.dev)
        self.gauss = Gaussians(self.n_gauss, 0, _ptr(self.rec).value)
        # tiles
        nt = C.c_int64(0)
        _check("bz_num_tiles", self.lib.bz_num_tiles(C.byref(self.opts), C.byref(nt)))
        self.n_tiles = int(nt.value)
        self.ranges = torch.zeros(2 * self.n_tiles, dtype=torch.int32, device=self.dev)
        self.status = torch.zeros(4, dtype=torch.int64, device=self.dev)
        # image and state: [3][H][W] and [H][W], or flat over the canvases of a batch
        HW = self.n_pixels
        ishape = (3 * HW,) if self.canvases is not None else (3, self.H, self.W)
        pshape = (HW,) if self.canvases is not None else (self.H, self.W)
        self.image = torch.empty(ishape, dtype=f32, device=self.dev)
        if self.recompute:         # no per-pixel state: the backward recomputes it per tile
            self.t_final = self.n_last = self.n_contrib = None
            self.state = None
        else:
            self.t_final = torch.empty(pshape, dtype=f32, device=self.dev)
            self.n_last = torch.empty(pshape, dtype=torch.int32, device=self.dev)
            self.n_contrib = torch.empty(pshape, dtype=torch.int32, device=self.dev)
            self.state = PixState(_ptr(self.t_final).value, _ptr(self.n_last).value,
                                  _ptr(self.n_contrib).value, None, 0)
        self._alloc_pairs(cap_pairs if cap_pairs is not None else max(4 * self.n_gauss, 1 << 16))
        # gradients
        self.d_image = torch.empty(ishape, dtype=f32, device=self.dev)
        self.d_ctrl = torch.empty_like(self.ctrl)
        self.d_width = torch.empty_like(self.stroke_w)
        self.d_color = torch.empty_like(self.color)
        self.d_opacity = torch.empty_like(self.opacity)
        self.d_gauss = torch.empty(max(9 * self.n_gauss, 1), dtype=f32, device=self.dev)
        self.grads = Grads(_ptr(self.d_ctrl).value, _ptr(self.d_width).value,
                           _ptr(self.d_color).value, _ptr(self.d_opacity).value,
                           _ptr(self.d_gauss).value)
        self.loss = torch.zeros(1, dtype=f32, device=self.dev)
        self.xing_value = torch.zeros(1, dtype=f32, device=self.dev)
        self._hw = HW
        self.area = torch.zeros(max(scene.n_curves, 1), dtype=f32, device=self.dev)
        if draw_order == "area":
            wb = C.c_int64(0)
            _check("bz_area_order_workspace",
                   self.lib.bz_area_order_workspace(scene.n_curves, C.byref(wb)))
            self.order_ws = torch.empty(int(wb.value) + 256, dtype=torch.uint8, device=self.dev)
            self._order_ws_ptr = (self.order_ws.data_ptr() + 255) & ~255
            self._order_ws_bytes = int(wb.value)

    # -- capacity ------------------------------------------------------------
    def _alloc_pairs(self, cap: int):
        torch = self.torch
        cap = int(min(max(cap, 1), (1 << 32) - 1))
        self.cap_pairs = cap
        self.ids = torch.empty(cap, dtype=torch.int32, device=self.dev)
        wsb = C.c_int64(0)
        _check("bz_workspace_size", self.lib.bz_workspace_size(C.byref(self.opts), self.n_gauss,
                                                               cap, C.byref(wsb)))
        self.workspace = torch.empty(int(wsb.value) + 256, dtype=torch.uint8, device=self.dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.bins = Bins(cap, _ptr(self.ids).value, _ptr(self.ranges).value, aligned,
                         int(wsb.value), _ptr(self.status).value)
        if self.state is None:
            return
        vw = C.c_int64(0)
        _check("bz_visit_words", self.lib.bz_visit_words(C.byref(self.opts), cap, C.byref(vw)))
        self.visit = torch.empty(int(vw.value), dtype=torch.int64, device=self.dev)
        self.state.visit = _ptr(self.visit).value
        self.state.visit_words = int(vw.value)

    def pairs_required(self) -> int:
        """Pair count of the last bz_bin (synchronises)."""
        return int(self.status[0].item())

    def flags(self) -> int:
        return int(self.status[1].item())

    def ensure_capacity(self, slack: float = 1.25) -> bool:
        """After a bz_bin: grow the pair buffer if it overflowed (synchronises).
        Returns True when it had to grow (the caller then bins again)."""
        f = self.flags()
        if f & STATUS_LIST_MISMATCH:
            raise RuntimeError("libbz tile lists inconsistent (emitted tiles differ from counts)")
        if f & STATUS_OVERFLOW:
            self._alloc_pairs(int(math.ceil(self.pairs_required() * slack)) + 1024)
            return True
        return False

    # -- batches -----------------------------------------------------------------
    def canvas_view(self, t, c: int):
        """Canvas c's [3, H, W] block of a flat batch image (or [H, W] block of
        a flat per-pixel array)."""
        W, H, off = self.canvas_host[c]
        if t.numel() == 3 * self.n_pixels:
            return t.view(-1)[3 * off: 3 * off + 3 * W * H].view(3, H, W)
        return t.view(-1)[off: off + W * H].view(H, W)

    def flat_images(self, imgs):
        """Concatenate per-canvas [3, H, W] arrays into the flat batch layout."""
        return np.concatenate([np.asarray(a, np.float32).reshape(-1) for a in imgs])

    # -- parameters --------------------------------------------------------------
    def set_params(self, ctrl=None, stroke_w=None, color=None, opacity=None):
        """Copy new curve parameters into the device buffers the curve set points
        at (shapes must match; the layout - kinds, S, K, R, draw order - is fixed
        at construction)."""
        for dst, src in ((self.ctrl, ctrl), (self.stroke_w, stroke_w), (self.color, color),
                         (self.opacity, opacity)):
            if src is None:
                continue
            src = self.torch.as_tensor(src, device=self.dev)
            if src.numel() != dst.numel():
                raise ValueError(f"parameter has {src.numel()} values, the curve set {dst.numel()}")
            dst.copy_(src.detach().reshape(dst.shape))

    # -- library calls ---------------------------------------------------------
    def _state_arg(self, count: bool = True):
        """The blend state for the library; count=False leaves out the
        per-pixel contributor counts (a diagnostic nothing downstream reads;
        the forward is ~3% faster without them)."""
        if self.state is None:
            return None
        if count:
            return C.byref(self.state)
        st = PixState(self.state.t_final, self.state.n_last, None, self.state.visit,
                      self.state.visit_words)
        return C.byref(st)

    def curve_area(self):
        """Per-curve areas (by curve index) into ``area``."""
        _check("bz_curve_area", self.lib.bz_curve_area(C.byref(self.curves), _ptr(self.area),
                                                       _stream()))
        return self.area

    def reorder(self):
        """Draw order by area (smallest in front), on the device, into the
        ``order`` / ``gauss_off`` the curve set points at."""
        _check("bz_area_order", self.lib.bz_area_order(
            C.byref(self.curves), C.byref(self.opts), _ptr(self.area), _ptr(self.order),
            _ptr(self.gauss_off), C.c_void_p(self._order_ws_ptr), self._order_ws_bytes,
            _stream()))

    def xing(self, weight: float):
        """Xing loss of the closed curves into ``xing_value``; weight times its
        gradient is added to ``d_ctrl``."""
        _check("bz_xing_loss", self.lib.bz_xing_loss(C.byref(self.curves), C.c_float(weight),
                                                     _ptr(self.xing_value), _ptr(self.d_ctrl),
                                                     _stream()))
        return self.xing_value

    def sample(self):
        if self.draw_order == "area":
            self.reorder()
        _check("bz_sample", self.lib.bz_sample(C.byref(self.curves), C.byref(self.opts),
                                               C.byref(self.gauss), _stream()))

    def sample_bin(self):
        """sample and bin in one call: the sampler also does the binning's
        counting pass; records and tile lists as from the two calls."""
        if self.draw_order == "area":
            self.reorder()
        _check("bz_sample_bin", self.lib.bz_sample_bin(C.byref(self.curves), C.byref(self.opts),
                                                       C.byref(self.gauss), C.byref(self.bins),
                                                       _stream()))

    def sample_bin_static(self):
        """sample_bin with the binning workspace in the library's fixed device
        array (bz_sample_bin_static: allocates nothing; limited to
        STATIC_SCRATCH_BYTES of workspace)."""
        if self.draw_order == "area":
            self.reorder()
        _check("bz_sample_bin_static", self.lib.bz_sample_bin_static(
            C.byref(self.curves), C.byref(self.opts), C.byref(self.gauss), C.byref(self.bins),
            _stream()))

    def bin(self):
        _check("bz_bin", self.lib.bz_bin(C.byref(self.gauss), C.byref(self.opts),
                                         C.byref(self.bins), _stream()))

    def forward(self):
        _check("bz_render_fwd", self.lib.bz_render_fwd(C.byref(self.gauss), C.byref(self.bins),
                                                       C.byref(self.opts), _ptr(self.image),
                                                       self._state_arg(), _stream()))
        return self.image

    def backward(self, d_image=None):
        d = self.d_image if d_image is None else d_image
        _check("bz_render_bwd", self.lib.bz_render_bwd(C.byref(self.curves), C.byref(self.gauss),
                                                       C.byref(self.bins), C.byref(self.opts),
                                                       _ptr(d), self._state_arg(),
                                                       C.byref(self.grads), _stream()))

    def backward_gauss(self, d_image=None):
        """Stage 1 only: per-Gaussian gradients into ``d_gauss``."""
        d = self.d_image if d_image is None else d_image
        _check("bz_render_bwd_gauss", self.lib.bz_render_bwd_gauss(
            C.byref(self.gauss), C.byref(self.bins), C.byref(self.opts), _ptr(d),
            self._state_arg(), _ptr(self.d_gauss), _stream()))

    def backward_curves(self):
        """Stage 2 only: ``d_gauss`` -> per-curve gradients."""
        _check("bz_render_bwd_curves", self.lib.bz_render_bwd_curves(
            C.byref(self.curves), C.byref(self.opts), _ptr(self.d_gauss), C.byref(self.grads),
            _stream()))

    def l2_grad(self, target, scale=None):
        """d_image = scale (image - target), scale defaults to 2 / (3 H W) (mean
        squared error); loss accumulates sum (image - target)^2."""
        n = 3 * self._hw
        s = 2.0 / n if scale is None else scale
        _check("bz_l2_grad", self.lib.bz_l2_grad(_ptr(self.image), _ptr(target), n, C.c_float(s),
                                                 _ptr(self.d_image), _ptr(self.loss), _stream()))

    def forward_l2(self, target, scale=None, count: bool = False):
        """forward and l2_grad in one pass: the image and blend state of
        ``forward``, ``d_image`` bit for bit as ``l2_grad`` writes it, ``loss``
        summed in another order.  The contributor counts ``n_contrib`` are
        written only with ``count``."""
        s = 2.0 / (3 * self._hw) if scale is None else scale
        _check("bz_render_fwd_l2", self.lib.bz_render_fwd_l2(
            C.byref(self.gauss), C.byref(self.bins), C.byref(self.opts), _ptr(self.image),
            self._state_arg(count), _ptr(target), C.c_float(s), _ptr(self.d_image),
            _ptr(self.loss), _stream()))
        return self.image

    def render(self):
        """sample + bin + forward, growing the pair buffer when needed (synchronises)."""
        self.sample()
        self.bin()
        if self.ensure_capacity():
            self.bin()
        return self.forward()

    def step(self, target):
        """One fwd+bwd of the mean squared error against ``target`` (no sync)."""
        self.sample_bin()
        self.forward_l2(target)
        self.backward()

    # -- host views --------------------------------------------------------------
    def gaussians_host(self) -> dict:
        r = self.rec[: 12 * self.n_gauss].view(-1, 12).cpu().numpy()
        mu = r[:, 0:2].astype(np.float64) + r[:, 2:4].astype(np.float64)
        # conic from the principal-frame shape: Q = e e^T + k^2 e' e'^T
        ex, ey, k = (r[:, j].astype(np.float64) for j in (4, 5, 6))
        k2 = k * k
        conic = np.stack([ex * ex + k2 * ey * ey, ex * ey * (1.0 - k2), ey * ey + k2 * ex * ex], 1)
        return dict(mu=mu, conic=conic, shape=r[:, 4:7].copy(), opac=r[:, 7].astype(np.float64),
                    color=r[:, 8:11].astype(np.float64), curve=r[:, 11].view(np.int32).copy(),
                    hi=r[:, 0:2].copy(), lo=r[:, 2:4].copy())

    def d_gauss_host(self) -> np.ndarray:
        """Per-Gaussian gradients as [n][9] (mean x, mean y, Qxx, Qxy, Qyy, o, r, g, b)."""
        return self.d_gauss[: 9 * self.n_gauss].view(9, -1).t().cpu().numpy().astype(np.float64)

    def tile_lists(self):
        ranges = self.ranges.view(-1, 2).cpu().numpy().astype(np.int64)
        n = self.pairs_required()
        ids = self.ids[:n].cpu().numpy().view(np.uint32).astype(np.int64)
        return ranges, ids
