"""ctypes front end of the double-precision CPU oracle (bz_oracle.c).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg, never by the product path.  Every function cites the part of
the paper it follows in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bz_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Readings of parameters the paper leaves open (density constant rho, screen
# dilation, kernel truncation, alpha clamp, termination transmittance).
DEFAULTS = dict(rho=2.0, sigma0_sq=0.3, g_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-6)

_lib = None


def lib_path() -> str:
    return _LIB


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, IEEE double, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB)
        _lib.orc_count_gaussians.restype = C.c_int64
        for name in ("orc_sample", "orc_render", "orc_render_pixels", "orc_chain",
                     "orc_tile_depth", "orc_num_threads"):
            getattr(_lib, name).restype = C.c_int
    return _lib


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads the oracle's parallel loops use from now on."""
    _load().orc_set_threads(C.c_int(int(n)))


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _opts(o):
    d = dict(DEFAULTS)
    if o:
        d.update(o)
    return d


def _scene_args(sc):
    return (C.c_int(sc.n_curves), _p(_c(sc.kind, np.int32)), _p(_c(sc.nseg, np.int32)),
            _p(_c(sc.k_samples, np.int32)), _p(_c(sc.r_interior, np.int32)),
            _p(_c(sc.ctrl, np.float64)), _p(_c(sc.ctrl_off, np.int32)),
            _p(_c(sc.tau, np.float64)), _p(_c(sc.tau_off, np.int32)),
            _p(_c(sc.stroke_w, np.float64)))


def sample(sc, opts=None) -> dict:
    """Gaussians of a scene in draw order (Sec. 3.3), all float64."""
    o = _opts(opts)
    lib = _load()
    # keep contiguous copies alive for the duration of the call
    arrs = [_c(sc.kind, np.int32), _c(sc.nseg, np.int32), _c(sc.k_samples, np.int32),
            _c(sc.r_interior, np.int32), _c(sc.ctrl, np.float64), _c(sc.ctrl_off, np.int32),
            _c(sc.tau, np.float64), _c(sc.tau_off, np.int32), _c(sc.stroke_w, np.float64),
            _c(sc.color, np.float64), _c(sc.opacity, np.float64), _c(sc.opa_off, np.int32),
            _c(sc.rank, np.int32)]
    n = sc.n_curves
    ng = int(lib.orc_count_gaussians(C.c_int(n), _p(arrs[0]), _p(arrs[2]), _p(arrs[3])))
    out = dict(mu=np.zeros((ng, 2)), conic=np.zeros((ng, 3)), sx2=np.zeros(ng),
               sy2=np.zeros(ng), tangent=np.zeros((ng, 2)), opac=np.zeros(ng),
               color=np.zeros((ng, 3)), curve=np.zeros(ng, np.int32),
               row=np.zeros(ng, np.int32), col=np.zeros(ng, np.int32),
               slot=np.zeros(ng, np.int32))
    st = lib.orc_sample(C.c_int(n), *[_p(a) for a in arrs], C.c_double(o["rho"]),
                        C.c_double(o["sigma0_sq"]), _p(out["mu"]), _p(out["conic"]),
                        _p(out["sx2"]), _p(out["sy2"]), _p(out["tangent"]), _p(out["opac"]),
                        _p(out["color"]), _p(out["curve"]), _p(out["row"]), _p(out["col"]),
                        _p(out["slot"]))
    if st != 0:
        raise ValueError(f"oracle sample rejected the scene (status {st})")
    return out


def render(g: dict, W: int, H: int, bg, opts=None, rows=None, d_image=None, brute=False) -> dict:
    """Front-to-back blend (Sec. 3.4) of rows [y0, y1); with d_image also the
    reverse pass to per-Gaussian gradients (mu_x, mu_y, Qxx, Qxy, Qyy, o, r, g, b)."""
    o = _opts(opts)
    lib = _load()
    mu, conic = _c(g["mu"], np.float64), _c(g["conic"], np.float64)
    opac, color = _c(g["opac"], np.float64), _c(g["color"], np.float64)
    ng = mu.shape[0]
    bgv = _c(bg, np.float64)
    y0, y1 = (0, H) if rows is None else rows
    image = np.zeros((3, H, W))
    t_final = np.ones((H, W))
    n_contrib = np.zeros((H, W), np.int32)
    margin = np.full((H, W), np.inf)
    counters = np.zeros(4, np.int64)
    dimg = None if d_image is None else _c(d_image, np.float64)
    d_gauss = None if d_image is None else np.zeros((ng, 9))
    st = lib.orc_render(C.c_int64(ng), _p(mu), _p(conic), _p(opac), _p(color), C.c_int(W),
                        C.c_int(H), _p(bgv), C.c_double(o["g_min"]), C.c_double(o["alpha_max"]),
                        C.c_double(o["t_min"]), C.c_int(y0), C.c_int(y1), C.c_int(int(brute)),
                        _p(image), _p(t_final), _p(n_contrib), _p(dimg), _p(d_gauss),
                        _p(counters), _p(margin))
    if st != 0:
        raise ValueError(f"oracle render rejected its arguments (status {st})")
    return dict(image=image, t_final=t_final, n_contrib=n_contrib, d_gauss=d_gauss,
                margin=margin, pairs=int(counters[0]), tested=int(counters[1]),
                terminated=int(counters[2]))


def render_pixels(g: dict, W: int, H: int, bg, xs, ys, opts=None) -> dict:
    """Forward value of individual pixels (each pixel scans every Gaussian)."""
    o = _opts(opts)
    lib = _load()
    mu, conic = _c(g["mu"], np.float64), _c(g["conic"], np.float64)
    opac, color = _c(g["opac"], np.float64), _c(g["color"], np.float64)
    xs, ys = _c(xs, np.int32), _c(ys, np.int32)
    npx = xs.shape[0]
    rgb = np.zeros((npx, 3))
    T = np.zeros(npx)
    nc = np.zeros(npx, np.int32)
    st = lib.orc_render_pixels(C.c_int64(mu.shape[0]), _p(mu), _p(conic), _p(opac), _p(color),
                               C.c_int(W), C.c_int(H), _p(_c(bg, np.float64)),
                               C.c_double(o["g_min"]), C.c_double(o["alpha_max"]),
                               C.c_double(o["t_min"]), C.c_int(npx), _p(xs), _p(ys), _p(rgb),
                               _p(T), _p(nc))
    if st != 0:
        raise ValueError(f"oracle render_pixels rejected its arguments (status {st})")
    return dict(rgb=rgb, t_final=T, n_contrib=nc)


def tile_depth(g: dict, n_curves: int, W: int, H: int, tile=(16, 16), opts=None) -> dict:
    """Depth complexity per tile (row-major tiles of tile[0] x tile[1] px):
    distinct curves contributing to a pixel of the tile (forward pass of Sec.
    3.4 re-run per tile) and distinct curves whose support box reaches it."""
    o = _opts(opts)
    lib = _load()
    mu, conic = _c(g["mu"], np.float64), _c(g["conic"], np.float64)
    opac, curve = _c(g["opac"], np.float64), _c(g["curve"], np.int32)
    tw, th = tile
    nt = (-(-W // tw)) * (-(-H // th))
    dc = np.zeros(nt, np.int32)
    ds = np.zeros(nt, np.int32)
    st = lib.orc_tile_depth(C.c_int64(mu.shape[0]), _p(mu), _p(conic), _p(opac), _p(curve),
                            C.c_int(n_curves), C.c_int(W), C.c_int(H), C.c_double(o["g_min"]),
                            C.c_double(o["alpha_max"]), C.c_double(o["t_min"]), C.c_int(tw),
                            C.c_int(th), _p(dc), _p(ds))
    if st != 0:
        raise ValueError(f"oracle tile_depth rejected its arguments (status {st})")
    return dict(contrib=dc, support=ds)


def chain(sc, d_gauss: np.ndarray, opts=None) -> dict:
    """Per-Gaussian gradients -> curve parameters (control points, widths,
    colours, opacities), through the sampling of Sec. 3.3."""
    o = _opts(opts)
    lib = _load()
    arrs = [_c(sc.kind, np.int32), _c(sc.nseg, np.int32), _c(sc.k_samples, np.int32),
            _c(sc.r_interior, np.int32), _c(sc.ctrl, np.float64), _c(sc.ctrl_off, np.int32),
            _c(sc.tau, np.float64), _c(sc.tau_off, np.int32), _c(sc.stroke_w, np.float64),
            _c(sc.opa_off, np.int32), _c(sc.rank, np.int32)]
    n = sc.n_curves
    out = dict(d_ctrl=np.zeros((sc.ctrl.shape[0], 2)), d_width=np.zeros(n),
               d_color=np.zeros((n, 3)), d_opacity=np.zeros(sc.opacity.shape[0]))
    dg = _c(d_gauss, np.float64)
    st = lib.orc_chain(C.c_int(n), *[_p(a) for a in arrs], C.c_double(o["rho"]),
                       C.c_double(o["sigma0_sq"]), _p(dg), _p(out["d_ctrl"]),
                       _p(out["d_width"]), _p(out["d_color"]), _p(out["d_opacity"]))
    if st != 0:
        raise ValueError(f"oracle chain rejected its arguments (status {st})")
    return out


def forward_backward(sc, d_image=None, opts=None, rows=None) -> dict:
    """Sample, render and (given d_image) differentiate a whole scene."""
    g = sample(sc, opts)
    r = render(g, sc.width, sc.height, sc.bg, opts, rows=rows, d_image=d_image)
    r["gauss"] = g
    if d_image is not None:
        r.update(chain(sc, r["d_gauss"], opts))
    return r
