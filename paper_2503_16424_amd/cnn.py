"""Binding of libbz's BF16 matrix-core convolutions (include/bz_cnn.h) and the
curve-proposal network built from them.

:class:`CurveNet` maps a 32x32 RGB patch to the parameters of 8 cubic curves
of that patch: four 3x3 convolutions with 64 channels (stride 1, 2, 2, 2, each
followed by max(0, .)) and a fully connected head (1024 -> 104 = 8 curves x
13 values).  Weights are kept in FP32 (the optimiser's copy) and converted to
BF16 for the kernels; activations between layers are BF16, gradients FP32.
Every layer runs in libbz's kernels: forward (``bz_conv_fwd``), input
gradient with the ReLU mask (``bz_conv_bwd_data``), filter and bias
gradients (``bz_conv_bwd_weight``).  torch supplies memory, the loss on the
decoded curves and the Adam update.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import bz


class ConvDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("h", C.c_int32), ("w", C.c_int32), ("c", C.c_int32),
                ("k", C.c_int32), ("r", C.c_int32), ("stride", C.c_int32), ("pad", C.c_int32),
                ("ho", C.c_int32), ("wo", C.c_int32)]


EXPORTS = ("bz_conv_shape", "bz_conv_fwd", "bz_conv_bwd_data", "bz_conv_bwd_weight",
           "bz_f32_to_bf16", "bz_extract_patches")

_ready = False


def lib():
    global _ready
    L = bz.load_library()
    if not _ready:
        P, V = C.POINTER, C.c_void_p
        L.bz_conv_shape.restype = C.c_int
        L.bz_conv_shape.argtypes = [P(ConvDesc)]
        L.bz_conv_fwd.restype = C.c_int
        L.bz_conv_fwd.argtypes = [P(ConvDesc), V, V, V, C.c_int32, V, V, V]
        L.bz_conv_bwd_data.restype = C.c_int
        L.bz_conv_bwd_data.argtypes = [P(ConvDesc), V, V, V, V, V]
        L.bz_conv_bwd_weight.restype = C.c_int
        L.bz_conv_bwd_weight.argtypes = [P(ConvDesc), V, V, V, V, V]
        L.bz_f32_to_bf16.restype = C.c_int
        L.bz_f32_to_bf16.argtypes = [V, V, C.c_int64, V]
        L.bz_extract_patches.restype = C.c_int
        L.bz_extract_patches.argtypes = [V, C.c_int32, C.c_int32, V, C.c_int32, C.c_int32,
                                         C.c_float, V, V]
        _ready = True
    return L


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def conv_desc(n, h, w, c, k, r, stride, pad) -> ConvDesc:
    d = ConvDesc(n, h, w, c, k, r, stride, pad, 0, 0)
    bz._check("bz_conv_shape", lib().bz_conv_shape(C.byref(d)))
    return d


def conv_fwd(d, x, w, bias=None, relu=False, y=None, y_bf16=None):
    bz._check("bz_conv_fwd", lib().bz_conv_fwd(C.byref(d), _p(x), _p(w), _p(bias), int(relu),
                                               _p(y), _p(y_bf16), bz._stream()))


def conv_bwd_data(d, dy, w, dx, x_mask=None):
    bz._check("bz_conv_bwd_data", lib().bz_conv_bwd_data(C.byref(d), _p(dy), _p(w), _p(x_mask),
                                                         _p(dx), bz._stream()))


def conv_bwd_weight(d, dy, x, dw, db=None):
    bz._check("bz_conv_bwd_weight", lib().bz_conv_bwd_weight(C.byref(d), _p(dy), _p(x), _p(dw),
                                                             _p(db), bz._stream()))


def to_bf16(src, dst):
    bz._check("bz_f32_to_bf16", lib().bz_f32_to_bf16(_p(src), _p(dst), src.numel(),
                                                     bz._stream()))


def extract_patches(image, xy, side, fill, out):
    """image [3, H, W] f32, xy [n, 2] int32 (top-left corners) -> out bf16 bits
    [n, side, side, 3] (int16 tensor)."""
    H, W = image.shape[1], image.shape[2]
    bz._check("bz_extract_patches", lib().bz_extract_patches(
        _p(image), W, H, _p(xy), xy.shape[0], side, float(fill), _p(out), bz._stream()))


def bf16_view(t):
    """A torch bfloat16 tensor's bits as the int16 tensor the kernels take."""
    return t.view(__import__("torch").int16)


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------
PATCH = 32
CURVES = 8
PER_CURVE = 13           # 4 control points (8), width, colour (3), opacity
OUT = CURVES * PER_CURVE
LAYERS = ((3, 64, 3, 1, 1), (64, 64, 3, 2, 1), (64, 64, 3, 2, 1), (64, 64, 3, 2, 1))  # c, k, r, s, p
HEAD_IN = 64 * 4 * 4
# Input channels of layer 0 as its forward reads them: the 3 of the patch and 5
# zeros, so that the convolution gathers 8 BF16 channels per 16-byte load; the
# weights of the zero channels are zero, so the outputs are those of 3.
C0 = 8


class CurveNet:
    """Weights, BF16 copies and the per-batch activations of the network."""

    def __init__(self, seed: int = 0, device="cuda"):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        g = torch.Generator().manual_seed(seed)
        self.params = []                       # (w [k, r, r, c], b [k]) per layer, FP32
        for (c, k, r, s, p) in LAYERS:
            std = math.sqrt(2.0 / (r * r * c))
            w = torch.randn((k, r, r, c), generator=g) * std
            self.params.append((w.to(self.dev).requires_grad_(), torch.zeros(k, device=self.dev)
                                .requires_grad_()))
        wh = torch.randn((OUT, 1, 1, HEAD_IN), generator=g) * math.sqrt(1.0 / HEAD_IN)
        self.params.append((wh.to(self.dev).requires_grad_(),
                            torch.zeros(OUT, device=self.dev).requires_grad_()))
        self._bf = [torch.empty(w.shape, dtype=torch.int16, device=self.dev) for w, _ in self.params]
        k0, r0 = LAYERS[0][1], LAYERS[0][2]
        self._bf[0] = torch.zeros((k0, r0, r0, C0), dtype=torch.int16, device=self.dev)
        self._acts = None
        self._x8 = None

    def tensors(self):
        return [t for wb in self.params for t in wb]

    def _shapes(self, n):
        """Descriptors of the layers (layer 0 with its 3 real input channels:
        the backward's)."""
        ds, h = [], PATCH
        for (c, k, r, s, p) in LAYERS:
            d = conv_desc(n, h, h, c, k, r, s, p)
            ds.append(d)
            h = d.ho
        ds.append(conv_desc(n, 1, 1, HEAD_IN, OUT, 1, 1, 0))
        return ds

    def _fwd_shapes(self, n):
        """The forward's descriptors: layer 0 reads C0 channels."""
        ds = self._shapes(n)
        c, k, r, s, p = LAYERS[0]
        ds[0] = conv_desc(n, PATCH, PATCH, C0, k, r, s, p)
        return ds

    def sync_weights(self):
        """FP32 weights -> the BF16 copies the kernels read (layer 0's padded
        to C0 input channels with zeros)."""
        torch = self.torch
        with torch.no_grad():
            for i, ((w, _), wb) in enumerate(zip(self.params, self._bf)):
                if i == 0:
                    wp = torch.zeros(wb.shape, dtype=torch.float32, device=self.dev)
                    wp[..., :w.shape[-1]] = w.detach()
                    to_bf16(wp, wb)
                else:
                    to_bf16(w.detach().contiguous(), wb)

    def forward(self, x):
        """x: BF16 bits (int16) [n, 32, 32, 3] -> raw outputs FP32 [n, 104]."""
        torch = self.torch
        n = x.shape[0]
        ds, dsf = self._shapes(n), self._fwd_shapes(n)
        x8 = torch.nn.functional.pad(x, (0, C0 - x.shape[-1]))      # BF16 zero bits
        acts = [x]
        for i in range(len(LAYERS)):
            d = dsf[i]
            y = torch.empty((n, d.ho, d.wo, d.k), dtype=torch.int16, device=self.dev)
            conv_fwd(d, x8 if i == 0 else acts[-1], self._bf[i], self.params[i][1], relu=True,
                     y_bf16=y)
            acts.append(y)
        z = torch.empty((n, OUT), dtype=torch.float32, device=self.dev)
        conv_fwd(ds[-1], acts[-1], self._bf[-1], self.params[-1][1], relu=False, y=z)
        self._acts, self._ds, self._dsf, self._x8 = acts, ds, dsf, x8
        return z

    def backward(self, dz):
        """dz: FP32 [n, 104] -> .grad of every weight and bias."""
        torch = self.torch
        acts, ds = self._acts, self._ds
        d = dz.contiguous()
        for i in range(len(self.params) - 1, -1, -1):
            w, b = self.params[i]
            dw = torch.empty_like(w)
            db = torch.empty_like(b)
            conv_bwd_weight(ds[i], d, acts[i], dw, db)
            w.grad, b.grad = dw, db
            if i > 0:
                dx = torch.empty(acts[i].shape, dtype=torch.float32, device=self.dev)
                conv_bwd_data(ds[i], d, self._bf[i], dx, x_mask=acts[i])
                d = dx

    def state_dict(self) -> dict:
        out = {}
        for i, (w, b) in enumerate(self.params):
            out[f"w{i}"] = w.detach().cpu().numpy()
            out[f"b{i}"] = b.detach().cpu().numpy()
        return out

    def load_state_dict(self, sd: dict):
        with self.torch.no_grad():
            for i, (w, b) in enumerate(self.params):
                w.copy_(self.torch.as_tensor(np.asarray(sd[f"w{i}"])))
                b.copy_(self.torch.as_tensor(np.asarray(sd[f"b{i}"])))
        self.sync_weights()


# ---------------------------------------------------------------------------
# curve parameters <-> network outputs
# ---------------------------------------------------------------------------
MARGIN = 0.25            # control points may leave the patch by a quarter side
W_MIN, W_SPAN = 0.5, 3.5


class TrainGraph:
    """Forward and backward of ``net`` on fixed buffers ``x`` (BF16 bits,
    [n, 32, 32, 3]) and ``dz`` (FP32 [n, 104]), recorded once as a HIP graph
    and replayed with one launch.  Eagerly the step issues ~25 small launches
    from Python and the GPU waits on the host between them.  After a replay
    ``z`` holds the outputs and every parameter's ``.grad`` the gradients
    (buffers of the graph, overwritten by the next replay); the BF16 weight
    copies are read as they are at replay time."""

    def __init__(self, net: "CurveNet", x, dz, warmup: int = 2):
        torch = net.torch
        self.net, self.x, self.dz = net, x, dz
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                net.forward(x)
                net.backward(dz)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.z = net.forward(x)
            net.backward(dz)

    def replay(self):
        self.graph.replay()
        return self.z


def decode(z, side=PATCH):
    """Raw outputs [n, 104] -> normalised curve parameters [n, 8, 13]:
    control points in patch sides (origin at the patch corner), then
    (width - 0.5) / 3.5, colour, opacity, each in [0, 1] for the last five."""
    torch = __import__("torch")
    s = torch.sigmoid(z.view(-1, CURVES, PER_CURVE))
    pts = s[..., :8] * (1.0 + 2.0 * MARGIN) - MARGIN
    return torch.cat([pts, s[..., 8:]], dim=-1)


def to_curves(u, origins, side=PATCH):
    """Normalised parameters [n, 8, 13] and patch corners [n, 2] (px) ->
    control points [n*8, 4, 2] px, widths [n*8], colours [n*8, 3], opacities [n*8]."""
    n = u.shape[0]
    pts = u[..., :8].reshape(n, CURVES, 4, 2) * side + origins.reshape(n, 1, 1, 2)
    return (pts.reshape(-1, 4, 2), (W_MIN + W_SPAN * u[..., 8]).reshape(-1),
            u[..., 9:12].reshape(-1, 3), u[..., 12].reshape(-1))


def normalise(ctrl, width, color, opacity, origins, side=PATCH):
    """Inverse of :func:`to_curves` (numpy): curves of n patches (8 each, in
    slot order) -> normalised targets [n, 8, 13]."""
    n = origins.shape[0]
    pts = (np.asarray(ctrl).reshape(n, CURVES, 4, 2) - origins.reshape(n, 1, 1, 2)) / side
    w = (np.asarray(width).reshape(n, CURVES, 1) - W_MIN) / W_SPAN
    return np.concatenate([pts.reshape(n, CURVES, 8), w, np.asarray(color).reshape(n, CURVES, 3),
                           np.asarray(opacity).reshape(n, CURVES, 1)], axis=-1)
