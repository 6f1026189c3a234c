"""Plain FP64 reference of the learned initialiser's convolutions.

TEST INFRASTRUCTURE ONLY: imported by tests/ alone (never by the package).

The network is project-defined (the paper initialises curves at random); this
module writes out, by definition, what its layers compute so that the BF16
matrix-core kernels can be checked against it:

* ``conv_fwd``: y[b, oy, ox, o] = bias[o] + sum_{ky, kx, i} x[b, oy s - p + ky,
  ox s - p + kx, i] w[o, ky, kx, i] with zero padding, then max(0, .);
* ``conv_bwd_data``: the adjoint of that sum, scattered tap by tap;
* ``conv_bwd_weight``: dw[o, ky, kx, i] = sum_{b, oy, ox} dy[b, oy, ox, o] x[b,
  oy s - p + ky, ox s - p + kx, i], db[o] = sum dy[..., o];
* ``bf16``: rounding of float32 values to bfloat16, to nearest even, the
  precision the kernels feed the matrix cores with.

Tensors are NHWC numpy arrays; filters are [k][r][r][c].  Plain loops over
the r x r taps, each tap one numpy multiply-add over whole slices.
"""
from __future__ import annotations

import numpy as np


def bf16(a) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); returned as
    float64 holding the rounded values."""
    f = np.ascontiguousarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def out_size(h, r, stride, pad):
    return (h + 2 * pad - r) // stride + 1


def _padded(x, pad):
    return np.pad(x, ((0, 0), (pad, pad), (pad, pad), (0, 0)))


def conv_fwd(x, w, bias=None, stride=1, pad=0, relu=False):
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    n, h, wd, c = x.shape
    k, r, _, _ = w.shape
    ho, wo = out_size(h, r, stride, pad), out_size(wd, r, stride, pad)
    xp = _padded(x, pad)
    y = np.zeros((n, ho, wo, k))
    for ky in range(r):
        for kx in range(r):
            sl = xp[:, ky: ky + stride * (ho - 1) + 1: stride,
                    kx: kx + stride * (wo - 1) + 1: stride, :]          # [n, ho, wo, c]
            y += sl @ w[:, ky, kx, :].T
    if bias is not None:
        y += np.asarray(bias, np.float64)
    return np.maximum(y, 0.0) if relu else y


def conv_bwd_data(dy, w, in_shape, stride=1, pad=0, x_mask=None):
    dy = np.asarray(dy, np.float64)
    w = np.asarray(w, np.float64)
    n, h, wd, c = in_shape
    k, r, _, _ = w.shape
    ho, wo = dy.shape[1], dy.shape[2]
    dxp = np.zeros((n, h + 2 * pad, wd + 2 * pad, c))
    for ky in range(r):
        for kx in range(r):
            dxp[:, ky: ky + stride * (ho - 1) + 1: stride,
                kx: kx + stride * (wo - 1) + 1: stride, :] += dy @ w[:, ky, kx, :]
    dx = dxp[:, pad: pad + h, pad: pad + wd, :]
    if x_mask is not None:
        dx = np.where(np.asarray(x_mask) > 0, dx, 0.0)
    return dx


def conv_bwd_weight(dy, x, r, stride=1, pad=0):
    dy = np.asarray(dy, np.float64)
    x = np.asarray(x, np.float64)
    n, ho, wo, k = dy.shape
    c = x.shape[3]
    xp = _padded(x, pad)
    dw = np.zeros((k, r, r, c))
    d2 = dy.reshape(-1, k)
    for ky in range(r):
        for kx in range(r):
            sl = xp[:, ky: ky + stride * (ho - 1) + 1: stride,
                    kx: kx + stride * (wo - 1) + 1: stride, :].reshape(-1, c)
            dw[:, ky, kx, :] = d2.T @ sl
    return dw, d2.sum(axis=0)
