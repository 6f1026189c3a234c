"""Pins of the FP64 convolution reference against independent facts (CPU).

* bf16 rounding equals torch's float32 -> bfloat16 conversion;
* the forward equals a sum of scipy 2-D correlations (then strided);
* a 1x1 convolution is a matrix product;
* the input gradient is the adjoint of the forward (<A x, y> = <x, A^T y>);
* the filter gradient satisfies <conv(x; w), dy> = <w, dW(dy, x)>, the bias
  gradient is the sum of dy;
* the ReLU mask of the input gradient matches central differences through
  max(0, .).
"""
import numpy as np
import pytest
import scipy.signal

from oracle import cnn_oracle as co


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.standard_normal(20000).astype(np.float32) * 10.0,
                        # exact ties: the low 16 bits are 0x8000
                        (rng.integers(1, 1 << 15, 200).astype(np.uint32) << 16 | 0x8000)
                        .view(np.float32), np.float32([0.0, -0.0, 1.0, 3.0e38])])
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(co.bf16(v), ref)


@pytest.mark.parametrize("stride,pad", [(1, 0), (1, 1), (2, 1), (2, 0), (3, 1)])
def test_forward_is_a_sum_of_correlations(stride, pad):
    rng = np.random.default_rng(stride * 10 + pad)
    n, h, w, c, k, r = 2, 7, 6, 3, 4, 3
    x = rng.standard_normal((n, h, w, c))
    wt = rng.standard_normal((k, r, r, c))
    b = rng.standard_normal(k)
    y = co.conv_fwd(x, wt, b, stride, pad)
    xp = np.pad(x, ((0, 0), (pad, pad), (pad, pad), (0, 0)))
    for bi in range(n):
        for o in range(k):
            full = sum(scipy.signal.correlate2d(xp[bi, :, :, i], wt[o, :, :, i], mode="valid")
                       for i in range(c))
            ref = full[::stride, ::stride] + b[o]
            assert np.allclose(y[bi, :, :, o], ref, atol=1e-12, rtol=0)


def test_one_by_one_convolution_is_a_matrix_product():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((5, 1, 1, 40))
    wt = rng.standard_normal((7, 1, 1, 40))
    y = co.conv_fwd(x, wt)
    assert np.allclose(y.reshape(5, 7), x.reshape(5, 40) @ wt.reshape(7, 40).T, atol=1e-12)


@pytest.mark.parametrize("stride,pad,r", [(1, 1, 3), (2, 1, 3), (2, 0, 3), (1, 0, 1)])
def test_input_gradient_is_the_adjoint(stride, pad, r):
    rng = np.random.default_rng(stride + 3 * pad + r)
    n, h, w, c, k = 2, 9, 8, 5, 6
    x = rng.standard_normal((n, h, w, c))
    wt = rng.standard_normal((k, r, r, c))
    y = co.conv_fwd(x, wt, None, stride, pad)
    dy = rng.standard_normal(y.shape)
    dx = co.conv_bwd_data(dy, wt, x.shape, stride, pad)
    assert abs(np.sum(y * dy) - np.sum(x * dx)) <= 1e-10 * np.sum(np.abs(y * dy))


@pytest.mark.parametrize("stride,pad,r", [(1, 1, 3), (2, 1, 3), (1, 0, 1)])
def test_filter_gradient_identity(stride, pad, r):
    rng = np.random.default_rng(7 + stride + pad + r)
    n, h, w, c, k = 3, 8, 9, 4, 5
    x = rng.standard_normal((n, h, w, c))
    wt = rng.standard_normal((k, r, r, c))
    y = co.conv_fwd(x, wt, None, stride, pad)
    dy = rng.standard_normal(y.shape)
    dw, db = co.conv_bwd_weight(dy, x, r, stride, pad)
    assert abs(np.sum(y * dy) - np.sum(wt * dw)) <= 1e-10 * np.sum(np.abs(y * dy))
    assert np.allclose(db, dy.reshape(-1, k).sum(0), atol=1e-12)


def test_relu_mask_matches_central_differences():
    rng = np.random.default_rng(11)
    z = rng.standard_normal((1, 6, 6, 3))
    z[np.abs(z) < 0.05] = 0.3                       # keep away from the kink
    wt = rng.standard_normal((4, 3, 3, 3))
    g = rng.standard_normal((1, 3, 3, 4))

    def loss(zz):
        return np.sum(co.conv_fwd(np.maximum(zz, 0.0), wt, None, 2, 1) * g)

    dz = co.conv_bwd_data(g, wt, z.shape, 2, 1, x_mask=np.maximum(z, 0.0))
    eps = 1e-6
    for idx in [(0, 1, 2, 0), (0, 3, 3, 2), (0, 5, 0, 1), (0, 2, 4, 1)]:
        zp, zm = z.copy(), z.copy()
        zp[idx] += eps
        zm[idx] -= eps
        fd = (loss(zp) - loss(zm)) / (2 * eps)
        assert abs(fd - dz[idx]) <= 1e-6 * max(1.0, abs(fd)), idx
