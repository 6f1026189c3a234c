"""BF16 matrix-core convolutions against the FP64 reference (GPU).

Both sides see the same BF16 operands (the reference rounds exactly where the
kernels do: inputs, filters, output gradients entering the matrix cores,
activations between layers), so single layers differ only by the FP32
accumulation order: bound 1e-5 of the sum of |terms|.  BF16 outputs may
differ by one BF16 step where that order moves a value across a rounding
boundary (bounded fraction), or by the accumulation bound where a sum near
zero lands on the other side of the ReLU.  The whole network (five layers, BF16 between
them) is compared to 1e-2 relative L2: one flipped BF16 rounding changes a
value by 2^-8 relative and propagates.
"""
import numpy as np
import pytest

from oracle import cnn_oracle as co
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return torch


def _bf16_bits(torch, a):
    """float array -> (int16 bits tensor on the GPU, float64 rounded values)."""
    t = torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).cuda(), t.to(torch.float64).numpy()


SHAPES = [  # n, h, w, c, k, r, stride, pad
    (3, 32, 32, 3, 64, 3, 1, 1),      # first layer (its own filter-gradient kernel)
    (2, 13, 32, 2, 64, 3, 1, 1),      # the same kernel: ragged rows per wave, 2 channels
    (1, 64, 32, 1, 64, 3, 1, 1),      # the same kernel: tallest image, 1 channel
    (1, 65, 32, 3, 64, 3, 1, 1),      # one row taller: the generic path
    (5, 32, 32, 64, 64, 3, 2, 1),     # strided layers
    (7, 8, 8, 64, 64, 3, 2, 1),
    (9, 1, 1, 1024, 104, 1, 1, 0),    # fully connected head
    (2, 7, 9, 5, 13, 3, 2, 1),        # ragged everything
    (3, 5, 6, 40, 70, 3, 1, 0),
    (1, 3, 3, 2, 1, 3, 3, 1),
]


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_layer_matches_reference(torch_cuda, shape):
    torch = torch_cuda
    from paper_2503_16424_amd import cnn
    n, h, w, c, k, r, s, p = shape
    rng = np.random.default_rng(sum(shape))
    xb, x = _bf16_bits(torch, rng.standard_normal((n, h, w, c)))
    wb, wt = _bf16_bits(torch, rng.standard_normal((k, r, r, c)) * 0.2)
    bias = rng.standard_normal(k).astype(np.float32)
    d = cnn.conv_desc(n, h, w, c, k, r, s, p)
    ho, wo = d.ho, d.wo
    assert (ho, wo) == (co.out_size(h, r, s, p), co.out_size(w, r, s, p))
    # forward, FP32 output without ReLU, BF16 output with it
    y = torch.empty((n, ho, wo, k), device="cuda")
    yb = torch.empty((n, ho, wo, k), dtype=torch.int16, device="cuda")
    bias_t = torch.as_tensor(bias, device="cuda")
    cnn.conv_fwd(d, xb, wb, bias_t, relu=False, y=y)
    cnn.conv_fwd(d, xb, wb, bias_t, relu=True, y_bf16=yb)
    ref = co.conv_fwd(x, wt, bias.astype(np.float64), s, p)
    scale = co.conv_fwd(np.abs(x), np.abs(wt), np.abs(bias), s, p) + 1e-30
    assert (np.abs(y.cpu().numpy() - ref) / scale).max() <= 1e-5
    got_b = yb.view(torch.bfloat16).to(torch.float64).cpu().numpy()
    ref_b = co.bf16(np.maximum(ref, 0.0).astype(np.float32))
    diff = got_b != ref_b
    assert diff.mean() <= 2e-3
    # one BF16 step, or (a sum near zero that the ReLU clips on one side only)
    # the FP32 accumulation-order bound of the FP32 output above
    bound = np.abs(ref_b) * 2.0 ** -7 + 1e-5 * scale
    assert np.all(np.abs(got_b - ref_b)[diff] <= bound[diff])
    # input gradient, with the ReLU mask of the input
    dy = rng.standard_normal((n, ho, wo, k)).astype(np.float32)
    dy_t = torch.as_tensor(dy, device="cuda")
    dx = torch.empty((n, h, w, c), device="cuda")
    cnn.conv_bwd_data(d, dy_t, wb, dx, x_mask=xb)
    dyb = co.bf16(dy)
    ref = co.conv_bwd_data(dyb, wt, (n, h, w, c), s, p, x_mask=x)
    scale = co.conv_bwd_data(np.abs(dyb), np.abs(wt), (n, h, w, c), s, p) + 1e-30
    assert (np.abs(dx.cpu().numpy() - ref) / scale).max() <= 1e-5
    # filter and bias gradients
    dw = torch.empty((k, r, r, c), device="cuda")
    db = torch.empty(k, device="cuda")
    cnn.conv_bwd_weight(d, dy_t, xb, dw, db)
    ref_w, _ = co.conv_bwd_weight(dyb, x, r, s, p)
    scale, _ = co.conv_bwd_weight(np.abs(dyb), np.abs(x), r, s, p)
    assert (np.abs(dw.cpu().numpy() - ref_w) / (scale + 1e-30)).max() <= 1e-5
    ref_b = dy.astype(np.float64).reshape(-1, k).sum(0)
    sc_b = np.abs(dy.astype(np.float64)).reshape(-1, k).sum(0)
    assert (np.abs(db.cpu().numpy() - ref_b) / sc_b).max() <= 1e-5


def test_bf16_conversion_and_patches(torch_cuda):
    torch = torch_cuda
    from paper_2503_16424_amd import cnn
    rng = np.random.default_rng(4)
    v = (rng.standard_normal(100003) * 50).astype(np.float32)
    out = torch.empty(v.size, dtype=torch.int16, device="cuda")
    cnn.to_bf16(torch.as_tensor(v, device="cuda"), out)
    ref = torch.as_tensor(v).to(torch.bfloat16).view(torch.int16).numpy()
    assert np.array_equal(out.cpu().numpy(), ref)
    img = rng.uniform(0, 1, (3, 37, 53)).astype(np.float32)
    xy = np.array([[0, 0], [40, 20], [-5, -3], [30, 30]], np.int32)
    pt = torch.empty((4, 16, 16, 3), dtype=torch.int16, device="cuda")
    cnn.extract_patches(torch.as_tensor(img, device="cuda"), torch.as_tensor(xy, device="cuda"),
                        16, 0.5, pt)
    got = pt.view(torch.bfloat16).to(torch.float64).cpu().numpy()
    pad = np.full((3, 37 + 64, 53 + 64), 0.5, np.float32)
    pad[:, 32:69, 32:85] = img
    for i, (x0, y0) in enumerate(xy):
        ref = pad[:, y0 + 32: y0 + 48, x0 + 32: x0 + 48].transpose(1, 2, 0)
        assert np.array_equal(got[i], co.bf16(ref)), i


def _reference_network(net, xs):
    """The network in FP64 on the kernels' BF16 operands, rounding where they do."""
    from paper_2503_16424_amd import cnn
    ps = [(co.bf16(w.detach().cpu().numpy()), b.detach().cpu().numpy().astype(np.float64))
          for w, b in net.params]
    acts = [xs]
    for (c, k, r, s, p), (w, b) in zip(cnn.LAYERS, ps[:-1]):
        acts.append(co.bf16(co.conv_fwd(acts[-1], w, b, s, p, relu=True).astype(np.float32)))
    n = xs.shape[0]
    z = co.conv_fwd(acts[-1].reshape(n, 1, 1, -1), ps[-1][0], ps[-1][1]).reshape(n, -1)
    return ps, acts, z


def test_network_forward_and_backward_match_reference(torch_cuda):
    torch = torch_cuda
    from paper_2503_16424_amd import cnn
    from tests.helpers import rel_l2
    rng = np.random.default_rng(6)
    net = cnn.CurveNet(seed=3)
    net.sync_weights()
    n = 20
    xb, xs = _bf16_bits(torch, rng.uniform(0, 1, (n, 32, 32, 3)))
    z = net.forward(xb)
    ps, acts, zr = _reference_network(net, xs)
    assert rel_l2(z.cpu().numpy(), zr) <= 1e-2
    dz = rng.standard_normal((n, cnn.OUT)).astype(np.float32)
    net.backward(torch.as_tensor(dz, device="cuda"))
    # reference backward, rounding dy to BF16 where the kernels do
    d = dz.astype(np.float64).reshape(n, 1, 1, -1)
    grads = []
    shapes = [a.shape for a in acts]
    for i in range(len(ps) - 1, -1, -1):
        w, _ = ps[i]
        r = w.shape[1]
        s, p = (1, 0) if i == len(ps) - 1 else cnn.LAYERS[i][3:5]
        a = acts[i] if i < len(ps) - 1 else acts[i].reshape(n, 1, 1, -1)
        dw, db = co.conv_bwd_weight(co.bf16(d.astype(np.float32)), a, r, s, p)
        grads.append((i, dw, db))
        if i > 0:
            dx = co.conv_bwd_data(co.bf16(d.astype(np.float32)), w, a.shape, s, p, x_mask=a)
            d = dx.reshape(shapes[i])
            d = d.astype(np.float32).astype(np.float64)
    for i, dw, db in grads:
        w, b = net.params[i]
        assert rel_l2(w.grad.cpu().numpy().reshape(dw.shape), dw) <= 1e-2, i
        assert rel_l2(b.grad.cpu().numpy(), db) <= 1e-2, i


def test_train_graph_replays_match_the_eager_step(torch_cuda):
    """The recorded forward+backward replayed four times, with eager work and
    synchronisations between the replays, gives the eager step's outputs and
    gradients each time (the filter gradients to float-atomic order)."""
    torch = torch_cuda
    from paper_2503_16424_amd import cnn
    net = cnn.CurveNet(seed=3)
    net.sync_weights()
    rng = np.random.default_rng(4)
    x = torch.as_tensor(rng.uniform(0, 1, (64, 32, 32, 3)).astype(np.float32),
                        device="cuda").to(torch.bfloat16).view(torch.int16)
    dz = torch.as_tensor(rng.standard_normal((64, cnn.OUT)).astype(np.float32), device="cuda")
    z_ref = net.forward(x).clone()
    net.backward(dz)
    torch.cuda.synchronize()
    g_ref = [(w.grad.clone(), b.grad.clone()) for w, b in net.params]
    tg = cnn.TrainGraph(net, x, dz)
    for rep in range(4):
        for w, b in net.params:                      # eager work between the replays
            w.grad.fill_(7.0)
            b.grad.fill_(7.0)
        torch.cuda.synchronize()
        z = tg.replay()
        torch.cuda.synchronize()
        assert torch.equal(z, z_ref), rep
        for (w, b), (gw, gb) in zip(net.params, g_ref):
            assert rel_l2(w.grad.cpu().numpy(), gw.cpu().numpy()) <= 1e-5, rep
            assert rel_l2(b.grad.cpu().numpy(), gb.cpu().numpy()) <= 1e-5, rep
