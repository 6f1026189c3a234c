"""What the trained curve-proposal network gains over the random start (GPU).

The committed weights (trained on the GPU by the project's own BF16
kernels) propose the curves of a held-out synthetic 512x512 target (a seed
outside the training and evaluation sets).  Under the learning rates of Sec.
4.1 the learned start must begin far above the uniform random start, reach
the random start's 300-step PSNR in at most 40% of the 300 steps, and end above
it.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def net():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    from paper_2503_16424_amd import cnn, learned_init
    assert os.path.exists(learned_init.WEIGHTS)
    n = cnn.CurveNet()
    with np.load(learned_init.WEIGHTS, allow_pickle=False) as f:
        n.load_state_dict({k: f[k] for k in f.files})
    return n


def test_learned_start_beats_random_start(net):
    from paper_2503_16424_amd import learned_init
    from paper_2503_16424_amd.optim import PAPER_LR
    out = learned_init.evaluate(net, size=512, steps=300, seed=4242,
                                sets={"paper_lr": dict(PAPER_LR)})["paper_lr"]
    rnd, lrn = out["random"], out["learned"]
    print(f"random {rnd['psnr_initial']:.2f} -> {rnd['psnr_final']:.2f}, learned "
          f"{lrn['psnr_initial']:.2f} -> {lrn['psnr_final']:.2f}, steps "
          f"{lrn['steps_to_random_final']}", flush=True)
    assert lrn["psnr_initial"] >= rnd["psnr_initial"] + 5.0
    assert lrn["steps_to_random_final"] is not None
    assert lrn["fraction_of_steps"] <= 0.4
    assert lrn["psnr_final"] > rnd["psnr_final"]


def test_proposal_is_a_valid_curve_set(net):
    import torch
    from paper_2503_16424_amd import bz, learned_init
    tgt = torch.as_tensor(learned_init.synthetic_target(4243, 96, 64), device="cuda")
    sc = learned_init.propose(net, tgt)
    assert sc.n_curves == 3 * 2 * 8
    assert np.all((sc.stroke_w >= 0.5) & (sc.stroke_w <= 4.0))
    assert np.all((sc.color >= 0) & (sc.color <= 1)) and np.all((sc.opacity >= 0) & (sc.opacity <= 1))
    pts = sc.ctrl.reshape(-1, 8, 4, 2)
    org = np.array([[x, y] for y in (0, 32) for x in (0, 32, 64)], np.float32)
    rel = pts - org[:, None, None, :]
    assert np.all(rel >= -8.0 - 1e-4) and np.all(rel <= 40.0 + 1e-4)     # a quarter side outside
    img = bz.Rasterizer(sc).render()
    assert torch.isfinite(img).all()
