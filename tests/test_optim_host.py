"""Host-side pieces of the optimisation loop (no GPU)."""
import math

import numpy as np

from paper_2503_16424_amd import scenes
from paper_2503_16424_amd.optim import noisy_target, psnr_from_mse


def test_psnr_closed_forms():
    assert psnr_from_mse(1.0) == 0.0
    assert abs(psnr_from_mse(1e-2) - 20.0) < 1e-12
    assert abs(psnr_from_mse(0.02 ** 2) - 20.0 * math.log10(50.0)) < 1e-12
    assert psnr_from_mse(0.0) == float("inf")


def test_noisy_target_is_seeded_clipped_and_has_the_stated_sigma():
    clean = np.full((3, 64, 64), 0.5)
    a = noisy_target(clean, 2, 0.02)
    b = noisy_target(clean, 2, 0.02)
    assert a.dtype == np.float32 and np.array_equal(a, b)
    assert not np.array_equal(a, noisy_target(clean, 3, 0.02))
    assert abs(float(np.std(a - 0.5)) - 0.02) < 1e-3          # far from the clip bounds
    edge = noisy_target(np.zeros((3, 8, 8)), 2, 0.5)
    assert edge.min() == 0.0 and edge.max() <= 1.0


def test_gaussian_noise_statistics():
    z = scenes.gaussian_noise(0, (200000,), 0.02)
    assert abs(z.mean()) < 2e-4 and abs(z.std() - 0.02) < 2e-4


def test_optimizer_state_round_trips_and_resumes_bit_for_bit(tmp_path):
    """Adam on the host: 30 steps straight, against 12 steps, a checkpoint of
    the parameters and moments through an .npz file, and 18 more steps from a
    fresh optimiser -- the same parameters bit for bit."""
    import torch
    from paper_2503_16424_amd.optim import load_optimizer_state, optimizer_state_arrays
    rng = np.random.default_rng(0)
    A = torch.as_tensor(rng.normal(size=(6, 6)), dtype=torch.float32)
    b = torch.as_tensor(rng.normal(size=6), dtype=torch.float32)

    def run(x, opt, steps):
        for _ in range(steps):
            opt.zero_grad()
            loss = ((A @ x - b) ** 2).sum()
            loss.backward()
            opt.step()

    x1 = torch.nn.Parameter(torch.zeros(6))
    o1 = torch.optim.Adam([x1], lr=0.05)
    run(x1, o1, 30)
    x2 = torch.nn.Parameter(torch.zeros(6))
    o2 = torch.optim.Adam([x2], lr=0.05)
    run(x2, o2, 12)
    path = str(tmp_path / "ckpt.npz")
    np.savez(path, x=x2.detach().numpy(), **optimizer_state_arrays(o2))
    with np.load(path, allow_pickle=False) as f:
        a = {k: f[k] for k in f.files}
    assert {"opt_0_0_step", "opt_0_0_exp_avg", "opt_0_0_exp_avg_sq"} <= set(a)
    x3 = torch.nn.Parameter(torch.as_tensor(a["x"]))
    o3 = torch.optim.Adam([x3], lr=0.05)
    load_optimizer_state(o3, a)
    run(x3, o3, 18)
    assert torch.equal(x1.detach(), x3.detach())
