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
