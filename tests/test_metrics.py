"""Pins of the image-quality metrics against closed forms."""
import numpy as np

from paper_2509_08574_amd import metrics


def test_psnr_closed_form():
    t = np.zeros((6, 7, 8))
    t[2, 3, 4] = 2.0
    x = t + 0.1                     # MSE = 0.01, peak 2
    assert abs(metrics.psnr(x, t) - 10 * np.log10(4.0 / 0.01)) < 1e-12
    assert metrics.psnr(t, t) == float("inf")


def test_ssim_identity_and_closed_forms():
    rng = np.random.default_rng(0)
    t = rng.uniform(size=(12, 13, 14))
    assert abs(metrics.ssim(t, t) - 1.0) < 1e-12
    # constant images a and b: only the luminance term remains,
    # (2ab + c1) / (a^2 + b^2 + c1) with c1 from the truth's range (here 0 ->
    # the truth has range L = 0 so use a truth with range 1 instead)
    a = np.zeros((10, 10, 10))
    a[0, 0, 0] = 1.0                # range 1, mean ~0
    b = a.copy()
    assert abs(metrics.ssim(b, a) - 1.0) < 1e-12


def test_ssim_and_psnr_decrease_with_noise():
    rng = np.random.default_rng(1)
    t = rng.uniform(size=(16, 16, 16))
    vals = [(metrics.ssim(t + s * rng.normal(size=t.shape), t),
             metrics.psnr(t + s * rng.normal(size=t.shape), t)) for s in (0.01, 0.05, 0.2)]
    assert vals[0][0] > vals[1][0] > vals[2][0]
    assert vals[0][1] > vals[1][1] > vals[2][1]


def test_ssim_of_a_scaled_image():
    """x = k t with constant-free structure: SSIM = (2k mu^2 + c1)(2k var + c2) /
    ((1 + k^2) mu^2 + c1)((1 + k^2) var + c2) where the local statistics are
    uniform, i.e. for a constant image the first factor only."""
    t = np.full((9, 9, 9), 0.5)
    t[0, 0, 0] = 1.5                # range L = 1
    t[0, 0, 1] = 0.5
    k = 0.8
    c1 = (0.01 * 1.0) ** 2
    s = metrics.ssim(k * t, t)
    # far from the corner the images are constant 0.5k vs 0.5
    mu = 0.5
    far = (2 * k * mu * mu + c1) / ((1 + k * k) * mu * mu + c1)
    assert abs(s - far) < 0.02


def test_change_recovery_endpoints():
    rng = np.random.default_rng(2)
    prior = rng.uniform(size=(10, 10, 10))
    truth = prior.copy()
    truth[4:6, 4:6, 4:6] += 1.0
    assert abs(metrics.change_recovery(prior, truth, prior) - 1.0) < 1e-12
    assert metrics.change_recovery(truth, truth, prior) == 0.0
    half = prior + 0.5 * (truth - prior)
    assert abs(metrics.change_recovery(half, truth, prior) - 0.5) < 1e-12
