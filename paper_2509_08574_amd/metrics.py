"""Image-quality metrics over whole 3-D volumes (as in the paper's Sec. 3 tables).

PSNR with the ground truth's peak as the signal range, SSIM of Wang, Bovik,
Sheikh & Simoncelli (2004) with an isotropic Gaussian window (sigma 1.5
voxels, the published default) averaged over all voxels, and the relative L2
error.  Plain NumPy/SciPy on the host.
"""
import numpy as np
from scipy.ndimage import gaussian_filter


def rel_l2(x, truth) -> float:
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(truth, dtype=np.float64)
    return float(np.linalg.norm(x - t) / np.linalg.norm(t))


def psnr(x, truth) -> float:
    """10 log10(peak^2 / MSE), peak = max |truth|."""
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(truth, dtype=np.float64)
    mse = float(np.mean((x - t) ** 2))
    peak = float(np.max(np.abs(t)))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(peak * peak / mse)


def ssim(x, truth, sigma: float = 1.5) -> float:
    """Mean SSIM with Gaussian-weighted local statistics; the dynamic range L is
    that of the ground truth, K1 = 0.01, K2 = 0.03."""
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(truth, dtype=np.float64)
    L = float(t.max() - t.min())
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    f = lambda a: gaussian_filter(a, sigma, mode="reflect", truncate=3.5)  # noqa: E731
    mx, mt = f(x), f(t)
    vx = f(x * x) - mx * mx
    vt = f(t * t) - mt * mt
    cxt = f(x * t) - mx * mt
    s = ((2 * mx * mt + c1) * (2 * cxt + c2)) / ((mx * mx + mt * mt + c1) * (vx + vt + c2))
    return float(s.mean())


def change_recovery(x, truth, prior, dilate: int = 2) -> float:
    """||x - truth|| / ||truth - prior|| over the voxels where truth and prior
    differ, grown by `dilate` voxels: 1 when x shows none of the change (x =
    prior there), 0 when it recovers it exactly."""
    from scipy.ndimage import binary_dilation
    t = np.asarray(truth, dtype=np.float64)
    p = np.asarray(prior, dtype=np.float64)
    m = binary_dilation(t != p, iterations=dilate)
    d = np.linalg.norm((t - p)[m])
    return float(np.linalg.norm((np.asarray(x, dtype=np.float64) - t)[m]) / d)
