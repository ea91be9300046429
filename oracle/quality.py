"""Float64 oracle of the frame-quality measures (test infrastructure only).

What is computed (paper §IV-C1, the reward of the decision predictor): the gain
in PSNR and SSIM of the frame an action produces over the frame the other
action would have produced, both measured against the ground-truth frame.
PSNR is 10 log10(peak^2 / MSE) with the 8-bit peak 255 in the paper; SSIM is
named without parameters.

Readings taken where the paper is silent:

* Frames here are float in [0, 1], so the peak is 1.0 (the float equivalent
  of 255 for 8-bit frames); it is an argument.
* MSE is the mean over all channels and pixels of a frame (holes of a warped
  frame count as errors like any other pixel). MSE = 0 gives PSNR = +inf.
* SSIM is the structural similarity index of Wang, Bovik, Sheikh and
  Simoncelli (2004) in its usual form: an 11 x 11 Gaussian window with
  standard deviation 1.5, normalised to sum 1; C1 = (0.01 peak)^2,
  C2 = (0.03 peak)^2; local means, variances and covariance are the
  window-weighted moments; the index map is evaluated where the window lies
  inside the frame (no padding), averaged over those positions and then over
  channels. Frames smaller than 11 x 11 have no SSIM.

Window sums use FFT convolution (``scipy.signal.fftconvolve``) as the
library step. Nothing here is shared with, or imported by, the HIP path.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.signal import fftconvolve

WIN = 11
SIGMA = 1.5
K1, K2 = 0.01, 0.03


def gaussian_window(size: int = WIN, sigma: float = SIGMA) -> np.ndarray:
    """The normalised size x size Gaussian weighting window (float64)."""
    r = np.arange(size, dtype=np.float64) - (size - 1) / 2
    g = np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / (2 * sigma * sigma))
    return g / g.sum()


def mse(a, b) -> float:
    """Mean squared difference over all elements of one frame."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return math.fsum((d * d).ravel().tolist()) / d.size


def psnr(a, b, peak: float = 1.0) -> float:
    """10 log10(peak^2 / MSE) of one frame (§IV-C1); +inf for identical frames."""
    m = mse(a, b)
    return math.inf if m == 0.0 else 10.0 * math.log10(peak * peak / m)


def ssim_map(x, y, peak: float = 1.0) -> np.ndarray:
    """SSIM index map of one channel [H, W] -> [H-10, W-10]."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.shape != y.shape or x.ndim != 2:
        raise ValueError("ssim_map takes two [H, W] planes of one shape")
    if x.shape[0] < WIN or x.shape[1] < WIN:
        raise ValueError("frames smaller than the 11 x 11 window have no SSIM")
    g = gaussian_window()

    def wsum(img):  # window-weighted sum at every position where the window fits
        return fftconvolve(img, g[::-1, ::-1], mode="valid")

    c1 = (K1 * peak) ** 2
    c2 = (K2 * peak) ** 2
    mx, my = wsum(x), wsum(y)
    sxx = wsum(x * x) - mx * mx
    syy = wsum(y * y) - my * my
    sxy = wsum(x * y) - mx * my
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))


def ssim(a, b, peak: float = 1.0) -> float:
    """Mean SSIM of one frame [C, H, W]: mean over positions, then channels."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.ndim == 2:
        a, b = a[None], b[None]
    return float(np.mean([ssim_map(a[c], b[c], peak).mean() for c in range(a.shape[0])]))


def frame_quality(pred, truth, peak: float = 1.0) -> np.ndarray:
    """Per-frame (MSE, PSNR, SSIM) of a batch [..., C, H, W] -> [..., 3]."""
    pred = np.asarray(pred)
    truth = np.asarray(truth)
    lead = pred.shape[:-3]
    out = np.empty(lead + (3,), dtype=np.float64)
    for idx in np.ndindex(*lead):
        m = mse(pred[idx], truth[idx])
        out[idx + (0,)] = m
        out[idx + (1,)] = math.inf if m == 0.0 else 10.0 * math.log10(peak * peak / m)
        out[idx + (2,)] = ssim(pred[idx], truth[idx], peak)
    return out
