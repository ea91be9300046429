"""Float64 oracle of the per-frame scene-state statistics (test infrastructure only).

What is computed (paper §IV-C, Eq. 1: the environment vector E_t of a frame F_t): the
variance of the motion-vector buffer, taken separately for the horizontal
and the vertical component (Var_x(F_mv), Var_y(F_mv); Table IV lists the
motion variance as the feature that reveals dynamic objects, §III-D), and
the rendering resolution R = R_h x R_w. §III-C (Fig. 2) measures how many
pixels of a warped frame have no source; the out-of-frame share of that is
the invalid fraction of a warp.

Readings taken where the paper is silent:

* The statistic is the population variance (divide by the number of
  vectors) over all H x W per-pixel vectors of the frame, with its mean
  reported beside it. A field given per 16 x 16 block is the special case of
  a per-pixel field whose blocks repeat one value.
* Any non-finite component makes that component's mean and variance
  non-finite (IEEE propagation); nothing is filtered out.
* The invalid fraction counts out-of-frame samples only (the G-buffer holes
  of Fig. 2 need the renderer's buffers, which are not modelled).

The mean and the variance follow their plain definitions in two passes:
mean = (sum of the values) / n with a correctly rounded sum (``math.fsum``),
then variance = (sum of squared deviations from that mean) / n, again with
``math.fsum``. Nothing here is shared with, or imported by, the HIP path.
"""

from __future__ import annotations

import math

import numpy as np


def _mean_var(values: np.ndarray) -> tuple[float, float]:
    """Population mean and variance of a flat float array (two passes)."""
    x = np.asarray(values, dtype=np.float64).ravel()
    n = x.size
    if n == 0:
        raise ValueError("empty component")
    mean = math.fsum(x.tolist()) / n
    with np.errstate(invalid="ignore", over="ignore"):
        dev = x - mean
        var = math.fsum((dev * dev).tolist()) / n
    return mean, var


def motion_stats(mv) -> np.ndarray:
    """Per-frame motion statistics (§IV-C, Eq. 1, E_t: Var_x(F_mv), Var_y(F_mv)).

    ``mv`` is [N, 2, H, W] (component 0 horizontal, 1 vertical) or [2, H, W].
    Returns float64 [N, 4] = (mean_x, var_x, mean_y, var_y) per frame.
    """
    a = np.asarray(mv)
    if a.ndim == 3:
        a = a[None]
    if a.ndim != 4 or a.shape[1] != 2:
        raise ValueError("mv must be [N, 2, H, W]")
    out = np.empty((a.shape[0], 4), dtype=np.float64)
    for n in range(a.shape[0]):
        out[n, 0], out[n, 1] = _mean_var(a[n, 0])
        out[n, 2], out[n, 3] = _mean_var(a[n, 1])
    return out


def resolution(h: int, w: int) -> int:
    """Rendering resolution R = R_h x R_w as one integer (§IV-C, Eq. 1, E_t)."""
    return int(h) * int(w)


def invalid_fraction(invalid_count, h: int, w: int) -> np.ndarray:
    """Share of out-of-frame samples per (frame, phase) (§III-C, Fig. 2)."""
    return np.asarray(invalid_count, dtype=np.float64) / (int(h) * int(w))
