"""Float64 oracle of the EMD features of the state vector (test infrastructure only).

What is computed (paper §III-D, State Representation; Table IV; the
environment vector E_t of §IV-C, Eq. 1): EMD_{W_N} and EMD_{W_P}, the Earth
Mover's Distance (Rubner et al.) between the world-normal buffer of F_t and
that of F_{t-1}, and likewise for the world-position buffer. The paper names
the metric and the buffers, not how a buffer becomes a distribution.

Readings taken here:

* Each channel of a buffer is a distribution of values over the frame's
  pixels, held as a histogram of ``bins`` uniform bins on [lo, hi]. A value v
  falls in bin floor((v - lo) * bins / (hi - lo)), computed in float64 (the
  scale bins / (hi - lo) first, then the difference, then the product),
  clamped to [0, bins - 1] (values outside the range join the end bins, +inf
  the last, -inf and NaN the first).
* The ground distance between bins i and j is |i - j| times the bin width
  (hi - lo) / bins. Both histograms hold the same mass (H * W pixels); the
  EMD of unit-mass histograms in one dimension is the L1 distance between
  their cumulative histograms times the bin width (the optimal transport in
  one dimension moves mass in order; the pins check this against the
  minimum-cost transport itself on small inputs):

      EMD = (sum_i |CA_i - CB_i|) / (H * W) * width,   CA_i = sum_{j <= i} A_j,

  with the integer sum formed exactly and the two float64 operations in
  that order.
* A buffer's feature is the sum of its channels' EMDs (three for normals and
  positions); the per-channel values are returned too.

Nothing here is shared with, or imported by, the HIP path.
"""

from __future__ import annotations

import numpy as np


def bin_index(values, lo: float, hi: float, bins: int) -> np.ndarray:
    """The histogram bin of every value (int64), as stated above."""
    v = np.asarray(values).astype(np.float64)
    scale = np.float64(bins) / (np.float64(hi) - np.float64(lo))
    with np.errstate(invalid="ignore", over="ignore"):
        t = np.floor((v - np.float64(lo)) * scale)
    # fmax / fmin return the non-NaN operand: NaN lands in bin 0
    t = np.fmin(np.fmax(t, 0.0), np.float64(bins - 1))
    return t.astype(np.int64)


def histogram(values, lo: float, hi: float, bins: int) -> np.ndarray:
    """Counts of every bin (int64)."""
    return np.bincount(bin_index(np.ravel(values), lo, hi, bins), minlength=bins).astype(np.int64)


def emd_from_histograms(ha: np.ndarray, hb: np.ndarray, width: float) -> float:
    """EMD of two histograms of equal mass with ground distance |i - j| * width."""
    ha = np.asarray(ha, np.int64)
    hb = np.asarray(hb, np.int64)
    mass = int(ha.sum())
    if mass != int(hb.sum()):
        raise ValueError("histograms of different mass")
    if mass == 0:
        return 0.0
    s = int(np.abs(np.cumsum(ha) - np.cumsum(hb)).sum())
    return float(np.float64(s) / np.float64(mass) * np.float64(width))


def channel_emd(a, b, lo: float, hi: float, bins: int) -> float:
    """EMD between the value distributions of two planes [H, W] of one channel."""
    width = (np.float64(hi) - np.float64(lo)) / np.float64(bins)
    return emd_from_histograms(histogram(a, lo, hi, bins), histogram(b, lo, hi, bins), width)


def buffer_emd(cur, prev, lo: float, hi: float, bins: int) -> np.ndarray:
    """Per-frame, per-channel EMD between buffers ``cur`` and ``prev``
    [N, C, H, W] (any float dtype; the stored values are used): [N, C] float64.
    The feature of a frame is the sum over its channels."""
    cur = np.asarray(cur)
    prev = np.asarray(prev)
    if cur.shape != prev.shape or cur.ndim != 4:
        raise ValueError("buffer_emd takes two [N, C, H, W] buffers of one shape")
    if not (bins >= 1 and np.isfinite(lo) and np.isfinite(hi) and hi > lo):
        raise ValueError("need bins >= 1 and finite lo < hi")
    n, c = cur.shape[:2]
    out = np.empty((n, c), dtype=np.float64)
    for i in range(n):
        for ch in range(c):
            out[i, ch] = channel_emd(cur[i, ch], prev[i, ch], lo, hi, bins)
    return out
