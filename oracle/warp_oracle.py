"""Float64 NumPy oracle of the motion-vector backward warp (test infrastructure only).

What is computed (paper §II-B: warping maps every location of one image to a
location in another; §IV-B: the predicted frame P_i is shown at t + i/4 and is
made from F_t alone; §III-B: warped pixels without a valid source are marked
invalid; §III-D: the motion-vector buffer holds each pixel's direction and
magnitude of motion):

    P(n, s)[c, y, x] = bilinear sample of F_n[c] at (x - s*u, y - s*v)

with ``(u, v) = mv[n, :, y, x]`` the screen-space motion of the content over
one rendered-frame interval (+x right, +y down, in pixels) and ``s`` the
phase. The paper does not spell out the arithmetic; the readings taken here
are:

* Backward warp (gather): the motion vector is read at the output pixel.
* Samples sit at integer pixel indices; bilinear interpolation over the four
  neighbours ``(x0, y0) .. (x0+1, y0+1)`` with ``x0 = floor(sx)``; the second
  index is clamped to the last column/row, where its weight is exactly zero.
* A pixel is valid iff ``0 <= sx <= W-1`` and ``0 <= sy <= H-1`` (a closed
  box: every tap with non-zero weight lies inside the frame). Invalid pixels
  are 0 in every channel, get mask 0, and are counted. NaN/Inf motion is
  invalid. The test is evaluated exactly (on the displacement against integer
  bounds), and the cell as ``x0 = x - ceil(d)`` with fraction ``ceil(d) - d``,
  so that a displacement far below an ulp of x is not rounded away.
* Two modes for the displacement ``d = s*u``. The exact mode
  (``exact=True``) is the plain definition: ``s*u`` in float64, which is
  exact because ``s`` and ``u`` are float32 (a product of two 24-bit
  significands fits in 53 bits). The default mode rounds ``s*u`` once to
  float32, the precision of the motion field, so that the validity decision
  is taken in the precision a float32 implementation takes it in. For phases
  0, 1/4, 1/2 and 1 the product is exact and the two modes agree; for 3/4
  they differ by at most 2^-24 relative in ``d``, so a mask can differ only
  where the exact sample point lies within half a float32 ulp of ``d`` from a
  frame bound. Everything after the displacement is exact or float64.
* Backward pass: the transpose of the bilinear gather for the image, and the
  derivative of the bilinear blend along the sampling coordinate for the
  motion, using the right-derivative at the floor kinks; summed over phases;
  zero at invalid pixels.

All values are returned in float64. Nothing here is shared with, or imported
by, the HIP path.
"""

from __future__ import annotations

import numpy as np


def displacement(comp: np.ndarray, phase: float, exact: bool = False) -> np.ndarray:
    """``s * mv`` as float64: exact, or rounded once to float32.

    The product of two float32 numbers is exact in float64, so it is the exact
    displacement, and rounding it to float32 gives the correctly rounded
    float32 product.
    """
    s = np.float64(np.float32(phase))
    prod = s * np.asarray(comp, dtype=np.float32).astype(np.float64)
    if exact:
        return prod
    return prod.astype(np.float32).astype(np.float64)


def taps(u: np.ndarray, v: np.ndarray, phase: float, xs: np.ndarray, ys: np.ndarray,
         h: int, w: int, exact: bool = False):
    """Bilinear taps of the output pixels ``(xs, ys)`` whose motion is ``(u, v)``.

    Returns ``valid, x0, x1, y0, y1, fx, fy`` (arrays shaped like ``xs``);
    indices and fractions of invalid pixels are set to 0.
    """
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    dx = displacement(u, phase, exact)
    dy = displacement(v, phase, exact)
    # 0 <= x - d <= W-1, stated on d against integer bounds: exact even where
    # |d| is below half an ulp of x and forming x - d would round.
    with np.errstate(invalid="ignore"):
        valid = ((dx <= xs) & (dx >= xs - (w - 1)) & (dy <= ys) & (dy >= ys - (h - 1)))
    dx = np.where(valid, dx, 0.0)
    dy = np.where(valid, dy, 0.0)
    # floor(x - d) = x - ceil(d) for integer x; the fraction is ceil(d) - d.
    cx = np.ceil(dx)
    cy = np.ceil(dy)
    x0 = np.where(valid, xs - cx.astype(np.int64), 0)
    y0 = np.where(valid, ys - cy.astype(np.int64), 0)
    fx = cx - dx
    fy = cy - dy
    x1 = np.minimum(x0 + 1, w - 1)
    y1 = np.minimum(y0 + 1, h - 1)
    return valid, x0, x1, y0, y1, fx, fy


def _as_f64(a) -> np.ndarray:
    return np.asarray(a).astype(np.float64)


def sample(img: np.ndarray, u, v, phase: float, xs, ys, exact: bool = False):
    """Warp of one frame ``img`` [C, H, W] at output pixels ``(xs, ys)``.

    ``u, v`` are the motion components at those output pixels. Returns
    ``(values [C, P] float64, valid [P] bool)`` for the flattened pixels.
    """
    img = _as_f64(img)
    h, w = img.shape[-2:]
    valid, x0, x1, y0, y1, fx, fy = taps(np.ravel(u), np.ravel(v), phase, np.ravel(xs),
                                         np.ravel(ys), h, w, exact)
    i00 = img[:, y0, x0]
    i01 = img[:, y0, x1]
    i10 = img[:, y1, x0]
    i11 = img[:, y1, x1]
    val = ((1.0 - fx) * (1.0 - fy) * i00 + fx * (1.0 - fy) * i01
           + (1.0 - fx) * fy * i10 + fx * fy * i11)
    return np.where(valid, val, 0.0), valid


def forward(src, mv, phases, exact: bool = False):
    """Warp every frame at every phase.

    ``src`` [N, C, H, W] (any float dtype: the stored values are upcast),
    ``mv`` [N, 2, H, W] float32, ``phases`` [K].
    Returns ``out`` [N, K, C, H, W] float64, ``mask`` [N, K, H, W] uint8 and
    ``invalid_count`` [N, K] int64.
    """
    src = _as_f64(src)
    mv = np.asarray(mv, dtype=np.float32)
    n, c, h, w = src.shape
    phases = np.asarray(phases, dtype=np.float32).reshape(-1)
    k = phases.size
    ys, xs = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    out = np.zeros((n, k, c, h, w), dtype=np.float64)
    mask = np.zeros((n, k, h, w), dtype=np.uint8)
    count = np.zeros((n, k), dtype=np.int64)
    for i in range(n):
        for j in range(k):
            val, valid = sample(src[i], mv[i, 0], mv[i, 1], phases[j], xs, ys, exact)
            out[i, j] = val.reshape(c, h, w)
            mask[i, j] = valid.reshape(h, w)
            count[i, j] = valid.size - int(valid.sum())
    return out, mask, count


def backward(src, mv, phases, grad_out, exact: bool = False):
    """Gradients of ``sum(grad_out * forward(src, mv, phases)[0])``.

    Returns ``grad_src`` [N, C, H, W] and ``grad_mv`` [N, 2, H, W], float64,
    each summed over the K phases.
    """
    src = _as_f64(src)
    g_all = _as_f64(grad_out)
    mv = np.asarray(mv, dtype=np.float32)
    n, c, h, w = src.shape
    phases = np.asarray(phases, dtype=np.float32).reshape(-1)
    ys, xs = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    xs = xs.ravel()
    ys = ys.ravel()
    grad_src = np.zeros_like(src)
    grad_mv = np.zeros((n, 2, h, w), dtype=np.float64)
    for i in range(n):
        img = src[i]
        for j, s in enumerate(phases):
            valid, x0, x1, y0, y1, fx, fy = taps(mv[i, 0].ravel(), mv[i, 1].ravel(), s, xs, ys,
                                                 h, w, exact)
            g = g_all[i, j].reshape(c, -1) * valid  # zero for invalid pixels
            # Image: transpose of the gather, one scatter per tap.
            for yy, xx, wt in ((y0, x0, (1 - fx) * (1 - fy)), (y0, x1, fx * (1 - fy)),
                               (y1, x0, (1 - fx) * fy), (y1, x1, fx * fy)):
                flat = yy * w + xx
                for ch in range(c):
                    grad_src[i, ch] += np.bincount(flat, weights=wt * g[ch],
                                                   minlength=h * w).reshape(h, w)
            # Motion: d out / d sx and d out / d sy of the bilinear blend, times
            # d sx / d u = d sy / d v = -s.
            i00 = img[:, y0, x0]
            i01 = img[:, y0, x1]
            i10 = img[:, y1, x0]
            i11 = img[:, y1, x1]
            d_sx = (1 - fy) * (i01 - i00) + fy * (i11 - i10)
            d_sy = (1 - fx) * (i10 - i00) + fx * (i11 - i01)
            s64 = np.float64(s)
            grad_mv[i, 0] += (-s64 * (g * d_sx).sum(axis=0)).reshape(h, w)
            grad_mv[i, 1] += (-s64 * (g * d_sy).sum(axis=0)).reshape(h, w)
    return grad_src, grad_mv


# ------------------------------------------------- point-wise (sampled) forms

def forward_at(src_frame, mv_frame, phase: float, ys, xs, exact: bool = False):
    """Outputs of one frame at one phase at the listed pixels only.

    ``src_frame`` [C, H, W], ``mv_frame`` [2, H, W]. Returns ``(values [C, P],
    valid [P])``; used to check full-size runs on a sample of pixels.
    """
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    mvf = np.asarray(mv_frame, dtype=np.float32)
    return sample(src_frame, mvf[0, ys, xs], mvf[1, ys, xs], phase, xs, ys, exact)


def grad_mv_at(src_frame, mv_frame, phases, grad_out_frame, ys, xs, exact: bool = False):
    """``grad_mv`` of one frame at the listed pixels: [2, P] float64.

    ``grad_out_frame`` is [K, C, H, W]. A pixel's motion gradient depends only
    on that pixel's own output, so it can be evaluated one pixel at a time.
    """
    img = _as_f64(src_frame)
    h, w = img.shape[-2:]
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    mvf = np.asarray(mv_frame, dtype=np.float32)
    out = np.zeros((2, ys.size), dtype=np.float64)
    for j, s in enumerate(np.asarray(phases, dtype=np.float32).reshape(-1)):
        valid, x0, x1, y0, y1, fx, fy = taps(mvf[0, ys, xs], mvf[1, ys, xs], s, xs, ys, h, w,
                                             exact)
        g = _as_f64(grad_out_frame[j][:, ys, xs]) * valid
        d_sx = (1 - fy) * (img[:, y0, x1] - img[:, y0, x0]) + fy * (img[:, y1, x1] - img[:, y1, x0])
        d_sy = (1 - fx) * (img[:, y1, x0] - img[:, y0, x0]) + fx * (img[:, y1, x1] - img[:, y0, x1])
        out[0] += -np.float64(s) * (g * d_sx).sum(axis=0)
        out[1] += -np.float64(s) * (g * d_sy).sum(axis=0)
    return out


def grad_src_at(mv_frame, phases, grad_out_frame, ys, xs, radius: int, exact: bool = False):
    """``grad_src`` of one frame at the listed source pixels: [C, P] float64.

    For each listed source pixel q, every output pixel within ``radius`` of q
    (Chebyshev distance) is examined and its bilinear weights onto q are
    summed, times its output gradient. ``radius`` must be at least
    ``ceil(max |s * mv|) + 1`` for the result to be complete.
    """
    mvf = np.asarray(mv_frame, dtype=np.float32)
    g_all = _as_f64(grad_out_frame)
    k, c, h, w = g_all.shape
    phases = np.asarray(phases, dtype=np.float32).reshape(-1)
    res = np.zeros((c, len(ys)), dtype=np.float64)
    off = np.arange(-radius, radius + 1)
    for idx, (qy, qx) in enumerate(zip(np.asarray(ys).tolist(), np.asarray(xs).tolist())):
        py = np.clip(qy + off, 0, h - 1)
        px = np.clip(qx + off, 0, w - 1)
        py = np.unique(py)
        px = np.unique(px)
        gy, gx = np.meshgrid(py, px, indexing="ij")
        gy = gy.ravel()
        gx = gx.ravel()
        for j, s in enumerate(phases):
            valid, x0, x1, y0, y1, fx, fy = taps(mvf[0, gy, gx], mvf[1, gy, gx], s, gx, gy, h, w,
                                                 exact)
            wsum = np.zeros(gy.size, dtype=np.float64)
            for yy, xx, wt in ((y0, x0, (1 - fx) * (1 - fy)), (y0, x1, fx * (1 - fy)),
                               (y1, x0, (1 - fx) * fy), (y1, x1, fx * fy)):
                wsum += np.where((yy == qy) & (xx == qx) & valid, wt, 0.0)
            res[:, idx] += (g_all[j][:, gy, gx] * wsum).sum(axis=1)
    return res
