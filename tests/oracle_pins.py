"""Pins of the warp oracle: checks against facts fixed outside the oracle itself.

Each pin takes an implementation ``O`` exposing ``forward(src, mv, phases)``
and ``backward(src, mv, phases, grad_out)`` with the oracle's conventions and
raises ``AssertionError`` when it disagrees with:

* exact special cases (zero motion, integer shifts, constant images),
* closed forms (affine, bilinear and quadratic images under sub-pixel motion),
* brute force with exact rational arithmetic on tiny frames,
* independent library routines (``torch.nn.functional.grid_sample`` in
  float64 and ``scipy.ndimage.map_coordinates``),
* the adjoint identity and finite differences,
* a hand-worked example (``tests/golden/hand_2x3.json``),
* the scene generator's own motion (an integer pan).

An implementation with ``O.exact`` true takes the displacement ``s*u``
exactly (the plain definition); otherwise ``s*u`` is rounded once to float32.
The pins that depend on the displacement compute it the same way, from the
phase and the motion alone.

The same pins run on planted mistakes in ``test_oracle_mutants.py`` to show
that each plausible mistake fails at least one of them.
"""

from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def _shift_ref(img, a, b):
    """img [C,H,W] moved by integer (a, b) with zero fill: out[y, x] = img[y-b, x-a]."""
    c, h, w = img.shape
    out = np.zeros_like(img)
    ys = np.arange(h)[:, None] - b
    xs = np.arange(w)[None, :] - a
    ok = (ys >= 0) & (ys < h) & (xs >= 0) & (xs < w)
    out[:, ok] = img[:, np.clip(ys, 0, h - 1), np.clip(xs, 0, w - 1)][:, ok]
    return out, ok


def pin_identity(O):
    """Zero phase or zero motion returns the input exactly, all valid."""
    src = _rng(1).random((2, 3, 7, 9))
    mv = _rng(2).uniform(-5, 5, (2, 2, 7, 9)).astype(np.float32)
    out, mask, cnt = O.forward(src, mv, [0.0])
    assert np.array_equal(out[:, 0], src), "phase 0 must return the input"
    assert mask.all() and (cnt == 0).all()
    out, mask, cnt = O.forward(src, np.zeros_like(mv), [0.25, 0.5, 0.75, 1.0])
    for k in range(4):
        assert np.array_equal(out[:, k], src), "zero motion must return the input"
    assert mask.all() and (cnt == 0).all()


def pin_integer_shift(O):
    """Integer motion moves pixels exactly, with zero fill; checks sign and axes."""
    src = _rng(3).random((1, 2, 11, 13))
    for (a, b) in [(2, -3), (-1, 4), (5, 0), (0, -2), (13, 1)]:
        for s, scale in [(1.0, 1), (0.25, 4), (0.5, 2)]:
            mv = np.zeros((1, 2, 11, 13), np.float32)
            mv[0, 0] = a * scale
            mv[0, 1] = b * scale
            out, mask, cnt = O.forward(src, mv, [s])
            ref, ok = _shift_ref(src[0], a, b)
            assert np.array_equal(out[0, 0], ref), f"integer shift {(a, b)} at phase {s}"
            assert np.array_equal(mask[0, 0].astype(bool), ok)
            assert cnt[0, 0] == ok.size - ok.sum()


def pin_constant(O):
    """A constant image stays constant on valid pixels (weights sum to one)."""
    src = np.full((1, 2, 9, 10), 0.3)
    mv = _rng(4).uniform(-3, 3, (1, 2, 9, 10)).astype(np.float32)
    out, mask, _ = O.forward(src, mv, [0.25, 0.75, 1.0])
    exp = 0.3 * mask[:, :, None].astype(np.float64)
    assert np.abs(out - exp).max() <= 1e-15


def _exact(O) -> bool:
    return bool(getattr(O, "exact", False))


def _disp(O, s, comp):
    """The displacement s*u in the mode of ``O``: the float64 product of the
    float32 phase and motion (exact), or that product rounded to float32."""
    prod = np.float64(np.float32(s)) * np.asarray(comp, np.float32).astype(np.float64)
    return prod if _exact(O) else prod.astype(np.float32).astype(np.float64)


def _sample_points(O, mv, s, h, w):
    """Float64 sample coordinates x - d, y - d of the displacement of ``O``'s mode
    (exact here: x and d are below 2^24 with at most 26 significant bits)."""
    ys, xs = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    return xs - _disp(O, s, mv[0]), ys - _disp(O, s, mv[1])


def pin_closed_forms(O):
    """Affine, bilinear (x*y) and quadratic (x^2) images under sub-pixel motion.

    Bilinear interpolation reproduces any function a + b*x + c*y + e*x*y
    exactly, and turns x^2 into x^2 + fx*(1 - fx) with fx the fractional part.
    """
    h, w = 12, 14
    ys, xs = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64),
                         indexing="ij")
    alpha, beta, gamma, eps = 0.375, -0.8125, 2.5, 0.0625
    img = np.stack([alpha * xs + beta * ys + gamma, eps * xs * ys, xs * xs])[None]
    mv = _rng(5).uniform(-4, 4, (1, 2, h, w)).astype(np.float32)
    for s in (0.25, 0.5, 0.75, 1.0):
        out, mask, _ = O.forward(img, mv, [s])
        sx, sy = _sample_points(O, mv[0], s, h, w)
        ok = (sx >= 0) & (sx <= w - 1) & (sy >= 0) & (sy <= h - 1)
        assert np.array_equal(mask[0, 0].astype(bool), ok)
        fx = sx - np.floor(sx)
        exp = [alpha * sx + beta * sy + gamma, eps * sx * sy, sx * sx + fx * (1 - fx)]
        for ch in range(3):
            err = np.abs(out[0, 0, ch] - exp[ch])[ok].max()
            assert err <= 1e-11, f"closed form channel {ch} phase {s}: err {err}"
        assert (out[0, 0][:, ~ok] == 0).all()


def _brute_valid(dx: Fraction, dy: Fraction, x, y, h, w):
    """Exact rational test: every tap with non-zero weight lies in the frame."""
    sx = Fraction(x) - dx
    sy = Fraction(y) - dy
    cols = {math.floor(sx), math.ceil(sx)}
    rows = {math.floor(sy), math.ceil(sy)}
    return all(0 <= c < w for c in cols) and all(0 <= r < h for r in rows)


def _disp_fraction(O, s, u):
    """The displacement as an exact rational (None when it is not finite)."""
    if _exact(O):
        if not np.isfinite(u):
            return None
        return Fraction(float(np.float32(s))) * Fraction(float(u))
    d = np.float32(np.float64(np.float32(s)) * np.float64(u))
    return Fraction(float(d)) if np.isfinite(d) else None


def pin_mask_bruteforce(O):
    """Masks on tiny frames equal exact brute force, including at the exact bounds
    and one float32 ulp either side, and at motions whose product with the phase
    3/4 lies within an ulp of a bound (where the exact and the float32-rounded
    displacement can fall on different sides of it); constant motion gives the
    closed-form count."""
    for h, w in [(1, 1), (1, 3), (2, 2), (3, 5), (5, 3), (8, 8)]:
        vals = []
        for b in range(-w - 1, w + 2):
            f = np.float32(b)
            vals += [f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))]
            g = np.float32(b / 0.75)
            vals += [g, np.nextafter(g, np.float32(np.inf)), np.nextafter(g, np.float32(-np.inf))]
        vals += [np.float32(0.5), np.float32(-0.25), np.float32(np.nan), np.float32(np.inf),
                 np.float32(1e-40), np.float32(-1e-40), np.float32(-0.0)]
        vals = np.array(vals, dtype=np.float32)
        r = _rng(h * 31 + w)
        for s in (1.0, 0.75, 0.5):
            mv = np.stack([r.choice(vals, (h, w)), r.choice(vals, (h, w))])[None].astype(np.float32)
            _, mask, cnt = O.forward(np.ones((1, 1, h, w)), mv, [s])
            for y in range(h):
                for x in range(w):
                    dx = _disp_fraction(O, s, mv[0, 0, y, x])
                    dy = _disp_fraction(O, s, mv[0, 1, y, x])
                    exp = (dx is not None and dy is not None
                           and _brute_valid(dx, dy, x, y, h, w))
                    assert bool(mask[0, 0, y, x]) == exp, (h, w, s, x, y, dx, dy)
            assert cnt[0, 0] == h * w - int(mask.sum())
    # Constant motion: valid count = max(0, W - ceil|dx|) * max(0, H - ceil|dy|).
    h, w = 9, 12
    for dx, dy in [(0.5, 0.0), (2.25, -1.0), (-3.0, 4.5), (11.5, 0.0), (12.0, 1.0), (0.0, -8.75)]:
        mv = np.zeros((1, 2, h, w), np.float32)
        mv[0, 0], mv[0, 1] = dx, dy
        _, mask, cnt = O.forward(np.zeros((1, 1, h, w)), mv, [1.0])
        nvalid = max(0, w - math.ceil(abs(dx))) * max(0, h - math.ceil(abs(dy)))
        assert int(mask.sum()) == nvalid and cnt[0, 0] == h * w - nvalid, (dx, dy)


def pin_library(O):
    """Forward and backward agree with torch grid_sample (float64, bilinear,
    align_corners=True, zero padding) on valid pixels and with
    scipy.ndimage.map_coordinates(order=1)."""
    import scipy.ndimage as nd
    import torch
    import torch.nn.functional as F

    n, c, h, w = 2, 3, 10, 13
    src = _rng(6).random((n, c, h, w))
    mv = _rng(7).uniform(-4, 4, (n, 2, h, w)).astype(np.float32)
    for s in (0.5, 1.0):
        out, mask, _ = O.forward(src, mv, [s])
        sx = np.empty((n, h, w))
        sy = np.empty((n, h, w))
        for i in range(n):
            sx[i], sy[i] = _sample_points(O, mv[i], s, h, w)
        gx = torch.tensor(2.0 * sx / (w - 1) - 1.0, requires_grad=True)
        gy = torch.tensor(2.0 * sy / (h - 1) - 1.0, requires_grad=True)
        t_src = torch.tensor(src, requires_grad=True)
        ref = F.grid_sample(t_src, torch.stack([gx, gy], dim=-1), mode="bilinear",
                            padding_mode="zeros", align_corners=True)
        m = torch.tensor(mask[:, 0].astype(np.float64))[:, None]
        ref_masked = (ref * m).detach().numpy()
        assert np.abs(out[:, 0] - ref_masked).max() <= 1e-12, "grid_sample forward"
        for i in range(n):
            for ch in range(c):
                mc = nd.map_coordinates(src[i, ch], [sy[i], sx[i]], order=1, mode="constant",
                                        cval=0.0)
                ok = mask[i, 0].astype(bool)
                assert np.abs(mc[ok] - out[i, 0, ch][ok]).max() <= 1e-12, "map_coordinates"
        # Backward through the library: L = sum(G * mask * grid_sample).
        g = _rng(8).standard_normal((n, 1, c, h, w))
        (ref * m * torch.tensor(g[:, 0])).sum().backward()
        gs, gm = O.backward(src, mv, [s], g)
        assert np.abs(gs - t_src.grad.numpy()).max() <= 1e-12, "grid_sample image gradient"
        fx = sx - np.floor(sx)
        fy = sy - np.floor(sy)
        away = (fx > 1e-6) & (fx < 1 - 1e-6) & (fy > 1e-6) & (fy < 1 - 1e-6)
        lib_gu = -s * (2.0 / (w - 1)) * gx.grad.numpy()
        lib_gv = -s * (2.0 / (h - 1)) * gy.grad.numpy()
        assert np.abs(gm[:, 0][away] - lib_gu[away]).max() <= 1e-10, "grid_sample motion grad x"
        assert np.abs(gm[:, 1][away] - lib_gv[away]).max() <= 1e-10, "grid_sample motion grad y"


def pin_adjoint(O):
    """<W x, y> = <x, W^T y> for a fixed motion field, all four phases at once."""
    n, c, h, w = 2, 3, 17, 19
    mv = _rng(9).uniform(-6, 6, (n, 2, h, w)).astype(np.float32)
    x = _rng(10).standard_normal((n, c, h, w))
    phases = [0.25, 0.5, 0.75, 1.0]
    y = _rng(11).standard_normal((n, 4, c, h, w))
    wx, _, _ = O.forward(x, mv, phases)
    wty, _ = O.backward(np.zeros_like(x), mv, phases, y)
    lhs = float((wx * y).sum())
    rhs = float((x * wty).sum())
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs)), (lhs, rhs)


def pin_finite_differences(O):
    """Motion gradient by central differences of each pixel's own loss term
    (an output pixel depends only on its own motion), away from floor kinks and
    frame bounds; image gradient by a directional difference (the loss is
    linear in the image)."""
    n, c, h, w = 1, 3, 16, 18
    src = _rng(12).random((n, c, h, w))
    mv = _rng(13).uniform(-4, 4, (n, 2, h, w)).astype(np.float32)
    phases = [0.5, 1.0]
    g = _rng(14).standard_normal((n, 2, c, h, w))
    _, gm = O.backward(src, mv, phases, g)
    hstep = np.float32(1e-3)
    for comp in (0, 1):
        plus = mv.copy()
        minus = mv.copy()
        plus[:, comp] = mv[:, comp] + hstep
        minus[:, comp] = mv[:, comp] - hstep
        step = (plus[:, comp].astype(np.float64) - minus[:, comp].astype(np.float64))
        op, mp, _ = O.forward(src, plus, phases)
        om, mm, _ = O.forward(src, minus, phases)
        lp = (g * op).sum(axis=(1, 2))
        lm = (g * om).sum(axis=(1, 2))
        fd = (lp - lm) / step
        # keep pixels whose cell and validity do not change over [-h, h] at any phase
        keep = np.ones((n, h, w), bool)
        ys, xs = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
        for s in phases:
            coord = (xs if comp == 0 else ys) - s * mv[:, comp].astype(np.float64)
            frac = coord - np.floor(coord)
            keep &= (frac > 4 * float(hstep)) & (frac < 1 - 4 * float(hstep))
        keep &= (mp == mm).all(axis=1)
        assert keep.sum() > 0.5 * keep.size
        err = np.abs(fd - gm[:, comp])[keep].max()
        scale = max(1.0, np.abs(gm[:, comp][keep]).max())
        assert err <= 1e-6 * scale, f"motion FD component {comp}: {err}"
    # image: L(I) = <G, W I> is linear, so a central difference is exact.
    d = _rng(15).standard_normal(src.shape)
    gs, _ = O.backward(src, mv, phases, g)
    lp = (g * O.forward(src + 0.5 * d, mv, phases)[0]).sum()
    lm = (g * O.forward(src - 0.5 * d, mv, phases)[0]).sum()
    assert abs((lp - lm) - (gs * d).sum()) <= 1e-9 * max(1.0, abs(lp - lm))


def pin_golden(O):
    """The hand-worked 2x3 example."""
    with open(os.path.join(GOLDEN, "hand_2x3.json")) as f:
        gold = json.load(f)
    img = np.array(gold["image"], dtype=np.float64)[None]
    for case in gold["cases"]:
        mv = np.zeros((1, 2, 2, 3), np.float32)
        mv[0, 0], mv[0, 1] = case["mv"]
        out, mask, cnt = O.forward(img, mv, [case["phase"]])
        assert np.array_equal(out[0, 0], np.array(case["out"], np.float64)), case["name"]
        assert np.array_equal(mask[0, 0], np.array(case["mask"])), case["name"]
        assert cnt[0, 0] == case["invalid_count"], case["name"]
        g = np.where(mask[0, 0] == 1, case["grad_out_valid"], case["grad_out_invalid"])
        gs, gm = O.backward(img, mv, [case["phase"]], g[None, None, None].astype(np.float64))
        assert np.array_equal(gs[0], np.array(case["grad_src"], np.float64)), case["name"]
        if case["grad_mv"] is not None:
            assert np.array_equal(gm[0], np.array(case["grad_mv"], np.float64)), case["name"]


def pin_generator_pan(O):
    """With an integer camera pan and no moving objects, warping frame i by its
    own motion at phase 1 gives frame i+1 on every valid pixel (paper §III-D:
    without dynamic objects, motion vectors and warping predict the next frame)."""
    from synth import pan_rect_sequence

    frames, mv, _ = pan_rect_sequence(_rng(16), 3, 20, 24, kind="rgb", n_rects=0,
                                      pan=(2.0, -3.0))
    out, mask, _ = O.forward(frames[:2], mv[:2], [1.0])
    ok = mask[:, 0].astype(bool)
    nxt = frames[1:3].astype(np.float64)
    assert ok.sum() > 0
    for ch in range(3):
        assert np.array_equal(out[:, 0, ch][ok], nxt[:, ch][ok])


def pin_phase_scaling(O):
    """Motion u at phase s and motion 2u at phase s/2 give the same displacement,
    hence identical outputs (exact for power-of-two phases)."""
    src = _rng(17).random((1, 2, 9, 11))
    mv = _rng(18).uniform(-3, 3, (1, 2, 9, 11)).astype(np.float32)
    a, ma, _ = O.forward(src, mv, [1.0, 0.5])
    b, mb, _ = O.forward(src, (2 * mv).astype(np.float32), [0.5, 0.25])
    assert np.array_equal(a, b) and np.array_equal(ma, mb)


ALL_PINS = [pin_identity, pin_integer_shift, pin_constant, pin_closed_forms,
            pin_mask_bruteforce, pin_library, pin_adjoint, pin_finite_differences,
            pin_golden, pin_generator_pan, pin_phase_scaling]
