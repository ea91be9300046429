"""Planted mistakes in the NumPy oracle must each fail at least one pin (CPU only).

Each mutant patches one step of the oracle (on the CPU, in this process) with
a plausible error: a flipped sign, swapped axes or weights, a dropped term, an
off-by-one bound, a missing phase factor. The pins in ``oracle_pins`` must
catch every one, so a passing oracle is not passing by accident. Every
mutant is planted in both displacement modes (float32-rounded and exact),
except the two that swap one mode's displacement for the other's, which are
planted only in the mode they contradict.
"""

import types

import numpy as np
import pytest

from oracle import warp_oracle

import oracle_pins

_taps = warp_oracle.taps
_displacement = warp_oracle.displacement
_sample = warp_oracle.sample
_backward = warp_oracle.backward


def _taps_sign(u, v, s, xs, ys, h, w, exact=False):
    return _taps(-np.asarray(u), -np.asarray(v), s, xs, ys, h, w, exact)


def _taps_axes(u, v, s, xs, ys, h, w, exact=False):
    return _taps(v, u, s, xs, ys, h, w, exact)


def _taps_weights(u, v, s, xs, ys, h, w, exact=False):
    valid, x0, x1, y0, y1, fx, fy = _taps(u, v, s, xs, ys, h, w, exact)
    return valid, x0, x1, y0, y1, np.where(valid, 1 - fx, 0.0), fy


def _taps_one_column(u, v, s, xs, ys, h, w, exact=False):
    valid, x0, x1, y0, y1, fx, fy = _taps(u, v, s, xs, ys, h, w, exact)
    return valid, x0, x0, y0, y1, fx, fy


def _taps_strict_bound(u, v, s, xs, ys, h, w, exact=False):
    valid, x0, x1, y0, y1, fx, fy = _taps(u, v, s, xs, ys, h, w, exact)
    sx = np.asarray(xs, np.float64) - _displacement(u, s, exact)
    with np.errstate(invalid="ignore"):
        valid = valid & (sx < w - 1)
    return valid, x0, x1, y0, y1, fx, fy


def _taps_floor_of_x_only(u, v, s, xs, ys, h, w, exact=False):
    # rounds the sample point to the nearest pixel instead of interpolating
    valid, x0, x1, y0, y1, fx, fy = _taps(u, v, s, xs, ys, h, w, exact)
    return valid, x0, x1, y0, y1, np.round(fx), np.round(fy)


def _disp_exact(comp, phase, exact=False):
    return _displacement(comp, phase, True)


def _disp_rounded(comp, phase, exact=False):
    return _displacement(comp, phase, False)


def _disp_unscaled(comp, phase, exact=False):
    return _displacement(comp, 1.0 if phase != 0 else 0.0, exact)


def _sample_drop_cross(img, u, v, phase, xs, ys, exact=False):
    img = np.asarray(img, np.float64)
    h, w = img.shape[-2:]
    valid, x0, x1, y0, y1, fx, fy = warp_oracle.taps(np.ravel(u), np.ravel(v), phase,
                                                     np.ravel(xs), np.ravel(ys), h, w, exact)
    val = ((1 - fx) * (1 - fy) * img[:, y0, x0] + fx * (1 - fy) * img[:, y0, x1]
           + (1 - fx) * fy * img[:, y1, x0])
    return np.where(valid, val, 0.0), valid


def _sample_no_zero(img, u, v, phase, xs, ys, exact=False):
    """Clamps the sample point into the frame instead of zeroing invalid pixels."""
    img = np.asarray(img, np.float64)
    h, w = img.shape[-2:]
    _, valid = _sample(img, u, v, phase, xs, ys, exact)
    with np.errstate(invalid="ignore"):
        sx = np.clip(np.ravel(xs) - _displacement(np.ravel(u), phase, exact), 0, w - 1)
        sy = np.clip(np.ravel(ys) - _displacement(np.ravel(v), phase, exact), 0, h - 1)
    sx = np.nan_to_num(sx)
    sy = np.nan_to_num(sy)
    x0 = np.floor(sx).astype(np.int64)
    y0 = np.floor(sy).astype(np.int64)
    fx, fy = sx - x0, sy - y0
    x1, y1 = np.minimum(x0 + 1, w - 1), np.minimum(y0 + 1, h - 1)
    val = ((1 - fx) * (1 - fy) * img[:, y0, x0] + fx * (1 - fy) * img[:, y0, x1]
           + (1 - fx) * fy * img[:, y1, x0] + fx * fy * img[:, y1, x1])
    return val, valid


def _backward_neg_motion(src, mv, phases, g, exact=False):
    gs, gm = _backward(src, mv, phases, g, exact)
    return gs, -gm


def _backward_no_phase(src, mv, phases, g, exact=False):
    gs, gm = _backward(src, mv, phases, g, exact)
    return gs, gm / float(np.asarray(phases, np.float32)[-1])


def _backward_swap_motion(src, mv, phases, g, exact=False):
    gs, gm = _backward(src, mv, phases, g, exact)
    return gs, gm[:, ::-1].copy()


def _backward_swapped_scatter(src, mv, phases, g, exact=False):
    """Sends each output gradient to the image through transposed weights."""
    n, c, h, w = np.asarray(src).shape
    gs = np.zeros((n, c, h, w))
    _, gm = _backward(src, mv, phases, g, exact)
    ys, xs = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    for i in range(n):
        for j, s in enumerate(np.asarray(phases, np.float32).reshape(-1)):
            valid, x0, x1, y0, y1, fx, fy = _taps(mv[i, 0].ravel(), mv[i, 1].ravel(), s,
                                                  xs.ravel(), ys.ravel(), h, w, exact)
            gg = np.asarray(g, np.float64)[i, j].reshape(c, -1) * valid
            for yy, xx, wt in ((y0, x0, (1 - fx) * (1 - fy)), (y0, x1, (1 - fx) * fy),
                               (y1, x0, fx * (1 - fy)), (y1, x1, fx * fy)):
                for ch in range(c):
                    gs[i, ch] += np.bincount(yy * w + xx, weights=wt * gg[ch],
                                             minlength=h * w).reshape(h, w)
    return gs, gm


MUTANTS = {
    "sign": ("taps", _taps_sign),
    "axes": ("taps", _taps_axes),
    "weights": ("taps", _taps_weights),
    "one_column": ("taps", _taps_one_column),
    "strict_bound": ("taps", _taps_strict_bound),
    "nearest": ("taps", _taps_floor_of_x_only),
    "exact_displacement": ("displacement", _disp_exact),
    "rounded_displacement": ("displacement", _disp_rounded),
    "unscaled": ("displacement", _disp_unscaled),
    "drop_cross_term": ("sample", _sample_drop_cross),
    "no_zero_fill": ("sample", _sample_no_zero),
    "neg_motion_grad": ("backward", _backward_neg_motion),
    "no_phase_factor": ("backward", _backward_no_phase),
    "swapped_motion_grad": ("backward", _backward_swap_motion),
    "swapped_scatter_weights": ("backward", _backward_swapped_scatter),
}


# mutants planted only in one mode: each one is that mode's correct behaviour
# in the other
ONLY_MODE = {"exact_displacement": False, "rounded_displacement": True}


def _oracle(exact):
    """The (possibly patched) oracle in one mode, resolved at call time."""
    return types.SimpleNamespace(
        exact=exact,
        forward=lambda src, mv, ph: warp_oracle.forward(src, mv, ph, exact=exact),
        backward=lambda src, mv, ph, g: warp_oracle.backward(src, mv, ph, g, exact=exact))


def _run_pins(O):
    failed = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(O)
        except Exception as exc:  # a crash counts as a caught mistake too
            failed.append((pin.__name__, type(exc).__name__))
    return failed


CASES = [(name, exact) for name in sorted(MUTANTS) for exact in (False, True)
         if ONLY_MODE.get(name, exact) == exact]


@pytest.mark.parametrize("name,exact", CASES,
                         ids=[f"{n}-{'exact' if e else 'rounded'}" for n, e in CASES])
def test_mutant_is_caught(name, exact, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(warp_oracle, attr, fn)
    assert _run_pins(_oracle(exact)), f"mutant {name} passed every pin"


@pytest.mark.parametrize("exact", [False, True], ids=["rounded", "exact"])
def test_count_mutant_is_caught(exact):
    def fwd(src, mv, phases):
        out, mask, cnt = warp_oracle.forward(src, mv, phases, exact=exact)
        return out, mask, mask.reshape(mask.shape[0], mask.shape[1], -1).sum(axis=2)
    O = types.SimpleNamespace(exact=exact, forward=fwd,
                              backward=lambda s, m, p, g: warp_oracle.backward(s, m, p, g, exact=exact))
    assert _run_pins(O)


@pytest.mark.parametrize("exact", [False, True], ids=["rounded", "exact"])
def test_unmutated_oracle_passes_every_pin(exact):
    assert _run_pins(_oracle(exact)) == []
