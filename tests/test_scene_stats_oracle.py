"""Pins of the scene-statistics oracle (CPU only).

The per-frame motion mean and population variance (paper §IV-C, Eq. 1, E_t) are
checked against facts fixed outside the oracle: exact rational arithmetic on
small fields, closed forms (constant, two-valued and ramp fields), the
invariances of a variance (shift, scale, permutation), and NumPy's own
variance as an independent routine. Planted mistakes (sample instead of
population variance, swapped components, a one-pass formula that cancels, a
dropped frame axis) must each fail one of them.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import scene_stats


def _exact(values):
    xs = [Fraction(float(v)) for v in np.asarray(values, dtype=np.float64).ravel()]
    n = len(xs)
    mean = sum(xs) / n
    var = sum((x - mean) ** 2 for x in xs) / n
    return mean, var


def pin_exact_rational(S):
    rng = np.random.default_rng(11)
    mv = rng.uniform(-20, 20, (3, 2, 5, 7)).astype(np.float32)
    got = S.motion_stats(mv)
    for n in range(3):
        for comp in range(2):
            mean, var = _exact(mv[n, comp])
            assert abs(got[n, 2 * comp] - float(mean)) <= 1e-15 * max(1.0, abs(float(mean)))
            assert abs(got[n, 2 * comp + 1] - float(var)) <= 1e-14 * float(var)


def pin_closed_forms(S):
    h, w = 6, 11
    const = np.full((1, 2, h, w), 3.25, dtype=np.float32)
    got = S.motion_stats(const)
    assert got[0, 0] == 3.25 and got[0, 2] == 3.25
    assert got[0, 1] == 0.0 and got[0, 3] == 0.0
    # ramp u = x: every row is 0..W-1, population variance (W^2 - 1) / 12;
    # v = 2y: variance 4 (H^2 - 1) / 12
    ys, xs = np.mgrid[0:h, 0:w]
    ramp = np.stack([xs, 2 * ys]).astype(np.float32)[None]
    got = S.motion_stats(ramp)
    assert got[0, 0] == (w - 1) / 2 and got[0, 2] == (h - 1)
    assert abs(got[0, 1] - (w * w - 1) / 12) <= 1e-13
    assert abs(got[0, 3] - 4 * (h * h - 1) / 12) <= 1e-13
    # two values a, b in equal numbers: variance ((a - b) / 2)^2
    two = np.zeros((1, 2, 4, 4), dtype=np.float32)
    two[0, 0, :2] = -1.5
    two[0, 0, 2:] = 4.5
    got = S.motion_stats(two)
    assert got[0, 0] == 1.5 and got[0, 1] == 9.0


def pin_invariances(S):
    rng = np.random.default_rng(12)
    base = rng.normal(0.0, 2.0, (2, 2, 16, 24))
    ref = S.motion_stats(base.astype(np.float32))
    # shifting by a large offset keeps the variance (a one-pass E[x^2] - E[x]^2
    # loses it to cancellation); values stay exact in float32 by construction
    q = np.round(base * 64) / 64
    shifted = S.motion_stats((q + 4096.0).astype(np.float32))
    plain = S.motion_stats(q.astype(np.float32))
    assert np.allclose(shifted[:, [1, 3]], plain[:, [1, 3]], rtol=1e-12, atol=0)
    assert np.allclose(shifted[:, [0, 2]], plain[:, [0, 2]] + 4096.0, rtol=1e-15, atol=1e-9)
    # scaling by 4 (exact in float32) multiplies the variance by 16
    scaled = S.motion_stats((base.astype(np.float32) * 4).astype(np.float32))
    assert np.allclose(scaled[:, [1, 3]], ref[:, [1, 3]] * 16, rtol=1e-13, atol=0)
    # permuting pixels changes nothing
    perm = base.reshape(2, 2, -1)[:, :, rng.permutation(16 * 24)].reshape(base.shape)
    assert np.allclose(S.motion_stats(perm.astype(np.float32)), ref, rtol=1e-13, atol=1e-15)
    # components and frames are independent
    assert np.allclose(S.motion_stats(base[:, ::-1].astype(np.float32))[:, [2, 3, 0, 1]], ref,
                       rtol=0, atol=0)
    assert np.allclose(S.motion_stats(base[::-1].astype(np.float32))[::-1], ref, rtol=0, atol=0)


def pin_library(S):
    rng = np.random.default_rng(13)
    mv = rng.uniform(-8, 8, (2, 2, 33, 17)).astype(np.float32)
    got = S.motion_stats(mv)
    flat = mv.astype(np.float64).reshape(2, 2, -1)
    assert np.allclose(got[:, [0, 2]], flat.mean(axis=2), rtol=1e-13, atol=1e-15)
    assert np.allclose(got[:, [1, 3]], flat.var(axis=2), rtol=1e-12, atol=0)


def pin_nonfinite(S):
    mv = np.zeros((1, 2, 3, 3), dtype=np.float32)
    mv[0, 0, 1, 1] = np.nan
    mv[0, 1, 2, 2] = np.inf
    got = S.motion_stats(mv)
    assert np.isnan(got[0, 0]) and np.isnan(got[0, 1])
    assert np.isinf(got[0, 2]) and not np.isfinite(got[0, 3])


ALL = [pin_exact_rational, pin_closed_forms, pin_invariances, pin_library, pin_nonfinite]


@pytest.mark.parametrize("pin", ALL, ids=[p.__name__ for p in ALL])
def test_pin(pin):
    pin(scene_stats)


def test_resolution_and_invalid_fraction():
    assert scene_stats.resolution(1080, 1920) == 2073600
    frac = scene_stats.invalid_fraction(np.array([[0, 518400]], dtype=np.uint32), 1080, 1920)
    assert frac.tolist() == [[0.0, 0.25]]


class _Mutant:
    def __init__(self, mean_var):
        self._mean_var = mean_var

    def motion_stats(self, mv):
        a = np.asarray(mv)
        if a.ndim == 3:
            a = a[None]
        out = np.empty((a.shape[0], 4))
        for n in range(a.shape[0]):
            out[n, 0], out[n, 1] = self._mean_var(a[n, 0])
            out[n, 2], out[n, 3] = self._mean_var(a[n, 1])
        return out


def _sample_var(x):
    x = np.asarray(x, dtype=np.float64).ravel()
    return x.mean(), x.var(ddof=1)


def _one_pass_f32(x):
    x = np.asarray(x, dtype=np.float32).ravel()
    m = np.float32(x.sum(dtype=np.float32) / np.float32(x.size))
    return float(m), float(np.float32((x * x).sum(dtype=np.float32) / np.float32(x.size)) - m * m)


def _no_square(x):
    x = np.asarray(x, dtype=np.float64).ravel()
    return x.mean(), np.abs(x - x.mean()).mean()


class _Swapped(_Mutant):
    def motion_stats(self, mv):
        return super().motion_stats(np.asarray(mv)[:, ::-1] if np.asarray(mv).ndim == 4
                                    else np.asarray(mv)[::-1])


class _FirstFrameOnly(_Mutant):
    def motion_stats(self, mv):
        out = super().motion_stats(mv)
        out[:] = out[0]
        return out


MUTANTS = {
    "sample_variance": _Mutant(_sample_var),
    "one_pass_float32": _Mutant(_one_pass_f32),
    "mean_abs_deviation": _Mutant(_no_square),
    "swapped_components": _Swapped(scene_stats._mean_var),
    "first_frame_only": _FirstFrameOnly(scene_stats._mean_var),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    mutant = MUTANTS[name]
    caught = False
    for pin in ALL:
        try:
            pin(mutant)
        except AssertionError:
            caught = True
            break
    assert caught, f"mutant {name} passes every pin"
