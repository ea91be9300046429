"""Pins of the frame-quality oracle, PSNR and SSIM (CPU only).

Checked against facts fixed outside the oracle: the closed form of PSNR for a
constant error, SSIM's closed form for constant frames and its value 1 for
identical frames, symmetry, the Gaussian window's own properties, and brute
force (explicit loops over positions and window taps with the window computed
independently) on small frames. Planted mistakes (the 8-bit peak on unit-range
frames, a box window, zero padding instead of valid positions, swapped
constants, a missing covariance term) must each fail one of them.
"""

import math

import numpy as np
import pytest

from oracle import quality


def _brute_ssim_map(x, y, peak=1.0):
    r = [i - 5 for i in range(11)]
    wts = [[math.exp(-(a * a + b * b) / (2 * 1.5 * 1.5)) for b in r] for a in r]
    tot = math.fsum(v for row in wts for v in row)
    c1, c2 = (0.01 * peak) ** 2, (0.03 * peak) ** 2
    h, w = x.shape
    out = np.empty((h - 10, w - 10))
    for i in range(h - 10):
        for j in range(w - 10):
            sx = sy = sxx = syy = sxy = 0.0
            for a in range(11):
                for b in range(11):
                    g = wts[a][b] / tot
                    p, q = float(x[i + a, j + b]), float(y[i + a, j + b])
                    sx += g * p
                    sy += g * q
                    sxx += g * p * p
                    syy += g * q * q
                    sxy += g * p * q
            vx, vy, cxy = sxx - sx * sx, syy - sy * sy, sxy - sx * sy
            out[i, j] = ((2 * sx * sy + c1) * (2 * cxy + c2)) / ((sx * sx + sy * sy + c1) * (vx + vy + c2))
    return out


def pin_psnr_closed_form(Q):
    rng = np.random.default_rng(21)
    a = rng.random((3, 20, 30))
    for c in (0.5, 0.1, 1e-3):
        got = Q.psnr(a, a + c)
        assert abs(got - (-20 * math.log10(c))) <= 1e-9, (c, got)
    assert Q.psnr(a, a) == math.inf
    # the peak enters squared: 8-bit-scaled frames with peak 255 give the same PSNR
    b = a + rng.normal(0, 0.05, a.shape)
    assert abs(Q.psnr(a * 255, b * 255, peak=255.0) - Q.psnr(a, b)) <= 1e-9
    # a known MSE: error +-0.1 on alternate pixels -> MSE 0.01 -> 20 dB
    e = np.where(np.indices(a.shape).sum(axis=0) % 2 == 0, 0.1, -0.1)
    assert abs(Q.psnr(a, a + e) - 20.0) <= 1e-9


def pin_ssim_identity_and_constants(Q):
    rng = np.random.default_rng(22)
    x = rng.random((2, 24, 31))
    assert Q.ssim(x, x) == 1.0
    for a, b in ((0.2, 0.7), (0.5, 0.5), (0.0, 1.0)):
        c1 = (0.01) ** 2
        expect = (2 * a * b + c1) / (a * a + b * b + c1)
        got = Q.ssim(np.full((1, 16, 20), a), np.full((1, 16, 20), b))
        assert abs(got - expect) <= 1e-12, (a, b, got, expect)


def pin_ssim_symmetry_and_window(Q):
    rng = np.random.default_rng(23)
    x, y = rng.random((1, 30, 25)), rng.random((1, 30, 25))
    assert abs(Q.ssim(x, y) - Q.ssim(y, x)) <= 1e-14
    g = Q.gaussian_window()
    assert g.shape == (11, 11) and abs(g.sum() - 1.0) <= 1e-15
    assert np.allclose(g, g.T, rtol=0, atol=0) and np.allclose(g, g[::-1, ::-1], rtol=0, atol=0)
    one = np.exp(-((np.arange(11) - 5.0) ** 2) / (2 * 1.5 ** 2))
    assert np.allclose(g, np.outer(one, one) / one.sum() ** 2, rtol=1e-14, atol=0)
    assert g.argmax() == 60  # centre tap


def pin_ssim_brute_force(Q):
    rng = np.random.default_rng(24)
    x = rng.random((15, 17))
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    ref = _brute_ssim_map(x, y)
    got = Q.ssim_map(x, y)
    assert got.shape == ref.shape == (5, 7)
    assert np.allclose(got, ref, rtol=0, atol=1e-12), float(np.abs(got - ref).max())
    assert abs(Q.ssim(x[None], y[None]) - ref.mean()) <= 1e-12


def pin_ssim_checkerboard_closed_form(Q):
    """A 1-px checkerboard chi against a negatively correlated copy.

    x = a + dx * chi and y = p - dy * chi. Under the separable window the
    weighted mean of chi at a position is m = e^2 + o^2 or 2 e o (by the
    parity of the position), where e and o are the sums of the normalised
    1-D Gaussian taps at even and at odd offsets; chi^2 = chi gives its
    weighted variance m (1 - m). Hence mu_x = a + dx m, mu_y = p - dy m,
    sigma_x^2 = dx^2 m (1 - m), sigma_y^2 = dy^2 m (1 - m) and the covariance
    -dx dy m (1 - m), which is negative: this pins the structure term's sign
    and its factor 2, which SSIM(x, x) = 1 and symmetry cannot."""
    one = [math.exp(-((k - 5) ** 2) / (2 * 1.5 ** 2)) for k in range(11)]
    tot = math.fsum(one)
    e = math.fsum(one[k] for k in range(0, 11, 2)) / tot
    o = math.fsum(one[k] for k in range(1, 11, 2)) / tot
    h, w = 17, 22
    chi = (np.indices((h, w)).sum(axis=0) % 2).astype(np.float64)
    for a, dx, p, dy, peak in ((0.0, 1.0, 1.0, 1.0, 1.0), (0.2, 0.5, 0.9, 0.3, 1.0),
                               (0.1, 0.05, 0.6, 0.4, 1.0), (30.0, 180.0, 250.0, 200.0, 255.0)):
        x = a + dx * chi
        y = p - dy * chi
        expect = np.empty((h - 10, w - 10))
        for i in range(h - 10):
            for j in range(w - 10):
                # chi = 1 where the offset parity differs from the corner's
                m = 2 * e * o if (i + j) % 2 == 0 else e * e + o * o
                mx, my = a + dx * m, p - dy * m
                vx, vy = dx * dx * m * (1 - m), dy * dy * m * (1 - m)
                cxy = -dx * dy * m * (1 - m)
                c1, c2 = (0.01 * peak) ** 2, (0.03 * peak) ** 2
                expect[i, j] = ((2 * mx * my + c1) * (2 * cxy + c2)) / (
                    (mx * mx + my * my + c1) * (vx + vy + c2))
        got = Q.ssim_map(x, y, peak)
        assert np.abs(got - expect).max() <= 1e-10, (a, dx, p, dy, float(np.abs(got - expect).max()))
        assert abs(Q.ssim(x[None], y[None], peak) - expect.mean()) <= 1e-10
        assert expect.max() < 0.5  # far from 1: the structure term is active


ALL = [pin_psnr_closed_form, pin_ssim_identity_and_constants, pin_ssim_symmetry_and_window,
       pin_ssim_brute_force, pin_ssim_checkerboard_closed_form]


@pytest.mark.parametrize("pin", ALL, ids=[p.__name__ for p in ALL])
def test_pin(pin):
    pin(quality)


def test_frame_quality_batches_and_rejects_small_frames():
    rng = np.random.default_rng(25)
    a = rng.random((2, 3, 1, 12, 13))
    b = np.clip(a + 0.05, 0, 1)
    q = quality.frame_quality(a, b)
    assert q.shape == (2, 3, 3)
    for i in range(2):
        for j in range(3):
            assert q[i, j, 0] == quality.mse(a[i, j], b[i, j])
            assert q[i, j, 2] == quality.ssim(a[i, j], b[i, j])
    with pytest.raises(ValueError):
        quality.ssim(np.zeros((1, 10, 40)), np.zeros((1, 10, 40)))


class _Mutant:
    """The oracle with one step replaced."""

    def __init__(self, **over):
        self.over = over

    def __getattr__(self, name):
        return self.over.get(name, getattr(quality, name))


def _psnr_255(a, b, peak=1.0):
    m = quality.mse(a, b)
    return math.inf if m == 0 else 10 * math.log10(255.0 ** 2 / m)


def _ssim_map_with(window=None, pad=False, k1=0.01, k2=0.03, cov=True, cov_sign=1.0,
                   cov_factor=2.0):
    from scipy.signal import fftconvolve

    def f(x, y, peak=1.0):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        g = quality.gaussian_window() if window is None else window

        def ws(img):
            return fftconvolve(img, g[::-1, ::-1], mode="same" if pad else "valid")
        c1, c2 = (k1 * peak) ** 2, (k2 * peak) ** 2
        mx, my = ws(x), ws(y)
        sxx, syy = ws(x * x) - mx * mx, ws(y * y) - my * my
        sxy = cov_sign * (ws(x * y) - mx * my) if cov else np.zeros_like(mx)
        return (((2 * mx * my + c1) * (cov_factor * sxy + c2))
                / ((mx * mx + my * my + c1) * (sxx + syy + c2)))
    return f


def _ssim_from(map_fn):
    def f(a, b, peak=1.0):
        a, b = np.asarray(a), np.asarray(b)
        if a.ndim == 2:
            a, b = a[None], b[None]
        return float(np.mean([map_fn(a[c], b[c], peak).mean() for c in range(a.shape[0])]))
    return f


def _mutant_ssim(**kw):
    m = _ssim_map_with(**kw)
    return _Mutant(ssim_map=m, ssim=_ssim_from(m))


MUTANTS = {
    "peak_255_on_unit_frames": _Mutant(psnr=_psnr_255),
    "box_window": _mutant_ssim(window=np.full((11, 11), 1 / 121)),
    "zero_padding": _mutant_ssim(pad=True),
    "swapped_constants": _mutant_ssim(k1=0.03, k2=0.01),
    "no_covariance": _mutant_ssim(cov=False),
    "covariance_sign": _mutant_ssim(cov_sign=-1.0),
    "covariance_without_factor_2": _mutant_ssim(cov_factor=1.0),
}


def test_checkerboard_pin_alone_catches_the_covariance_mutants():
    """The closed form with negative covariance is what pins the structure term:
    it rejects a flipped sign and a dropped factor 2 on its own."""
    for name in ("covariance_sign", "covariance_without_factor_2", "no_covariance"):
        with pytest.raises(AssertionError):
            pin_ssim_checkerboard_closed_form(MUTANTS[name])


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    caught = False
    for pin in ALL:
        try:
            pin(MUTANTS[name])
        except (AssertionError, ValueError):
            caught = True
            break
    assert caught, f"mutant {name} passes every pin"
