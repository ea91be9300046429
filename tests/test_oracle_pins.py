"""The float64 oracles (NumPy and C) against their pins; CPU only."""

import numpy as np
import pytest

from oracle import ref_c, warp_oracle
from synth import make_config

import oracle_pins


class _COracle:
    exact = False
    forward = staticmethod(ref_c.forward)
    backward = staticmethod(ref_c.backward)


class _COracleExact:
    exact = True

    @staticmethod
    def forward(src, mv, phases):
        return ref_c.forward(src, mv, phases, exact=True)

    @staticmethod
    def backward(src, mv, phases, grad_out):
        return ref_c.backward(src, mv, phases, grad_out, exact=True)


class _NumpyExact:
    exact = True

    @staticmethod
    def forward(src, mv, phases):
        return warp_oracle.forward(src, mv, phases, exact=True)

    @staticmethod
    def backward(src, mv, phases, grad_out):
        return warp_oracle.backward(src, mv, phases, grad_out, exact=True)


# The float32-rounded displacement (the default) and the exact one.
ORACLES = {"numpy": warp_oracle, "c": _COracle, "numpy_exact": _NumpyExact,
           "c_exact": _COracleExact}


@pytest.mark.parametrize("impl", sorted(ORACLES))
@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin, impl):
    pin(ORACLES[impl])


# Reduced sizes of the five workloads: several tiles and ragged edges, seconds on a CPU.
SMALL = {1: dict(), 2: dict(n=2, h=75, w=131), 3: dict(n=2, h=90, w=160),
         4: dict(n=2, h=70, w=97), 5: dict(n=1, h=60, w=107)}


@pytest.mark.parametrize("exact", [False, True], ids=["rounded", "exact"])
@pytest.mark.parametrize("index", sorted(SMALL))
def test_numpy_and_c_oracles_agree(index, exact):
    d = make_config(index, **SMALL[index])
    phases = d["phases"]
    o1, m1, c1 = warp_oracle.forward(d["src"], d["mv"], phases, exact=exact)
    o2, m2, c2 = ref_c.forward(d["src"], d["mv"], phases, exact=exact)
    assert np.abs(o1 - o2).max() <= 1e-12
    assert np.array_equal(m1, m2) and np.array_equal(c1, c2)
    g = np.random.default_rng(index).standard_normal(o1.shape)
    a1, b1 = warp_oracle.backward(d["src"], d["mv"], phases, g, exact=exact)
    a2, b2 = ref_c.backward(d["src"], d["mv"], phases, g, exact=exact)
    assert np.abs(a1 - a2).max() <= 1e-12
    assert np.abs(b1 - b2).max() <= 1e-12


def test_modes_differ_only_where_the_rounding_of_three_quarters_moves_d():
    """The two displacement modes agree exactly at phases 1/4, 1/2 and 1 (the
    product is exact there); at 3/4 they differ by no more than the rounding
    of d (half a float32 ulp) times the image's largest gradient, and masks
    differ only where an integer bound lies within that half ulp."""
    d = make_config(2, n=1, h=80, w=120)
    src, mv = d["src"], d["mv"]
    for s in (0.25, 0.5, 1.0):
        a = ref_c.forward(src, mv, [s], exact=True)
        b = ref_c.forward(src, mv, [s], exact=False)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    a, ma, _ = ref_c.forward(src, mv, [0.75], exact=True)
    b, mb, _ = ref_c.forward(src, mv, [0.75], exact=False)
    d32 = np.float32(0.75) * mv.astype(np.float64)
    half_ulp = np.abs(np.spacing(d32.astype(np.float32))).astype(np.float64) / 2
    # the largest difference between neighbouring pixels bounds the slope
    slope = max(np.abs(np.diff(src, axis=-1)).max(), np.abs(np.diff(src, axis=-2)).max())
    both = (ma == 1) & (mb == 1)
    assert np.abs(a - b)[:, :, :, both[0, 0]].max() <= 2 * slope * half_ulp.max() + 1e-15
    diff = ma != mb
    if diff.any():
        ys, xs = np.nonzero(diff[0, 0])
        frac_x = np.abs(d32[0, 0, ys, xs] - np.round(d32[0, 0, ys, xs]))
        frac_y = np.abs(d32[0, 1, ys, xs] - np.round(d32[0, 1, ys, xs]))
        assert (np.minimum(frac_x, frac_y) <= half_ulp[0].max()).all()


def test_pointwise_forms_match_full_frames():
    """The sampled evaluators used at full size agree with the full-frame oracle."""
    d = make_config(2, n=1, h=64, w=96)
    src, mv, phases = d["src"], d["mv"], d["phases"]
    out, mask, _ = warp_oracle.forward(src, mv, phases)
    g = np.random.default_rng(0).standard_normal(out.shape)
    gs, gm = warp_oracle.backward(src, mv, phases, g)
    rng = np.random.default_rng(1)
    ys = rng.integers(0, 64, 40)
    xs = rng.integers(0, 96, 40)
    for k, s in enumerate(phases):
        v, ok = warp_oracle.forward_at(src[0], mv[0], s, ys, xs)
        assert np.array_equal(v, out[0, k][:, ys, xs])
        assert np.array_equal(ok, mask[0, k][ys, xs].astype(bool))
    gmv = warp_oracle.grad_mv_at(src[0], mv[0], phases, g[0], ys, xs)
    assert np.abs(gmv - gm[0][:, ys, xs]).max() <= 1e-12
    radius = int(np.ceil(np.abs(mv).max() * max(phases))) + 1
    gsrc = warp_oracle.grad_src_at(mv[0], phases, g[0], ys, xs, radius)
    assert np.abs(gsrc - gs[0][:, ys, xs]).max() <= 1e-12
