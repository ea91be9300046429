"""The float64 oracles (NumPy and C) against their pins; CPU only."""

import numpy as np
import pytest

from oracle import ref_c, warp_oracle
from synth import make_config

import oracle_pins


class _COracle:
    forward = staticmethod(ref_c.forward)
    backward = staticmethod(ref_c.backward)


ORACLES = {"numpy": warp_oracle, "c": _COracle}


@pytest.mark.parametrize("impl", sorted(ORACLES))
@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin, impl):
    pin(ORACLES[impl])


# Reduced sizes of the five workloads: several tiles and ragged edges, seconds on a CPU.
SMALL = {1: dict(), 2: dict(n=2, h=75, w=131), 3: dict(n=2, h=90, w=160),
         4: dict(n=2, h=70, w=97), 5: dict(n=1, h=60, w=107)}


@pytest.mark.parametrize("index", sorted(SMALL))
def test_numpy_and_c_oracles_agree(index):
    d = make_config(index, **SMALL[index])
    phases = d["phases"]
    o1, m1, c1 = warp_oracle.forward(d["src"], d["mv"], phases)
    o2, m2, c2 = ref_c.forward(d["src"], d["mv"], phases)
    assert np.abs(o1 - o2).max() <= 1e-12
    assert np.array_equal(m1, m2) and np.array_equal(c1, c2)
    g = np.random.default_rng(index).standard_normal(o1.shape)
    a1, b1 = warp_oracle.backward(d["src"], d["mv"], phases, g)
    a2, b2 = ref_c.backward(d["src"], d["mv"], phases, g)
    assert np.abs(a1 - a2).max() <= 1e-12
    assert np.abs(b1 - b2).max() <= 1e-12


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
