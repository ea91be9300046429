"""Pins of the decision-path and chained-warp oracle (CPU only).

The decision tree must reproduce Table V exactly (``tests/golden/
table5_scenarios.json``, typed from the paper): every scenario reached by
exactly one combination of decisions, with its frames and its frame-rate
upsampling. Chained warps are pinned to exact integer shifts (three quarter
steps of a 4-px motion are three 1-px shifts with zero fill), to the identity
under zero motion, and to constant images staying constant where every
step was valid. Planted mistakes must fail a pin.
"""

import itertools
import json
import os

import numpy as np
import pytest

from oracle import decision_paths as D

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "table5_scenarios.json")


def all_decisions():
    for d1, d_last in itertools.product((D.WARP, D.EXTRAPOLATE), repeat=2):
        if d1 == D.WARP:
            for d2 in (D.WARP, D.EXTRAPOLATE):
                yield d1, d2, d_last
        else:
            yield d1, None, d_last


def pin_table_v(P):
    table = {s["name"]: s for s in json.load(open(GOLDEN))["scenarios"]}
    seen = {}
    for dec in all_decisions():
        p = P.plan(*dec)
        name = p["scenario"]
        assert name not in seen, f"{name} reached twice: {seen.get(name)} and {dec}"
        seen[name] = dec
        row = table[name]
        for k in ("P1", "P2", "P3"):
            assert list(p[k]) == row[k], (name, k, p[k], row[k])
        assert p["new_frames"] + 1 == row["upsampling"], (name, p["new_frames"])
        # each decision picks its frame: warping at a node shows a warped frame there
        d1, d2, d_last = dec
        assert (d1 == D.WARP) == (p["P1"][0] == "warp"), (name, dec)
        if d2 is not None:
            assert (d2 == D.WARP) == (p["P2"][0] == "warp"), (name, dec)
        assert (d_last == D.WARP) == (p["P3"][0] == "warp"), (name, dec)
    assert sorted(seen) == sorted(table), seen


def _shift(img, a, b):
    out = np.zeros_like(img)
    h, w = img.shape[-2:]
    ys, xs = np.mgrid[0:h, 0:w]
    ok = (ys - b >= 0) & (ys - b < h) & (xs - a >= 0) & (xs - a < w)
    out[..., ok] = img[..., (ys - b)[ok], (xs - a)[ok]]
    return out, ok


def pin_chain_integer_steps(P):
    rng = np.random.default_rng(31)
    src = rng.random((2, 3, 9, 12))
    mv = np.zeros((2, 2, 9, 12), dtype=np.float32)
    mv[:, 0] = 4.0   # 1 px right per quarter step
    mv[:, 1] = -8.0  # 2 px up per quarter step
    out, mask, cnt = P.chained_warp(src, mv, 0.25, 3)
    for i in range(3):
        ref, ok = _shift(src, i + 1, -2 * (i + 1))
        assert np.array_equal(out[i], ref), i
        # a step's mask is that step's own out-of-frame test: one shift of (1, -2)
        _, ok1 = _shift(src, 1, -2)
        assert np.array_equal(mask[i].astype(bool), np.broadcast_to(ok1, mask[i].shape)), i
        assert (cnt[i] == (~ok1).sum()).all()


def pin_chain_identity_and_constant(P):
    rng = np.random.default_rng(32)
    src = rng.random((1, 2, 8, 10))
    out, mask, cnt = P.chained_warp(src, np.zeros((1, 2, 8, 10), np.float32), 0.25, 3)
    assert all(np.array_equal(out[i], src) for i in range(3)) and mask.all()
    const = np.full((1, 1, 16, 16), 0.625)
    mv = rng.uniform(-3, 3, (1, 2, 16, 16)).astype(np.float32)
    out, mask, _ = P.chained_warp(const, mv, 0.25, 3)
    # where every step so far was valid and sampled only valid pixels the value stays
    assert np.allclose(out[0][mask[0].astype(bool)[:, None].repeat(1, 1)], 0.625, atol=1e-15)


def pin_policy(P):
    calm = (0.0, 0.0, 0.0, 0.0)
    assert P.threshold_policy(calm, [0, 0, 0], 1.0, 0.01) == (D.WARP, D.WARP, D.WARP)
    wild = (0.0, 50.0, 0.0, 50.0)
    assert P.threshold_policy(wild, [0, 0, 0], 1.0, 0.01) == (D.EXTRAPOLATE, None, D.EXTRAPOLATE)
    # holes growing with the phase: warp first, then extrapolate
    assert P.threshold_policy(calm, [0.001, 0.005, 0.02], 1.0, 0.01) == (D.WARP, D.WARP, D.EXTRAPOLATE)
    for stats in (calm, wild):
        for inv in ([0, 0, 0], [0.5, 0.5, 0.5]):
            d1, d2, d3 = P.threshold_policy(stats, inv, 1.0, 0.01)
            P.plan(d1, d2, d3)  # always a valid path


ALL = [pin_table_v, pin_chain_integer_steps, pin_chain_identity_and_constant, pin_policy]


@pytest.mark.parametrize("pin", ALL, ids=[p.__name__ for p in ALL])
def test_pin(pin):
    pin(D)


class _Mutant:
    def __init__(self, **over):
        self.over = over

    def __getattr__(self, name):
        return self.over.get(name, getattr(D, name))


def _plan_swapped_last(d1, d2, d_last):
    return D.plan(d1, d2, 1 - d_last if d1 == D.WARP else d_last)


def _plan_p3_from_f(d1, d2, d_last):
    p = dict(D.plan(d1, d2, d_last))
    if p["P3"][0] == "extrapolate":
        p["P3"] = ("extrapolate", "F")
    return p


def _chain_direct(src, mv, phase, steps, store=None):
    # the direct warp at phase i/4 instead of the chain
    from oracle import warp_oracle
    outs, masks, counts = [], [], []
    for i in range(steps):
        o, m, c = warp_oracle.forward(src, mv, [phase * (i + 1)])
        outs.append(o[:, 0]), masks.append(m[:, 0]), counts.append(c[:, 0])
    return np.stack(outs), np.stack(masks), np.stack(counts)


MUTANTS = {
    "swapped_last_decision": _Mutant(plan=_plan_swapped_last),
    "p3_extrapolated_from_rendered": _Mutant(plan=_plan_p3_from_f),
    "direct_instead_of_chained": _Mutant(chained_warp=_chain_direct),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    caught = False
    for pin in ALL:
        try:
            pin(MUTANTS[name])
        except AssertionError:
            caught = True
            break
    assert caught, f"mutant {name} passes every pin"
