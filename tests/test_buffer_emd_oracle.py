"""Pins of the EMD oracle of the state features EMD_{W_N}, EMD_{W_P} (CPU only).

Checked against facts fixed outside the oracle: the Earth Mover's Distance
by its definition (the minimum-cost transport between the two histograms,
solved as a linear programme with scipy), the library's one-dimensional
Wasserstein distance, closed forms (a shifted spike, nested uniform
histograms), bin edges worked by hand, symmetry, the triangle inequality and
invariance under permuting pixels. Planted mistakes (the bin rounded instead
of floored, no clamping, a squared ground distance, no normalisation by the
mass, cumulative sums taken over one histogram twice) must each fail one.
"""


import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.stats import wasserstein_distance

from oracle import buffer_emd


def _transport_lp(ha, hb, width):
    """The EMD by its definition: minimum total cost of moving unit mass from
    distribution ha to hb with cost |i - j| * width per unit (dense LP)."""
    a = np.asarray(ha, np.float64) / np.sum(ha)
    b = np.asarray(hb, np.float64) / np.sum(hb)
    m = len(a)
    cost = np.array([[abs(i - j) * width for j in range(m)] for i in range(m)]).ravel()
    a_eq, b_eq = [], []
    for i in range(m):  # row sums: mass leaving bin i
        row = np.zeros((m, m)); row[i, :] = 1; a_eq.append(row.ravel()); b_eq.append(a[i])
    for j in range(m):  # column sums: mass arriving in bin j
        col = np.zeros((m, m)); col[:, j] = 1; a_eq.append(col.ravel()); b_eq.append(b[j])
    res = linprog(cost, A_eq=np.array(a_eq), b_eq=np.array(b_eq), bounds=(0, None),
                  method="highs")
    assert res.success
    return res.fun


def pin_definition_by_transport(E):
    rng = np.random.default_rng(31)
    for m in (2, 5, 8):
        for _ in range(6):
            ha = rng.integers(0, 7, m)
            hb = rng.integers(0, 7, m)
            ha[0] += 1
            # equal mass: adjust the larger side's last bins
            d = int(ha.sum() - hb.sum())
            hb[-1] += max(d, 0)
            ha[-1] += max(-d, 0)
            width = 0.125 * (1 + int(rng.integers(0, 4)))
            got = E.emd_from_histograms(ha, hb, width)
            ref = _transport_lp(ha, hb, width)
            assert abs(got - ref) <= 1e-9, (ha, hb, got, ref)


def pin_library_wasserstein(E):
    rng = np.random.default_rng(32)
    lo, hi, bins = -1.0, 1.0, 32
    centers = lo + (np.arange(bins) + 0.5) * (hi - lo) / bins
    for _ in range(5):
        a = np.clip(rng.normal(0.1, 0.3, (40, 50)), -1, 0.999)
        b = np.clip(rng.normal(-0.2, 0.4, (40, 50)), -1, 0.999)
        ha = E.histogram(a, lo, hi, bins)
        hb = E.histogram(b, lo, hi, bins)
        ref = wasserstein_distance(centers, centers, ha, hb)
        assert abs(E.channel_emd(a, b, lo, hi, bins) - ref) <= 1e-12
        # the histograms themselves agree with numpy's on interior values
        ref_h, _ = np.histogram(a, bins=bins, range=(lo, hi))
        assert np.array_equal(ha, ref_h)


def pin_closed_forms(E):
    lo, hi, bins = 0.0, 4.0, 64
    width = (hi - lo) / bins
    centers = lo + (np.arange(bins) + 0.5) * width
    # a spike moved by k bins costs k bin widths
    for i, k in ((3, 5), (10, 0), (60, -17)):
        a = np.full((9, 11), centers[i])
        b = np.full((9, 11), centers[i + k])
        assert abs(E.channel_emd(a, b, lo, hi, bins) - abs(k) * width) <= 1e-15
    # uniform over bins [0, m) against uniform over [j, j + m): j widths
    for m, j in ((4, 3), (16, 20), (1, 63)):
        a = np.repeat(centers[:m], 12)
        b = np.repeat(centers[j:j + m], 12)
        assert abs(E.channel_emd(a, b, lo, hi, bins) - j * width) <= 1e-13
    # uniform over [0, m) against uniform over [0, 2m): m/2 widths
    for m in (2, 8, 32):
        a = np.repeat(centers[:m], 2 * 6)
        b = np.repeat(centers[:2 * m], 6)
        assert abs(E.channel_emd(a, b, lo, hi, bins) - m / 2 * width) <= 1e-13


def pin_bin_edges(E):
    lo, hi, bins = -1.0, 1.0, 8  # width 1/4, exact in binary
    vals = np.array([-1.0, -0.75, -0.5000001, 0.0, 0.2499999, 0.25, 0.999, 1.0, 7.0, -3.0,
                     np.inf, -np.inf, np.nan, -1.0000001])
    exp = np.array([0, 1, 1, 4, 4, 5, 7, 7, 7, 0, 7, 0, 0, 0])
    assert np.array_equal(E.bin_index(vals, lo, hi, bins), exp)
    # float16 / bfloat16 buffers are binned by their stored values
    h = np.array([0.25, -0.75], np.float16)
    assert np.array_equal(E.bin_index(h, lo, hi, bins), [5, 1])


def pin_metric_properties(E):
    rng = np.random.default_rng(33)
    lo, hi, bins = -2.0, 2.0, 40
    x, y, z = (rng.normal(m, 0.5, (20, 30)) for m in (-0.5, 0.0, 0.7))
    dxy = E.channel_emd(x, y, lo, hi, bins)
    assert dxy == E.channel_emd(y, x, lo, hi, bins)
    assert E.channel_emd(x, x, lo, hi, bins) == 0.0
    assert dxy <= E.channel_emd(x, z, lo, hi, bins) + E.channel_emd(z, y, lo, hi, bins) + 1e-15
    perm = rng.permutation(x.size)
    assert E.channel_emd(x.ravel()[perm].reshape(x.shape), y, lo, hi, bins) == dxy
    # a frame against itself is 0 in every channel; the batch form equals the planes
    buf = rng.normal(0, 0.4, (2, 3, 12, 14))
    assert (E.buffer_emd(buf, buf, lo, hi, bins) == 0).all()
    other = rng.normal(0.2, 0.4, (2, 3, 12, 14))
    got = E.buffer_emd(buf, other, lo, hi, bins)
    for i in range(2):
        for ch in range(3):
            assert got[i, ch] == E.channel_emd(buf[i, ch], other[i, ch], lo, hi, bins)


ALL = [pin_definition_by_transport, pin_library_wasserstein, pin_closed_forms, pin_bin_edges,
       pin_metric_properties]


@pytest.mark.parametrize("pin", ALL, ids=[p.__name__ for p in ALL])
def test_pin(pin):
    pin(buffer_emd)


class _Mutant:
    def __init__(self, **over):
        self.over = over

    def __getattr__(self, name):
        return self.over.get(name, getattr(buffer_emd, name))


def _bin_round(values, lo, hi, bins):
    v = np.asarray(values).astype(np.float64)
    t = np.round((v - lo) * (bins / (hi - lo)))
    t = np.fmin(np.fmax(np.nan_to_num(t, nan=0.0), 0.0), bins - 1)
    return t.astype(np.int64)


def _bin_no_clamp(values, lo, hi, bins):
    v = np.asarray(values).astype(np.float64)
    with np.errstate(invalid="ignore", over="ignore"):
        t = np.floor((v - lo) * (bins / (hi - lo)))
    ok = (t >= 0) & (t < bins)
    return t[ok].astype(np.int64)  # values outside the range are dropped


def _emd_squared(ha, hb, width):
    s = (np.cumsum(ha) - np.cumsum(hb)).astype(np.float64)
    return float((s * s).sum() / np.sum(ha) * width)


def _emd_unnormalised(ha, hb, width):
    return float(np.abs(np.cumsum(ha) - np.cumsum(hb)).sum() * width)


def _emd_one_sided(ha, hb, width):
    return float(np.abs(np.cumsum(ha) - hb).sum() / np.sum(ha) * width)


def _mut(**kw):
    m = _Mutant(**kw)
    # the wrappers must route through the patched steps
    def histogram(values, lo, hi, bins):
        idx = m.bin_index(np.ravel(values), lo, hi, bins)
        return np.bincount(idx, minlength=bins).astype(np.int64)
    def channel_emd(a, b, lo, hi, bins):
        width = (hi - lo) / bins
        return m.emd_from_histograms(histogram(a, lo, hi, bins), histogram(b, lo, hi, bins), width)
    def buffer_emd_(cur, prev, lo, hi, bins):
        cur, prev = np.asarray(cur), np.asarray(prev)
        return np.array([[channel_emd(cur[i, c], prev[i, c], lo, hi, bins)
                          for c in range(cur.shape[1])] for i in range(cur.shape[0])])
    m.over.update(histogram=histogram, channel_emd=channel_emd, buffer_emd=buffer_emd_)
    return m


MUTANTS = {
    "bin_rounded": _mut(bin_index=_bin_round),
    "no_clamp": _mut(bin_index=_bin_no_clamp),
    "squared_ground_distance": _mut(emd_from_histograms=_emd_squared),
    "not_normalised": _mut(emd_from_histograms=_emd_unnormalised),
    "one_sided_cumsum": _mut(emd_from_histograms=_emd_one_sided),
}


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


def test_unmutated_routes_pass():
    for pin in ALL:
        pin(_mut())
