"""Pins of the N_D oracle (number of dynamic objects: connected components of
the marked stencil pixels), CPU only.

Checked against facts fixed outside the oracle: a breadth-first flood fill
written out here on small random frames, closed forms (empty and full
frames, separated rectangles, corner contact, checkerboards, stripes,
diagonals, a ring), invariance under transposes and flips, and the count's
behaviour under the two connectivities. Planted mistakes (4 for 8
connectivity, marked means > 1, counting pixels, counting the background's
components, a frame that wraps around) must each fail one.
"""

from collections import deque

import numpy as np
import pytest

from oracle import dynamic_objects


def flood_fill_count(stencil, connectivity=8):
    """Components by their definition: start a new one at each marked pixel
    not yet reached and walk its neighbours breadth first."""
    mask = np.asarray(stencil) != 0
    h, w = mask.shape
    steps = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    if connectivity == 8:
        steps += [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    seen = np.zeros_like(mask)
    count = 0
    for y in range(h):
        for x in range(w):
            if not mask[y, x] or seen[y, x]:
                continue
            count += 1
            seen[y, x] = True
            todo = deque([(y, x)])
            while todo:
                cy, cx = todo.popleft()
                for dy, dx in steps:
                    ny, nx = cy + dy, cx + dx
                    if 0 <= ny < h and 0 <= nx < w and mask[ny, nx] and not seen[ny, nx]:
                        seen[ny, nx] = True
                        todo.append((ny, nx))
    return count


def pin_flood_fill(D):
    rng = np.random.default_rng(51)
    for _ in range(60):
        h, w = (int(v) for v in rng.integers(1, 14, 2))
        p = float(rng.uniform(0.1, 0.9))
        st = (rng.random((h, w)) < p).astype(np.uint8) * rng.integers(1, 256, (h, w)).astype(np.uint8)
        for conn in (4, 8):
            assert D.frame_objects(st, conn) == flood_fill_count(st, conn), (h, w, p, conn)


def pin_closed_forms(D):
    for conn in (4, 8):
        assert D.frame_objects(np.zeros((7, 9), np.uint8), conn) == 0
        assert D.frame_objects(np.ones((7, 9), np.uint8), conn) == 1
        # k rectangles with a gap of one pixel between them
        st = np.zeros((20, 60), np.uint8)
        for i in range(5):
            st[3:15, 12 * i:12 * i + 11] = 1
        assert D.frame_objects(st, conn) == 5
        # vertical stripes on every other column: one object each
        st = np.zeros((9, 14), np.uint8)
        st[:, ::2] = 1
        assert D.frame_objects(st, conn) == 7
        # a ring: one object; its hole is background
        st = np.ones((11, 11), np.uint8)
        st[3:8, 3:8] = 0
        assert D.frame_objects(st, conn) == 1
    # two squares touching at a corner: one object under 8, two under 4
    st = np.zeros((10, 10), np.uint8)
    st[1:4, 1:4] = 1
    st[4:7, 4:7] = 1
    assert D.frame_objects(st, 8) == 1 and D.frame_objects(st, 4) == 2
    # checkerboard: every marked cell alone under 4, all joined under 8
    for h, w in ((2, 2), (5, 8), (9, 9)):
        cb = ((np.arange(h)[:, None] + np.arange(w)[None, :]) % 2 == 0).astype(np.uint8)
        assert D.frame_objects(cb, 4) == int(cb.sum())
        assert D.frame_objects(cb, 8) == 1
    # a diagonal line of n pixels
    st = np.eye(12, dtype=np.uint8)
    assert D.frame_objects(st, 4) == 12 and D.frame_objects(st, 8) == 1
    # marked pixels at opposite edges stay apart (no wrap-around)
    st = np.zeros((6, 8), np.uint8)
    st[:, 0] = 1
    st[:, 7] = 1
    assert D.frame_objects(st, 8) == 2


def pin_invariants_and_batch(D):
    rng = np.random.default_rng(52)
    st = (rng.random((4, 23, 31)) < 0.45).astype(np.uint8) * 3
    n4 = D.dynamic_objects(st, 4)
    n8 = D.dynamic_objects(st, 8)
    assert n4.dtype == np.int64 and n4.shape == (4,)
    assert (n8 <= n4).all()
    for i in range(4):
        for conn, ref in ((4, n4[i]), (8, n8[i])):
            f = st[i]
            assert D.frame_objects(f.T, conn) == ref
            assert D.frame_objects(f[::-1], conn) == ref
            assert D.frame_objects(f[:, ::-1], conn) == ref
    # any non-zero value marks a pixel
    vals = st * rng.integers(1, 86, st.shape).astype(np.uint8)
    assert np.array_equal(D.dynamic_objects(vals, 8), n8)


ALL = [pin_flood_fill, pin_closed_forms, pin_invariants_and_batch]


@pytest.mark.parametrize("pin", ALL, ids=[p.__name__ for p in ALL])
def test_pin(pin):
    pin(dynamic_objects)


class _Mutant:
    def __init__(self, frame_objects):
        self.frame_objects = frame_objects

    def dynamic_objects(self, stencil, connectivity=8):
        return np.array([self.frame_objects(f, connectivity) for f in np.asarray(stencil)],
                        dtype=np.int64)


def _always_four(st, conn=8):
    return dynamic_objects.frame_objects(st, 4)


def _marked_above_one(st, conn=8):
    return dynamic_objects.frame_objects((np.asarray(st) > 1).astype(np.uint8), conn)


def _pixels(st, conn=8):
    return int((np.asarray(st) != 0).sum())


def _background(st, conn=8):
    return dynamic_objects.frame_objects((np.asarray(st) == 0).astype(np.uint8), conn)


def _wrapping(st, conn=8):
    st = np.asarray(st)
    tiled = np.tile(st != 0, (3, 3)).astype(np.uint8)  # the frame on a torus, seen 3 x 3 times
    h, w = st.shape
    from scipy import ndimage
    lab, _ = ndimage.label(tiled, structure=dynamic_objects.structure(conn))
    centre = lab[h:2 * h, w:2 * w]
    return int(len(np.unique(centre[centre > 0])))


MUTANTS = {"four_for_eight": _always_four, "marked_above_one": _marked_above_one,
           "counts_pixels": _pixels, "counts_background": _background,
           "wraps_around": _wrapping}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    m = _Mutant(MUTANTS[name])
    caught = False
    for pin in ALL:
        try:
            pin(m)
        except AssertionError:
            caught = True
            break
    assert caught, f"mutant {name} passes every pin"


def test_synthetic_stencil_marks_the_rectangles():
    from synth import make_config
    d = make_config(2, n=2, h=90, w=160)
    st = d["stencil"]
    assert st.shape == (2, 90, 160) and st.dtype == np.uint8
    assert set(np.unique(st)) <= {0, 1}
    # moving rectangles cover part of the frame, and carry their own motion
    assert 0 < st.mean() < 1
    pan = np.asarray(d["info"]["pan"], np.float32)
    bg = st[0] == 0
    assert np.allclose(d["mv"][0, 0][bg], pan[0]) and np.allclose(d["mv"][0, 1][bg], pan[1])
    n = dynamic_objects.dynamic_objects(st)
    assert (n >= 1).all() and (n <= d["info"]["n_rects"]).all()
