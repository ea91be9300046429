"""N_D (dynamic objects: connected components of the marked stencil pixels)
on the GPU, through the C-ABI, against the oracle. Counts are integers, so
they must be equal.

The cases stress the two passes: random masks near the percolation density
(components that cross many 32 x 32 tiles and their borders in every
direction), checkerboards (every diagonal contact matters under
8-connectivity, none under 4), long diagonals and a spiral crossing tile
borders many times, frames smaller than a tile and ragged edges, and the
synthetic scenes' stencils at full size."""

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from oracle import dynamic_objects
from synth import make_config
from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


def gpu_count(st: np.ndarray, conn: int, dev) -> np.ndarray:
    t = torch.from_numpy(np.ascontiguousarray(st, dtype=np.uint8)).to(dev)
    out = exw.dynamic_objects(t, conn)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.int64)


def check(st, what, dev):
    for conn in (4, 8):
        got = gpu_count(st, conn, dev)
        ref = dynamic_objects.dynamic_objects(st, conn)
        assert np.array_equal(got, ref), (what, conn, got, ref)


@pytest.mark.parametrize("density", [0.2, 0.45, 0.55, 0.6, 0.75])
def test_random_masks(density):
    dev = need_gpu()
    rng = np.random.default_rng(int(density * 100))
    st = (rng.random((3, 157, 211)) < density).astype(np.uint8) * rng.integers(1, 256, (3, 157, 211)).astype(np.uint8)
    announce("dynamic objects random", density)
    check(st, f"density {density}", dev)


def test_structured_masks():
    dev = need_gpu()
    cases = []
    h, w = 130, 200
    cb = ((np.arange(h)[:, None] + np.arange(w)[None, :]) % 2 == 0).astype(np.uint8)
    cases.append(("checkerboard", cb))
    diag = np.zeros((h, w), np.uint8)
    for i in range(h):
        diag[i, (i * 3) % w] = 1          # steep diagonal: apart under 4, joined pairs under 8
        diag[i, min(i, w - 1)] = 1        # a 45-degree line through many tiles
    cases.append(("diagonals", diag))
    sp = np.zeros((h, w), np.uint8)       # a one-pixel spiral
    y0, y1, x0, x1 = 0, h - 1, 0, w - 1
    while y0 <= y1 and x0 <= x1:
        sp[y0, x0:x1 + 1] = 1
        sp[y0:y1 + 1, x1] = 1
        if y1 - y0 >= 2:
            sp[y1, x0 + 2:x1 + 1] = 1
        if x1 - x0 >= 2:
            sp[y0 + 2:y1 + 1, x0] = 1
        y0, y1, x0, x1 = y0 + 2, y1 - 2, x0 + 2, x1 - 2
        if y0 <= y1 and x0 <= x1:
            sp[y0, x0 - 2:x0] = 0
    cases.append(("spiral", sp))
    grid = np.zeros((h, w), np.uint8)     # lines exactly on the tile borders
    grid[31::32, :] = 1
    grid[:, 31::32] = 1
    grid[32::32, 32::32] = 0
    cases.append(("tile borders", grid))
    stripes = np.zeros((h, w), np.uint8)
    stripes[:, ::2] = 1
    cases.append(("stripes", stripes))
    for name, m in cases:
        announce("dynamic objects", name)
        check(m[None], name, dev)


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 1, 40), (2, 40, 1), (1, 31, 33), (1, 32, 32),
                                   (3, 33, 65), (1, 5, 1000), (1, 1000, 5)])
def test_shapes_and_edges(shape):
    dev = need_gpu()
    rng = np.random.default_rng(shape[1] * 7 + shape[2])
    st = (rng.random(shape) < 0.55).astype(np.uint8)
    announce("dynamic objects shape", shape)
    check(st, f"shape {shape}", dev)
    for fill in (0, 1):
        check(np.full(shape, fill, np.uint8), f"constant {fill} {shape}", dev)


def test_empty_frames_and_repeated_calls():
    dev = need_gpu()
    t = torch.zeros((3, 0, 17), dtype=torch.uint8, device=dev)
    count = torch.full((3,), 7, dtype=torch.int32, device=dev)
    exw.exw_dynamic_objects(t, count, None, 8)
    torch.cuda.synchronize()
    assert count.cpu().tolist() == [0, 0, 0]
    # the same workspace twice, the second time on a smaller batch
    rng = np.random.default_rng(3)
    big = (rng.random((4, 90, 120)) < 0.5).astype(np.uint8)
    small = big[:2, :50, :70].copy()
    ws = torch.empty(exw.exw_dynamic_objects_workspace_bytes(4, 90, 120), dtype=torch.uint8,
                     device=dev)
    for st in (big, small):
        s = torch.from_numpy(st).to(dev)
        c = torch.empty((st.shape[0],), dtype=torch.int32, device=dev)
        exw.exw_dynamic_objects(s, c, ws, 8)
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy(), dynamic_objects.dynamic_objects(st, 8))


@pytest.mark.parametrize("index", [2, 5])
def test_synthetic_stencils_full_size(index):
    dev = need_gpu()
    d = make_config(index)
    st = d["stencil"]
    announce("dynamic objects full size", index, st.shape)
    check(st, f"workload {index}", dev)
    assert (dynamic_objects.dynamic_objects(st) >= 1).all()


def test_frame_at_the_size_limit():
    """H * W = 2^30 (32768 x 32768, the C ABI's limit): a grid of 48 x 48
    squares 16 pixels apart has one object per square in either
    connectivity, (32768 / 64)^2 = 262144 (closed form; the 1 GiB stencil
    is built on the GPU)."""
    dev = need_gpu()
    side = 1 << 15
    announce("dynamic objects at the size limit", side, side)
    r = (torch.arange(side, device=dev) % 64) < 48
    st = (r[:, None] & r[None, :]).to(torch.uint8)[None]
    del r
    for conn in (4, 8):
        got = exw.dynamic_objects(st, conn)
        torch.cuda.synchronize()
        assert got.cpu().tolist() == [(side // 64) ** 2], (conn, got)
    del st
    torch.cuda.empty_cache()
