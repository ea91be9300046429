"""Rigid-motion cases of the warp on the GPU, against the float64 oracle.

Under a constant motion field every 64-pixel row segment away from the frame
borders is valid in all its lanes with one integer tap offset per phase, so
the kernels take their uniform-segment paths: shared gathers in the forward,
scalar tap offsets and boxes in the footprint pass, the pattern scatter
without per-lane tests and the coalesced motion-gradient gathers in the
adjoint. The cases cover phases that share their offsets and phases that do
not, both signs, integer displacements (zero fractions), offsets past the
128-pixel replay limit, partial last segments, one, three and four phases,
and all storage types. The tolerances are those of the general tests.
"""

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from oracle import warp_oracle
from gpu_util import announce, assert_close_kernel, half_ulp, need_gpu, stored, to_dev, to_host

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-5  # as in the general adjoint tests

# (pan_x, pan_y, phases): ceil(s * pan) is the same for all phases in the
# first two cases and differs between phases in the others.
PANS = [
    (0.6, -0.8, (0.25, 0.5, 0.75)),
    (-0.45, 0.3, (0.25, 0.5, 0.75)),
    (2.5, -3.0, (0.25, 0.5, 0.75)),
    (-7.3, 5.2, (0.25, 0.5, 0.75)),
    (2.0, -4.0, (0.25, 0.5, 0.75, 1.0)),   # integer displacements at every phase
    (40.0, -9.5, (1.0,)),                  # one phase, long reach
    (150.0, 2.0, (1.0,)),                  # beyond the replay limit: far segments
]


def pan_field(n, h, w, px, py, rect=None):
    mv = np.empty((n, 2, h, w), np.float32)
    mv[:, 0], mv[:, 1] = px, py
    if rect is not None:  # a block moving differently: segments crossing its edges are not uniform
        y0, y1, x0, x1, rx, ry = rect
        mv[:, 0, y0:y1, x0:x1], mv[:, 1, y0:y1, x0:x1] = rx, ry
    return mv


def check_grad(got, ref, what):
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert float(err.max()) <= GRAD_TOL, f"{what}: rel err {float(err.max())}"


def run_case(src, mv, phases, dtype, dev, label):
    n, c, h, w = src.shape
    g = np.random.default_rng(h * w + c).standard_normal((n, len(phases), c, h, w)).astype(np.float32)
    src_q, g_q = stored(src, dtype), stored(g, dtype)
    s = to_dev(src, dtype, dev)
    m = torch.from_numpy(np.ascontiguousarray(mv)).to(dev)
    announce("uniform segments forward", label, dtype, src.shape, phases)
    out, mask, cnt = exw.warp(s, m, phases, return_mask=True, return_count=True)
    torch.cuda.synchronize()
    ref, ref_mask, ref_cnt = warp_oracle.forward(src_q, mv, list(phases))
    assert np.array_equal(mask.cpu().numpy(), ref_mask), label
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), ref_cnt), label
    assert_close_kernel(to_host(out), ref, dtype, f"forward {label} {dtype}")
    announce("uniform segments backward", label, dtype, src.shape, phases)
    gs, gm = exw.warp_backward(s, m, phases, to_dev(g, dtype, dev))
    torch.cuda.synchronize()
    ref_gs, ref_gm = warp_oracle.backward(src_q, mv, list(phases), g_q)
    check_grad(to_host(gm), ref_gm, f"grad_mv {label} {dtype}")
    if dtype == "f32":
        check_grad(to_host(gs), ref_gs, f"grad_src {label}")
    else:
        bound = half_ulp(ref_gs, dtype) + GRAD_TOL * np.maximum(1.0, np.abs(ref_gs))
        assert (np.abs(to_host(gs) - ref_gs) <= bound).all(), f"grad_src {label} {dtype}"


@pytest.mark.parametrize("pan", PANS, ids=[f"{p[0]}_{p[1]}_k{len(p[2])}" for p in PANS])
def test_pan_fields_f32(pan):
    dev = need_gpu()
    px, py, phases = pan
    # 300 = 4 full segments + 44 columns; 70 rows span several 3-row tiles
    src = np.random.default_rng(7).random((2, 4, 70, 300)).astype(np.float32)
    run_case(src, pan_field(2, 70, 300, px, py), phases, "f32", dev, f"pan {px},{py}")


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("pan", PANS[:4], ids=[f"{p[0]}_{p[1]}" for p in PANS[:4]])
def test_pan_fields_16bit(pan, dtype):
    dev = need_gpu()
    px, py, phases = pan
    src = np.random.default_rng(8).random((1, 4, 45, 260)).astype(np.float32)
    run_case(src, pan_field(1, 45, 260, px, py), phases, dtype, dev, f"pan {px},{py}")


@pytest.mark.parametrize("c", [1, 3, 12])
def test_pan_with_moving_block_other_channel_counts(c):
    # a block with its own motion: uniform segments around it, non-uniform ones on its edges
    dev = need_gpu()
    src = np.random.default_rng(9 + c).random((1, c, 64, 256)).astype(np.float32)
    mv = pan_field(1, 64, 256, 1.7, -0.6, rect=(20, 44, 70, 150, -5.5, 3.25))
    run_case(src, mv, (0.25, 0.5, 0.75) if c <= 4 else (1.0,), "f32", dev, f"block c={c}")


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("c,phases", [(1, (1.0,)), (3, (0.25, 0.5)), (4, (0.25, 0.5, 0.75)),
                                       (4, (0.25, 0.5, 0.75, 1.0)), (12, (0.5, 1.0)),
                                       (12, (1.0,))])
def test_rigid_forward_16bit_channel_counts(c, phases, dtype):
    """16-bit storage under rigid motion for every specialised channel count:
    widths of whole 128-pixel segments (256, 1024) and a ragged tail (600);
    a moving block makes some segments fall back to the one-pixel paths."""
    dev = need_gpu()
    rng = np.random.default_rng(20 + c + len(phases))
    for h, w, px, py, rect in ((9, 256, 1.25, -0.5, None), (13, 600, -2.75, 3.5, None),
                               (10, 1024, 0.3, 0.7, (2, 8, 300, 420, -9.0, 4.5))):
        src = rng.random((2, c, h, w)).astype(np.float32)
        mv = pan_field(2, h, w, px, py, rect)
        announce("rigid 16-bit forward", c, phases, dtype, (h, w))
        s = to_dev(src, dtype, dev)
        m = torch.from_numpy(np.ascontiguousarray(mv)).to(dev)
        out, mask, cnt = exw.warp(s, m, phases, return_mask=True, return_count=True)
        torch.cuda.synchronize()
        ref, ref_mask, ref_cnt = warp_oracle.forward(stored(src, dtype), mv, list(phases))
        assert np.array_equal(mask.cpu().numpy(), ref_mask)
        assert np.array_equal(cnt.cpu().numpy().astype(np.int64), ref_cnt)
        assert_close_kernel(to_host(out), ref, dtype, f"rigid c={c} {dtype} {w}")
