"""A frame of 4 GiB on the GPU (16384 x 16384 RGBA float32), against the oracle.

Below 4 GiB per frame the forward's all-phase gathers and the adjoint's
uniform motion-gradient gathers address the whole frame with 32-bit offsets;
at 4 GiB and above both fall back to per-plane addressing. This case checks
that fallback, with rigid motion (uniform segments), a block moving
differently (segment edges) and the frame borders, on sampled pixels: the
forward values, mask and counts, the motion gradient, and the image gradient;
then the training pair (recording forward, adjoint from the records) on the
same buffers against those results. About 21 GiB of device memory and 30 GiB
of host memory.
"""

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from oracle import warp_oracle
from gpu_util import announce, need_gpu, to_host

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-5   # as in the general adjoint tests
FWD_TOL = 1e-5    # as in the general forward tests


def test_frame_of_4gib():
    dev = need_gpu()
    c, h, w = 4, 16384, 16384  # C*H*W*4 bytes = 2^32: beyond 32-bit frame offsets
    phase = 0.75
    gen = torch.Generator(device=dev).manual_seed(2307)
    announce("4 GiB frame: inputs")
    src = torch.rand((1, c, h, w), device=dev, generator=gen)
    mv = torch.empty((1, 2, h, w), device=dev)
    mv[:, 0], mv[:, 1] = 1.3, -0.7
    mv[:, 0, 5000:5600, 7000:8000], mv[:, 1, 5000:5600, 7000:8000] = -6.2, 3.4
    g = torch.randn((1, 1, c, h, w), device=dev, generator=gen)
    announce("4 GiB frame: forward")
    out, mask, cnt = exw.warp(src, mv, (phase,), return_mask=True, return_count=True)
    announce("4 GiB frame: backward")
    gs, gm = exw.warp_backward(src, mv, (phase,), g)
    torch.cuda.synchronize()
    assert int(cnt[0, 0]) == int((mask[0, 0] == 0).sum())

    rng = np.random.default_rng(7)
    ys = np.concatenate([rng.integers(0, h, 120), rng.integers(4990, 5610, 40), [0, h - 1, 0, h - 1, 1]])
    xs = np.concatenate([rng.integers(0, w, 120), rng.integers(6990, 8010, 40), [0, 0, w - 1, w - 1, w - 2]])
    yd, xd = torch.from_numpy(ys).to(dev), torch.from_numpy(xs).to(dev)
    got = to_host(out[0, 0][:, yd, xd])
    got_mask = mask[0, 0][yd, xd].cpu().numpy()
    got_gm = to_host(gm[0][:, yd, xd])
    got_gs = to_host(gs[0][:, yd[:60], xd[:60]])
    cnt_plain = cnt.clone()

    # the training pair on the same buffers: the forward records the footprint
    # (one-pixel paths only at this size), the adjoint takes it from there
    announce("4 GiB frame: recording forward and recorded adjoint")
    ws = torch.empty(exw.exw_warp_backward_workspace_bytes(torch.float32, 1, c, h, w),
                     dtype=torch.uint8, device=dev)
    exw.exw_warp_forward_batched_record(src, mv, (phase,), out, ws, mask, cnt)
    exw.exw_warp_backward_batched_recorded(src, mv, (phase,), g, gs, gm, ws)
    torch.cuda.synchronize()
    assert torch.equal(cnt, cnt_plain)
    assert np.array_equal(to_host(out[0, 0][:, yd, xd]), got)
    assert np.array_equal(mask[0, 0][yd, xd].cpu().numpy(), got_mask)
    assert np.array_equal(to_host(gm[0][:, yd, xd]), got_gm)
    rec_gs = to_host(gs[0][:, yd[:60], xd[:60]])
    assert float((np.abs(rec_gs - got_gs) / np.maximum(1.0, np.abs(got_gs))).max()) <= GRAD_TOL
    del ws

    src_h = src[0].cpu().numpy()
    mv_h = mv[0].cpu().numpy()
    g_h = g[0].cpu().numpy()
    del out, mask, gs, gm, src, mv, g
    torch.cuda.empty_cache()

    ref, valid = warp_oracle.forward_at(src_h, mv_h, phase, ys, xs)
    assert np.array_equal(got_mask.astype(bool), valid)
    assert float(np.abs(got - ref).max()) <= FWD_TOL
    ref_gm = warp_oracle.grad_mv_at(src_h, mv_h, [phase], g_h, ys, xs)
    err = np.abs(got_gm - ref_gm) / np.maximum(1.0, np.abs(ref_gm))
    assert float(err.max()) <= GRAD_TOL, float(err.max())
    ref_gs = warp_oracle.grad_src_at(mv_h, [phase], g_h, ys[:60], xs[:60], radius=7)
    err = np.abs(got_gs - ref_gs) / np.maximum(1.0, np.abs(ref_gs))
    assert float(err.max()) <= GRAD_TOL, float(err.max())
