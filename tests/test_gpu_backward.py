"""Adjoint (backward) kernels on the GPU, through the C-ABI: against the float64
oracle, the adjoint identity, finite differences and autograd."""

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from oracle import warp_oracle
from synth import make_config
from gpu_util import announce, half_ulp, need_gpu, stored, to_dev, to_host

pytestmark = pytest.mark.gpu

SMALL = {1: dict(), 2: dict(n=2, h=75, w=131), 3: dict(n=1, h=90, w=200),
         4: dict(n=2, h=70, w=97), 5: dict(n=1, h=61, w=107)}

# Gradients are sums of up to 4*K*C float32 products of O(1) terms; 1e-5
# relative to max(1, |value|) leaves a wide margin over float32 rounding.
GRAD_TOL = 1e-5


# Half an ulp, relative, of each storage type: rounding the forward output and
# the image gradient into it moves each side of the adjoint identity by at
# most this much times the sum of the absolute terms.
REL_ROUND = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def assert_adjoint(wx, y, x, wty, dtype):
    """<W x, y> = <x, W^T y>: for float32 storage to 1e-4 relative; for
    f16/bf16 within the rounding bound of the two stored results."""
    lhs = float((wx.double() * y.double()).sum())
    rhs = float((x.double() * wty.double()).sum())
    if dtype == "f32":
        assert abs(lhs - rhs) <= 1e-4 * max(1.0, abs(lhs)), (lhs, rhs)
        return
    scale = float((wx.double().abs() * y.double().abs()).sum()
                  + (x.double().abs() * wty.double().abs()).sum())
    assert abs(lhs - rhs) <= 2 * REL_ROUND[dtype] * scale + 1e-6 * scale, (lhs, rhs, scale)


def grads_gpu(src, mv, phases, g, dtype, dev):
    s = to_dev(src, dtype, dev)
    gd = to_dev(g, dtype, dev)
    m = torch.from_numpy(np.ascontiguousarray(mv)).to(dev)
    gs, gm = exw.warp_backward(s, m, phases, gd)
    torch.cuda.synchronize()
    return to_host(gs), to_host(gm)


def check_grad(got, ref, what):
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert float(err.max()) <= GRAD_TOL, f"{what}: rel err {float(err.max())}"


@pytest.mark.parametrize("index", sorted(SMALL))
def test_backward_matches_oracle(index):
    dev = need_gpu()
    d = make_config(index, **SMALL[index])
    phases = list(d["phases"]) if index != 1 else [0.25, 0.5, 0.75, 1.0]
    n, c, h, w = d["src"].shape
    g = np.random.default_rng(index).standard_normal((n, len(phases), c, h, w)).astype(np.float32)
    for dtype in d["spec"].storage:
        announce("backward", index, dtype, d["src"].shape, phases)
        src_q = stored(d["src"], dtype)
        g_q = stored(g, dtype)
        ref_gs, ref_gm = warp_oracle.backward(src_q, d["mv"], phases, g_q)
        gs, gm = grads_gpu(d["src"], d["mv"], phases, g, dtype, dev)
        check_grad(gm, ref_gm, f"grad_mv config {index} {dtype}")
        if dtype == "f32":
            check_grad(gs, ref_gs, f"grad_src config {index}")
        else:
            bound = half_ulp(ref_gs, dtype) + GRAD_TOL * np.maximum(1.0, np.abs(ref_gs))
            assert (np.abs(gs - ref_gs) <= bound).all(), f"grad_src config {index} {dtype}"


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_adjoint_identity(dtype):
    """<W x, y> = <x, W^T y> with the GPU's own forward and backward."""
    dev = need_gpu()
    d = make_config(2, n=2, h=130, w=257)
    rng = np.random.default_rng(10)
    x = rng.random(d["src"].shape, dtype=np.float32)
    phases = list(d["phases"])
    n, c, h, w = x.shape
    y = rng.standard_normal((n, len(phases), c, h, w)).astype(np.float32)
    announce("adjoint", dtype)
    xd, yd = to_dev(x, dtype, dev), to_dev(y, dtype, dev)
    m = torch.from_numpy(d["mv"]).to(dev)
    wx = exw.warp(xd, m, phases)
    wty, _ = exw.warp_backward(xd, m, phases, yd, need_mv=False)
    assert_adjoint(wx, yd, xd, wty, dtype)


def test_finite_differences_on_crops():
    """Config-4 style: 8 crops of 64x64 px, L = sum((warp(I, mv) - tgt)^2) with
    tgt = warp(I, mv + delta). Within a bilinear cell L is quadratic in one
    pixel's motion and in the image, so central differences of the GPU forward
    are exact up to float32 rounding; pixels near a cell edge or the frame
    bound are excluded."""
    dev = need_gpu()
    d = make_config(4, n=8, h=64, w=64)
    src, mv, delta = d["src"], d["mv"], d["delta"]
    phases = [1.0]
    sd = to_dev(src, "f32", dev)
    md = torch.from_numpy(mv).to(dev)
    announce("finite differences")
    tgt = exw.warp(sd, torch.from_numpy(mv + delta).to(dev), phases)
    out = exw.warp(sd, md, phases)
    g = 2.0 * (out - tgt)
    gs, gm = exw.warp_backward(sd, md, phases, g.contiguous())
    # against the oracle's analytic gradients
    ref_gs, ref_gm = warp_oracle.backward(src, mv, phases, to_host(g))
    check_grad(to_host(gs), ref_gs, "grad_src")
    check_grad(to_host(gm), ref_gm, "grad_mv")
    # motion: per-pixel central differences (each output pixel sees only its own motion)
    hstep = 1e-2
    for comp in (0, 1):
        plus, minus = mv.copy(), mv.copy()
        plus[:, comp] += hstep
        minus[:, comp] -= hstep
        step = plus[:, comp].astype(np.float64) - minus[:, comp].astype(np.float64)
        lp = ((exw.warp(sd, torch.from_numpy(plus).to(dev), phases) - tgt) ** 2).sum(dim=(1, 2))
        lm = ((exw.warp(sd, torch.from_numpy(minus).to(dev), phases) - tgt) ** 2).sum(dim=(1, 2))
        fd = (to_host(lp) - to_host(lm)) / step
        ys, xs = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
        coord = (xs if comp == 0 else ys)[None] - mv[:, comp].astype(np.float64)
        frac = coord - np.floor(coord)
        keep = (frac > 2 * hstep) & (frac < 1 - 2 * hstep)
        keep &= (coord > 1) & (coord < 62)
        other = (ys if comp == 0 else xs)[None] - mv[:, 1 - comp].astype(np.float64)
        keep &= (other >= 0) & (other <= 63)
        assert keep.sum() > 0.5 * keep.size
        ref = to_host(gm)[:, comp]
        err = np.abs(fd - ref)[keep] / np.maximum(np.abs(ref[keep]), 1e-1)
        assert float(np.quantile(err, 0.999)) <= 1e-2 and float(err.max()) <= 5e-2
    # image: directional difference
    dirn = torch.randn_like(sd)
    lp = ((exw.warp(sd + 0.5 * dirn, md, phases) - tgt) ** 2).double().sum()
    lm = ((exw.warp(sd - 0.5 * dirn, md, phases) - tgt) ** 2).double().sum()
    lin = float((gs.double() * dirn.double()).sum())
    assert abs(float(lp - lm) - lin) <= 1e-3 * max(1.0, abs(lin))


def test_autograd_function():
    dev = need_gpu()
    d = make_config(5, n=1, h=40, w=70)
    phases = [1.0]
    for dtype in ("f32", "bf16"):
        announce("autograd", dtype)
        src = to_dev(d["src"], dtype, dev).requires_grad_(True)
        mv = torch.from_numpy(d["mv"]).to(dev).requires_grad_(True)
        out = exw.warp_differentiable(src, mv, phases)
        w8 = torch.linspace(-1, 1, out.numel(), device=dev).reshape(out.shape).to(out.dtype)
        (out.float() * w8.float()).sum().backward()
        gs, gm = exw.warp_backward(src.detach(), mv.detach(), phases, w8)
        assert torch.equal(src.grad, gs) or torch.allclose(src.grad.float(), gs.float(),
                                                            rtol=1e-2, atol=1e-2)
        assert torch.allclose(mv.grad, gm, rtol=1e-4, atol=1e-4)
    # only the motion, or only the image
    src = to_dev(d["src"], "f32", dev)
    mv = torch.from_numpy(d["mv"]).to(dev).requires_grad_(True)
    exw.warp_differentiable(src, mv, phases).sum().backward()
    assert mv.grad is not None and src.grad is None


def test_backward_specials_and_single_frame():
    dev = need_gpu()
    rng = np.random.default_rng(11)
    h, w = 9, 75
    src = rng.random((1, 3, h, w), dtype=np.float32)
    mv = rng.uniform(-3, 3, (1, 2, h, w)).astype(np.float32)
    mv[0, 0, 0, :10] = np.nan
    mv[0, 1, 1, :10] = np.inf
    mv[0, 0, 2, :10] = 1e30
    g = rng.standard_normal((1, 2, 3, h, w)).astype(np.float32)
    phases = [0.5, 1.0]
    announce("backward specials")
    gs, gm = grads_gpu(src, mv, phases, g, "f32", dev)
    ref_gs, ref_gm = warp_oracle.backward(src, mv, phases, g)
    assert np.isfinite(gs).all() and np.isfinite(gm).all()
    check_grad(gs, ref_gs, "grad_src specials")
    check_grad(gm, ref_gm, "grad_mv specials")
    # single-frame entry point
    sd = to_dev(src[0], "f16", dev)
    md = torch.from_numpy(mv[0]).to(dev)
    gd = to_dev(g[0, 1], "f16", dev)
    gsrc = torch.empty_like(sd)
    gmv = torch.empty((2, h, w), device=dev)
    ws = torch.empty(exw.exw_warp_backward_workspace_bytes(torch.float16, 1, 3, h, w),
                     dtype=torch.uint8, device=dev)
    exw.exw_warp_backward(sd, md, 1.0, gd, gsrc, gmv, ws)
    ref_s, ref_m = exw.warp_backward(sd[None], md[None], [1.0], gd[None, None])
    torch.cuda.synchronize()
    assert torch.allclose(gsrc.float(), ref_s[0].float(), atol=2e-3, rtol=2e-3)
    assert torch.allclose(gmv, ref_m[0], atol=1e-5, rtol=1e-5)


@pytest.mark.parametrize("index,dtype", [(2, "f32"), (5, "bf16")])
def test_full_size_backward_sampled(index, dtype):
    """Full-size batches in the benchmark's launch configuration: sampled motion
    and image gradients against the oracle, and the adjoint identity."""
    dev = need_gpu()
    d = make_config(index)
    src, mv, phases = d["src"], d["mv"], list(d["phases"])
    n, c, h, w = src.shape
    k = len(phases)
    announce("full backward", index, dtype)
    sd = to_dev(src, dtype, dev)
    md = torch.from_numpy(mv).to(dev)
    gen = torch.Generator(device=dev).manual_seed(index)
    gd = torch.randn((n, k, c, h, w), device=dev, generator=gen).to(sd.dtype)
    gs, gm = exw.warp_backward(sd, md, phases, gd)
    wx = exw.warp(sd, md, phases)
    assert_adjoint(wx, gd, sd, gs, dtype)
    rng = np.random.default_rng(index)
    radius = int(np.ceil(np.nanmax(np.abs(mv)) * max(phases))) + 1
    for i in (0, n - 1):
        ys = np.concatenate([rng.integers(0, h, 150), [0, h - 1, 0, h - 1]])
        xs = np.concatenate([rng.integers(0, w, 150), [0, 0, w - 1, w - 1]])
        src_q = stored(src[i], dtype)
        g_q = to_host(gd[i])
        ref_m = warp_oracle.grad_mv_at(src_q, mv[i], phases, g_q, ys, xs)
        got_m = to_host(gm[i][:, torch.from_numpy(ys).to(dev), torch.from_numpy(xs).to(dev)])
        check_grad(got_m, ref_m, f"full grad_mv frame {i}")
        ref_s = warp_oracle.grad_src_at(mv[i], phases, g_q, ys[:60], xs[:60], radius)
        got_s = to_host(gs[i][:, torch.from_numpy(ys[:60]).to(dev),
                              torch.from_numpy(xs[:60]).to(dev)])
        if dtype == "f32":
            check_grad(got_s, ref_s, f"full grad_src frame {i}")
        else:
            bound = half_ulp(ref_s, dtype) + GRAD_TOL * np.maximum(1.0, np.abs(ref_s))
            assert (np.abs(got_s - ref_s) <= bound).all()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_far_motion_fallback(dtype):
    """Motion reaching further than the tile gather covers (> 128 px) goes
    through the atomic fallback; mixed with near motion in the same frame."""
    dev = need_gpu()
    rng = np.random.default_rng(20)
    n, c, h, w = 2, 4, 150, 400
    src = rng.random((n, c, h, w), dtype=np.float32)
    mv = rng.uniform(-3, 3, (n, 2, h, w)).astype(np.float32)
    mv[0, 0, 40:60, 100:300] = rng.uniform(-250, 250, (20, 200)).astype(np.float32)
    mv[0, 1, 70:75, :] = 140.5
    phases = [0.25, 0.5, 1.0]
    g = rng.standard_normal((n, 3, c, h, w)).astype(np.float32)
    announce("far motion", dtype)
    gs, gm = grads_gpu(src, mv, phases, g, dtype, dev)
    ref_gs, ref_gm = warp_oracle.backward(stored(src, dtype), mv, phases, stored(g, dtype))
    check_grad(gm, ref_gm, f"grad_mv far {dtype}")
    if dtype == "f32":
        check_grad(gs, ref_gs, "grad_src far")
    else:
        bound = half_ulp(ref_gs, dtype) + GRAD_TOL * np.maximum(1.0, np.abs(ref_gs))
        assert (np.abs(gs - ref_gs) <= bound).all()


def test_backward_shapes_channels_and_partial_requests():
    dev = need_gpu()
    rng = np.random.default_rng(21)
    for (n, c, h, w, k) in [(1, 1, 1, 1, 1), (2, 2, 7, 1, 3), (3, 5, 5, 65, 4),
                            (1, 12, 9, 130, 1), (1, 64, 3, 5, 1), (2, 3, 67, 257, 2),
                            (1, 4, 1, 300, 3)]:
        src = rng.random((n, c, h, w), dtype=np.float32)
        mv = rng.uniform(-3, 3, (n, 2, h, w)).astype(np.float32)
        phases = [0.25, 0.5, 0.75, 1.0][:k]
        g = rng.standard_normal((n, k, c, h, w)).astype(np.float32)
        for dtype in ("f32", "f16", "bf16"):
            announce("backward shapes", n, c, h, w, k, dtype)
            ref_gs, ref_gm = warp_oracle.backward(stored(src, dtype), mv, phases, stored(g, dtype))
            gs, gm = grads_gpu(src, mv, phases, g, dtype, dev)
            check_grad(gm, ref_gm, f"grad_mv {(n, c, h, w, k)} {dtype}")
            if dtype == "f32":
                check_grad(gs, ref_gs, f"grad_src {(n, c, h, w, k)}")
            else:
                bound = half_ulp(ref_gs, dtype) + GRAD_TOL * np.maximum(1.0, np.abs(ref_gs))
                assert (np.abs(gs - ref_gs) <= bound).all(), (n, c, h, w, k)
            # one gradient at a time
            sd, gd = to_dev(src, dtype, dev), to_dev(g, dtype, dev)
            md = torch.from_numpy(mv).to(dev)
            only_s, none_m = exw.warp_backward(sd, md, phases, gd, need_mv=False)
            none_s, only_m = exw.warp_backward(sd, md, phases, gd, need_src=False)
            assert none_m is None and none_s is None
            check_grad(to_host(only_m), ref_gm, "motion only")
            if dtype == "f32":
                check_grad(to_host(only_s), ref_gs, "image only")
