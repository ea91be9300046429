"""Forward warp on the GPU, through the C-ABI, against the float64 oracle."""

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from oracle import warp_oracle
from synth import make_config
from gpu_util import (E2E_TOL, announce, assert_close_kernel, compare_with_exact, need_gpu,
                      rounding_band, stored, to_dev, to_host)

pytestmark = pytest.mark.gpu

# Reduced sizes of the five workloads: several 64x4 tiles and ragged edges.
SMALL = {1: dict(), 2: dict(n=2, h=75, w=131), 3: dict(n=2, h=90, w=200),
         4: dict(n=2, h=70, w=97), 5: dict(n=1, h=61, w=107)}


def run_forward(src, mv, phases, dtype, dev):
    s = to_dev(src, dtype, dev)
    m = torch.from_numpy(mv).to(dev)
    out, mask, cnt = exw.warp(s, m, phases, return_mask=True, return_count=True)
    torch.cuda.synchronize()
    return to_host(out), mask.cpu().numpy(), cnt.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("index", sorted(SMALL))
def test_forward_matches_oracle(index):
    dev = need_gpu()
    d = make_config(index, **SMALL[index])
    phases = list(d["phases"])
    if index == 1:
        phases = [0.25, 0.5, 0.75, 1.0]
    for dtype in d["spec"].storage:
        announce("forward", index, dtype, d["src"].shape, phases)
        src_q = stored(d["src"], dtype)
        ref, ref_mask, ref_cnt = warp_oracle.forward(src_q, d["mv"], phases)
        out, mask, cnt = run_forward(d["src"], d["mv"], phases, dtype, dev)
        assert np.array_equal(mask, ref_mask), f"mask differs in {int((mask != ref_mask).sum())}"
        assert np.array_equal(cnt, ref_cnt)
        assert_close_kernel(out, ref, dtype, f"config {index} {dtype}")
        ex, ex_mask, _ = warp_oracle.forward(src_q, d["mv"], phases, exact=True)
        compare_with_exact(out, mask, ex, ex_mask, d["mv"], phases, dtype,
                           f"config {index} {dtype}")
        # end to end: against the oracle on the float32 original frames
        ref32, _, _ = warp_oracle.forward(d["src"], d["mv"], phases)
        assert np.abs(out - ref32).max() <= E2E_TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_identity_is_bitwise(dtype):
    dev = need_gpu()
    rng = np.random.default_rng(0)
    src = rng.random((2, 3, 37, 70), dtype=np.float32)
    mv = rng.uniform(-9, 9, (2, 2, 37, 70)).astype(np.float32)
    s = to_dev(src, dtype, dev)
    announce("identity", dtype)
    out, mask = exw.warp(s, torch.from_numpy(mv).to(dev), [0.0], return_mask=True)
    assert torch.equal(out[:, 0], s) and bool(mask.all())
    out, mask = exw.warp(s, torch.zeros(2, 2, 37, 70, device=dev), [0.25, 0.5, 0.75, 1.0],
                         return_mask=True)
    for k in range(4):
        assert torch.equal(out[:, k], s)
    assert bool(mask.all())


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_integer_shift_is_bitwise(dtype):
    dev = need_gpu()
    rng = np.random.default_rng(1)
    h, w = 29, 67
    src = rng.random((1, 4, h, w), dtype=np.float32)
    s = to_dev(src, dtype, dev)
    ref_src = torch.from_numpy(src).to(torch.float32)
    for a, b in [(3, -2), (-7, 5), (0, 11), (66, 0)]:
        for phase, scale in [(1.0, 1), (0.25, 4), (0.5, 2), (0.75, 4 / 3)]:
            if phase == 0.75 and (a % 3 or b % 3):
                continue
            mv = np.zeros((1, 2, h, w), np.float32)
            mv[0, 0], mv[0, 1] = a * scale, b * scale
            announce("shift", dtype, a, b, phase)
            out = exw.warp(s, torch.from_numpy(mv).to(dev), [phase])[0, 0].cpu()
            exp = torch.zeros_like(out)
            ys = slice(max(b, 0), h + min(b, 0))
            xs = slice(max(a, 0), w + min(a, 0))
            ys0 = slice(max(-b, 0), h + min(-b, 0))
            xs0 = slice(max(-a, 0), w + min(-a, 0))
            exp[:, ys, xs] = s[0].cpu()[:, ys0, xs0]
            assert torch.equal(out, exp), (a, b, phase)
    del ref_src


def test_constant_and_ramp_closed_forms():
    dev = need_gpu()
    h, w = 50, 131
    ys, xs = np.meshgrid(np.arange(h, dtype=np.float64), np.arange(w, dtype=np.float64),
                         indexing="ij")
    img = np.stack([np.full((h, w), 0.625), 0.00390625 * xs + 0.0078125 * ys + 0.125,
                    (xs * ys) / (h * w)])[None].astype(np.float32)
    mv = np.random.default_rng(2).uniform(-6, 6, (1, 2, h, w)).astype(np.float32)
    for phase in (0.25, 0.5, 0.75, 1.0):
        announce("closed forms", phase)
        out, mask, _ = run_forward(img, mv, [phase], "f32", dev)
        ref, ref_mask, _ = warp_oracle.forward(img, mv, [phase])
        assert np.array_equal(mask, ref_mask)
        ok = mask[0, 0].astype(bool)
        # constant: weights sum to one up to float32 rounding
        assert np.abs(out[0, 0, 0][ok] - 0.625).max() <= 1e-6
        assert np.abs(out - ref).max() <= 1e-5


def test_precision_far_from_origin_4k():
    """A one-pixel checkerboard near the right and bottom edges of a 4K frame
    with fractional motion: forming x - d in float32 would be off by ~1e-4."""
    dev = need_gpu()
    h, w = 2160, 3840
    ys, xs = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    img = ((xs + ys) % 2).astype(np.float32)[None, None].repeat(2, axis=1)
    rng = np.random.default_rng(3)
    mv = rng.uniform(-5, 5, (1, 2, h, w)).astype(np.float32)
    announce("precision 4k")
    s = to_dev(img, "f32", dev)
    out = exw.warp(s, torch.from_numpy(mv).to(dev), [0.25, 0.75, 1.0])
    torch.cuda.synchronize()
    py, px = np.meshgrid(np.arange(h - 40, h), np.arange(w - 300, w), indexing="ij")
    py, px = py.ravel(), px.ravel()
    for k, phase in enumerate([0.25, 0.75, 1.0]):
        ref, _ = warp_oracle.forward_at(img[0], mv[0], phase, py, px)
        got = out[0, k][:, torch.from_numpy(py).to(dev), torch.from_numpy(px).to(dev)]
        assert np.abs(to_host(got) - ref).max() <= 1e-5


def test_edge_cases_shapes_and_channels():
    dev = need_gpu()
    rng = np.random.default_rng(4)
    for (n, c, h, w, k) in [(1, 1, 1, 1, 1), (1, 3, 1, 9, 2), (2, 2, 7, 1, 3), (3, 5, 5, 65, 4),
                            (1, 12, 9, 130, 1), (2, 7, 4, 64, 2), (1, 64, 3, 5, 1),
                            (1, 4, 67, 257, 3)]:
        src = rng.random((n, c, h, w), dtype=np.float32)
        mv = rng.uniform(-3, 3, (n, 2, h, w)).astype(np.float32)
        phases = [0.25, 0.5, 0.75, 1.0][:k]
        for dtype in ("f32", "bf16"):
            announce("edge shapes", n, c, h, w, k, dtype)
            out, mask, cnt = run_forward(src, mv, phases, dtype, dev)
            ref, ref_mask, ref_cnt = warp_oracle.forward(stored(src, dtype), mv, phases)
            assert np.array_equal(mask, ref_mask) and np.array_equal(cnt, ref_cnt)
            assert_close_kernel(out, ref, dtype, f"shape {(n, c, h, w, k)}")
            ex, ex_mask, _ = warp_oracle.forward(stored(src, dtype), mv, phases, exact=True)
            compare_with_exact(out, mask, ex, ex_mask, mv, phases, dtype,
                               f"shape {(n, c, h, w, k)} {dtype}")


def test_non_finite_huge_and_denormal_motion():
    dev = need_gpu()
    h, w = 6, 70
    src = np.random.default_rng(5).random((1, 3, h, w), dtype=np.float32)
    specials = np.array([np.nan, np.inf, -np.inf, 1e30, -1e30, 3e38, 1e-40, -1e-40, 1e-45,
                         -0.0, 0.0, 69.0, -69.0, 70.0, 5.0, -5.0], np.float32)
    rng = np.random.default_rng(6)
    mv = np.stack([rng.choice(specials, (h, w)), rng.choice(specials, (h, w))])[None]
    mv = mv.astype(np.float32)
    for phases in ([1.0], [0.0], [0.5, 0.75], [-1.0, 2.0, 0.25, 1.0]):
        announce("specials", phases)
        out, mask, cnt = run_forward(src, mv, phases, "f32", dev)
        ref, ref_mask, ref_cnt = warp_oracle.forward(src, mv, phases)
        assert np.array_equal(mask, ref_mask), phases
        assert np.array_equal(cnt, ref_cnt)
        assert np.isfinite(out).all()
        assert np.abs(out - ref).max() <= 1e-5
        ex, ex_mask, _ = warp_oracle.forward(src, mv, phases, exact=True)
        compare_with_exact(out, mask, ex, ex_mask, mv, phases, "f32", f"specials {phases}")


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_non_finite_huge_and_denormal_motion_16bit(dtype):
    """The same special motion values on 16-bit frames of 1, 3, 4 and 12
    channels: the one-pixel paths load for invalid lanes too (the plane's
    first pair, unused), and those lanes must still come out 0 and unmasked."""
    dev = need_gpu()
    h, w = 6, 70
    specials = np.array([np.nan, np.inf, -np.inf, 1e30, -1e30, 3e38, 1e-40, -1e-40, 1e-45,
                         -0.0, 0.0, 69.0, -69.0, 70.0, 5.0, -5.0], np.float32)
    rng = np.random.default_rng(16)
    for c in (1, 3, 4, 12):
        src = rng.random((2, c, h, w), dtype=np.float32)
        mv = np.stack([rng.choice(specials, (2, h, w)), rng.choice(specials, (2, h, w))], axis=1)
        mv = mv.astype(np.float32)
        for phases in ([1.0], [0.5, 0.75], [-1.0, 2.0, 0.25, 1.0]):
            announce("specials 16-bit", dtype, c, phases)
            out, mask, cnt = run_forward(src, mv, phases, dtype, dev)
            ref, ref_mask, ref_cnt = warp_oracle.forward(stored(src, dtype), mv, phases)
            assert np.array_equal(mask, ref_mask), (c, phases)
            assert np.array_equal(cnt, ref_cnt)
            assert np.isfinite(out).all()
            invalid = np.broadcast_to((mask == 0)[:, :, None], out.shape)
            assert (out[invalid] == 0).all(), (c, phases)
            assert_close_kernel(out, ref, dtype, f"specials {dtype} c={c} {phases}")


def test_three_quarter_phase_at_the_bounds_exact_vs_rounded():
    """Motions whose product with the phase 3/4 lies within an ulp of a frame
    bound: the GPU decides validity on the float32-rounded displacement, so
    its masks equal the rounded-mode oracle bit for bit, and may differ from
    the exact mode only inside the rounding band (where some of them do)."""
    dev = need_gpu()
    h, w = 9, 130
    vals = []
    for b in range(-w, w + 1):
        g = np.float32(b / 0.75)
        vals += [g, np.nextafter(g, np.float32(np.inf)), np.nextafter(g, np.float32(-np.inf))]
    vals = np.array(vals, np.float32)
    rng = np.random.default_rng(8)
    mv = np.stack([rng.choice(vals, (h, w)), rng.uniform(-2, 2, (h, w)).astype(np.float32)])
    mv = mv[None].astype(np.float32)
    src = rng.random((1, 3, h, w), dtype=np.float32)
    announce("3/4 phase at the bounds")
    out, mask, cnt = run_forward(src, mv, [0.75], "f32", dev)
    ref, ref_mask, ref_cnt = warp_oracle.forward(src, mv, [0.75])
    assert np.array_equal(mask, ref_mask) and np.array_equal(cnt, ref_cnt)
    assert np.abs(out - ref).max() <= 1e-5
    ex, ex_mask, _ = warp_oracle.forward(src, mv, [0.75], exact=True)
    st = compare_with_exact(out, mask, ex, ex_mask, mv, [0.75], "f32", "3/4 at the bounds")
    assert st["band_pixels"] > 0
    assert rounding_band(mv, 0.75, h, w).sum() == st["band_pixels"]


def test_empty_batch_is_a_no_op():
    dev = need_gpu()
    src = torch.zeros((0, 3, 8, 8), device=dev)
    out, cnt = exw.warp(src, torch.zeros((0, 2, 8, 8), device=dev), [0.5], return_count=True)
    assert out.shape == (0, 1, 3, 8, 8) and cnt.shape == (0, 1)
    src = torch.zeros((2, 3, 0, 8), device=dev)
    out, cnt = exw.warp(src, torch.zeros((2, 2, 0, 8), device=dev), [0.5, 1.0],
                        return_count=True)
    torch.cuda.synchronize()
    assert (cnt == 0).all()


def test_single_frame_entry_point_matches_batched():
    dev = need_gpu()
    rng = np.random.default_rng(7)
    src = to_dev(rng.random((4, 33, 90), dtype=np.float32), "f16", dev)
    mv = torch.from_numpy(rng.uniform(-4, 4, (2, 33, 90)).astype(np.float32)).to(dev)
    out = torch.empty_like(src)
    mask = torch.empty((33, 90), dtype=torch.uint8, device=dev)
    announce("single frame")
    exw.exw_warp_forward(src, mv, 0.75, out, mask)
    ref, ref_mask = exw.warp(src[None], mv[None], [0.75], return_mask=True)
    assert torch.equal(out, ref[0, 0]) and torch.equal(mask, ref_mask[0, 0])


def test_binding_rejects_bad_shapes():
    dev = need_gpu()
    src = torch.zeros((1, 3, 8, 8), device=dev)
    mv = torch.zeros((1, 2, 8, 8), device=dev)
    with pytest.raises(ValueError):
        exw.exw_warp_forward_batched(src, mv, [1.0], torch.zeros((1, 2, 3, 8, 8), device=dev))
    with pytest.raises(ValueError):
        exw.exw_warp_forward_batched(src, mv.double(), [1.0],
                                     torch.zeros((1, 1, 3, 8, 8), device=dev))
    with pytest.raises(ValueError):
        exw.warp(src, mv, [1.0] * 5)
    with pytest.raises(exw.ExwError):
        exw.warp(src, mv, [float("nan")])


FULL = {2: ["f32", "f16"], 3: ["f32", "f16"]}


@pytest.mark.parametrize("index", sorted(FULL))
def test_full_size_forward_sampled(index):
    """Full-size workloads in the benchmark's launch configuration: the whole
    mask and invalid counts, and sampled pixel values, against the oracle."""
    dev = need_gpu()
    d = make_config(index)
    src, mv, phases = d["src"], d["mv"], list(d["phases"])
    n, c, h, w = src.shape
    rng = np.random.default_rng(index)
    ys = rng.integers(0, h, 4000)
    xs = rng.integers(0, w, 4000)
    # add the frame border, where invalid pixels live
    ys = np.concatenate([ys, np.zeros(w, int), np.full(w, h - 1), np.arange(h), np.arange(h)])
    xs = np.concatenate([xs, np.arange(w), np.arange(w), np.zeros(h, int), np.full(h, w - 1)])
    m_dev = torch.from_numpy(mv).to(dev)
    for dtype in FULL[index]:
        announce("full forward", index, dtype)
        s = to_dev(src, dtype, dev)
        out, mask, cnt = exw.warp(s, m_dev, phases, return_mask=True, return_count=True)
        torch.cuda.synchronize()
        cnt = cnt.cpu().numpy()
        yi = torch.from_numpy(ys).to(dev)
        xi = torch.from_numpy(xs).to(dev)
        for i in range(n):
            src_q = stored(src[i], dtype)
            for k, phase in enumerate(phases):
                valid, *_ = warp_oracle.taps(mv[i, 0], mv[i, 1], phase,
                                             np.arange(w)[None, :], np.arange(h)[:, None], h, w)
                assert np.array_equal(mask[i, k].cpu().numpy().astype(bool), valid)
                assert cnt[i, k] == valid.size - valid.sum()
                ref, _ = warp_oracle.forward_at(src_q, mv[i], phase, ys, xs)
                got = to_host(out[i, k][:, yi, xi])
                assert_close_kernel(got, ref, dtype, f"full config {index} {dtype} n={i} k={k}")
        del s, out, mask
        torch.cuda.empty_cache()
