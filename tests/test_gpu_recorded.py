"""The training pair on the GPU: the forward that records the adjoint's
footprint, and the adjoint that takes it from the workspace.

The forward's records must be byte for byte those of the adjoint's own
footprint pass (boxes, tap offsets and the per-frame figures); its outputs
those of the plain forward; and the recorded adjoint's gradients must match
the float64 oracle to the tolerances of the general adjoint tests. The cases
cover the two-pixel path (rigid motion), the one-pixel paths (moving
rectangles, random motion), ragged widths and heights, far segments, the
channel counts whose forward has no recording kernel (C = 2, width 1) and
one whose adjoint reads no footprint (C = 5), in every storage type.
"""

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from oracle import warp_oracle
from synth import make_config
from gpu_util import TORCH_DT, announce, half_ulp, need_gpu, stored, to_dev, to_host

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-5  # as in the general adjoint tests


def pan(n, h, w, px, py, rect=None):
    mv = np.empty((n, 2, h, w), np.float32)
    mv[:, 0], mv[:, 1] = px, py
    if rect is not None:
        y0, y1, x0, x1, rx, ry = rect
        mv[:, 0, y0:y1, x0:x1], mv[:, 1, y0:y1, x0:x1] = rx, ry
    return mv


def random_field(n, h, w, reach, seed):
    return np.random.default_rng(seed).uniform(-reach, reach, (n, 2, h, w)).astype(np.float32)


def records(ws: torch.Tensor, n: int, h: int, w: int) -> dict:
    """The footprint part of the adjoint workspace (layout of exwarp.h: boxes
    and offsets, 32 bytes per 64-pixel segment, then 8 bytes per frame at the
    next 256-byte boundary)."""
    seg_bytes = 32 * n * h * ((w + 63) // 64)
    info = (seg_bytes + 255) // 256 * 256
    host = ws.cpu().numpy()
    return {"segments": host[:seg_bytes].copy(), "frames": host[info:info + 8 * n].copy()}


# (label, n, c, h, w, motion, phases, dtype)
CASES = [
    ("pan two-pixel f32", 2, 4, 70, 300, pan(2, 70, 300, 2.5, -3.0), (0.25, 0.5, 0.75), "f32"),
    ("pan shared offsets f16", 1, 4, 45, 260, pan(1, 45, 260, 0.6, -0.8), (0.25, 0.5, 0.75), "f16"),
    ("pan + block C=3 K=4", 1, 3, 66, 390, pan(1, 66, 390, 1.7, -0.6, (20, 44, 70, 150, -5.5, 3.25)),
     (0.25, 0.5, 0.75, 1.0), "f32"),
    ("far pan K=1", 1, 4, 40, 400, pan(1, 40, 400, 150.0, 2.0), (1.0,), "f32"),
    ("random C=3 K=1", 2, 3, 37, 131, random_field(2, 37, 131, 4.0, 3), (1.0,), "f32"),
    ("random C=1 K=2 bf16", 1, 1, 29, 77, random_field(1, 29, 77, 6.0, 4), (0.5, 1.0), "bf16"),
    ("G-buffer C=12 K=1 bf16", 1, 12, 23, 200, pan(1, 23, 200, -3.5, 1.25, (5, 15, 40, 120, 9.0, -4.0)),
     (1.0,), "bf16"),
    ("G-buffer C=12 K=3", 1, 12, 19, 140, pan(1, 19, 140, 1.0, 2.0), (0.25, 0.5, 0.75), "f32"),
    ("C=2 (separate footprint pass)", 2, 2, 21, 150, random_field(2, 21, 150, 3.0, 5),
     (0.25, 0.75), "f16"),
    ("width 1", 1, 3, 17, 1, random_field(1, 17, 1, 2.0, 6), (0.5,), "f32"),
    ("C=5 (no footprint)", 1, 5, 20, 70, random_field(1, 20, 70, 2.0, 7), (1.0,), "f32"),
    ("narrow ragged", 3, 4, 6, 45, pan(3, 6, 45, -0.3, 0.7), (0.25, 0.5, 0.75), "f32"),
    # 16-bit storage, several 128-pixel segments per row, a moving block, C = 12
    ("wide pan f16", 2, 4, 21, 600, pan(2, 21, 600, 2.5, -3.0), (0.25, 0.5, 0.75), "f16"),
    ("wide pan + block bf16 C=3", 1, 3, 30, 520,
     pan(1, 30, 520, -1.3, 0.9, (8, 20, 200, 290, 6.5, -2.25)), (0.25, 0.5, 0.75, 1.0), "bf16"),
    ("wide G-buffer C=12 K=2 f16", 1, 12, 11, 512, pan(1, 11, 512, 0.4, -1.6),
     (0.5, 1.0), "f16"),
]


def run_case(label, n, c, h, w, mv, phases, dtype, dev):
    src = np.random.default_rng(h * w + c).random((n, c, h, w)).astype(np.float32)
    k = len(phases)
    g = np.random.default_rng(c + 31).standard_normal((n, k, c, h, w)).astype(np.float32)
    tdt = TORCH_DT[dtype]
    s = to_dev(src, dtype, dev)
    m = torch.from_numpy(np.ascontiguousarray(mv)).to(dev)
    gd = to_dev(g, dtype, dev)
    nbytes = exw.exw_warp_backward_workspace_bytes(tdt, n, c, h, w)

    announce("recorded: plain forward and adjoint", label, dtype, (n, c, h, w), phases)
    out0 = torch.empty((n, k, c, h, w), dtype=tdt, device=dev)
    mask0 = torch.empty((n, k, h, w), dtype=torch.uint8, device=dev)
    cnt0 = torch.empty((n, k), dtype=torch.int32, device=dev)
    exw.exw_warp_forward_batched(s, m, phases, out0, mask0, cnt0)
    ws0 = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device=dev)
    gs0 = torch.empty_like(s)
    gm0 = torch.empty((n, 2, h, w), device=dev)
    exw.exw_warp_backward_batched(s, m, phases, gd, gs0, gm0, ws0)

    announce("recorded: recording forward", label)
    out1 = torch.empty_like(out0)
    mask1 = torch.empty_like(mask0)
    cnt1 = torch.empty_like(cnt0)
    ws1 = torch.full((nbytes,), 0x5A, dtype=torch.uint8, device=dev)
    exw.exw_warp_forward_batched_record(s, m, phases, out1, ws1, mask1, cnt1)
    torch.cuda.synchronize()
    assert torch.equal(out0, out1) and torch.equal(mask0, mask1) and torch.equal(cnt0, cnt1), label
    if c in (1, 2, 3, 4, 12):  # adjoints that read the footprint
        r0, r1 = records(ws0, n, h, w), records(ws1, n, h, w)
        assert np.array_equal(r0["segments"], r1["segments"]), f"{label}: segment records differ"
        assert np.array_equal(r0["frames"], r1["frames"]), f"{label}: frame records differ"

    announce("recorded: adjoint from the records", label)
    gs1 = torch.empty_like(s)
    gm1 = torch.empty_like(gm0)
    exw.exw_warp_backward_batched_recorded(s, m, phases, gd, gs1, gm1, ws1)
    torch.cuda.synchronize()
    ref_gs, ref_gm = warp_oracle.backward(stored(src, dtype), mv, list(phases), stored(g, dtype))
    for got, ref, what in ((to_host(gm1), ref_gm, "grad_mv"), (to_host(gs1), ref_gs, "grad_src")):
        if what == "grad_src" and dtype != "f32":
            bound = half_ulp(ref, dtype) + GRAD_TOL * np.maximum(1.0, np.abs(ref))
            assert (np.abs(got - ref) <= bound).all(), f"{what} {label}"
        else:
            err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
            assert float(err.max()) <= GRAD_TOL, f"{what} {label}: rel err {float(err.max())}"
    # the motion gradient does not depend on the records: same kernels, same order
    assert torch.equal(gm0, gm1), label


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_recorded_pair(case):
    run_case(*case, need_gpu())


def test_recorded_pair_full_size_workload():
    """8 x 1920 x 1080 RGBA, three phases, moving rectangles: the records of
    the benchmark's batch, and sampled gradients against the oracle."""
    dev = need_gpu()
    d = make_config(2)
    src, mv, phases = d["src"], d["mv"], list(d["phases"])
    n, c, h, w = src.shape
    k = len(phases)
    announce("recorded: full-size workload 2")
    s = to_dev(src, "f32", dev)
    m = torch.from_numpy(mv).to(dev)
    gen = torch.Generator(device=dev).manual_seed(12)
    gd = torch.randn((n, k, c, h, w), device=dev, generator=gen)
    nbytes = exw.exw_warp_backward_workspace_bytes(torch.float32, n, c, h, w)
    ws0 = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    ws1 = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    gs0, gm0 = torch.empty_like(s), torch.empty((n, 2, h, w), device=dev)
    exw.exw_warp_backward_batched(s, m, phases, gd, gs0, gm0, ws0)
    out = torch.empty((n, k, c, h, w), device=dev)
    exw.exw_warp_forward_batched_record(s, m, phases, out, ws1)
    gs1, gm1 = torch.empty_like(s), torch.empty_like(gm0)
    exw.exw_warp_backward_batched_recorded(s, m, phases, gd, gs1, gm1, ws1)
    torch.cuda.synchronize()
    r0, r1 = records(ws0, n, h, w), records(ws1, n, h, w)
    assert np.array_equal(r0["segments"], r1["segments"])
    assert np.array_equal(r0["frames"], r1["frames"])
    assert torch.equal(gm0, gm1)
    # image gradients: same replays in the same order, up to the order of LDS
    # atomics at motion boundaries
    err = ((gs1 - gs0).abs() / gs0.abs().clamp(min=1.0)).max().item()
    assert err <= GRAD_TOL, err
    # sampled pixels against the oracle
    rng = np.random.default_rng(13)
    fr = 3
    ys, xs = rng.integers(0, h, 200), rng.integers(0, w, 200)
    ref_gm = warp_oracle.grad_mv_at(src[fr], mv[fr], phases, to_host(gd[fr]), ys, xs)
    got_gm = to_host(gm1[fr][:, torch.from_numpy(ys).to(dev), torch.from_numpy(xs).to(dev)])
    err = np.abs(got_gm - ref_gm) / np.maximum(1.0, np.abs(ref_gm))
    assert float(err.max()) <= GRAD_TOL


def test_autograd_uses_the_recorded_pair(monkeypatch):
    """warp_differentiable records in its forward and skips the footprint pass
    in its backward: gradients equal those of the plain adjoint."""
    dev = need_gpu()
    d = make_config(2, n=2, h=75, w=131)
    phases = list(d["phases"])
    calls = []
    rec_fwd, bwd = exw.exw_warp_forward_batched_record, exw.exw_warp_backward_batched

    def spy_fwd(*args, **kwargs):
        calls.append("record")
        return rec_fwd(*args, **kwargs)

    def spy_bwd(*args, **kwargs):
        calls.append("recorded" if kwargs.get("recorded") else "plain")
        return bwd(*args, **kwargs)

    monkeypatch.setattr(exw, "exw_warp_forward_batched_record", spy_fwd)
    monkeypatch.setattr(exw, "exw_warp_backward_batched", spy_bwd)
    for dtype in ("f32", "f16"):
        announce("recorded: autograd", dtype)
        src = to_dev(d["src"], dtype, dev).requires_grad_(True)
        mv = torch.from_numpy(d["mv"]).to(dev).requires_grad_(True)
        calls.clear()
        out = exw.warp_differentiable(src, mv, phases)
        wgt = torch.linspace(-1, 1, out.numel(), device=dev).reshape(out.shape).to(out.dtype)
        (out.float() * wgt.float()).sum().backward()
        assert calls == ["record", "recorded"], calls
        gs, gm = exw.warp_backward(src.detach(), mv.detach(), phases, wgt)
        assert torch.equal(out.detach(), exw.warp(src.detach(), mv.detach(), phases))
        assert torch.equal(mv.grad, gm)
        tol = 1e-5 if dtype == "f32" else 2e-3
        assert torch.allclose(src.grad.float(), gs.float(), rtol=tol, atol=tol)


def test_recorded_pair_many_small_frames():
    """More frames than a second grid dimension could hold (70000 frames of
    5 x 7 px, random motion): the training pair's records, outputs and
    gradients against the plain calls, and three frames against the oracle."""
    dev = need_gpu()
    n, c, h, w, phases = 70000, 3, 5, 7, (0.5, 1.0)
    k = len(phases)
    rng = np.random.default_rng(21)
    src = rng.random((n, c, h, w), dtype=np.float32)
    mv = rng.uniform(-3, 3, (n, 2, h, w)).astype(np.float32)
    g = rng.standard_normal((n, k, c, h, w)).astype(np.float32)
    s, m, gd = (torch.from_numpy(a).to(dev) for a in (src, mv, g))
    nbytes = exw.exw_warp_backward_workspace_bytes(torch.float32, n, c, h, w)
    announce("recorded: 70000 small frames")
    outs = [torch.empty((n, k, c, h, w), device=dev) for _ in range(2)]
    masks = [torch.empty((n, k, h, w), dtype=torch.uint8, device=dev) for _ in range(2)]
    cnts = [torch.empty((n, k), dtype=torch.int32, device=dev) for _ in range(2)]
    wss = [torch.empty(nbytes, dtype=torch.uint8, device=dev) for _ in range(2)]
    gss = [torch.empty_like(s) for _ in range(2)]
    gms = [torch.empty((n, 2, h, w), device=dev) for _ in range(2)]
    exw.exw_warp_forward_batched(s, m, phases, outs[0], masks[0], cnts[0])
    exw.exw_warp_backward_batched(s, m, phases, gd, gss[0], gms[0], wss[0])
    exw.exw_warp_forward_batched_record(s, m, phases, outs[1], wss[1], masks[1], cnts[1])
    exw.exw_warp_backward_batched_recorded(s, m, phases, gd, gss[1], gms[1], wss[1])
    torch.cuda.synchronize()
    r0, r1 = records(wss[0], n, h, w), records(wss[1], n, h, w)
    assert np.array_equal(r0["segments"], r1["segments"])
    assert np.array_equal(r0["frames"], r1["frames"])
    assert torch.equal(outs[0], outs[1]) and torch.equal(masks[0], masks[1])
    assert torch.equal(cnts[0], cnts[1]) and torch.equal(gms[0], gms[1])
    err = ((gss[1] - gss[0]).abs() / gss[0].abs().clamp(min=1.0)).max().item()
    assert err <= GRAD_TOL, err
    pick = [0, 65536, n - 1]
    ref_gs, ref_gm = warp_oracle.backward(src[pick], mv[pick], list(phases), g[pick])
    for got, ref in ((to_host(gss[1][pick]), ref_gs), (to_host(gms[1][pick]), ref_gm)):
        assert float((np.abs(got - ref) / np.maximum(1.0, np.abs(ref))).max()) <= GRAD_TOL
