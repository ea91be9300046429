"""Thin Python binding of libexwarp: the C-ABI entry points under the same
names, taking torch tensors (device memory) and the current HIP stream.

Each function checks that tensor shapes, dtypes, devices and contiguity match
the layouts of include/exwarp.h (the library trusts the sizes it is given),
then passes raw pointers. All arithmetic happens in the library's kernels.
"""

from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _capi
from ._capi import EXW_BF16, EXW_F16, EXW_F32, EXW_MAX_PHASES, ExwError, check, lib

DTYPES = {torch.float32: EXW_F32, torch.float16: EXW_F16, torch.bfloat16: EXW_BF16}


def exw_dtype(t: torch.dtype) -> int:
    try:
        return DTYPES[t]
    except KeyError:
        raise TypeError(f"unsupported frame dtype {t}; use float32, float16 or bfloat16") from None


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, name: str, device: torch.device) -> None:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _expect(t: Optional[torch.Tensor], name: str, shape: Sequence[int], dtype: torch.dtype,
            device: torch.device) -> None:
    if t is None:
        return
    _dev(t, name, device)
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")


def _phases(phases) -> tuple:
    ph = [float(s) for s in phases]
    if not 1 <= len(ph) <= EXW_MAX_PHASES:
        raise ValueError(f"need 1..{EXW_MAX_PHASES} phases, got {len(ph)}")
    arr = (ctypes.c_float * len(ph))(*ph)
    return arr, len(ph)


def _stream(device: torch.device, stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def exw_warp_forward_batched(src: torch.Tensor, mv: torch.Tensor, phases, out: torch.Tensor,
                             mask: Optional[torch.Tensor] = None,
                             invalid_count: Optional[torch.Tensor] = None, stream=None) -> None:
    """src [N,C,H,W], mv [N,2,H,W] f32, out [N,K,C,H,W], mask [N,K,H,W] u8,
    invalid_count [N,K] int32 (read as uint32)."""
    dev = src.device
    _dev(src, "src", dev)
    n, c, h, w = src.shape
    arr, k = _phases(phases)
    _expect(mv, "mv", (n, 2, h, w), torch.float32, dev)
    _expect(out, "out", (n, k, c, h, w), src.dtype, dev)
    _expect(mask, "mask", (n, k, h, w), torch.uint8, dev)
    _expect(invalid_count, "invalid_count", (n, k), torch.int32, dev)
    st = lib().exw_warp_forward_batched(_ptr(src), exw_dtype(src.dtype), n, c, h, w, _ptr(mv),
                                        arr, k, _ptr(out), _ptr(mask), _ptr(invalid_count),
                                        _stream(dev, stream))
    check(st, "exw_warp_forward_batched")


def exw_warp_forward_batched_record(src: torch.Tensor, mv: torch.Tensor, phases, out: torch.Tensor,
                                    workspace: torch.Tensor, mask: Optional[torch.Tensor] = None,
                                    invalid_count: Optional[torch.Tensor] = None,
                                    motion_stats: Optional[torch.Tensor] = None,
                                    stream=None) -> None:
    """exw_warp_forward_batched, also leaving the adjoint's footprint of this
    motion and these phases in ``workspace`` (a byte tensor of at least
    ``exw_warp_backward_workspace_bytes`` bytes) for
    exw_warp_backward_batched_recorded; with ``motion_stats`` ([N,4] float64)
    also the per-frame motion statistics, from the same motion read."""
    dev = src.device
    _dev(src, "src", dev)
    n, c, h, w = src.shape
    arr, k = _phases(phases)
    _expect(mv, "mv", (n, 2, h, w), torch.float32, dev)
    _expect(out, "out", (n, k, c, h, w), src.dtype, dev)
    _expect(mask, "mask", (n, k, h, w), torch.uint8, dev)
    _expect(invalid_count, "invalid_count", (n, k), torch.int32, dev)
    _expect(motion_stats, "motion_stats", (n, 4), torch.float64, dev)
    _dev(workspace, "workspace", dev)
    st = lib().exw_warp_forward_batched_record(
        _ptr(src), exw_dtype(src.dtype), n, c, h, w, _ptr(mv), arr, k, _ptr(out), _ptr(mask),
        _ptr(invalid_count), _ptr(motion_stats), _ptr(workspace),
        workspace.numel() * workspace.element_size(), _stream(dev, stream))
    check(st, "exw_warp_forward_batched_record")


def exw_warp_forward(src: torch.Tensor, mv: torch.Tensor, phase: float, out: torch.Tensor,
                     mask: Optional[torch.Tensor] = None, stream=None) -> None:
    """One frame: src [C,H,W], mv [2,H,W] f32, out [C,H,W], mask [H,W] u8."""
    dev = src.device
    _dev(src, "src", dev)
    c, h, w = src.shape
    _expect(mv, "mv", (2, h, w), torch.float32, dev)
    _expect(out, "out", (c, h, w), src.dtype, dev)
    _expect(mask, "mask", (h, w), torch.uint8, dev)
    st = lib().exw_warp_forward(_ptr(src), exw_dtype(src.dtype), c, h, w, _ptr(mv),
                                ctypes.c_float(phase), _ptr(out), _ptr(mask),
                                _stream(dev, stream))
    check(st, "exw_warp_forward")


def exw_warp_backward_workspace_bytes(dtype: torch.dtype, n: int, c: int, h: int, w: int) -> int:
    return int(lib().exw_warp_backward_workspace_bytes(exw_dtype(dtype), n, c, h, w))


def exw_warp_backward_batched(src: Optional[torch.Tensor], mv: torch.Tensor, phases,
                              grad_out: torch.Tensor, grad_src: Optional[torch.Tensor] = None,
                              grad_mv: Optional[torch.Tensor] = None,
                              workspace: Optional[torch.Tensor] = None, stream=None,
                              recorded: bool = False) -> None:
    """grad_out [N,K,C,H,W] -> grad_src [N,C,H,W] (dtype of grad_out) and/or
    grad_mv [N,2,H,W] f32. ``workspace``: a byte tensor of at least
    ``exw_warp_backward_workspace_bytes`` bytes (needed for f16/bf16 grad_src)."""
    dev = grad_out.device
    _dev(grad_out, "grad_out", dev)
    n, k, c, h, w = grad_out.shape
    arr, k2 = _phases(phases)
    if k2 != k:
        raise ValueError(f"grad_out has {k} phases, got {k2} phase values")
    dt = grad_out.dtype
    _expect(src, "src", (n, c, h, w), dt, dev)
    _expect(mv, "mv", (n, 2, h, w), torch.float32, dev)
    _expect(grad_src, "grad_src", (n, c, h, w), dt, dev)
    _expect(grad_mv, "grad_mv", (n, 2, h, w), torch.float32, dev)
    ws_bytes = 0
    if workspace is not None:
        _dev(workspace, "workspace", dev)
        ws_bytes = workspace.numel() * workspace.element_size()
    name = "exw_warp_backward_batched_recorded" if recorded else "exw_warp_backward_batched"
    st = getattr(lib(), name)(_ptr(src), exw_dtype(dt), n, c, h, w, _ptr(mv), arr, k,
                              _ptr(grad_out), _ptr(grad_src), _ptr(grad_mv),
                              _ptr(workspace), ws_bytes, _stream(dev, stream))
    check(st, name)


def exw_warp_backward_batched_recorded(src: Optional[torch.Tensor], mv: torch.Tensor, phases,
                                       grad_out: torch.Tensor,
                                       grad_src: Optional[torch.Tensor] = None,
                                       grad_mv: Optional[torch.Tensor] = None,
                                       workspace: Optional[torch.Tensor] = None,
                                       stream=None) -> None:
    """exw_warp_backward_batched with the footprint that
    exw_warp_forward_batched_record left in ``workspace`` for the same motion,
    phases, dtype and shape."""
    exw_warp_backward_batched(src, mv, phases, grad_out, grad_src, grad_mv, workspace, stream,
                              recorded=True)


def exw_warp_backward(src: Optional[torch.Tensor], mv: torch.Tensor, phase: float,
                      grad_out: torch.Tensor, grad_src: Optional[torch.Tensor] = None,
                      grad_mv: Optional[torch.Tensor] = None,
                      workspace: Optional[torch.Tensor] = None, stream=None) -> None:
    """One frame: grad_out [C,H,W] -> grad_src [C,H,W], grad_mv [2,H,W]."""
    dev = grad_out.device
    _dev(grad_out, "grad_out", dev)
    c, h, w = grad_out.shape
    dt = grad_out.dtype
    _expect(src, "src", (c, h, w), dt, dev)
    _expect(mv, "mv", (2, h, w), torch.float32, dev)
    _expect(grad_src, "grad_src", (c, h, w), dt, dev)
    _expect(grad_mv, "grad_mv", (2, h, w), torch.float32, dev)
    ws_bytes = 0
    if workspace is not None:
        _dev(workspace, "workspace", dev)
        ws_bytes = workspace.numel() * workspace.element_size()
    st = lib().exw_warp_backward(_ptr(src), exw_dtype(dt), c, h, w, _ptr(mv),
                                 ctypes.c_float(phase), _ptr(grad_out), _ptr(grad_src),
                                 _ptr(grad_mv), _ptr(workspace), ws_bytes, _stream(dev, stream))
    check(st, "exw_warp_backward")


def exw_motion_stats_workspace_bytes(n: int, h: int, w: int) -> int:
    return int(lib().exw_motion_stats_workspace_bytes(n, h, w))


def exw_motion_stats(mv: torch.Tensor, stats: torch.Tensor,
                     workspace: Optional[torch.Tensor] = None, stream=None) -> None:
    """mv [N,2,H,W] f32 -> stats [N,4] f64 = (mean_x, var_x, mean_y, var_y).
    ``workspace``: a byte tensor of at least ``exw_motion_stats_workspace_bytes``."""
    dev = mv.device
    _dev(mv, "mv", dev)
    if mv.dim() != 4 or mv.shape[1] != 2:
        raise ValueError(f"mv has shape {tuple(mv.shape)}, expected [N, 2, H, W]")
    if mv.dtype != torch.float32:
        raise ValueError(f"mv has dtype {mv.dtype}, expected torch.float32")
    n, _, h, w = mv.shape
    _expect(stats, "stats", (n, 4), torch.float64, dev)
    ws_bytes = 0
    if workspace is not None:
        _dev(workspace, "workspace", dev)
        ws_bytes = workspace.numel() * workspace.element_size()
    st = lib().exw_motion_stats(_ptr(mv), n, h, w, _ptr(stats), _ptr(workspace), ws_bytes,
                                _stream(dev, stream))
    check(st, "exw_motion_stats")


def exw_motion_stats_no_alloc(mv: torch.Tensor, stats: torch.Tensor, stream=None) -> None:
    """exw_motion_stats with the library's static device scratch instead of a
    workspace (no allocation; calls that overlap on one GPU race)."""
    dev = mv.device
    _dev(mv, "mv", dev)
    if mv.dim() != 4 or mv.shape[1] != 2:
        raise ValueError(f"mv has shape {tuple(mv.shape)}, expected [N, 2, H, W]")
    if mv.dtype != torch.float32:
        raise ValueError(f"mv has dtype {mv.dtype}, expected torch.float32")
    n, _, h, w = mv.shape
    _expect(stats, "stats", (n, 4), torch.float64, dev)
    st = lib().exw_motion_stats_no_alloc(_ptr(mv), n, h, w, _ptr(stats), _stream(dev, stream))
    check(st, "exw_motion_stats_no_alloc")


def exw_buffer_emd_workspace_bytes(n: int, c: int, bins: int) -> int:
    return int(lib().exw_buffer_emd_workspace_bytes(n, c, bins))


def exw_buffer_emd(cur: torch.Tensor, prev: torch.Tensor, lo: float, hi: float, bins: int,
                   emd: torch.Tensor, workspace: Optional[torch.Tensor] = None,
                   stream=None) -> None:
    """cur, prev [N,C,H,W] (one dtype) -> emd [N,C] f64: per-channel EMD between
    the value histograms (``bins`` bins on [lo, hi]). ``workspace``: a byte
    tensor of at least ``exw_buffer_emd_workspace_bytes`` bytes."""
    dev = cur.device
    _dev(cur, "cur", dev)
    if cur.dim() != 4:
        raise ValueError(f"cur has shape {tuple(cur.shape)}, expected [N, C, H, W]")
    n, c, h, w = cur.shape
    _expect(prev, "prev", (n, c, h, w), cur.dtype, dev)
    _expect(emd, "emd", (n, c), torch.float64, dev)
    ws_bytes = 0
    if workspace is not None:
        _dev(workspace, "workspace", dev)
        ws_bytes = workspace.numel() * workspace.element_size()
    st = lib().exw_buffer_emd(_ptr(cur), _ptr(prev), exw_dtype(cur.dtype), n, c, h, w,
                              ctypes.c_double(lo), ctypes.c_double(hi), bins, _ptr(emd),
                              _ptr(workspace), ws_bytes, _stream(dev, stream))
    check(st, "exw_buffer_emd")


def exw_dynamic_objects_workspace_bytes(n: int, h: int, w: int) -> int:
    return int(lib().exw_dynamic_objects_workspace_bytes(n, h, w))


def exw_dynamic_objects(stencil: torch.Tensor, count: torch.Tensor,
                        workspace: Optional[torch.Tensor] = None, connectivity: int = 8,
                        stream=None) -> None:
    """stencil [N,H,W] uint8 -> count [N] int32 (bit pattern of the C ABI's
    uint32): the number of connected components of the marked (non-zero)
    pixels of each frame. ``workspace``: a byte tensor of at least
    ``exw_dynamic_objects_workspace_bytes`` bytes."""
    dev = stencil.device
    _dev(stencil, "stencil", dev)
    if stencil.dim() != 3:
        raise ValueError(f"stencil has shape {tuple(stencil.shape)}, expected [N, H, W]")
    n, h, w = stencil.shape
    _expect(stencil, "stencil", (n, h, w), torch.uint8, dev)
    _expect(count, "count", (n,), torch.int32, dev)
    ws_bytes = 0
    if workspace is not None:
        _dev(workspace, "workspace", dev)
        ws_bytes = workspace.numel() * workspace.element_size()
    st = lib().exw_dynamic_objects(_ptr(stencil), n, h, w, connectivity, _ptr(count),
                                   _ptr(workspace), ws_bytes, _stream(dev, stream))
    check(st, "exw_dynamic_objects")


def exw_frame_quality_workspace_bytes(b: int, c: int, h: int, w: int) -> int:
    return int(lib().exw_frame_quality_workspace_bytes(b, c, h, w))


def exw_frame_quality(pred: torch.Tensor, truth: torch.Tensor, quality: torch.Tensor,
                      workspace: Optional[torch.Tensor] = None, peak: float = 1.0,
                      stream=None) -> None:
    """pred, truth [B,C,H,W] (same dtype) -> quality [B,3] f64 = (MSE, PSNR, SSIM).
    ``workspace``: a byte tensor of at least ``exw_frame_quality_workspace_bytes``."""
    dev = pred.device
    _dev(pred, "pred", dev)
    if pred.dim() != 4:
        raise ValueError(f"pred has shape {tuple(pred.shape)}, expected [B, C, H, W]")
    b, c, h, w = pred.shape
    _expect(truth, "truth", (b, c, h, w), pred.dtype, dev)
    _expect(quality, "quality", (b, 3), torch.float64, dev)
    ws_bytes = 0
    if workspace is not None:
        _dev(workspace, "workspace", dev)
        ws_bytes = workspace.numel() * workspace.element_size()
    st = lib().exw_frame_quality(_ptr(pred), _ptr(truth), exw_dtype(pred.dtype), b, c, h, w,
                                 ctypes.c_double(peak), _ptr(quality), _ptr(workspace), ws_bytes,
                                 _stream(dev, stream))
    check(st, "exw_frame_quality")


def exw_warp_chain(src: torch.Tensor, mv: torch.Tensor, phase: float, steps: int,
                   out: torch.Tensor, mask: Optional[torch.Tensor] = None,
                   invalid_count: Optional[torch.Tensor] = None, stream=None) -> None:
    """src [N,C,H,W], mv [N,2,H,W] f32 -> out [S,N,C,H,W] (step-major), mask
    [S,N,H,W] u8, invalid_count [S,N] u32/i32: out[i] = W(out[i-1], phase)."""
    dev = src.device
    _dev(src, "src", dev)
    n, c, h, w = src.shape
    dt = src.dtype
    _expect(mv, "mv", (n, 2, h, w), torch.float32, dev)
    _expect(out, "out", (steps, n, c, h, w), dt, dev)
    _expect(mask, "mask", (steps, n, h, w), torch.uint8, dev)
    if invalid_count is not None:
        _dev(invalid_count, "invalid_count", dev)
        if tuple(invalid_count.shape) != (steps, n) or invalid_count.dtype not in (torch.int32,
                                                                                 torch.uint32):
            raise ValueError("invalid_count must be [S, N] int32/uint32")
    st = lib().exw_warp_chain(_ptr(src), exw_dtype(dt), n, c, h, w, _ptr(mv),
                              ctypes.c_float(phase), steps, _ptr(out), _ptr(mask),
                              _ptr(invalid_count), _stream(dev, stream))
    check(st, "exw_warp_chain")


def exw_decision_plan(d1: int, d2: int, d_last: int) -> "_capi.DisplayPlan":
    """Host-only: the frames shown for decisions (d1, d2, d_last)."""
    plan = _capi.DisplayPlan()
    check(lib().exw_decision_plan(d1, d2, d_last, ctypes.byref(plan)), "exw_decision_plan")
    return plan


def exw_threshold_policy(motion_stats, invalid_fraction, max_variance: float,
                         max_invalid: float) -> tuple:
    """Host-only: (d1, d2, d_last) of the fixed policy for one frame."""
    st = (ctypes.c_double * 4)(*[float(v) for v in motion_stats])
    inv = (ctypes.c_double * 3)(*[float(v) for v in invalid_fraction])
    dec = (ctypes.c_int32 * 3)()
    check(lib().exw_threshold_policy(st, inv, ctypes.c_double(max_variance),
                                     ctypes.c_double(max_invalid), dec), "exw_threshold_policy")
    return tuple(dec)


__all__ = ["ExwError", "exw_dtype", "exw_warp_forward_batched", "exw_warp_forward_batched_record",
           "exw_warp_forward", "exw_warp_backward_workspace_bytes", "exw_warp_backward_batched",
           "exw_warp_backward_batched_recorded", "exw_warp_backward",
           "exw_motion_stats_workspace_bytes", "exw_motion_stats",
           "exw_frame_quality_workspace_bytes", "exw_frame_quality", "exw_warp_chain",
           "exw_decision_plan", "exw_threshold_policy", "_capi"]


def _bytes_of(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def exw_stream_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """dst <- src (same byte size, contiguous device tensors): the plain HBM copy
    the warp kernels are measured against."""
    dev = src.device
    _dev(src, "src", dev)
    _dev(dst, "dst", dev)
    if _bytes_of(src) != _bytes_of(dst):
        raise ValueError("src and dst differ in size")
    check(lib().exw_stream_copy(_ptr(src), _ptr(dst), _bytes_of(src), _stream(dev, stream)),
          "exw_stream_copy")


def exw_stream_read(src: torch.Tensor, sink: torch.Tensor, stream=None) -> None:
    """Reads every byte of src (sink: a float32 device tensor, never written)."""
    dev = src.device
    _dev(src, "src", dev)
    _expect(sink, "sink", tuple(sink.shape), torch.float32, dev)
    check(lib().exw_stream_read(_ptr(src), _bytes_of(src), _ptr(sink), _stream(dev, stream)),
          "exw_stream_read")


def exw_stream_write(dst: torch.Tensor, stream=None) -> None:
    """Writes zeros over every byte of dst."""
    dev = dst.device
    _dev(dst, "dst", dev)
    check(lib().exw_stream_write(_ptr(dst), _bytes_of(dst), _stream(dev, stream)),
          "exw_stream_write")
