"""exwarp: motion-vector frame warping for ExWarp's fast branch on MI355X.

The last rendered frame is warped with its per-pixel motion vectors, scaled
by the extrapolation phase, to predict the frames shown between rendered
frames (paper §II-B, §III-D, §IV-B). The work runs in hand-written HIP
kernels behind the C-ABI of ``libexwarp.so`` (``include/exwarp.h``); this
package marshals torch tensors to that ABI:

* ``binding.exw_*``: the C-ABI entry points under the same names.
* ``warp``: allocate outputs and run the batched forward warp.
* ``WarpFunction`` / ``warp_differentiable``: autograd over the hand-written
  adjoint (gradients for the frames and the motion vectors).
* ``motion_stats``: per-frame mean and variance of the motion field, the
  scene-state feature the warp/extrapolate decision is taken on (§IV-C, Eq. 1).
* ``frame_quality``: per-frame MSE, PSNR and SSIM against the ground truth,
  the quality terms of the decision's reward (§IV-C1).
* ``warp_chain``, ``plan``, ``threshold_policy``, ``decision_path_frames``:
  the decision paths of §IV-B / Table V (chained warps W(P_i) on the GPU,
  the decision tree and a fixed policy in native host code).
"""

from __future__ import annotations

from typing import Sequence

import torch

from ._capi import ExwError, lib  # noqa: F401  (lib() raises if the library is missing)
from .binding import (  # noqa: F401
    exw_warp_backward,
    exw_warp_backward_batched,
    exw_warp_backward_batched_recorded,
    exw_warp_backward_workspace_bytes,
    exw_decision_plan,
    exw_frame_quality,
    exw_frame_quality_workspace_bytes,
    exw_threshold_policy,
    exw_warp_chain,
    exw_motion_stats,
    exw_motion_stats_workspace_bytes,
    exw_motion_stats_no_alloc,
    exw_buffer_emd,
    exw_buffer_emd_workspace_bytes,
    exw_dynamic_objects,
    exw_dynamic_objects_workspace_bytes,
    exw_warp_forward,
    exw_warp_forward_batched,
    exw_warp_forward_batched_record,
    exw_stream_copy,
    exw_stream_read,
    exw_stream_write,
)

# Fail at import, not at first use, when the native library is absent.
lib()


def warp(src: torch.Tensor, mv: torch.Tensor, phases: Sequence[float] = (1.0,), *,
         return_mask: bool = False, return_count: bool = False):
    """Warp ``src`` [N,C,H,W] by ``mv`` [N,2,H,W] at each phase.

    Returns ``out`` [N,K,C,H,W] (dtype of ``src``), plus ``mask`` [N,K,H,W]
    uint8 and/or ``invalid_count`` [N,K] int32 when asked for.
    """
    src = src.contiguous()
    mv = mv.contiguous()
    n, c, h, w = src.shape
    k = len(phases)
    out = torch.empty((n, k, c, h, w), dtype=src.dtype, device=src.device)
    mask = torch.empty((n, k, h, w), dtype=torch.uint8, device=src.device) if return_mask else None
    cnt = torch.empty((n, k), dtype=torch.int32, device=src.device) if return_count else None
    exw_warp_forward_batched(src, mv, phases, out, mask, cnt)
    res = [out]
    if return_mask:
        res.append(mask)
    if return_count:
        res.append(cnt)
    return res[0] if len(res) == 1 else tuple(res)


def warp_backward(src, mv, phases, grad_out, *, need_src: bool = True, need_mv: bool = True,
                  recorded_workspace: torch.Tensor | None = None):
    """Gradients of the batched warp: ``(grad_src or None, grad_mv or None)``.

    ``recorded_workspace``: the workspace a recording forward
    (``exw_warp_forward_batched_record``) filled for this motion and these
    phases; the adjoint then skips its footprint pass.
    """
    grad_out = grad_out.contiguous()
    n, k, c, h, w = grad_out.shape
    dev = grad_out.device
    gs = torch.empty((n, c, h, w), dtype=grad_out.dtype, device=dev) if need_src else None
    gm = torch.empty((n, 2, h, w), dtype=torch.float32, device=dev) if need_mv else None
    ws = recorded_workspace
    if need_src and ws is None:
        nbytes = exw_warp_backward_workspace_bytes(grad_out.dtype, n, c, h, w)
        if nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    exw_warp_backward_batched(src.contiguous() if need_mv else None, mv.contiguous(), phases,
                              grad_out, gs, gm, ws, recorded=recorded_workspace is not None)
    return gs, gm


class WarpFunction(torch.autograd.Function):
    """Differentiable warp: ``out = WarpFunction.apply(src, mv, phases)``.

    Gradients flow to ``src`` (the frames) and ``mv`` (the motion vectors);
    the phases and the validity mask are not differentiated.
    """

    @staticmethod
    def forward(ctx, src, mv, phases):
        phases = tuple(float(s) for s in phases)
        src, mv = src.contiguous(), mv.contiguous()
        n, c, h, w = src.shape
        out = torch.empty((n, len(phases), c, h, w), dtype=src.dtype, device=src.device)
        ctx.ws = None
        if ctx.needs_input_grad[0]:
            # the image gradient will be needed: the forward also records the
            # adjoint's footprint, and the backward skips that pass (the
            # workspace, which for 16-bit frames includes the adjoint's float32
            # accumulator, is held from here to the backward)
            nbytes = exw_warp_backward_workspace_bytes(src.dtype, n, c, h, w)
            ctx.ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=src.device)
            exw_warp_forward_batched_record(src, mv, phases, out, ctx.ws)
        else:
            exw_warp_forward_batched(src, mv, phases, out)
        ctx.phases = phases
        ctx.save_for_backward(src, mv)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        src, mv = ctx.saved_tensors
        need_src, need_mv = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_src or need_mv):
            return None, None, None
        gs, gm = warp_backward(src, mv, ctx.phases, grad_out.to(src.dtype),
                               need_src=need_src, need_mv=need_mv,
                               recorded_workspace=ctx.ws if need_src else None)
        return gs, gm, None


def warp_differentiable(src, mv, phases=(1.0,)):
    return WarpFunction.apply(src, mv, tuple(phases))


def motion_stats(mv: torch.Tensor) -> torch.Tensor:
    """Per-frame ``(mean_x, var_x, mean_y, var_y)`` of ``mv`` [N,2,H,W] as a
    float64 [N,4] device tensor (population variance over all pixels)."""
    mv = mv.contiguous()
    n, _, h, w = mv.shape
    stats = torch.empty((n, 4), dtype=torch.float64, device=mv.device)
    nbytes = exw_motion_stats_workspace_bytes(n, h, w)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=mv.device)
    exw_motion_stats(mv, stats, ws)
    return stats


def buffer_emd(cur: torch.Tensor, prev: torch.Tensor, lo: float, hi: float,
               bins: int = 256) -> torch.Tensor:
    """Per-frame, per-channel EMD between buffers ``cur`` (of F_t) and ``prev``
    (of F_t-1), both [N,C,H,W] of one dtype, over ``bins`` histogram bins on
    [lo, hi]: a float64 [N,C] device tensor. The state feature of a buffer
    (EMD_{W_N}, EMD_{W_P}) is its sum over channels."""
    cur = cur.contiguous()
    prev = prev.contiguous()
    n, c = cur.shape[:2]
    emd = torch.empty((n, c), dtype=torch.float64, device=cur.device)
    nbytes = exw_buffer_emd_workspace_bytes(n, c, bins)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=cur.device)
    exw_buffer_emd(cur, prev, lo, hi, bins, emd, ws)
    return emd


def dynamic_objects(stencil: torch.Tensor, connectivity: int = 8) -> torch.Tensor:
    """N_D of every frame: the number of connected components of the marked
    (non-zero) pixels of the custom stencil ``stencil`` [N,H,W] uint8, as an
    int32 [N] device tensor."""
    stencil = stencil.contiguous()
    n, h, w = stencil.shape
    count = torch.empty((n,), dtype=torch.int32, device=stencil.device)
    nbytes = exw_dynamic_objects_workspace_bytes(n, h, w)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=stencil.device)
    exw_dynamic_objects(stencil, count, ws, connectivity)
    return count


def frame_quality(pred: torch.Tensor, truth: torch.Tensor, peak: float = 1.0) -> torch.Tensor:
    """Per-frame ``(MSE, PSNR, SSIM)`` of ``pred`` against ``truth``, both
    [..., C, H, W] of one dtype, as a float64 [..., 3] device tensor."""
    if pred.shape != truth.shape or pred.dim() < 3:
        raise ValueError("pred and truth must both be [..., C, H, W] of one shape")
    lead = pred.shape[:-3]
    c, h, w = pred.shape[-3:]
    p = pred.contiguous().reshape(-1, c, h, w)
    t = truth.contiguous().reshape(-1, c, h, w)
    q = torch.empty((p.shape[0], 3), dtype=torch.float64, device=pred.device)
    nbytes = exw_frame_quality_workspace_bytes(p.shape[0], c, h, w)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=pred.device)
    exw_frame_quality(p, t, q, ws, peak)
    return q.reshape(*lead, 3)


def warp_chain(src: torch.Tensor, mv: torch.Tensor, phase: float = 0.25, steps: int = 3, *,
               return_mask: bool = False, return_count: bool = False):
    """Chained warps ``out[i] = W(out[i-1], phase)``, ``out[0] = W(src, phase)``:
    ``out`` [S,N,C,H,W] (+ ``mask`` [S,N,H,W], ``invalid_count`` [S,N])."""
    src = src.contiguous()
    mv = mv.contiguous()
    n, c, h, w = src.shape
    out = torch.empty((steps, n, c, h, w), dtype=src.dtype, device=src.device)
    mask = (torch.empty((steps, n, h, w), dtype=torch.uint8, device=src.device)
            if return_mask else None)
    cnt = torch.empty((steps, n), dtype=torch.int32, device=src.device) if return_count else None
    exw_warp_chain(src, mv, phase, steps, out, mask, cnt)
    res = [out] + ([mask] if return_mask else []) + ([cnt] if return_count else [])
    return res[0] if len(res) == 1 else tuple(res)


_KINDS = {0: "repeat", 1: "warp", 2: "extrapolate"}
_SOURCES = {0: "F", 1: "P1", 2: "P2"}
WARP, EXTRAPOLATE, NONE = 0, 1, -1


def plan(d1: int, d2, d_last: int) -> dict:
    """The frames shown for decisions (d1, d2, d_last) (§IV-B, Table V):
    ``{"scenario": "S1".."S6", "P1": (kind, source), "P2": ..., "P3": ...,
    "nodes": (...), "new_frames": n}``."""
    p = exw_decision_plan(d1, NONE if d2 is None else d2, d_last)
    out = {"scenario": f"S{p.scenario}", "new_frames": p.new_frames,
           "nodes": tuple(None if v == 0 else v for v in p.node)}
    for i in range(3):
        out[f"P{i + 1}"] = (_KINDS[p.kind[i]], _SOURCES[p.source[i]])
    return out


def threshold_policy(motion_stats, invalid_fraction, max_variance: float, max_invalid: float):
    """Decisions ``(d1, d2 or None, d_last)`` of the fixed policy for one frame."""
    d1, d2, d3 = exw_threshold_policy(motion_stats, invalid_fraction, max_variance, max_invalid)
    return d1, (None if d2 == NONE else d2), d3


def decision_path_frames(src: torch.Tensor, mv: torch.Tensor, path: dict, extrapolate=None):
    """Make the frames P1, P2, P3 of a decision path (a ``plan`` result) on the
    GPU: warps are the forward warp at phase 1/4 with the motion of ``src``;
    ``extrapolate(frame) -> frame`` makes extrapolated frames (the paper's
    extrapolation network is not part of this library; without it those
    frames are None). Returns ``[P1, P2, P3]``, each [N,C,H,W] or None."""
    made = {"F": src}
    frames = []
    for i in range(3):
        kind, source = path[f"P{i + 1}"]
        base = made[source]
        if kind == "repeat":
            f = base
        elif kind == "warp":
            f = None if base is None else warp(base, mv, (0.25,))[:, 0]
        else:
            f = None if (extrapolate is None or base is None) else extrapolate(base)
        made[f"P{i + 1}"] = f
        frames.append(f)
    return frames


__all__ = ["ExwError", "warp", "warp_backward", "WarpFunction", "warp_differentiable",
           "motion_stats", "frame_quality", "warp_chain", "plan", "threshold_policy",
           "decision_path_frames", "exw_warp_forward", "exw_warp_forward_batched",
           "exw_warp_forward_batched_record", "exw_warp_backward", "exw_warp_backward_batched",
           "exw_warp_backward_batched_recorded", "exw_warp_backward_workspace_bytes",
           "exw_motion_stats",
           "exw_motion_stats_workspace_bytes", "exw_frame_quality",
           "exw_frame_quality_workspace_bytes", "exw_warp_chain", "exw_decision_plan",
           "exw_threshold_policy", "exw_stream_copy", "exw_stream_read", "exw_stream_write",
           "exw_motion_stats_no_alloc", "exw_buffer_emd", "exw_buffer_emd_workspace_bytes",
           "buffer_emd", "exw_dynamic_objects", "exw_dynamic_objects_workspace_bytes",
           "dynamic_objects"]
