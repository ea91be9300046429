"""Seeded frame and motion-vector generators.

The paper evaluates on Unreal Engine scenes (Table I: 480p to 1080p game
frames with a moving camera and dynamically moving objects, paper §III-A and
§III-D). Those scenes are not available here, so these generators draw
stand-ins with the same structure:

* ``SinTexture``: a smooth colour texture, ``clip(0.5 + sum of 8 random 2-D
  sinusoids, 0, 1)`` per channel.
* ``random_field_frames``: independent textured frames with i.i.d. uniform
  per-pixel motion vectors (a stress test for the gather, no scene
  structure).
* ``pan_rect_sequence``: a camera pan with a constant sub-pixel offset per
  frame plus axis-aligned textured rectangles that each move with their own
  velocity (the "dynamic objects" of paper §III-D). The motion vector of a
  pixel is the velocity of the topmost surface there, in pixels per rendered
  frame, +x right and +y down.

Everything is drawn from ``numpy.random.default_rng(seed)`` and evaluated in
float64, then stored as float32. Nothing here resamples a frame through a
motion field: the warp itself lives elsewhere.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

N_WAVES = 8


class SinTexture:
    """``clip(0.5 + sum_k a_k sin(2 pi (f_k . (x, y)) + phi_k), 0, 1)`` per channel.

    ``a_k ~ U(0.05, 0.25)``, ``|f_k| ~ U(1/128, 1/8)`` cycles per pixel in a
    uniformly random direction, ``phi_k ~ U(0, 2 pi)``.
    """

    def __init__(self, rng: np.random.Generator, channels: int, n_waves: int = N_WAVES):
        self.channels = channels
        shape = (channels, n_waves)
        self.amp = rng.uniform(0.05, 0.25, size=shape)
        mag = rng.uniform(1.0 / 128.0, 1.0 / 8.0, size=shape)
        ang = rng.uniform(0.0, 2.0 * math.pi, size=shape)
        self.fx = mag * np.cos(ang)
        self.fy = mag * np.sin(ang)
        self.phi = rng.uniform(0.0, 2.0 * math.pi, size=shape)

    def eval(self, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
        """Evaluate on the grid ``ys x xs`` (1-D float64 arrays) -> [C, H, W] float64.

        Uses sin(a + b) = sin(a) cos(b) + cos(a) sin(b) so that each channel is
        one small [H, 2K] @ [2K, W] product instead of K full-grid sines.
        """
        xs = np.asarray(xs, dtype=np.float64)
        ys = np.asarray(ys, dtype=np.float64)
        out = np.empty((self.channels, ys.size, xs.size), dtype=np.float64)
        two_pi = 2.0 * math.pi
        for c in range(self.channels):
            ax = two_pi * np.outer(self.fx[c], xs) + self.phi[c][:, None]  # [K, W]
            by = two_pi * np.outer(ys, self.fy[c])  # [H, K]
            left = np.concatenate([np.cos(by), np.sin(by)], axis=1) * np.concatenate(
                [self.amp[c], self.amp[c]])[None, :]
            right = np.concatenate([np.sin(ax), np.cos(ax)], axis=0)
            np.matmul(left, right, out=out[c])
            out[c] += 0.5
        np.clip(out, 0.0, 1.0, out=out)
        return out


def random_field_frames(rng: np.random.Generator, n: int, c: int, h: int, w: int,
                        mv_range: float = 4.0):
    """Independent textured frames with i.i.d. ``U(-mv_range, mv_range)`` motion vectors.

    Returns ``(frames [n, c, h, w] float32, mv [n, 2, h, w] float32)``.
    """
    frames = np.empty((n, c, h, w), dtype=np.float32)
    xs = np.arange(w, dtype=np.float64)
    ys = np.arange(h, dtype=np.float64)
    for i in range(n):
        frames[i] = SinTexture(rng, c).eval(xs, ys)
    mv = rng.uniform(-mv_range, mv_range, size=(n, 2, h, w)).astype(np.float32)
    return frames, mv


# ---------------------------------------------------------------- pan + rects

GBUFFER_CHANNELS = ("color_r", "color_g", "color_b", "depth", "normal_x", "normal_y",
                    "normal_z", "albedo_r", "albedo_g", "albedo_b", "roughness", "metallic")


class _Surface:
    """One rigid surface: the background or one rectangle."""

    def __init__(self, rng: np.random.Generator, kind: str, background: bool):
        self.kind = kind
        if kind == "gbuffer":
            self.tex = SinTexture(rng, 10)
            self.depth_base = 0.95 if background else rng.uniform(0.1, 0.9)
            self.depth_slope = rng.uniform(-2e-4, 2e-4, size=2)
            self.rough_base = rng.uniform(0.0, 1.0)
            self.metal_base = rng.uniform(0.0, 1.0)
        else:
            self.tex = SinTexture(rng, 4 if kind == "rgba" else 3)

    @property
    def channels(self) -> int:
        return 12 if self.kind == "gbuffer" else self.tex.channels

    def eval(self, lx: np.ndarray, ly: np.ndarray) -> np.ndarray:
        """Surface attributes at local coordinates -> [C, len(ly), len(lx)] float64."""
        t = self.tex.eval(lx, ly)
        if self.kind != "gbuffer":
            return t
        out = np.empty((12, ly.size, lx.size), dtype=np.float64)
        out[0:3] = t[0:3]
        depth = (self.depth_base + self.depth_slope[0] * lx[None, :]
                 + self.depth_slope[1] * ly[:, None])
        out[3] = np.clip(depth, 0.0, 1.0)
        a = 0.3 * (2.0 * t[3] - 1.0)
        b = 0.3 * (2.0 * t[4] - 1.0)
        norm = np.sqrt(a * a + b * b + 1.0)
        out[4] = a / norm
        out[5] = b / norm
        out[6] = 1.0 / norm
        out[7:10] = 0.8 * t[5:8]
        out[10] = np.clip(self.rough_base + 0.05 * t[8], 0.0, 1.0)
        out[11] = np.clip(self.metal_base + 0.05 * t[9], 0.0, 1.0)
        return out


def pan_rect_sequence(rng: np.random.Generator, n: int, h: int, w: int, *, kind: str = "rgba",
                      n_rects: int = 16, vmax: float = 32.0, pan_max: float = 3.0,
                      rect_size: Sequence[int] = (32, 256), pan: Optional[Sequence[float]] = None,
                      truth_phases: Optional[Sequence[float]] = None):
    """Camera pan plus moving rectangles; returns ``(frames, mv, info)``.

    * Pan ``(px, py) ~ U(-pan_max, pan_max)^2`` px per frame (or ``pan``):
      frame ``i`` shows the background texture at world coordinate
      ``(x - i*px, y - i*py)``, so background content moves by ``(px, py)``.
    * ``n_rects`` rectangles with integer sizes drawn from ``rect_size``
      (clipped to the frame), top-left uniform over the frame, velocity
      ``~ U(-vmax, vmax)^2`` px per frame, each with its own rigidly attached
      texture; painted in index order at ``top_left + i * velocity``.
    * ``mv[i, :, y, x]`` is the velocity of the topmost surface at ``(x, y)``.

    ``kind`` is ``"rgb"`` (3 channels), ``"rgba"`` (4) or ``"gbuffer"`` (12,
    in the order of ``GBUFFER_CHANNELS``). With ``truth_phases``, ``info["truth"]``
    [N, K, C, H, W] holds the scene rendered at times ``i + s`` (the ground
    truth of the frames predicted between rendered frames).
    """
    if pan is None:
        pan = rng.uniform(-pan_max, pan_max, size=2)
    pan = np.asarray(pan, dtype=np.float64)
    bg = _Surface(rng, kind, background=True)
    rects = []
    for _ in range(n_rects):
        rw = int(min(max(rng.integers(rect_size[0], rect_size[1] + 1), 1), w))
        rh = int(min(max(rng.integers(rect_size[0], rect_size[1] + 1), 1), h))
        x0 = rng.uniform(0.0, float(w - rw))
        y0 = rng.uniform(0.0, float(h - rh))
        vel = rng.uniform(-vmax, vmax, size=2)
        rects.append((rw, rh, x0, y0, vel, _Surface(rng, kind, background=False)))

    c = bg.channels
    xs = np.arange(w, dtype=np.float64)
    ys = np.arange(h, dtype=np.float64)

    def render(t: float, stencil=None):
        # the scene at time t (in rendered-frame intervals): image and motion;
        # with `stencil` [H, W] u8, also the custom stencil (1 where a moving
        # rectangle is the topmost surface, 0 on the background)
        frame = bg.eval(xs - t * pan[0], ys - t * pan[1])
        motion = np.empty((2, h, w), dtype=np.float32)
        motion[0] = np.float32(pan[0])
        motion[1] = np.float32(pan[1])
        if stencil is not None:
            stencil[...] = 0
        for rw, rh, rx, ry, vel, surf in rects:
            left = rx + t * vel[0]
            top = ry + t * vel[1]
            xa, xb = max(0, math.ceil(left)), min(w, math.ceil(left + rw))
            ya, yb = max(0, math.ceil(top)), min(h, math.ceil(top + rh))
            if xa >= xb or ya >= yb:
                continue
            frame[:, ya:yb, xa:xb] = surf.eval(xs[xa:xb] - left, ys[ya:yb] - top)
            motion[0, ya:yb, xa:xb] = np.float32(vel[0])
            motion[1, ya:yb, xa:xb] = np.float32(vel[1])
            if stencil is not None:
                stencil[ya:yb, xa:xb] = 1
        return frame, motion

    frames = np.empty((n, c, h, w), dtype=np.float32)
    mv = np.empty((n, 2, h, w), dtype=np.float32)
    stencil = np.empty((n, h, w), dtype=np.uint8)
    for i in range(n):
        frames[i], mv[i] = render(float(i), stencil[i])
    info = {"pan": pan.tolist(), "n_rects": n_rects, "vmax": vmax,
            "velocities": [r[4].tolist() for r in rects], "stencil": stencil}
    if truth_phases is not None:
        # the exact scene between rendered frames: what a perfect predictor shows
        truth = np.empty((n, len(truth_phases), c, h, w), dtype=np.float32)
        for i in range(n):
            for k, s in enumerate(truth_phases):
                truth[i, k] = render(i + float(s))[0]
        info["truth"] = truth
    return frames, mv, info


# ----------------------------------------------------------- named workloads

@dataclasses.dataclass(frozen=True)
class ConfigSpec:
    index: int
    name: str
    generator: str  # "field" or "pan_rect"
    n: int
    c: int
    h: int
    w: int
    phases: tuple
    storage: tuple  # storage dtypes exercised: "f32", "f16", "bf16"
    kind: str = "rgb"
    n_rects: int = 0
    vmax: float = 0.0
    mv_range: float = 4.0
    delta_std: float = 0.0  # std of the motion perturbation of the L2 target
    grads: bool = False


QUARTERS = (0.25, 0.5, 0.75)

CONFIGS = {
    1: ConfigSpec(1, "256x256 RGB fp32, i.i.d. U(-4,4) motion", "field", 1, 3, 256, 256,
                  (1.0,), ("f32",)),
    2: ConfigSpec(2, "1080p RGBA, 8 frames, pan + 16 rectangles (|v|<=32), 3 phases",
                  "pan_rect", 8, 4, 1080, 1920, QUARTERS, ("f32", "f16"), kind="rgba",
                  n_rects=16, vmax=32.0),
    3: ConfigSpec(3, "4K RGBA, 8 frames, pan + 16 rectangles (|v|<=32), 3 phases",
                  "pan_rect", 8, 4, 2160, 3840, QUARTERS, ("f32", "f16"), kind="rgba",
                  n_rects=16, vmax=32.0),
    4: ConfigSpec(4, "8 x 1080p RGB fp32, i.i.d. U(-4,4) motion, L2 loss vs perturbed warp",
                  "field", 8, 3, 1080, 1920, (1.0,), ("f32",), delta_std=0.5, grads=True),
    5: ConfigSpec(5, "4 x 1440p 12-channel G-buffer, pan + 32 rectangles (|v|<=48)",
                  "pan_rect", 4, 12, 1440, 2560, (1.0,), ("bf16", "f32"), kind="gbuffer",
                  n_rects=32, vmax=48.0, delta_std=0.5, grads=True),
}


def make_config(index: int, *, n: Optional[int] = None, h: Optional[int] = None,
                w: Optional[int] = None, seed: Optional[int] = None,
                with_truth: bool = False) -> dict:
    """Draw the inputs of workload ``index`` (1..5), optionally at a reduced size.

    Returns a dict with ``src`` [N,C,H,W] float32, ``mv`` [N,2,H,W] float32,
    ``phases`` [K] float32, ``delta`` [N,2,H,W] float32 or None (the motion
    perturbation of the L2 target), ``truth`` [N,K,C,H,W] float32 (the scene
    at times n + phase, pan-and-rectangle workloads with ``with_truth``) or
    None, ``stencil`` [N,H,W] uint8 (the custom stencil of the
    pan-and-rectangle workloads: 1 on moving rectangles, 0 on the
    background) or None, plus the spec. The default seed is
    ``1000 + index``. At a reduced size rectangle sizes shrink with the frame,
    velocities do not.
    """
    spec = CONFIGS[index]
    n = spec.n if n is None else n
    h = spec.h if h is None else h
    w = spec.w if w is None else w
    rng = np.random.default_rng(1000 + index if seed is None else seed)
    info = {}
    if spec.generator == "field":
        src, mv = random_field_frames(rng, n, spec.c, h, w, spec.mv_range)
    else:
        scale = min(1.0, h / spec.h, w / spec.w)
        lo = max(4, int(round(32 * scale)))
        hi = max(lo, int(round(256 * scale)))
        src, mv, info = pan_rect_sequence(rng, n, h, w, kind=spec.kind, n_rects=spec.n_rects,
                                          vmax=spec.vmax, rect_size=(lo, hi),
                                          truth_phases=spec.phases if with_truth else None)
    delta = None
    if spec.delta_std > 0:
        delta = rng.normal(0.0, spec.delta_std, size=mv.shape).astype(np.float32)
    truth = info.pop("truth", None)
    stencil = info.pop("stencil", None)
    return {"spec": spec, "src": src, "mv": mv, "phases": np.asarray(spec.phases, np.float32),
            "delta": delta, "info": info, "truth": truth, "stencil": stencil}


def quantize(x: np.ndarray, dtype: str) -> np.ndarray:
    """Round float32 values to a storage dtype (RNE) and return them as float32."""
    if dtype == "f32":
        return np.asarray(x, dtype=np.float32)
    if dtype == "f16":
        return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)
    if dtype == "bf16":
        import torch
        t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32))
        return t.to(torch.bfloat16).to(torch.float32).numpy()
    raise ValueError(f"unknown storage dtype {dtype!r}")


def upstream_gradient(seed: int, shape) -> np.ndarray:
    """A stand-in for dL/d out: i.i.d. uniform values in [-1, 1), float32.

    Drawn per frame from its own seed, so that any frame of a batch can be
    drawn again on its own (uniform rather than normal: four times cheaper to
    draw at the size of a 4K batch).
    """
    rng = np.random.default_rng(seed)
    g = rng.random(size=tuple(shape), dtype=np.float32)
    g *= 2.0
    g -= 1.0
    return g


# World position of the G-buffer scene: a pinhole camera of focal length W px
# looks down +z; a pixel's view depth is near + depth * (far - near) (depth =
# G-buffer channel 3); the camera moves with the pan, so that a point of the
# background keeps its world position from frame to frame.
WORLD_NEAR, WORLD_FAR = 1.0, 100.0


def world_position(depth: np.ndarray, pan, frame0: int = 0) -> np.ndarray:
    """World-position buffer [N, 3, H, W] float32 (x, y, z) of frames
    frame0 .. frame0 + N - 1 from their depth channel [N, H, W] and the
    sequence's camera pan (px per frame)."""
    depth = np.asarray(depth, dtype=np.float64)
    n, h, w = depth.shape
    f = float(w)
    z = WORLD_NEAR + depth * (WORLD_FAR - WORLD_NEAR)
    z_bg = WORLD_NEAR + 0.95 * (WORLD_FAR - WORLD_NEAR)  # the background's depth
    xs = np.arange(w, dtype=np.float64)[None, None, :] - w / 2.0
    ys = np.arange(h, dtype=np.float64)[None, :, None] - h / 2.0
    t = (frame0 + np.arange(n, dtype=np.float64))[:, None, None]
    cam_x = -t * float(pan[0]) * z_bg / f
    cam_y = -t * float(pan[1]) * z_bg / f
    out = np.empty((n, 3, h, w), dtype=np.float32)
    out[:, 0] = xs * z / f + cam_x
    out[:, 1] = ys * z / f + cam_y
    out[:, 2] = z
    return out
