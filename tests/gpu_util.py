"""Helpers shared by the GPU parity tests (not collected by pytest)."""

from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

TORCH_DT = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
MANTISSA_BITS = {"f32": 23, "f16": 10, "bf16": 7}

# Forward tolerance against the float64 oracle on the same stored inputs.
FWD_TOL_F32 = 1e-5
# End-to-end forward tolerance against the oracle on the float32 original frames.
E2E_TOL = {"f32": 1e-5, "f16": 1e-3, "bf16": 4e-3}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch.device("cuda:0")


def announce(*parts) -> None:
    """Name the case on stdout before a GPU step, so a fault leaves a trace."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray, dtype: str, device) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device).to(TORCH_DT[dtype])


def stored(a: np.ndarray, dtype: str) -> np.ndarray:
    """The values a storage dtype holds for float32 input (RNE), as float64."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(
        TORCH_DT[dtype]).to(torch.float64).numpy()


def to_host(t: torch.Tensor) -> np.ndarray:
    return t.detach().to(torch.float64).cpu().numpy()


def half_ulp(ref: np.ndarray, dtype: str) -> np.ndarray:
    """Half a unit in the last place of ``dtype`` at |ref| (normal range)."""
    mag = np.abs(ref)
    _, e = np.frexp(np.maximum(mag, 1e-30))
    return np.ldexp(0.5, e - 1 - MANTISSA_BITS[dtype])


def assert_close_kernel(gpu: np.ndarray, ref: np.ndarray, dtype: str, what: str) -> float:
    """GPU vs float64 oracle on the same stored inputs: float32 within 1e-5;
    f16/bf16 within half an ulp of the storage type plus the float32 blend error."""
    err = np.abs(gpu - ref)
    if dtype == "f32":
        bound = FWD_TOL_F32
        worst = float(err.max()) if err.size else 0.0
        assert worst <= bound, f"{what}: max err {worst} > {bound}"
        return worst
    bound = half_ulp(ref, dtype) + 1e-6 * np.maximum(1.0, np.abs(ref))
    bad = err > bound
    assert not bad.any(), (f"{what}: {int(bad.sum())} elements beyond half an ulp; worst "
                           f"{float(err.max())}")
    return float(err.max()) if err.size else 0.0


def rounding_band(mv: np.ndarray, phase: float, h: int, w: int) -> np.ndarray:
    """Pixels [.., H, W] where the float32 rounding of d = s*u (or s*v) can move
    the validity decision: an integer bound of the box test (x, x - (W-1); y,
    y - (H-1)) lies within half a float32 ulp of d of the exact d. Outside this
    band the exact and the float32-rounded displacement decide alike."""
    s32 = np.float32(phase)
    mvf = np.asarray(mv, np.float32)
    d32 = (s32 * mvf).astype(np.float32)
    dex = np.float64(s32) * mvf.astype(np.float64)
    with np.errstate(invalid="ignore"):
        half = np.abs(np.spacing(d32)).astype(np.float64) / 2
        xs = np.arange(w, dtype=np.float64)[None, :]
        ys = np.arange(h, dtype=np.float64)[:, None]
        bx, by = dex[..., 0, :, :], dex[..., 1, :, :]
        hx, hy = half[..., 0, :, :], half[..., 1, :, :]
        return ((np.abs(bx - xs) <= hx) | (np.abs(bx - (xs - (w - 1))) <= hx)
                | (np.abs(by - ys) <= hy) | (np.abs(by - (ys - (h - 1))) <= hy))


def compare_with_exact(gpu_out: np.ndarray, gpu_mask: np.ndarray, ex_out: np.ndarray,
                       ex_mask: np.ndarray, mv: np.ndarray, phases, dtype: str,
                       what: str) -> dict:
    """The GPU forward [N,K,C,H,W] against the oracle's exact mode (d = s*u in
    float64): mask mismatches only inside the rounding band, counted; values
    of pixels valid on both sides within 1e-5 (f32) or half an ulp of the
    storage type plus 1e-5 (f16/bf16). Returns the counts and the worst error."""
    n, k = gpu_mask.shape[:2]
    h, w = gpu_mask.shape[-2:]
    in_band = mismatches = 0
    worst = 0.0
    for j, s in enumerate(phases):
        band = rounding_band(mv, s, h, w)  # [N, H, W]
        diff = gpu_mask[:, j] != ex_mask[:, j]
        assert not (diff & ~band).any(), (
            f"{what}: {int((diff & ~band).sum())} mask mismatches outside the rounding band")
        mismatches += int(diff.sum())
        in_band += int(band.sum())
        both = (gpu_mask[:, j] == 1) & (ex_mask[:, j] == 1)
        err = np.abs(gpu_out[:, j] - ex_out[:, j]) * both[:, None]
        if dtype == "f32":
            bound = 1e-5
        else:
            bound = half_ulp(ex_out[:, j], dtype) + 1e-5
        assert (err <= bound).all(), f"{what}: phase {s} value error {float(err.max())} vs exact"
        worst = max(worst, float(err.max()) if err.size else 0.0)
    print(f"[exact-mode] {what}: band pixels {in_band}, mask mismatches in band "
          f"{mismatches}, max value error {worst:.3g}", flush=True)
    return {"band_pixels": in_band, "band_mismatches": mismatches, "max_abs_vs_exact": worst}
