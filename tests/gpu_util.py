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
