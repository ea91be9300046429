"""Per-frame MSE / PSNR / SSIM on the GPU, through the C-ABI, against the oracle.

Tolerance: every window sum, index and total is float64 on both sides; they
differ only in summation order (FFT convolution in the oracle, direct sums
in the kernel), so MSE agrees to 1e-12 relative, PSNR to 1e-9 dB and SSIM to
1e-11 absolute.
"""

import math

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from oracle import quality
from synth import make_config
from gpu_util import announce, need_gpu, stored, to_dev

pytestmark = pytest.mark.gpu


def gpu_quality(pred: np.ndarray, truth: np.ndarray, dtype: str, dev, peak=1.0) -> np.ndarray:
    p, t = to_dev(pred, dtype, dev), to_dev(truth, dtype, dev)
    q = exw.frame_quality(p, t, peak)
    torch.cuda.synchronize()
    return q.cpu().numpy()


def assert_quality(got: np.ndarray, pred: np.ndarray, truth: np.ndarray, dtype: str,
                   what: str, peak=1.0) -> None:
    ref = quality.frame_quality(stored(pred, dtype), stored(truth, dtype), peak)
    assert got.shape == ref.shape
    mse_err = np.abs(got[..., 0] - ref[..., 0])
    assert (mse_err <= 1e-12 * ref[..., 0]).all(), (what, mse_err, ref[..., 0])
    fin = np.isfinite(ref[..., 1])
    assert np.array_equal(np.isfinite(got[..., 1]), fin), what
    assert (np.abs(got[..., 1][fin] - ref[..., 1][fin]) <= 1e-9).all(), (what, got[..., 1], ref[..., 1])
    assert (np.abs(got[..., 2] - ref[..., 2]) <= 1e-11).all(), (what, got[..., 2], ref[..., 2])


@pytest.mark.parametrize("shape", [(2, 3, 40, 50), (1, 1, 11, 11), (1, 2, 11, 75), (1, 1, 77, 11),
                                   (2, 1, 76, 74), (1, 3, 77, 75), (1, 4, 143, 139)])
def test_quality_matches_oracle_ragged(shape):
    dev = need_gpu()
    rng = np.random.default_rng(sum(shape))
    truth = rng.random(shape).astype(np.float32)
    pred = np.clip(truth + rng.normal(0, 0.05, shape), 0, 1).astype(np.float32)
    announce("frame quality", shape)
    assert_quality(gpu_quality(pred, truth, "f32", dev), pred, truth, "f32", f"shape {shape}")


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_quality_16bit_storage(dtype):
    dev = need_gpu()
    rng = np.random.default_rng(7)
    truth = rng.random((2, 3, 60, 90)).astype(np.float32)
    pred = np.clip(truth + rng.normal(0, 0.1, truth.shape), 0, 1).astype(np.float32)
    announce("frame quality", dtype)
    assert_quality(gpu_quality(pred, truth, dtype, dev), pred, truth, dtype, dtype)


def test_quality_identical_frames_and_peak():
    dev = need_gpu()
    x = np.random.default_rng(8).random((2, 3, 30, 40)).astype(np.float32)
    announce("frame quality identical")
    q = gpu_quality(x, x, "f32", dev)
    assert (q[:, 0] == 0.0).all() and (q[:, 1] == math.inf).all() and (q[:, 2] == 1.0).all()
    y = np.clip(x + 0.03, 0, 1).astype(np.float32)
    announce("frame quality peak 255")
    q255 = gpu_quality(x * 255, y * 255, "f32", dev, peak=255.0)
    assert_quality(q255, x * 255, y * 255, "f32", "peak 255", peak=255.0)


def test_quality_of_warped_frames_against_the_analytic_scene():
    # P_i = W(F_t, i/4) against the scene rendered at t + i/4 (workload 2 generator)
    dev = need_gpu()
    d = make_config(2, n=2, h=270, w=480, with_truth=True)
    phases = [float(s) for s in d["phases"]]
    src = torch.from_numpy(d["src"]).to(dev)
    mv = torch.from_numpy(d["mv"]).to(dev)
    announce("frame quality of warped frames", d["truth"].shape)
    out = exw.warp(src, mv, phases)
    pred = out.cpu().numpy()
    q = gpu_quality(pred, d["truth"], "f32", dev)
    assert_quality(q, pred, d["truth"], "f32", "warped vs truth")
    # the prediction degrades with the distance from the rendered frame
    assert (q[:, 0, 1] > q[:, 2, 1]).all() and (q[:, 0, 2] > q[:, 2, 2]).all()


def test_quality_full_size_frames():
    dev = need_gpu()
    d = make_config(2, n=1, with_truth=True)
    phases = [float(s) for s in d["phases"]]
    out = exw.warp(torch.from_numpy(d["src"]).to(dev), torch.from_numpy(d["mv"]).to(dev), phases)
    announce("frame quality full size", d["truth"].shape)
    pred = out.cpu().numpy()
    q = gpu_quality(pred, d["truth"], "f32", dev)
    assert_quality(q, pred, d["truth"], "f32", "1080p")


def test_quality_reproducible_and_binding_checks():
    dev = need_gpu()
    rng = np.random.default_rng(9)
    x = torch.from_numpy(rng.random((3, 2, 50, 70)).astype(np.float32)).to(dev)
    y = torch.from_numpy(rng.random((3, 2, 50, 70)).astype(np.float32)).to(dev)
    announce("frame quality reproducible")
    a, b = exw.frame_quality(x, y), exw.frame_quality(x, y)
    assert torch.equal(a, b)
    with pytest.raises(ValueError):
        exw.frame_quality(x, y[:, :1])
    with pytest.raises(exw.ExwError):
        exw.frame_quality(x[..., :10, :], y[..., :10, :])
