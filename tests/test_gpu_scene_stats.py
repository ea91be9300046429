"""Per-frame motion statistics on the GPU, through the C-ABI, against the oracle.

Tolerance: the kernel folds (count, mean, M2) in float64 through about thirty
levels (chunks, lanes, wavefronts, workgroups), each contributing a few ulp,
so the mean is within 1e-12 of the mean absolute value and the variance
within 1e-11 relative of the correctly rounded two-pass oracle.
"""

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from oracle import scene_stats
from synth import make_config
from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu

MEAN_TOL = 1e-12
VAR_TOL = 1e-11


def gpu_stats(mv: np.ndarray, dev) -> np.ndarray:
    m = torch.from_numpy(np.ascontiguousarray(mv, dtype=np.float32)).to(dev)
    out = exw.motion_stats(m)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def assert_stats(got: np.ndarray, mv: np.ndarray, what: str) -> None:
    ref = scene_stats.motion_stats(mv)
    scale = np.abs(mv.astype(np.float64)).reshape(mv.shape[0], 2, -1).mean(axis=2)
    for comp in range(2):
        em = np.abs(got[:, 2 * comp] - ref[:, 2 * comp])
        assert (em <= MEAN_TOL * np.maximum(scale[:, comp], 1e-300)).all(), (what, comp, em)
        ev = np.abs(got[:, 2 * comp + 1] - ref[:, 2 * comp + 1])
        assert (ev <= VAR_TOL * ref[:, 2 * comp + 1]).all(), (what, comp, ev, ref[:, 2 * comp + 1])


SMALL = {1: dict(), 2: dict(n=2, h=75, w=131), 3: dict(n=2, h=90, w=200),
         4: dict(n=2, h=70, w=97), 5: dict(n=1, h=61, w=107)}


@pytest.mark.parametrize("index", sorted(SMALL))
def test_stats_match_oracle_small(index):
    dev = need_gpu()
    d = make_config(index, **SMALL[index])
    announce("motion stats", index, d["mv"].shape)
    assert_stats(gpu_stats(d["mv"], dev), d["mv"], f"workload {index}")


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 1, 7), (2, 32, 64), (1, 2048, 1), (1, 1, 2049),
                                   (2, 45, 46), (1, 517, 1031)])
def test_stats_ragged_shapes(shape):
    dev = need_gpu()
    n, h, w = shape
    mv = np.random.default_rng(h * 7 + w).normal(1.5, 3.0, (n, 2, h, w)).astype(np.float32)
    announce("motion stats ragged", shape)
    assert_stats(gpu_stats(mv, dev), mv, f"shape {shape}")


def test_stats_full_size_workload_2():
    dev = need_gpu()
    d = make_config(2)
    announce("motion stats full size", d["mv"].shape)
    assert_stats(gpu_stats(d["mv"], dev), d["mv"], "workload 2")


def test_stats_many_passes_per_workgroup():
    # 2160 x 3840 = 8.3 M pixels: 4050 passes of 2048 over 256 workgroups
    dev = need_gpu()
    mv = np.random.default_rng(5).uniform(-40, 40, (2, 2, 2160, 3840)).astype(np.float32)
    announce("motion stats 4K", mv.shape)
    assert_stats(gpu_stats(mv, dev), mv, "4K")


def test_stats_constant_field_is_exact_and_large_offset_does_not_cancel():
    dev = need_gpu()
    const = np.full((2, 2, 33, 70), 7.125, dtype=np.float32)
    announce("motion stats constant")
    got = gpu_stats(const, dev)
    assert (got[:, [0, 2]] == 7.125).all() and (got[:, [1, 3]] == 0.0).all()
    rng = np.random.default_rng(6)
    off = (4096.0 + np.round(rng.normal(0, 1, (2, 2, 100, 300)) * 64) / 64).astype(np.float32)
    announce("motion stats offset")
    assert_stats(gpu_stats(off, dev), off, "offset 4096")


def test_stats_reproducible_and_nonfinite():
    dev = need_gpu()
    d = make_config(2, n=2, h=200, w=300)
    announce("motion stats reproducible")
    a, b = gpu_stats(d["mv"], dev), gpu_stats(d["mv"], dev)
    assert np.array_equal(a, b)
    mv = d["mv"].copy()
    mv[1, 0, 10, 10] = np.nan
    announce("motion stats nan")
    got = gpu_stats(mv, dev)
    assert np.isnan(got[1, 0]) and np.isnan(got[1, 1])
    assert np.isfinite(got[1, 2:]).all() and np.isfinite(got[0]).all()
    assert np.array_equal(got[0], a[0])


def test_stats_empty_batch_and_binding_checks():
    dev = need_gpu()
    announce("motion stats empty")
    out = exw.motion_stats(torch.zeros((0, 2, 4, 4), device=dev))
    assert out.shape == (0, 4)
    with pytest.raises(ValueError):
        exw.exw_motion_stats(torch.zeros((1, 2, 4, 4), device=dev, dtype=torch.float64),
                             torch.empty((1, 4), device=dev, dtype=torch.float64))
    with pytest.raises(ValueError):
        exw.exw_motion_stats(torch.zeros((1, 2, 4, 4), device=dev),
                             torch.empty((1, 4), device=dev, dtype=torch.float32))


# ------------------------------------------ statistics from the recording forward

def record_stats(mv: np.ndarray, c: int, dev, dtype=torch.float32, phases=(0.25, 0.75)):
    """The recording forward with motion_stats: (stats, out, ws, plain out, plain ws)."""
    n, _, h, w = mv.shape
    src = torch.from_numpy(np.random.default_rng(h + w + c).random((n, c, h, w),
                                                                    dtype=np.float32)).to(dev).to(dtype)
    m = torch.from_numpy(np.ascontiguousarray(mv, dtype=np.float32)).to(dev)
    k = len(phases)
    nbytes = exw.exw_warp_backward_workspace_bytes(dtype, n, c, h, w)
    outs, wss = [], []
    stats = torch.full((n, 4), float("nan"), dtype=torch.float64, device=dev)
    for with_stats in (True, False):
        out = torch.empty((n, k, c, h, w), dtype=dtype, device=dev)
        ws = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        exw.exw_warp_forward_batched_record(src, m, phases, out, ws,
                                            motion_stats=stats if with_stats else None)
        outs.append(out)
        wss.append(ws)
    torch.cuda.synchronize()
    return stats.cpu().numpy(), outs, wss


def footprint_bytes(ws, n, h, w):
    seg = 32 * n * h * ((w + 63) // 64)
    info = (seg + 255) // 256 * 256
    host = ws.cpu().numpy()
    return np.concatenate([host[:seg], host[info:info + 8 * n]])


@pytest.mark.parametrize("index", sorted(SMALL))
def test_recording_forward_stats_match_oracle(index):
    """The statistics the recording forward folds from its own motion read
    equal the oracle's within the statistics pass's tolerances, and asking for
    them changes neither the forward's outputs nor its footprint records."""
    dev = need_gpu()
    d = make_config(index, **SMALL[index])
    mv = d["mv"]
    n, _, h, w = mv.shape
    c = d["src"].shape[1]
    announce("recording forward statistics", index, mv.shape, c)
    got, outs, wss = record_stats(mv, c, dev)
    assert_stats(got, mv, f"recording forward, workload {index}")
    assert torch.equal(outs[0], outs[1])
    assert np.array_equal(footprint_bytes(wss[0], n, h, w), footprint_bytes(wss[1], n, h, w))


@pytest.mark.parametrize("c,shape", [(4, (1, 1, 1)), (4, (3, 1, 7)), (3, (2, 5, 129)),
                                     (1, (1, 2048, 2)), (12, (1, 7, 300)), (4, (2, 45, 46)),
                                     (4, (1, 517, 1031)),
                                     (2, (2, 33, 70)),    # plain forward + statistics pass
                                     (3, (2, 40, 1))])    # width 1: plain forward
def test_recording_forward_stats_shapes(c, shape):
    dev = need_gpu()
    n, h, w = shape
    mv = np.random.default_rng(h * 5 + w).normal(1.5, 3.0, (n, 2, h, w)).astype(np.float32)
    announce("recording forward statistics", c, shape)
    got, outs, _ = record_stats(mv, c, dev)
    assert_stats(got, mv, f"recording forward c={c} {shape}")
    assert torch.equal(outs[0], outs[1])


def test_recording_forward_stats_large_mean_constant_and_nonfinite():
    dev = need_gpu()
    rng = np.random.default_rng(12)
    # a mean large against the spread (no cancellation), a constant frame
    mv = np.empty((4, 2, 37, 301), np.float32)
    mv[0] = 1.0e4 + rng.normal(0.0, 0.01, (2, 37, 301))
    mv[1] = -2.5
    mv[2] = rng.normal(0.0, 1.0, (2, 37, 301))
    mv[2, 0, 17, 200] = np.nan
    mv[2, 1, 3, 3] = np.inf
    # one outlier far from the first tile, tiny spread about a large mean
    mv[3, 0] = 0.0
    mv[3, 0, 30, 250] = 1.0e6
    mv[3, 1] = 5.0e3 + rng.normal(0.0, 1.0e-3, (37, 301))
    announce("recording forward statistics: large mean, constant, outlier, non-finite")
    got, _, _ = record_stats(mv, 4, dev, dtype=torch.float16)
    finite = [0, 1, 3]
    assert_stats(got[finite], mv[finite], "large mean / constant / outlier")
    assert got[1, 1] == 0.0 and got[1, 3] == 0.0 and got[1, 0] == -2.5
    assert not np.isfinite(got[2, 0]) and not np.isfinite(got[2, 1])
    assert not np.isfinite(got[2, 2]) and not np.isfinite(got[2, 3])


def test_recording_forward_stats_full_size():
    dev = need_gpu()
    d = make_config(2)
    announce("recording forward statistics, full size", d["mv"].shape)
    got, _, _ = record_stats(d["mv"], 4, dev, phases=(0.25, 0.5, 0.75))
    assert_stats(got, d["mv"], "recording forward, workload 2 full size")
