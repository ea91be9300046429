"""EMD features (EMD_{W_N}, EMD_{W_P}) on the GPU, through the C-ABI, against the
float64 oracle. Counts are integers and the final value is the same float64
expression on both sides, so results must be equal bit for bit."""

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from oracle import buffer_emd
from synth import make_config, world_position
from gpu_util import TORCH_DT, announce, need_gpu, stored, to_dev

pytestmark = pytest.mark.gpu


def gpu_emd(cur, prev, lo, hi, bins, dtype, dev):
    c = to_dev(cur, dtype, dev)
    p = to_dev(prev, dtype, dev)
    out = exw.buffer_emd(c, p, lo, hi, bins)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_normals_and_positions_match_oracle(dtype):
    dev = need_gpu()
    d = make_config(5, n=4, h=90, w=171)
    g = d["src"]
    normals = g[:, 4:7]
    pos = world_position(g[:, 3], d["info"]["pan"])
    for what, buf, lo, hi, bins in (("normals", normals, -1.0, 1.0, 256),
                                    ("positions", pos, -64.0, 128.0, 1024)):
        announce("buffer EMD", what, dtype)
        cur, prev = buf[1:], buf[:-1]
        got = gpu_emd(cur, prev, lo, hi, bins, dtype, dev)
        ref = buffer_emd.buffer_emd(stored(cur, dtype), stored(prev, dtype), lo, hi, bins)
        assert np.array_equal(got, ref), (what, dtype, np.abs(got - ref).max())
        assert (ref > 0).all()


def test_edge_cases():
    dev = need_gpu()
    rng = np.random.default_rng(41)
    cases = [
        # (n, c, h, w, lo, hi, bins)
        (1, 1, 1, 1, 0.0, 1.0, 1),
        (2, 3, 5, 7, -1.0, 1.0, 4096),
        (1, 2, 33, 65, -0.5, 0.25, 3),
        (3, 1, 129, 131, -2.0, 2.0, 100),
        (2, 2, 64, 300, -3.0, 3.0, 1500),   # two LDS copies of the histograms
        (1, 3, 50, 77, -1.0, 1.0, 2048),    # two copies, the largest such bin count
        (1, 1, 70, 90, -1.0, 1.0, 2049),    # one copy
    ]
    for n, c, h, w, lo, hi, bins in cases:
        announce("buffer EMD edge", n, c, h, w, bins)
        cur = rng.normal(0.0, 1.0, (n, c, h, w)).astype(np.float32)
        prev = rng.normal(0.3, 1.5, (n, c, h, w)).astype(np.float32)
        # values beyond the range, at the bounds, NaN and infinities
        flat = cur.reshape(-1)
        special = np.array([np.nan, np.inf, -np.inf, lo, hi, 1e30], np.float32)
        flat[:min(6, flat.size)] = special[:min(6, flat.size)]
        got = gpu_emd(cur, prev, lo, hi, bins, "f32", dev)
        ref = buffer_emd.buffer_emd(cur, prev, lo, hi, bins)
        assert np.array_equal(got, ref), (n, c, h, w, bins, got, ref)
        same = gpu_emd(cur, cur, lo, hi, bins, "f32", dev)
        assert (same == 0).all()
        if bins == 1:
            assert (got == 0).all()


def test_full_size_gbuffer_normals_bf16():
    """The G-buffer workload at full size (4 x 2560 x 1440, bfloat16): the
    normal channels of each frame against the previous frame."""
    dev = need_gpu()
    d = make_config(5)
    normals = d["src"][:, 4:7]
    announce("buffer EMD full size", normals.shape)
    cur, prev = normals[1:], normals[:-1]
    got = gpu_emd(cur, prev, -1.0, 1.0, 256, "bf16", dev)
    ref = buffer_emd.buffer_emd(stored(cur, "bf16"), stored(prev, "bf16"), -1.0, 1.0, 256)
    assert np.array_equal(got, ref)


def test_plane_at_the_size_limit():
    """One plane of 2^30 values (the C ABI's limit; 4 GiB per buffer): every
    value of cur in bin 5 and of prev in bin 2 of 8 on [0, 1] moves all the
    mass 3 bins, so the EMD is 3 bin widths exactly (closed form); the counts
    and their cumulative sums reach 2^30."""
    dev = need_gpu()
    side = 1 << 15
    announce("buffer EMD at the size limit", side, side)
    cur = torch.full((1, 1, side, side), 0.70, dtype=torch.float32, device=dev)   # bin 5
    prev = torch.full((1, 1, side, side), 0.30, dtype=torch.float32, device=dev)  # bin 2
    got = exw.buffer_emd(cur, prev, 0.0, 1.0, 8)
    torch.cuda.synchronize()
    assert got.cpu().tolist() == [[3 * 0.125]]
    same = exw.buffer_emd(cur, cur, 0.0, 1.0, 8)
    torch.cuda.synchronize()
    assert same.cpu().tolist() == [[0.0]]
    del cur, prev
    torch.cuda.empty_cache()
