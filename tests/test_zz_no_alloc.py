"""exw_motion_stats_no_alloc (the call that allocates nothing) against
exw_motion_stats (the same kernels with a caller's workspace), through the
C-ABI: two calls in a row on one GPU, the second on a smaller batch, so that
the static scratch still holds the first call's partials when the second
runs. Both calls must equal the workspace call's results bit for bit."""

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from paper_2307_12607_amd import _capi
from synth import make_config
from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


def _with_workspace(mv):
    n, _, h, w = mv.shape
    ws = torch.empty(exw.exw_motion_stats_workspace_bytes(n, h, w), dtype=torch.uint8,
                     device=mv.device)
    out = torch.empty((n, 4), dtype=torch.float64, device=mv.device)
    exw.exw_motion_stats(mv, out, ws)
    return out


def test_no_alloc_matches_workspace_call_twice():
    dev = need_gpu()
    big = make_config(2, n=6, h=700, w=1100)["mv"]       # 6 x 256 partials: 72 KB of scratch
    small = make_config(5, n=2, h=90, w=130)["mv"]       # 2 x 6 partials
    cap = _capi.EXW_NO_ALLOC_SCRATCH_BYTES
    assert exw.exw_motion_stats_workspace_bytes(*big.shape[:1], *big.shape[2:]) <= cap
    results = []
    for label, mv_host in (("larger batch", big), ("smaller batch", small)):
        announce("no-alloc motion statistics", label, mv_host.shape)
        mv = torch.from_numpy(mv_host).to(dev)
        got = torch.full((mv.shape[0], 4), float("nan"), dtype=torch.float64, device=dev)
        exw.exw_motion_stats_no_alloc(mv, got)
        ref = _with_workspace(mv)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(g, r), (label, np.abs(g - r).max())
        assert np.isfinite(g).all()
        results.append(g)
    # the second call saw none of the first call's partials
    assert results[1].shape == (2, 4)


def test_no_alloc_rejects_batches_beyond_its_scratch():
    dev = need_gpu()
    # 200 frames of 1920 x 1080 need 200 x 256 partials of 48 bytes: 2.4 MB
    mv = torch.zeros((200, 2, 8, 8), dtype=torch.float32, device=dev)
    st = _capi.lib().exw_motion_stats_no_alloc(mv.data_ptr(), 200, 1080, 1920, mv.data_ptr(), None)
    assert st == _capi.EXW_ERROR_UNSUPPORTED
    assert "static scratch" in _capi.last_error()
