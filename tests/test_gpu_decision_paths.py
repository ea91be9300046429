"""Chained warps and decision-path frames on the GPU, against the oracle.

Each chain step is the forward warp applied to the previous step's stored
output, so it is checked like the forward (kernel-only tolerance) against
the oracle run on the GPU's own previous step, and end to end against the
oracle chain that rounds every step to the storage type.
"""

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from oracle import decision_paths as D
from oracle import warp_oracle
from synth import make_config, quantize
from gpu_util import announce, assert_close_kernel, need_gpu, stored, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_chain_each_step_matches_oracle(dtype):
    dev = need_gpu()
    d = make_config(2, n=2, h=75, w=131)
    src = to_dev(d["src"], dtype, dev)
    mv = torch.from_numpy(d["mv"]).to(dev)
    announce("warp chain", dtype, d["src"].shape)
    out, mask, cnt = exw.warp_chain(src, mv, 0.25, 3, return_mask=True, return_count=True)
    torch.cuda.synchronize()
    out_h = to_host(out)
    prev = stored(d["src"], dtype)
    for i in range(3):
        ref, ref_mask, ref_cnt = warp_oracle.forward(prev, d["mv"], [0.25])
        assert np.array_equal(mask[i].cpu().numpy(), ref_mask[:, 0]), i
        assert np.array_equal(cnt[i].cpu().numpy().astype(np.int64), ref_cnt[:, 0]), i
        assert_close_kernel(out_h[i], ref[:, 0], dtype, f"chain step {i}")
        prev = out_h[i]  # the GPU's stored step feeds the next one


def test_chain_end_to_end_and_integer_steps():
    dev = need_gpu()
    d = make_config(2, n=2, h=64, w=96)
    announce("warp chain end to end")
    out = exw.warp_chain(torch.from_numpy(d["src"]).to(dev), torch.from_numpy(d["mv"]).to(dev),
                         0.25, 3)
    ref, _, _ = D.chained_warp(d["src"], d["mv"], 0.25, 3, store=lambda x: quantize(x, "f32"))
    # three float32 steps, each within 1e-5 of its own oracle step and a
    # contraction of the previous error (bilinear weights sum to at most 1)
    assert float(np.abs(to_host(out) - ref).max()) <= 3e-5
    # integer quarter steps: exact shifts with zero fill
    rng = np.random.default_rng(3)
    src = rng.random((1, 3, 20, 30)).astype(np.float32)
    mv = np.zeros((1, 2, 20, 30), np.float32)
    mv[:, 0], mv[:, 1] = 8.0, -4.0
    announce("warp chain integer steps")
    out = exw.warp_chain(torch.from_numpy(src).to(dev), torch.from_numpy(mv).to(dev), 0.25, 4)
    ref, _, _ = D.chained_warp(src, mv, 0.25, 4)
    assert np.array_equal(to_host(out), ref)


def test_decision_path_frames():
    dev = need_gpu()
    d = make_config(2, n=1, h=90, w=160)
    src = torch.from_numpy(d["src"]).to(dev)
    mv = torch.from_numpy(d["mv"]).to(dev)
    announce("decision path frames")
    chain = exw.warp_chain(src, mv, 0.25, 3)

    def extrap(frame):  # a stand-in extrapolator: brightens, so its output is recognisable
        return frame * 0.5 + 0.25

    s6 = exw.decision_path_frames(src, mv, exw.plan(D.WARP, D.WARP, D.WARP), extrap)
    for i in range(3):
        assert torch.equal(s6[i], chain[i])
    s4 = exw.decision_path_frames(src, mv, exw.plan(D.WARP, D.EXTRAPOLATE, D.WARP), extrap)
    assert torch.equal(s4[0], chain[0])
    assert torch.equal(s4[1], extrap(src))
    assert torch.equal(s4[2], exw.warp(extrap(src), mv, (0.25,))[:, 0])
    s1 = exw.decision_path_frames(src, mv, exw.plan(D.EXTRAPOLATE, None, D.EXTRAPOLATE), extrap)
    assert torch.equal(s1[0], src) and torch.equal(s1[2], s1[1])
    s5 = exw.decision_path_frames(src, mv, exw.plan(D.WARP, D.WARP, D.EXTRAPOLATE))
    assert torch.equal(s5[1], chain[1]) and s5[2] is None  # no extrapolator given
