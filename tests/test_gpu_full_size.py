"""The benchmark's training step at full size, against the float64 C oracle.

For every workload line the benchmark times (1080p and 4K RGBA in float32 and
float16 storage with three fused phases, 8 x 1080p RGB under random motion,
4 x 1440p twelve-channel G-buffers in bfloat16 and float32), the step is run
exactly as timed: the forward that records the adjoint's footprint, then the
adjoint that reads it, on the whole batch. The first and last frames are then
compared element by element with the C oracle (OpenMP) on the same stored
inputs: output, mask, invalid counts, image gradient and motion gradient;
the output also against the oracle's exact displacement mode (mask
differences allowed only in the float32 rounding band of s*u, counted) and,
for 16-bit storage, end to end against the oracle on the float32 frames.
Every frame of the batch, the middle ones included, is checked by the
adjoint identity <W x, g> = <x, W^T g> of its own outputs.

The measured errors are printed and, when EXW_PARITY_REPORT names a file,
written there as JSON.
"""

import json
import os

import numpy as np
import pytest
import torch

import paper_2307_12607_amd as exw
from oracle import ref_c
from synth import make_config, upstream_gradient
from gpu_util import (E2E_TOL, TORCH_DT, announce, assert_close_kernel, compare_with_exact,
                      half_ulp, need_gpu, stored, to_dev, to_host)

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-5  # relative to max(1, |oracle|), as in the other adjoint tests
REL_ROUND = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}

ROWS = [(2, "f32"), (2, "f16"), (3, "f32"), (3, "f16"), (4, "f32"), (5, "bf16"), (5, "f32")]

_cache = {}
_report = {}


def inputs(index):
    """One workload's inputs at a time (a 4K batch is 1.6 GB on the host)."""
    if index not in _cache:
        _cache.clear()
        _cache[index] = make_config(index)
    return _cache[index]


def gradient_seed(index, frame):
    return 50_000 + 100 * index + frame


def _write_report():
    path = os.environ.get("EXW_PARITY_REPORT")
    if path:
        with open(path, "w") as f:
            json.dump(_report, f, indent=1, sort_keys=True)


@pytest.mark.parametrize("index,dtype", ROWS, ids=[f"config{i}-{t}" for i, t in ROWS])
def test_training_step_full_size(index, dtype):
    dev = need_gpu()
    d = inputs(index)
    src32, mv = d["src"], d["mv"]
    phases = [float(s) for s in d["phases"]]
    n, c, h, w = src32.shape
    k = len(phases)
    tdt = TORCH_DT[dtype]
    announce("full-size training step", f"config{index}", dtype, (n, c, h, w, k))
    checked = [0, n - 1]
    sd = to_dev(src32, dtype, dev)
    md = torch.from_numpy(mv).to(dev)
    # dL/d out: host-drawn for the frames compared with the oracle, drawn on
    # the device for the others (checked by the adjoint identity only)
    gd = torch.empty((n, k, c, h, w), dtype=tdt, device=dev)
    gd.uniform_(-1.0, 1.0, generator=torch.Generator(device=dev).manual_seed(index))
    g_host = {}
    for i in checked:
        gi = upstream_gradient(gradient_seed(index, i), (k, c, h, w))
        gd[i].copy_(to_dev(gi, dtype, dev))
        g_host[i] = stored(gi, dtype)
        del gi
    out = torch.empty((n, k, c, h, w), dtype=tdt, device=dev)
    mask = torch.empty((n, k, h, w), dtype=torch.uint8, device=dev)
    cnt = torch.empty((n, k), dtype=torch.int32, device=dev)
    gsrc = torch.empty((n, c, h, w), dtype=tdt, device=dev)
    gmv = torch.empty((n, 2, h, w), dtype=torch.float32, device=dev)
    ws = torch.empty(exw.exw_warp_backward_workspace_bytes(tdt, n, c, h, w), dtype=torch.uint8,
                     device=dev)
    exw.exw_warp_forward_batched_record(sd, md, phases, out, ws, mask, cnt)
    exw.exw_warp_backward_batched_recorded(sd, md, phases, gd, gsrc, gmv, ws)
    torch.cuda.synchronize()

    # every frame: the adjoint identity of the GPU's own outputs
    for i in range(n):
        lhs = float((out[i].double() * gd[i].double()).sum())
        rhs = float((sd[i].double() * gsrc[i].double()).sum())
        scale = float((out[i].double().abs() * gd[i].double().abs()).sum()
                      + (sd[i].double().abs() * gsrc[i].double().abs()).sum())
        tol = (1e-4 * max(1.0, abs(lhs)) if dtype == "f32"
               else 2 * REL_ROUND[dtype] * scale + 1e-6 * scale)
        assert abs(lhs - rhs) <= tol, ("adjoint identity", i, lhs, rhs, tol)

    rec = {"frames_checked": checked}
    errs = {"out": 0.0, "grad_src_rel": 0.0, "grad_mv_rel": 0.0, "out_e2e": 0.0}
    exact_stats = {"band_pixels": 0, "band_mismatches": 0, "max_abs_vs_exact": 0.0}
    for i in checked:
        src_q = stored(src32[i], dtype)[None]
        mv_i = mv[i:i + 1]
        what = f"config{index} {dtype} frame {i}"
        ref_out, ref_mask, ref_cnt = ref_c.forward(src_q, mv_i, phases)
        got_out = to_host(out[i:i + 1])
        got_mask = mask[i:i + 1].cpu().numpy()
        assert np.array_equal(got_mask, ref_mask), f"{what}: mask"
        assert np.array_equal(cnt[i:i + 1].cpu().numpy().astype(np.int64), ref_cnt), f"{what}: count"
        errs["out"] = max(errs["out"], assert_close_kernel(got_out, ref_out, dtype, f"{what} out"))
        ex_out, ex_mask, _ = ref_c.forward(src_q, mv_i, phases, exact=True)
        st = compare_with_exact(got_out, got_mask, ex_out, ex_mask, mv_i, phases, dtype, what)
        exact_stats["band_pixels"] += st["band_pixels"]
        exact_stats["band_mismatches"] += st["band_mismatches"]
        exact_stats["max_abs_vs_exact"] = max(exact_stats["max_abs_vs_exact"],
                                              st["max_abs_vs_exact"])
        del ex_out, ex_mask
        if dtype != "f32":  # end to end: against the oracle on the float32 frames
            e2e, _, _ = ref_c.forward(src32[i:i + 1], mv_i, phases)
            err = float(np.abs(got_out - e2e).max())
            assert err <= E2E_TOL[dtype], f"{what}: end-to-end error {err}"
            errs["out_e2e"] = max(errs["out_e2e"], err)
            del e2e
        del ref_out, got_out
        ref_gs, ref_gm = ref_c.backward(src_q, mv_i, phases, g_host[i][None])
        got_gs = to_host(gsrc[i:i + 1])
        got_gm = to_host(gmv[i:i + 1])
        rel_s = np.abs(got_gs - ref_gs) / np.maximum(1.0, np.abs(ref_gs))
        if dtype == "f32":
            assert float(rel_s.max()) <= GRAD_TOL, f"{what}: grad_src rel err {float(rel_s.max())}"
        else:
            bound = half_ulp(ref_gs, dtype) + GRAD_TOL * np.maximum(1.0, np.abs(ref_gs))
            assert (np.abs(got_gs - ref_gs) <= bound).all(), f"{what}: grad_src"
        rel_m = np.abs(got_gm - ref_gm) / np.maximum(1.0, np.abs(ref_gm))
        assert float(rel_m.max()) <= GRAD_TOL, f"{what}: grad_mv rel err {float(rel_m.max())}"
        errs["grad_src_rel"] = max(errs["grad_src_rel"], float(rel_s.max()))
        errs["grad_mv_rel"] = max(errs["grad_mv_rel"], float(rel_m.max()))
        del ref_gs, ref_gm, got_gs, got_gm
    rec.update({k2: float(v) for k2, v in errs.items()})
    rec["exact_mode"] = exact_stats
    print(f"[full-size] config{index} {dtype}: {json.dumps(rec)}", flush=True)
    _report[f"config{index}-{dtype}"] = rec
    _write_report()
    del sd, md, gd, out, mask, gsrc, gmv, ws
    torch.cuda.empty_cache()
