"""The C-ABI library without a GPU: it loads, exports what the header declares,
and rejects bad arguments before any HIP call."""

import ctypes
import os
import re
import subprocess

import pytest

from paper_2307_12607_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exwarp.h")

F = ctypes.c_float
FAKE = 0x7f0000000000  # aligned fake device address; never dereferenced on the CPU


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(exw_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_functions()
    assert names == sorted(_capi.SIGNATURES), names


def test_library_exports_every_declared_symbol():
    L = _capi.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _capi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (exw_\w+)", out))
    assert set(declared_functions()) <= exported


def test_abi_version_and_status_strings():
    L = _capi.lib()
    assert L.exw_abi_version() == 2
    assert _capi.status_string(0) == "EXW_SUCCESS"
    assert _capi.status_string(1) == "EXW_ERROR_INVALID_VALUE"
    assert _capi.status_string(2) == "EXW_ERROR_UNSUPPORTED"
    assert _capi.status_string(3) == "EXW_ERROR_LAUNCH"
    assert _capi.status_string(99) == "EXW_UNKNOWN_STATUS"


def _phases(*vals):
    return (F * len(vals))(*vals)


def fwd(src=FAKE, dtype=0, n=1, c=3, h=8, w=8, mv=FAKE + (1 << 30), phases=None, k=1,
        out=FAKE + (2 << 30), mask=None, count=None):
    if phases is None:
        phases = _phases(1.0)
    return _capi.lib().exw_warp_forward_batched(src, dtype, n, c, h, w, mv, phases, k, out, mask,
                                                count, None)


def bwd(src=FAKE, dtype=0, n=1, c=3, h=8, w=8, mv=FAKE + (1 << 30), phases=None, k=1,
        gout=FAKE + (2 << 30), gsrc=FAKE + (3 << 30), gmv=FAKE + (4 << 30), ws=FAKE + (6 << 30),
        ws_bytes=1 << 30):
    if phases is None:
        phases = _phases(1.0)
    return _capi.lib().exw_warp_backward_batched(src, dtype, n, c, h, w, mv, phases, k, gout,
                                                 gsrc, gmv, ws, ws_bytes, None)


INVALID, UNSUPPORTED = _capi.EXW_ERROR_INVALID_VALUE, _capi.EXW_ERROR_UNSUPPORTED


@pytest.mark.parametrize("kwargs,status,needle", [
    (dict(dtype=7), INVALID, "dtype"),
    (dict(n=-1), INVALID, "negative"),
    (dict(h=-2), INVALID, "negative"),
    (dict(c=0), INVALID, "channel"),
    (dict(c=65), UNSUPPORTED, "channel"),
    (dict(k=0), INVALID, "phase count"),
    (dict(k=5, phases=(F * 5)(1, 1, 1, 1, 1)), UNSUPPORTED, "phase count"),
    (dict(phases=_phases(float("nan"))), INVALID, "not finite"),
    (dict(phases=_phases(float("inf"))), INVALID, "not finite"),
    (dict(src=None), INVALID, "src is NULL"),
    (dict(mv=None), INVALID, "mv is NULL"),
    (dict(out=None), INVALID, "out is NULL"),
    (dict(src=FAKE + 2), INVALID, "aligned"),
    (dict(mask=FAKE + 64), INVALID, "mask overlaps input src"),
    (dict(mv=FAKE + 1 + (1 << 30)), INVALID, "aligned"),
    (dict(out=FAKE + 100), INVALID, "overlaps input src"),
    (dict(mask=FAKE + (2 << 30) + 16), INVALID, "out overlaps output mask"),
    (dict(count=FAKE + (1 << 30) + 8), INVALID, "overlaps input mv"),
    (dict(count=FAKE + 2 + (5 << 30)), INVALID, "aligned"),
    (dict(h=1 << 24, w=1), UNSUPPORTED, "2^24"),
    (dict(h=1 << 16, w=1 << 15), UNSUPPORTED, "2^30"),
    (dict(n=1 << 20, c=64, h=4096, w=4096, k=1), UNSUPPORTED, "too large"),
    # twelve 16-bit channels: 129 * (2^22 - 1) * 4 >= 2^31 row segments, while the
    # 64 x 4 tiles (129 * (2^22 - 1)), H*W and the element count are in range
    (dict(dtype=1, n=129, c=12, h=(1 << 24) - 4, w=2), UNSUPPORTED, "row segments"),
])
def test_forward_rejects(kwargs, status, needle):
    st = fwd(**kwargs)
    assert st == status, (_capi.status_string(st), _capi.last_error())
    assert needle in _capi.last_error()


@pytest.mark.parametrize("kwargs,status,needle", [
    (dict(dtype=3), INVALID, "dtype"),
    (dict(gout=None), INVALID, "grad_out is NULL"),
    (dict(src=None), INVALID, "src is NULL"),
    (dict(mv=None), INVALID, "mv is NULL"),
    (dict(ws=None), INVALID, "workspace is NULL"),
    (dict(dtype=1, ws=None), INVALID, "workspace is NULL"),
    (dict(dtype=2, ws_bytes=16), INVALID, "needs"),
    (dict(ws=FAKE + (6 << 30) + 128), INVALID, "256-byte aligned"),
    (dict(ws=FAKE + (3 << 30) + 512), INVALID, "overlaps output workspace"),
    (dict(gsrc=FAKE + (2 << 30)), INVALID, "grad_src overlaps input grad_out"),
    (dict(gmv=FAKE), INVALID, "grad_mv overlaps input src"),
    (dict(gmv=FAKE + (3 << 30) + 64), INVALID, "grad_src overlaps output grad_mv"),
    (dict(gsrc=FAKE + 1 + (3 << 30)), INVALID, "aligned"),
    (dict(k=9, phases=(F * 9)(*[1] * 9)), UNSUPPORTED, "phase count"),
])
def test_backward_rejects(kwargs, status, needle):
    st = bwd(**kwargs)
    assert st == status, (_capi.status_string(st), _capi.last_error())
    assert needle in _capi.last_error()


def fwd_rec(src=FAKE, dtype=0, n=1, c=3, h=8, w=8, mv=FAKE + (1 << 30), phases=None, k=1,
            out=FAKE + (2 << 30), mask=None, count=None, stats=None, ws=FAKE + (6 << 30),
            ws_bytes=1 << 30):
    if phases is None:
        phases = _phases(1.0)
    return _capi.lib().exw_warp_forward_batched_record(src, dtype, n, c, h, w, mv, phases, k, out,
                                                       mask, count, stats, ws, ws_bytes, None)


def bwd_rec(**kwargs):
    a = dict(src=FAKE, dtype=0, n=1, c=3, h=8, w=8, mv=FAKE + (1 << 30), phases=_phases(1.0), k=1,
             gout=FAKE + (2 << 30), gsrc=FAKE + (3 << 30), gmv=FAKE + (4 << 30),
             ws=FAKE + (6 << 30), ws_bytes=1 << 30)
    a.update(kwargs)
    return _capi.lib().exw_warp_backward_batched_recorded(
        a["src"], a["dtype"], a["n"], a["c"], a["h"], a["w"], a["mv"], a["phases"], a["k"],
        a["gout"], a["gsrc"], a["gmv"], a["ws"], a["ws_bytes"], None)


@pytest.mark.parametrize("kwargs,status,needle", [
    (dict(dtype=5), INVALID, "dtype"),
    (dict(c=65), UNSUPPORTED, "channel"),
    (dict(src=None), INVALID, "src is NULL"),
    (dict(out=FAKE + 100), INVALID, "overlaps input src"),
    (dict(ws=None), INVALID, "workspace is NULL"),
    (dict(ws_bytes=16), INVALID, "needs"),
    (dict(dtype=1, ws_bytes=1000), INVALID, "needs"),
    (dict(ws=FAKE + (6 << 30) + 64), INVALID, "256-byte aligned"),
    (dict(ws=FAKE + (2 << 30)), INVALID, "overlaps output workspace"),
    (dict(ws=FAKE), INVALID, "workspace overlaps input src"),
    (dict(mask=FAKE + (6 << 30) + 64), INVALID, "mask overlaps output workspace"),
    (dict(stats=FAKE + (7 << 30) + 4), INVALID, "motion_stats is not 8-byte aligned"),
    (dict(stats=FAKE + (6 << 30) + 256), INVALID, "workspace overlaps output motion_stats"),
    (dict(stats=FAKE + 8), INVALID, "motion_stats overlaps input src"),
    (dict(stats=FAKE + (7 << 30), h=0), INVALID, "no variance"),
])
def test_recording_forward_rejects(kwargs, status, needle):
    st = fwd_rec(**kwargs)
    assert st == status, (_capi.status_string(st), _capi.last_error())
    assert needle in _capi.last_error()


@pytest.mark.parametrize("kwargs,status,needle", [
    (dict(dtype=3), INVALID, "dtype"),
    (dict(gout=None), INVALID, "grad_out is NULL"),
    (dict(ws=None), INVALID, "workspace is NULL"),
    (dict(dtype=2, ws_bytes=16), INVALID, "needs"),
    (dict(ws=FAKE + (6 << 30) + 128), INVALID, "256-byte aligned"),
    (dict(gsrc=FAKE + (2 << 30)), INVALID, "grad_src overlaps input grad_out"),
])
def test_recorded_backward_rejects(kwargs, status, needle):
    st = bwd_rec(**kwargs)
    assert st == status, (_capi.status_string(st), _capi.last_error())
    assert needle in _capi.last_error()


def test_recording_pair_on_empty_batches_is_a_no_op():
    assert fwd_rec(n=0, src=None, mv=None, out=None, ws=None, ws_bytes=0) == 0
    assert fwd_rec(w=0, src=None, mv=None, out=None, ws=None, ws_bytes=0) == 0
    assert _capi.last_error() == ""
    assert bwd_rec(n=0, src=None, mv=None, gout=None, gsrc=None, gmv=None, ws=None) == 0
    assert bwd_rec(gsrc=None, gmv=None) == 0


def test_empty_batches_and_no_requested_gradient_are_no_ops():
    # No pointer is needed, and nothing is launched (this host has no GPU).
    assert fwd(n=0, src=None, mv=None, out=None) == 0
    assert fwd(h=0, src=None, mv=None, out=None) == 0
    assert _capi.last_error() == ""
    assert bwd(n=0, src=None, mv=None, gout=None, gsrc=None, gmv=None) == 0
    assert bwd(gsrc=None, gmv=None) == 0


def test_workspace_size():
    L = _capi.lib()
    # per 64-pixel row segment a 16 B tap box and 16 B of tap offsets; 8 B per
    # frame; 2 x 24 B of motion-statistics partials per 128 x 4 tile (at least
    # one per 2048 pixels, at most 256, per frame), 2 x 8 x 24 B of fold slots
    # and 2 x 4 B of counters per frame; float32 accumulator for 16-bit storage
    def expect(dtype, n, c, h, w):
        boxes = 32 * n * h * ((w + 63) // 64)
        info = (boxes + 255) // 256 * 256
        stats = (info + 8 * n + 255) // 256 * 256
        tiles = ((w + 127) // 128) * ((h + 3) // 4)
        parts = max(tiles, min(256, (h * w + 2047) // 2048))
        accum = (stats + 48 * n * parts + 384 * n + 8 * n + 255) // 256 * 256
        return accum + (0 if dtype == 0 else 4 * n * c * h * w)
    for args in [(0, 2, 3, 4, 5), (1, 2, 3, 4, 5), (2, 8, 12, 1440, 2560), (0, 8, 4, 1080, 1920)]:
        assert L.exw_warp_backward_workspace_bytes(*args) == expect(*args), args
    assert L.exw_warp_backward_workspace_bytes(2, 0, 3, 4, 5) == 0
    assert L.exw_warp_backward_workspace_bytes(9, 1, 3, 4, 5) == 0


def stats(mv=FAKE, n=2, h=8, w=8, out=FAKE + (1 << 30), ws=FAKE + (2 << 30), ws_bytes=1 << 20):
    L = _capi.lib()
    return L.exw_motion_stats(mv, n, h, w, out, ws, ws_bytes, None)


@pytest.mark.parametrize("kwargs,status,needle", [
    (dict(n=-1), INVALID, "negative size"),
    (dict(h=0), INVALID, "empty frames"),
    (dict(h=1 << 24), UNSUPPORTED, "2^24"),
    (dict(h=1 << 16, w=1 << 15), UNSUPPORTED, "2^30"),
    (dict(n=1 << 21), UNSUPPORTED, "2^21"),
    (dict(mv=None), INVALID, "mv is NULL"),
    (dict(mv=FAKE + 2), INVALID, "aligned"),
    (dict(out=None), INVALID, "stats is NULL"),
    (dict(out=FAKE + (1 << 30) + 4), INVALID, "aligned"),
    (dict(ws=None), INVALID, "workspace is NULL"),
    (dict(ws=FAKE + (2 << 30) + 64), INVALID, "256-byte aligned"),
    (dict(ws_bytes=8), INVALID, "workspace has 8 bytes"),
    (dict(out=FAKE + 64), INVALID, "stats overlaps input mv"),
    (dict(ws=FAKE + (1 << 30)), INVALID, "stats overlaps output workspace"),
])
def test_motion_stats_rejects(kwargs, status, needle):
    st = stats(**kwargs)
    assert st == status, (_capi.status_string(st), _capi.last_error())
    assert needle in _capi.last_error()


def test_motion_stats_empty_batch_and_workspace_size():
    assert stats(n=0, mv=None, out=None, ws=None, ws_bytes=0) == 0
    L = _capi.lib()
    # 48 bytes per workgroup partial (count, mean, M2 of both components in
    # float64); ceil(H*W / 2048) partials per frame, at most 256
    for (n, h, w) in [(1, 1, 1), (2, 45, 46), (3, 64, 64), (8, 1080, 1920), (4, 1440, 2560),
                      (2, 2160, 3840)]:
        parts = min(-(-h * w // 2048), 256)
        assert L.exw_motion_stats_workspace_bytes(n, h, w) == 48 * n * parts
    assert L.exw_motion_stats_workspace_bytes(0, 4, 4) == 0


def qual(pred=FAKE, truth=FAKE + (1 << 30), dtype=0, b=2, c=3, h=16, w=20, peak=1.0,
         out=FAKE + (2 << 30), ws=FAKE + (3 << 30), ws_bytes=1 << 20):
    return _capi.lib().exw_frame_quality(pred, truth, dtype, b, c, h, w, peak, out, ws, ws_bytes,
                                         None)


@pytest.mark.parametrize("kwargs,status,needle", [
    (dict(dtype=7), INVALID, "unknown dtype"),
    (dict(b=-1), INVALID, "negative size"),
    (dict(peak=0.0), INVALID, "peak"),
    (dict(peak=float("nan")), INVALID, "peak"),
    (dict(c=0), INVALID, "channel count"),
    (dict(h=10), INVALID, "11x11"),
    (dict(w=3), INVALID, "11x11"),
    (dict(h=1 << 24), UNSUPPORTED, "2^24"),
    (dict(pred=None), INVALID, "pred is NULL"),
    (dict(truth=FAKE + 2 + (1 << 30)), INVALID, "aligned"),
    (dict(dtype=1, pred=FAKE + 1), INVALID, "aligned"),
    (dict(out=FAKE + (2 << 30) + 4), INVALID, "aligned"),
    (dict(ws=None), INVALID, "workspace is NULL"),
    (dict(ws_bytes=8), INVALID, "workspace has 8 bytes"),
    (dict(out=FAKE + 64), INVALID, "quality overlaps input pred"),
    (dict(ws=FAKE + 256), INVALID, "workspace overlaps input pred"),
])
def test_frame_quality_rejects(kwargs, status, needle):
    st = qual(**kwargs)
    assert st == status, (_capi.status_string(st), _capi.last_error())
    assert needle in _capi.last_error()


def test_frame_quality_empty_batch_and_workspace_size():
    assert qual(b=0, pred=None, truth=None, out=None, ws=None, ws_bytes=0) == 0
    L = _capi.lib()
    # 16 bytes (SSIM sum, squared-error sum) per strip of 64 x 66 SSIM positions
    for (b, c, h, w) in [(1, 1, 11, 11), (2, 3, 76, 74), (3, 4, 77, 75), (24, 4, 1080, 1920)]:
        strips = -(-(w - 10) // 64) * -(-(h - 10) // 66)
        assert L.exw_frame_quality_workspace_bytes(b, c, h, w) == 16 * b * c * strips
    assert L.exw_frame_quality_workspace_bytes(1, 1, 10, 40) == 0


def chain(src=FAKE, dtype=0, n=1, c=3, h=8, w=8, mv=FAKE + (1 << 30), phase=0.25, steps=3,
          out=FAKE + (2 << 30), mask=None, count=None):
    return _capi.lib().exw_warp_chain(src, dtype, n, c, h, w, mv, F(phase), steps, out, mask,
                                      count, None)


@pytest.mark.parametrize("kwargs,status,needle", [
    (dict(steps=0), INVALID, "steps 0 < 1"),
    (dict(phase=float("inf")), INVALID, "not finite"),
    (dict(c=65), UNSUPPORTED, "channel count"),
    (dict(src=None), INVALID, "src is NULL"),
    (dict(out=FAKE + 100), INVALID, "out overlaps input src"),
    (dict(mask=FAKE + (2 << 30) + 3 * 3 * 64 * 4 - 8), INVALID, "out overlaps output mask"),
    (dict(count=FAKE + (1 << 30) + 4), INVALID, "overlaps input mv"),
    (dict(n=1 << 20, h=1 << 10, w=1 << 10, steps=4), UNSUPPORTED, "too large"),
])
def test_chain_rejects(kwargs, status, needle):
    st = chain(**kwargs)
    assert st == status, (_capi.status_string(st), _capi.last_error())
    assert needle in _capi.last_error()


def test_chain_empty_batch_is_a_no_op():
    assert chain(n=0, src=None, mv=None, out=None) == 0


def test_missing_library_fails_loudly(tmp_path):
    code = ("import paper_2307_12607_amd._capi as c; c.LIB_PATH = '/nonexistent/libexwarp.so'; "
            "c._lib = None\ntry:\n    c.lib()\nexcept ImportError as e:\n    print('RAISED', e)")
    res = subprocess.run(["python", "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert "RAISED" in res.stdout and "build" in res.stdout


def test_product_path_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2307_12607_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b|warp_ref|synth", text), f


@pytest.mark.parametrize("call,args,needle", [
    ("exw_stream_copy", (FAKE, FAKE + (1 << 30), 100, None), "multiple of 16"),
    ("exw_stream_copy", (None, FAKE, 64, None), "src is NULL"),
    ("exw_stream_copy", (FAKE + 8, FAKE + (1 << 30), 64, None), "src is not 16-byte aligned"),
    ("exw_stream_copy", (FAKE, FAKE + 32, 64, None), "overlaps"),
    ("exw_stream_read", (FAKE, 64, None, None), "sink is NULL"),
    ("exw_stream_read", (FAKE, 48, FAKE + 2, None), "sink is not 4-byte aligned"),
    ("exw_stream_write", (FAKE + 4, 64, None), "dst is not 16-byte aligned"),
])
def test_stream_calls_reject(call, args, needle):
    st = getattr(_capi.lib(), call)(*args)
    assert st == _capi.EXW_ERROR_INVALID_VALUE
    assert needle in _capi.last_error()


def test_stream_calls_of_zero_bytes_are_no_ops():
    for call, args in (("exw_stream_copy", (FAKE, FAKE, 0, None)),
                       ("exw_stream_read", (FAKE, 0, FAKE, None)),
                       ("exw_stream_write", (FAKE, 0, None))):
        assert getattr(_capi.lib(), call)(*args) == _capi.EXW_SUCCESS


def test_motion_stats_no_alloc_rejects_before_any_hip_call():
    L = _capi.lib()
    # beyond the static scratch: 200 x 1080p needs 200 x 256 partials of 48 bytes
    assert L.exw_motion_stats_no_alloc(FAKE, 200, 1080, 1920, FAKE + (1 << 30), None) == \
        _capi.EXW_ERROR_UNSUPPORTED
    assert "static scratch" in _capi.last_error()
    assert L.exw_motion_stats_no_alloc(None, 1, 8, 8, FAKE, None) == _capi.EXW_ERROR_INVALID_VALUE
    assert L.exw_motion_stats_no_alloc(FAKE, 1, 0, 8, FAKE, None) == _capi.EXW_ERROR_INVALID_VALUE
    assert L.exw_motion_stats_no_alloc(FAKE, 0, 8, 8, FAKE, None) == _capi.EXW_SUCCESS


def emd(cur=FAKE, prev=FAKE + (1 << 30), dtype=0, n=1, c=3, h=8, w=8, lo=-1.0, hi=1.0, bins=64,
        out=FAKE + (2 << 30), ws=FAKE + (3 << 30), ws_bytes=1 << 20):
    return _capi.lib().exw_buffer_emd(cur, prev, dtype, n, c, h, w, lo, hi, bins, out, ws,
                                      ws_bytes, None)


@pytest.mark.parametrize("kwargs,status,needle", [
    (dict(dtype=7), 1, "unknown dtype"),
    (dict(c=0), 1, "channel count"),
    (dict(c=65), 2, "channel count"),
    (dict(lo=1.0, hi=1.0), 1, "finite lo < hi"),
    (dict(lo=float("nan")), 1, "finite lo < hi"),
    (dict(hi=float("inf")), 1, "finite lo < hi"),
    (dict(bins=0), 1, "bins 0"),
    (dict(bins=4097), 1, "bins 4097"),
    (dict(h=0), 1, "empty frames"),
    (dict(cur=None), 1, "cur is NULL"),
    (dict(prev=FAKE + 2), 1, "prev is not 4-byte aligned"),
    (dict(ws_bytes=100), 1, "workspace has 100 bytes"),
    (dict(out=FAKE + 64), 1, "emd overlaps input cur"),
])
def test_buffer_emd_rejects(kwargs, status, needle):
    assert emd(**kwargs) == status
    assert needle in _capi.last_error(), _capi.last_error()


def test_buffer_emd_empty_batch_and_workspace_size():
    assert emd(n=0) == _capi.EXW_SUCCESS
    L = _capi.lib()
    assert L.exw_buffer_emd_workspace_bytes(2, 3, 100) == 2 * 3 * 2 * 100 * 4
    assert L.exw_buffer_emd_workspace_bytes(0, 3, 100) == 0
    assert L.exw_buffer_emd_workspace_bytes(1, 3, 4097) == 0


def dyn(st=FAKE, n=2, h=40, w=70, conn=8, count=FAKE + (1 << 30), ws=FAKE + (2 << 30),
        ws_bytes=1 << 20):
    return _capi.lib().exw_dynamic_objects(st, n, h, w, conn, count, ws, ws_bytes, None)


@pytest.mark.parametrize("kwargs,status,needle", [
    (dict(n=-1), 1, "negative size"),
    (dict(conn=6), 1, "connectivity 6 is not 4 or 8"),
    (dict(h=1 << 15, w=1 << 16), 2, "h*w"),
    (dict(st=None), 1, "stencil is NULL"),
    (dict(count=None), 1, "count is NULL"),
    (dict(count=FAKE + (1 << 30) + 2), 1, "count is not 4-byte aligned"),
    (dict(ws=FAKE + (2 << 30) + 16), 1, "workspace is not 256-byte aligned"),
    (dict(ws_bytes=100), 1, "workspace has 100 bytes"),
    (dict(count=FAKE + 64), 1, "count overlaps input stencil"),
    (dict(ws=FAKE + (1 << 30)), 1, "overlaps"),
])
def test_dynamic_objects_rejects(kwargs, status, needle):
    assert dyn(**kwargs) == status
    assert needle in _capi.last_error(), _capi.last_error()


def test_dynamic_objects_empty_batch_and_workspace_size():
    L = _capi.lib()
    assert dyn(n=0) == _capi.EXW_SUCCESS
    assert dyn(n=0, st=None, count=None, ws=None) == _capi.EXW_SUCCESS
    assert L.exw_dynamic_objects_workspace_bytes(2, 40, 70) == 4 * 2 * 40 * 70
    assert L.exw_dynamic_objects_workspace_bytes(0, 40, 70) == 0
    assert L.exw_dynamic_objects_workspace_bytes(2, 0, 70) == 0
