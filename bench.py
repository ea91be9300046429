#!/usr/bin/env python3
"""Throughput of the motion-vector warp on one MI355X.

One step = the whole hot path over one batch: the fused K-phase forward warp
(output frames, validity mask, invalid counts) followed by the adjoint
(image and motion gradients) for the same batch, as a training step runs
them: the forward also records the adjoint's footprint (the tap box and
offsets of every row segment) and the adjoint takes it from there. The same
calls on their own are timed too and reported beside. Default workload: 8 frames
of 1920x1080 RGBA stored as float32, pan + 16 moving rectangles, 3 phases
(1/4, 2/4, 3/4). Inputs are resident in device memory before timing starts;
two complete buffer sets alternate between steps so that one step's data is
not served from the previous step's caches.

Prints one JSON line. ``value`` = output pixels (N*K*H*W) per second of a
forward+backward step, in Mpix/s. Beside it: the other workloads (4K, 16-bit
storage, random motion, G-buffers), the measured HBM ceilings (hand-written
copy, read and write streams), the motion statistics (their own pass, and
folded by the recording forward), the EMD features of the G-buffers, the
frame quality of the predicted frames against the scene's analytic frames,
and the CPU leg: the float64 C oracle
timed on the host (one thread and the process's CPU share) and, from the same
oracle, each workload's measured error on its first frame.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
FP64_VECTOR_PEAK_GFLOPS = 78600.0  # MI355X float64 vector peak (256 CUs x 2.4 GHz)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
GRAD_SEED = 90_001  # seed of the host-drawn upstream gradient of frame 0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=30)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--config", type=int, default=2, choices=[2, 3, 4, 5])
    p.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    p.add_argument("--no-variants", action="store_true",
                   help="skip the other workloads (FP16, 4K, loss-gradient, G-buffer lines)")
    p.add_argument("--no-cpu-baseline", action="store_true",
                   help="skip the CPU leg (oracle timing and the error figures)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run a plain 1 GiB device copy first (for counter scaling)")
    p.add_argument("--only-step", action="store_true",
                   help="time the step alone: no statistics, EMD, quality, chain or ceiling "
                        "lines (for profiler runs)")
    return p.parse_args()


def algorithmic_bytes(n, c, h, w, k, b):
    """Bytes the method must move once per launch (each input read once, each
    output written once)."""
    px = n * h * w
    fwd = px * c * b + px * 8 + px * k * c * b + px * k * 1 + n * k * 4
    bwd = px * k * c * b + px * c * b + px * 8 + px * c * b + px * 8
    return fwd, bwd


def ssim_flops_per_position() -> float:
    """Float64 operations of the SSIM filter per output position and channel
    (an FMA counts 2), from the strip kernel's separable scheme: each input
    row is filtered horizontally (11 taps x (2 mul + 2 add + 3 FMA) = 110)
    and added into the 11 output rows it feeds (11 x 5 FMA = 110); a strip of
    66 output rows reads 76 input rows, so both are paid 76/66 times per
    output row; the index itself is ~20 operations (3 products, 3
    differences, the numerator's and denominator's sums and products, the
    quotient, the running sum) and the squared error 3 (difference + FMA)."""
    return (110.0 + 110.0) * 76.0 / 66.0 + 20.0 + 3.0


def _elf_section(path, name):
    """Bytes of one section of an ELF64 little-endian file (None if absent)."""
    with open(path, "rb") as f:
        data = f.read()
    if data[:4] != b"\x7fELF" or data[4] != 2:
        return None
    u16 = lambda o: int.from_bytes(data[o:o + 2], "little")
    u64 = lambda o: int.from_bytes(data[o:o + 8], "little")
    shoff, shentsize, shnum, shstrndx = u64(0x28), u16(0x3A), u16(0x3C), u16(0x3E)
    def header(i):
        b = shoff + i * shentsize
        return int.from_bytes(data[b:b + 4], "little"), u64(b + 0x18), u64(b + 0x20)
    _, str_off, _ = header(shstrndx)
    for i in range(shnum):
        name_off, off, size = header(i)
        end = data.index(b"\0", str_off + name_off)
        if data[str_off + name_off:end].decode() == name:
            return data[off:off + size]
    return None


def code_objects(lib_path):
    """The gfx950 code objects (ELF images) in a library's .hip_fatbin
    section, which holds one clang offload bundle per translation unit: a
    24-byte magic, the entry count, then per entry its offset (from the
    bundle's start), size, and target triple."""
    sec = _elf_section(lib_path, ".hip_fatbin") or b""
    magic = b"__CLANG_OFFLOAD_BUNDLE__"
    u64 = lambda o: int.from_bytes(sec[o:o + 8], "little")
    objs = []
    pos = sec.find(magic)
    while pos >= 0:
        off = pos + len(magic) + 8
        for _ in range(u64(pos + len(magic))):
            e_off, e_size, t_size = u64(off), u64(off + 8), u64(off + 16)
            triple = sec[off + 24:off + 24 + t_size].decode(errors="replace")
            off += 24 + t_size
            if "gfx950" in triple and e_size:
                objs.append(sec[pos + e_off:pos + e_off + e_size])
        pos = sec.find(magic, off)
    return objs


def elf_symbols(data):
    """{symbol name: bytes} of the sized symbols of an ELF64 image (kernel
    code in .text, kernel descriptors `<name>.kd`)."""
    u16 = lambda o: int.from_bytes(data[o:o + 2], "little")
    u32 = lambda o: int.from_bytes(data[o:o + 4], "little")
    u64 = lambda o: int.from_bytes(data[o:o + 8], "little")
    shoff, shentsize, shnum = u64(0x28), u16(0x3A), u16(0x3C)
    secs = []
    for i in range(shnum):
        b = shoff + i * shentsize
        secs.append({"type": u32(b + 4), "addr": u64(b + 0x10), "offset": u64(b + 0x18),
                     "size": u64(b + 0x20), "link": u32(b + 0x28)})
    out = {}
    for sec in secs:
        if sec["type"] != 2:  # SHT_SYMTAB
            continue
        strtab = secs[sec["link"]]["offset"]
        for e in range(sec["offset"], sec["offset"] + sec["size"], 24):
            name_off, shndx, value, size = u32(e), u16(e + 6), u64(e + 8), u64(e + 16)
            if size == 0 or shndx == 0 or shndx >= len(secs):
                continue
            end = data.index(b"\0", strtab + name_off)
            name = data[strtab + name_off:end].decode(errors="replace")
            tgt = secs[shndx]
            start = tgt["offset"] + (value - tgt["addr"])
            out[name] = data[start:start + size]
    return out


def kernel_code_sha(names, lib_path=None):
    """Hash of the named kernels' machine code and descriptors in the built
    library (None if one is missing): stored counter readings apply only
    while the kernels they were taken on are unchanged. Other kernels,
    comments and host code do not change it."""
    if lib_path is None:
        import paper_2307_12607_amd._capi as capi
        lib_path = capi.LIB_PATH
    syms = {}
    for obj in code_objects(lib_path):
        syms.update(elf_symbols(obj))
    h = hashlib.sha256()
    for name in sorted(names):
        if name not in syms:
            return None
        h.update(name.encode() + syms[name] + syms.get(name + ".kd", b""))
    return h.hexdigest()[:16]


def load_traffic(call, workload):
    """HBM bytes per call from stored rocprofv3 counter runs, if they were
    taken on the kernels the library now holds; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    entry = rec.get("calls", {}).get(f"{call}|{workload}")
    if not entry or kernel_code_sha(entry["kernels"]) != entry.get("code_sha"):
        return None
    return entry.get("hbm_bytes_per_launch")


class Workload:
    def __init__(self, index, dtype, dev, sets=2, with_truth=False):
        import numpy as np
        import torch
        import paper_2307_12607_amd as exw
        from synth import make_config, upstream_gradient

        self.torch = torch
        d = make_config(index, with_truth=with_truth)
        self.spec = d["spec"]
        self.dtype = dtype
        tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dtype]
        self.tdt = tdt
        self.phases = [float(s) for s in d["phases"]]
        n, c, h, w = d["src"].shape
        k = len(self.phases)
        self.shape = (n, c, h, w, k)
        src = torch.from_numpy(d["src"]).to(dev).to(tdt)
        mv = torch.from_numpy(d["mv"]).to(dev)
        self.truth = (torch.from_numpy(d["truth"]).to(dev).to(tdt)
                      if d.get("truth") is not None else None)
        # frame 0 as the host drew it, for the CPU leg's error figures
        self.frame0 = {"src32": d["src"][0].copy(), "mv": d["mv"][0].copy(),
                       "gout32": upstream_gradient(GRAD_SEED, (k, c, h, w))}
        gen = torch.Generator(device=dev).manual_seed(1234)
        self.sets = []
        for i in range(sets):
            s = {
                "src": src if i == 0 else src.clone(),
                "mv": mv if i == 0 else mv.clone(),
                "out": torch.empty((n, k, c, h, w), dtype=tdt, device=dev),
                "mask": torch.empty((n, k, h, w), dtype=torch.uint8, device=dev),
                "count": torch.empty((n, k), dtype=torch.int32, device=dev),
                # upstream gradient dL/d out (stands in for a loss gradient)
                "gout": torch.randn((n, k, c, h, w), device=dev, generator=gen).to(tdt),
                "gsrc": torch.empty((n, c, h, w), dtype=tdt, device=dev),
                "gmv": torch.empty((n, 2, h, w), dtype=torch.float32, device=dev),
            }
            nb = exw.exw_warp_backward_workspace_bytes(tdt, n, c, h, w)
            s["ws"] = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
            self.sets.append(s)
        self.sets[0]["gout"][0].copy_(torch.from_numpy(self.frame0["gout32"]).to(dev).to(tdt))
        del d
        self.b = 4 if dtype == "f32" else 2
        self.fwd_bytes, self.bwd_bytes = algorithmic_bytes(n, c, h, w, k, self.b)
        self.out_px = n * k * h * w
        self.np = np

    def name(self):
        n, c, h, w, k = self.shape
        return f"config{self.spec.index}: {n}x{w}x{h} C={c} K={k} {self.dtype}"

    def run(self, steps, warmup, recorded=True):
        """Time forward + backward steps. recorded: the training pair (the
        forward records the adjoint's footprint, the adjoint skips that pass);
        else the standalone calls."""
        import paper_2307_12607_amd as exw
        torch = self.torch
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]

        def step(i, ev=None):
            s = self.sets[i % len(self.sets)]
            if ev:
                ev[0].record()
            if recorded:
                exw.exw_warp_forward_batched_record(s["src"], s["mv"], self.phases, s["out"],
                                                    s["ws"], s["mask"], s["count"])
            else:
                exw.exw_warp_forward_batched(s["src"], s["mv"], self.phases, s["out"], s["mask"],
                                             s["count"])
            if ev:
                ev[1].record()
            exw.exw_warp_backward_batched(s["src"], s["mv"], self.phases, s["gout"], s["gsrc"],
                                          s["gmv"], s["ws"], recorded=recorded)
            if ev:
                ev[2].record()

        for i in range(warmup):
            step(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(warmup + i, evs[i])
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        fwd_each = sorted(e[0].elapsed_time(e[1]) for e in evs)
        bwd_each = sorted(e[1].elapsed_time(e[2]) for e in evs)
        fwd_ms = sum(fwd_each) / steps
        bwd_ms = sum(bwd_each) / steps
        ms = 1e3 * elapsed / steps

        def spread(xs):  # median, min, max of the per-step event times (ms)
            return [round(xs[len(xs) // 2], 4), round(xs[0], 4), round(xs[-1], 4)]

        return {
            "ms_per_step": ms,
            "fwd_ms": fwd_ms,
            "bwd_ms": bwd_ms,
            "fwd_ms_median_min_max": spread(fwd_each),
            "bwd_ms_median_min_max": spread(bwd_each),
            "mpix_s": self.out_px / (ms * 1e-3) / 1e6,
            "fwd_mpix_s": self.out_px / (fwd_ms * 1e-3) / 1e6,
            "fwd_gbs": self.fwd_bytes / (fwd_ms * 1e-3) / 1e9,
            "bwd_gbs": self.bwd_bytes / (bwd_ms * 1e-3) / 1e9,
        }

    def capture_frame0(self):
        """Frame 0 of buffer set 0 after a timed run (the step's outputs for the
        host-drawn upstream gradient), for the CPU leg's error figures."""
        torch = self.torch
        torch.cuda.synchronize()
        s = self.sets[0]
        f = lambda t: t[0].detach().float().cpu().numpy()
        self.frame0.update({
            "src_stored": f(s["src"]), "gout_stored": f(s["gout"]), "out": f(s["out"]),
            "mask": s["mask"][0].cpu().numpy(), "count": s["count"][0].cpu().numpy(),
            "gsrc": f(s["gsrc"]), "gmv": f(s["gmv"])})
        return self.frame0

    def run_motion_stats(self, reps=20):
        """Per-frame motion mean/variance (one read of the motion planes)."""
        import paper_2307_12607_amd as exw
        torch = self.torch
        n, c, h, w, k = self.shape
        nb = exw.exw_motion_stats_workspace_bytes(n, h, w)
        ws = torch.empty(nb, dtype=torch.uint8, device=self.sets[0]["mv"].device)
        out = torch.empty((n, 4), dtype=torch.float64, device=ws.device)
        for i in range(3):
            exw.exw_motion_stats(self.sets[i % len(self.sets)]["mv"], out, ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(reps):
            exw.exw_motion_stats(self.sets[i % len(self.sets)]["mv"], out, ws)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        gbs = 8 * n * h * w / (us * 1e-6) / 1e9

        # The same statistics folded by the recording forward from its own
        # motion read: the forward's time with and without them, alternated.
        s = self.sets[0]

        def rec(stats):
            exw.exw_warp_forward_batched_record(s["src"], s["mv"], self.phases, s["out"],
                                                s["ws"], s["mask"], s["count"],
                                                motion_stats=stats)
        fused = {None: [], "stats": []}
        for _ in range(3):
            for key, stats in ((None, None), ("stats", out)):
                for _ in range(3):
                    rec(stats)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(reps):
                    rec(stats)
                e1.record()
                torch.cuda.synchronize()
                fused[key].append(e0.elapsed_time(e1) / reps * 1e3)
        plain_us, with_us = min(fused[None]), min(fused["stats"])
        return {"workload": f"config{self.spec.index}: motion statistics of {n}x{w}x{h}",
                "us": round(us, 2), "alg_bytes": 8 * n * h * w, "gbs": round(gbs, 1),
                "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                "fused_in_recording_forward": {
                    "forward_us": round(plain_us, 2), "forward_with_stats_us": round(with_us, 2),
                    "extra_us": round(with_us - plain_us, 2)}}

    def run_quality_and_chain(self, reps=5):
        """Frame quality (MSE/PSNR/SSIM) of the N*K predicted frames against the
        scene's analytic frames at the same instants, and the K-step chained
        warp."""
        import paper_2307_12607_amd as exw
        torch = self.torch
        n, c, h, w, k = self.shape
        s0 = self.sets[0]
        exw.exw_warp_forward_batched(s0["src"], s0["mv"], self.phases, s0["out"], None, None)
        pred = s0["out"].reshape(n * k, c, h, w)
        truth = self.truth.reshape(n * k, c, h, w)
        nb = exw.exw_frame_quality_workspace_bytes(n * k, c, h, w)
        ws = torch.empty(nb, dtype=torch.uint8, device=pred.device)
        q = torch.empty((n * k, 3), dtype=torch.float64, device=pred.device)
        chain = torch.empty((k, n, c, h, w), dtype=pred.dtype, device=pred.device)

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps * 1e3

        q_us = timed(lambda: exw.exw_frame_quality(pred, truth, q, ws))
        qh = q.cpu().numpy().reshape(n, k, 3)
        ch_us = timed(lambda: exw.exw_warp_chain(s0["src"], s0["mv"], 0.25, k, chain))
        flops = n * k * c * (h - 10) * (w - 10) * ssim_flops_per_position()
        per_phase = {f"{s:g}": {"psnr_db_mean": round(float(qh[:, j, 1].mean()), 3),
                                "psnr_db_min": round(float(qh[:, j, 1].min()), 3),
                                "ssim_mean": round(float(qh[:, j, 2].mean()), 5)}
                     for j, s in enumerate(self.phases)}
        return ({"workload": f"config{self.spec.index}: MSE/PSNR/SSIM of the {n * k} predicted "
                             f"frames {w}x{h} C={c} {self.dtype} against the scene's analytic "
                             f"frames at t + phase",
                 "us": round(q_us, 1), "bound": "alu",
                 "fp64_flops_per_position": round(ssim_flops_per_position(), 1),
                 "fp64_gflop_s": round(flops / (q_us * 1e-6) / 1e9, 1),
                 "peak_fp64_gflop_s": FP64_VECTOR_PEAK_GFLOPS,
                 "frac": round(flops / (q_us * 1e-6) / 1e9 / FP64_VECTOR_PEAK_GFLOPS, 4),
                 "quality_by_phase": per_phase},
                {"workload": f"config{self.spec.index}: {k} chained quarter-step warps "
                             f"of {n}x{w}x{h} C={c} {self.dtype}",
                 "us": round(ch_us, 1),
                 "direct_fwd_phases_us": None})

    def free(self):
        self.sets = []
        self.truth = None
        self.torch.cuda.empty_cache()


def buffer_emd_line(dev, reps=20):
    """The EMD features of the G-buffer workload (4 x 1440p): world normals
    (3 channels, bfloat16 storage, 256 bins on [-1, 1]) and world positions
    (3 channels, float32, 1024 bins on [-64, 128]) of frames 1..3 against
    frames 0..2 (algorithmic bytes: one read of both buffers); and N_D, the
    number of dynamic objects, of its 4 frames' custom stencil."""
    import numpy as np
    import torch
    import paper_2307_12607_amd as exw
    from synth import make_config, world_position

    d = make_config(5)
    g = d["src"]
    pos = world_position(g[:, 3], d["info"]["pan"])
    stencil = torch.from_numpy(d["stencil"]).to(dev)
    bufs = (("normals", torch.from_numpy(np.ascontiguousarray(g[:, 4:7])).to(dev).to(torch.bfloat16),
             -1.0, 1.0, 256),
            ("positions", torch.from_numpy(pos).to(dev), -64.0, 128.0, 1024))
    del d, g, pos
    out = {}
    for name, buf, lo, hi, bins in bufs:
        cur, prev = buf[1:], buf[:-1]
        n, c, h, w = cur.shape
        emd = torch.empty((n, c), dtype=torch.float64, device=dev)
        ws = torch.empty(exw.exw_buffer_emd_workspace_bytes(n, c, bins), dtype=torch.uint8,
                         device=dev)
        for _ in range(3):
            exw.exw_buffer_emd(cur, prev, lo, hi, bins, emd, ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            exw.exw_buffer_emd(cur, prev, lo, hi, bins, emd, ws)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        nbytes = 2 * cur.numel() * cur.element_size()
        out[name] = {"workload": f"config5: EMD of {n} frames {w}x{h} C={c} "
                                 f"{str(cur.dtype).replace('torch.', '')}, {bins} bins",
                     "us": round(us, 2), "alg_bytes": nbytes,
                     "gbs": round(nbytes / (us * 1e-6) / 1e9, 1),
                     "hbm_frac": round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "emd_sum_frame1": round(float(emd[0].sum()), 6)}
        del cur, prev, buf, emd, ws
    # N_D of the same frames: connected components of the custom stencil
    n, h, w = stencil.shape
    count = torch.empty((n,), dtype=torch.int32, device=dev)
    ws = torch.empty(exw.exw_dynamic_objects_workspace_bytes(n, h, w), dtype=torch.uint8,
                     device=dev)
    for _ in range(3):
        exw.exw_dynamic_objects(stencil, count, ws, 8)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        exw.exw_dynamic_objects(stencil, count, ws, 8)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / reps * 1e3
    out["dynamic_objects"] = {"workload": f"config5: N_D of {n} frames {w}x{h} (custom stencil, "
                                          f"8-connectivity)",
                              "us": round(us, 2), "gpix_s": round(n * h * w / (us * 1e-6) / 1e9, 1),
                              "n_d": count.cpu().tolist()}
    del stencil, count, ws
    torch.cuda.empty_cache()
    return out


def stream_ceilings(dev, nbytes=1 << 30, reps=10):
    """GB/s of the library's plain HBM streams on 1 GiB buffers: a copy (read +
    write counted), a read-only and a write-only sweep."""
    import torch
    import paper_2307_12607_amd as exw
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    sink = torch.zeros(1, dtype=torch.float32, device=dev)
    out = {}
    for name, moved, fn in (("copy_gbs", 2 * nbytes, lambda: exw.exw_stream_copy(a, b)),
                            ("read_gbs", nbytes, lambda: exw.exw_stream_read(a, sink)),
                            ("write_gbs", nbytes, lambda: exw.exw_stream_write(b))):
        fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / reps
        out[name] = round(moved / (ms * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------------ CPU leg

def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(index, budget_s=8.0):
    """The float64 C oracle (as it stands) on the host cores: forward + backward
    over a bounded sample of the same workload (its first frame), on one
    thread and on every thread OpenMP gives this process (its CPU share)."""
    import numpy as np
    from oracle import ref_c
    from synth import make_config

    d = make_config(index, n=1)
    s, m, ph = ref_c.prepare(d["src"], d["mv"], d["phases"])
    n, c, h, w = s.shape
    k = ph.size
    out = np.empty((n, k, c, h, w))
    mask = np.empty((n, k, h, w), np.uint8)
    cnt = np.empty((n, k), np.int64)
    g = np.random.default_rng(0).standard_normal((n, k, c, h, w))
    gs = np.empty_like(s)
    gm = np.empty((n, 2, h, w))

    def rate(threads):
        ref_c.set_threads(threads)
        reps = 0
        t0 = time.perf_counter()
        while True:
            ref_c.forward_prepared(s, m, ph, out, mask, cnt)
            ref_c.backward_prepared(s, m, ph, g, gs, gm)
            reps += 1
            if time.perf_counter() - t0 > budget_s or reps >= 50:
                break
        dt = (time.perf_counter() - t0) / reps
        return n * k * h * w / dt / 1e6, reps

    share = ref_c.max_threads()  # OMP_NUM_THREADS / the affinity mask of this process
    multi, reps_m = rate(share)
    single, reps_s = rate(1)
    ref_c.set_threads(share)
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"value": round(multi, 3), "unit": "Mpix/s", "cores": share, "kind": "oracle",
            "single_thread_value": round(single, 3),
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "affinity_cpus": affinity,
            "sample": f"float64 C oracle, forward+backward of frame 0 of the workload "
                      f"({w}x{h}, C={c}, K={k}): {reps_m} reps on {share} OpenMP threads "
                      f"(this process's CPU share), {reps_s} reps on 1 thread"}


def oracle_errors(frame0, phases, dtype):
    """Frame 0 of a timed step against the float64 C oracle on the same stored
    inputs (kernel-only), against the oracle's exact displacement mode, and
    for 16-bit storage end to end against the oracle on the float32 frame."""
    import numpy as np
    from oracle import ref_c

    f = frame0
    src = f["src_stored"][None].astype(np.float64)
    mv = f["mv"][None]
    ref, rmask, rcnt = ref_c.forward(src, mv, phases)
    got = f["out"][None].astype(np.float64)
    res = {"frame": 0,
           "fwd_max_abs": float(np.abs(got - ref).max()),
           "mask_mismatches": int((f["mask"][None] != rmask).sum()),
           "count_mismatches": int((f["count"][None].astype(np.int64) != rcnt).sum())}
    del ref
    ex, emask, _ = ref_c.forward(src, mv, phases, exact=True)
    both = (f["mask"][None] == 1) & (emask == 1)
    res["exact_mode"] = {
        "fwd_max_abs": float((np.abs(got - ex) * both[:, :, None]).max()),
        "mask_mismatches": int((f["mask"][None] != emask).sum())}
    del ex
    if dtype != "f32":
        e2e, _, _ = ref_c.forward(f["src32"][None].astype(np.float64), mv, phases)
        res["fwd_e2e_max_abs"] = float(np.abs(got - e2e).max())
        del e2e
    gs, gm = ref_c.backward(src, mv, phases, f["gout_stored"][None].astype(np.float64))
    for name, g_gpu, g_ref in (("grad_src", f["gsrc"][None], gs), ("grad_mv", f["gmv"][None], gm)):
        diff = np.abs(g_gpu.astype(np.float64) - g_ref)
        res[f"{name}_max_abs"] = float(diff.max())
        res[f"{name}_max_rel"] = float((diff / np.maximum(1.0, np.abs(g_ref))).max())
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the warp's frames and "
              "phases are independent, so N GPUs would each run this same step on their own "
              "batch.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2307_12607_amd as exw  # fails loudly if the HIP library is missing

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        a = torch.ones((1 << 30) // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            exw.exw_stream_copy(a, b)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()

    main_wl = Workload(args.config, args.dtype, dev, with_truth=args.config in (2, 3, 5))
    r = main_wl.run(args.steps, args.warmup)
    captured = [(main_wl.name(), main_wl.phases, args.dtype, main_wl.capture_frame0())]
    # the same calls without the recorded footprint (an adjoint called on its own)
    alone = main_wl.run(max(5, args.steps // 3), 2, recorded=False)
    n, c, h, w, k = main_wl.shape
    dominant = "warp_backward" if r["bwd_ms"] >= r["fwd_ms"] else "warp_forward"
    dom_ms = r["bwd_ms"] if dominant == "warp_backward" else r["fwd_ms"]
    dom_bytes = main_wl.bwd_bytes if dominant == "warp_backward" else main_wl.fwd_bytes
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    wl_name = main_wl.name()
    traffic = load_traffic(dominant, wl_name)
    stats_line = None if args.only_step else main_wl.run_motion_stats()
    quality_line = chain_line = None
    if main_wl.truth is not None and not args.only_step:
        quality_line, chain_line = main_wl.run_quality_and_chain()
        chain_line["direct_fwd_phases_us"] = round(r["fwd_ms"] * 1e3, 1)
    main_wl.free()

    variants = []
    if not args.no_variants:
        todo = [(args.config, "f16" if args.dtype == "f32" else "f32")]
        if args.config == 2:
            # 4K RGBA; 8 x 1080p RGB with s = 1 (the loss-gradient workload: the
            # upstream gradient is a precomputed tensor, the loss is not timed);
            # 4 x 1440p 12-channel G-buffers in bf16 and f32 storage
            todo += [(3, "f32"), (3, "f16"), (4, "f32"), (5, "bf16"), (5, "f32")]
        for idx, dt in todo:
            wl = Workload(idx, dt, dev)
            vr = wl.run(max(5, args.steps // 3), 2)
            captured.append((wl.name(), wl.phases, dt, wl.capture_frame0()))
            variants.append({"workload": wl.name(), "fwd_bwd_mpix_s": round(vr["mpix_s"], 1),
                             "fwd_mpix_s": round(vr["fwd_mpix_s"], 1),
                             "fwd_ms": round(vr["fwd_ms"], 4), "bwd_ms": round(vr["bwd_ms"], 4),
                             "fwd_ms_median_min_max": vr["fwd_ms_median_min_max"],
                             "bwd_ms_median_min_max": vr["bwd_ms_median_min_max"],
                             "fwd_hbm_frac": round(vr["fwd_gbs"] / HBM_PEAK_GBS, 4),
                             "bwd_hbm_frac": round(vr["bwd_gbs"] / HBM_PEAK_GBS, 4)})
            wl.free()

    emd_line = None if args.no_variants or args.only_step else buffer_emd_line(dev)
    ceilings = None if args.only_step else stream_ceilings(dev)
    cpu = None
    errors = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.config)
        errors = {name: oracle_errors(f0, ph, dt) for name, ph, dt, f0 in captured}
    del captured

    rec = {
        "metric": "Mpix/s warp fwd+bwd (output pixels per second)",
        "value": round(r["mpix_s"], 1),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": wl_name, "frames": n, "channels": c, "height": h, "width": w,
                   "phases": k, "storage": args.dtype, "motion": "fp32"},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "frac_of_measured_copy": (round(achieved / ceilings["copy_gbs"], 4)
                                               if ceilings else None)},
        "cpu_baseline": cpu,
        "errors": errors,
        "breakdown": {"fwd_ms": round(r["fwd_ms"], 4), "bwd_ms": round(r["bwd_ms"], 4),
                      "fwd_ms_median_min_max": r["fwd_ms_median_min_max"],
                      "bwd_ms_median_min_max": r["bwd_ms_median_min_max"],
                      "fwd_mpix_s": round(r["fwd_mpix_s"], 1),
                      "fwd_gbs": round(r["fwd_gbs"], 1), "bwd_gbs": round(r["bwd_gbs"], 1),
                      "fwd_hbm_frac": round(r["fwd_gbs"] / HBM_PEAK_GBS, 4),
                      "fwd_alg_bytes": main_wl.fwd_bytes, "bwd_alg_bytes": main_wl.bwd_bytes,
                      "hbm_ceilings_measured": ceilings,
                      "step": "forward recording the adjoint's footprint + adjoint from it",
                      "standalone_calls": {"fwd_ms": round(alone["fwd_ms"], 4),
                                           "bwd_ms": round(alone["bwd_ms"], 4),
                                           "fwd_bwd_mpix_s": round(alone["mpix_s"], 1)}},
        "variants": variants,
        "motion_stats": stats_line,
        "buffer_emd": emd_line,
        "frame_quality": quality_line,
        "warp_chain": chain_line,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
