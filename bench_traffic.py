#!/usr/bin/env python3
"""Summaries of rocprofv3 runs of bench.py, for `profiles/`.

Two subcommands, each reading the CSV files rocprofv3 wrote:

  trace   --stats <run_kernel_stats.csv> --summary <txt> --command "<cmd>"
      per-kernel calls and average / min / max duration of a
      `rocprofv3 --kernel-trace --stats` run.

  traffic --workload "<bench workload name>" --fetch <FETCH_SIZE csv>
          --write <WRITE_SIZE csv> --summary <txt> --json <traffic json>
          --command "<fetch cmd>" --command "<write cmd>"
      HBM bytes per library call from two `rocprofv3 --pmc` runs of the same
      bench command with --copy-calibration. Each counter is scaled by what it
      reads for the library's plain copy of 1 GiB (stream_copy_kernel: 1 GiB
      read, 1 GiB written), then summed over the call's kernels:
        warp_forward  = the recording forward kernel + frame_reach_kernel
        warp_backward = adjoint_tiles_kernel + adjoint_far_kernel
                        (+ cast_far_frames_kernel)
      The json entry names the kernels' symbols and the hash of their code
      (bench.kernel_code_sha); bench.py reports the traffic only while the
      built library still holds those kernels unchanged.

  counters --workload "<name>" --csv <counter csv> [--csv ...] --summary <txt>
           --command "<cmd>" [--command ...]
      per-kernel figures from `rocprofv3 --pmc` runs of three counter sets
      (TCC_HIT_sum TCC_MISS_sum | SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES
      SQ_INSTS_VALU SQ_INSTS_VMEM_RD SQ_INSTS_SALU SQ_INSTS_LDS
      SQ_LDS_BANK_CONFLICT | TA_TA_BUSY_sum TD_TD_BUSY_sum GRBM_GUI_ACTIVE
      SQ_ACTIVE_INST_VALU), means over dispatches. SQ, TA, TD and GRBM
      counters are summed over the device (8 XCDs, 256 CUs, 1024 SIMDs):
        kernel cycles  = GRBM_GUI_ACTIVE / 8
        L2 hit rate    = TCC_HIT / (TCC_HIT + TCC_MISS)
        VALU busy      = 4 * SQ_INSTS_VALU / (1024 * cycles)   (a wave64 VALU
                         instruction holds a SIMD for 4 cycles)
        TA, TD busy    = TA_TA_BUSY, TD_TD_BUSY / (256 * cycles)
        waves / SIMD   = 4 * SQ_WAVE_CYCLES / (1024 * cycles)  (SQ_WAVE_CYCLES
                         counts in units of 4 cycles)
      with the kernel's VGPRs (from its descriptor) and workgroup size.

  requests --workload "<name>" --csv <counter csv> --summary <txt> --command "<cmd>"
      per-kernel L1-to-L2 requests from one `rocprofv3 --pmc` run of
      TCP_TCC_READ_REQ_sum TCP_TCC_READ_REQ_LATENCY_sum TCP_TCC_WRITE_REQ_sum
      TCP_TOTAL_CACHE_ACCESSES_sum GRBM_GUI_ACTIVE, means over dispatches:
        mean read latency (cycles)  = TCP_TCC_READ_REQ_LATENCY / TCP_TCC_READ_REQ
        reads in flight per CU      = TCP_TCC_READ_REQ_LATENCY / (256 * cycles)
      (the latency counter sums every read's cycles over the device's 256
      vector L1 caches, so by Little's law it is the mean number of reads
      outstanding times the cycles elapsed).

Symbol names are matched to the profiler's kernel names with c++filt.
"""

from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (code-object parsing and the hash bench.py checks)

LIB = os.path.join(ROOT, "paper_2307_12607_amd", "libexwarp.so")
KIB = 1024
GIB = 1 << 30

CALLS = {
    "warp_forward": [r"^exw::warp_forward_kernel<.*, true, false>$", r"^exw::frame_reach_kernel$"],
    "warp_backward": [r"^exw::adjoint_tiles_kernel<", r"^exw::adjoint_far_kernel<",
                      r"^exw::cast_far_frames_kernel<"],
}


def key(name: str) -> str:
    """A kernel's name without return type, anonymous namespace or parameters."""
    name = name.replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    depth = 0
    for i, ch in enumerate(name):  # cut at the parameter list (outside template brackets)
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def demangle(names):
    """c++filt over mangled names. The 16-bit floating types' codes (DF16_ for
    _Float16, DF16b for __bf16), which this c++filt and the profiler leave
    mangled, are first given the codes of `half` and of a vendor type
    `__bf16`, so such kernels read e.g. adjoint_tiles_kernel<half, 4, 3>."""
    subst = [n.replace("DF16_", "Dh").replace("DF16b", "u6__bf16") if n.startswith("_Z") else n
             for n in names]
    out = subprocess.run(["c++filt"], input="\n".join(subst), capture_output=True, text=True,
                         check=True).stdout.splitlines()
    return [key(d) for d in out]


def symbols_by_key():
    """{kernel key: mangled symbol} of every kernel function in the library."""
    names = set()
    for obj in bench.code_objects(LIB):
        names.update(n for n in bench.elf_symbols(obj) if n.startswith("_Z")
                     and not n.endswith(".kd"))
    names = sorted(names)
    return dict(zip(demangle(names), names))


def load_counter(path):
    """{kernel key: [value per dispatch]} of one counter CSV (values summed
    over the rows of a dispatch)."""
    per = collections.defaultdict(float)
    names = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            per[d] += float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
    raw = sorted(set(names.values()))
    keys = dict(zip(raw, demangle(raw)))
    out = collections.defaultdict(list)
    for d, v in per.items():
        out[keys[names[d]]].append(v)
    return out


def mean(xs):
    return sum(xs) / len(xs)


def cmd_trace(a):
    rows = []
    with open(a.stats) as f:
        for r in csv.DictReader(f):
            rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                         float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                         float(r["Percentage"])))
    names = demangle([r[0] for r in rows])
    rows = [(n,) + r[1:] for n, r in zip(names, rows)]
    rows.sort(key=lambda r: -r[1] * r[2])
    with open(a.summary, "w") as f:
        f.write(f"# rocprofv3 kernel trace: {a.title}\n")
        for c in a.command:
            f.write(f"# command: {c}\n")
        f.write(f"\n{'kernel':76s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} "
                f"{'max_us':>9s} {'%time':>6s}\n")
        for k, calls, avg, lo, hi, pct in rows:
            f.write(f"{k[:76]:76s} {calls:6d} {avg:9.1f} {lo:9.1f} {hi:9.1f} {pct:6.2f}\n")
    print(open(a.summary).read())


def cmd_traffic(a):
    fetch = load_counter(a.fetch)
    write = load_counter(a.write)
    copy = "exw::stream_copy_kernel"
    if copy not in fetch or copy not in write:
        sys.exit("no stream_copy_kernel dispatch: run the bench with --copy-calibration")
    fetch_scale = (GIB / KIB) / mean(fetch[copy])
    write_scale = (GIB / KIB) / mean(write[copy])
    syms = symbols_by_key()
    try:
        with open(a.json) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    rec.setdefault("calls", {})
    lines = []
    for call, pats in CALLS.items():
        ks = sorted(k for k in fetch if any(re.search(p, k) for p in pats))
        if not ks:
            continue
        fb = sum(mean(fetch[k]) for k in ks) * KIB * fetch_scale
        wb = sum(mean(write.get(k, [0.0])) for k in ks) * KIB * write_scale
        mangled = [syms[k] for k in ks]
        rec["calls"][f"{call}|{a.workload}"] = {
            "kernels": mangled, "code_sha": bench.kernel_code_sha(mangled, LIB),
            "fetch_bytes_per_launch": round(fb), "write_bytes_per_launch": round(wb),
            "hbm_bytes_per_launch": round(fb + wb), "fetch_scale": round(fetch_scale, 4),
            "write_scale": round(write_scale, 4)}
        lines.append(f"{call:14s} fetch {fb / 1e6:9.1f} MB  write {wb / 1e6:9.1f} MB  "
                     f"total {(fb + wb) / 1e6:9.1f} MB   kernels: {', '.join(ks)}")
    with open(a.json, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    with open(a.summary, "w") as f:
        f.write(f"# HBM traffic per call from rocprofv3 counters, {a.workload}\n")
        for c in a.command:
            f.write(f"# command: {c}\n")
        f.write(f"# calibration: the library's copy of 1 GiB reads FETCH_SIZE="
                f"{mean(fetch[copy]):.0f} KiB and WRITE_SIZE={mean(write[copy]):.0f} KiB, "
                f"so FETCH is scaled by {fetch_scale:.3f} and WRITE by {write_scale:.3f}\n\n")
        f.write("\n".join(lines) + "\n\n")
        f.write(f"{'kernel':76s} {'fetch_MB':>10s} {'write_MB':>10s}  (per dispatch, scaled)\n")
        for k in sorted(fetch):
            fm = mean(fetch[k]) * KIB * fetch_scale / 1e6
            wm = mean(write.get(k, [0.0])) * KIB * write_scale / 1e6
            f.write(f"{k[:76]:76s} {fm:10.2f} {wm:10.2f}\n")
    print(open(a.summary).read())


_KD = None


def vgprs(kernel_key):
    """(VGPRs used, VGPRs allocated) of a kernel from its descriptor: the
    accumulation offset (compute_pgm_rsrc3 bits 5:0, in units of 4) ends the
    architectural VGPRs, and compute_pgm_rsrc1 bits 5:0 hold the allocation
    in granules of 8, minus one."""
    global _KD
    if _KD is None:
        syms = {}
        for obj in bench.code_objects(LIB):
            syms.update(bench.elf_symbols(obj))
        _KD = {k: syms.get(m + ".kd") for k, m in symbols_by_key().items()}
    kd = _KD.get(kernel_key)
    if not kd or len(kd) < 64:
        return None
    rsrc3 = int.from_bytes(kd[44:48], "little")
    rsrc1 = int.from_bytes(kd[48:52], "little")
    return ((rsrc3 & 0x3F) + 1) * 4, ((rsrc1 & 0x3F) + 1) * 8


def cmd_counters(a):
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    res = {}
    raw_names = set()
    rows = []
    for path in a.csv:
        per = collections.defaultdict(float)
        meta = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                d = (path, int(r["Dispatch_Id"]), r["Counter_Name"])
                per[d] += float(r["Counter_Value"])
                meta[d] = r
        for (p, disp, ctr), v in per.items():
            r = meta[(p, disp, ctr)]
            rows.append((r["Kernel_Name"], ctr, v))
            raw_names.add(r["Kernel_Name"])
            res[r["Kernel_Name"]] = (int(r["VGPR_Count"]), int(r["LDS_Block_Size"]),
                                     int(r["Workgroup_Size"]))
    keys = dict(zip(sorted(raw_names), demangle(sorted(raw_names))))
    for name, ctr, v in rows:
        vals[keys[name]][ctr].append(v)
    out = [f"# rocprofv3 counters per dispatch (mean over dispatches), {a.workload}"]
    out += [f"# command: {c}" for c in a.command]
    out.append("# SQ/TA/TD/GRBM counters summed over the device (8 XCDs, 256 CUs, 1024 "
               "SIMDs); definitions in bench_traffic.py")
    for k in sorted(vals, key=lambda k: -mean(vals[k].get("GRBM_GUI_ACTIVE", [0.0]))):
        if not k.startswith("exw::"):
            continue
        m = {c: mean(v) for c, v in vals[k].items()}
        _, _, wg = next(res[n] for n in raw_names if keys[n] == k)
        out.append(f"\n{k}")
        regs = vgprs(k)
        if regs:
            out.append(f"  VGPRs (descriptor: used, allocated; waves/SIMD they allow)   "
                       f"{regs[0]}, {regs[1]}; {min(8, 512 // regs[1])}")
        out.append(f"  workgroup size                 {wg}")
        cyc = m.get("GRBM_GUI_ACTIVE", 0.0) / 8.0
        if "TCC_HIT_sum" in m:
            hit, miss = m["TCC_HIT_sum"], m["TCC_MISS_sum"]
            out.append(f"  L2 hit rate                    {hit / max(hit + miss, 1.0):.3f}   "
                       f"(hits {hit / 1e6:.2f} M, misses {miss / 1e6:.2f} M)")
        if cyc:
            out.append(f"  kernel cycles (per XCD)        {cyc / 1e6:.3f} M")
            if "SQ_INSTS_VALU" in m:
                out.append(f"  VALU busy                      "
                           f"{4 * m['SQ_INSTS_VALU'] / (1024 * cyc):.3f}")
            out.append(f"  TA busy / TD busy              {m['TA_TA_BUSY_sum'] / (256 * cyc):.3f}"
                       f" / {m['TD_TD_BUSY_sum'] / (256 * cyc):.3f}")
            if "SQ_WAVE_CYCLES" in m:
                out.append(f"  mean resident waves / SIMD     "
                           f"{4 * m['SQ_WAVE_CYCLES'] / (1024 * cyc):.2f}")
        for c in ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD",
                  "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT"):
            if c in m:
                out.append(f"  {c:30s} {m[c] / 1e6:.3f} M")
    with open(a.summary, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


def per_kernel_means(paths):
    """{kernel key: {counter: mean over dispatches}} of counter CSV files (a
    dispatch's rows summed per counter)."""
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    raw = set()
    rows = []
    for path in paths:
        per = collections.defaultdict(float)
        names = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                d = (int(r["Dispatch_Id"]), r["Counter_Name"])
                per[d] += float(r["Counter_Value"])
                names[d] = r["Kernel_Name"]
        for (disp, ctr), v in per.items():
            rows.append((names[(disp, ctr)], ctr, v))
            raw.add(names[(disp, ctr)])
    keys = dict(zip(sorted(raw), demangle(sorted(raw))))
    for name, ctr, v in rows:
        vals[keys[name]][ctr].append(v)
    return {k: {c: mean(v) for c, v in m.items()} for k, m in vals.items()}


def cmd_requests(a):
    means = per_kernel_means(a.csv)
    out = [f"# rocprofv3 L1-to-L2 requests per dispatch (mean over dispatches), {a.workload}"]
    out += [f"# command: {c}" for c in a.command]
    out.append("# summed over the device's 256 vector L1 caches; definitions in bench_traffic.py")
    out.append(f"\n{'kernel':76s} {'reads':>9s} {'writes':>9s} {'read latency':>13s} "
               f"{'reads in flight':>16s}")
    out.append(f"{'':76s} {'(M)':>9s} {'(M)':>9s} {'(cycles)':>13s} {'(per CU)':>16s}")
    for k in sorted(means, key=lambda k: -means[k].get("GRBM_GUI_ACTIVE", 0.0)):
        if not k.startswith("exw::"):
            continue
        m = means[k]
        cyc = m["GRBM_GUI_ACTIVE"] / 8.0
        rd, lat = m["TCP_TCC_READ_REQ_sum"], m["TCP_TCC_READ_REQ_LATENCY_sum"]
        out.append(f"{k[:76]:76s} {rd / 1e6:9.2f} {m['TCP_TCC_WRITE_REQ_sum'] / 1e6:9.2f} "
                   f"{lat / max(rd, 1.0):13.0f} {lat / (256 * cyc):16.1f}")
    with open(a.summary, "w") as f:
        f.write("\n".join(out) + "\n")
    print("\n".join(out))


def main():
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--stats", required=True)
    t.add_argument("--summary", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--command", action="append", default=[])
    r = sub.add_parser("traffic")
    r.add_argument("--workload", required=True)
    r.add_argument("--fetch", required=True)
    r.add_argument("--write", required=True)
    r.add_argument("--summary", required=True)
    r.add_argument("--json", default=bench.TRAFFIC_FILE)
    r.add_argument("--command", action="append", default=[])
    c = sub.add_parser("counters")
    c.add_argument("--workload", required=True)
    c.add_argument("--csv", action="append", required=True)
    c.add_argument("--summary", required=True)
    c.add_argument("--command", action="append", default=[])
    q = sub.add_parser("requests")
    q.add_argument("--workload", required=True)
    q.add_argument("--csv", action="append", required=True)
    q.add_argument("--summary", required=True)
    q.add_argument("--command", action="append", default=[])
    a = p.parse_args()
    {"trace": cmd_trace, "traffic": cmd_traffic, "counters": cmd_counters,
     "requests": cmd_requests}[a.cmd](a)


if __name__ == "__main__":
    main()
