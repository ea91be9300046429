"""Host-side logic of bench.py (no GPU): the one-GPU contract, the algorithmic
byte counts the roofline figure is built on, and the per-kernel code key of
the traffic counters (with the profile summariser's kernel names)."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_of_the_main_workload():
    # 8 x 1920 x 1080 RGBA float32, three phases. Forward: source, motion,
    # outputs, masks once each, plus the N*K uint32 invalid counts; adjoint:
    # upstream gradient, source, motion, image and motion gradients.
    n, c, h, w, k, b = 8, 4, 1080, 1920, 3, 4
    px = n * h * w
    fwd, bwd = bench.algorithmic_bytes(n, c, h, w, k, b)
    assert fwd == px * (c * b + 8) + px * k * (c * b + 1) + 4 * n * k
    assert bwd == px * k * c * b + px * (c * b + 8 + c * b + 8)
    assert (fwd, bwd) == (1244160096, 1592524800)
    # 16-bit storage halves the frame terms only
    f16, b16 = bench.algorithmic_bytes(n, c, h, w, k, 2)
    assert f16 == px * (c * 2 + 8) + px * k * (c * 2 + 1) + 4 * n * k
    assert b16 == px * k * c * 2 + px * (c * 2 + 8 + c * 2 + 8)


def _lib():
    import paper_2307_12607_amd._capi as capi
    return capi.LIB_PATH


def test_code_objects_and_kernel_symbols_of_the_library():
    objs = bench.code_objects(_lib())
    assert len(objs) >= 5  # one per translation unit with device code
    syms = {}
    for o in objs:
        assert o[:4] == b"\x7fELF"
        syms.update(bench.elf_symbols(o))
    tiles = [n for n in syms if "adjoint_tiles_kernelIfLi4ELi3E" in n and not n.endswith(".kd")]
    assert len(tiles) == 1 and tiles[0] + ".kd" in syms
    assert len(syms[tiles[0] + ".kd"]) == 64  # an AMDGPU kernel descriptor


def test_kernel_code_key_and_traffic_lookup():
    syms = {}
    for o in bench.code_objects(_lib()):
        syms.update(bench.elf_symbols(o))
    names = sorted(n for n in syms if ("adjoint_tiles_kernelIfLi4ELi3E" in n
                                       or "adjoint_far_kernelIfLi4ELi3E" in n)
                   and not n.endswith(".kd"))
    sha = bench.kernel_code_sha(names, _lib())
    assert len(sha) == 16 and all(ch in "0123456789abcdef" for ch in sha)
    assert bench.kernel_code_sha(list(reversed(names)), _lib()) == sha  # order-free
    assert bench.kernel_code_sha(names[:1], _lib()) != sha
    assert bench.kernel_code_sha(names + ["_Z_no_such_kernel"], _lib()) is None
    t = bench.load_traffic("warp_backward", "config2: 8x1920x1080 C=4 K=3 f32")
    assert t is None or (isinstance(t, int) and t > 0)
    assert bench.load_traffic("no_such_call", "no workload") is None


def test_profile_names_match_symbols():
    import bench_traffic as bt
    assert bt.key("void exw::(anonymous namespace)::adjoint_tiles_kernel<float, 4, 3>"
                  "(exw::(anonymous namespace)::BwdArgs<float>)") == "exw::adjoint_tiles_kernel<float, 4, 3>"
    # the profiler leaves the 16-bit instantiations mangled; both sides read them alike
    m = "_ZN3exw12_GLOBAL__N_120adjoint_tiles_kernelIDF16bLi12ELi1EEEvNS0_7BwdArgsIT_EE"
    assert bt.demangle([m]) == ["exw::adjoint_tiles_kernel<__bf16, 12, 1>"]
    keys = bt.symbols_by_key()
    assert keys["exw::adjoint_tiles_kernel<__bf16, 12, 1>"] == m
    assert "exw::warp_forward_kernel<half, 4, 3, true, false>" in keys
    assert "exw::stream_copy_kernel" in keys


def _counter_csv(path, counter, rows):
    """A rocprofv3 counter-collection CSV with the columns the summariser reads."""
    import csv
    cols = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
            "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
            "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
            "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(cols)
        for i, (name, value) in enumerate(rows, 1):
            w.writerow([i, i, "Agent 1", 1, 1, 1, 64, 1, name, 256, 0, 0, 8, 0, 16, counter, value,
                        0, 1])


def test_traffic_summary_scales_by_the_copy(tmp_path):
    import json
    import bench_traffic as bt
    tiles = "void exw::(anonymous namespace)::adjoint_tiles_kernel<float, 4, 3>(exw::(anonymous namespace)::BwdArgs<float>)"
    far = "void exw::(anonymous namespace)::adjoint_far_kernel<float, 4, 3>(exw::(anonymous namespace)::BwdArgs<float>, float*)"
    copy = "void exw::(anonymous namespace)::stream_copy_kernel(float __vector(4) const*, float __vector(4)*, long)"
    # the copy of 1 GiB reads FETCH = 512 Ki KiB (half of its bytes) and WRITE = 1 Mi KiB;
    # two dispatches of the tile kernel average 1000 KiB fetched
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE",
                 [(copy, 524288.0), (tiles, 900.0), (tiles, 1100.0), (far, 10.0)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE",
                 [(copy, 1048576.0), (tiles, 300.0), (tiles, 300.0), (far, 0.0)])
    js = tmp_path / "t.json"
    import sys
    argv = sys.argv
    sys.argv = ["bench_traffic.py", "traffic", "--workload", "wl", "--fetch", str(tmp_path / "f.csv"),
                "--write", str(tmp_path / "w.csv"), "--summary", str(tmp_path / "s.txt"),
                "--json", str(js), "--command", "x"]
    try:
        bt.main()
    finally:
        sys.argv = argv
    e = json.loads(js.read_text())["calls"]["warp_backward|wl"]
    assert e["fetch_scale"] == 2.0 and e["write_scale"] == 1.0
    assert e["fetch_bytes_per_launch"] == round((1000.0 + 10.0) * 1024 * 2)
    assert e["write_bytes_per_launch"] == round(300.0 * 1024)
    assert e["hbm_bytes_per_launch"] == e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]
    assert len(e["kernels"]) == 2 and all(k.startswith("_Z") for k in e["kernels"])
    assert e["code_sha"] == bench.kernel_code_sha(e["kernels"], _lib())


def test_request_summary_applies_littles_law(tmp_path):
    """Reads in flight per CU = summed read latency / (256 caches * kernel
    cycles), the kernel cycles being GRBM_GUI_ACTIVE over the 8 XCDs; the
    mean latency = summed latency / reads. Two dispatches are averaged."""
    import csv
    import bench_traffic as bt
    fwd = "void exw::(anonymous namespace)::warp_forward_kernel<float, 4, 3, true, false>(exw::(anonymous namespace)::FwdArgs<float>)"
    cols = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
            "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
            "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
            "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    # dispatch 1: 1000 cycles per XCD, 2e6 reads of 500 cycles each; dispatch 2: the
    # same cycles, 4e6 reads of 500 cycles (the latency counter is split over two rows)
    per = {1: {"GRBM_GUI_ACTIVE": [8000.0], "TCP_TCC_READ_REQ_sum": [2e6],
               "TCP_TCC_READ_REQ_LATENCY_sum": [1e9], "TCP_TCC_WRITE_REQ_sum": [1e6],
               "TCP_TOTAL_CACHE_ACCESSES_sum": [5e6]},
           2: {"GRBM_GUI_ACTIVE": [8000.0], "TCP_TCC_READ_REQ_sum": [4e6],
               "TCP_TCC_READ_REQ_LATENCY_sum": [1.5e9, 0.5e9], "TCP_TCC_WRITE_REQ_sum": [3e6],
               "TCP_TOTAL_CACHE_ACCESSES_sum": [5e6]}}
    path = tmp_path / "r.csv"
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(cols)
        for disp, ctrs in per.items():
            for ctr, values in ctrs.items():
                for v in values:
                    w.writerow([disp, disp, "Agent 1", 1, 1, 1, 64, 1, fwd, 256, 0, 0, 8, 0, 16,
                                ctr, v, 0, 1])
    import sys
    argv = sys.argv
    sys.argv = ["bench_traffic.py", "requests", "--workload", "wl", "--csv", str(path),
                "--summary", str(tmp_path / "s.txt"), "--command", "x"]
    try:
        bt.main()
    finally:
        sys.argv = argv
    line = next(l for l in (tmp_path / "s.txt").read_text().splitlines()
                if l.startswith("exw::warp_forward_kernel"))
    reads, writes, latency, in_flight = (float(v) for v in line.split()[-4:])
    assert reads == 3.0 and writes == 2.0          # millions, mean of the two dispatches
    assert latency == 500.0                        # 1.5e9 / 3e6
    assert abs(in_flight - 1.5e9 / (256 * 1000.0)) < 0.05
