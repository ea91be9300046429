"""Host-side logic of bench.py (no GPU): the one-GPU contract, the algorithmic
byte counts the roofline figure is built on, and the device-code key of the
traffic counters."""

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


def test_device_code_key_and_traffic_lookup():
    sha = bench.device_code_sha()
    assert sha is None or (len(sha) == 16 and all(ch in "0123456789abcdef" for ch in sha))
    t = bench.load_traffic("warp_backward", "config2: 8x1920x1080 C=4 K=3 f32")
    assert t is None or (isinstance(t, int) and t > 0)
    assert bench.load_traffic("no_such_kernel", "no workload") is None
