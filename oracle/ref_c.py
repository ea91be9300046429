"""ctypes wrapper of the C float64 oracle (test infrastructure only).

Same definition as ``warp_oracle`` (paper §II-B, §III-B, §III-D, §IV-B), as
plain scalar loops; see ``warp_ref.c``.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        i64 = ctypes.c_int64
        p = ctypes.c_void_p
        L.warp_ref_forward.argtypes = [p, p, i64, i64, i64, i64, p, i64, p, p, p, ctypes.c_int]
        L.warp_ref_forward.restype = ctypes.c_int
        L.warp_ref_backward.argtypes = [p, p, i64, i64, i64, i64, p, i64, p, p, p, ctypes.c_int]
        L.warp_ref_backward.restype = ctypes.c_int
        L.warp_ref_max_threads.restype = ctypes.c_int
        L.warp_ref_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    lib().warp_ref_set_threads(int(n))


def max_threads() -> int:
    return int(lib().warp_ref_max_threads())


def prepare(src, mv, phases):
    """Dense float64 src, float32 mv and phases, as the C oracle takes them."""
    return (np.ascontiguousarray(np.asarray(src).astype(np.float64)),
            np.ascontiguousarray(mv, dtype=np.float32),
            np.ascontiguousarray(np.asarray(phases, dtype=np.float32).reshape(-1)))


def forward(src, mv, phases, exact: bool = False):
    """Returns ``(out [N,K,C,H,W] f64, mask [N,K,H,W] u8, invalid_count [N,K] i64)``.

    ``exact``: the displacement s*u exactly (float64), else rounded once to
    float32 (see ``warp_ref.c``)."""
    s, m, ph = prepare(src, mv, phases)
    n, c, h, w = s.shape
    k = ph.size
    out = np.empty((n, k, c, h, w), dtype=np.float64)
    mask = np.empty((n, k, h, w), dtype=np.uint8)
    cnt = np.empty((n, k), dtype=np.int64)
    rc = lib().warp_ref_forward(_ptr(s), _ptr(m), n, c, h, w, _ptr(ph), k, _ptr(out), _ptr(mask),
                                _ptr(cnt), int(bool(exact)))
    if rc != 0:
        raise ValueError("warp_ref_forward rejected its arguments")
    return out, mask, cnt


def forward_prepared(s, m, ph, out, mask, cnt, exact: bool = False):
    """Forward on already-converted buffers (used to time the oracle alone)."""
    n, c, h, w = s.shape
    rc = lib().warp_ref_forward(_ptr(s), _ptr(m), n, c, h, w, _ptr(ph), ph.size, _ptr(out),
                                _ptr(mask), _ptr(cnt), int(bool(exact)))
    if rc != 0:
        raise ValueError("warp_ref_forward rejected its arguments")


def backward(src, mv, phases, grad_out, exact: bool = False):
    """Returns ``(grad_src [N,C,H,W] f64, grad_mv [N,2,H,W] f64)``."""
    s, m, ph = prepare(src, mv, phases)
    g = np.ascontiguousarray(np.asarray(grad_out).astype(np.float64))
    n, c, h, w = s.shape
    gs = np.empty_like(s)
    gm = np.empty((n, 2, h, w), dtype=np.float64)
    backward_prepared(s, m, ph, g, gs, gm, exact)
    return gs, gm


def backward_prepared(s, m, ph, g, gs, gm, exact: bool = False):
    n, c, h, w = s.shape
    if g.shape != (n, ph.size, c, h, w):
        raise ValueError("grad_out shape mismatch")
    rc = lib().warp_ref_backward(_ptr(s), _ptr(m), n, c, h, w, _ptr(ph), ph.size, _ptr(g),
                                 _ptr(gs), _ptr(gm), int(bool(exact)))
    if rc != 0:
        raise ValueError("warp_ref_backward rejected its arguments")
