"""Binding of libhh_probe.so, the measurement utilities (include/hh_probe.h):
the issue-rate probe behind the arithmetic roofline's denominators and the
barrier floor of the network time loop.  They are not part of the method
and live in their own library, next to libhh.so."""
from __future__ import annotations

import ctypes
import os

import torch

from .hh import _ok, _ptr, _stream

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhh_probe.so")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhh_probe.so is not built (%s); run python -m "
                          "paper_2601_21407_amd.build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    i32, sz, vp = ctypes.c_int32, ctypes.c_size_t, ctypes.c_void_p
    L.hh_probe_issue.argtypes = [i32, i32, i32, vp, i32, vp]
    L.hh_probe_issue.restype = i32
    L.hh_probe_barrier_bytes.argtypes = [i32]
    L.hh_probe_barrier_bytes.restype = sz
    L.hh_probe_barrier.argtypes = [i32, i32, i32, vp, sz, vp]
    L.hh_probe_barrier.restype = i32
    return L


lib = _load()

PROBE_OPS = {"fma": 0, "exp2": 1, "rcp": 2, "sqrt": 3, "sin": 4, "mul64": 5, "mix": 6,
             "pkfma16": 7, "exp16": 8, "mfma16": 9, "mfma16_valu": 10}


def probe_issue(op: str, iters: int, blocks: int, out):
    """Launch the issue-rate probe; blocks * 256 * 8 * iters operations of
    kind `op`."""
    _ok(lib.hh_probe_issue(PROBE_OPS[op], int(iters), int(blocks), _ptr(out), int(out.numel()),
                           _stream()), "hh_probe_issue")


def probe_barrier(steps: int, blocks: int, mode: int, work=None):
    """Launch the barrier-floor probe; returns the work buffer for reuse."""
    need = int(lib.hh_probe_barrier_bytes(int(blocks)))
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.uint8, device="cuda")
    _ok(lib.hh_probe_barrier(int(steps), int(blocks), int(mode), _ptr(work), work.numel(),
                             _stream()), "hh_probe_barrier")
    return work
