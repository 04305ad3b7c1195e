"""The paper's tiled CPU algorithm (Sec. 3, Algorithm 2), for comparison with the GPU kernels.

A separate library (``libdd_cpu.so``, plain C + OpenMP); nothing in the GPU
path calls it.  It takes the plan's FP64-derived integer shift table and
computes the same exact sums as the GPU kernels.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "cpu", "tiled.c")
LIB = os.path.join(_HERE, "libdd_cpu.so")
_lib = None

#: Default tiles (D_t samples, D_dm trials, D_f channels): the best of a small sweep on 8192-channel
#: 8-bit rows (64 trials, 2^18 samples) on an 8-core host.
DEFAULT_TILES = (4096, 32, 128)


def build() -> str:
    """Compile libdd_cpu.so with gcc (-O3, OpenMP, run-time AVX-512/AVX2 dispatch)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError("libdd_cpu.so is not built: run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        lib.dd_cpu_tiled_forward_u8.argtypes = [vp, i64, i32, vp, i32, i64, vp, i64, i32, i32, i32]
        lib.dd_cpu_tiled_forward_u8.restype = i32
        _lib = lib
    return _lib


def forward_u8(x: np.ndarray, shift: np.ndarray, n_out: int, tiles=DEFAULT_TILES) -> np.ndarray:
    """float32 [n_dm][n_out]: the transform of 8-bit rows x [n_chan][>= n_out + max shift]."""
    lib = _load()
    assert x.dtype == np.uint8 and x.ndim == 2 and x.flags.c_contiguous
    sh = np.ascontiguousarray(shift, dtype=np.int32)
    n_dm, n_chan = sh.shape
    assert x.shape[0] == n_chan and x.shape[1] >= n_out + int(sh.max()) and int(sh.min()) >= 0
    out = np.empty((n_dm, n_out), dtype=np.float32)
    d_t, d_dm, d_f = tiles
    rc = lib.dd_cpu_tiled_forward_u8(x.ctypes.data, x.shape[1], n_chan, sh.ctypes.data, n_dm, n_out,
                                     out.ctypes.data, out.shape[1], d_t, d_dm, d_f)
    if rc != 0:
        raise ValueError("dd_cpu_tiled_forward_u8 failed (%d)" % rc)
    return out
