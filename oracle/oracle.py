"""ctypes front end of the C oracle (``oracle.c``) -- TEST INFRASTRUCTURE.

Builds ``liboracle.so`` with gcc (FP64, no FMA contraction, OpenMP) and exposes
the shift table (Eq. 1 with the per-channel form of Sec. 4.1), the forward
transform (Eq. 3 / Algorithm 1), the scatter-form adjoint, time binning and the
input corner turn.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

#: Dispersion constant in s MHz^2 cm^3 / pc (Eq. 1; the value 4.148808e3 is the
#: reading taken for the garbled constant printed with Eq. 1).
KDM = 4.148808e3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def lib_path() -> str:
    return _LIB


def build() -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (always recompiles)."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def compile_source(src: str, out: str) -> str:
    """Compile C source text with the oracle's flags into a shared library at ``out``."""
    tmp_c = out + ".c"
    with open(tmp_c, "w") as fh:
        fh.write(src)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", tmp_c, "-o", out, "-lm"], check=True)
    return out


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()


def use_library(path):
    """Point the front end at another build of the oracle (None restores the default).

    Used only by the tests that plant a mistake in a copy of the oracle and
    check that the pins catch it.
    """
    global _lib
    _lib = None if path is None else _configure(ctypes.CDLL(path))


def _gpu_started() -> bool:
    """True once this process has initialised a GPU through torch (no compiler may be started then)."""
    import sys
    torch = sys.modules.get("torch")
    return bool(torch is not None and torch.cuda.is_initialized())


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        if _gpu_started():
            raise RuntimeError("liboracle.so is missing or older than oracle.c: run oracle.build() "
                               "(or __graft_entry__.build()) before using a GPU in this process")
        build()
    _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def _configure(lib):
    i32, i64, dbl, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.oracle_shift_table.argtypes = [i32, dbl, dbl, vp, dbl, dbl, dbl, i32, vp]
    lib.oracle_shift_table.restype = i32
    lib.oracle_forward_int.argtypes = [i32, vp, i64, i32, i64, vp, i32, i64, vp, i32, vp]
    lib.oracle_forward_int.restype = i32
    lib.oracle_forward_f32.argtypes = [vp, i64, i32, i64, vp, i32, i64, vp, i32, vp, vp]
    lib.oracle_forward_f32.restype = i32
    lib.oracle_adjoint_f64.argtypes = [vp, i64, i32, i64, vp, i32, i64, vp]
    lib.oracle_adjoint_f64.restype = i32
    lib.oracle_bin_int.argtypes = [i32, vp, i64, i32, i64, i32, vp, i64]
    lib.oracle_bin_int.restype = i32
    lib.oracle_bin_f32.argtypes = [vp, i64, i32, i64, i32, vp, i64]
    lib.oracle_bin_f32.restype = i32
    lib.oracle_corner_turn.argtypes = [i32, vp, i64, i32, i64, vp, i64]
    lib.oracle_corner_turn.restype = i32
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def shift_table(n_chan, f_high, chan_bw, t_samp, dm_start, dm_step, n_dm, freqs=None):
    """int32 [n_dm][n_chan] shift table, in samples (Eq. 1 / Sec. 4.1)."""
    lib = _load()
    out = np.empty((n_dm, n_chan), dtype=np.int32)
    fp = None
    if freqs is not None:
        freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        assert freqs.shape == (n_chan,)
        fp = _ptr(freqs)
    rc = lib.oracle_shift_table(n_chan, float(f_high), float(chan_bw), fp, float(t_samp),
                                float(dm_start), float(dm_step), n_dm, _ptr(out))
    if rc != 0:
        raise ValueError("shift table out of range (non-positive frequency or int32 overflow)")
    return out


def n_out_for(shift: np.ndarray, n_samp: int) -> int:
    """Number of valid output samples, N_t minus the largest shift."""
    return int(n_samp) - int(shift.max())


def _rows_arg(rows, n_dm):
    if rows is None:
        return None, n_dm
    r = np.ascontiguousarray(rows, dtype=np.int32)
    return r, len(r)


def forward(x: np.ndarray, dtype: str, n_samp: int, shift: np.ndarray, rows=None) -> np.ndarray:
    """Forward transform of integer input; float32 [len(rows)][n_out].

    x is uint8 [n_chan][pitch]; for dtype "u4" the pitch is in bytes and holds
    two samples per byte, the even sample in the low nibble.  For dtype "u16"
    x is uint16 [n_chan][pitch] (little-endian samples), for "u32" uint32
    (time-binned 16-bit data).
    """
    lib = _load()
    assert x.ndim == 2 and x.flags.c_contiguous
    n_dm, n_chan = shift.shape
    assert x.shape[0] == n_chan
    code = {"u8": 1, "u4": 2, "u16": 4, "u32": 5}[dtype]
    if code == 4:
        assert x.dtype == np.uint16 and x.shape[1] >= n_samp
        x = x.astype("<u2", copy=False).view(np.uint8)
    elif code == 5:
        assert x.dtype == np.uint32 and x.shape[1] >= n_samp
        x = x.astype("<u4", copy=False).view(np.uint8)
    else:
        assert x.dtype == np.uint8
    if code == 1:
        assert x.shape[1] >= n_samp
    elif code == 2:
        assert n_samp % 2 == 0 and x.shape[1] >= n_samp // 2
    n_out = n_out_for(shift, n_samp)
    r, nr = _rows_arg(rows, n_dm)
    out = np.empty((nr, max(n_out, 0)), dtype=np.float32)
    sh = np.ascontiguousarray(shift, dtype=np.int32)
    rc = lib.oracle_forward_int(code, _ptr(x), x.shape[1], n_chan, n_samp, _ptr(sh), n_dm, n_out,
                                None if r is None else _ptr(r), nr, _ptr(out))
    if rc != 0:
        raise ValueError("oracle forward: bad arguments")
    return out


def forward_f32(x: np.ndarray, n_samp: int, shift: np.ndarray, rows=None, with_abs=True):
    """Forward transform of float32 input in FP64: (sum, sum of |terms|)."""
    lib = _load()
    assert x.dtype == np.float32 and x.ndim == 2 and x.flags.c_contiguous
    n_dm, n_chan = shift.shape
    assert x.shape[0] == n_chan and x.shape[1] >= n_samp
    n_out = n_out_for(shift, n_samp)
    r, nr = _rows_arg(rows, n_dm)
    # NaN-filled, so that a sum the C code fails to start from zero cannot pass for one
    out = np.full((nr, max(n_out, 0)), np.nan, dtype=np.float64)
    ab = np.full_like(out, np.nan) if with_abs else None
    sh = np.ascontiguousarray(shift, dtype=np.int32)
    rc = lib.oracle_forward_f32(_ptr(x), x.shape[1], n_chan, n_samp, _ptr(sh), n_dm, n_out,
                                None if r is None else _ptr(r), nr, _ptr(out),
                                None if ab is None else _ptr(ab))
    if rc != 0:
        raise ValueError("oracle forward_f32: bad arguments")
    return out, ab


def adjoint(y: np.ndarray, n_chan: int, n_samp: int, shift: np.ndarray) -> np.ndarray:
    """Scatter-form adjoint in FP64: float64 [n_chan][n_samp]."""
    lib = _load()
    assert y.dtype == np.float32 and y.ndim == 2 and y.flags.c_contiguous
    n_dm = shift.shape[0]
    assert shift.shape[1] == n_chan and y.shape[0] == n_dm
    n_out = n_out_for(shift, n_samp)
    assert y.shape[1] >= n_out
    g = np.empty((n_chan, n_samp), dtype=np.float64)
    sh = np.ascontiguousarray(shift, dtype=np.int32)
    rc = lib.oracle_adjoint_f64(_ptr(y), y.shape[1], n_chan, n_samp, _ptr(sh), n_dm, n_out, _ptr(g))
    if rc != 0:
        raise ValueError("oracle adjoint: bad arguments")
    return g


def bin_time(x: np.ndarray, dtype: str, n_samp: int, factor: int) -> np.ndarray:
    """Time binning by ``factor``: sums of ``factor`` consecutive samples, trailing partial bin dropped.

    Integer input (uint8 for "u8"/"u4", uint16 for "u16") gives int64 [n_chan][n_samp // factor];
    float32 input gives float64 sums.
    """
    lib = _load()
    assert x.ndim == 2 and x.flags.c_contiguous
    n_chan = x.shape[0]
    n_bins = n_samp // factor
    if dtype == "f32":
        assert x.dtype == np.float32 and x.shape[1] >= n_samp
        out = np.empty((n_chan, max(n_bins, 1)), dtype=np.float64)
        rc = lib.oracle_bin_f32(_ptr(x), x.shape[1], n_chan, n_samp, factor, _ptr(out), out.shape[1])
    else:
        code = {"u8": 1, "u4": 2, "u16": 4}[dtype]
        if code == 4:
            assert x.dtype == np.uint16 and x.shape[1] >= n_samp
            x = x.astype("<u2", copy=False).view(np.uint8)
        else:
            assert x.dtype == np.uint8
            assert x.shape[1] >= (n_samp + 1) // 2 if code == 2 else x.shape[1] >= n_samp
        out = np.empty((n_chan, max(n_bins, 1)), dtype=np.int64)
        rc = lib.oracle_bin_int(code, _ptr(x), x.shape[1], n_chan, n_samp, factor, _ptr(out), out.shape[1])
    if rc != 0:
        raise ValueError("oracle bin: bad arguments")
    return out[:, :n_bins]


_CT_CODE = {"u8": 1, "u4": 2, "f32": 3, "u16": 4}
_CT_ES = {"u8": 1, "u16": 2, "f32": 4}


def corner_turn(spectra: np.ndarray, dtype: str, n_chan: int, n_samp: int) -> np.ndarray:
    """Time-major spectra [n_samp][>= row] to channel-major rows [n_chan][row] (see oracle.c).

    u8/u16/f32: element transpose; u4: channel pairs per byte in, time pairs per byte out."""
    lib = _load()
    assert spectra.ndim == 2 and spectra.flags.c_contiguous and spectra.shape[0] >= n_samp
    raw = spectra.view(np.uint8)
    if dtype == "u4":
        out = np.empty((n_chan, n_samp // 2), dtype=np.uint8)
        ob = out
    else:
        dt = {"u8": np.uint8, "u16": np.dtype("<u2"), "f32": np.float32}[dtype]
        assert spectra.dtype == dt
        out = np.empty((n_chan, n_samp), dtype=dt)
        ob = out.view(np.uint8)
    rc = lib.oracle_corner_turn(_CT_CODE[dtype], _ptr(raw), raw.shape[1], n_chan, n_samp, _ptr(ob), ob.shape[1])
    if rc != 0:
        raise ValueError("oracle corner turn: bad arguments")
    return out

