"""Seeded synthetic filterbanks shaped like the paper's workloads.

The only input source shared by the CPU oracle (through the tests and the
benchmark's CPU-baseline leg) and the GPU library.  It holds none of the
transform's arithmetic: pulse injection takes the per-channel delays of the
pulse's DM from the caller.  These stand in for the SIGPROC ``fake`` files the
paper generated its test signals with (Sec. 5), which are not available.

Recipe:

* 8-bit and 4-bit samples come from a counter-based generator (``gen_common.h``):
  SplitMix64's output function over a per-row counter, 16 bits per sample, so
  any time slice of any row can be produced on its own, on the CPU (``gen.c``)
  or directly in GPU memory (``gen.hip``), with identical bytes.
* 8-bit Gaussian noise N(mean, sigma), rounded to nearest and clipped to
  0..255, is the 16-bit draw looked up in a quantile table:
  ``clip(rint(mean + sigma * Phi^-1((i + 0.5) / 65536)), 0, 255)``.
* 4-bit noise: uniform 0..15 (the low 4 bits of the draw), two samples per
  byte, the even sample in the low nibble.
* float noise: standard normal float32, one ``PCG64(SeedSequence([seed, c]))``
  stream per channel row.
* Pulses: a boxcar of amplitude A and width W starting at arrival time t0 at
  the top of the band, added at ``x[c][t0 + k + delay[c]]`` for k < W and
  clipped at 255, after the noise.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_CPU_LIB = os.path.join(_HERE, "libsynth_cpu.so")
_GPU_LIB = os.path.join(_HERE, "libsynth_gpu.so")
_cpu = None
_gpu = None


def build(gpu: bool = True) -> None:
    """Compile the CPU generator (gcc) and, if asked, the GPU generator (hipcc, gfx950)."""
    tmp = _CPU_LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                    os.path.join(_HERE, "gen.c"), "-o", tmp], check=True)
    os.replace(tmp, _CPU_LIB)
    if gpu:
        tmp = _GPU_LIB + ".tmp%d" % os.getpid()
        subprocess.run(["hipcc", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        os.path.join(_HERE, "gen.hip"), "-o", tmp],
                       check=True, stderr=subprocess.DEVNULL)
        os.replace(tmp, _GPU_LIB)


def _cpu_lib():
    global _cpu
    if _cpu is None:
        src = os.path.join(_HERE, "gen.c")
        if not os.path.exists(_CPU_LIB) or os.path.getmtime(_CPU_LIB) < os.path.getmtime(src):
            torch = sys.modules.get("torch")
            if torch is not None and torch.cuda.is_initialized():  # no compiler after GPU start
                raise RuntimeError("libsynth_cpu.so is missing or stale: run synth.build() first")
            build(gpu=False)
        lib = ctypes.CDLL(_CPU_LIB)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
        lib.synth_u8_table.argtypes = [vp, i32, i64, i64, u64, i64, vp]
        lib.synth_u8_table.restype = None
        lib.synth_u4_packed.argtypes = [vp, i32, i64, i64, u64, i64]
        lib.synth_u16_table.argtypes = [vp, i32, i64, i64, u64, i64, vp]
        lib.synth_u16_table.restype = None
        lib.synth_u4_packed.restype = None
        _cpu = lib
    return _cpu


def _gpu_lib():
    global _gpu
    if _gpu is None:
        if not os.path.exists(_GPU_LIB):
            raise RuntimeError("synthetic GPU generator not built: run synth.build()")
        lib = ctypes.CDLL(_GPU_LIB)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
        lib.synth_u8_table_gpu.argtypes = [vp, i32, i64, i64, u64, i64, vp, vp]
        lib.synth_u8_table_gpu.restype = i32
        lib.synth_u4_packed_gpu.argtypes = [vp, i32, i64, i64, u64, i64, vp]
        lib.synth_u16_table_gpu.argtypes = [vp, i32, i64, i64, u64, i64, vp, vp]
        lib.synth_u16_table_gpu.restype = ctypes.c_int
        lib.synth_u4_packed_gpu.restype = i32
        _gpu = lib
    return _gpu


@lru_cache(maxsize=8)
def gaussian_table(mean: float = 128.0, sigma: float = 16.0) -> np.ndarray:
    """uint8[65536] quantile table of N(mean, sigma), rounded to nearest, clipped to 0..255."""
    from scipy.special import ndtri
    p = (np.arange(65536, dtype=np.float64) + 0.5) / 65536.0
    v = np.clip(np.rint(mean + sigma * ndtri(p)), 0.0, 255.0)
    return v.astype(np.uint8)


def gaussian_u8(n_chan: int, n_samp: int, seed: int, mean: float = 128.0, sigma: float = 16.0,
                pitch: int | None = None, t_start: int = 0) -> np.ndarray:
    """uint8 [n_chan][pitch]: samples t_start .. t_start + n_samp - 1 of every row; padding is 0."""
    pitch = n_samp if pitch is None else pitch
    assert pitch >= n_samp and n_chan > 0 and n_samp > 0
    out = np.zeros((n_chan, pitch), dtype=np.uint8)
    table = gaussian_table(mean, sigma)
    _cpu_lib().synth_u8_table(out.ctypes.data, n_chan, n_samp, pitch, seed, t_start, table.ctypes.data)
    return out


def gaussian_table16(mean: float = 32768.0, sigma: float = 4096.0) -> np.ndarray:
    """uint16[65536] quantile table of N(mean, sigma), rounded to nearest, clipped to 0..65535."""
    from scipy.special import ndtri
    p = (np.arange(65536, dtype=np.float64) + 0.5) / 65536.0
    v = np.clip(np.rint(mean + sigma * ndtri(p)), 0.0, 65535.0)
    return v.astype(np.uint16)


def gaussian_u16(n_chan: int, n_samp: int, seed: int, mean: float = 32768.0, sigma: float = 4096.0,
                 pitch: int | None = None, t_start: int = 0) -> np.ndarray:
    """uint16 [n_chan][pitch] (pitch in samples): the same draws as gaussian_u8 through a 16-bit table."""
    pitch = n_samp if pitch is None else pitch
    assert pitch >= n_samp and n_chan > 0 and n_samp > 0
    out = np.zeros((n_chan, pitch), dtype=np.uint16)
    table = gaussian_table16(mean, sigma)
    _cpu_lib().synth_u16_table(out.ctypes.data, n_chan, n_samp, pitch, seed, t_start, table.ctypes.data)
    return out


def gaussian_u16_device(ptr: int, n_chan: int, n_samp: int, pitch: int, seed: int, table_ptr: int,
                        stream: int = 0, t_start: int = 0) -> None:
    """Fill device memory at ``ptr`` exactly as :func:`gaussian_u16` would (16-bit table on the device)."""
    rc = _gpu_lib().synth_u16_table_gpu(ptr, n_chan, n_samp, pitch, seed, t_start, table_ptr, stream)
    if rc != 0:
        raise RuntimeError("synth_u16_table_gpu failed (%d)" % rc)


def uniform_u4_packed(n_chan: int, n_samp: int, seed: int, pitch_bytes: int | None = None,
                      t_start: int = 0) -> np.ndarray:
    """uint8 [n_chan][pitch_bytes]: uniform 0..15 samples, two per byte, even sample low."""
    assert n_samp % 2 == 0 and t_start % 2 == 0
    pb = n_samp // 2 if pitch_bytes is None else pitch_bytes
    assert pb >= n_samp // 2
    out = np.zeros((n_chan, pb), dtype=np.uint8)
    _cpu_lib().synth_u4_packed(out.ctypes.data, n_chan, n_samp, pb, seed, t_start)
    return out


def gaussian_u8_device(ptr: int, n_chan: int, n_samp: int, pitch: int, seed: int, table_ptr: int,
                       stream: int = 0, t_start: int = 0) -> None:
    """Fill device memory at ``ptr`` exactly as :func:`gaussian_u8` would (table on the device)."""
    rc = _gpu_lib().synth_u8_table_gpu(ptr, n_chan, n_samp, pitch, seed, t_start, table_ptr, stream)
    if rc != 0:
        raise RuntimeError("synth_u8_table_gpu failed (%d)" % rc)


def uniform_u4_device(ptr: int, n_chan: int, n_samp: int, pitch_bytes: int, seed: int,
                      stream: int = 0, t_start: int = 0) -> None:
    rc = _gpu_lib().synth_u4_packed_gpu(ptr, n_chan, n_samp, pitch_bytes, seed, t_start, stream)
    if rc != 0:
        raise RuntimeError("synth_u4_packed_gpu failed (%d)" % rc)


def unpack_u4(packed: np.ndarray, n_samp: int) -> np.ndarray:
    """Inverse of the 4-bit packing: uint8 [n_chan][n_samp] of values 0..15."""
    out = np.empty((packed.shape[0], n_samp), dtype=np.uint8)
    out[:, 0::2] = packed[:, : n_samp // 2] & 15
    out[:, 1::2] = packed[:, : n_samp // 2] >> 4
    return out


def normal_f32(n_chan: int, n_samp: int, seed: int, pitch: int | None = None) -> np.ndarray:
    """float32 [n_chan][pitch] standard-normal noise, one PCG64 stream per row; padding 0."""
    pitch = n_samp if pitch is None else pitch
    out = np.zeros((n_chan, pitch), dtype=np.float32)
    for c in range(n_chan):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), c])))
        out[c, :n_samp] = rng.standard_normal(n_samp, dtype=np.float32)
    return out


def boxcar_updates(x_at, delay: np.ndarray, t0: int, width: int, amp: int, top: int = 255):
    """Positions and new values of a dispersed boxcar pulse, clipped at ``top`` (255 for 8-bit).

    ``x_at(rows, cols)`` returns the current uint8 values at those positions
    (from a host array, or regenerated from the counter generator).  Returns
    (rows, cols, new_values, applied) where applied[c][k] is the increment that
    survived clipping; its column sums are the exact gain of the dedispersed
    pulse at its DM.
    """
    n_chan = delay.shape[0]
    rows = np.repeat(np.arange(n_chan, dtype=np.int64), width)
    cols = (t0 + delay.astype(np.int64)[:, None] + np.arange(width, dtype=np.int64)[None, :]).reshape(-1)
    before = np.asarray(x_at(rows, cols), dtype=np.int64)
    after = np.minimum(before + amp, top)
    applied = (after - before).reshape(n_chan, width)
    return rows, cols, after.astype(np.uint8 if top <= 255 else np.uint16), applied


def inject_boxcar_u8(x: np.ndarray, delay: np.ndarray, t0: int, width: int, amp: int) -> np.ndarray:
    """Add a dispersed boxcar to a host array (uint8 or uint16) in place; returns the applied increments."""
    top = 65535 if x.dtype == np.uint16 else 255
    rows, cols, vals, applied = boxcar_updates(lambda r, c: x[r, c], delay, t0, width, amp, top)
    x[rows, cols] = vals
    return applied


#: The workloads: shapes, bands, DM plans and seeds.  Channel c sits at
#: f_high - c * chan_bw.  Pulses are (dm_index, width, t0).
CONFIGS = {
    "small": dict(dtype="u8", n_chan=128, n_samp=32768, f_high=1500.0, chan_bw=1.5625,
                  t_samp=64e-6, dm_start=0.0, dm_step=1.0, n_dm=256, seed=1,
                  pulses=[(100, 4, 8000)], amp=40),
    "headline": dict(dtype="u8", n_chan=8192, n_samp=1 << 20, f_high=1500.0, chan_bw=300.0 / 8192,
                     t_samp=64e-6, dm_start=0.0, dm_step=0.5, n_dm=4000, seed=2,
                     pulses=[(100, 1, 100_000), (600, 2, 280_000), (1600, 4, 460_000),
                             (3000, 8, 640_000), (3800, 16, 820_000)], amp=40),
    # One GPU's share of the headline under 8-way DM sharding: the last of eight
    # 500-DM slices (the largest delays), with the headline's DM-1900 pulse.
    "headline_shard8": dict(dtype="u8", n_chan=8192, n_samp=1 << 20, f_high=1500.0, chan_bw=300.0 / 8192,
                            t_samp=64e-6, dm_start=1750.0, dm_step=0.5, n_dm=500, seed=2,
                            pulses=[(300, 16, 820_000)], amp=40),
    "lowfreq_u4": dict(dtype="u4", n_chan=4096, n_samp=1 << 19, f_high=190.0, chan_bw=70.0 / 4096,
                       t_samp=327.68e-6, dm_start=0.0, dm_step=0.1, n_dm=2048, seed=3,
                       pulses=[], amp=0),
    # The headline plan on packed 4-bit input (two samples per byte), for the
    # 4-bit against 8-bit comparison on one plan.
    "headline_u4": dict(dtype="u4", n_chan=8192, n_samp=1 << 20, f_high=1500.0, chan_bw=300.0 / 8192,
                        t_samp=64e-6, dm_start=0.0, dm_step=0.5, n_dm=4000, seed=7,
                        pulses=[], amp=0),
    "headline_u16": dict(dtype="u16", n_chan=8192, n_samp=1 << 20, f_high=1500.0, chan_bw=300.0 / 8192,
                         t_samp=64e-6, dm_start=0.0, dm_step=0.5, n_dm=4000, seed=6,
                         pulses=[(100, 1, 100_000), (1600, 4, 460_000), (3800, 16, 820_000)], amp=2560),
    # Large delay spread: 264 samples more delay per DM step at the band bottom,
    # too wide for LDS staging to pay; runs on the direct-read kernel.
    "lowfreq_wide": dict(dtype="u8", n_chan=4096, n_samp=1 << 20, f_high=190.0, chan_bw=70.0 / 4096,
                         t_samp=327.68e-6, dm_start=0.0, dm_step=0.5, n_dm=1024, seed=10,
                         pulses=[(200, 2, 100_000), (700, 4, 400_000)], amp=40),
    # The same plan on 16-bit samples (the direct kernel's 16-bit form).
    "lowfreq_wide_u16": dict(dtype="u16", n_chan=4096, n_samp=1 << 20, f_high=190.0, chan_bw=70.0 / 4096,
                             t_samp=327.68e-6, dm_start=0.0, dm_step=0.5, n_dm=1024, seed=11,
                             pulses=[(200, 2, 100_000), (700, 4, 400_000)], amp=2560),
    "grad_f32": dict(dtype="f32", n_chan=1024, n_samp=1 << 17, f_high=1500.0, chan_bw=300.0 / 1024,
                     t_samp=128e-6, dm_start=0.0, dm_step=1.0, n_dm=1024, seed=4,
                     target_seed=40, fd_seed=41, pulses=[], amp=0),
}


#: Multi-range DM plans over one filterbank: ranges are (dm_start, dm_step,
#: n_dm, time-binning factor); pulses are (DM, width in samples, t0), injected
#: along the unbinned delays of that DM.
#:   survey_small    a small mixed plan for exhaustive parity (factors 1, 2, 4 and 3).
#:   tab_plans_8192  the three-range plan of Table tab:plans (Sec. 5.2): 10 s at
#:                   64 us, 1400 MHz centre, 300 MHz band, 8192 channels, no binning.
#:   pipeline_high   the "High" pipeline case of Sec. 5.3 (1400 MHz centre, 300 MHz
#:                   band, 64 us, 4096 channels, ~50 s, DM 0-3000): the three ranges
#:                   above, then ranges binned by 2, 4 and 8 whose step doubles with
#:                   the factor (about 3.6 binned samples of band-edge delay per step).
SURVEYS = {
    "survey_small": dict(dtype="u8", n_chan=128, n_samp=32770, f_high=1500.0, chan_bw=1.5625, t_samp=64e-6,
                         ranges=[(0.0, 1.0, 100, 1), (100.0, 2.0, 60, 2), (220.0, 4.0, 40, 4), (380.0, 3.0, 30, 3)],
                         seed=9, pulses=[(50.0, 2, 9000), (300.0, 4, 15000)], amp=40),
    "tab_plans_8192": dict(dtype="u8", n_chan=8192, n_samp=156250, f_high=1550.0, chan_bw=300.0 / 8192,
                           t_samp=64e-6, ranges=[(0.0, 0.1, 1500, 1), (150.0, 0.2, 750, 1), (300.0, 0.25, 800, 1)],
                           seed=7, pulses=[(75.0, 1, 40_000), (250.0, 2, 80_000), (450.0, 4, 120_000)], amp=40),
    "pipeline_high": dict(dtype="u8", n_chan=4096, n_samp=781250, f_high=1550.0, chan_bw=300.0 / 4096,
                          t_samp=64e-6, ranges=[(0.0, 0.1, 1500, 1), (150.0, 0.2, 750, 1), (300.0, 0.25, 800, 1),
                                                (500.0, 0.5, 1000, 2), (1000.0, 1.0, 1000, 4), (2000.0, 2.0, 500, 8)],
                          seed=8, pulses=[(100.0, 1, 100_000), (700.0, 2, 300_000), (1500.0, 4, 500_000),
                                          (2600.0, 8, 600_000)], amp=40),
}


def wide_beams(dtype: str = "u8", n_beams: int = 8, seed: int = 3):
    """Per-beam parameters of a batch of wide-spread beams (8 by default).

    Channel counts from {1024, 2048}, lengths uniform in [2^18, 2^19) rounded
    down to 64 samples, 256..1024 DM trials at step 0.5; 190 MHz top of a 70
    MHz band, 327.68 us sampling: a spread of ~4000 samples per 16 DM trials,
    too wide to stage, so every plan reads directly.  Beam b's data seed is
    600 + b.
    """
    rng = np.random.default_rng(seed)
    beams = []
    for b in range(n_beams):
        n_chan = int(rng.choice([1024, 2048]))
        n_samp = int(rng.integers(1 << 18, 1 << 19)) // 64 * 64
        n_dm = int(rng.integers(256, 1025))
        beams.append(dict(dtype=dtype, n_chan=n_chan, n_samp=n_samp, f_high=190.0, chan_bw=70.0 / n_chan,
                          t_samp=327.68e-6, dm_start=0.0, dm_step=0.5, n_dm=n_dm, seed=600 + b))
    return beams


def small_beams(dtype: str = "u8", n_beams: int = 64, seed: int = 4):
    """Per-beam parameters of a batch of many small beams (64 by default).

    Channel counts from {256, 512, 1024}, lengths uniform in [2^15, 2^17)
    rounded down to 64 samples, 64..512 DM trials with a step from {0.25, 0.5,
    1.0}; 1500 MHz top of a 300 MHz band, 64 us sampling (staged plans).  Beam
    b's data seed is 700 + b.
    """
    rng = np.random.default_rng(seed)
    beams = []
    for b in range(n_beams):
        n_chan = int(rng.choice([256, 512, 1024]))
        n_samp = int(rng.integers(1 << 15, 1 << 17)) // 64 * 64
        n_dm = int(rng.integers(64, 513))
        step = float(rng.choice([0.25, 0.5, 1.0]))
        beams.append(dict(dtype=dtype, n_chan=n_chan, n_samp=n_samp, f_high=1500.0, chan_bw=300.0 / n_chan,
                          t_samp=64e-6, dm_start=0.0, dm_step=step, n_dm=n_dm, seed=700 + b))
    return beams


def batch_beams(n_beams: int = 48, seed: int = 5):
    """Per-beam parameters of the multi-beam workload (48 beams by default).

    Channel counts from {1024, 2048, 4096, 8192}, lengths uniform in
    [2^16, 2^20], 500..4000 DM trials with a step from {0.25, 0.5, 0.75, 1.0};
    1500 MHz top of band, 300 MHz band, 64 us sampling.  Beam b's data seed is
    500 + b; rows are padded to a pitch that is a multiple of 64 samples.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    beams = []
    for b in range(n_beams):
        n_chan = int(rng.choice([1024, 2048, 4096, 8192]))
        n_samp = int(rng.integers(1 << 16, (1 << 20) + 1))
        n_dm = int(rng.integers(500, 4001))
        step = float(rng.choice([0.25, 0.5, 0.75, 1.0]))
        beams.append(dict(dtype="u8", n_chan=n_chan, n_samp=n_samp, f_high=1500.0,
                          chan_bw=300.0 / n_chan, t_samp=64e-6, dm_start=0.0, dm_step=step,
                          n_dm=n_dm, seed=500 + b, pitch=(n_samp + 63) // 64 * 64))
    return beams
