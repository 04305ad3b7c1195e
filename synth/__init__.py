"""Seeded synthetic filterbanks shaped like the paper's workloads.

Shared by the tests, the benchmark and the smoke check as the only common
input source for the CPU oracle and the GPU library.  It holds none of the
transform's arithmetic: pulse injection takes the per-channel delays of the
pulse's DM as an argument from the caller.

Recipe (stands in for the SIGPROC ``fake`` files the paper generated its test
signals with, Sec. 5):

* Every channel row c draws from its own stream ``PCG64(SeedSequence([seed, c]))``,
  so a row's values do not depend on how many rows are generated or in which
  order, and rows can be generated in parallel.
* 8-bit noise: ``normal(mean, sigma)``, rounded to nearest (``np.rint``),
  clipped to 0..255.
* 4-bit noise: uniform integers 0..15, packed two per byte, the even sample in
  the low nibble.
* float noise: standard normal, float32.
* Pulses: a boxcar of amplitude A and width W starting at arrival time t0 at the
  top of the band, added at ``x[c][t0 + k + delay[c]]`` for k < W and clipped
  at 255 (8-bit) after the noise is clipped.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_WORKERS = max(1, min(16, os.cpu_count() or 1))


def _rng(seed: int, row: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(row)])))


def _fill_rows(out: np.ndarray, fn, workers: int | None = None) -> np.ndarray:
    n = out.shape[0]
    w = workers or _WORKERS
    if n * out.shape[1] < (1 << 22) or w == 1:
        for c in range(n):
            fn(c, out[c])
    else:
        with ThreadPoolExecutor(max_workers=w) as ex:
            list(ex.map(lambda c: fn(c, out[c]), range(n)))
    return out


def gaussian_u8(n_chan: int, n_samp: int, seed: int, mean: float = 128.0, sigma: float = 16.0,
                pitch: int | None = None) -> np.ndarray:
    """uint8 [n_chan][pitch] of rounded, clipped Gaussian noise; columns >= n_samp are 0."""
    pitch = n_samp if pitch is None else pitch
    assert pitch >= n_samp
    out = np.zeros((n_chan, pitch), dtype=np.uint8)

    def row(c, dst):
        v = _rng(seed, c).normal(mean, sigma, n_samp)
        np.rint(v, out=v)
        np.clip(v, 0.0, 255.0, out=v)
        dst[:n_samp] = v.astype(np.uint8)

    return _fill_rows(out, row)


def uniform_u4_packed(n_chan: int, n_samp: int, seed: int, pitch_bytes: int | None = None) -> np.ndarray:
    """uint8 [n_chan][pitch_bytes]: uniform 0..15 samples, two per byte, even sample low."""
    assert n_samp % 2 == 0
    pb = n_samp // 2 if pitch_bytes is None else pitch_bytes
    assert pb >= n_samp // 2
    out = np.zeros((n_chan, pb), dtype=np.uint8)

    def row(c, dst):
        v = _rng(seed, c).integers(0, 16, n_samp, dtype=np.uint8)
        dst[: n_samp // 2] = v[0::2] | (v[1::2] << 4)

    return _fill_rows(out, row)


def unpack_u4(packed: np.ndarray, n_samp: int) -> np.ndarray:
    """Inverse of the 4-bit packing: uint8 [n_chan][n_samp] of values 0..15."""
    out = np.empty((packed.shape[0], n_samp), dtype=np.uint8)
    out[:, 0::2] = packed[:, : n_samp // 2] & 15
    out[:, 1::2] = packed[:, : n_samp // 2] >> 4
    return out


def normal_f32(n_chan: int, n_samp: int, seed: int, pitch: int | None = None) -> np.ndarray:
    """float32 [n_chan][pitch] standard-normal noise; columns >= n_samp are 0."""
    pitch = n_samp if pitch is None else pitch
    out = np.zeros((n_chan, pitch), dtype=np.float32)

    def row(c, dst):
        dst[:n_samp] = _rng(seed, c).standard_normal(n_samp, dtype=np.float32)

    return _fill_rows(out, row)


def inject_boxcar_u8(x: np.ndarray, delay: np.ndarray, t0: int, width: int, amp: int) -> np.ndarray:
    """Add a dispersed boxcar in place: x[c][t0 + k + delay[c]] += amp, clipped at 255.

    ``delay`` is the integer per-channel delay of the pulse's DM, supplied by
    the caller.  Returns the int64 [n_chan][width] array of increments actually
    applied (after clipping), whose column sums are the exact amplitude the
    dedispersed pulse gains at its DM.
    """
    n_chan = x.shape[0]
    assert delay.shape == (n_chan,)
    applied = np.zeros((n_chan, width), dtype=np.int64)
    for k in range(width):
        cols = t0 + k + delay.astype(np.int64)
        rows = np.arange(n_chan)
        before = x[rows, cols].astype(np.int64)
        after = np.minimum(before + amp, 255)
        x[rows, cols] = after.astype(np.uint8)
        applied[:, k] = after - before
    return applied


#: The five workloads: shapes, bands, DM plans and seeds.  Channel c sits at
#: f_high - c * chan_bw_mhz.  Pulses are (dm_index, width, t0).
CONFIGS = {
    "small": dict(dtype="u8", n_chan=128, n_samp=32768, f_high=1500.0, chan_bw=1.5625,
                  t_samp=64e-6, dm_start=0.0, dm_step=1.0, n_dm=256, seed=1,
                  pulses=[(100, 4, 8000)], amp=40),
    "headline": dict(dtype="u8", n_chan=8192, n_samp=1 << 20, f_high=1500.0, chan_bw=300.0 / 8192,
                     t_samp=64e-6, dm_start=0.0, dm_step=0.5, n_dm=4000, seed=2,
                     pulses=[(100, 1, 100_000), (600, 2, 280_000), (1600, 4, 460_000),
                             (3000, 8, 640_000), (3800, 16, 820_000)], amp=40),
    "lowfreq_u4": dict(dtype="u4", n_chan=4096, n_samp=1 << 19, f_high=190.0, chan_bw=70.0 / 4096,
                       t_samp=327.68e-6, dm_start=0.0, dm_step=0.1, n_dm=2048, seed=3,
                       pulses=[], amp=0),
    "grad_f32": dict(dtype="f32", n_chan=1024, n_samp=1 << 17, f_high=1500.0, chan_bw=300.0 / 1024,
                     t_samp=128e-6, dm_start=0.0, dm_step=1.0, n_dm=1024, seed=4,
                     target_seed=40, fd_seed=41, pulses=[], amp=0),
}


def batch_beams(n_beams: int = 48, seed: int = 5):
    """Per-beam parameters of the multi-beam workload (48 beams by default).

    Channel counts from {1024, 2048, 4096, 8192}, lengths uniform in
    [2^16, 2^20], 500..4000 DM trials with a step from {0.25, 0.5, 0.75, 1.0};
    1500 MHz top of band, 300 MHz band, 64 us sampling.  Beam b's data seed is
    500 + b.
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
                          n_dm=n_dm, seed=500 + b))
    return beams
