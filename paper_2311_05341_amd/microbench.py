"""Measured denominators for the roofline fractions: VALU issue rate per add form,
LDS read bandwidth per access width and alignment, and HBM copy bandwidth.

The kernels live in ``csrc/microbench.hip`` (library ``libddmb.so``, built by
``build()``); this module only launches them on torch-allocated buffers and times
each launch with HIP events on the current stream.  Rates are reported per second
and per clock and CU at the nominal 2.4 GHz shader clock (the sampled clock, when
given, as well).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "microbench.hip")
LIB = os.path.join(HERE, "libddmb.so")
N_CU = 256
NOMINAL_SCLK_HZ = 2.4e9

VALU_FORMS = {"v_add_u32": (0, 1), "v_add3_u32": (1, 2), "v_pk_add_u16": (2, 2), "v_add_u32_sdwa": (3, 1),
              "v_perm_b32": (4, 0), "swar_pair_8bit": (5, 2)}  # name: (form id, sample-adds per lane-op)
LDS_CASES = [  # (name: the instruction the kernel issues, bytes per lane and read, byte misalignment)
    ("ds_read2st64_b32", 4, 0), ("ds_read2st64_b64", 8, 0), ("ds_read_b128", 16, 0),
    ("ds_read2st64_b32_at_1", 4, 1), ("ds_read2st64_b64_at_4", 8, 4), ("ds_read_b128_at_4", 16, 4),
    ("ds_read_b128_at_8", 16, 8)]


def build() -> str:
    from . import _build
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", *_build.HIPCC_FLAGS, SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def _lib():
    if not os.path.exists(LIB):
        raise ImportError("libddmb.so is not built: run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB)
    vp, i32 = ctypes.c_void_p, ctypes.c_int
    lib.ddmb_valu.argtypes = [i32, i32, i32, vp, vp, vp]
    lib.ddmb_lds.argtypes = [i32, i32, i32, i32, vp, vp]
    lib.ddmb_copy.argtypes = [vp, vp, ctypes.c_size_t, i32, vp]
    lib.ddmb_valu_instructions_per_lane.argtypes = [i32, i32]
    lib.ddmb_lds_bytes_per_lane.argtypes = [i32, i32]
    for f in (lib.ddmb_valu, lib.ddmb_lds, lib.ddmb_copy, lib.ddmb_valu_instructions_per_lane,
              lib.ddmb_lds_bytes_per_lane):
        f.restype = i32
    return lib


def _time(torch, launch, reps=5):
    """Median launch time in seconds (one warm-up launch, HIP events on the current stream)."""
    stream = torch.cuda.current_stream()
    rc = launch(stream.cuda_stream)
    if rc != 0:
        raise RuntimeError("microbenchmark launch failed: hipError %d" % rc)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        launch(stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    ms.sort()
    return ms[len(ms) // 2] * 1e-3


def measure(torch, sclk_hz=None, copy_bytes=1 << 31):
    """Run every microbenchmark once on the current device; returns a dict of rates."""
    lib = _lib()
    clk = NOMINAL_SCLK_HZ
    per = lambda rate: rate / (N_CU * clk)  # noqa: E731  (per clock and CU at the nominal clock)
    res = {"n_cu": N_CU, "nominal_sclk_hz": clk, "sampled_sclk_hz": sclk_hz, "valu": {}, "lds": {}, "hbm": {}}

    inp = (torch.arange(128, dtype=torch.int64) * 2654435761 % (1 << 31)).to(torch.int32).cuda()
    blocks, iters = N_CU * 32, 400
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    for name, (form, adds_per_op) in VALU_FORMS.items():
        lane_ops = float(blocks) * 256 * lib.ddmb_valu_instructions_per_lane(form, iters)
        t = _time(torch, lambda s: lib.ddmb_valu(form, blocks, iters, inp.data_ptr(), out.data_ptr(), s))
        rate = lane_ops / t
        res["valu"][name] = {"lane_ops_per_s": rate, "lane_ops_per_clk_cu": per(rate),
                             "sample_adds_per_s": rate * adds_per_op}
    del out

    blocks, iters = N_CU * 24, 400
    out = torch.empty(blocks * 256, dtype=torch.int32, device="cuda")
    for name, width, mis in LDS_CASES:
        it = iters if mis % width == 0 else iters // 16  # misaligned reads are far slower
        nbytes = float(blocks) * 256 * lib.ddmb_lds_bytes_per_lane(width, it)
        t = _time(torch, lambda s: lib.ddmb_lds(width, mis, blocks, it, out.data_ptr(), s))
        rate = nbytes / t
        res["lds"][name] = {"bytes_per_s": rate, "bytes_per_clk_cu": per(rate)}
    del out

    src = torch.ones(copy_bytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    t = _time(torch, lambda s: lib.ddmb_copy(src.data_ptr(), dst.data_ptr(), copy_bytes, N_CU * 16, s))
    res["hbm"]["copy"] = {"bytes": 2 * copy_bytes, "GB_per_s": 2 * copy_bytes / t / 1e9}
    del src, dst
    torch.cuda.empty_cache()
    return res
