"""Benchmark: brute-force dedispersion throughput on one MI355X.

Default workload (the paper-shaped headline case): 8192 channels of 8-bit
input, 2^20 samples at 64 us, 1500 MHz top of a 300 MHz band, 4000 trial DMs
0..1999.5 in steps of 0.5, five injected pulses.  A step is one full forward
transform of that filterbank, input already resident in HBM.

Prints one JSON line with Tadds/s (adds = N_dm * N_out * N_ch), the
x-real-time factor (N_t * t_samp / t_step), the VALU roofline fraction of the
forward kernel, the GPU clocks sampled during the timed steps, and the CPU
oracle timed on a bounded sample of the same workload.  The headline line also
carries the rest of the metric, each form against the plain forward on the
same GPU: the float adjoint against the float forward (1024 ch x 2^17 x 1024
DMs, and one autograd forward + backward step) and the 48-beam batched launch
against the same work as plain calls.

  python bench.py [--steps K] [--warmup W]
                  [--workload headline|headline_shard8|lowfreq_u4|headline_u4|lowfreq_wide|lowfreq_wide_u16|headline_u16|grad_f32|small|
                              batch48|batch_wide8|batch_wide8_u4|batch_wide8_u16|batch_small64|tab_plans_8192|pipeline_high]
                  [--adjoint] [--time-major] [--tiles SHAPE,ORDER] [--no-cpu-baseline] [--no-autotune]
                  [--autotune] [--no-extras] [--copy-calibration]

The headline plan runs its default tiles unless --autotune is given (the
autotuner's pick on that plan); the other workloads autotune unless
--no-autotune or --tiles is given.

The multi-range workloads (tab_plans_8192, pipeline_high) time one step as the
whole survey: binning of the input once per factor plus every range's transform.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 lanes x 2.4 GHz = 39.32e12 32-bit VALU lane-operations per second.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# LDS: 128 bytes per clock per CU for 4- and 8-byte reads (the widths the accumulate loops use).
LDS_PEAK_TBS = 256 * 128 * 2.4e9 / 1e12
# LDS bytes the accumulate loop reads per add: one byte per 8- or 4-bit sample
# (4-bit samples are unpacked to bytes when staged), four per float.
LDS_BYTES_PER_ADD = {"u8": 1, "u4": 1, "u16": 2, "f32": 4}
# The integer kernels add four 8-bit samples per 32-bit word and two channels per
# v_add3_u32 (one v_perm_b32 + one v_add3_u32 per two channel-words for each of
# the even/odd byte lanes): 8 sample-adds per 4 VALU ops, so twice the one-add-per-lane peak.
INT_FORM = "SWAR bytes in 32-bit words, v_perm_b32 + v_add3_u32 (2 sample-adds per VALU lane-op)"
F32_FORM = "v_add_f32 (1 add per VALU lane-op)"
# 16-bit: per two channel-words (4 sample-adds) one v_add3_u32 for the low halves and
# one SDWA v_add_u32 per word for the high halves: 3 VALU ops.
U16_FORM = ("two 16-bit samples per word, v_add3_u32 over two channels + one SDWA v_add_u32 per word "
            "(4 sample-adds per 3 VALU lane-ops)")
FORMS = {"u8": (INT_FORM, 2), "u4": (INT_FORM, 2), "u16": (U16_FORM, 4.0 / 3.0), "f32": (F32_FORM, 1)}
# Packed 4-bit phase-load shapes add nibbles in place: per two channel words (16 samples) two
# v_and_b32, two v_lshrrev_b32 and two v_add3_u32; their windows are read packed (half a byte per add).
U4_NIBBLE_FORM = ("SWAR nibbles in 32-bit words, v_and_b32 + v_lshrrev_b32 + v_add3_u32 "
                  "(16 sample-adds per 6 VALU lane-ops)")
# The direct-read kernel first aligns each window word with one v_alignbit_b32, then adds it in
# the same SWAR forms (two channels per v_add3_u32): per two channel words 2 v_alignbit_b32 plus
# 2 v_perm_b32 + 2 v_add3_u32 (8-bit, 8 sample-adds), 2 v_and_b32 + 2 v_lshrrev_b32 + 2
# v_add3_u32 (4-bit, 16) or 2 v_lshrrev_b32 + 2 v_add3_u32 (16-bit, 4).  No LDS.
DIRECT_FORMS = {
    "u8": ("direct reads: v_alignbit_b32 per word, SWAR bytes v_perm_b32 + v_add3_u32 "
           "(8 sample-adds per 6 VALU lane-ops)", 8.0 / 6.0),
    "u4": ("direct reads: v_alignbit_b32 per word, SWAR nibbles v_and_b32 + v_lshrrev_b32 + v_add3_u32 "
           "(16 sample-adds per 8 VALU lane-ops)", 2.0),
    "u16": ("direct reads: v_alignbit_b32 per word, 16-bit halves v_lshrrev_b32 + v_add3_u32 "
            "(4 sample-adds per 6 VALU lane-ops)", 4.0 / 6.0),
}
# (v_alignbit_b32, v_perm_b32, single-rate VOP2 (v_and/v_lshrrev), v_add3_u32) per two channel
# words, and the sample-adds they make, for pricing the direct forms at measured rates.
DIRECT_OPS = {"u8": (2, 2, 0, 2, 8), "u4": (2, 0, 4, 2, 16), "u16": (2, 0, 2, 2, 4)}


def accumulate_form(dtype, tiles):
    """(instruction form, sample-adds per VALU lane-op, LDS bytes read per add) of a kernel choice."""
    if dtype != "f32" and tiles.get("row_block", 0) == 0:
        return DIRECT_FORMS[dtype][0], DIRECT_FORMS[dtype][1], 0
    if dtype == "u4" and tiles.get("segs", 0) > 0:
        return U4_NIBBLE_FORM, 16.0 / 6.0, 0.5
    return FORMS[dtype][0], FORMS[dtype][1], LDS_BYTES_PER_ADD[dtype]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    """CPU model and thread counts of the host, read from /proc (no program is started)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu_model": model, "nproc": usable, "os_cpu_count": os.cpu_count()}


class SysfsClocks:
    """Samples the GPU's current shader (sclk) and memory (mclk) clocks during a timed region.

    Plain reads of the amdgpu hwmon files (freq1_input = sclk, freq2_input = mclk,
    in Hz) every `period` seconds from a thread of this process: no program is
    started, so nothing is exec'd from a process that holds the GPU.  Falls back
    to the DPM table's current level (pp_dpm_sclk / pp_dpm_mclk, the line marked
    '*') when hwmon has no frequency files.  Reports the median and range per card."""

    def __init__(self, period=0.05):
        import threading
        self.period = period
        self.samples = {}
        self._stop = threading.Event()
        self._thread = threading.Thread(target=self._run, daemon=True)
        self.sources = self._find()

    @staticmethod
    def _find():
        out = {}
        for dev in sorted(glob.glob("/sys/class/drm/card[0-9]*/device")):
            card = dev.split("/")[-2]
            srcs = {}
            for hw in sorted(glob.glob(os.path.join(dev, "hwmon", "hwmon*"))):
                for key, fn in (("sclk_mhz", "freq1_input"), ("mclk_mhz", "freq2_input")):
                    f = os.path.join(hw, fn)
                    if os.path.isfile(f) and key not in srcs:
                        srcs[key] = ("hz", f)
            for key, fn in (("sclk_mhz", "pp_dpm_sclk"), ("mclk_mhz", "pp_dpm_mclk")):
                f = os.path.join(dev, fn)
                if key not in srcs and os.path.isfile(f):
                    srcs[key] = ("dpm", f)
            if srcs:
                out[card] = srcs
        return out

    @staticmethod
    def _read(kind, path):
        try:
            with open(path) as fh:
                text = fh.read()
        except OSError:
            return None
        if kind == "hz":
            try:
                return int(text.strip()) / 1e6
            except ValueError:
                return None
        for line in text.splitlines():
            if line.rstrip().endswith("*"):
                m = re.search(r"(\d+)\s*Mhz", line, re.I)
                return float(m.group(1)) if m else None
        return None

    def _run(self):
        while not self._stop.is_set():
            for card, srcs in self.sources.items():
                for key, (kind, path) in srcs.items():
                    v = self._read(kind, path)
                    if v is not None:
                        self.samples.setdefault(card, {}).setdefault(key, []).append(v)
            self._stop.wait(self.period)

    def __enter__(self):
        if self.sources:
            self._thread.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        if self._thread.is_alive():
            self._thread.join()

    def report(self):
        rep = {}
        for card, keys in self.samples.items():
            rep[card] = {k: {"median": float(np.median(v)), "min": float(min(v)), "max": float(max(v)), "n": len(v),
                             "source": self.sources[card][k][0]} for k, v in keys.items()}
        return rep or None


# Which microbenchmarked rate prices each input type's accumulate loop: the VALU
# form it issues and the LDS read instruction it reads windows with.
# (Float input adds with v_add_f32, priced at the measured v_add_u32 issue rate: both
# are single-rate 32-bit VALU operations.)
MEASURED_FORM = {"u8": "swar_pair_8bit", "u4": "swar_pair_8bit", "u16": "v_add3_u32", "f32": "v_add_u32"}
MEASURED_LDS = "ds_read2st64_b32"


def attach_measured_peaks(rec, dd, torch, dtype):
    """Run the microbenchmarks (libddmb.so) and put the measured rates beside the datasheet
    denominators: the VALU rate of the accumulate loop's own instruction form (sample-adds per
    second) and the LDS read bandwidth of the read instruction it uses."""
    from paper_2311_05341_amd import microbench
    clocks = rec.get("clocks") or {}
    sclk = None
    for card in clocks.values():
        if "sclk_mhz" in card:
            sclk = card["sclk_mhz"]["median"] * 1e6
            break
    mb = microbench.measure(torch, sclk_hz=sclk)
    rec["microbench"] = mb
    achieved = rec["roofline"]["achieved"]
    form = mb["valu"][MEASURED_FORM[dtype]]
    direct = [k for k, v in DIRECT_FORMS.items() if v[0] == rec["roofline"]["instruction_form"]]
    if direct:
        # each op priced at its measured rate: v_alignbit_b32 as v_perm_b32 (both single-rate VOP3)
        n_align, n_perm, n_vop2, n_add3, adds = DIRECT_OPS[direct[0]]
        v = mb["valu"]
        t = ((n_align + n_perm) / v["v_perm_b32"]["lane_ops_per_s"] + n_vop2 / v["v_add_u32"]["lane_ops_per_s"]
             + n_add3 / v["v_add3_u32"]["lane_ops_per_s"])
        peak = adds / t / 1e12
    elif dtype == "u4" and rec["roofline"]["instruction_form"] == U4_NIBBLE_FORM:
        # 16 sample-adds per two v_and_b32, two v_lshrrev_b32 (priced at the v_add_u32 rate: single-
        # rate VOP2) and two v_add3_u32, each at its own measured rate
        r_a = mb["valu"]["v_add3_u32"]["lane_ops_per_s"]
        r_1 = mb["valu"]["v_add_u32"]["lane_ops_per_s"]
        peak = 16.0 / (2.0 / r_a + 4.0 / r_1) / 1e12
    elif dtype == "u16":
        # 4 sample-adds per one v_add3_u32 and two SDWA adds, each at its own measured rate
        r_a = mb["valu"]["v_add3_u32"]["lane_ops_per_s"]
        r_s = mb["valu"]["v_add_u32_sdwa"]["lane_ops_per_s"]
        peak = 4.0 / (1.0 / r_a + 2.0 / r_s) / 1e12
    else:
        peak = form["sample_adds_per_s"] / 1e12
    rec["roofline"]["peak_measured_instruction_form"] = peak
    rec["roofline"]["frac_measured_instruction_form"] = achieved / peak
    if rec.get("lds_roofline") is None:
        return
    lds = mb["lds"][MEASURED_LDS]["bytes_per_s"] / 1e12
    rec["lds_roofline"]["peak_measured"] = lds
    rec["lds_roofline"]["peak_measured_instruction"] = MEASURED_LDS
    rec["lds_roofline"]["frac_measured"] = rec["lds_roofline"]["achieved"] / lds


def measured_traffic(workload, tiles):
    """Memory traffic per launch from a committed rocprofv3 counter summary.

    profiles/*_counters.md hold a ```traffic block (FETCH_SIZE + WRITE_SIZE per
    launch, calibrated against a 1 GiB copy) with the workload, the tile choice
    and the SHA-256 of the kernel source they were measured on.  The figure is
    used only if all three match the run; otherwise the traffic is unknown (None).
    """
    want_tiles = "%d,%d" % (tiles["shape"], tiles["order"])
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_counters.md"))):
        with open(path) as fh:
            text = fh.read()
        for block in re.findall(r"```traffic\n(.*?)```", text, re.S):
            kv = dict(line.split(": ", 1) for line in block.strip().splitlines() if ": " in line)
            if kv.get("workload") != workload or kv.get("tiles") != want_tiles:
                continue
            src = os.path.join(ROOT, kv.get("source", ""))
            if not os.path.isfile(src):
                continue
            with open(src, "rb") as fh:
                if hashlib.sha256(fh.read()).hexdigest() != kv.get("source_sha256"):
                    continue
            return int(kv["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


def make_input(dd, torch, synth, cfg, plan):
    """Seeded synthetic filterbank generated directly in device memory (pulses included)."""
    n_chan, n_samp = cfg["n_chan"], cfg["n_samp"]
    stream = torch.cuda.current_stream().cuda_stream
    if cfg["dtype"] == "u8":
        x = torch.empty((n_chan, plan.in_pitch_bytes), dtype=torch.uint8, device="cuda")
        table = torch.from_numpy(synth.gaussian_table()).cuda()
        synth.gaussian_u8_device(x.data_ptr(), n_chan, n_samp, plan.in_pitch_bytes, cfg["seed"],
                                 table.data_ptr(), stream)
        shift = plan.shift
        for dp, width, t0 in cfg.get("pulses", []):
            def at(r, c):
                v = x[torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()]
                return v.cpu().numpy()
            rows, cols, vals, _ = synth.boxcar_updates(at, shift[dp], t0, width, cfg["amp"])
            x[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()] = torch.from_numpy(vals).cuda()
    elif cfg["dtype"] == "u4":
        x = torch.empty((n_chan, plan.in_pitch_bytes), dtype=torch.uint8, device="cuda")
        synth.uniform_u4_device(x.data_ptr(), n_chan, n_samp, plan.in_pitch_bytes, cfg["seed"], stream)
    elif cfg["dtype"] == "u16":
        pitch = plan.in_pitch_bytes // 2
        x = torch.empty((n_chan, pitch), dtype=torch.uint16, device="cuda")
        table = torch.from_numpy(synth.gaussian_table16()).cuda()
        synth.gaussian_u16_device(x.data_ptr(), n_chan, n_samp, pitch, cfg["seed"], table.data_ptr(), stream)
        shift = plan.shift
        xi = x.view(torch.int16)  # torch has no uint16 gather/scatter on the GPU; same bytes as int16
        for dp, width, t0 in cfg.get("pulses", []):
            def at(r, c):
                return xi[torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()].cpu().numpy().view(np.uint16)
            rows, cols, vals, _ = synth.boxcar_updates(at, shift[dp], t0, width, cfg["amp"], 65535)
            xi[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()] = torch.from_numpy(vals.view(np.int16)).cuda()
    else:
        x = torch.from_numpy(synth.normal_f32(cfg["n_chan"], n_samp, cfg["seed"])).cuda()
    torch.cuda.synchronize()
    return x


def cpu_baseline(cfg, seconds_target=15.0):
    """Time the CPU oracle on a bounded sample: whole DM rows (all channels, all samples)."""
    import oracle
    import synth

    s = oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], cfg["dm_start"],
                           cfg["dm_step"], cfg["n_dm"])
    n_out = oracle.n_out_for(s, cfg["n_samp"])
    if cfg["dtype"] == "u8":
        x = synth.gaussian_u8(cfg["n_chan"], cfg["n_samp"], cfg["seed"])
        run = lambda rows: oracle.forward(x, "u8", cfg["n_samp"], s, rows=rows)  # noqa: E731
    elif cfg["dtype"] == "u4":
        x = synth.uniform_u4_packed(cfg["n_chan"], cfg["n_samp"], cfg["seed"])
        run = lambda rows: oracle.forward(x, "u4", cfg["n_samp"], s, rows=rows)  # noqa: E731
    elif cfg["dtype"] == "u16":
        x = synth.gaussian_u16(cfg["n_chan"], cfg["n_samp"], cfg["seed"])
        run = lambda rows: oracle.forward(x, "u16", cfg["n_samp"], s, rows=rows)  # noqa: E731
    else:
        x = synth.normal_f32(cfg["n_chan"], cfg["n_samp"], cfg["seed"])
        run = lambda rows: oracle.forward_f32(x, cfg["n_samp"], s, rows=rows, with_abs=False)  # noqa: E731
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # calibrate with a few rows, then size the sample to the time target
    probe = list(range(0, cfg["n_dm"], max(1, cfg["n_dm"] // max(1, threads))))[:threads]
    t = time.perf_counter()
    run(probe)
    dt = time.perf_counter() - t
    per_row = dt / len(probe)
    n_rows = int(max(len(probe), min(cfg["n_dm"], seconds_target / per_row)))
    rows = np.linspace(0, cfg["n_dm"] - 1, n_rows).round().astype(int).tolist()
    t = time.perf_counter()
    run(rows)
    dt = time.perf_counter() - t
    adds = float(len(rows)) * n_out * cfg["n_chan"]
    return dict({"value": adds / dt / 1e12, "unit": "Tadds/s", "cores": threads, "kind": "oracle",
                 "sample": "%d of %d DM rows, all %d channels x %d output samples (%.2e adds, %.1f s)"
                           % (len(rows), cfg["n_dm"], cfg["n_chan"], n_out, adds, dt)}, **host_cpu())


def cpu_tiled_baseline(cfg, seconds_target=15.0):
    """Time the paper's tiled CPU algorithm (Algorithm 2, libdd_cpu.so) on a bounded sample:
    the first DM rows of the plan (neighbouring trials are what its tiling reuses), all
    channels and output samples.  8-bit input only."""
    import oracle
    import synth
    from paper_2311_05341_amd import cpu_tiled

    s = oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], cfg["dm_start"],
                           cfg["dm_step"], cfg["n_dm"])
    n_out = oracle.n_out_for(s, cfg["n_samp"])
    x = synth.gaussian_u8(cfg["n_chan"], cfg["n_samp"], cfg["seed"])
    d_dm = cpu_tiled.DEFAULT_TILES[1]
    probe = min(cfg["n_dm"], 2 * d_dm)
    t = time.perf_counter()
    cpu_tiled.forward_u8(x, s[:probe], n_out)
    per_row = (time.perf_counter() - t) / probe
    n_rows = int(min(cfg["n_dm"], max(probe, seconds_target / per_row // d_dm * d_dm)))
    t = time.perf_counter()
    cpu_tiled.forward_u8(x, s[:n_rows], n_out)
    dt = time.perf_counter() - t
    adds = float(n_rows) * n_out * cfg["n_chan"]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": adds / dt / 1e12, "unit": "Tadds/s", "cores": threads, "kind": "tiled (Algorithm 2)",
            "tiles": list(cpu_tiled.DEFAULT_TILES),
            "sample": "first %d of %d DM rows, all %d channels x %d output samples (%.2e adds, %.1f s)"
                      % (n_rows, cfg["n_dm"], cfg["n_chan"], n_out, adds, dt)}


BATCH_CHUNKS = 2  # time chunks per beam of the 48-beam job (its outputs would not fit HBM at once)


def setup_batch48(dd, torch, synth, n_chunks=BATCH_CHUNKS, log=log):
    """The 48-beam job: inputs resident in HBM, one persistent batch per time chunk.

    Every beam's whole filterbank (99 GB in total) is generated in device
    memory.  The whole job's outputs (217 GB) plus inputs exceed one MI355X's
    288 GB, so each beam's outputs are produced in n_chunks time chunks into
    one reused per-beam buffer, as a streaming search would consume them; chunk
    k of every beam is one dd.Batch (one graph-replayed persistent launch).
    Returns (beams, chunkers, inputs, outputs, batches)."""
    from concurrent.futures import ThreadPoolExecutor

    beams = synth.batch_beams()
    keys = ["n_chan", "n_samp", "dtype", "f_high", "chan_bw", "t_samp", "dm_start", "dm_step", "n_dm"]
    t = time.perf_counter()

    def chunker(b):
        return dd.TimeChunks(dict({k: b[k] for k in keys}, in_pitch_bytes=b["pitch"]), n_chunks, bind=False)

    with ThreadPoolExecutor(8) as pool:
        chunkers = list(pool.map(chunker, beams))
    log("batch: %d beams, %d plans in %.1f s" % (len(beams), sum(len(set(map(id, c.plans))) for c in chunkers),
                                                   time.perf_counter() - t))
    dev = torch.device("cuda", torch.cuda.current_device())
    in_bytes = sum(b["n_chan"] * b["pitch"] for b in beams)
    out_bytes = sum(b["n_dm"] * ((c.chunk_len + 3) // 4 * 4) * 4 for b, c in zip(beams, chunkers))
    free, _ = torch.cuda.mem_get_info()
    log("batch: inputs %.1f GB, chunk outputs %.1f GB, device free %.1f GB" % (in_bytes / 1e9, out_bytes / 1e9,
                                                                               free / 1e9))
    if in_bytes + out_bytes > 0.95 * free:
        raise SystemExit("the 48-beam job needs %.1f GB of device memory, %.1f GB are free"
                         % ((in_bytes + out_bytes) / 1e9, free / 1e9))
    for c in chunkers:
        for p in set(c.plans):
            p.bind(dev)
    table = torch.from_numpy(synth.gaussian_table()).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    inputs, outputs = [], []
    for b, c in zip(beams, chunkers):
        x = torch.empty((b["n_chan"], b["pitch"]), dtype=torch.uint8, device=dev)
        synth.gaussian_u8_device(x.data_ptr(), b["n_chan"], b["n_samp"], b["pitch"], b["seed"], table.data_ptr(),
                                 stream)
        inputs.append(x)
        outputs.append(torch.empty((b["n_dm"], (c.chunk_len + 3) // 4 * 4), dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    t = time.perf_counter()
    batches = []
    for k in range(n_chunks):
        idx = [i for i, c in enumerate(chunkers) if k < len(c)]
        batches.append((idx, dd.Batch([chunkers[i].plans[k] for i in idx],
                                      [chunkers[i].input_view(inputs[i], k) for i in idx],
                                      [outputs[i] for i in idx])))
    torch.cuda.synchronize()
    log("batch: %d batches bound in %.1f s" % (len(batches), time.perf_counter() - t))
    return beams, chunkers, inputs, outputs, batches


def batch_shapes(batch):
    """Tile shapes a batch's beams run: {shape index: number of beams}."""
    counts = {}
    for b in range(len(batch.plans)):
        s = batch.beam_tiles(b)["shape"]
        counts[s] = counts.get(s, 0) + 1
    return {str(k): v for k, v in sorted(counts.items())}


def timed_events(torch, fn, steps, warmup):
    """Mean and median kernel time (ms) of fn() over `steps` calls, each bracketed by HIP events on
    the current stream (the stream every call here launches on)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in ev:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    return float(np.mean(ms)), float(np.median(ms))


def adjoint_vs_forward(dd, torch, synth, steps=10):
    """The float differentiation workload (1024 ch f32 x 2^17 x 1024 DMs): the forward and the
    adjoint (gather form) of one plan, each timed alone, and one forward + backward step through
    DedisperseFn (the backward being the adjoint; the incoming gradient has row pitch n_out).
    Both directions run in float32 with the same fixed-order sums and the same stated bound
    (1e-5 of the sum of |terms|)."""
    cfg = synth.CONFIGS["grad_f32"]
    plan = dd.Plan(cfg["n_chan"], cfg["n_samp"], "f32", cfg["f_high"], cfg["chan_bw"], cfg["t_samp"],
                   cfg["dm_start"], cfg["dm_step"], cfg["n_dm"])
    x = torch.from_numpy(synth.normal_f32(cfg["n_chan"], cfg["n_samp"], cfg["seed"])).cuda()
    gen = torch.Generator(device="cpu").manual_seed(cfg["target_seed"])
    y = torch.randn((cfg["n_dm"], plan.n_out), generator=gen).cuda()
    out = torch.empty((plan.n_dm, plan.out_pitch), device="cuda")
    g = torch.empty((plan.n_chan, plan.in_row_elems), device="cuda")
    adds = float(plan.n_dm) * plan.n_out * plan.n_chan
    f_ms, f_med = timed_events(torch, lambda: plan.forward(x, out=out), steps, 3)
    a_ms, a_med = timed_events(torch, lambda: plan.adjoint(y, out=g), steps, 3)
    xg = x.clone().requires_grad_(True)

    def fwd_bwd():
        xg.grad = None
        dd.DedisperseFn.apply(xg, plan).backward(y)
    s_ms, _ = timed_events(torch, fwd_bwd, steps, 2)
    rec = {"workload": "grad_f32", "n_chan": cfg["n_chan"], "n_samp": cfg["n_samp"], "n_dm": cfg["n_dm"],
           "adds": adds, "forward": {"ms": f_ms, "ms_median": f_med, "Tadds_s": adds / f_ms / 1e9,
                                     "tiles": plan.tiles(0)},
           "adjoint": {"ms": a_ms, "ms_median": a_med, "Tadds_s": adds / a_ms / 1e9, "tiles": plan.tiles(1)},
           "adjoint_over_forward_throughput": f_ms / a_ms,
           "autograd_step": {"ms": s_ms, "what": "DedisperseFn forward + backward (adjoint), incoming gradient "
                                                 "[n_dm][n_out] passed to the adjoint without a copy"},
           "accuracy": "both float32, fixed-order sums, |err| <= 1e-5 * sum|terms| (tests)"}
    del x, y, out, g, xg, plan
    torch.cuda.empty_cache()
    return rec


def batched_vs_plain(dd, torch, synth):
    """The 48-beam job (2 time chunks per beam), batched persistent graph-replayed launches against
    the same work as plain dd_execute calls, both bit-exact; one warm-up and one timed pass each,
    the plan's default tile shape (no tuning inside the benchmark)."""
    beams, chunkers, inputs, outputs, batches = setup_batch48(dd, torch, synth)
    adds = float(sum(b["n_dm"] * c.n_out * b["n_chan"] for b, c in zip(beams, chunkers)))

    def batched():
        for _, bt in batches:
            bt.run()

    def plain():
        for k in range(len(batches)):
            for i, c in enumerate(chunkers):
                if k < len(c):
                    c.plans[k].forward(c.input_view(inputs[i], k), out=outputs[i])
    b_ms, _ = timed_events(torch, batched, 1, 1)
    p_ms, _ = timed_events(torch, plain, 1, 1)
    rec = {"workload": "batch48", "beams": len(beams), "time_chunks": len(batches), "adds": adds,
           "batched": {"ms": b_ms, "Tadds_s": adds / b_ms / 1e9, "tiles": batches[0][1].tiles(),
                       "beams_per_shape": batch_shapes(batches[0][1])},
           "plain": {"ms": p_ms, "Tadds_s": adds / p_ms / 1e9, "calls": sum(len(c) for c in chunkers)},
           "batched_over_plain_throughput": p_ms / b_ms,
           "accuracy": "both bit-exact (integer input; tests compare every beam)"}
    del beams, chunkers, inputs, outputs, batches
    torch.cuda.empty_cache()
    return rec


def bench_batch48(args, dd, torch, synth):
    beams, chunkers, inputs, outputs, batches = setup_batch48(dd, torch, synth)
    adds = float(sum(b["n_dm"] * c.n_out * b["n_chan"] for b, c in zip(beams, chunkers)))
    stream = torch.cuda.current_stream()
    tune = None
    if not args.no_autotune:
        # the batch autotuner on the first chunk's batch; the other chunks take its shape
        t = time.perf_counter()
        tune = batches[0][1].autotune()
        for _, bt in batches[1:]:
            bt.set_tiles(tune["best"]["shape"])
        torch.cuda.synchronize()
        tune["seconds"] = time.perf_counter() - t
        log("batch autotune: %s" % tune)

    def batched():
        for _, bt in batches:
            bt.run()

    def plain():
        for k in range(len(batches)):
            for i, c in enumerate(chunkers):
                if k < len(c):
                    c.plans[k].forward(c.input_view(inputs[i], k), out=outputs[i])

    def timed(step, steps, per_launch=False):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        launch_ms, wall = [], []
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if per_launch:
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(batches) + 1)]
                ev[0].record(stream)
                for j, (_, bt) in enumerate(batches):
                    bt.run()
                    ev[j + 1].record(stream)
            else:
                step()
            torch.cuda.synchronize()
            wall.append(time.perf_counter() - t0)
            if per_launch:
                launch_ms += [ev[j].elapsed_time(ev[j + 1]) for j in range(len(batches))]
        return float(np.mean(wall)) * 1e3, launch_ms

    log("timing batched ...")
    ms_batched, launch_ms = timed(batched, args.steps, per_launch=True)
    log("batched: %.1f ms/step, launches %s ms" % (ms_batched, ["%.1f" % v for v in launch_ms]))
    log("timing 48 plain calls per chunk ...")
    ms_plain, _ = timed(plain, args.steps)
    log("plain: %.1f ms/step" % ms_plain)
    value = adds / (ms_batched * 1e-3) / 1e12
    kernel_ms = float(np.sum(launch_ms)) / args.steps
    achieved = adds / (kernel_ms * 1e-3) / 1e12
    beam_seconds = sum(b["n_samp"] * b["t_samp"] for b in beams)
    rec = {
        "metric": "Tadds/s (48 beams, batched)",
        "value": value,
        "unit": "Tadds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_batched,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "batch48", "beams": len(beams), "time_chunks": len(batches),
                   "adds_per_step": adds, "input_bytes": sum(b["n_chan"] * b["pitch"] for b in beams),
                   "n_chan_set": sorted(set(b["n_chan"] for b in beams)),
                   "n_samp_range": [min(b["n_samp"] for b in beams), max(b["n_samp"] for b in beams)],
                   "n_dm_range": [min(b["n_dm"] for b in beams), max(b["n_dm"] for b in beams)]},
        "plain_calls": {"value": adds / (ms_plain * 1e-3) / 1e12, "unit": "Tadds/s", "ms_per_step": ms_plain,
                        "calls_per_step": sum(len(c) for c in chunkers)},
        "batched_over_plain": ms_plain / ms_batched,
        "x_realtime_beams": beam_seconds / (ms_batched * 1e-3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tadds/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": None, "kernel": "fwd_int_batched_kernel",
                     "kernel_ms": kernel_ms, "instruction_form": INT_FORM, "peak_instruction_form": 2 * VALU_PEAK_TOPS,
                     "frac_instruction_form": achieved / (2 * VALU_PEAK_TOPS)},
        "lds_roofline": {"achieved": achieved, "peak": LDS_PEAK_TBS, "unit": "TB/s", "frac": achieved / LDS_PEAK_TBS,
                         "bytes_per_add": 1},
        "batch_tiles": batches[0][1].tiles(),
        "beams_per_shape": batch_shapes(batches[0][1]),
        "batch_autotune": tune,
    }
    if not args.no_cpu_baseline:
        big = max(beams, key=lambda b: b["n_chan"] * b["n_samp"] * b["n_dm"])
        log("cpu baseline on the largest beam ...")
        rec["cpu_baseline"] = cpu_baseline(dict(big, pulses=[]), seconds_target=12.0)
        rec["cpu_baseline"]["sample"] = "largest beam: " + rec["cpu_baseline"]["sample"]
    print(json.dumps(rec), flush=True)


# Batches of wide-spread beams (every plan on a direct-read shape), by input type, and a batch of
# many small staged beams: (input type, beam generator in synth).
BATCH_SETS = {"batch_wide8": ("u8", "wide_beams"), "batch_wide8_u4": ("u4", "wide_beams"),
              "batch_wide8_u16": ("u16", "wide_beams"), "batch_small64": ("u8", "small_beams")}


def bench_batch_set(args, dd, torch, synth):
    """A batch of beams from synth.wide_beams (8 beams at 120-190 MHz, whose plans all read directly)
    or synth.small_beams (64 small staged beams): one graph replay of the batch per step against the
    plain calls, one per beam, each step bracketed by HIP events on the stream both launch on."""
    dtype, gen = BATCH_SETS[args.workload]
    beams = getattr(synth, gen)(dtype)
    plans, inputs, outputs = [], [], []
    for b in beams:
        p = dd.Plan(b["n_chan"], b["n_samp"], dtype, b["f_high"], b["chan_bw"], b["t_samp"], b["dm_start"],
                    b["dm_step"], b["n_dm"])
        plans.append(p)
        inputs.append(make_input(dd, torch, synth, b, p))
        outputs.append(torch.empty((p.n_dm, p.out_pitch), dtype=torch.float32, device="cuda"))
    adds = float(sum(b["n_chan"] * b["n_dm"] * p.n_out for b, p in zip(beams, plans)))
    log("%s: %d %s beams, %.3e adds, plan shapes %s" % (args.workload, len(beams), dtype, adds,
                                                         sorted(set(p.tiles(0)["shape"] for p in plans))))
    batch = dd.Batch(plans, inputs)
    tune = None
    if args.tiles:
        batch.set_tiles(int(args.tiles.split(",")[0]))
    elif not args.no_autotune:
        tune = batch.autotune()
        log("batch autotune: %s" % tune)

    def plain():
        for p, x, o in zip(plans, inputs, outputs):
            p.forward(x, out=o)

    b_ms, b_med = timed_events(torch, batch.run, args.steps, args.warmup)
    p_ms, _ = timed_events(torch, plain, args.steps, args.warmup)
    got = batch.run()
    plain()
    torch.cuda.synchronize()
    same = all(torch.equal(g, o[:, : p.n_out]) for g, o, p in zip(got, outputs, plans))
    direct = all(p.tiles(0)["row_block"] == 0 for p in plans)
    form, per_op, lds_b = accumulate_form(dtype, plans[0].tiles(0))
    achieved = adds / (b_ms * 1e-3) / 1e12
    rec = {
        "metric": "Tadds/s (%d %s beams, batched)" % (len(beams), "wide-spread" if direct else "small"),
        "value": achieved,
        "unit": "Tadds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": b_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": args.workload, "beams": len(beams), "adds_per_step": adds,
                   "n_chan_set": sorted(set(b["n_chan"] for b in beams)),
                   "n_samp_range": [min(b["n_samp"] for b in beams), max(b["n_samp"] for b in beams)],
                   "n_dm_range": [min(b["n_dm"] for b in beams), max(b["n_dm"] for b in beams)],
                   "band_mhz": [beams[0]["f_high"] - 70.0, beams[0]["f_high"]], "t_samp": beams[0]["t_samp"],
                   "dm_step": beams[0]["dm_step"]},
        "plain_calls": {"value": adds / (p_ms * 1e-3) / 1e12, "unit": "Tadds/s", "ms_per_step": p_ms,
                        "calls_per_step": len(plans)},
        "batched_over_plain": p_ms / b_ms,
        "batched_equals_plain": same,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tadds/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "kernel": "fwd_direct_batched_kernel" if direct else "fwd_int_batched_kernel",
                     "kernel_ms": b_ms, "kernel_ms_median": b_med, "instruction_form": form,
                     "peak_instruction_form": per_op * VALU_PEAK_TOPS,
                     "frac_instruction_form": achieved / (per_op * VALU_PEAK_TOPS)},
        "lds_roofline": None if not lds_b else {"achieved": achieved * lds_b, "peak": LDS_PEAK_TBS, "unit": "TB/s",
                                                "frac": achieved * lds_b / LDS_PEAK_TBS, "bytes_per_add": lds_b},
        "batch_tiles": batch.tiles(),
        "beams_per_shape": batch_shapes(batch),
        "batch_autotune": tune,
    }
    if not args.no_cpu_baseline:
        big = max(beams, key=lambda b: b["n_chan"] * b["n_samp"] * b["n_dm"])
        log("cpu baseline on the largest beam ...")
        rec["cpu_baseline"] = cpu_baseline(dict(big, pulses=[]), seconds_target=12.0)
        rec["cpu_baseline"]["sample"] = "largest beam: " + rec["cpu_baseline"]["sample"]
    print(json.dumps(rec), flush=True)
    if not same:
        sys.exit("batched outputs differ from the plain calls")


def bench_survey(args, dd, torch, synth):
    """Multi-range DM plan (binning + one transform per range) over one 8-bit filterbank.

    With --time-major the input is time-major spectra and every step starts with
    the corner turn, as the paper's pipelines (and their real-time factor) do."""
    cfg = synth.SURVEYS[args.workload]
    n_chan, n_samp, t_samp = cfg["n_chan"], cfg["n_samp"], cfg["t_samp"]
    tm = args.time_major
    pitch = (n_samp + 63) // 64 * 64
    log("survey %s%s: %s" % (args.workload, " (time-major input)" if tm else "",
                             {k: v for k, v in cfg.items() if k != "pulses"}))
    sv = dd.Survey(n_chan, n_samp, "u8", cfg["f_high"], cfg["chan_bw"], t_samp, cfg["ranges"],
                   in_pitch_bytes=n_chan if tm else pitch, time_major=tm)
    stream = torch.cuda.current_stream()
    table = torch.from_numpy(synth.gaussian_table()).cuda()
    if tm:  # spectra [n_samp][n_chan]: the generator's rows are time samples
        x = torch.empty((n_samp, n_chan), dtype=torch.uint8, device="cuda")
        synth.gaussian_u8_device(x.data_ptr(), n_samp, n_chan, n_chan, cfg["seed"], table.data_ptr(),
                                 stream.cuda_stream)
    else:
        x = torch.empty((n_chan, pitch), dtype=torch.uint8, device="cuda")
        synth.gaussian_u8_device(x.data_ptr(), n_chan, n_samp, pitch, cfg["seed"], table.data_ptr(),
                                 stream.cuda_stream)
    for dm, width, t0 in cfg["pulses"]:
        delay = dd.Plan(n_chan, n_samp, "u8", cfg["f_high"], cfg["chan_bw"], t_samp, dm, 0.0, 1,
                        in_pitch_bytes=pitch, bind=False).shift[0]

        def index(r, c):  # (channels, samples) as indices of x
            r, c = torch.from_numpy(r).cuda(), torch.from_numpy(c).cuda()
            return (c, r) if tm else (r, c)

        def at(r, c):
            return x[index(r, c)].cpu().numpy()
        rows, cols, vals, _ = synth.boxcar_updates(at, delay, t0, width, cfg["amp"])
        x[index(rows, cols)] = torch.from_numpy(vals).cuda()
    outs = sv.empty_outputs()
    torch.cuda.synchronize()
    tune_s = None
    if not args.no_autotune:
        t = time.perf_counter()
        sv.autotune(x, outs)
        tune_s = time.perf_counter() - t
        log("autotune %.1f s" % tune_s)
    for _ in range(args.warmup):
        sv.run(x, outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sv.run(x, outs)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    adds = float(sum(ri["n_dm"] * ri["n_out"] for ri in sv.range_info)) * n_chan

    # Per-kernel breakdown: the same kernels launched one by one (binning into
    # buffers of the survey's layout, each range through a plan with the survey's
    # tile choice), each timed with HIP events on the current stream.
    def timed(fn, reps):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    turn = None
    rows_in = x
    if tm:
        rows_in = torch.empty((n_chan, pitch), dtype=torch.uint8, device="cuda")
        ms = timed(lambda: dd.corner_turn(x, "u8", n_chan, n_samp, out=rows_in), 5)
        nbytes = 2.0 * n_chan * n_samp
        turn = {"ms": ms, "bytes": nbytes, "GB_s": nbytes / ms / 1e6, "frac_hbm": nbytes / ms / 1e6 / HBM_PEAK_GBS}
    binned, bins = {}, []
    for f in sorted({r[3] for r in cfg["ranges"] if r[3] > 1}):
        nb = n_samp // f
        binned[f] = torch.empty((n_chan, (2 * nb + 255) // 256 * 128), dtype=torch.uint16, device="cuda")
        ms = timed(lambda f=f: dd.bin_time(rows_in, "u8", n_samp, f, out=binned[f]), 5)
        nbytes = float(n_chan) * (nb * f + 2 * nb)  # whole bins read once, uint16 sums written once
        bins.append({"factor": f, "ms": ms, "bytes": nbytes, "GB_s": nbytes / ms / 1e6,
                     "frac_hbm": nbytes / ms / 1e6 / HBM_PEAK_GBS})
    parts = []
    for r, (start, step, n_dm, b) in enumerate(cfg["ranges"]):
        ri = sv.range_info[r]
        src = rows_in if b == 1 else binned[b]
        p = dd.Plan(n_chan, ri["n_samp"], ri["dtype"], cfg["f_high"], cfg["chan_bw"], ri["t_samp"], start, step,
                    n_dm, in_pitch_bytes=src.stride(0) * src.element_size())
        tl = sv.tiles(r)
        p.set_tiles(0, tl["shape"], tl["order"])
        ms = timed(lambda: p.forward(src, out=outs[r]), max(1, args.steps // 2))
        a = float(n_dm) * ri["n_out"] * n_chan
        parts.append({"range": r, "dm_start": start, "dm_step": step, "n_dm": n_dm, "bin": b, "input": ri["dtype"],
                      "n_out": ri["n_out"], "ms": ms, "Tadds_s": a / ms / 1e9, "tiles": tl})
        del p
    dom = max(parts, key=lambda q: q["ms"])
    log("survey parts: %s; bins: %s; corner turn: %s" % (parts, bins, turn))
    rec = {
        "metric": "Tadds/s (multi-range survey)", "value": adds / ms_step / 1e9, "unit": "Tadds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": args.workload, "n_chan": n_chan, "n_samp": n_samp, "t_samp_s": t_samp,
                   "f_high_mhz": cfg["f_high"], "band_mhz": cfg["chan_bw"] * n_chan, "ranges": cfg["ranges"],
                   "adds_per_step": adds, "input_layout": "time-major spectra" if tm else "channel-major rows"},
        "x_realtime": n_samp * t_samp / (ms_step * 1e-3),
        "roofline": {"bound": "alu", "achieved": dom["Tadds_s"], "peak": VALU_PEAK_TOPS, "unit": "Tadds/s",
                     "frac": dom["Tadds_s"] / VALU_PEAK_TOPS, "traffic": None, "kernel": "fwd_int_kernel",
                     "range": dom["range"], "kernel_ms": dom["ms"]},
        "parts": parts, "binning": bins, "corner_turn": turn, "autotune_s": tune_s,
        "sum_of_parts_ms": sum(q["ms"] for q in parts) + sum(q["ms"] for q in bins) + (turn["ms"] if turn else 0.0),
    }
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20; 5 for the multi-range workloads, 2 for the 48-beam job)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default 3; 1 for the 48-beam job)")
    ap.add_argument("--workload", default="headline")
    ap.add_argument("--adjoint", action="store_true", help="time the adjoint instead of the forward")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default tile choice")
    ap.add_argument("--tiles", default=None, metavar="SHAPE,ORDER",
                    help="use this compiled tile shape index and workgroup order instead of autotuning")
    ap.add_argument("--time-major", action="store_true",
                    help="multi-range workloads: time-major spectra in, corner turn inside every step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy first, as a known-size reference for memory counters")
    ap.add_argument("--autotune", action="store_true",
                    help="headline: autotune the tiles first (its default shape is the tuner's pick there)")
    ap.add_argument("--no-microbench", action="store_true",
                    help="skip the measured VALU/LDS/HBM rates reported beside the datasheet peaks")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline: skip the adjoint-vs-forward and batched-vs-plain records")
    args = ap.parse_args()
    long_steps = {"batch48": 2, "tab_plans_8192": 5, "pipeline_high": 5}
    if args.steps is None:
        args.steps = long_steps.get(args.workload, 20)
    if args.warmup is None:
        args.warmup = 1 if args.workload == "batch48" else 3
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2311_05341_amd as dd
    import synth

    if args.copy_calibration:
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 1 GiB read + 1 GiB written")
    if args.workload == "batch48":
        return bench_batch48(args, dd, torch, synth)
    if args.workload in BATCH_SETS:
        return bench_batch_set(args, dd, torch, synth)
    if args.workload in synth.SURVEYS:
        return bench_survey(args, dd, torch, synth)
    cfg = synth.CONFIGS[args.workload]
    log("workload %s: %s" % (args.workload, {k: v for k, v in cfg.items() if k != "pulses"}))
    t = time.perf_counter()
    plan = dd.Plan(cfg["n_chan"], cfg["n_samp"], cfg["dtype"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"],
                   cfg["dm_start"], cfg["dm_step"], cfg["n_dm"])
    log("plan %.2f s: n_out=%d max_shift=%d tile ns=%d dm/wave=%d waves=%d chan_block=%d" % (
        time.perf_counter() - t, plan.n_out, plan.max_shift, plan.info.kernel_ns, plan.info.kernel_dm_per_wave,
        plan.info.kernel_waves, plan.info.kernel_chan_block))
    x = make_input(dd, torch, synth, cfg, plan)
    out = torch.empty((plan.n_dm, plan.out_pitch), dtype=torch.float32, device="cuda")
    direction = 1 if args.adjoint else 0
    if args.adjoint:
        y = torch.randn((plan.n_dm, plan.out_pitch), device="cuda")
        g = torch.empty((plan.n_chan, plan.in_row_elems), dtype=torch.float32, device="cuda")
        step = lambda: plan.adjoint(y, out=g)  # noqa: E731
    else:
        step = lambda: plan.forward(x, out=out)  # noqa: E731
    tune = None
    if args.tiles:
        shape, order = (int(v) for v in args.tiles.split(","))
        plan.set_tiles(direction, shape, order)
    elif not args.no_autotune and (args.autotune or args.workload != "headline"):
        t = time.perf_counter()
        tune = plan.autotune(y, g, direction=1) if args.adjoint else plan.autotune(x, out)
        tune["seconds"] = time.perf_counter() - t
        log("autotune %.1f s: %s" % (tune["seconds"], tune))
    tiles = plan.tiles(direction)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")
    stream = torch.cuda.current_stream()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    with SysfsClocks() as clocks:
        t0 = time.perf_counter()
        for e0, e1 in events:
            e0.record(stream)
            step()
            e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    kernel_ms = [e0.elapsed_time(e1) for e0, e1 in events]
    ms_step = wall * 1e3 / args.steps
    adds = float(plan.n_dm) * plan.n_out * plan.n_chan
    value = adds / (ms_step * 1e-3) / 1e12
    k_avg = float(np.mean(kernel_ms))
    k_med = float(np.median(kernel_ms))
    achieved = adds / (k_avg * 1e-3) / 1e12
    traffic, traffic_src = (None, None) if args.adjoint else measured_traffic(args.workload, tiles)
    form = accumulate_form(cfg["dtype"], tiles)
    log("steps: kernel ms %s, wall ms/step %.3f" % (["%.3f" % v for v in kernel_ms], ms_step))
    rec = {
        "metric": "Tadds/s" + (" (adjoint)" if args.adjoint else ""),
        "value": value,
        "unit": "Tadds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": cfg["dtype"],
        "data": "synthetic",
        "config": {"workload": args.workload, "n_chan": cfg["n_chan"], "n_samp": cfg["n_samp"],
                   "n_dm": cfg["n_dm"], "dm_step": cfg["dm_step"], "t_samp_s": cfg["t_samp"],
                   "f_high_mhz": cfg["f_high"], "band_mhz": cfg["chan_bw"] * cfg["n_chan"],
                   "n_out": plan.n_out, "adds_per_step": adds, "input": cfg["dtype"],
                   "direction": "adjoint" if args.adjoint else "forward"},
        "x_realtime": cfg["n_samp"] * cfg["t_samp"] / (ms_step * 1e-3),
        "x_realtime_streaming": plan.n_out * cfg["t_samp"] / (ms_step * 1e-3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tadds/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic, "traffic_unit": "bytes per launch",
                     "traffic_source": traffic_src,
                     "kernel": ("f32_kernel" if cfg["dtype"] == "f32" else
                                "fwd_direct_kernel" if tiles["row_block"] == 0 else "fwd_int_kernel"),
                     "kernel_ms": k_avg, "kernel_ms_median": k_med,
                     "instruction_form": form[0],
                     "peak_instruction_form": VALU_PEAK_TOPS * form[1],
                     "frac_instruction_form": achieved / (VALU_PEAK_TOPS * form[1])},
        "lds_roofline": None if form[2] == 0 else {
            "achieved": achieved * form[2], "peak": LDS_PEAK_TBS, "unit": "TB/s",
            "frac": achieved * form[2] / LDS_PEAK_TBS, "bytes_per_add": form[2]},
        "tiles": tiles,
        "autotune": tune,
        "clocks": clocks.report(),
        "host": host_cpu(),
    }
    if tiles["row_block"] == 0 and cfg["dtype"] != "f32":
        # The direct-read kernel loads 16 bytes per 16 samples of 8-bit (or 32 of 4-bit) input from
        # L1/L2 for every (channel, DM) pair (the word after them comes from the next lane); lane 63
        # of each wave loads a window only for lane 62 and outputs nothing, so 64 loads per 63.
        per_add = {"u8": 16 / 16, "u4": 16 / 32, "u16": 32 / 16}[cfg["dtype"]] * 64 / 63
        rec["load_path"] = {"bytes_per_add": per_add, "achieved_TB_s": achieved * per_add}
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        rec["cpu_baseline"] = cpu_baseline(cfg)
        if cfg["dtype"] == "u8":
            log("tiled cpu baseline ...")
            rec["cpu_tiled"] = cpu_tiled_baseline(cfg)
    if not args.no_microbench:
        log("microbenchmarks (measured VALU, LDS and HBM rates) ...")
        attach_measured_peaks(rec, dd, torch, cfg["dtype"])
    if args.workload == "headline" and not args.adjoint and not args.no_extras:
        # the rest of the metric: the adjoint and the batched form against the plain forward, same GPU
        del x, out
        torch.cuda.empty_cache()
        log("adjoint vs forward (grad_f32) ...")
        rec["adjoint_vs_forward"] = adjoint_vs_forward(dd, torch, synth)
        log("adjoint vs forward: %s" % rec["adjoint_vs_forward"])
        log("batched vs plain (batch48) ...")
        rec["batched_vs_plain"] = batched_vs_plain(dd, torch, synth)
        log("batched vs plain: %s" % rec["batched_vs_plain"])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
