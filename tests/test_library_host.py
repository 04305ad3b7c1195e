"""Host-side checks of the C-ABI library (no GPU needed).

The plan's FP64 table must equal the oracle's entry for entry; every symbol the
header declares must be exported; argument checks must return the documented
status codes before touching a device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dd():
    import paper_2311_05341_amd as dd
    return dd


def _plan(dd, cfg, **kw):
    args = dict(n_chan=cfg["n_chan"], n_samp=cfg["n_samp"], dtype=cfg["dtype"], f_high=cfg["f_high"],
                chan_bw=cfg["chan_bw"], t_samp=cfg["t_samp"], dm_start=cfg["dm_start"],
                dm_step=cfg["dm_step"], n_dm=cfg["n_dm"], bind=False)
    args.update(kw)
    return dd.Plan(**args)


def test_header_symbols_exported(dd):
    with open(os.path.join(ROOT, "include", "dd.h")) as fh:
        text = fh.read()
    names = sorted(set(re.findall(r"\b(dd_[a-z_]+)\s*\(", text)))
    assert len(names) >= 12
    lib = ctypes.CDLL(dd.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), "missing export " + n


def test_microbench_header_symbols_exported():
    from paper_2311_05341_amd import microbench
    with open(os.path.join(ROOT, "include", "ddmb.h")) as fh:
        text = fh.read()
    names = sorted(set(re.findall(r"\b(ddmb_[a-z_]+)\s*\(", text)))
    assert len(names) == 5
    lib = ctypes.CDLL(microbench.LIB)
    for n in names:
        assert hasattr(lib, n), "missing export " + n
    assert lib.ddmb_valu_instructions_per_lane(5, 3) == 2 * lib.ddmb_valu_instructions_per_lane(1, 3)


@pytest.mark.parametrize("name", ["small", "headline", "lowfreq_u4", "headline_u16", "grad_f32"])
def test_library_table_equals_oracle(dd, name):
    cfg = synth.CONFIGS[name]
    p = _plan(dd, cfg)
    s = oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], cfg["dm_start"],
                           cfg["dm_step"], cfg["n_dm"])
    assert np.array_equal(p.shift, s)
    assert p.n_out == oracle.n_out_for(s, cfg["n_samp"])
    assert p.max_shift == int(s.max())


def test_library_table_random_plans(dd):
    rng = np.random.default_rng(21)
    for _ in range(20):
        n_chan = int(rng.integers(1, 300))
        f_high = float(rng.uniform(100, 3000))
        bw = float(rng.uniform(0.01, 0.5)) * f_high / n_chan
        t_samp = float(rng.choice([10.24e-6, 64e-6, 327.68e-6, 1e-3]))
        n_dm = int(rng.integers(1, 200))
        start, step = float(rng.uniform(0, 50)), float(rng.choice([0.01, 0.1, 0.25, 1.0, 3.7]))
        s = oracle.shift_table(n_chan, f_high, bw, t_samp, start, step, n_dm)
        n_samp = int(s.max()) + int(rng.integers(1, 5000))
        p = dd.Plan(n_chan, n_samp, "u8", f_high, bw, t_samp, start, step, n_dm,
                    in_pitch_bytes=(n_samp + 15) // 16 * 16, bind=False)
        assert np.array_equal(p.shift, s)
        freqs = np.sort(rng.uniform(0.3 * f_high, f_high, n_chan))[::-1].copy()
        freqs[0] = f_high
        s2 = oracle.shift_table(n_chan, f_high, 0.0, t_samp, start, step, n_dm, freqs=freqs)
        n2 = int(s2.max()) + 7
        p2 = dd.Plan(n_chan, n2, "f32", f_high, 0.0, t_samp, start, step, n_dm,
                     chan_freq=freqs, in_pitch_bytes=(n2 + 3) // 4 * 16, bind=False)
        assert np.array_equal(p2.shift, s2)


def _status(dd, fn):
    with pytest.raises(dd.DDError) as e:
        fn()
    return e.value.name


def test_error_codes(dd):
    cfg = dict(synth.CONFIGS["small"])
    assert _status(dd, lambda: _plan(dd, cfg, n_chan=0)) == "DD_ERR_ARG"
    assert _status(dd, lambda: _plan(dd, cfg, n_samp=2400)) == "DD_ERR_TOO_SHORT"
    assert _status(dd, lambda: _plan(dd, cfg, chan_bw=20.0)) == "DD_ERR_RANGE"   # band below 0 MHz
    assert _status(dd, lambda: _plan(dd, cfg, dm_start=-1.0)) == "DD_ERR_RANGE"
    assert _status(dd, lambda: _plan(dd, cfg, dtype="u4", n_samp=32767)) == "DD_ERR_ARG"
    assert _status(dd, lambda: _plan(dd, cfg, in_pitch_bytes=32770)) == "DD_ERR_ALIGN"
    assert _status(dd, lambda: _plan(dd, cfg, in_pitch_bytes=1000)) == "DD_ERR_ARG"
    assert _status(dd, lambda: _plan(dd, cfg, n_chan=70000, chan_bw=0.001)) == "DD_ERR_RANGE"
    assert _status(dd, lambda: _plan(dd, cfg, dtype="u16", n_chan=65538, chan_bw=0.001)) == "DD_ERR_RANGE"
    _plan(dd, cfg, dtype="u16", n_chan=65537, chan_bw=0.001, n_dm=2)  # the largest exact 16-bit plan
    assert _status(dd, lambda: _plan(dd, cfg, dtype="u4", n_chan=1118482, chan_bw=1e-5, n_dm=2)) == "DD_ERR_RANGE"
    assert _status(dd, lambda: _plan(dd, cfg, n_samp=1 << 29)) == "DD_ERR_RANGE"
    _plan(dd, cfg, n_samp=(1 << 29) - 32, n_dm=2)  # the longest rows
    assert _status(dd, lambda: _plan(dd, cfg, dtype="f32", n_samp=(1 << 29) - 32, n_dm=2,
                                     in_pitch_bytes=1 << 31)) == "DD_ERR_RANGE"
    assert _status(dd, lambda: _plan(dd, cfg, chan_freq=np.full(128, 1600.0))) == "DD_ERR_RANGE"  # above f_high
    p = _plan(dd, cfg)
    lib = ctypes.CDLL(dd.LIB_PATH)
    lib.dd_execute.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_void_p]
    lib.dd_execute_adjoint.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_void_p]
    assert lib.dd_execute(p._h, 16, 16, p.out_pitch, None) == -6          # not bound
    assert lib.dd_execute_adjoint(p._h, 16, p.out_pitch, 16, None) == -5  # integer plan
    assert lib.dd_execute(None, 16, 16, 4, None) == -1


def test_plan_tile_shapes(dd):
    for name in ["small", "headline", "lowfreq_u4", "grad_f32"]:
        p = _plan(dd, synth.CONFIGS[name])
        i = p.info
        assert i.kernel_ns in (8, 16, 32) and i.kernel_waves >= 1 and i.kernel_dm_per_wave >= 1
        assert i.kernel_chan_block == 0 or 256 % i.kernel_chan_block == 0  # 0: a direct-read shape


def _bin_lib(dd):
    lib = ctypes.CDLL(dd.LIB_PATH)
    lib.dd_bin_time.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    return lib


def test_bin_argument_checks(dd):
    """Every rejected call returns its status before any device work."""
    lib = _bin_lib(dd)
    a, b = 1 << 20, 1 << 30  # 16-byte aligned addresses that are never dereferenced
    ok = dict(dtype=1, d_in=a, in_pitch=1024, n_chan=4, n_samp=1000, factor=4, d_out=b, out_pitch=512)

    def call(**kw):
        k = dict(ok, **kw)
        return lib.dd_bin_time(k["dtype"], k["d_in"], k["in_pitch"], k["n_chan"], k["n_samp"], k["factor"],
                               k["d_out"], k["out_pitch"], None)
    assert call(dtype=9) == -1
    assert call(d_in=0) == -1 and call(d_out=0) == -1
    assert call(n_chan=0) == -1 and call(n_samp=0) == -1
    assert call(factor=0) == -1 and call(factor=257) == -1
    assert call(n_samp=3) == -2
    assert call(d_in=a + 8) == -4 and call(d_out=b + 4) == -4
    assert call(in_pitch=992) == -1                      # shorter than a row of 1000 bytes
    assert call(in_pitch=1032) == -4                     # not a multiple of 16
    assert call(out_pitch=496) == -1                     # 250 bins of 2 bytes need 500
    assert call(out_pitch=504) == -4
    assert call(d_out=a + 2048) == -1                    # overlaps the input rows
    assert call(dtype=2, in_pitch=496) == -1             # 4-bit rows of 1000 samples take 500 bytes
    assert call(dtype=4, in_pitch=1024) == -1            # 16-bit rows take 2000 bytes
    assert call(dtype=4, in_pitch=2000, out_pitch=992) == -1  # float sums take 4 bytes
    assert [lib.dd_bin_out_dtype(t) for t in (1, 2, 3, 4, 7)] == [4, 4, 3, 3, 0]


SURVEY_RANGES = [(0.0, 1.0, 60, 1), (60.0, 2.0, 40, 2), (140.0, 3.0, 30, 3), (230.0, 4.0, 8, 4)]


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "f32"])
def test_survey_range_plans_equal_oracle(dd, dtype):
    """Range r is planned on the binned grid: t_samp * bin, n_samp // bin, the binned encoding."""
    cfg = synth.CONFIGS["small"]
    n_samp = cfg["n_samp"]
    s = dd.Survey(cfg["n_chan"], n_samp, dtype, cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], SURVEY_RANGES,
                  bind=False)
    need = 0
    for r, (start, step, n_dm, b) in enumerate(SURVEY_RANGES):
        want = oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"] * b, start, step, n_dm)
        assert np.array_equal(s.shift(r), want)
        ri = s.range_info[r]
        assert ri["n_out"] == oracle.n_out_for(want, n_samp // b) and ri["n_samp"] == n_samp // b
        assert ri["dtype"] == (dtype if b == 1 else dd.SURVEY_BIN_DTYPE[dtype])
        assert ri["split_planes"] == (dtype == "u16" and b > 1)
        if b > 1:  # binned sums: uint16 for 8/4-bit input, two uint16 planes for 16-bit, float32 for float
            need += cfg["n_chan"] * (n_samp // b) * (2 if dd.BIN_OUT[dtype] == "u16" else 4)
    assert s.workspace_bytes >= need


def test_survey_errors(dd):
    cfg = synth.CONFIGS["small"]
    base = (cfg["n_chan"], cfg["n_samp"], "u8", cfg["f_high"], cfg["chan_bw"], cfg["t_samp"])

    def make(ranges, **kw):
        args = list(base)
        for i, k in enumerate(["n_chan", "n_samp", "dtype"]):
            if k in kw:
                args[i] = kw[k]
        return dd.Survey(*args, ranges, bind=False)
    assert _status(dd, lambda: make([(0.0, 1.0, 10, 0)])) == "DD_ERR_ARG"
    assert _status(dd, lambda: make([(0.0, 1.0, 10, 257)])) == "DD_ERR_ARG"
    assert _status(dd, lambda: make([(0.0, 1.0, 10, 64)], n_samp=48)) == "DD_ERR_TOO_SHORT"
    with pytest.raises(dd.DDError) as e:  # the binned range is too short for its delays
        make([(0.0, 1.0, 10, 1), (0.0, 20.0, 256, 16)])
    assert e.value.name == "DD_ERR_TOO_SHORT" and "range 1" in str(e.value)
    assert _status(dd, lambda: make([(0.0, 1.0, 10, 1)], dtype="u4", n_samp=32767)) == "DD_ERR_ARG"
    make([(0.0, 1.0, 10, 2)], dtype="u4", n_samp=32767)  # odd length is fine once binned
    assert _status(dd, lambda: make([])) == "DD_ERR_ARG"


def test_corner_turn_argument_checks(dd):
    lib = ctypes.CDLL(dd.LIB_PATH)
    lib.dd_corner_turn.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    a, b = 1 << 20, 1 << 30
    ok = dict(dtype=1, d_in=a, in_pitch=112, n_chan=100, n_samp=1000, d_out=b, out_pitch=1008)

    def call(**kw):
        k = dict(ok, **kw)
        return lib.dd_corner_turn(k["dtype"], k["d_in"], k["in_pitch"], k["n_chan"], k["n_samp"], k["d_out"],
                                  k["out_pitch"], None)
    assert call(dtype=0) == -1 and call(d_in=0) == -1 and call(n_chan=0) == -1 and call(n_samp=0) == -1
    assert call(dtype=2, n_samp=999) == -1            # 4-bit rows pack time pairs
    assert call(in_pitch=96) == -1                    # a spectrum of 100 channels needs 100 bytes
    assert call(in_pitch=104) == -4                   # not a multiple of 16
    assert call(out_pitch=992) == -1 and call(out_pitch=1000) == -4
    assert call(d_in=a + 4) == -4
    assert call(d_out=a + 64) == -1                   # overlaps the spectra
    assert call(dtype=4, in_pitch=192) == -1          # 16-bit spectra of 100 channels take 200 bytes
    assert call(dtype=2, in_pitch=48, out_pitch=496) == -1  # 4-bit rows of 1000 samples take 500 bytes


def test_survey_time_major_layout(dd):
    """A time-major survey plans the same ranges and adds the turned copy to its workspace."""
    cfg = synth.CONFIGS["small"]
    args = (cfg["n_chan"], cfg["n_samp"], "u8", cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], SURVEY_RANGES)
    cm = dd.Survey(*args, bind=False)
    tm = dd.Survey(*args, in_pitch_bytes=128, bind=False, time_major=True)
    for r in range(len(SURVEY_RANGES)):
        assert np.array_equal(cm.shift(r), tm.shift(r))
        assert cm.range_info[r]["n_out"] == tm.range_info[r]["n_out"]
    assert tm.workspace_bytes >= cm.workspace_bytes + cfg["n_chan"] * cfg["n_samp"]
    with pytest.raises(dd.DDError) as e:  # spectrum pitch below one spectrum of 128 channels
        dd.Survey(*args, in_pitch_bytes=112, bind=False, time_major=True)
    assert e.value.name == "DD_ERR_ARG"


def test_large_spread_plan_uses_direct_kernel(dd):
    """8- and 16-bit plans whose delay spread leaves only LDS stages of at most 4 channels (16-bit:
    other than its preferred 8-wave shape), and every 4-bit plan, default to the direct-read
    kernel (no staging: row_block 0), whose table is the plain shift table: 4 rows x 4 waves for
    8- and 16-bit samples, 2 rows x 8 waves for 4-bit samples; grid order 1, except 8-bit plans
    too wide for 4-channel stages (order 2)."""
    cfg = synth.CONFIGS["lowfreq_wide"]
    p = _plan(dd, cfg)
    t = p.tiles(0)
    assert t["row_block"] == 0 and t["shape"] >= p.n_shapes - 2  # the two direct-read shapes come last
    assert t["per_wave"] == 4 and t["waves"] == 4
    t16 = _plan(dd, synth.CONFIGS["lowfreq_wide_u16"]).tiles(0)
    assert t16["row_block"] == 0 and t16["per_wave"] == 4 and t16["waves"] == 4
    assert p.info.dev_table_bytes >= cfg["n_dm"] * cfg["n_chan"] * 4
    assert p.info.tune_ws_bytes >= p.info.dev_table_bytes
    for name in ["small", "headline", "headline_u16"]:  # narrow spreads keep LDS staging
        assert _plan(dd, synth.CONFIGS[name]).tiles(0)["row_block"] > 0
    # a moderate spread (4-channel stages at best) reads directly for 8- and 16-bit samples
    mid = dict(cfg, n_samp=1 << 19, dm_step=0.1, n_dm=2048)
    for dt in ("u8", "u16"):
        tm = _plan(dd, dict(mid, dtype=dt)).tiles(0)
        assert tm["row_block"] == 0 and tm["per_wave"] == 4 and tm["order"] == 1, (dt, tm)
    for c in [synth.CONFIGS["lowfreq_u4"], synth.CONFIGS["headline_u4"], dict(cfg, dtype="u4"),
              dict(synth.CONFIGS["small"], dtype="u4")]:  # 4-bit: direct reads for any spread
        t4 = _plan(dd, c).tiles(0)
        assert t4["row_block"] == 0 and t4["per_wave"] == 2 and t4["waves"] == 8 and t4["order"] == 1


def test_batch_tile_choice_host(dd):
    """Batch shape selection on the host: by default each beam runs its plan's own shape (staged,
    or direct-read for a wide delay spread), set_tiles switches or refuses (DD_ERR_RANGE, batch
    unchanged), and the workspace size does not depend on the shape."""
    lib = ctypes.CDLL(dd.LIB_PATH)
    lib.dd_batch_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]
    lib.dd_batch_workspace_bytes.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]
    lib.dd_batch_get_tiles.argtypes = [ctypes.c_void_p, ctypes.POINTER(dd.binding.Tiles)]
    lib.dd_batch_set_tiles.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.dd_batch_destroy.argtypes = [ctypes.c_void_p]
    small = synth.CONFIGS["small"]
    wide = dict(small, n_chan=64, chan_bw=0.3, dm_step=40.0, n_dm=40, n_samp=1 << 17)  # a wide delay spread
    # a spread of ~4000 samples per 16 DM rows at 120-190 MHz: the plan reads directly
    widest = dict(small, n_chan=256, f_high=190.0, chan_bw=70.0 / 256, t_samp=327.68e-6, dm_step=0.5, n_dm=100,
                  n_samp=1 << 17)
    plans = [_plan(dd, small), _plan(dd, wide), _plan(dd, widest)]
    assert plans[2].tiles(0)["row_block"] == 0
    arr = (ctypes.c_void_p * 3)(*[p._h for p in plans])
    h = ctypes.c_void_p()
    assert lib.dd_batch_create(arr, 3, ctypes.byref(h)) == 0
    try:
        t = dd.binding.Tiles()
        assert lib.dd_batch_get_tiles(h, ctypes.byref(t)) == 0
        ws0 = ctypes.c_size_t()
        lib.dd_batch_workspace_bytes(h, ctypes.byref(ws0))
        first = t.shape
        n_staged = plans[0].n_shapes - 2  # the staged shapes; the two direct-read shapes follow them
        assert lib.dd_batch_set_tiles(h, n_staged + 2) == -1 and lib.dd_batch_set_tiles(h, -1) == -1
        ok, segs = [], {}
        for s in range(n_staged + 2):
            rc = lib.dd_batch_set_tiles(h, s)
            assert rc in (0, -3), rc
            lib.dd_batch_get_tiles(h, ctypes.byref(t))
            if rc == 0:
                ok.append(s)
                segs[s] = t.segs
                assert t.shape == s
            ws = ctypes.c_size_t()
            lib.dd_batch_workspace_bytes(h, ctypes.byref(ws))
            assert ws.value == ws0.value
        assert ok and len(ok) < n_staged + 2  # the wide beam rules some staged shapes out
        assert n_staged in ok and n_staged + 1 in ok  # the direct-read shapes take any spread
        lib.dd_batch_set_tiles(h, n_staged + 1)
        lib.dd_batch_get_tiles(h, ctypes.byref(t))
        assert t.row_block == 0 and t.per_wave == 2 and t.waves == 8
        # the default: every beam on its plan's own shape, staged or direct-read, else (a staged
        # shape whose LDS need falls in the persistent kernel's own 64 bytes) on the first staged
        # shape that holds it (phase-load shapes first); here the two beams differ
        assert first == -1
    finally:
        lib.dd_batch_destroy(h)
    # a fresh batch reports each beam's default
    lib.dd_batch_get_beam_tiles.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(dd.binding.Tiles)]
    h = ctypes.c_void_p()
    assert lib.dd_batch_create(arr, 3, ctypes.byref(h)) == 0
    try:
        for b, p in enumerate(plans):
            t = dd.binding.Tiles()
            assert lib.dd_batch_get_beam_tiles(h, b, ctypes.byref(t)) == 0
            own = p.tiles(0)
            assert (t.row_block > 0) == (own["row_block"] > 0)
            if own["row_block"] == 0:
                assert t.shape == own["shape"]  # the plan's direct-read shape
            else:
                # the plan's own shape, unless its LDS need falls in the 64 bytes the persistent
                # kernel keeps for itself: then a later staged shape
                assert t.shape >= own["shape"]
                if b == 0:
                    assert t.shape == own["shape"]
        assert lib.dd_batch_get_beam_tiles(h, 3, ctypes.byref(t)) == -1
    finally:
        lib.dd_batch_destroy(h)


def test_package_without_library_fails_loudly(tmp_path):
    """A copy of the package without libdd.so must refuse to import: there is no
    other execution path (no CPU fallback, no route through the oracle)."""
    import shutil
    import subprocess
    import sys
    src = os.path.join(ROOT, "paper_2311_05341_amd")
    dst = tmp_path / "paper_2311_05341_amd"
    shutil.copytree(src, dst, ignore=shutil.ignore_patterns("*.so", "__pycache__", "csrc", "cpu"))
    assert not list(dst.glob("*.so"))
    code = ("import sys\n"
            "try:\n"
            "    import paper_2311_05341_amd\n"
            "except ImportError as e:\n"
            "    print('refused:', e); sys.exit(0)\n"
            "sys.exit('imported without libdd.so')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True, text=True,
                       timeout=300, env=dict(os.environ, PYTHONPATH=str(tmp_path)))
    assert r.returncode == 0, r.stdout + r.stderr
    assert "libdd.so is not built" in r.stdout
