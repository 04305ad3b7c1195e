"""Host-side checks of tile-shape selection (no GPU needed).

Every compiled shape either holds a plan's delay spread (then its tables fit
the tuning workspace bound) or is refused with DD_ERR_RANGE, leaving the plan
as it was.  The tuning cache applies a recorded choice to an identical plan
and ignores lines whose shape parameters do not match the library's.
"""
import ctypes

import numpy as np
import pytest

import synth


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


def _status(dd, fn):
    with pytest.raises(dd.DDError) as e:
        fn()
    return e.value.name


@pytest.mark.parametrize("name", ["small", "lowfreq_u4", "headline_u16", "grad_f32"])
def test_every_shape_feasible_or_refused(dd, name):
    cfg = synth.CONFIGS[name]
    p = _plan(dd, cfg)
    dirs = [0, 1] if cfg["dtype"] == "f32" else [0]
    bound = p.info.tune_ws_bytes
    assert p.info.dev_table_bytes <= bound
    for direction in dirs:
        ok = 0
        for s in range(p.n_shapes):
            for o in (0, 1, 2, 3):
                before = p.tiles(direction)
                try:
                    p.set_tiles(direction, s, o)
                except dd.DDError as e:
                    assert e.name == "DD_ERR_RANGE"
                    assert p.tiles(direction) == before
                    continue
                ok += 1
                t = p.tiles(direction)
                assert (t["shape"], t["order"]) == (s, o)
                assert p.info.dev_table_bytes <= bound
                if direction == 0:
                    assert (p.info.kernel_ns, p.info.kernel_dm_per_wave, p.info.kernel_waves,
                            p.info.kernel_chan_block, p.info.kernel_order) == (
                        t["ns"], t["per_wave"], t["waves"], t["row_block"], o)
        assert ok >= 2  # at least one shape, in both orders


def test_tiles_argument_errors(dd):
    p = _plan(dd, synth.CONFIGS["small"])
    assert _status(dd, lambda: p.tiles(1)) == "DD_ERR_DTYPE"
    assert _status(dd, lambda: p.set_tiles(1, 0, 0)) == "DD_ERR_DTYPE"
    assert _status(dd, lambda: p.set_tiles(0, p.n_shapes, 0)) == "DD_ERR_ARG"
    assert _status(dd, lambda: p.set_tiles(0, -1, 0)) == "DD_ERR_ARG"
    assert _status(dd, lambda: p.set_tiles(0, 0, 4)) == "DD_ERR_ARG"


def test_default_tiles_grouped_order(dd):
    for name in ["small", "headline", "headline_u16", "grad_f32", "lowfreq_wide"]:
        p = _plan(dd, synth.CONFIGS[name])
        assert p.tiles(0)["order"] == 2
        assert p.info.kernel_order == 2
    # direct-read plans (every 4-bit plan, 16-bit ones, 8-bit ones of moderate spread): whole
    # time tiles per XCD; the widest 8-bit plans (at most 2 channels per stage) keep order 2
    for name in ["lowfreq_u4", "headline_u4", "lowfreq_wide_u16"]:
        p = _plan(dd, synth.CONFIGS[name])
        assert p.tiles(0)["row_block"] == 0 and p.tiles(0)["order"] == 1 and p.info.kernel_order == 1


_KEY_FMT = (b"dtype=%d,nchan=%d,nsamp=%lld,fhigh=%a,bw=%a,freqs=%016llx,tsamp=%a,dm0=%a,dmstep=%a,ndm=%d,"
            b"pitch=%lld,dir=%d")


def _cache_key(cfg, dtype_code, pitch, direction):
    """The cache's plan key, formatted by the C library's own printf (hex-float doubles)."""
    libc = ctypes.CDLL(None)
    buf = ctypes.create_string_buffer(600)
    d = ctypes.c_double
    libc.snprintf(buf, 600, _KEY_FMT, ctypes.c_int(dtype_code), ctypes.c_int(cfg["n_chan"]),
                  ctypes.c_longlong(cfg["n_samp"]), d(cfg["f_high"]), d(cfg["chan_bw"]), ctypes.c_ulonglong(0),
                  d(cfg["t_samp"]), d(cfg["dm_start"]), d(cfg["dm_step"]), ctypes.c_int(cfg["n_dm"]),
                  ctypes.c_longlong(pitch), ctypes.c_int(direction))
    return buf.value.decode()


def test_tune_cache_applied(dd, tmp_path, monkeypatch):
    cfg = synth.CONFIGS["small"]
    p0 = _plan(dd, cfg)
    feasible = []
    for s in range(p0.n_shapes):
        try:
            p0.set_tiles(0, s, 1)
            feasible.append((s, p0.tiles(0)))
        except dd.DDError:
            pass
    assert len(feasible) >= 2
    shape, t = feasible[-1]
    key = _cache_key(cfg, 1, p0.in_pitch_bytes, 0)
    path = tmp_path / "tune.txt"
    other_key = key.replace("ndm=%d" % cfg["n_dm"], "ndm=%d" % (cfg["n_dm"] + 1))
    params = "%d %d %d %d" % (t["ns"], t["per_wave"], t["waves"], t["row_block"])
    path.write_text("dd-tune-v2 %s %d 1 %s 1.0\n" % (key, shape, params) +
                    "dd-tune-v2 %s 0 0 %s 1.0\n" % (other_key, params) +
                    "garbage line\n")
    monkeypatch.setenv("DD_TUNE_CACHE", str(path))
    p = _plan(dd, cfg)
    assert (p.tiles(0)["shape"], p.tiles(0)["order"]) == (shape, 1)
    # a line whose shape parameters disagree with the compiled shape is ignored
    path.write_text("dd-tune-v2 %s %d 1 %d %s 1.0\n" % (key, shape, t["ns"] + 1, params.split(" ", 1)[1]))
    p = _plan(dd, cfg)
    assert p.tiles(0)["order"] == 2
    # a different plan does not pick up the line
    path.write_text("dd-tune-v2 %s %d 1 %s 1.0\n" % (key, shape, params))
    p = _plan(dd, cfg, n_dm=cfg["n_dm"] - 1)
    assert p.tiles(0)["order"] == 2
    monkeypatch.delenv("DD_TUNE_CACHE")
    p = _plan(dd, cfg)
    assert p.tiles(0)["order"] == 2


@pytest.mark.parametrize("dtype,n_chunks", [("u8", 1), ("u8", 3), ("u4", 4), ("u16", 3), ("f32", 5)])
def test_time_chunks_cover_the_output(dd, dtype, n_chunks):
    cfg = dict(synth.CONFIGS["small"], dtype=dtype)
    desc = {k: cfg[k] for k in ["n_chan", "n_samp", "dtype", "f_high", "chan_bw", "t_samp", "dm_start", "dm_step",
                                "n_dm"]}
    tc = dd.TimeChunks(desc, n_chunks, bind=False)
    whole = _plan(dd, cfg)
    assert tc.n_out == whole.n_out and tc.max_shift == whole.max_shift
    assert len(tc) == n_chunks
    unit = {"u8": 16, "u4": 32, "u16": 8, "f32": 4}[dtype]
    t = 0
    for (t0, n), p in zip(tc.spans, tc.plans):
        assert t0 == t and t0 % unit == 0 and n > 0
        assert p.max_shift == whole.max_shift and p.in_pitch_bytes == whole.in_pitch_bytes
        assert p.n_out == n or (dtype == "u4" and p.n_out == n + 1 and t0 + n < whole.n_out)
        assert np.array_equal(p.shift, whole.shift)
        t += n
    assert t == whole.n_out


def test_16bit_default_takes_the_phase_load_shape(dd):
    """16-bit plans take the 8-wave, 4-rows-per-wave, 4-channel shape in its phase-load form
    when two of its workgroups fit in a CU's LDS (the headline plan), its raw-ring form
    otherwise when that fits twice; when neither does, the first staged shape that holds the
    spread, or the direct-read shape when that one stages at most 4 channels."""
    def key(t):
        return (t["ns"], t["per_wave"], t["waves"], t["row_block"])
    p = _plan(dd, synth.CONFIGS["headline_u16"])
    t = p.tiles(0)
    assert key(t) == (16, 4, 8, 4) and t["segs"] > 0 and t["order"] == 2
    # the 120-190 MHz plan with 16-bit samples: 32 DMs spread over 1638 samples, rows too
    # long for two workgroups of either form; the first staged shape that holds it stages 4
    # channels at a time, so the plan reads directly
    p = _plan(dd, dict(synth.CONFIGS["lowfreq_u4"], dtype="u16"))
    t = p.tiles(0)
    assert t["row_block"] == 0 and key(t) == (16, 4, 4, 0) and t["order"] == 1
    first = None
    for s in range(p.n_shapes - 2):
        try:
            p.set_tiles(0, s, 2)
        except dd.DDError:
            continue
        first = p.tiles(0)
        break
    assert first is not None and first["row_block"] <= 4 and key(first) != (16, 4, 8, 4)
