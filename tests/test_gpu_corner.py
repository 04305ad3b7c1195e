"""GPU parity of the input corner turn and of time-major surveys against the oracle.

The corner turn moves bytes only, so every output byte must equal the
oracle's; bytes of the row pitch beyond the row must stay untouched.  A
time-major survey (turn + binning + every range) must equal the oracle's
corner turn followed by its binning and transform, bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import sample_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import paper_2311_05341_amd as dd
    assert torch.cuda.is_available()
    return dd


_ES = {"u8": 1, "u16": 2, "f32": 4}
_NP = {"u8": np.uint8, "u4": np.uint8, "u16": np.uint16, "f32": np.float32}


def _to_dev(x):
    if x.dtype == np.uint16:
        return torch.from_numpy(x.view(np.int16)).cuda().view(torch.uint16)
    return torch.from_numpy(x).cuda()


def _bytes_of(t):
    if t.dtype == torch.uint16:
        t = t.view(torch.int16)
    return t.cpu().numpy().view(np.uint8)


def _spectra(dtype, n_chan, n_samp, seed):
    """Random spectra with a padded pitch whose padding holds the largest value."""
    rng = np.random.default_rng(seed)
    sb = (n_chan + 1) // 2 if dtype == "u4" else n_chan * _ES[dtype]
    pitch = (sb + 16 + 15) // 16 * 16
    if dtype == "f32":
        x = np.full((n_samp, pitch // 4), 3.0e38, dtype=np.float32)
        x[:, :n_chan] = rng.standard_normal((n_samp, n_chan))
    elif dtype == "u16":
        x = np.full((n_samp, pitch // 2), 65535, dtype=np.uint16)
        x[:, :n_chan] = rng.integers(0, 65536, (n_samp, n_chan))
    else:
        x = np.full((n_samp, pitch), 255, dtype=np.uint8)
        x[:, :sb] = rng.integers(0, 256, (n_samp, sb))
    return x


def _check_turn(dd, dtype, n_chan, n_samp, seed):
    spec = _spectra(dtype, n_chan, n_samp, seed)
    row = n_samp // 2 if dtype == "u4" else n_samp * _ES[dtype]
    opitch = (row + 16 + 15) // 16 * 16
    es = 1 if dtype == "u4" else _ES[dtype]
    out_h = np.full((n_chan, opitch // es), 0, dtype=_NP[dtype])
    out_h.view(np.uint8)[:] = 0xA5
    out = _to_dev(out_h)
    print("corner turn %s n_chan=%d n_samp=%d" % (dtype, n_chan, n_samp), flush=True)
    dd.corner_turn(_to_dev(spec), dtype, n_chan, n_samp, out=out)
    torch.cuda.synchronize()
    got = _bytes_of(out)
    want = oracle.corner_turn(spec, dtype, n_chan, n_samp).view(np.uint8)
    assert np.array_equal(got[:, :row], want[:, :row])
    assert np.all(got[:, row:] == 0xA5), "wrote past the row"


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "f32"])
def test_corner_turn_shapes(dtype, dd):
    """Whole and partial tiles in both directions, single channel or sample pair, odd channel counts."""
    for i, (n_chan, n_samp) in enumerate([(1, 2), (5, 130), (257, 1000), (300, 4098), (1000, 514), (64, 32),
                                          (513, 258)]):
        _check_turn(dd, dtype, n_chan, n_samp, seed=10 + i)


def test_corner_turn_large(dd):
    _check_turn(dd, "u8", 8192, 20000, seed=3)
    _check_turn(dd, "u4", 4097, 30000, seed=4)


def _survey_args(cfg, n_samp):
    return (cfg["n_chan"], n_samp, cfg["dtype"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], cfg["ranges"])


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "f32"])
def test_time_major_survey_small_exact(dtype, dd):
    """Spectra in, every range out: the oracle's corner turn, binning and transform. Integer
    encodings bit for bit (binned 16-bit ranges too: the oracle sums the exact 32-bit bin sums);
    float spectra within 1e-5 of the sum of |terms|."""
    cfg = dict(synth.SURVEYS["survey_small"], dtype=dtype)
    n_chan, n_samp = cfg["n_chan"], cfg["n_samp"]
    spec = _spectra(dtype, n_chan, n_samp, seed=21)
    rows = oracle.corner_turn(spec, dtype, n_chan, n_samp)
    sv = dd.Survey(*_survey_args(cfg, n_samp), in_pitch_bytes=spec.strides[0], time_major=True)
    outs = sv.run(_to_dev(spec))
    torch.cuda.synchronize()
    for r, (start, step, n_dm, b) in enumerate(cfg["ranges"]):
        s = oracle.shift_table(n_chan, cfg["f_high"], cfg["chan_bw"], cfg["t_samp"] * b, start, step, n_dm)
        got = outs[r].cpu().numpy()
        if b == 1 and dtype != "f32":
            assert np.array_equal(got, oracle.forward(rows, dtype, n_samp, s)), r
        elif b == 1:
            want, ab = oracle.forward_f32(rows, n_samp, s)
            assert np.all(np.abs(got.astype(np.float64) - want) <= 1e-5 * ab + 1e-30), r
        elif dtype in ("u8", "u4"):
            xb = oracle.bin_time(rows, dtype, n_samp, b).astype(np.uint16)
            assert np.array_equal(got, oracle.forward(xb, "u16", xb.shape[1], s)), r
        elif dtype == "u16":
            xb = oracle.bin_time(rows, dtype, n_samp, b).astype(np.uint32)
            assert np.array_equal(got, oracle.forward(xb, "u32", xb.shape[1], s)), r
        else:  # float rows bin to float sums
            xb = oracle.bin_time(rows, dtype, n_samp, b)
            ab_b = oracle.bin_time(np.abs(rows.astype(np.float64)).astype(np.float32), dtype, n_samp, b)
            want, _ = oracle.forward_f32(np.ascontiguousarray(xb.astype(np.float32)), xb.shape[1], s)
            ab, _ = oracle.forward_f32(np.ascontiguousarray(ab_b.astype(np.float32)), xb.shape[1], s)
            assert np.all(np.abs(got.astype(np.float64) - want) <= 1e-5 * ab + 1e-30), r


def test_time_major_pipeline_full_size(dd):
    """pipeline_high with time-major input, as bench.py --time-major runs it: spectra generated
    on the device and reproduced on the host; sampled rows of every range bit-exact."""
    cfg = synth.SURVEYS["pipeline_high"]
    n_chan, n_samp = cfg["n_chan"], cfg["n_samp"]
    print("time-major pipeline_high: generating spectra", flush=True)
    spec_d = torch.empty((n_samp, n_chan), dtype=torch.uint8, device="cuda")
    table = torch.from_numpy(synth.gaussian_table()).cuda()
    synth.gaussian_u8_device(spec_d.data_ptr(), n_samp, n_chan, n_chan, cfg["seed"], table.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    spec = synth.gaussian_u8(n_samp, n_chan, cfg["seed"])
    torch.cuda.synchronize()
    for t in (0, 12345, n_samp - 1):
        assert np.array_equal(spec_d[t].cpu().numpy(), spec[t])
    sv = dd.Survey(*_survey_args(cfg, n_samp), in_pitch_bytes=n_chan, time_major=True)
    outs = sv.run(spec_d)
    torch.cuda.synchronize()
    print("time-major pipeline_high: oracle corner turn", flush=True)
    rows = oracle.corner_turn(spec, "u8", n_chan, n_samp)
    del spec
    for r, (start, step, n_dm, b) in enumerate(cfg["ranges"]):
        print("time-major pipeline_high: range %d" % r, flush=True)
        s = oracle.shift_table(n_chan, cfg["f_high"], cfg["chan_bw"], cfg["t_samp"] * b, start, step, n_dm)
        picks = sample_rows(n_dm, extra=2, seed=30 + r)
        if b == 1:
            want = oracle.forward(rows, "u8", n_samp, s, rows=picks)
        else:
            xb = np.empty((n_chan, n_samp // b), dtype=np.uint16)
            for c0 in range(0, n_chan, 512):
                xb[c0:c0 + 512] = oracle.bin_time(np.ascontiguousarray(rows[c0:c0 + 512]), "u8", n_samp, b)
            want = oracle.forward(xb, "u16", n_samp // b, s, rows=picks)
        assert np.array_equal(outs[r][picks].cpu().numpy(), want), r
