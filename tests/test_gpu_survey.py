"""GPU parity of time binning and of multi-range (binned) DM plans against the oracle.

Binning: integer inputs bit-exact; float input within the recursive-summation
bound (factor - 1) * 2^-24 * sum|x| per bin.  Surveys: every range compared
with the oracle's binning followed by the oracle's transform on the binned
grid (t_samp * bin), bit-exact for integer input.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import row_sums_by_prefix, sample_rows

pytestmark = pytest.mark.gpu

FACTORS = [1, 2, 3, 4, 5, 7, 8, 16, 32, 64, 100, 128, 255, 256]


@pytest.fixture(scope="module")
def dd():
    import paper_2311_05341_amd as dd
    assert torch.cuda.is_available()
    return dd


def _host(dtype, n_chan, n_samp, pitch_elems, seed):
    """Random rows with the padding beyond the row filled with the largest value."""
    rng = np.random.default_rng(seed)
    if dtype == "u8":
        x = np.full((n_chan, pitch_elems), 255, dtype=np.uint8)
        x[:, :n_samp] = rng.integers(0, 256, (n_chan, n_samp))
    elif dtype == "u4":
        x = np.full((n_chan, pitch_elems), 255, dtype=np.uint8)
        v = rng.integers(0, 16, (n_chan, n_samp + (n_samp & 1))).astype(np.uint8)
        x[:, :(n_samp + 1) // 2] = v[:, 0::2] | (v[:, 1::2] << 4)
        if n_samp & 1:  # the unused high nibble of the last byte
            x[:, n_samp // 2] |= 0xF0
    elif dtype == "u16":
        x = np.full((n_chan, pitch_elems), 65535, dtype=np.uint16)
        x[:, :n_samp] = rng.integers(0, 65536, (n_chan, n_samp))
    else:
        x = np.full((n_chan, pitch_elems), 3.0e38, dtype=np.float32)
        x[:, :n_samp] = rng.standard_normal((n_chan, n_samp)).astype(np.float32)
    return x


def _to_dev(x):
    if x.dtype == np.uint16:  # no uint16 host-to-device path in torch: copy the bytes
        return torch.from_numpy(x.view(np.int16)).cuda().view(torch.uint16)
    return torch.from_numpy(x).cuda()


def _to_host(t):
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


_ELEM = {"u8": 1, "u4": 1, "u16": 2, "f32": 4}


def _check_bin(dd, dtype, n_chan, n_samp, factor, seed):
    row_bytes = {"u8": n_samp, "u4": (n_samp + 1) // 2, "u16": 2 * n_samp, "f32": 4 * n_samp}[dtype]
    pitch = (row_bytes + 16 + 15) // 16 * 16  # one spare 16-byte chunk of padding per row
    xh = _host(dtype, n_chan, n_samp, pitch // _ELEM[dtype], seed)
    n_bins = n_samp // factor
    odt = dd.BIN_OUT[dtype]
    ob = _ELEM[odt]
    opitch = (n_bins * ob + 16 + 15) // 16 * 16
    sentinel = 12345 if odt == "u16" else -7.5
    out_h = np.full((n_chan, opitch // ob), sentinel, dtype=np.uint16 if odt == "u16" else np.float32)
    out = _to_dev(out_h)
    print("bin %s n_chan=%d n_samp=%d factor=%d" % (dtype, n_chan, n_samp, factor), flush=True)
    dd.bin_time(_to_dev(xh), dtype, n_samp, factor, out=out)
    torch.cuda.synchronize()
    got = _to_host(out)
    assert np.all(got[:, n_bins:] == sentinel), "wrote past the last whole bin"
    want = oracle.bin_time(np.ascontiguousarray(xh), dtype, n_samp, factor)
    if dtype == "f32":
        absum = oracle.bin_time(np.abs(xh), "f32", n_samp, factor)
        err = np.abs(got[:, :n_bins].astype(np.float64) - want)
        assert np.all(err <= 1.01 * (factor - 1) * 2.0 ** -24 * absum + 1e-30), (factor, float(err.max()))
    else:
        assert np.array_equal(got[:, :n_bins].astype(np.int64), want)


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "f32"])
def test_bin_every_kernel_form(dtype, dd):
    """Chunk, group and generic kernels; ragged lengths (partial chunks, a dropped partial bin)."""
    for i, f in enumerate(FACTORS):
        _check_bin(dd, dtype, 5, 20011 + 2 * i, f, seed=100 + i)


def test_bin_edge_cases(dd):
    # exactly one bin; a row of one chunk; more rows than one grid dimension holds
    _check_bin(dd, "u8", 3, 256, 256, seed=1)
    _check_bin(dd, "u4", 2, 33, 32, seed=2)
    _check_bin(dd, "u16", 70000, 48, 2, seed=3)
    _check_bin(dd, "f32", 70000, 12, 3, seed=4)


def test_bin_zero_bins_rejected(dd):
    x = torch.zeros((2, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(dd.DDError) as e:
        dd.bin_time(x, "u8", 10, 16)
    assert e.value.name == "DD_ERR_TOO_SHORT"


def _oracle_range(xh, dtype, n_samp, cfg, rng_):
    """Oracle result of one range of an integer-input survey: (table, values).

    The oracle bins exactly (int64) and sums the bins of 8- and 4-bit input as
    16-bit samples, of 16-bit input as 32-bit samples (bin sums reach 2^24)."""
    start, step, n_dm, b = rng_
    s = oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"] * b, start, step, n_dm)
    if b == 1:
        return s, oracle.forward(xh, dtype, n_samp, s)
    xb = oracle.bin_time(xh, dtype, n_samp, b)
    wide = "u16" if dtype in ("u8", "u4") else "u32"
    return s, oracle.forward(np.ascontiguousarray(xb.astype(np.uint16 if wide == "u16" else np.uint32)), wide,
                             xb.shape[1], s)


def _survey(dd, cfg, dtype, n_samp, pitch_bytes=0):
    return dd.Survey(cfg["n_chan"], n_samp, dtype, cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], cfg["ranges"],
                     in_pitch_bytes=pitch_bytes)


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16"])
def test_survey_small_exact(dtype, dd):
    """Every output of every range bit-exact: binned ranges run the 16-bit kernel on exact uint16 sums
    (8- and 4-bit input), or on the low and high uint16 halves of the exact bin sums (16-bit input)
    combined once into the float32 of the exact total."""
    cfg = synth.SURVEYS["survey_small"]
    n_samp = cfg["n_samp"]
    row = {"u8": n_samp, "u4": n_samp // 2, "u16": 2 * n_samp}[dtype]
    pitch = (row + 64 + 15) // 16 * 16
    xh = _host(dtype, cfg["n_chan"], n_samp, pitch // _ELEM[dtype], seed=cfg["seed"])
    if dtype == "u8":
        for dm, width, t0 in cfg["pulses"]:
            sh = oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], dm, 0.0, 1)[0]
            synth.inject_boxcar_u8(xh, sh, t0, width, cfg["amp"])
    sv = _survey(dd, cfg, dtype, n_samp, pitch)
    print("survey_small %s" % dtype, flush=True)
    outs = sv.run(_to_dev(xh))
    torch.cuda.synchronize()
    for r, rg in enumerate(cfg["ranges"]):
        s, want = _oracle_range(xh, dtype, n_samp, cfg, rg)
        assert np.array_equal(sv.shift(r), s)
        assert np.array_equal(outs[r].cpu().numpy(), want), r


def test_survey_u16_binned_exact_large_sums(dd):
    """Binned 16-bit ranges for factors whose sums need the high plane (8, 16, 256; and 6, an even
    factor that is not a multiple of 8), on uniform data and on all-65535 data: with bin sums up to
    256 * 65535 and channel sums up to 72 * 256 * 65535 (far past 2^24), every output equals the
    oracle's exact sum rounded once to float32."""
    n_chan, n_samp = 72, 1 << 16
    cfg = dict(n_chan=n_chan, f_high=1500.0, chan_bw=300.0 / n_chan, t_samp=64e-6)
    ranges = [(0.0, 1.0, 16, 8), (10.0, 2.0, 16, 16), (50.0, 4.0, 8, 256), (5.0, 1.5, 12, 6)]
    pitch = 2 * n_samp + 32
    for seed, fill in ((41, None), (42, 65535)):
        xh = _host("u16", n_chan, n_samp, pitch // 2, seed=seed)
        if fill is not None:
            xh[:, :n_samp] = fill
        sv = dd.Survey(n_chan, n_samp, "u16", cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], ranges,
                       in_pitch_bytes=pitch)
        assert all(ri["split_planes"] for ri in sv.range_info)
        outs = sv.run(_to_dev(xh))
        torch.cuda.synchronize()
        for r, rg in enumerate(ranges):
            s, want = _oracle_range(xh, "u16", n_samp, cfg, rg)
            got = outs[r].cpu().numpy()
            assert np.array_equal(got, want), (seed, r)
        if fill is not None:  # every output is the float32 of n_chan * factor * 65535
            for r, (_, _, _, b) in enumerate(ranges):
                assert (outs[r] == float(np.float32(n_chan * b * 65535))).all(), r


def test_survey_small_f32(dd):
    """Float input: binned float sums, then the float kernel; within 1e-5 of the sum of |terms|."""
    cfg = synth.SURVEYS["survey_small"]
    n_samp = cfg["n_samp"]
    xh = synth.normal_f32(cfg["n_chan"], n_samp, 11, pitch=(n_samp + 3) // 4 * 4)
    sv = _survey(dd, cfg, "f32", n_samp, xh.shape[1] * 4)
    outs = sv.run(torch.from_numpy(xh).cuda())
    torch.cuda.synchronize()
    for r, (start, step, n_dm, b) in enumerate(cfg["ranges"]):
        s = oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"] * b, start, step, n_dm)
        if b == 1:
            want, ab = oracle.forward_f32(xh, n_samp, s)
        else:
            xb = oracle.bin_time(xh, "f32", n_samp, b)
            abs_b = oracle.bin_time(np.abs(xh), "f32", n_samp, b)
            want, _ = oracle.forward_f32(np.ascontiguousarray(xb.astype(np.float32)), xb.shape[1], s)
            ab, _ = oracle.forward_f32(np.ascontiguousarray(abs_b.astype(np.float32)), xb.shape[1], s)
        got = outs[r].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - want) <= 1e-5 * ab + 1e-30), r


def test_survey_autotune_keeps_results(dd):
    cfg = synth.SURVEYS["survey_small"]
    n_samp = cfg["n_samp"]
    pitch = (n_samp + 15) // 16 * 16
    xh = _host("u8", cfg["n_chan"], n_samp, pitch, seed=5)
    sv = _survey(dd, cfg, "u8", n_samp, pitch)
    xd = _to_dev(xh)
    before = [o.cpu().numpy() for o in sv.run(xd)]
    sv.autotune(xd)
    after = [o.cpu().numpy() for o in sv.run(xd)]
    torch.cuda.synchronize()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)


def _device_survey_input(dd, cfg):
    n_chan, n_samp = cfg["n_chan"], cfg["n_samp"]
    pitch = (n_samp + 63) // 64 * 64
    xd = torch.empty((n_chan, pitch), dtype=torch.uint8, device="cuda")
    table = torch.from_numpy(synth.gaussian_table()).cuda()
    synth.gaussian_u8_device(xd.data_ptr(), n_chan, n_samp, pitch, cfg["seed"], table.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    xh = synth.gaussian_u8(n_chan, n_samp, cfg["seed"], pitch=pitch)
    for dm, width, t0 in cfg["pulses"]:
        sh = oracle.shift_table(n_chan, cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], dm, 0.0, 1)[0]
        rows, cols, vals, _ = synth.boxcar_updates(lambda r, c: xh[r, c], sh, t0, width, cfg["amp"])
        xh[rows, cols] = vals
        xd[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()] = torch.from_numpy(vals).cuda()
    torch.cuda.synchronize()
    return xd, xh, pitch


def _binned_u16(xh, n_samp, b, block=512):
    """The oracle's binning of a large u8 filterbank, a block of channels at a time, as uint16."""
    n_bins = n_samp // b
    out = np.empty((xh.shape[0], n_bins), dtype=np.uint16)
    for c0 in range(0, xh.shape[0], block):
        part = oracle.bin_time(np.ascontiguousarray(xh[c0:c0 + block]), "u8", n_samp, b)
        out[c0:c0 + block] = part
    return out


@pytest.mark.parametrize("name", ["tab_plans_8192", "pipeline_high"])
def test_survey_full_size_sampled(name, dd):
    """The benchmark's survey workloads at full size: sampled rows of every range bit-exact,
    every row of the unbinned ranges by the prefix-sum row-sum identity, pulses found."""
    cfg = synth.SURVEYS[name]
    print("survey %s: generating input" % name, flush=True)
    xd, xh, pitch = _device_survey_input(dd, cfg)
    sv = _survey(dd, cfg, "u8", cfg["n_samp"], pitch)
    outs = sv.run(xd)
    torch.cuda.synchronize()
    n_samp = cfg["n_samp"]
    binned = {}
    for r, (start, step, n_dm, b) in enumerate(cfg["ranges"]):
        print("survey %s: range %d" % (name, r), flush=True)
        s = oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"] * b, start, step, n_dm)
        assert np.array_equal(sv.shift(r), s)
        pulse_rows = [int(round((dm - start) / step)) for dm, _, _ in cfg["pulses"] if start <= dm < start + n_dm * step]
        rows = sample_rows(n_dm, [(p, 0, 0) for p in pulse_rows], extra=3, seed=r)
        if b == 1:
            want = oracle.forward(xh, "u8", n_samp, s, rows=rows)
        else:
            if b not in binned:
                binned[b] = _binned_u16(xh, n_samp, b)
            want = oracle.forward(binned[b], "u16", n_samp // b, s, rows=rows)
        got = outs[r][rows].cpu().numpy()
        assert np.array_equal(got, want), (r, rows)
        if b == 1:
            n_out = sv.range_info[r]["n_out"]
            gpu_rowsum = outs[r].double().sum(dim=1).cpu().numpy().astype(np.int64)
            assert np.array_equal(gpu_rowsum, row_sums_by_prefix(lambda c: xh[c, :n_samp], s, n_out))
        for (dm, width, t0), p in zip([q for q in cfg["pulses"] if start <= q[0] < start + n_dm * step], pulse_rows):
            col = outs[r][:, t0 // b].cpu().numpy()
            assert abs(int(np.argmax(col)) - p) <= 2, (r, dm, int(np.argmax(col)), p)
