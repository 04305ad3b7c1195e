"""GPU parity of the forward transform (Eq. 3) against the CPU oracle.

Integer inputs must match bit for bit.  Float inputs must satisfy
|gpu - oracle_fp64| <= 1e-5 * sum_c |terms| per element.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import host_input, oracle_table, plan_for, row_sums_by_prefix, sample_rows

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5


@pytest.fixture(scope="module")
def dd():
    import paper_2311_05341_amd as dd
    assert torch.cuda.is_available()
    return dd


def _to_dev(x):
    return torch.from_numpy(x).cuda()


def _gpu_forward(dd, plan, x_host):
    out = plan.forward(_to_dev(x_host))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_small_workload_exact(dd):
    """128 channels, 32768 samples, 256 DMs, injected pulse: every output bit-exact."""
    cfg = synth.CONFIGS["small"]
    s = oracle_table(cfg)
    x, applied = host_input(cfg, s)
    plan = plan_for(dd, cfg)
    assert np.array_equal(plan.shift, s)
    got = _gpu_forward(dd, plan, x)
    want = oracle.forward(x, "u8", cfg["n_samp"], s)
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    dp, width, t0 = cfg["pulses"][0]
    assert int(np.argmax(got[:, t0])) == dp


def _random_case(rng, dtype, n_chan, n_samp, n_dm):
    f_high = float(rng.uniform(300, 1600))
    bw = float(rng.uniform(0.05, 0.3)) * f_high / n_chan
    t_samp = float(rng.choice([64e-6, 128e-6, 256e-6]))
    k = 1 / (f_high - (n_chan - 1) * bw) ** 2 - 1 / f_high**2
    frac = float(rng.uniform(0.05, 0.7))
    dm_max = frac * n_samp * t_samp / (4.148808e3 * k) if k > 0 else 100.0
    start = float(rng.uniform(0, 0.3)) * dm_max
    step = (dm_max - start) / max(n_dm - 1, 1)
    return dict(dtype=dtype, n_chan=n_chan, n_samp=n_samp, f_high=f_high, chan_bw=bw, t_samp=t_samp,
                dm_start=start, dm_step=step, n_dm=n_dm)


RAGGED = [  # (n_chan, n_samp, n_dm): tails in every tile dimension, >256 channels, tiny outputs
    (1, 3000, 1), (5, 4111, 3), (17, 9000, 17), (33, 20000, 40), (130, 7001, 35),
    (300, 12345, 70), (600, 6000, 21), (257, 40000, 16), (64, 2050, 128),
]


@pytest.mark.parametrize("case", RAGGED)
@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "f32"])
def test_ragged_shapes(dd, dtype, case):
    n_chan, n_samp, n_dm = case
    if dtype == "u4":
        n_samp += n_samp & 1
    rng = np.random.default_rng(n_chan * 1000 + n_dm + {"u8": 0, "u4": 1, "f32": 2, "u16": 3}[dtype])
    cfg = _random_case(rng, dtype, n_chan, n_samp, n_dm)
    s = oracle_table(cfg)
    n_out = oracle.n_out_for(s, n_samp)
    if n_out <= 0:
        pytest.skip("plan leaves no output")
    elem = {"f32": 4, "u16": 2}.get(dtype, 1)
    row = n_samp // 2 if dtype == "u4" else n_samp * elem
    pitch_bytes = (row + 15) // 16 * 16 + 16 * int(rng.integers(0, 3))  # padded rows
    pitch = pitch_bytes // elem
    if dtype == "u8":
        x = rng.integers(0, 256, (n_chan, pitch)).astype(np.uint8)
        x[:, ::13] = 255
    elif dtype == "u4":
        x = rng.integers(0, 256, (n_chan, pitch)).astype(np.uint8)
    elif dtype == "u16":
        x = rng.integers(0, 65536, (n_chan, pitch)).astype(np.uint16)
        x[:, ::13] = 65535
    else:
        x = rng.standard_normal((n_chan, pitch)).astype(np.float32)
    plan = plan_for(dd, cfg, in_pitch_bytes=pitch_bytes)
    assert plan.n_out == n_out
    got = _gpu_forward(dd, plan, x)
    if dtype == "f32":
        want, ab = oracle.forward_f32(np.ascontiguousarray(x), n_samp, s)
        err = np.abs(got.astype(np.float64) - want)
        assert (err <= F32_TOL * ab + 1e-30).all(), float((err / np.maximum(ab, 1e-30)).max())
    else:
        want = oracle.forward(np.ascontiguousarray(x), dtype, n_samp, s)
        assert np.array_equal(got, want)


def test_zero_dm_step_and_single_channel(dd):
    """All delays zero (DM step 0): every row is the plain channel sum."""
    rng = np.random.default_rng(4)
    cfg = dict(dtype="u8", n_chan=40, n_samp=5000, f_high=1400.0, chan_bw=1.0, t_samp=64e-6,
               dm_start=0.0, dm_step=0.0, n_dm=9)
    x = rng.integers(0, 256, (40, 5008)).astype(np.uint8)
    plan = plan_for(dd, cfg, in_pitch_bytes=5008)
    got = _gpu_forward(dd, plan, x)
    want = x[:, :5000].sum(axis=0, dtype=np.int64).astype(np.float32)
    assert (got == want[None, :]).all()


def test_repeat_runs_bitwise_identical(dd):
    cfg = synth.CONFIGS["small"]
    s = oracle_table(cfg)
    x, _ = host_input(cfg, s)
    plan = plan_for(dd, cfg)
    xd = _to_dev(x)
    a = plan.forward(xd).clone()
    b = plan.forward(xd).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    xf = torch.randn(64, 8192, device="cuda")
    cf = dict(dtype="f32", n_chan=64, n_samp=8192, f_high=1500.0, chan_bw=2.0, t_samp=64e-6,
              dm_start=0.0, dm_step=2.0, n_dm=50)
    pf = plan_for(dd, cf)
    assert torch.equal(pf.forward(xf).clone(), pf.forward(xf).clone())


def _device_u8(cfg, s, pitch=None):
    """Generate a workload directly in GPU memory and on the host; apply pulses to both."""
    n_chan, n_samp = cfg["n_chan"], cfg["n_samp"]
    pitch = pitch or n_samp
    xd = torch.empty((n_chan, pitch), dtype=torch.uint8, device="cuda")
    table = torch.from_numpy(synth.gaussian_table()).cuda()
    synth.gaussian_u8_device(xd.data_ptr(), n_chan, n_samp, pitch, cfg["seed"], table.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    xh = synth.gaussian_u8(n_chan, n_samp, cfg["seed"], pitch=pitch)
    applied = {}
    for i, (dp, width, t0) in enumerate(cfg.get("pulses", [])):
        rows, cols, vals, app = synth.boxcar_updates(lambda r, c: xh[r, c], s[dp], t0, width, cfg["amp"])
        xh[rows, cols] = vals
        xd[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()] = torch.from_numpy(vals).cuda()
        applied[i] = app
    torch.cuda.synchronize()
    return xd, xh, applied


def test_headline_workload_sampled(dd):
    """8192 channels x 2^20 samples x 4000 DMs, as the benchmark times it.

    Sampled rows (DM 0, the pulse rows, the last row, every 400th and random
    rows) bit-exact against the oracle; every row checked by the prefix-sum
    row-sum identity and DM 0 by the plain channel sum; narrow pulses peak at
    their DM.
    """
    cfg = synth.CONFIGS["headline"]
    s = oracle_table(cfg)
    xd, xh, applied = _device_u8(cfg, s)
    for c in [0, 1, 4095, 8191]:  # the device generator reproduces the host bytes
        assert torch.equal(xd[c].cpu(), torch.from_numpy(xh[c]))
    plan = plan_for(dd, cfg)
    out = plan.forward(xd)
    torch.cuda.synchronize()
    n_out = plan.n_out
    rows = sample_rows(cfg["n_dm"], cfg["pulses"], every=400, extra=6, seed=2)
    got = out[rows].cpu().numpy()
    want = oracle.forward(xh, "u8", cfg["n_samp"], s, rows=rows)
    assert np.array_equal(got, want)
    gpu_rowsum = out.double().sum(dim=1).cpu().numpy().astype(np.int64)
    cpu_rowsum = row_sums_by_prefix(lambda c: xh[c], s, n_out)
    assert np.array_equal(gpu_rowsum, cpu_rowsum)
    dm0 = xh[:, :n_out].sum(axis=0, dtype=np.int64)
    assert np.array_equal(out[0].cpu().numpy().astype(np.int64), dm0)
    for i, (dp, width, t0) in enumerate(cfg["pulses"]):
        assert dp in rows and applied[i].sum() > 0  # the pulse rows were compared bit for bit above
        if width <= 4:
            # narrow pulses peak at their own DM; for wider boxcars the next DM up, whose
            # extra delay is smaller than the width, collects almost the whole pulse too
            col = out[:, t0].cpu().numpy()
            assert int(np.argmax(col)) == dp, (dp, int(np.argmax(col)))


def test_headline_shard8_workload_sampled(dd):
    """One GPU's share of the headline under 8-way DM sharding (DMs 1750..1999.5), as the
    benchmark times it: sampled rows, the pulse row among them, bit-exact; every row by the
    row-sum identity."""
    cfg = synth.CONFIGS["headline_shard8"]
    s = oracle_table(cfg)
    xd, xh, applied = _device_u8(cfg, s)
    plan = plan_for(dd, cfg)
    out = plan.forward(xd)
    torch.cuda.synchronize()
    rows = sample_rows(cfg["n_dm"], cfg["pulses"], extra=3, seed=8)
    assert np.array_equal(out[rows].cpu().numpy(), oracle.forward(xh, "u8", cfg["n_samp"], s, rows=rows))
    gpu_rowsum = out.double().sum(dim=1).cpu().numpy().astype(np.int64)
    assert np.array_equal(gpu_rowsum, row_sums_by_prefix(lambda c: xh[c], s, plan.n_out))
    assert applied[0].sum() > 0


def test_lowfreq_wide_workload_sampled(dd):
    """4096 channels at 120-190 MHz, 2^20 samples, 1024 DMs in steps of 0.5 (264 samples of extra
    delay per step): the direct-read kernel, as the benchmark runs it.  Sampled rows bit-exact,
    every row by the row-sum identity, DM 0 by the channel sum, pulses at their DM."""
    cfg = synth.CONFIGS["lowfreq_wide"]
    s = oracle_table(cfg)
    xd, xh, applied = _device_u8(cfg, s)
    plan = plan_for(dd, cfg)
    assert plan.tiles(0)["row_block"] == 0
    out = plan.forward(xd)
    torch.cuda.synchronize()
    n_out = plan.n_out
    rows = sample_rows(cfg["n_dm"], cfg["pulses"], every=128, extra=4, seed=10)
    assert np.array_equal(out[rows].cpu().numpy(), oracle.forward(xh, "u8", cfg["n_samp"], s, rows=rows))
    gpu_rowsum = out.double().sum(dim=1).cpu().numpy().astype(np.int64)
    assert np.array_equal(gpu_rowsum, row_sums_by_prefix(lambda c: xh[c], s, n_out))
    assert np.array_equal(out[0].cpu().numpy().astype(np.int64), xh[:, :n_out].sum(axis=0, dtype=np.int64))
    for i, (dp, width, t0) in enumerate(cfg["pulses"]):
        assert applied[i].sum() > 0
        assert int(np.argmax(out[:, t0].cpu().numpy())) == dp


def test_lowfreq_u4_workload_sampled(dd):
    """4096 channels of packed 4-bit input at 120-190 MHz, 2^19 samples, 2048 DMs (delays > 10^5)."""
    cfg = synth.CONFIGS["lowfreq_u4"]
    s = oracle_table(cfg)
    n_chan, n_samp = cfg["n_chan"], cfg["n_samp"]
    xd = torch.empty((n_chan, n_samp // 2), dtype=torch.uint8, device="cuda")
    synth.uniform_u4_device(xd.data_ptr(), n_chan, n_samp, n_samp // 2, cfg["seed"],
                            torch.cuda.current_stream().cuda_stream)
    xh = synth.uniform_u4_packed(n_chan, n_samp, cfg["seed"])
    torch.cuda.synchronize()
    for c in [0, 2047, 4095]:
        assert torch.equal(xd[c].cpu(), torch.from_numpy(xh[c]))
    plan = plan_for(dd, cfg)
    out = plan.forward(xd)
    torch.cuda.synchronize()
    rows = sample_rows(cfg["n_dm"], every=256, extra=6, seed=3)
    got = out[rows].cpu().numpy()
    want = oracle.forward(xh, "u4", n_samp, s, rows=rows)
    assert np.array_equal(got, want)
    unpacked = synth.unpack_u4
    gpu_rowsum = out.double().sum(dim=1).cpu().numpy().astype(np.int64)
    cpu_rowsum = row_sums_by_prefix(lambda c: unpacked(xh[c:c + 1], n_samp)[0], s, plan.n_out)
    assert np.array_equal(gpu_rowsum, cpu_rowsum)


def test_headline_u16_workload_sampled(dd):
    """The headline shape with 16-bit samples (8192 ch x 2^20 x 4000 DMs), as bench.py times it.

    Sums reach 2^29, so outputs above 2^24 are rounded once to float32; the
    oracle rounds its exact int64 sums the same way, so sampled rows (DM 0, the
    pulse rows, every 400th, random rows) compare bit for bit, and DM 0 equals
    the float32 of the plain channel sum.
    """
    cfg = synth.CONFIGS["headline_u16"]
    s = oracle_table(cfg)
    n_chan, n_samp = cfg["n_chan"], cfg["n_samp"]
    xd = torch.empty((n_chan, n_samp), dtype=torch.uint16, device="cuda")
    table = torch.from_numpy(synth.gaussian_table16()).cuda()
    synth.gaussian_u16_device(xd.data_ptr(), n_chan, n_samp, n_samp, cfg["seed"], table.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
    xh = synth.gaussian_u16(n_chan, n_samp, cfg["seed"])
    for dp, width, t0 in cfg["pulses"]:
        rows, cols, vals, _ = synth.boxcar_updates(lambda r, c: xh[r, c], s[dp], t0, width, cfg["amp"], 65535)
        xh[rows, cols] = vals
        # torch has no uint16 scatter on the GPU: write the same bytes through an int16 view
        xd.view(torch.int16)[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()] = \
            torch.from_numpy(vals.view(np.int16)).cuda()
    torch.cuda.synchronize()
    for c in [0, 4095, 8191]:
        assert np.array_equal(xd[c].cpu().numpy(), xh[c])
    plan = plan_for(dd, cfg)
    out = plan.forward(xd)
    torch.cuda.synchronize()
    rows = sample_rows(cfg["n_dm"], cfg["pulses"], every=400, extra=6, seed=6)
    got = out[rows].cpu().numpy()
    want = oracle.forward(xh, "u16", n_samp, s, rows=rows)
    assert np.array_equal(got, want)
    dm0 = xh[:, :plan.n_out].sum(axis=0, dtype=np.int64).astype(np.float32)
    assert np.array_equal(out[0].cpu().numpy(), dm0)
    for dp, width, t0 in cfg["pulses"]:
        if width <= 4:
            assert int(np.argmax(out[:, t0].cpu().numpy())) == dp


def test_lowfreq_wide_u16_workload_sampled(dd):
    """The wide-spread low-frequency plan on 16-bit samples (4096 ch x 2^20 x 1024 DMs, 264
    samples of extra delay per DM step): the direct-read kernel's 16-bit form, as the benchmark
    runs it.  Sampled rows bit-exact against the oracle, DM 0 against the plain channel sum."""
    cfg = synth.CONFIGS["lowfreq_wide_u16"]
    s = oracle_table(cfg)
    n_chan, n_samp = cfg["n_chan"], cfg["n_samp"]
    xd = torch.empty((n_chan, n_samp), dtype=torch.uint16, device="cuda")
    table = torch.from_numpy(synth.gaussian_table16()).cuda()
    synth.gaussian_u16_device(xd.data_ptr(), n_chan, n_samp, n_samp, cfg["seed"], table.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
    xh = synth.gaussian_u16(n_chan, n_samp, cfg["seed"])
    for dp, width, t0 in cfg["pulses"]:
        rows, cols, vals, _ = synth.boxcar_updates(lambda r, c: xh[r, c], s[dp], t0, width, cfg["amp"], 65535)
        xh[rows, cols] = vals
        xd.view(torch.int16)[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()] = \
            torch.from_numpy(vals.view(np.int16)).cuda()
    torch.cuda.synchronize()
    plan = plan_for(dd, cfg)
    assert plan.tiles(0)["row_block"] == 0, plan.tiles(0)
    out = plan.forward(xd)
    torch.cuda.synchronize()
    rows = sample_rows(cfg["n_dm"], cfg["pulses"], every=128, extra=4, seed=11)
    assert np.array_equal(out[rows].cpu().numpy(), oracle.forward(xh, "u16", n_samp, s, rows=rows))
    dm0 = xh[:, :plan.n_out].sum(axis=0, dtype=np.int64).astype(np.float32)
    assert np.array_equal(out[0].cpu().numpy(), dm0)
    for dp, width, t0 in cfg["pulses"]:
        assert int(np.argmax(out[:, t0].cpu().numpy())) == dp


def test_grad_workload_forward_sampled(dd):
    """1024 float channels x 2^17 samples x 1024 DMs: sampled rows within the FP32 bound."""
    cfg = synth.CONFIGS["grad_f32"]
    s = oracle_table(cfg)
    x = synth.normal_f32(cfg["n_chan"], cfg["n_samp"], cfg["seed"])
    plan = plan_for(dd, cfg)
    out = plan.forward(_to_dev(x))
    torch.cuda.synchronize()
    rows = sample_rows(cfg["n_dm"], every=64, extra=8, seed=4)
    got = out[rows].cpu().numpy().astype(np.float64)
    want, ab = oracle.forward_f32(x, cfg["n_samp"], s, rows=rows)
    err = np.abs(got - want)
    assert (err <= F32_TOL * ab).all(), float((err / ab).max())


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "f32"])
def test_explicit_unordered_frequencies(dd, dtype):
    """Channels given by an explicit frequency list in random order (delays no longer grow with
    the channel index, the staging bases jump between neighbouring channels): the forward, and
    for float input the adjoint, against the oracle's table built from the same list."""
    rng = np.random.default_rng({"u8": 51, "u4": 52, "u16": 53, "f32": 54}[dtype])
    n_chan, n_samp, n_dm = 301, 12000, 45
    f_high, t_samp = 1450.0, 64e-6
    freqs = rng.permutation(np.concatenate([[f_high], rng.uniform(1150.0, f_high, n_chan - 1)]))
    k = 1 / freqs.min() ** 2 - 1 / f_high**2
    dm_max = 0.6 * n_samp * t_samp / (4.148808e3 * k)
    start, step = 0.05 * dm_max, 0.95 * dm_max / (n_dm - 1)
    s = oracle.shift_table(n_chan, f_high, 0.0, t_samp, start, step, n_dm, freqs=freqs)
    assert (np.diff(s[-1].astype(np.int64)) < 0).any()  # delays are not monotone in the channel index
    n_out = oracle.n_out_for(s, n_samp)
    elem = {"f32": 4, "u16": 2}.get(dtype, 1)
    row = n_samp // 2 if dtype == "u4" else n_samp * elem
    pitch_bytes = (row + 15) // 16 * 16 + 32
    pitch = pitch_bytes // elem
    if dtype in ("u8", "u4"):
        x = rng.integers(0, 256, (n_chan, pitch)).astype(np.uint8)
    elif dtype == "u16":
        x = rng.integers(0, 65536, (n_chan, pitch)).astype(np.uint16)
    else:
        x = rng.standard_normal((n_chan, pitch)).astype(np.float32)
    plan = dd.Plan(n_chan=n_chan, n_samp=n_samp, dtype=dtype, f_high=f_high, chan_bw=0.0, t_samp=t_samp,
                   dm_start=start, dm_step=step, n_dm=n_dm, chan_freq=freqs, in_pitch_bytes=pitch_bytes)
    assert np.array_equal(plan.shift, s) and plan.n_out == n_out
    print("explicit frequencies %s: n_chan=%d n_samp=%d n_dm=%d n_out=%d" % (dtype, n_chan, n_samp, n_dm, n_out),
          flush=True)
    got = plan.forward(_to_dev(x))
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    if dtype != "f32":
        want = oracle.forward(np.ascontiguousarray(x), dtype, n_samp, s)
        assert np.array_equal(got, want)
        # the other kernel families on the same plan: direct reads and the ring-staged form if staged
        # (8-bit plans stage by phase loads by default), staged shapes if direct
        other = [plan.n_shapes - 2, 0] if plan.tiles(0)["row_block"] > 0 else [5, 6, 7]
        for shape in other:
            try:
                plan.set_tiles(0, shape, 2)
            except dd.DDError:
                continue
            print("  shape %d" % shape, flush=True)
            got = plan.forward(_to_dev(x))
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want), shape
            break
        else:
            raise AssertionError("no second kernel family fits this plan")
        return
    want, ab = oracle.forward_f32(np.ascontiguousarray(x), n_samp, s)
    assert (np.abs(got.astype(np.float64) - want) <= F32_TOL * ab + 1e-30).all()
    y = rng.standard_normal((n_dm, n_out)).astype(np.float32)
    g = plan.adjoint(torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    want_g = oracle.adjoint(y, n_chan, n_samp, s)
    ab_g = oracle.adjoint(np.abs(y), n_chan, n_samp, s)
    assert (np.abs(g - want_g) <= F32_TOL * ab_g).all()
    assert (g[ab_g == 0] == 0).all()
