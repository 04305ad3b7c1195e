"""GPU batched (persistent, graph-replayed) forward: per-beam bit-exact results."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import host_input, oracle_table, plan_for, sample_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import paper_2311_05341_amd as dd
    return dd


def _beams(n, seed, max_samp):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        n_chan = int(rng.choice([16, 96, 256, 300, 1024]))
        n_samp = int(rng.integers(20000, max_samp))
        n_dm = int(rng.integers(5, 300))
        step = float(rng.choice([0.25, 0.5, 0.75, 1.0]))
        out.append(dict(dtype="u8", n_chan=n_chan, n_samp=n_samp, f_high=1500.0, chan_bw=300.0 / n_chan,
                        t_samp=64e-6, dm_start=0.0, dm_step=step, n_dm=n_dm, seed=900 + b,
                        pitch=(n_samp + 63) // 64 * 64))
    return out


def test_batched_matches_oracle_and_plain(dd):
    beams = _beams(7, 77, 120000)
    plans, xs, hosts, tables = [], [], [], []
    for cfg in beams:
        s = oracle_table(cfg)
        x = synth.gaussian_u8(cfg["n_chan"], cfg["n_samp"], cfg["seed"], pitch=cfg["pitch"])
        plans.append(plan_for(dd, cfg, in_pitch_bytes=cfg["pitch"]))
        xs.append(torch.from_numpy(x).cuda())
        hosts.append(x)
        tables.append(s)
    batch = dd.Batch(plans, xs)
    outs = [o.clone() for o in batch.run()]
    outs2 = batch.run()  # a second replay of the same graph
    torch.cuda.synchronize()
    for b, (cfg, plan) in enumerate(zip(beams, plans)):
        assert torch.equal(outs[b], outs2[b])
        plain = plan.forward(xs[b])
        torch.cuda.synchronize()
        assert torch.equal(outs[b], plain)
        rows = sample_rows(cfg["n_dm"], every=37)
        want = oracle.forward(hosts[b], "u8", cfg["n_samp"], tables[b], rows=rows)
        assert np.array_equal(outs[b][rows].cpu().numpy(), want)


def test_batched_mixed_shapes_and_tuned_plan(dd):
    """Beams whose plans run different staged shapes (a narrow and a wide delay spread, and a
    plan set to a third shape) run in one batch as several groups, each beam on its plan's own
    shape: bit-exact against plain calls and the oracle, over two replays."""
    base = dict(dtype="u8", f_high=1500.0, t_samp=64e-6, dm_start=0.0)
    beams = [dict(base, n_chan=256, chan_bw=300.0 / 256, n_samp=70016, dm_step=0.25, n_dm=150, seed=951),
             dict(base, n_chan=300, chan_bw=1.0, n_samp=60032, dm_step=1.0, n_dm=97, seed=952),
             dict(base, n_chan=96, chan_bw=3.0, n_samp=50048, dm_step=0.5, n_dm=64, seed=953)]
    plans, xs, hosts, tables = [], [], [], []
    for cfg in beams:
        tables.append(oracle_table(cfg))
        x = synth.gaussian_u8(cfg["n_chan"], cfg["n_samp"], cfg["seed"])
        plans.append(plan_for(dd, cfg))
        xs.append(torch.from_numpy(x).cuda())
        hosts.append(x)
    plans[2].set_tiles(0, 0, 2)  # a ring-staged shape for the third beam
    shapes = [p.tiles(0)["shape"] for p in plans]
    batch = dd.Batch(plans, xs)
    assert [batch.beam_tiles(b)["shape"] for b in range(3)] == shapes
    assert len(set(shapes)) >= 2 and batch.tiles()["shape"] == -1
    outs = [o.clone() for o in batch.run()]
    outs2 = batch.run()
    torch.cuda.synchronize()
    for b, cfg in enumerate(beams):
        assert torch.equal(outs[b], outs2[b])
        assert torch.equal(outs[b], plans[b].forward(xs[b]))
        rows = sample_rows(cfg["n_dm"], every=17)
        want = oracle.forward(hosts[b], "u8", cfg["n_samp"], tables[b], rows=rows)
        assert np.array_equal(outs[b][rows].cpu().numpy(), want), b


def test_batched_single_beam_and_u4(dd):
    cfg = dict(dtype="u4", n_chan=200, n_samp=50016, f_high=400.0, chan_bw=0.5, t_samp=256e-6,
               dm_start=0.0, dm_step=0.3, n_dm=70)
    s = oracle_table(cfg)
    x = synth.uniform_u4_packed(cfg["n_chan"], cfg["n_samp"], 11)
    plan = plan_for(dd, cfg)
    batch = dd.Batch([plan], [torch.from_numpy(x).cuda()])
    out = batch.run()[0]
    torch.cuda.synchronize()
    want = oracle.forward(x, "u4", cfg["n_samp"], s)
    assert np.array_equal(out.cpu().numpy(), want)


def test_batched_u16_beams(dd):
    """Three 16-bit beams of different shapes in one batch: bit-exact against the oracle."""
    beams = [dict(dtype="u16", n_chan=96, n_samp=40000, f_high=1400.0, chan_bw=1.5, t_samp=64e-6,
                  dm_start=0.0, dm_step=0.5, n_dm=40, seed=61),
             dict(dtype="u16", n_chan=300, n_samp=30008, f_high=1500.0, chan_bw=0.8, t_samp=128e-6,
                  dm_start=5.0, dm_step=1.0, n_dm=33, seed=62),
             dict(dtype="u16", n_chan=17, n_samp=20000, f_high=800.0, chan_bw=2.0, t_samp=64e-6,
                  dm_start=0.0, dm_step=0.25, n_dm=65, seed=63)]
    plans, xs, hosts, tables = [], [], [], []
    for cfg in beams:
        s = oracle_table(cfg)
        x = synth.gaussian_u16(cfg["n_chan"], cfg["n_samp"], cfg["seed"])
        plans.append(plan_for(dd, cfg))
        xs.append(torch.from_numpy(x).cuda())
        hosts.append(x)
        tables.append(s)
    outs = dd.Batch(plans, xs).run()
    torch.cuda.synchronize()
    for b, cfg in enumerate(beams):
        want = oracle.forward(hosts[b], "u16", cfg["n_samp"], tables[b])
        assert np.array_equal(outs[b].cpu().numpy(), want), b


def test_batched_every_shape_and_autotune(dd):
    """Every staged shape that holds the beams and both direct-read shapes give the same bits (equal
    to plain calls), and the batch autotuner leaves the batch bound with one of them, results
    unchanged."""
    beams = _beams(5, 78, 60000)
    plans, xs = [], []
    for cfg in beams:
        x = synth.gaussian_u8(cfg["n_chan"], cfg["n_samp"], cfg["seed"], pitch=cfg["pitch"])
        plans.append(plan_for(dd, cfg, in_pitch_bytes=cfg["pitch"]))
        xs.append(torch.from_numpy(x).cuda())
    plain = [p.forward(x).clone() for p, x in zip(plans, xs)]
    batch = dd.Batch(plans, xs)
    n_ok = 0
    for shape in range(plans[0].n_shapes):  # every staged shape, then the two direct-read shapes
        try:
            batch.set_tiles(shape)
        except dd.DDError as e:
            assert e.name == "DD_ERR_RANGE"
            continue
        assert batch.tiles()["shape"] == shape
        outs = batch.run()
        torch.cuda.synchronize()
        print("batch shape", shape, flush=True)
        for b in range(len(beams)):
            assert torch.equal(outs[b], plain[b]), (shape, b)
        n_ok += 1
    assert n_ok >= 7
    rep = batch.autotune()
    assert rep["n_tried"] >= 2 and rep["best"]["shape"] == batch.tiles()["shape"]
    outs = batch.run()
    torch.cuda.synchronize()
    for b in range(len(beams)):
        assert torch.equal(outs[b], plain[b])


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16"])
def test_batched_beam_with_one_output_sample(dd, dtype):
    """A beam whose input is the shortest its plan accepts (one output sample per DM row)
    next to an ordinary beam, in one persistent launch: both bit-exact."""
    base = dict(dtype=dtype, n_chan=150, n_samp=1 << 20, f_high=1400.0, chan_bw=0.9, t_samp=64e-6,
                dm_start=3.0, dm_step=0.77, n_dm=50)
    ms = int(oracle_table(base).max())
    short = dict(base, n_samp=ms + 1 + ((ms + 1) & 1 if dtype == "u4" else 0))
    normal = dict(base, n_chan=97, n_samp=40000, n_dm=33)
    rng = np.random.default_rng(12)
    plans, xs, wants = [], [], []
    for cfg in (short, normal):
        s = oracle_table(cfg)
        elem = 2 if dtype == "u16" else 1
        pitch_bytes = ((cfg["n_samp"] // 2 if dtype == "u4" else cfg["n_samp"] * elem) + 15) // 16 * 16
        top, npt = (65536, np.uint16) if dtype == "u16" else (256, np.uint8)
        x = rng.integers(0, top, (cfg["n_chan"], pitch_bytes // elem)).astype(npt)
        wants.append(oracle.forward(x, dtype, cfg["n_samp"], s))
        plans.append(plan_for(dd, cfg, in_pitch_bytes=pitch_bytes))
        xs.append(torch.from_numpy(x).cuda())
    assert plans[0].n_out in (1, 2)
    print("batch with a one-output beam: %s" % dtype, flush=True)
    batch = dd.Batch(plans, xs)
    outs = batch.run()
    torch.cuda.synchronize()
    for o, w in zip(outs, wants):
        assert np.array_equal(o.cpu().numpy(), w)
    for shape in (plans[0].n_shapes - 2, plans[0].n_shapes - 1):  # both beams on a direct-read shape
        batch.set_tiles(shape)
        outs = batch.run()
        torch.cuda.synchronize()
        for o, w in zip(outs, wants):
            assert np.array_equal(o.cpu().numpy(), w), shape


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16"])
def test_batched_wide_beams_read_directly(dtype):
    """Beams whose delay spread is too wide to stage (120-190 MHz, ~4000 samples of spread per
    16 DM rows) run their plans' direct-read shape inside a batch, next to a narrow beam (staged
    for 8- and 16-bit input): two direct beams (100 and a ragged 37 DM rows) and the narrow one,
    over two replays, bit-exact against plain calls and the oracle."""
    import paper_2311_05341_amd as dd
    wide = dict(dtype=dtype, n_chan=256, n_samp=1 << 17, f_high=190.0, chan_bw=70.0 / 256, t_samp=327.68e-6,
                dm_start=0.0, dm_step=0.5, n_dm=100, seed=71)
    beams = [wide, dict(wide, n_chan=200, chan_bw=70.0 / 200, n_samp=100000, n_dm=37, dm_start=3.0, seed=72),
             dict(dtype=dtype, n_chan=96, n_samp=50016, f_high=1500.0, chan_bw=3.0, t_samp=64e-6,
                  dm_start=0.0, dm_step=0.5, n_dm=64, seed=73)]
    plans, xs, hosts, tables = [], [], [], []
    for cfg in beams:
        tables.append(oracle_table(cfg))
        x, _ = host_input(cfg)
        plans.append(plan_for(dd, cfg))
        xs.append(torch.from_numpy(x).cuda())
        hosts.append(x)
    # the narrow beam is staged, except 4-bit, whose plans all read directly
    assert [p.tiles(0)["row_block"] == 0 for p in plans] == [True, True, dtype == "u4"]
    batch = dd.Batch(plans, xs)
    for b, p in enumerate(plans):
        assert batch.beam_tiles(b)["shape"] == p.tiles(0)["shape"]
    print("batch with direct-read beams: %s" % dtype, flush=True)
    outs = [o.clone() for o in batch.run()]
    outs2 = batch.run()
    torch.cuda.synchronize()
    for b, cfg in enumerate(beams):
        assert torch.equal(outs[b], outs2[b]), b
        assert torch.equal(outs[b], plans[b].forward(xs[b])), b
        rows = sample_rows(cfg["n_dm"], every=13)
        want = oracle.forward(hosts[b], dtype, cfg["n_samp"], tables[b], rows=rows)
        assert np.array_equal(outs[b][rows].cpu().numpy(), want), b


def test_batched_two_direct_shapes_in_one_graph():
    """Two 4-bit wide-spread beams, one set to each direct-read shape (4 x 4 and 2 x 8), run as
    two direct-read groups of one graph: bit-exact against plain calls on the same shapes."""
    import paper_2311_05341_amd as dd
    base = dict(dtype="u4", n_chan=256, n_samp=1 << 17, f_high=190.0, chan_bw=70.0 / 256, t_samp=327.68e-6,
                dm_start=0.0, dm_step=0.5, n_dm=90, seed=81)
    beams = [base, dict(base, n_dm=51, dm_start=7.0, seed=82)]
    plans, xs = [], []
    for cfg in beams:
        x, _ = host_input(cfg)
        plans.append(plan_for(dd, cfg))
        xs.append(torch.from_numpy(x).cuda())
    n = plans[0].n_shapes
    plans[0].set_tiles(0, n - 2, 2)  # 4 rows x 4 waves
    plans[1].set_tiles(0, n - 1, 1)  # 2 rows x 8 waves
    plain = [p.forward(x).clone() for p, x in zip(plans, xs)]
    batch = dd.Batch(plans, xs)
    assert [batch.beam_tiles(b)["shape"] for b in range(2)] == [n - 2, n - 1]
    assert batch.tiles()["shape"] == -1
    print("batch with both direct-read shapes", flush=True)
    outs = batch.run()
    torch.cuda.synchronize()
    for b in range(2):
        assert torch.equal(outs[b], plain[b]), b
