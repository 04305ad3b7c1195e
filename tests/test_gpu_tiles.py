"""GPU checks that the tile choice changes speed only.

For every compiled shape that holds a plan's delay spread, in both workgroup
orders, the forward (and for float plans the adjoint) must give bitwise the
same result as the oracle-checked default.  The autotuner must leave a
feasible choice with the same results, and its cache line must reproduce that
choice for an identical plan.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import host_input, oracle_table, plan_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import paper_2311_05341_amd as dd
    assert torch.cuda.is_available()
    return dd


def _case(dtype):
    # several time tiles with a ragged tail, DM blocks with a tail, channels
    # not a multiple of any staging block
    return dict(dtype=dtype, n_chan=203, n_samp=30016, f_high=1400.0, chan_bw=0.9, t_samp=64e-6,
                dm_start=3.0, dm_step=0.77, n_dm=77, seed=41)


def _choices(dd, plan, direction):
    out = []
    for s in range(plan.n_shapes):
        for o in (0, 1, 2, 3):
            try:
                plan.set_tiles(direction, s, o)
            except dd.DDError as e:
                assert e.name == "DD_ERR_RANGE"
                continue
            out.append((s, o))
    return out


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16"])
def test_integer_tiles_bit_exact(dd, dtype):
    cfg = _case(dtype)
    s = oracle_table(cfg)
    x, _ = host_input(cfg, s)
    want = oracle.forward(x, dtype, cfg["n_samp"], s)
    plan = plan_for(dd, cfg)
    xd = torch.from_numpy(x).cuda()
    choices = _choices(dd, plan, 0)
    assert len(choices) >= 4
    for s_, o in choices:
        plan.set_tiles(0, s_, o)
        print("shape", s_, "order", o, plan.tiles(0), flush=True)
        got = plan.forward(xd)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want), (s_, o)


def test_float_tiles_bitwise_invariant(dd):
    cfg = _case("f32")
    s = oracle_table(cfg)
    x, _ = host_input(cfg, s)
    plan = plan_for(dd, cfg)
    xd = torch.from_numpy(x).cuda()
    n_out = plan.n_out
    y = synth.normal_f32(cfg["n_dm"], n_out, 77)
    yd = torch.from_numpy(np.ascontiguousarray(np.pad(y, ((0, 0), (0, plan.out_pitch - n_out))))).cuda()
    want_f, abs_f = oracle.forward_f32(x, cfg["n_samp"], s)
    want_a = oracle.adjoint(y, cfg["n_chan"], cfg["n_samp"], s)
    ref = {}
    for direction in (0, 1):
        for s_, o in _choices(dd, plan, direction):
            plan.set_tiles(direction, s_, o)
            print("direction", direction, "shape", s_, "order", o, flush=True)
            got = (plan.forward(xd) if direction == 0 else plan.adjoint(yd)).cpu().numpy()
            if direction not in ref:
                ref[direction] = got
                if direction == 0:
                    assert np.all(np.abs(got - want_f) <= 1e-5 * abs_f)
                else:
                    abs_a = oracle.adjoint(np.abs(y), cfg["n_chan"], cfg["n_samp"], s)
                    assert np.all(np.abs(got - want_a) <= 1e-5 * abs_a)
            assert np.array_equal(got, ref[direction]), (direction, s_, o)


def test_autotune_forward_and_cache(dd, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DD_TUNE_CACHE", str(cache))
    cfg = synth.CONFIGS["small"]
    s = oracle_table(cfg)
    x, _ = host_input(cfg, s)
    want = oracle.forward(x, "u8", cfg["n_samp"], s)
    plan = plan_for(dd, cfg)
    xd = torch.from_numpy(x).cuda()
    out = torch.empty((plan.n_dm, plan.out_pitch), dtype=torch.float32, device="cuda")
    rep = plan.autotune(xd, out)
    print(rep, flush=True)
    assert rep["n_tried"] >= 2 and rep["best_ms"] > 0 and rep["best_ms"] <= rep["default_ms"]
    assert rep["timed_out_samples"] == plan.n_out
    t = plan.tiles(0)
    assert t == rep["best"]
    got = plan.forward(xd, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
    line = cache.read_text().strip().splitlines()[-1].split()
    assert line[0] == "dd-tune-v2" and int(line[2]) == t["shape"] and int(line[3]) == t["order"]
    again = plan_for(dd, cfg)
    assert again.tiles(0) == t


def test_autotune_adjoint(dd, monkeypatch):
    monkeypatch.delenv("DD_TUNE_CACHE", raising=False)
    cfg = _case("f32")
    s = oracle_table(cfg)
    plan = plan_for(dd, cfg)
    y = synth.normal_f32(cfg["n_dm"], plan.n_out, 78)
    yd = torch.from_numpy(np.ascontiguousarray(np.pad(y, ((0, 0), (0, plan.out_pitch - plan.n_out))))).cuda()
    before = plan.adjoint(yd).cpu().numpy()
    g = torch.empty((plan.n_chan, plan.in_row_elems), dtype=torch.float32, device="cuda")
    rep = plan.autotune(yd, g, direction=1)
    print(rep, flush=True)
    assert rep["n_tried"] >= 2 and plan.tiles(1) == rep["best"]
    after = plan.adjoint(yd).cpu().numpy()
    assert np.array_equal(after, before)
    want = oracle.adjoint(y, cfg["n_chan"], cfg["n_samp"], s)
    abs_a = oracle.adjoint(np.abs(y), cfg["n_chan"], cfg["n_samp"], s)
    assert np.all(np.abs(after - want) <= 1e-5 * abs_a)


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "f32"])
def test_time_chunks_equal_whole(dd, dtype):
    """Chunks over column views of one input give the whole-input columns bit for bit."""
    cfg = _case(dtype)
    s = oracle_table(cfg)
    x, _ = host_input(cfg, s)
    desc = {k: cfg[k] for k in ["n_chan", "n_samp", "dtype", "f_high", "chan_bw", "t_samp", "dm_start", "dm_step",
                                "n_dm"]}
    whole = plan_for(dd, cfg)
    xd = torch.from_numpy(x).cuda()
    ref = whole.forward(xd).clone()
    tc = dd.TimeChunks(desc, 3)
    out = torch.full((whole.n_dm, whole.out_pitch), -1.0, device="cuda")
    for k, p in enumerate(tc.plans):
        p.forward(tc.input_view(xd, k), out=tc.output_view(out, k))
    torch.cuda.synchronize()
    assert torch.equal(out[:, : whole.n_out], ref)


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16"])
def test_direct_kernel_large_spread(dd, dtype):
    """The direct-read kernel on a plan it is chosen for: 264 samples of delay per DM step,
    more than 256 channels (exact flushes), a ragged last tile, odd delays for 4-bit input,
    padded rows; every output bit-exact, both direct shapes, all orders."""
    cfg = dict(dtype=dtype, n_chan=300, n_samp=50012, f_high=190.0, chan_bw=70.0 / 300, t_samp=327.68e-6,
               dm_start=1.0, dm_step=0.5, n_dm=37, seed=43)
    s = oracle_table(cfg)
    pitch = {"u8": 50048, "u4": 25024, "u16": 50048}[dtype]
    x, _ = host_input(cfg, s, pitch=pitch)
    want = oracle.forward(x, dtype, cfg["n_samp"], s)
    plan = plan_for(dd, cfg, in_pitch_bytes=pitch * (2 if dtype == "u16" else 1))
    assert plan.tiles(0)["row_block"] == 0, plan.tiles(0)
    xd = torch.from_numpy(x.view(np.int16)).cuda().view(torch.uint16) if dtype == "u16" else torch.from_numpy(x).cuda()
    for shape in range(plan.n_shapes):
        try:
            plan.set_tiles(0, shape, 0)
        except dd.DDError as e:  # an LDS shape that cannot stage this spread
            assert e.name == "DD_ERR_RANGE"
            continue
        if plan.tiles(0)["row_block"] != 0:
            continue
        for o in (0, 1, 2, 3):
            plan.set_tiles(0, shape, o)
            print("direct shape", shape, "order", o, flush=True)
            got = plan.forward(xd)
            torch.cuda.synchronize()
            assert np.array_equal(got.cpu().numpy(), want), (shape, o)


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "f32"])
def test_shortest_input_every_shape(dd, dtype):
    """The shortest input a plan accepts: n_samp = largest delay + 1 (+1 more for 4-bit input,
    whose sample count is even), so one or two output samples per DM row, on every compiled
    shape and order; float plans also through the adjoint."""
    base = dict(dtype=dtype, n_chan=203, n_samp=1 << 20, f_high=1400.0, chan_bw=0.9, t_samp=64e-6,
                dm_start=3.0, dm_step=0.77, n_dm=77)
    ms = int(oracle_table(base).max())
    n_samp = ms + 1 + ((ms + 1) & 1 if dtype == "u4" else 0)
    cfg = dict(base, n_samp=n_samp)
    s = oracle_table(cfg)
    n_out = oracle.n_out_for(s, n_samp)
    assert n_out in (1, 2)
    rng = np.random.default_rng(77)
    elem = {"f32": 4, "u16": 2}.get(dtype, 1)
    pitch_bytes = ((n_samp // 2 if dtype == "u4" else n_samp * elem) + 15) // 16 * 16
    cols = pitch_bytes // elem
    if dtype == "f32":
        x = rng.standard_normal((cfg["n_chan"], cols)).astype(np.float32)
        want, ab = oracle.forward_f32(x, n_samp, s)
    else:
        top = 65536 if dtype == "u16" else 256
        x = rng.integers(0, top, (cfg["n_chan"], cols)).astype(np.uint16 if dtype == "u16" else np.uint8)
        want = oracle.forward(x, dtype, n_samp, s)
    plan = plan_for(dd, cfg, in_pitch_bytes=pitch_bytes)
    assert plan.n_out == n_out
    xd = torch.from_numpy(x).cuda()
    choices = _choices(dd, plan, 0)
    assert choices
    for s_, o in choices:
        plan.set_tiles(0, s_, o)
        print("shortest %s: n_samp=%d n_out=%d shape %d order %d" % (dtype, n_samp, n_out, s_, o), flush=True)
        got = plan.forward(xd)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        if dtype == "f32":
            assert (np.abs(got.astype(np.float64) - want) <= 1e-5 * ab + 1e-30).all(), (s_, o)
        else:
            assert np.array_equal(got, want), (s_, o)
    if dtype != "f32":
        return
    y = rng.standard_normal((cfg["n_dm"], n_out)).astype(np.float32)
    gw = oracle.adjoint(y, cfg["n_chan"], n_samp, s)
    ga = oracle.adjoint(np.abs(y), cfg["n_chan"], n_samp, s)
    for s_, o in _choices(dd, plan, 1):
        plan.set_tiles(1, s_, o)
        print("shortest f32 adjoint: shape %d order %d" % (s_, o), flush=True)
        g = plan.adjoint(torch.from_numpy(y).cuda())
        torch.cuda.synchronize()
        g = g.cpu().numpy().astype(np.float64)
        assert (np.abs(g - gw) <= 1e-5 * ga).all(), (s_, o)
        assert (g[ga == 0] == 0).all(), (s_, o)
