"""Host-side checks of bench.py (no GPU): the one-GPU contract and the committed
counter summaries it reads its memory-traffic figures from."""
import glob
import importlib.util
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_blocks_parse_and_name_sources():
    blocks = 0
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_counters.md")):
        for block in re.findall(r"```traffic\n(.*?)```", open(path).read(), re.S):
            kv = dict(line.split(": ", 1) for line in block.strip().splitlines() if ": " in line)
            assert {"workload", "kernel", "source", "source_sha256"} <= set(kv)
            assert os.path.isfile(os.path.join(ROOT, kv["source"])), kv["source"]
            figures = [k for k in kv if k.startswith("traffic_bytes_per_launch")]  # per factor for binning
            assert figures and all(int(kv[k]) > 0 for k in figures)
            blocks += 1
    assert blocks >= 4


def test_headline_traffic_matches_the_current_kernel():
    """The headline's default tiles have counters taken on the kernel source as committed;
    after a change to that source the counters must be taken again (bench.py then reports
    the traffic as unknown)."""
    import paper_2311_05341_amd as dd
    import synth
    c = synth.CONFIGS["headline"]
    plan = dd.Plan(c["n_chan"], c["n_samp"], c["dtype"], c["f_high"], c["chan_bw"], c["t_samp"], c["dm_start"],
                   c["dm_step"], c["n_dm"], bind=False)
    traffic, src = _bench().measured_traffic("headline", plan.tiles(0))
    assert traffic is not None and src.startswith("profiles" + os.sep)
    assert traffic > 24.85e9  # at least the algorithmic bytes (input once + output once)


def test_accumulate_forms_follow_the_kernel():
    """The instruction form (and LDS bytes per add) the bench line prices a run against is the
    one its tile choice runs: direct-read shapes read no LDS, packed 4-bit phase loads add
    nibbles in place, the raw ring adds unpacked bytes."""
    b = _bench()
    direct = {"row_block": 0, "segs": 0}
    phase = {"row_block": 8, "segs": 1}
    ring = {"row_block": 4, "segs": 0}
    assert b.accumulate_form("u4", direct)[1:] == (2.0, 0)
    assert b.accumulate_form("u8", direct)[1:] == (8.0 / 6.0, 0)
    assert b.accumulate_form("u16", direct)[1:] == (4.0 / 6.0, 0)
    assert b.accumulate_form("u4", phase) == (b.U4_NIBBLE_FORM, 16.0 / 6.0, 0.5)
    assert b.accumulate_form("u4", ring)[1:] == (2, 1)
    assert b.accumulate_form("u8", phase)[1:] == (2, 1)
    assert b.accumulate_form("f32", {"row_block": 8, "segs": 0})[1:] == (1, 4)
    for dtype, ops in b.DIRECT_OPS.items():  # the op counts and the stated rate agree
        assert ops[4] / sum(ops[:4]) == b.DIRECT_FORMS[dtype][1]


def test_wide_beam_batches_read_directly():
    """The wide-spread beam batches bench.py times (batch_wide8*) put every plan on a direct-read
    shape by default, for each input type."""
    import paper_2311_05341_amd as dd
    import synth
    b = _bench()
    assert {v[0] for k, v in b.BATCH_SETS.items() if v[1] == "wide_beams"} == {"u8", "u4", "u16"}
    for dtype in ("u8", "u4", "u16"):
        for c in synth.wide_beams(dtype):
            p = dd.Plan(c["n_chan"], c["n_samp"], dtype, c["f_high"], c["chan_bw"], c["t_samp"], c["dm_start"],
                        c["dm_step"], c["n_dm"], bind=False)
            assert p.tiles(0)["row_block"] == 0, (dtype, c)
