"""The paper's tiled CPU algorithm (Algorithm 2) against the oracle: every output bit-exact.

It is a comparison implementation (libdd_cpu.so), not part of the GPU path;
these run on the CPU.
"""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def ct():
    from paper_2311_05341_amd import cpu_tiled
    return cpu_tiled


def _case(n_chan, n_samp, n_dm, step, seed):
    cfg = synth.CONFIGS["small"]
    bw = 200.0 / n_chan
    s = oracle.shift_table(n_chan, cfg["f_high"], bw, cfg["t_samp"], 0.5, step, n_dm)
    x = synth.gaussian_u8(n_chan, n_samp, seed, pitch=(n_samp + 63) // 64 * 64)
    x[:, ::97] = 255  # extremes: sums of up to 256 channels of 255 must stay exact in the 16-bit partials
    return x, s, oracle.n_out_for(s, n_samp)


@pytest.mark.parametrize("tiles", [(4096, 8, 256), (1000, 3, 7), (64, 1, 1), (333, 16, 256), (8192, 5, 100)])
def test_tiled_equals_oracle(ct, tiles):
    x, s, n_out = _case(300, 20000, 45, 1.7, seed=3)
    want = oracle.forward(x, "u8", x.shape[1], s)[:, :n_out]
    got = ct.forward_u8(x, s, n_out, tiles=tiles)
    assert np.array_equal(got, want)


def test_tiled_small_workload_and_saturated_input(ct):
    cfg = synth.CONFIGS["small"]
    s = oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"], cfg["dm_start"],
                           cfg["dm_step"], cfg["n_dm"])
    x = synth.gaussian_u8(cfg["n_chan"], cfg["n_samp"], cfg["seed"])
    n_out = oracle.n_out_for(s, cfg["n_samp"])
    assert np.array_equal(ct.forward_u8(x, s, n_out), oracle.forward(x, "u8", cfg["n_samp"], s))
    full = np.full((600, 3000), 255, dtype=np.uint8)  # 600 channels of 255: 3 channel blocks
    s0 = np.zeros((4, 600), dtype=np.int32)
    assert np.all(ct.forward_u8(full, s0, 3000, tiles=(512, 2, 256)) == 600 * 255)


def test_tiled_rejects_bad_tiles(ct):
    x, s, n_out = _case(16, 4000, 4, 1.0, seed=4)
    for tiles in [(0, 8, 256), (64, 0, 256), (64, 8, 0), (64, 8, 257)]:
        with pytest.raises(ValueError):
            ct.forward_u8(x, s, n_out, tiles=tiles)
