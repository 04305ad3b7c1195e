"""Largest channel counts each integer input form allows, with saturated samples.

8-bit: 65793 channels of 255 sum to 2^24 - 1, the largest exact float32
integer; 4-bit: 1118481 channels of 15 likewise; 16-bit: 65537 channels of
65535 sum to 4294901760 < 2^32 (exact in the 32-bit accumulators, rounded
once to float32).  The closed form n_chan * max pins every output; the oracle
checks a row of random data at the same channel counts.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

CASES = [("u8", 65793, 255), ("u4", 1118481, 15), ("u16", 65537, 65535)]


@pytest.fixture(scope="module")
def dd():
    import paper_2311_05341_amd as dd
    assert torch.cuda.is_available()
    return dd


def _dev(x):
    if x.dtype == np.uint16:
        return torch.from_numpy(x.view(np.int16)).cuda().view(torch.uint16)
    return torch.from_numpy(x).cuda()


@pytest.mark.parametrize("dtype,n_chan,top", CASES)
def test_max_channels_saturated(dd, dtype, n_chan, top):
    n_samp, n_dm = 2048, 3
    f_high, bw = 1500.0, 300.0 / n_chan
    cols = n_samp // 2 if dtype == "u4" else n_samp
    if dtype == "u16":
        x = np.full((n_chan, cols), top, dtype=np.uint16)
    else:
        x = np.full((n_chan, cols), 0xFF if dtype == "u4" else top, dtype=np.uint8)
    plan = dd.Plan(n_chan, n_samp, dtype, f_high, bw, 64e-6, 0.0, 0.5, n_dm)
    print("max channels %s %d" % (dtype, n_chan), flush=True)
    out = plan.forward(_dev(x))
    torch.cuda.synchronize()
    want = np.float32(float(n_chan * top))  # exact sum, rounded once to float32
    got = out.cpu().numpy()
    assert np.all(got == want), (dtype, float(got.min()), float(got.max()), float(want))
    if dtype != "u16":
        assert float(want) == n_chan * top < 2 ** 24


@pytest.mark.parametrize("dtype,n_chan,top", CASES[:1] + CASES[2:])
def test_max_channels_random_rows(dd, dtype, n_chan, top):
    """Random samples at the largest channel count: one DM row against the oracle."""
    n_samp, n_dm = 4096, 2
    rng = np.random.default_rng(7)
    x = rng.integers(0, top + 1, (n_chan, n_samp)).astype(np.uint16 if dtype == "u16" else np.uint8)
    bw = 300.0 / n_chan
    s = oracle.shift_table(n_chan, 1500.0, bw, 64e-6, 0.0, 0.5, n_dm)
    plan = dd.Plan(n_chan, n_samp, dtype, 1500.0, bw, 64e-6, 0.0, 0.5, n_dm)
    assert np.array_equal(plan.shift, s)
    out = plan.forward(_dev(x))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.forward(x, dtype, n_samp, s))
