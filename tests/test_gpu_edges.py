"""Largest sizes a plan accepts: the channel counts of each integer input form, with
saturated samples, and the longest rows.

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


LONGEST = (1 << 29) - 32  # plans take n_samp < 2^29; this keeps every row a multiple of 16 bytes


def _host(t):
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "f32"])
def test_longest_rows(dd, dtype):
    """Rows of 2^29 - 32 samples (1 GiB of 16-bit, 2 GiB of float input per channel): the
    first and the last 2^16 outputs of every DM row against the oracle, which sees only the
    head of the input and, by time-shift equivariance, its tail; integer plans also run their
    other kernel family (direct reads or LDS staging), float plans the adjoint."""
    n_chan, n_dm, n_samp, h = 3, 2, LONGEST, 1 << 16
    f_high, bw, t_samp = 1500.0, 100.0, 64e-6
    s = oracle.shift_table(n_chan, f_high, bw, t_samp, 0.0, 500.0, n_dm)
    ms = int(s.max())
    n_out = n_samp - ms
    t0 = (n_out - h) & ~1  # even, so that 4-bit tails start on a byte
    gen = torch.Generator(device="cuda").manual_seed(61)
    cols = n_samp // 2 if dtype == "u4" else n_samp
    print("longest rows %s: n_samp=%d n_out=%d" % (dtype, n_samp, n_out), flush=True)
    if dtype == "f32":
        x = torch.randn((n_chan, cols), generator=gen, device="cuda")
    elif dtype == "u16":
        x = torch.randint(-32768, 32768, (n_chan, cols), generator=gen, device="cuda", dtype=torch.int16)
        x = x.view(torch.uint16)
    else:
        x = torch.randint(0, 256, (n_chan, cols), generator=gen, device="cuda", dtype=torch.uint8)
    plan = dd.Plan(n_chan, n_samp, dtype, f_high, bw, t_samp, 0.0, 500.0, n_dm)
    assert np.array_equal(plan.shift, s) and plan.n_out == n_out

    def cut(lo, hi):  # input samples [lo, hi) on the host
        return np.ascontiguousarray(_host(x[:, lo // 2:hi // 2] if dtype == "u4" else x[:, lo:hi]))

    head_in, tail_in = cut(0, h + ms + 1 & ~1), cut(t0, n_samp)

    def check(out):
        head, tail = out[:, :h].cpu().numpy(), out[:, t0:].cpu().numpy()
        if dtype == "f32":
            for part, xin, lo in ((head, head_in, 0), (tail, tail_in, t0)):
                ns = xin.shape[1]
                want, ab = oracle.forward_f32(xin, ns, s)
                want, ab = want[:, : part.shape[1]], ab[:, : part.shape[1]]
                assert (np.abs(part.astype(np.float64) - want) <= 1e-5 * ab + 1e-30).all(), lo
            return
        ns_head = head_in.shape[1] * (2 if dtype == "u4" else 1)
        assert np.array_equal(head, oracle.forward(head_in, dtype, ns_head, s)[:, :h])
        assert np.array_equal(tail, oracle.forward(tail_in, dtype, n_samp - t0, s))

    check(plan.forward(x))
    torch.cuda.synchronize()
    if dtype != "f32":
        # the other kernel families: direct reads and the ring-staged form if staged, staged shapes if direct
        for shape in ([plan.n_shapes - 2, 0] if plan.tiles(0)["row_block"] > 0 else [5, 6, 7]):
            try:
                plan.set_tiles(0, shape, 2)
            except dd.DDError:
                continue
            print("  shape %d" % shape, flush=True)
            check(plan.forward(x))
            break
        else:
            raise AssertionError("no second kernel family fits this plan")
        return
    del x
    y = torch.randn((n_dm, n_out), generator=gen, device="cuda")
    g = plan.adjoint(y)
    torch.cuda.synchronize()
    yh = np.ascontiguousarray(y[:, :h].cpu().numpy())
    want = oracle.adjoint(yh, n_chan, h + ms, s)[:, :h]
    ab = oracle.adjoint(np.abs(yh), n_chan, h + ms, s)[:, :h]
    got = g[:, :h].cpu().numpy().astype(np.float64)
    assert (np.abs(got - want) <= 1e-5 * ab).all()
    yt = np.ascontiguousarray(y[:, t0:].cpu().numpy())  # outputs t0.. feed samples t0 + shift..: the gradient's tail
    want = oracle.adjoint(yt, n_chan, n_samp - t0, s)[:, ms:]
    ab = oracle.adjoint(np.abs(yt), n_chan, n_samp - t0, s)[:, ms:]
    got = g[:, t0 + ms:].cpu().numpy().astype(np.float64)
    assert (np.abs(got - want) <= 1e-5 * ab).all()
