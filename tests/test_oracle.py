"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formula in the same arithmetic: each
compares it with exact rational arithmetic, a closed form, a different
approximation from the paper (Eq. 4), a library routine, brute force, or an
invariant of Eq. 3.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KDM_EXACT = Fraction("4148.808")


def _plan(cfg, n_dm=None):
    return oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"],
                              cfg["dm_start"], cfg["dm_step"], n_dm or cfg["n_dm"])


# --------------------------------------------------------------------------------------
# Shift table: Eq. 1 with channel c at f_high - c*df (Sec. 4.1), rounded half up.
# --------------------------------------------------------------------------------------

def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


def test_shift_hand_derived_delays():
    """Textbook delays worked out by hand from Eq. 1 (tests/golden/dispersion_delays.txt)."""
    for fh, f, dm, ts, want in _golden_rows("dispersion_delays.txt"):
        fh, f, dm, ts, want = float(fh), float(f), float(dm), float(ts), int(want)
        s = oracle.shift_table(1, fh, 0.0, ts, dm, 1.0, 1, freqs=np.array([f]))
        assert int(s[0, 0]) == want, (fh, f, dm, ts)
        # the same delay through the uniform-band form: channel 1 of a band with df = fh - f
        s2 = oracle.shift_table(2, fh, fh - f, ts, dm, 1.0, 1)
        assert int(s2[0, 1]) == want and int(s2[0, 0]) == 0


@pytest.mark.parametrize("name", ["small", "headline", "lowfreq_u4", "grad_f32"])
def test_shift_plan_max(name):
    """Largest shift of each workload, computed by hand (tests/golden/plan_facts.txt)."""
    facts = {r[0]: int(r[1]) for r in _golden_rows("plan_facts.txt")}
    s = _plan(synth.CONFIGS[name])
    assert int(s.max()) == facts[name]
    assert int(s[-1, -1]) == facts[name]  # lowest channel, largest DM


@pytest.mark.parametrize("name", ["small", "headline", "lowfreq_u4", "grad_f32"])
def test_shift_special_cases_and_monotone(name):
    """DM = 0 and the top channel have no delay; lower frequencies and larger DMs arrive later (Sec. 1)."""
    s = _plan(synth.CONFIGS[name])
    assert (s[0] == 0).all()
    assert (s[:, 0] == 0).all()
    assert (np.diff(s, axis=0) >= 0).all()
    assert (np.diff(s, axis=1) >= 0).all()
    assert s.dtype == np.int32


def _exact_delay(dm, f, f_high, t_samp):
    return dm * KDM_EXACT * (1 / (f * f) - 1 / (f_high * f_high)) / t_samp


@pytest.mark.parametrize("name", ["small", "headline", "lowfreq_u4", "grad_f32"])
def test_shift_matches_exact_rational(name):
    """Every FP64 entry equals round-half-up of the exact rational delay, away from ties."""
    cfg = synth.CONFIGS[name]
    s = _plan(cfg)
    fh = Fraction(repr(cfg["f_high"]))
    df = Fraction(cfg["chan_bw"])  # the band splits exactly in binary for all workloads
    ts = Fraction(repr(cfg["t_samp"]))
    step = Fraction(repr(cfg["dm_step"]))
    rng = np.random.default_rng(7)
    n = s.size if s.size <= 40000 else 20000
    idx = np.arange(s.size) if n == s.size else rng.choice(s.size, n, replace=False)
    checked = 0
    for i in idx:
        d, c = divmod(int(i), cfg["n_chan"])
        v = _exact_delay(Fraction(cfg["dm_start"]) + d * step, fh - c * df, fh, ts)
        frac = v - math.floor(v)
        if abs(frac - Fraction(1, 2)) < Fraction(1, 10**6):
            continue  # too near a tie for FP64 to be held to the exact result
        assert int(s[d, c]) == math.floor(v + Fraction(1, 2)), (d, c, float(v))
        checked += 1
    assert checked >= 0.99 * n


@pytest.mark.parametrize("name", ["headline", "lowfreq_u4", "grad_f32"])
def test_shift_against_narrow_band_form(name):
    """Across m channels the delay slope agrees with the narrow-band form of Eq. 4.

    Eq. 4 gives the delay across a channel of width df at centre f_c as
    2 * K * DM * df / f_c^3 (K = 4.148808e3), an independent statement of the
    f^-2 law's slope.  Over m adjacent channels the rounded table differs from
    it only by rounding (<= 1 sample) and the curvature of the law.
    """
    cfg = synth.CONFIGS[name]
    s = _plan(cfg)
    m = 64
    df = cfg["chan_bw"]
    for d in [cfg["n_dm"] // 3, cfg["n_dm"] - 1]:
        dm = cfg["dm_start"] + d * cfg["dm_step"]
        for c in [0, cfg["n_chan"] // 2, cfg["n_chan"] - 1 - m]:
            fc = cfg["f_high"] - (c + m / 2) * df
            pred = 2 * 4.148808e3 * dm * (m * df) / fc**3 / cfg["t_samp"]
            got = int(s[d, c + m]) - int(s[d, c])
            curv = pred * 1.5 * (m * df / fc) ** 2 + 1e-9
            assert abs(got - pred) <= 1.0 + curv, (d, c, got, pred)


def test_shift_rejects_bad_band():
    with pytest.raises(ValueError):
        oracle.shift_table(4, 100.0, 40.0, 1e-3, 0.0, 1.0, 2)  # channel 3 at -20 MHz


# --------------------------------------------------------------------------------------
# Forward transform: Eq. 3 / Algorithm 1.
# --------------------------------------------------------------------------------------

def _tiny_case(rng, dtype):
    n_chan = int(rng.integers(1, 9))
    n_samp = int(rng.integers(40, 97)) & ~1
    f_high = float(rng.uniform(300, 1600))
    bw = float(rng.uniform(0.05, 0.4)) * f_high / max(n_chan, 1)
    t_samp = float(rng.choice([64e-6, 128e-6, 1e-3]))
    # pick a DM range whose largest delay fits comfortably in the window
    k_max = 1 / (f_high - (n_chan - 1) * bw) ** 2 - 1 / f_high**2
    dm_max = 0.6 * n_samp * t_samp / (4.148808e3 * k_max) if k_max > 0 else 10.0
    n_dm = int(rng.integers(1, 6))
    step = dm_max / max(n_dm - 1, 1)
    start = float(rng.uniform(0, 0.2)) * dm_max if n_dm > 1 else dm_max * 0.5
    step = (dm_max - start) / max(n_dm - 1, 1)
    if dtype == "u8":
        x = rng.integers(0, 256, (n_chan, n_samp)).astype(np.uint8)
        x[:, ::7] = 0
        x[:, 3::11] = 255
    elif dtype == "u4":
        x = rng.integers(0, 16, (n_chan, n_samp)).astype(np.uint8)
    elif dtype == "u16":
        x = rng.integers(0, 65536, (n_chan, n_samp)).astype(np.uint16)
        x[:, ::7] = 0
        x[:, 3::11] = 65535
    elif dtype == "u32":  # binned 16-bit sums: up to 256 * 65535 < 2^24
        x = rng.integers(0, 256 * 65535 + 1, (n_chan, n_samp)).astype(np.uint32)
        x[:, ::7] = 0
        x[:, 3::11] = 256 * 65535
    else:
        x = rng.standard_normal((n_chan, n_samp)).astype(np.float32)
        x[:, ::5] = 0.0
    return dict(n_chan=n_chan, n_samp=n_samp, f_high=f_high, bw=bw, t_samp=t_samp,
                start=start, step=step, n_dm=n_dm, x=x)


def _pack_u4(v):
    return (v[:, 0::2] | (v[:, 1::2] << 4)).astype(np.uint8)


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "u32", "f32"])
def test_forward_equals_literal_eq3(dtype):
    """Brute-force Eq. 3 (oracle/eq3_literal.py, independent code) on tiny random inputs."""
    rng = np.random.default_rng({"u8": 11, "u4": 12, "f32": 13, "u16": 14, "u32": 15}[dtype])
    for _ in range(12):
        k = _tiny_case(rng, dtype)
        dms = [k["start"] + d * k["step"] for d in range(k["n_dm"])]
        ref, table, n_out = oracle.eq3_literal(
            [list(map(float, r)) if dtype == "f32" else list(map(int, r)) for r in k["x"]],
            k["n_samp"], k["f_high"], k["bw"], k["t_samp"], dms)
        s = oracle.shift_table(k["n_chan"], k["f_high"], k["bw"], k["t_samp"], k["start"],
                               k["step"], k["n_dm"])
        assert s.tolist() == table
        if n_out <= 0:
            continue
        if dtype == "u8":
            got = oracle.forward(k["x"], "u8", k["n_samp"], s)
            assert got.tolist() == ref
        elif dtype == "u4":
            got = oracle.forward(_pack_u4(k["x"]), "u4", k["n_samp"], s)
            assert got.tolist() == ref
        elif dtype == "u16":  # at most 8 channels: every sum is below 2^24, so float32 is exact
            got = oracle.forward(k["x"], "u16", k["n_samp"], s)
            assert got.tolist() == ref
        elif dtype == "u32":  # sums up to 2^27: the exact integer (a double here) rounded once to float32
            got = oracle.forward(k["x"], "u32", k["n_samp"], s)
            assert got.tolist() == [[float(np.float32(v)) for v in row] for row in ref]
        else:
            got, _ = oracle.forward_f32(k["x"], k["n_samp"], s)
            np.testing.assert_allclose(got, np.array(ref), rtol=0, atol=1e-12)


def _small():
    cfg = synth.CONFIGS["small"]
    s = _plan(cfg)
    x = synth.gaussian_u8(cfg["n_chan"], cfg["n_samp"], cfg["seed"])
    return cfg, s, x


def test_forward_dm0_is_channel_sum():
    """At DM = 0 every delay is 0, so the output is the plain channel sum."""
    cfg, s, x = _small()
    n_out = oracle.n_out_for(s, cfg["n_samp"])
    out = oracle.forward(x, "u8", cfg["n_samp"], s, rows=[0])
    assert np.array_equal(out[0], x[:, :n_out].sum(axis=0, dtype=np.int64).astype(np.float32))


def test_forward_injected_pulse():
    """A pulse injected along the plan's own delays adds exactly its amplitude at its DM
    and peaks there (the paper's injected-signal comparison, Sec. 5.3)."""
    cfg, s, x = _small()
    (dp, width, t0), = cfg["pulses"]
    xp = x.copy()
    applied = synth.inject_boxcar_u8(xp, s[dp], t0, width, cfg["amp"])
    rows = list(range(256))
    base = oracle.forward(x, "u8", cfg["n_samp"], s, rows=rows)
    withp = oracle.forward(xp, "u8", cfg["n_samp"], s, rows=rows)
    gain = (withp[dp, t0:t0 + width].astype(np.int64) - base[dp, t0:t0 + width].astype(np.int64))
    assert np.array_equal(gain, applied.sum(axis=0))
    assert gain.min() > 0.9 * cfg["amp"] * cfg["n_chan"]
    for k in range(width):
        assert int(np.argmax(withp[:, t0 + k])) == dp


def test_forward_linear():
    """A(x1 + x2) = A x1 + A x2 exactly for integer input without overflow."""
    rng = np.random.default_rng(3)
    n_chan, n_samp = 24, 4096
    s = oracle.shift_table(n_chan, 1500.0, 300.0 / n_chan, 64e-6, 0.0, 2.0, 40)
    x1 = rng.integers(0, 128, (n_chan, n_samp)).astype(np.uint8)
    x2 = rng.integers(0, 128, (n_chan, n_samp)).astype(np.uint8)
    a = oracle.forward(x1, "u8", n_samp, s)
    b = oracle.forward(x2, "u8", n_samp, s)
    ab = oracle.forward((x1 + x2).astype(np.uint8), "u8", n_samp, s)
    assert np.array_equal(ab.astype(np.int64), a.astype(np.int64) + b.astype(np.int64))


def test_forward_time_shift_and_chunking():
    """Delaying the input delays the output; chunks with a max-delay overlap reassemble the whole."""
    cfg, s, x = _small()
    n_samp = cfg["n_samp"]
    full = oracle.forward(x, "u8", n_samp, s)
    tau = 777
    shifted = oracle.forward(np.ascontiguousarray(x[:, tau:]), "u8", n_samp - tau, s)
    assert np.array_equal(shifted, full[:, tau:])
    max_shift = int(s.max())
    n_out = n_samp - max_shift
    parts, t = [], 0
    for chunk in [5000, 9999, 4096, n_out]:
        m = min(chunk, n_out - t)
        if m <= 0:
            break
        xs = np.ascontiguousarray(x[:, t:t + m + max_shift])
        parts.append(oracle.forward(xs, "u8", m + max_shift, s))
        t += m
    assert np.array_equal(np.concatenate(parts, axis=1), full)


def test_forward_row_sum_identity():
    """Sum over t of S(d,t) equals sum over c of (P_c[s + N_out] - P_c[s]) with P_c the prefix sums."""
    cfg, s, x = _small()
    n_out = oracle.n_out_for(s, cfg["n_samp"])
    out = oracle.forward(x, "u8", cfg["n_samp"], s)
    p = np.zeros((x.shape[0], x.shape[1] + 1), dtype=np.int64)
    np.cumsum(x, axis=1, out=p[:, 1:])
    c = np.arange(x.shape[0])
    want = (p[c[None, :], s + n_out] - p[c[None, :], s]).sum(axis=1)
    assert np.array_equal(out.astype(np.int64).sum(axis=1), want)


def test_forward_u4_equals_u8_equals_f32():
    """Packed 4-bit input equals its unpacked 8-bit and float forms."""
    cfg = synth.CONFIGS["lowfreq_u4"]
    n_chan, n_samp = 64, 8192
    s = oracle.shift_table(n_chan, cfg["f_high"], 70.0 / n_chan, cfg["t_samp"], 0.0, 0.5, 30)
    packed = synth.uniform_u4_packed(n_chan, n_samp, 3)
    unpacked = synth.unpack_u4(packed, n_samp)
    a = oracle.forward(packed, "u4", n_samp, s)
    b = oracle.forward(unpacked, "u8", n_samp, s)
    c, _ = oracle.forward_f32(unpacked.astype(np.float32), n_samp, s)
    assert np.array_equal(a, b)
    assert np.array_equal(a.astype(np.float64), c)


def test_forward_u16_small_values_equal_u8():
    """16-bit samples below 256 give exactly the 8-bit result."""
    cfg, s, x = _small()
    a = oracle.forward(x, "u8", cfg["n_samp"], s, rows=[0, 7, 100, 255])
    b = oracle.forward(x.astype(np.uint16), "u16", cfg["n_samp"], s, rows=[0, 7, 100, 255])
    assert np.array_equal(a, b)


def test_forward_u16_little_endian_samples():
    """A 16-bit sample is its low byte plus 256 times its high byte (little-endian)."""
    raw = np.zeros((1, 2 * 64), dtype=np.uint8)
    raw[0, 2 * 5], raw[0, 2 * 5 + 1] = 0x01, 0x02  # sample 5 = 0x0201 = 513
    raw[0, 2 * 9 + 1] = 0xFF                         # sample 9 = 0xFF00 = 65280
    x = raw.view("<u2")
    s = np.zeros((1, 1), dtype=np.int32)  # one channel, one DM, no delay
    out = oracle.forward(np.ascontiguousarray(x), "u16", 64, s)
    want = np.zeros(64, dtype=np.float32)
    want[5], want[9] = 513.0, 65280.0
    assert np.array_equal(out[0], want)


def test_forward_u32_little_endian_samples_and_u16_agreement():
    """A 32-bit sample is its bytes in little-endian order; 32-bit data of 16-bit values gives
    the 16-bit transform, and a value above 2^16 adds its high part on top of it."""
    raw = np.zeros((1, 4 * 64), dtype=np.uint8)
    raw[0, 4 * 5: 4 * 5 + 4] = [0x01, 0x02, 0x03, 0x00]  # sample 5 = 0x030201 = 197121
    raw[0, 4 * 9 + 2] = 0xFF                            # sample 9 = 0xFF0000 = 16711680
    raw[0, 4 * 12 + 3] = 0x02                           # sample 12 = 0x02000000 = 2^25
    s0 = np.zeros((1, 1), dtype=np.int32)
    out = oracle.forward(np.ascontiguousarray(raw.view("<u4")), "u32", 64, s0)
    want = np.zeros(64, dtype=np.float32)
    want[5], want[9], want[12] = 197121.0, 16711680.0, 2.0 ** 25
    assert np.array_equal(out[0], want)
    rng = np.random.default_rng(44)
    cfg, s, _ = _small()
    x16 = rng.integers(0, 65536, (cfg["n_chan"], 4000)).astype(np.uint16)
    s = s[:: 16, :]
    s = s[:, :] // 4  # small delays that fit 4000 samples
    assert np.array_equal(oracle.forward(x16.astype(np.uint32), "u32", 4000, s), oracle.forward(x16, "u16", 4000, s))
    hi = rng.integers(0, 256, (cfg["n_chan"], 4000)).astype(np.uint32)
    got = oracle.forward(x16.astype(np.uint32) + (hi << 16), "u32", 4000, s)
    lo_sum = oracle.forward(x16, "u16", 4000, s).astype(np.float64)     # exact: 128 * 65535 < 2^24
    hi_sum = oracle.forward(hi.astype(np.uint8), "u8", 4000, s).astype(np.float64)
    assert np.array_equal(got, (lo_sum + 65536.0 * hi_sum).astype(np.float32))


def test_forward_u16_sums_round_to_float32_nearest_even():
    """Sums above 2^24 are converted once to float32, rounding to nearest even."""
    n_chan, n_samp = 257, 32
    x = np.full((n_chan, n_samp), 65535, dtype=np.uint16)
    x[256, :] = 257                      # 256 * 65535 + 257 = 2^24 + 1, halfway between two floats
    x[256, 1] = 258                      # 2^24 + 2 is a float32
    x[256, 2] = 259                      # 2^24 + 3 rounds up to 2^24 + 4 (even mantissa)
    s = np.zeros((1, n_chan), dtype=np.int32)
    out = oracle.forward(x, "u16", n_samp, s)[0]
    assert out[0] == np.float32(2 ** 24) and out[1] == np.float32(2 ** 24 + 2) and out[2] == np.float32(2 ** 24 + 4)
    assert 256 * 65535 + 257 == 2 ** 24 + 1


def _dense_matrix(s, n_samp):
    n_dm, n_chan = s.shape
    n_out = n_samp - int(s.max())
    a = np.zeros((n_dm * n_out, n_chan * n_samp))
    for d in range(n_dm):
        for c in range(n_chan):
            for t in range(n_out):
                a[d * n_out + t, c * n_samp + t + s[d, c]] += 1.0
    return a, n_out


def test_forward_and_adjoint_against_dense_matrix():
    """Both directions agree with an explicit 0/1 matrix built term by term."""
    rng = np.random.default_rng(5)
    n_chan, n_samp = 6, 80
    s = oracle.shift_table(n_chan, 400.0, 20.0, 1e-3, 0.5, 0.5, 5)
    a, n_out = _dense_matrix(s, n_samp)
    x = rng.integers(0, 256, (n_chan, n_samp)).astype(np.uint8)
    got = oracle.forward(x, "u8", n_samp, s)
    assert np.array_equal(got.reshape(-1), a @ x.reshape(-1).astype(np.float64))
    y = rng.standard_normal((s.shape[0], n_out)).astype(np.float32)
    g = oracle.adjoint(y, n_chan, n_samp, s)
    np.testing.assert_allclose(g.reshape(-1), a.T @ y.reshape(-1).astype(np.float64), rtol=0, atol=1e-12)


def test_forward_f32_abs_sum_against_dense_matrix():
    """The second output of the float forward, the sum of |terms| that scales every
    float tolerance, is |A| |x| for the 0/1 matrix of Eq. 3 and equals the forward of
    |x|; with signed terms it is strictly larger than |sum| where signs cancel."""
    rng = np.random.default_rng(15)
    n_chan, n_samp = 7, 90
    s = oracle.shift_table(n_chan, 400.0, 20.0, 1e-3, 0.1, 0.4, 6)
    a, n_out = _dense_matrix(s, n_samp)
    # small integers and halves: every FP64 sum below is exact, so equality is exact
    x = (rng.integers(-16, 17, (n_chan, n_samp)) * 0.5).astype(np.float32)
    out, ab = oracle.forward_f32(x, n_samp, s)
    assert np.array_equal(out.reshape(-1), a @ x.reshape(-1).astype(np.float64))
    assert np.array_equal(ab.reshape(-1), a @ np.abs(x.reshape(-1)).astype(np.float64))
    out_abs, _ = oracle.forward_f32(np.abs(x), n_samp, s)
    assert np.array_equal(ab, out_abs)
    assert np.all(ab >= np.abs(out)) and np.any(ab > np.abs(out))
    # a row subset returns the same rows of both outputs, each started from zero
    rows = [5, 0, 3]
    out_r, ab_r = oracle.forward_f32(x, n_samp, s, rows=rows)
    assert np.array_equal(out_r, out[rows]) and np.array_equal(ab_r, ab[rows])


# --------------------------------------------------------------------------------------
# Adjoint: transpose of Eq. 3 (scatter form).
# --------------------------------------------------------------------------------------

def _grad_case(n_chan=96, n_samp=6000, n_dm=48):
    cfg = synth.CONFIGS["grad_f32"]
    s = oracle.shift_table(n_chan, cfg["f_high"], 300.0 / n_chan, cfg["t_samp"], 0.0, 4.0, n_dm)
    return s, n_samp


def test_adjoint_exact_dot_test_small_integers():
    """<Ax, y> = <x, A^T y> exactly: small integers make every sum exact in FP64."""
    s, n_samp = _grad_case()
    rng = np.random.default_rng(9)
    n_dm, n_chan = s.shape
    n_out = oracle.n_out_for(s, n_samp)
    x = rng.integers(-15, 16, (n_chan, n_samp)).astype(np.float32)
    y = rng.integers(-3, 4, (n_dm, n_out)).astype(np.float32)
    ax, _ = oracle.forward_f32(x, n_samp, s)
    aty = oracle.adjoint(y, n_chan, n_samp, s)
    lhs = float((ax * y.astype(np.float64)).sum())
    rhs = float((x.astype(np.float64) * aty).sum())
    assert lhs == rhs


def test_adjoint_dot_test_gaussian():
    s, n_samp = _grad_case()
    rng = np.random.default_rng(10)
    n_dm, n_chan = s.shape
    n_out = oracle.n_out_for(s, n_samp)
    x = rng.standard_normal((n_chan, n_samp)).astype(np.float32)
    y = rng.standard_normal((n_dm, n_out)).astype(np.float32)
    ax, _ = oracle.forward_f32(x, n_samp, s)
    aty = oracle.adjoint(y, n_chan, n_samp, s)
    lhs = float((ax * y.astype(np.float64)).sum())
    rhs = float((x.astype(np.float64) * aty).sum())
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), abs(rhs))


def test_adjoint_unread_entries_are_zero():
    """Input samples that no output reads get exactly zero gradient."""
    s, n_samp = _grad_case()
    n_dm, n_chan = s.shape
    n_out = oracle.n_out_for(s, n_samp)
    y = np.ones((n_dm, n_out), dtype=np.float32)
    g = oracle.adjoint(y, n_chan, n_samp, s)
    read = np.zeros((n_chan, n_samp), dtype=bool)
    for c in range(n_chan):
        for d in range(n_dm):
            read[c, s[d, c]:s[d, c] + n_out] = True
    assert (g[~read] == 0).all()
    assert (g[read] > 0).all()


def test_gradient_by_central_differences():
    """loss = sum (A x - target)^2 is exactly quadratic, so central differences with
    h = 0.5 have no truncation error; they must match 2 A^T (A x - target)."""
    s, n_samp = _grad_case(n_chan=32, n_samp=3000, n_dm=20)
    rng = np.random.default_rng(41)
    n_dm, n_chan = s.shape
    n_out = oracle.n_out_for(s, n_samp)
    x = rng.standard_normal((n_chan, n_samp)).astype(np.float32)
    target = rng.standard_normal((n_dm, n_out))

    def loss(xx):
        ax, _ = oracle.forward_f32(xx, n_samp, s)
        return float(((ax - target) ** 2).sum())

    ax, _ = oracle.forward_f32(x, n_samp, s)
    grad = 2.0 * oracle.adjoint((ax - target).astype(np.float32), n_chan, n_samp, s)
    picks = [(int(c), int(t)) for c, t in zip(rng.integers(0, n_chan, 24), rng.integers(0, n_samp, 24))]
    picks += [(0, n_samp - 1), (0, n_out), (n_chan - 1, n_samp - 1)]  # the first two feed no output
    h = 0.5
    for c, t in picks:
        xp, xm = x.copy(), x.copy()
        xp[c, t] += h
        xm[c, t] -= h
        fd = (loss(xp) - loss(xm)) / (2 * h)
        assert abs(fd - grad[c, t]) <= 1e-6 * max(1.0, abs(fd)), (c, t, fd, grad[c, t])
    assert grad[0, n_samp - 1] == 0.0 and grad[0, n_out] == 0.0  # channel 0 never delays


# --------------------------------------------------------------------------------------
# Time binning (the downsampling of Secs. 5.2, 5.3, 5.5 and 6): sums of `factor` consecutive samples
# per channel, a trailing partial bin dropped.
# --------------------------------------------------------------------------------------

def _unpack_u4_numpy(packed, n_samp):
    out = np.empty((packed.shape[0], packed.shape[1] * 2), dtype=np.int64)
    out[:, 0::2] = packed & 15
    out[:, 1::2] = packed >> 4
    return out[:, :n_samp]


def _bin_case(rng, dtype, n_chan, n_samp):
    if dtype == "u8":
        x = rng.integers(0, 256, (n_chan, n_samp)).astype(np.uint8)
        return x, x.astype(np.int64)
    if dtype == "u4":
        v = rng.integers(0, 16, (n_chan, n_samp + (n_samp & 1))).astype(np.uint8)
        packed = _pack_u4(v)
        return packed, _unpack_u4_numpy(packed, n_samp)
    if dtype == "u16":
        x = rng.integers(0, 65536, (n_chan, n_samp)).astype(np.uint16)
        return x, x.astype(np.int64)
    x = rng.standard_normal((n_chan, n_samp)).astype(np.float32)
    return x, x.astype(np.float64)


@pytest.mark.parametrize("dtype", ["u8", "u4", "u16", "f32"])
def test_bin_equals_reshape_sum(dtype):
    """Binning equals numpy's reshape-and-sum over the whole bins, for ragged lengths."""
    rng = np.random.default_rng({"u8": 31, "u4": 32, "u16": 33, "f32": 34}[dtype])
    for n_samp, factor in [(1000, 1), (1000, 2), (1001, 3), (997, 7), (4099, 16), (300, 256), (255, 256)]:
        x, vals = _bin_case(rng, dtype, 5, n_samp)
        got = oracle.bin_time(x, dtype, n_samp, factor)
        nb = n_samp // factor
        want = vals[:, :nb * factor].reshape(5, nb, factor).sum(axis=2)
        assert got.shape == (5, nb)
        if dtype == "f32":
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-9)
        else:
            assert np.array_equal(got, want)


def test_bin_factor_one_identity_constant_and_impulse():
    rng = np.random.default_rng(35)
    x, _ = _bin_case(rng, "u8", 3, 640)
    assert np.array_equal(oracle.bin_time(x, "u8", 640, 1), x.astype(np.int64))
    const = np.full((2, 640), 9, dtype=np.uint8)
    for f in (2, 5, 64):
        assert np.all(oracle.bin_time(const, "u8", 640, f) == 9 * f)
    # one sample: lands in bin t // f of its own channel, or nowhere past the last whole bin
    for t in (0, 1, 399, 400, 639):
        imp = np.zeros((2, 640), dtype=np.uint8)
        imp[1, t] = 200
        got = oracle.bin_time(imp, "u8", 640, 8)
        assert got[0].sum() == 0
        assert got[1].sum() == 200 and got[1, t // 8] == 200
        got3 = oracle.bin_time(imp, "u8", 640, 3)  # 213 whole bins cover samples 0..638
        assert got3[1].sum() == (200 if t < 639 else 0)


def test_bin_factors_compose():
    """Binning by 2 and then by 3 equals binning by 6 (sums regroup)."""
    rng = np.random.default_rng(36)
    x, _ = _bin_case(rng, "u8", 4, 1203)
    b2 = oracle.bin_time(x, "u8", 1203, 2)
    b23 = oracle.bin_time(np.ascontiguousarray(b2.astype(np.uint16)), "u16", b2.shape[1], 3)
    assert np.array_equal(b23, oracle.bin_time(x, "u8", 1203, 6))


def test_binned_forward_dm0_is_sum_of_unbinned_dm0():
    """At DM 0 every delay is zero, so the binned transform is the binned channel sum."""
    cfg, s, x = _small()
    n_samp, f = cfg["n_samp"], 4
    b = oracle.bin_time(x, "u8", n_samp, f).astype(np.uint16)
    sb = oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"] * f, 0.0, 1.0, 1)
    assert not sb.any()
    got = oracle.forward(b, "u16", b.shape[1], sb)
    assert s[0].max() == 0  # the unbinned plan's first row is DM 0 as well
    row0 = oracle.forward(x, "u8", n_samp, s, rows=[0])[0].astype(np.int64)
    n = len(row0) // f
    assert np.array_equal(got[0, :n].astype(np.int64), row0[:n * f].reshape(-1, f).sum(1))
    want = x.astype(np.int64).sum(axis=0)[:b.shape[1] * f].reshape(-1, f).sum(1)
    assert np.array_equal(got[0].astype(np.int64), want)


def test_binned_forward_with_delays_in_whole_bins():
    """When every delay is a whole number of bins, binning commutes with the transform.

    Channel frequencies are chosen (explicit table) so that Eq. 1 gives delays of
    exactly f*m_c samples at the plan's single DM; on the grid of t_samp*f the same
    frequencies give m_c bins, and S_binned(j) = sum_i S(j*f + i).
    """
    f_high, t_samp, dm, f = 1500.0, 64e-6, 400.0, 4
    m = np.array([0, 1, 3, 4, 9, 13, 20, 31])
    # f_c^-2 = f_high^-2 + f*m_c*t_samp/(k*DM), chosen with a small safety margin inside the rounding interval
    freqs = (f_high ** -2 + f * m * t_samp / (4.148808e3 * dm)) ** -0.5
    s1 = oracle.shift_table(len(m), f_high, 0.0, t_samp, dm, 0.0, 1, freqs=freqs)
    sf = oracle.shift_table(len(m), f_high, 0.0, t_samp * f, dm, 0.0, 1, freqs=freqs)
    assert s1[0].tolist() == (f * m).tolist() and sf[0].tolist() == m.tolist()
    rng = np.random.default_rng(37)
    n_samp = 4000
    x = rng.integers(0, 256, (len(m), n_samp)).astype(np.uint8)
    full = oracle.forward(x, "u8", n_samp, s1)[0].astype(np.int64)
    b = oracle.bin_time(x, "u8", n_samp, f).astype(np.uint16)
    got = oracle.forward(b, "u16", b.shape[1], sf)[0].astype(np.int64)
    assert np.array_equal(got, full[:len(got) * f].reshape(-1, f).sum(1))


# --------------------------------------------------------------------------------------
# Corner turn (the input transpose of the pipelines, Secs. 5.3 and 5.5): time-major
# spectra to the channel-major rows Eq. 3 reads.
# --------------------------------------------------------------------------------------

def _nibbles_numpy(packed, n):
    """Unpack nibble pairs (element 2k in the low nibble) along the last axis."""
    out = np.empty(packed.shape[:-1] + (packed.shape[-1] * 2,), dtype=np.uint8)
    out[..., 0::2] = packed & 15
    out[..., 1::2] = packed >> 4
    return out[..., :n]


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_corner_turn_is_numpy_transpose(dtype):
    rng = np.random.default_rng(41)
    for n_chan, n_samp, pad in [(1, 1, 0), (7, 13, 3), (300, 257, 16), (64, 1000, 0)]:
        if dtype == "f32":
            cm = rng.standard_normal((n_chan, n_samp)).astype(np.float32)
        else:
            cm = rng.integers(0, 256 if dtype == "u8" else 65536, (n_chan, n_samp)).astype(
                np.uint8 if dtype == "u8" else np.uint16)
        tm = np.zeros((n_samp, n_chan + pad), dtype=cm.dtype)
        tm[:, :n_chan] = cm.T
        got = oracle.corner_turn(tm, dtype, n_chan, n_samp)
        assert got.dtype == cm.dtype and np.array_equal(got, cm)


def test_corner_turn_u4_nibble_orders():
    """4-bit spectra pack channel pairs, 4-bit rows pack time pairs, low nibble first."""
    rng = np.random.default_rng(42)
    for n_chan, n_samp in [(1, 2), (5, 10), (64, 200), (33, 64)]:
        v = rng.integers(0, 16, (n_chan, n_samp)).astype(np.uint8)  # v[c][t]
        vt = np.zeros((n_samp, n_chan + (n_chan & 1)), dtype=np.uint8)
        vt[:, :n_chan] = v.T
        spectra = (vt[:, 0::2] | (vt[:, 1::2] << 4)).astype(np.uint8)
        rows = oracle.corner_turn(np.ascontiguousarray(spectra), "u4", n_chan, n_samp)
        assert np.array_equal(_nibbles_numpy(rows, n_samp), v)
    # one hand-made case: spectrum t holds channels (0, 1) = (t, 15 - t)
    spectra = np.array([[t | ((15 - t) << 4)] for t in range(4)], dtype=np.uint8)
    rows = oracle.corner_turn(spectra, "u4", 2, 4)
    assert rows.tolist() == [[0x10, 0x32], [0xEF, 0xCD]]


def test_corner_turn_round_trip_and_forward():
    """Turning twice (roles of channels and times swapped) is the identity, and the turned
    spectra dedisperse exactly as the channel-major original."""
    cfg, s, x = _small()
    n_chan, n_samp = cfg["n_chan"], cfg["n_samp"]
    spectra = np.ascontiguousarray(x[:, :n_samp].T)
    rows = oracle.corner_turn(spectra, "u8", n_chan, n_samp)
    assert np.array_equal(oracle.corner_turn(rows, "u8", n_samp, n_chan), spectra)
    assert np.array_equal(oracle.forward(rows, "u8", n_samp, s, rows=[0, 100, 255]),
                          oracle.forward(x, "u8", n_samp, s, rows=[0, 100, 255]))
    rng = np.random.default_rng(43)
    v = rng.integers(0, 16, (6, 40)).astype(np.uint8)
    packed_rows = (v[:, 0::2] | (v[:, 1::2] << 4)).astype(np.uint8)
    vt = np.ascontiguousarray(v.T)
    spectra4 = (vt[:, 0::2] | (vt[:, 1::2] << 4)).astype(np.uint8)
    assert np.array_equal(oracle.corner_turn(np.ascontiguousarray(spectra4), "u4", 6, 40), packed_rows)
    assert np.array_equal(oracle.corner_turn(packed_rows, "u4", 40, 6), spectra4)
