"""Shared test helpers: build plans and seeded inputs for both the oracle and the GPU."""
import numpy as np

import oracle
import synth


def oracle_table(cfg):
    return oracle.shift_table(cfg["n_chan"], cfg["f_high"], cfg["chan_bw"], cfg["t_samp"],
                              cfg["dm_start"], cfg["dm_step"], cfg["n_dm"])


def host_input(cfg, shift=None, pitch=None):
    """Seeded host input of a workload, with its pulses injected along the oracle's delays.

    Returns (x, applied) where applied maps pulse index -> increments array.
    """
    dt = cfg["dtype"]
    if dt == "u8":
        x = synth.gaussian_u8(cfg["n_chan"], cfg["n_samp"], cfg["seed"], pitch=pitch)
    elif dt == "u4":
        x = synth.uniform_u4_packed(cfg["n_chan"], cfg["n_samp"], cfg["seed"], pitch_bytes=pitch)
    elif dt == "u16":
        x = synth.gaussian_u16(cfg["n_chan"], cfg["n_samp"], cfg["seed"], pitch=pitch)
    else:
        x = synth.normal_f32(cfg["n_chan"], cfg["n_samp"], cfg["seed"], pitch=pitch)
    applied = {}
    for i, (dp, width, t0) in enumerate(cfg.get("pulses", [])):
        applied[i] = synth.inject_boxcar_u8(x, shift[dp], t0, width, cfg["amp"])
    return x, applied


def plan_for(dd, cfg, **kw):
    args = dict(n_chan=cfg["n_chan"], n_samp=cfg["n_samp"], dtype=cfg["dtype"], f_high=cfg["f_high"],
                chan_bw=cfg["chan_bw"], t_samp=cfg["t_samp"], dm_start=cfg["dm_start"],
                dm_step=cfg["dm_step"], n_dm=cfg["n_dm"])
    args.update(kw)
    return dd.Plan(**args)


def sample_rows(n_dm, pulses=(), every=None, extra=0, seed=0):
    rows = {0, n_dm - 1}
    rows.update(p[0] for p in pulses)
    if every:
        rows.update(range(0, n_dm, every))
    if extra:
        rng = np.random.default_rng(seed)
        rows.update(int(v) for v in rng.integers(0, n_dm, extra))
    return sorted(rows)


def row_sums_by_prefix(x_rows, shift, n_out, workers=16):
    """Sum over t of S(d, t) for every d, from per-channel prefix sums (integer input).

    x_rows(c) returns channel c's samples as a 1-D integer array.
    """
    from concurrent.futures import ThreadPoolExecutor

    n_dm, n_chan = shift.shape
    total = np.zeros(n_dm, dtype=np.int64)

    def part(cs):
        acc = np.zeros(n_dm, dtype=np.int64)
        for c in cs:
            v = x_rows(c)
            p = np.zeros(v.shape[0] + 1, dtype=np.int64)
            np.cumsum(v, out=p[1:])
            s = shift[:, c].astype(np.int64)
            acc += p[s + n_out] - p[s]
        return acc

    chunks = np.array_split(np.arange(n_chan), workers)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for a in ex.map(part, chunks):
            total += a
    return total
