"""Eq. 3 evaluated literally, term by term -- TEST INFRASTRUCTURE, tiny inputs only.

Every term's delay is recomputed inline from Eq. 1 (channel c at
f_high - c*df as in Sec. 4.1, constant 4.148808e3 s MHz^2 cm^3/pc, rounded half
up) with Python floats, and the sum is taken with Python integers (or exact
fractions for float input).  It shares no code with ``oracle.c``; it exists to
check the C oracle by brute force.
"""
from __future__ import annotations

import math
from fractions import Fraction


def shift_literal(dm: float, f: float, f_high: float, t_samp: float) -> int:
    """Delay of frequency f relative to f_high, in whole samples (Eq. 1)."""
    delay_s = dm * 4.148808e3 * (1.0 / (f * f) - 1.0 / (f_high * f_high))
    return int(math.floor(delay_s / t_samp + 0.5))


def eq3_literal(x, n_samp, f_high, chan_bw, t_samp, dms, sample=None):
    """S(d, t) = sum over channels of x(c, t + delay(c, d)) for every t < N_out.

    x is a list of channel rows; ``sample(row, t)`` decodes one input sample
    (default: row[t]).  Integer samples sum exactly as ints; float samples are
    summed exactly as Fractions and returned as floats.
    """
    if sample is None:
        def sample(row, t):
            return row[t]
    n_chan = len(x)
    table = [[shift_literal(dm, f_high - c * chan_bw, f_high, t_samp) for c in range(n_chan)]
             for dm in dms]
    n_out = n_samp - max(max(r) for r in table)
    out = []
    for d in range(len(dms)):
        row = []
        for t in range(n_out):
            acc = 0
            for c in range(n_chan):
                v = sample(x[c], t + table[d][c])
                acc += Fraction(v) if isinstance(v, float) else v
            row.append(float(acc))
        out.append(row)
    return out, table, n_out
