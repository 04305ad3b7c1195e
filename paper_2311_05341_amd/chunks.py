"""Time chunks of one long filterbank that share its buffers.

The transform's output column t reads input columns t .. t + max_shift only
(Eq. 3 with integer delays), so outputs [t0, t0 + L) of the whole input equal
the outputs of the same plan applied to input columns [t0, t0 + L + max_shift).
A chunk is therefore a plan for n_samp = L + max_shift whose input is a view
of the full input starting at column t0 (same row pitch, so no copy), and
whose output can go to a view of a full output buffer at column t0 or to a
smaller buffer that is reused chunk after chunk (streaming).
"""
from __future__ import annotations

from .binding import Plan

_UNIT = {"u8": 16, "u4": 32, "u16": 8, "f32": 4}  # samples per 16 bytes: chunk starts stay 16-byte aligned


class TimeChunks:
    """Split the output time axis of a plan description into n_chunks chunks.

    ``desc`` holds the keyword arguments of ``Plan`` for the whole input
    (n_chan, n_samp, dtype, f_high, chan_bw, t_samp, dm_start, dm_step, n_dm,
    and optionally chan_freq and in_pitch_bytes).  Chunk starts are multiples
    of 16 bytes of input; every chunk but the last has the same length.
    """

    def __init__(self, desc: dict, n_chunks: int, device=None, whole: Plan | None = None, bind=True):
        if n_chunks < 1:
            raise ValueError("n_chunks must be >= 1")
        self.desc = dict(desc)
        whole = whole or Plan(**self.desc, bind=False)
        self.max_shift = whole.max_shift
        self.n_out = whole.n_out
        self.in_pitch_bytes = whole.in_pitch_bytes
        unit = _UNIT[self.desc["dtype"]]
        length = -(-self.n_out // n_chunks)
        length = -(-length // unit) * unit
        self.spans = []  # (first output sample, output samples)
        t = 0
        while t < self.n_out:
            self.spans.append((t, min(length, self.n_out - t)))
            t += length
        args = dict(self.desc, in_pitch_bytes=self.in_pitch_bytes, device=device, bind=bind)
        plans = {}
        for _, n in self.spans:
            if n not in plans:
                n_samp = n + self.max_shift
                if self.desc["dtype"] == "u4":
                    # 4-bit rows hold whole bytes: with an odd max shift a chunk computes
                    # one more column, the next chunk's first (identical values)
                    n_samp += n_samp & 1
                plans[n] = Plan(**dict(args, n_samp=n_samp))
        self.plans = [plans[n] for _, n in self.spans]
        for p, (_, n) in zip(self.plans, self.spans):
            assert p.max_shift == self.max_shift and n <= p.n_out <= n + 1

    @property
    def chunk_len(self) -> int:
        """Output columns a per-chunk output buffer must hold (any chunk)."""
        return max(p.n_out for p in self.plans)

    def input_view(self, x, k: int):
        """Input columns of chunk k: a view of the whole input x (rows of in_pitch_bytes)."""
        t0 = self.spans[k][0]
        dt = self.desc["dtype"]
        col = t0 // 2 if dt == "u4" else t0
        return x[:, col:]

    def output_view(self, out, k: int):
        """Output columns of chunk k inside a whole-length output buffer."""
        return out[:, self.spans[k][0]:]

    def __len__(self):
        return len(self.spans)
