// Host side of a plan: validation, the FP64 integer shift table, delay spans
// and the tile shape.  No device code here.
//
// The shift table follows Sec. 1, Eq. 1 (cold-plasma delay relative to the top
// of the band) with channel c at f_high - c*df as in Sec. 4.1, the constant
// 4.148808e3 s MHz^2 cm^3/pc, divided by the sampling time and rounded half up.
// It is evaluated in IEEE FP64 with no contraction, in one fixed order, so the
// table is bit-for-bit reproducible; the device only receives the integers.
#pragma clang fp contract(off)

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <new>
#include <thread>

#include "dd_internal.h"

namespace dd {

static const double kDispersionConstant = 4.148808e3;  // s MHz^2 cm^3 / pc

static double channel_freq(const dd_plan &p, int c) {
  if (!p.freqs.empty()) return p.freqs[c];
  return p.desc.f_high_mhz - (double)c * p.desc.chan_bw_mhz;
}

dd_status build_shift_table(dd_plan &p) {
  const int nc = p.desc.n_chan, nd = p.desc.n_dm;
  const double fh = p.desc.f_high_mhz;
  std::vector<double> k(nc);
  for (int c = 0; c < nc; ++c) {
    double f = channel_freq(p, c);
    if (!(f > 0.0) || !(f <= fh) || !isfinite(f))
      return fail(DD_ERR_RANGE, "channel " + std::to_string(c) + " frequency " + std::to_string(f) +
                                    " MHz is not in (0, f_high]");
    k[c] = 1.0 / (f * f) - 1.0 / (fh * fh);
  }
  try {
    p.shift.assign((size_t)nd * nc, 0);
  } catch (const std::bad_alloc &) {
    return fail(DD_ERR_NOMEM, "shift table allocation failed");
  }
  const double t = p.desc.t_samp_s, d0 = p.desc.dm_start, step = p.desc.dm_step;
  int bad = 0;
  auto rows = [&](int lo, int hi, int *flag) {
    for (int d = lo; d < hi; ++d) {
      const double dm = d0 + (double)d * step;
      int32_t *row = p.shift.data() + (size_t)d * nc;
      for (int c = 0; c < nc; ++c) {
        const double v = ((dm * kDispersionConstant) * k[c]) / t;
        const double s = floor(v + 0.5);
        if (!(s >= 0.0 && s <= 2147483647.0)) { *flag = 1; return; }
        row[c] = (int32_t)s;
      }
    }
  };
  const size_t work = (size_t)nd * nc;
  int nthr = work < (1u << 20) ? 1 : (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
  if (nthr == 1) {
    rows(0, nd, &bad);
  } else {
    std::vector<std::thread> th;
    std::vector<int> flags(nthr, 0);
    for (int i = 0; i < nthr; ++i) {
      int lo = (int)((int64_t)nd * i / nthr), hi = (int)((int64_t)nd * (i + 1) / nthr);
      th.emplace_back(rows, lo, hi, &flags[i]);
    }
    for (auto &x : th) x.join();
    for (int f : flags) bad |= f;
  }
  if (bad) return fail(DD_ERR_RANGE, "a shift does not fit in int32");
  // The kernels rely on delays never decreasing with d (each DM block is
  // staged from its first row's delays); Eq. 1 with dm_step >= 0 and
  // f_c <= f_high guarantees it, and so does monotone FP64 rounding.  Check.
  for (int d = 1; d < nd; ++d) {
    const int32_t *a = p.shift.data() + (size_t)(d - 1) * nc, *b = a + nc;
    for (int c = 0; c < nc; ++c)
      if (b[c] < a[c]) return fail(DD_ERR_RANGE, "shift table decreases with DM");
  }
  int32_t mx = 0;
  for (int32_t v : p.shift) mx = std::max(mx, v);
  p.max_shift = mx;
  p.n_out = p.desc.n_samp - (int64_t)mx;
  if (p.n_out <= 0)
    return fail(DD_ERR_TOO_SHORT, "n_samp " + std::to_string(p.desc.n_samp) + " <= largest shift " +
                                      std::to_string(mx));
  return DD_OK;
}

// Largest delay spread max_c(shift[d_hi][c] - shift[d_lo][c]) over the DM blocks
// [b*dm_block, b*dm_block + dm_block) (the last block clipped).  Shifts never
// decrease with d, so the spread inside a block is last row minus first row.
int32_t max_dm_block_span(const dd_plan &p, int dm_block) {
  const int nc = p.desc.n_chan, nd = p.desc.n_dm;
  int32_t span = 0;
  for (int lo = 0; lo < nd; lo += dm_block) {
    const int hi = std::min(lo + dm_block, nd) - 1;
    const int32_t *a = p.shift.data() + (size_t)lo * nc, *b = p.shift.data() + (size_t)hi * nc;
    for (int c = 0; c < nc; ++c) span = std::max(span, b[c] - a[c]);
  }
  return span;
}

static const int kLdsLimit = 160 * 1024;

static int round_up(int64_t v, int a) { return (int)((v + a - 1) / a * a); }

// Tables of the integer forward kernel for tile shape (ns, dm_per_wave, waves).
// For DM block b, channel c: sbase = shift(c, first DM of b) rounded down to
// the staging unit (the samples in 16 bytes: 16 for u8, 32 for u4, 8 for u16);
// for each DM d of the block, with v = shift(c, d) - sbase the window's offset
// in the staged row, the entry is the LDS byte offset of its first word inside
// the channel's shifted copies (each row_bytes long): for 8- and 4-bit samples
// (one byte each once staged) four copies, (v % 4) * row_bytes + (v - v % 4);
// for 16-bit samples (byte offset 2v) two copies,
// (v % 2) * row_bytes + 2 * (v - v % 2).  Phase-load shapes (segs > 0) add
// the channel's place in the staging slot; for packed 4-bit samples the copies
// are the eight nibble phases of the packed row and the entry is
// (v % 8) * row_bytes + 4 * (v / 8).
// Fails with DD_ERR_RANGE if even one channel per LDS stage does not fit.
dd_status build_int_tables(const dd_plan &p, int ns, int dm_per_wave, int waves, int chan_block, int segs,
                           int lds_limit, IntTables *t, bool fill) {
  const int nc = p.desc.n_chan, nd = p.desc.n_dm;
  const int dblk = waves * dm_per_wave;
  const bool u16 = p.desc.dtype == DD_U16;
  const bool u4 = p.desc.dtype == DD_U4;
  const int unit = u4 ? 32 : u16 ? 8 : 16;
  const bool phase = segs > 0;  // phase-load staging (8-bit, packed 4-bit)
  if (phase && p.desc.dtype == DD_F32) return fail(DD_ERR_RANGE, "phase-load staging is for integer input");
  if (phase && u4 && (ns % 8 || chan_block > 16)) return fail(DD_ERR_RANGE, "shape not compiled for 4-bit phase loads");
  // copies of a staged row: byte phases (4, or 2 for 16-bit samples); packed
  // 4-bit phase loads keep the eight nibble phases of the packed row
  const int copies = phase && u4 ? 8 : u16 ? 2 : 4;
  const int span = max_dm_block_span(p, dblk);
  // samples of a staged row: the tile, the spread, the rounding of the stage base
  // (ring form: and the extra word the phase build reads past a chunk; packed
  // 4-bit phase loads: a spare word, which the odd nibble copies never fill)
  const int64_t rs = (int64_t)64 * ns + span + unit + (phase ? (u4 ? 8 : 0) : 16);
  if (rs > (1 << 23)) return fail(DD_ERR_RANGE, "delay spread too large");
  t->row_bytes = u16 ? round_up(2 * rs, 16) : phase && u4 ? round_up((rs + 1) / 2, 16) : round_up(rs, unit);
  int64_t lds;
  if (phase) {
    // LDS: kPhaseSlots slots of chan_block x copies, 1 KB load sink; a copy row
    // is loaded in at most `segs` 1 KB segments; entries are slot offsets
    lds = (int64_t)kPhaseSlots * chan_block * copies * t->row_bytes + 1024;
    if ((t->row_bytes + 1023) / 1024 > segs) return fail(DD_ERR_RANGE, "staged rows longer than the shape's loads");
    if ((int64_t)chan_block * copies * t->row_bytes > 65536)
      return fail(DD_ERR_RANGE, "staging slot too large for 16-bit LDS offsets");
  } else {
    // LDS: two buffers of the shifted copies, a ring of 3 raw slots (rows of raw
    // bytes + 16), 1 KB of scratch.  Loads per block: 1 KB segments of raw rows.
    const int raw = p.desc.dtype == DD_U4 ? t->row_bytes / 2 : t->row_bytes;
    lds = (int64_t)2 * chan_block * copies * t->row_bytes + (int64_t)3 * chan_block * (raw + 16) + 1024;
    if (chan_block * ((raw + 1023) / 1024) > 16) return fail(DD_ERR_RANGE, "too many staging segments");  // kStageSegs
    if ((int64_t)copies * t->row_bytes > 65536) return fail(DD_ERR_RANGE, "staged rows too long for 16-bit LDS offsets");
  }
  if (lds > lds_limit) return fail(DD_ERR_RANGE, "staged channel block exceeds LDS");
  t->chan_block = chan_block;
  t->segs = segs;
  t->lds_bytes = (int)lds;
  if (!fill) return DD_OK;
  const int n_dblk = (nd + dblk - 1) / dblk;
  const int ew = int_entry_words(dm_per_wave, segs);  // 32-bit words per channel
  const int ncp = (nc + chan_block - 1) / chan_block * chan_block;  // channels rounded up to whole blocks
  try {
    t->offs.assign((size_t)n_dblk * waves * ncp * ew, 0);
    t->sbase.assign((size_t)n_dblk * nc, 0);
  } catch (const std::bad_alloc &) {
    return fail(DD_ERR_NOMEM, "table allocation failed");
  }
  for (int b = 0; b < n_dblk; ++b) {
    const int32_t *s0 = p.shift.data() + (size_t)(b * dblk) * nc;
    int32_t *sb = t->sbase.data() + (size_t)b * nc;
    for (int c = 0; c < nc; ++c) sb[c] = s0[c] & ~(unit - 1);
    for (int w = 0; w < waves; ++w)
      for (int r = 0; r < dm_per_wave; ++r) {
        const int d = std::min(b * dblk + w * dm_per_wave + r, nd - 1);
        const int32_t *sd = p.shift.data() + (size_t)d * nc;
        uint32_t *o = t->offs.data() + (((size_t)b * waves + w) * ncp) * ew;
        for (int c = 0; c < ncp; ++c) {
          // window offset v (samples) inside the staged row -> byte offset of
          // its first word inside the channel's shifted copies; padding
          // channels (c >= nc, staged as zero rows) read their own row at 0
          const int32_t v = c < nc ? sd[c] - sb[c] : 0;
          const int32_t slot = phase ? (c % chan_block) * copies * t->row_bytes : 0;  // channel's copies in the slot
          const uint32_t e = u16             ? (uint32_t)(slot + (v & 1) * t->row_bytes + 2 * (v & ~1))
                             : phase && u4 ? (uint32_t)(slot + (v & 7) * t->row_bytes + 4 * (v >> 3))
                                           : (uint32_t)(slot + (v & 3) * t->row_bytes + (v & ~3));
          if (phase)
            o[(size_t)c * ew + r] = e;
          else
            o[(size_t)c * ew + (r >> 1)] |= e << (16 * (r & 1));
        }
      }
  }
  return DD_OK;
}

// Tables of the float kernel in direction `adjoint` for shape (ns, per_wave,
// waves, row_block); see FloatTables.
static dd_status build_float_tables(const dd_plan &p, bool adjoint, const int *shape, int lds_limit,
                                    FloatTables *t) {
  const int nc = p.desc.n_chan, nd = p.desc.n_dm;
  const int ns = shape[0], per_wave = shape[1], waves = shape[2], rb = shape[3];
  const int n_rows = adjoint ? nd : nc, n_out = adjoint ? nc : nd;
  const int oblk = waves * per_wave;
  const int n_oblk = (n_out + oblk - 1) / oblk;
  auto sh = [&](int o, int k) -> int32_t {
    return adjoint ? -p.shift[(size_t)k * nc + o] : p.shift[(size_t)o * nc + k];
  };
  // staging bases and the largest spread
  std::vector<int32_t> sbase;
  try {
    sbase.assign((size_t)n_oblk * n_rows, 0);
  } catch (const std::bad_alloc &) {
    return fail(DD_ERR_NOMEM, "table allocation failed");
  }
  int64_t span = 0;
  for (int b = 0; b < n_oblk; ++b)
    for (int k = 0; k < n_rows; ++k) {
      int32_t mn = INT32_MAX, mx = INT32_MIN;
      for (int o = b * oblk; o < std::min(n_out, (b + 1) * oblk); ++o) {
        const int32_t v = sh(o, k);
        mn = std::min(mn, v);
        mx = std::max(mx, v);
      }
      sbase[(size_t)b * n_rows + k] = mn & ~3;  // rounds toward minus infinity
      span = std::max<int64_t>(span, (int64_t)mx - mn);
    }
  const int64_t floats = ((int64_t)64 * ns + span + 4 + 3) / 4 * 4;
  if (floats * 4 > (1 << 24)) return fail(DD_ERR_RANGE, "delay spread too large");
  t->row_bytes = (int)(floats * 4);
  const int64_t lds = (int64_t)3 * rb * t->row_bytes + 1024;  // ring of 3 slots and a 1 KiB load sink
  if (lds > lds_limit) return fail(DD_ERR_RANGE, "staged row block exceeds LDS");
  if (rb * ((t->row_bytes + 1023) / 1024) > std::min(64, 16 * waves))  // the kernel's load segments per block
    return fail(DD_ERR_RANGE, "too many staging segments");
  if (t->row_bytes > 65536) return fail(DD_ERR_RANGE, "staged rows too long for 16-bit LDS offsets");
  t->ns = ns;
  t->per_wave = per_wave;
  t->waves = waves;
  t->row_block = rb;
  t->lds_bytes = (int)lds;
  const int rp = per_wave < 2 ? 2 : per_wave;
  const int nrp = (n_rows + rb - 1) / rb * rb;
  try {
    t->offs.assign((size_t)n_oblk * waves * nrp * rp, 0);
  } catch (const std::bad_alloc &) {
    return fail(DD_ERR_NOMEM, "table allocation failed");
  }
  for (int b = 0; b < n_oblk; ++b)
    for (int w = 0; w < waves; ++w)
      for (int r = 0; r < per_wave; ++r) {
        const int o = std::min(b * oblk + w * per_wave + r, n_out - 1);
        uint16_t *dst = t->offs.data() + (((size_t)b * waves + w) * nrp) * rp + r;
        for (int k = 0; k < n_rows; ++k)
          dst[(size_t)k * rp] = (uint16_t)(4 * (sh(o, k) - sbase[(size_t)b * n_rows + k]));
      }
  t->sbase = std::move(sbase);
  return DD_OK;
}

int num_shapes(const dd_plan &p) {
  return p.desc.dtype == DD_F32 ? kNumF32Shapes : kNumIntShapes + kNumDirectShapes;
}

dd_status set_tiles(dd_plan &p, int direction, int shape, int order) {
  if (direction != 0 && !(direction == 1 && p.desc.dtype == DD_F32))
    return fail(DD_ERR_ARG, "direction must be 0 (forward) or 1 (adjoint, float plans)");
  if (shape < 0 || shape >= num_shapes(p)) return fail(DD_ERR_ARG, "no such tile shape");
  if (order < 0 || order >= kNumOrders) return fail(DD_ERR_ARG, "no such workgroup order");
  TileCfg t;
  t.shape = shape;
  t.order = order;
  if (p.desc.dtype == DD_F32) {
    FloatTables ft;
    const dd_status st = build_float_tables(p, direction == 1, kF32Shapes[shape], kLdsLimit, &ft);
    if (st != DD_OK) return st;
    ft.shape = shape;
    ft.order = order;
    if (direction == 1) {
      p.ftab_adj = std::move(ft);
      return DD_OK;
    }
    t.ns = ft.ns;
    t.dm_per_wave = ft.per_wave;
    t.waves = ft.waves;
    t.chan_block = ft.row_block;
    t.row_bytes = ft.row_bytes;
    t.lds_bytes = ft.lds_bytes;
    p.ftab_fwd = std::move(ft);
    p.fwd = t;
    return DD_OK;
  }
  const int *k = int_shape(shape);
  IntTables tab;
  if (k[3] == 0) {  // direct-read kernel: no staging tables, any delay spread
    t.ns = k[0];
    t.dm_per_wave = k[1];
    t.waves = k[2];
    t.chan_block = 0;
    t.row_bytes = t.lds_bytes = 0;
    p.fwd = t;
    p.span_fwd = max_dm_block_span(p, t.waves * t.dm_per_wave);
    p.itab = IntTables();
    return DD_OK;
  }
  const dd_status st = build_int_tables(p, k[0], k[1], k[2], k[3], int_shape_segs(shape), kLdsLimit, &tab);
  if (st != DD_OK) return st;
  t.ns = k[0];
  t.dm_per_wave = k[1];
  t.waves = k[2];
  t.chan_block = k[3];
  t.segs = tab.segs;
  t.row_bytes = tab.row_bytes;
  t.lds_bytes = tab.lds_bytes;
  p.fwd = t;
  p.span_fwd = max_dm_block_span(p, t.waves * t.dm_per_wave);
  p.itab = std::move(tab);
  return DD_OK;
}

// Default tiles: the first compiled shape (they are listed fastest first; for
// 8-bit plans the phase-load shapes before the others, an 8-wave one
// only where two of its workgroups fit in a CU's LDS) that holds the plan's
// delay spread, in the grouped workgroup order (as fast as time tiles fastest
// on the headline plan, with a third of its L2 fetch traffic).
// For an integer plan whose spread leaves only LDS shapes staging 1 or 2
// channels at a time, the direct-read kernel is faster (measured: 12.7 against
// 8.5-10 Tadds/s at 264-395 samples of delay per DM step) and is chosen.
// 4-bit plans read directly whatever their spread: 2 rows x 8 waves, each XCD
// taking whole time tiles.  Its packed 16-byte windows and in-place nibble adds
// beat staging even on narrow spreads (8192 ch x 2^20 x 4000 DMs at 1200-1500
// MHz: 50.1 against 44.1 Tadds/s for the best staged shape, the phase-load
// form; 4096 ch x 2^19 x 2048 DMs at 120-190 MHz: 50.0 against 25.3 for the
// best staged shape; grid order 1 there against 46.2 for the grouped order).
dd_status choose_forward_tiles(dd_plan &p) {
  if (p.desc.dtype == DD_U4) return set_tiles(p, 0, kNumIntShapes + 1, kOrderXcdTiles);
  const int dirs = p.desc.dtype == DD_F32 ? 2 : 1;
  for (int dir = 0; dir < dirs; ++dir) {
    dd_status last = DD_ERR_RANGE;
    for (int pass = 0; pass < 2 && last != DD_OK && last != DD_ERR_NOMEM; ++pass)
      for (int i = 0; i < num_shapes(p); ++i) {
        const bool phase = p.desc.dtype == DD_U8 && int_shape_segs(i) > 0;
        if (phase != (pass == 0)) continue;
        last = set_tiles(p, dir, i, kOrderDmGroups);
        // an 8-wave phase-load shape pays only when two of its workgroups share a CU
        if (last == DD_OK && phase && p.fwd.waves == 8 && 2 * p.fwd.lds_bytes > kLdsLimit) last = DD_ERR_RANGE;
        if (last == DD_OK || last == DD_ERR_NOMEM) break;
      }
    if (last == DD_ERR_NOMEM) return last;
    if (last != DD_OK) return fail(DD_ERR_RANGE, "delay spread exceeds every compiled staging shape");
  }
  // Direct shape for 8- and 16-bit samples: 4 rows x 4 waves (4096 ch x 2^20 at 120-190 MHz,
  // DM step 0.5: 30.0 against 25.9 Tadds/s for 2 x 8 with 8-bit samples, 11.7 against 8.2 with
  // 16-bit), each XCD taking whole time tiles (on 4096-channel plans at 120-190, 300-400 and
  // 1200-1500 MHz: 8-bit 33.0-34.3 against 30.5-31.2 Tadds/s for the grouped order, 16-bit
  // 17.0-17.8 against 16.1-16.7), except 8-bit plans too wide for 4-channel stages, which
  // keep the grouped order (4096 ch x 2^20 at 120-190 MHz, DM step 0.5: 30.0 against 29.3).
  // An 8-bit plan reads directly when its staged shape holds at most 4 channels per stage: on
  // those four plans (staged shapes 16, 17, 18 and 5) 33.0-34.3 against 15.0-24.4 Tadds/s.
  const int direct = kNumIntShapes;
  if (p.desc.dtype == DD_U8 && !is_direct(p.fwd) && p.fwd.chan_block <= 4)
    return set_tiles(p, 0, direct, p.fwd.chan_block <= 2 ? kOrderDmGroups : kOrderXcdTiles);
  // 16-bit plans: the 8-wave shape with 4 rows per wave and 4 channels per stage,
  // where two of its workgroups fit in a CU's LDS, so that one's barrier waits
  // overlap the other's adds: first in its phase-load form (the two copies loaded
  // straight into LDS: 1111.5 against 1326.9 ms on 8192 ch x 2^20 x 4000 DMs),
  // else in its raw-ring form (13-16% faster than the 16-wave default on 8192 x
  // 2^20 and on binned 4096-channel ranges; 11% slower on a plan with ~1000
  // samples of spread per 32 DMs, where only one fits).  Otherwise a plan left
  // with at most 4 channels per stage reads directly (4096-channel plans whose
  // staged shape was the 1-row, 16-wave raw ring: 17.0-17.8 against 14.6-15.1
  // Tadds/s), as does one with at most 2.
  if (p.desc.dtype == DD_U16 && !is_direct(p.fwd)) {
    if (p.fwd.chan_block <= 2) return set_tiles(p, 0, direct, kOrderXcdTiles);
    const int keep_shape = p.fwd.shape, keep_order = p.fwd.order;
    bool moved = false;
    for (int want_phase = 1; want_phase >= 0; --want_phase)
      for (int i = 0; i < kNumIntShapes; ++i) {
        const int *k = kIntShapes[i];
        if (k[0] != 16 || k[1] != 4 || k[2] != 8 || k[3] != 4 || (k[4] > 0) != (want_phase == 1)) continue;
        if (i == keep_shape) return moved ? set_tiles(p, 0, keep_shape, keep_order) : DD_OK;
        const dd_status st = set_tiles(p, 0, i, kOrderDmGroups);
        if (st == DD_ERR_NOMEM) return st;
        if (st == DD_OK && 2 * p.fwd.lds_bytes <= kLdsLimit) return DD_OK;
        moved = moved || st == DD_OK;
        break;
      }
    if (moved) {
      const dd_status st = set_tiles(p, 0, keep_shape, keep_order);
      if (st != DD_OK) return st;
    }
    if (p.fwd.chan_block <= 4) return set_tiles(p, 0, direct, kOrderXcdTiles);
  }
  return DD_OK;
}

static size_t up256(size_t v) { return (v + 255) / 256 * 256; }

// Device workspace layout.  Integer plans: [offs words][sbase int32].
// Float plans: [forward offs][forward sbase][adjoint offs][adjoint sbase].
TableLayout table_layout(const dd_plan &p) {
  TableLayout L;
  if (p.desc.dtype != DD_F32) {
    if (!is_direct(p.fwd)) L.int_sbase = up256(p.itab.offs.size() * sizeof(uint32_t));
    return L;
  }
  size_t off = 0;
  const FloatTables *tabs[2] = {&p.ftab_fwd, &p.ftab_adj};
  for (int k = 0; k < 2; ++k) {
    L.f_offs[k] = off;
    off += up256(tabs[k]->offs.size() * 2);
    L.f_sbase[k] = off;
    off += up256(tabs[k]->sbase.size() * 4);
  }
  return L;
}

size_t table_bytes(const dd_plan &p) {
  if (p.desc.dtype != DD_F32 && is_direct(p.fwd)) return up256(p.shift.size() * sizeof(int32_t));
  if (p.desc.dtype != DD_F32)
    return up256(p.itab.offs.size() * sizeof(uint32_t)) + up256(p.itab.sbase.size() * sizeof(int32_t));
  return up256(p.ftab_fwd.offs.size() * 2) + up256(p.ftab_fwd.sbase.size() * 4) + up256(p.ftab_adj.offs.size() * 2) +
         up256(p.ftab_adj.sbase.size() * 4);
}

// Table sizes follow the layouts of build_int_tables / build_float_tables
// (offs: per output block, wave and padded row, `entry_bytes` bytes of
// entries; sbase: per output block and row, one int32).
static size_t shape_table_bytes(int64_t n_out, int64_t n_rows, const int *k, int64_t entry_bytes) {
  const int64_t per_wave = k[1], waves = k[2], rb = k[3];
  const int64_t n_oblk = (n_out + waves * per_wave - 1) / (waves * per_wave);
  const int64_t rows_pad = (n_rows + rb - 1) / rb * rb;
  return up256((size_t)(n_oblk * waves * rows_pad * entry_bytes)) + up256((size_t)(n_oblk * n_rows * 4));
}

size_t tune_table_bytes(const dd_plan &p) {
  const int64_t nc = p.desc.n_chan, nd = p.desc.n_dm;
  size_t fwd = 0, adj = 0;
  if (p.desc.dtype != DD_F32) {
    for (int i = 0; i < kNumIntShapes; ++i)
      fwd = std::max(fwd, shape_table_bytes(nd, nc, kIntShapes[i], 4 * int_entry_words(kIntShapes[i][1], kIntShapes[i][4])));
    return std::max(fwd, up256((size_t)nd * (size_t)nc * sizeof(int32_t)));  // direct shapes: the shift table
  }
  for (int i = 0; i < kNumF32Shapes; ++i) {
    const int64_t eb = 2 * std::max(kF32Shapes[i][1], 2);  // max(per_wave, 2) uint16 entries
    fwd = std::max(fwd, shape_table_bytes(nd, nc, kF32Shapes[i], eb));
    adj = std::max(adj, shape_table_bytes(nc, nd, kF32Shapes[i], eb));
  }
  return fwd + adj;
}

}  // namespace dd
