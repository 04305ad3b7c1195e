// Input corner turn, time binning and multi-range DM plans ("surveys"): the C
// ABI of the corner-turn and binning kernels, and a survey object that turns
// the input (if it arrives time-major), bins it once per factor and runs one
// ordinary plan per DM range.  Declarations and contracts are in include/dd.h.
#include <hip/hip_runtime.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "dd_internal.h"

struct dd_survey {
  int32_t n_chan = 0;
  int64_t n_samp = 0;
  int32_t dtype = 0;
  int64_t in_pitch = 0;        // channel-major rows the binning and unbinned ranges read
  bool time_major = false;     // input arrives as spectra; turned into the copy at turn_off
  int64_t spectrum_pitch = 0;  // bytes between input spectra (time-major input)
  size_t turn_off = 0;
  std::vector<dd_range> ranges;
  std::vector<dd_plan *> plans;     // one per range, owned
  std::vector<int> slot_factor;     // distinct binning factors > 1, in first-use order
  std::vector<int64_t> slot_pitch;  // bytes per binned row
  // 16-bit input: every binned copy holds two uint16 planes per row, the low
  // and the high halves of the exact bin sums, the high one split_off[k] bytes
  // after the low one; the range's plan is a 16-bit plan over the low plane
  bool split16 = false;
  std::vector<int64_t> split_off;
  std::vector<size_t> slot_off;     // workspace offset of each binned copy
  std::vector<int> range_slot;      // per range: its binned copy, or -1 for the input itself
  std::vector<size_t> tab_off, tab_bytes;  // per range: its tables in the workspace
  size_t ws_bytes = 0;
  // binding
  uint8_t *ws = nullptr;
  int device = -1;
  bool bound = false;

  ~dd_survey() {
    for (dd_plan *p : plans) dd_plan_destroy(p);
  }
};

namespace dd {
namespace {

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int64_t input_row_bytes(int dtype, int64_t n_samp) {
  switch (dtype) {
    case DD_U8: return n_samp;
    case DD_U4: return (n_samp + 1) / 2;
    case DD_U16: return 2 * n_samp;
    case DD_F32: return 4 * n_samp;
  }
  return -1;
}

bool valid_dtype(int dtype) { return dtype == DD_U8 || dtype == DD_U4 || dtype == DD_U16 || dtype == DD_F32; }

int64_t spectrum_bytes(int dtype, int32_t n_chan) {
  return dtype == DD_U4 ? ((int64_t)n_chan + 1) / 2 : input_row_bytes(dtype, 1) * n_chan;
}

bool overlap(const void *a, int64_t na, const void *b, int64_t nb) {
  const uintptr_t a0 = (uintptr_t)a, a1 = a0 + (uintptr_t)na, b0 = (uintptr_t)b, b1 = b0 + (uintptr_t)nb;
  return a0 < b1 && b0 < a1;
}

// The channel-major input: the caller's, or the turned copy.
const void *rows_input(const dd_survey &s, const void *d_in) {
  return s.time_major ? (const void *)(s.ws + s.turn_off) : d_in;
}

// Input sources of every range: the channel-major input or a binned copy.
const void *range_input(const dd_survey &s, int r, const void *d_in) {
  const int slot = s.range_slot[r];
  return slot < 0 ? rows_input(s, d_in) : (const void *)(s.ws + s.slot_off[slot]);
}

dd_status check_survey_exec(const dd_survey *s, const void *d_in, float *const *d_out, const int64_t *out_pitch) {
  if (!s || !d_in || !d_out || !out_pitch) return fail(DD_ERR_ARG, "null argument");
  if (!s->bound) return fail(DD_ERR_NOT_BOUND, "survey is not bound to device workspace");
  int dev = -1;
  if (hipGetDevice(&dev) == hipSuccess && dev != s->device) return fail(DD_ERR_ARG, "survey is bound on another device");
  if (!aligned16(d_in)) return fail(DD_ERR_ALIGN, "input must be 16-byte aligned");
  if (s->time_major && overlap(d_in, s->spectrum_pitch * s->n_samp, s->ws, (int64_t)s->ws_bytes))
    return fail(DD_ERR_ARG, "input overlaps the survey workspace");
  for (size_t r = 0; r < s->plans.size(); ++r) {
    const dd_plan &p = *s->plans[r];
    if (!p.bound) return fail(DD_ERR_NOT_BOUND, "range " + std::to_string(r) + " was re-tiled: bind the survey again");
    if (!d_out[r]) return fail(DD_ERR_ARG, "null output of range " + std::to_string(r));
    if (!aligned16(d_out[r])) return fail(DD_ERR_ALIGN, "outputs must be 16-byte aligned");
    if (out_pitch[r] < p.n_out) return fail(DD_ERR_ARG, "out_pitch < n_out for range " + std::to_string(r));
    if (out_pitch[r] % 4) return fail(DD_ERR_ALIGN, "out_pitch must be a multiple of 4 elements");
  }
  return DD_OK;
}

// Corner turn (time-major input) and binning, in that order, on `stream`.
dd_status prepare_inputs(const dd_survey &s, const void *d_in, void *stream) {
  if (s.time_major) {
    const int e = launch_corner_turn(s.dtype, d_in, s.spectrum_pitch, s.n_chan, s.n_samp, s.ws + s.turn_off,
                                     s.in_pitch, stream);
    if (e) return hip_error(e, "corner-turn launch");
  }
  const void *rows = rows_input(s, d_in);
  for (size_t k = 0; k < s.slot_factor.size(); ++k) {
    const int e = s.split16 ? launch_bin_u16_split(rows, s.in_pitch, s.n_chan, s.n_samp, s.slot_factor[k],
                                                   s.ws + s.slot_off[k], s.slot_pitch[k], s.split_off[k], stream)
                            : launch_bin(s.dtype, rows, s.in_pitch, s.n_chan, s.n_samp, s.slot_factor[k],
                                         s.ws + s.slot_off[k], s.slot_pitch[k], stream);
    if (e) return hip_error(e, "binning launch");
  }
  return DD_OK;
}

// Forward transform of range r into d_out.  A binned range of 16-bit input
// sums its low-half plane exactly into raw 32-bit totals, then its high-half
// plane, combining both into the float32 of the exact sum.
dd_status range_forward(const dd_survey &s, int r, const void *d_in, float *d_out, int64_t out_pitch, void *stream) {
  const int slot = s.range_slot[r];
  if (!s.split16 || slot < 0) return dd_execute(s.plans[r], range_input(s, r, d_in), d_out, out_pitch, stream);
  const uint8_t *lo = s.ws + s.slot_off[slot];
  const dd_plan &p = *s.plans[r];
  int e = launch_forward_int(p, p.d_tables, lo, d_out, out_pitch, stream, 0, kOutRawTotals);
  if (!e) e = launch_forward_int(p, p.d_tables, lo + s.split_off[slot], d_out, out_pitch, stream, 0, kOutCombineHigh);
  if (e) return hip_error(e, "forward launch");
  return DD_OK;
}

}  // namespace
}  // namespace dd

using namespace dd;

extern "C" {

int32_t dd_bin_out_dtype(int32_t dtype) {
  if (dtype == DD_U8 || dtype == DD_U4) return DD_U16;
  if (dtype == DD_U16 || dtype == DD_F32) return DD_F32;
  return 0;
}

dd_status dd_bin_time(int32_t dtype, const void *d_in, int64_t in_pitch, int32_t n_chan, int64_t n_samp,
                      int32_t factor, void *d_out, int64_t out_pitch, void *stream) {
  if (!valid_dtype(dtype)) return fail(DD_ERR_ARG, "unknown dtype");
  if (!d_in || !d_out) return fail(DD_ERR_ARG, "null buffer");
  if (n_chan <= 0 || n_samp <= 0) return fail(DD_ERR_ARG, "n_chan and n_samp must be positive");
  if (factor < 1 || factor > 256) return fail(DD_ERR_ARG, "factor must be in 1..256");
  if (n_samp >= ((int64_t)1 << 40)) return fail(DD_ERR_RANGE, "n_samp must be below 2^40");
  const int64_t n_bins = n_samp / factor;
  if (n_bins == 0) return fail(DD_ERR_TOO_SHORT, "n_samp < factor: no whole bin");
  if (!aligned16(d_in) || !aligned16(d_out)) return fail(DD_ERR_ALIGN, "buffers must be 16-byte aligned");
  if (in_pitch < input_row_bytes(dtype, n_samp)) return fail(DD_ERR_ARG, "in_pitch_bytes smaller than one row");
  if (out_pitch < n_bins * bin_out_bytes(dtype)) return fail(DD_ERR_ARG, "out_pitch_bytes smaller than one binned row");
  if (in_pitch % 16 || out_pitch % 16) return fail(DD_ERR_ALIGN, "row pitches must be multiples of 16 bytes");
  if ((double)in_pitch * n_chan > 9.0e18 || (double)out_pitch * n_chan > 9.0e18) return fail(DD_ERR_RANGE, "size overflow");
  if (overlap(d_in, in_pitch * n_chan, d_out, out_pitch * n_chan)) return fail(DD_ERR_ARG, "input and output overlap");
  const int e = launch_bin(dtype, d_in, in_pitch, n_chan, n_samp, factor, d_out, out_pitch, stream);
  if (e) return hip_error(e, "binning launch");
  return DD_OK;
}

dd_status dd_corner_turn(int32_t dtype, const void *d_in, int64_t in_pitch, int32_t n_chan, int64_t n_samp,
                         void *d_out, int64_t out_pitch, void *stream) {
  if (!valid_dtype(dtype)) return fail(DD_ERR_ARG, "unknown dtype");
  if (!d_in || !d_out) return fail(DD_ERR_ARG, "null buffer");
  if (n_chan <= 0 || n_samp <= 0) return fail(DD_ERR_ARG, "n_chan and n_samp must be positive");
  if (dtype == DD_U4 && (n_samp & 1)) return fail(DD_ERR_ARG, "n_samp must be even for 4-bit rows");
  if (n_samp >= ((int64_t)1 << 36)) return fail(DD_ERR_RANGE, "n_samp must be below 2^36");
  if (!aligned16(d_in) || !aligned16(d_out)) return fail(DD_ERR_ALIGN, "buffers must be 16-byte aligned");
  if (in_pitch < spectrum_bytes(dtype, n_chan)) return fail(DD_ERR_ARG, "in_pitch_bytes smaller than one spectrum");
  if (out_pitch < input_row_bytes(dtype, n_samp)) return fail(DD_ERR_ARG, "out_pitch_bytes smaller than one row");
  if (in_pitch % 16 || out_pitch % 16) return fail(DD_ERR_ALIGN, "pitches must be multiples of 16 bytes");
  if ((double)in_pitch * n_samp > 9.0e18 || (double)out_pitch * n_chan > 9.0e18) return fail(DD_ERR_RANGE, "size overflow");
  if (overlap(d_in, in_pitch * n_samp, d_out, out_pitch * n_chan)) return fail(DD_ERR_ARG, "input and output overlap");
  {  // one workgroup per tile of (256 bytes of a spectrum) x (128 bytes of a row)
    const int64_t tc = dtype == DD_U4 ? 256 : 256 / input_row_bytes(dtype, 1);
    const int64_t tt = dtype == DD_U4 ? 256 : 128 / input_row_bytes(dtype, 1);
    if (((int64_t)n_chan + tc - 1) / tc * ((n_samp + tt - 1) / tt) > 0x7fffffff)
      return fail(DD_ERR_RANGE, "too many tiles for one launch");
  }
  const int e = launch_corner_turn(dtype, d_in, in_pitch, n_chan, n_samp, d_out, out_pitch, stream);
  if (e) return hip_error(e, "corner-turn launch");
  return DD_OK;
}

dd_status dd_survey_create(const dd_plan_desc *base, const dd_range *ranges, int32_t n_ranges, int32_t flags,
                           dd_survey **out) {
  if (!base || !ranges || !out) return fail(DD_ERR_ARG, "null argument");
  *out = nullptr;
  if (n_ranges <= 0) return fail(DD_ERR_ARG, "a survey needs at least one range");
  if (flags & ~DD_SURVEY_TIME_MAJOR) return fail(DD_ERR_ARG, "unknown survey flags");
  if (!valid_dtype(base->dtype)) return fail(DD_ERR_ARG, "unknown dtype");
  if (base->n_chan <= 0 || base->n_samp <= 0) return fail(DD_ERR_ARG, "n_chan and n_samp must be positive");
  const bool time_major = (flags & DD_SURVEY_TIME_MAJOR) != 0;
  const int64_t row = input_row_bytes(base->dtype, base->n_samp);
  int64_t pitch, spitch = 0;
  if (time_major) {
    // the caller's pitch is between spectra; the turned copy gets 256-byte rows
    const int64_t sb = spectrum_bytes(base->dtype, base->n_chan);
    spitch = base->in_pitch_bytes ? base->in_pitch_bytes : sb;
    if (spitch < sb) return fail(DD_ERR_ARG, "in_pitch_bytes smaller than one spectrum");
    if (spitch % 16) return fail(DD_ERR_ALIGN, "spectrum pitch must be a multiple of 16 bytes");
    if (base->dtype == DD_U4 && (base->n_samp & 1)) return fail(DD_ERR_ARG, "n_samp must be even for 4-bit input");
    pitch = (int64_t)round_up((size_t)row, 256);
  } else {
    pitch = base->in_pitch_bytes ? base->in_pitch_bytes : row;
    if (pitch < row) return fail(DD_ERR_ARG, "in_pitch_bytes smaller than one row");
    if (pitch % 16) return fail(DD_ERR_ALIGN, "input row pitch must be a multiple of 16 bytes");
  }
  for (int r = 0; r < n_ranges; ++r) {
    if (ranges[r].bin < 1 || ranges[r].bin > 256) return fail(DD_ERR_ARG, "range " + std::to_string(r) + ": bin must be in 1..256");
    if (base->n_samp / ranges[r].bin == 0) return fail(DD_ERR_TOO_SHORT, "range " + std::to_string(r) + ": no whole bin");
  }

  dd_survey *s = new (std::nothrow) dd_survey();
  if (!s) return fail(DD_ERR_NOMEM, "survey allocation failed");
  try {
    s->n_chan = base->n_chan;
    s->n_samp = base->n_samp;
    s->dtype = base->dtype;
    s->in_pitch = pitch;
    s->time_major = time_major;
    s->spectrum_pitch = spitch;
    s->ranges.assign(ranges, ranges + n_ranges);
    s->split16 = base->dtype == DD_U16;
    const int ob = s->split16 ? 2 : bin_out_bytes(base->dtype);
    size_t off = 0;
    if (time_major) {
      s->turn_off = 0;
      off = round_up((size_t)pitch * (size_t)base->n_chan, 256);
    }
    for (int r = 0; r < n_ranges; ++r) {
      const int f = ranges[r].bin;
      int slot = -1;
      if (f > 1) {
        for (size_t k = 0; k < s->slot_factor.size(); ++k)
          if (s->slot_factor[k] == f) slot = (int)k;
        if (slot < 0) {
          slot = (int)s->slot_factor.size();
          const int64_t plane = (int64_t)round_up((size_t)(base->n_samp / f) * ob, 256);
          const int64_t bp = s->split16 ? 2 * plane : plane;  // split rows: low plane, then high plane
          s->slot_factor.push_back(f);
          s->slot_pitch.push_back(bp);
          s->split_off.push_back(s->split16 ? plane : 0);
          s->slot_off.push_back(off);
          off += round_up((size_t)bp * (size_t)base->n_chan, 256);
        }
      }
      s->range_slot.push_back(slot);
      dd_plan_desc d = *base;
      d.dm_start = ranges[r].dm_start;
      d.dm_step = ranges[r].dm_step;
      d.n_dm = ranges[r].n_dm;
      if (f > 1) {
        d.dtype = s->split16 ? DD_U16 : dd_bin_out_dtype(base->dtype);
        d.n_samp = base->n_samp / f;
        d.t_samp_s = base->t_samp_s * f;
        d.in_pitch_bytes = s->slot_pitch[slot];
      } else {
        d.in_pitch_bytes = pitch;
      }
      dd_plan *p = nullptr;
      const dd_status st = dd_plan_create(&d, &p);
      if (st != DD_OK) {
        const std::string msg = "range " + std::to_string(r) + ": " + dd_last_error();
        delete s;
        return fail(st, msg);
      }
      s->plans.push_back(p);
    }
    for (dd_plan *p : s->plans) {
      const size_t tb = round_up(tune_table_bytes(*p), 256);
      s->tab_off.push_back(off);
      s->tab_bytes.push_back(tb);
      off += tb;
    }
    s->ws_bytes = off;
  } catch (const std::bad_alloc &) {
    delete s;
    return fail(DD_ERR_NOMEM, "survey allocation failed");
  }
  *out = s;
  return DD_OK;
}

dd_status dd_survey_plan(const dd_survey *s, int32_t r, dd_plan **plan) {
  if (!s || !plan) return fail(DD_ERR_ARG, "null argument");
  if (r < 0 || r >= (int32_t)s->plans.size()) return fail(DD_ERR_ARG, "range index out of range");
  *plan = s->plans[r];
  return DD_OK;
}

dd_status dd_survey_workspace_bytes(const dd_survey *s, size_t *bytes) {
  if (!s || !bytes) return fail(DD_ERR_ARG, "null argument");
  *bytes = s->ws_bytes;
  return DD_OK;
}

dd_status dd_survey_bind(dd_survey *s, void *ws, size_t bytes, void *stream) {
  if (!s || !ws) return fail(DD_ERR_ARG, "null argument");
  if (!aligned16(ws)) return fail(DD_ERR_ALIGN, "workspace must be 16-byte aligned");
  if (bytes < s->ws_bytes) return fail(DD_ERR_ARG, "workspace smaller than dd_survey_workspace_bytes");
  s->bound = false;
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "hipGetDevice");
  for (size_t r = 0; r < s->plans.size(); ++r) {
    const dd_status st = dd_plan_bind(s->plans[r], (uint8_t *)ws + s->tab_off[r], s->tab_bytes[r], stream);
    if (st != DD_OK) return st;
  }
  s->ws = (uint8_t *)ws;
  s->device = dev;
  s->bound = true;
  return DD_OK;
}

dd_status dd_survey_autotune(dd_survey *s, const void *d_in, float *const *d_out, const int64_t *out_pitch,
                             void *stream) {
  dd_status st = check_survey_exec(s, d_in, d_out, out_pitch);
  if (st != DD_OK) return st;
  st = prepare_inputs(*s, d_in, stream);
  for (size_t r = 0; r < s->plans.size() && st == DD_OK; ++r)
    st = dd_plan_autotune(s->plans[r], 0, range_input(*s, (int)r, d_in), d_out[r], out_pitch[r], s->ws + s->tab_off[r],
                          s->tab_bytes[r], stream, nullptr);
  return st;
}

dd_status dd_survey_execute(const dd_survey *s, const void *d_in, float *const *d_out, const int64_t *out_pitch,
                            void *stream) {
  dd_status st = check_survey_exec(s, d_in, d_out, out_pitch);
  if (st != DD_OK) return st;
  st = prepare_inputs(*s, d_in, stream);
  for (size_t r = 0; r < s->plans.size() && st == DD_OK; ++r)
    st = range_forward(*s, (int)r, d_in, d_out[r], out_pitch[r], stream);
  return st;
}

void dd_survey_destroy(dd_survey *s) { delete s; }

}  // extern "C"
