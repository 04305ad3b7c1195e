// Internal declarations shared by the host plan code, the C ABI and the kernels.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dd.h"

namespace dd {

// Thread-local error detail; returns the status for chaining.
dd_status fail(dd_status st, const std::string &msg);

// Tile shape of the forward kernels.  A workgroup covers `waves * dm_per_wave`
// DM rows and `64 * ns` output samples; each lane owns `ns` consecutive samples
// of `dm_per_wave` rows.  Channels are staged `chan_block` at a time into LDS
// rows of `row_bytes` bytes (unpacked samples).
struct TileCfg {
  int shape = 0;         // index into kIntShapes / kF32Shapes
  int order = 0;         // workgroup order, a TileOrder
  int ns = 32;           // samples per lane (16 or 32)
  int dm_per_wave = 4;   // DM rows per wave
  int waves = 4;         // waves per workgroup
  int chan_block = 16;   // channels per LDS stage
  int segs = 0;          // 8-bit phase-load staging: 1 KiB load segments per copy row; 0 = raw ring + phase build
  int row_bytes = 0;     // LDS bytes per staged channel row
  int lds_bytes = 0;     // total dynamic LDS
};

// Order of the workgroups of a 1-D grid over (time tile, output block) pairs.
// Workgroup w runs on XCD w % 8 (round-robin dispatch).
enum TileOrder {
  kOrderTimeFirst = 0,  // consecutive workgroups take consecutive time tiles of one output block
  kOrderXcdTiles = 1,   // each XCD takes whole time tiles, every output block of a tile in turn
  kOrderDmGroups = 2,   // each XCD takes its time tiles for 4 output blocks at a time (tile_order.h)
  kOrderXcdRuns = 3,    // each XCD takes a contiguous run of time tiles, time tiles fastest
  kNumOrders = 4
};

// Device tables of the integer forward kernel for one tile shape: per DM
// block the staging base of every channel (its first-DM delay rounded down to
// the staging unit) and, per (block, wave, channel, row), the LDS byte offset
// of the window's first word as uint16 (inside the channel's shifted copies
// for the ring form, from the start of the staging slot for the phase-load form).
// Entries are 32-bit words: raw-ring shapes pack two uint16 entries per word
// (row r at bits 16 * (r % 2) of word r / 2); phase-load shapes hold one
// entry per word (the byte offset from the staging slot's start).
inline int int_entry_words(int dm_per_wave, int segs) {
  return segs > 0 ? dm_per_wave : (dm_per_wave < 2 ? 2 : dm_per_wave) / 2;
}
struct IntTables {
  std::vector<uint32_t> offs;  // [n_dblk][waves][n_chan rounded up to chan_block][int_entry_words]
  std::vector<int32_t> sbase;  // [n_dblk][n_chan]
  int row_bytes = 0, chan_block = 0, segs = 0, lds_bytes = 0;
};
// Tables of the float kernel (forward or adjoint) for one tile shape.  The
// kernel sums staged rows k (channels forward, DM rows adjoint) into outputs o
// (DM rows forward, channels adjoint) at delay sh(o, k) = +shift (forward) or
// -shift (adjoint).  Per output block: sbase = the block's smallest sh of row
// k rounded down to 4 floats; per (block, wave, row, output of the wave): the
// LDS byte offset 4 * (sh - sbase) of the window in the staged row.
struct FloatTables {
  int shape = 0, order = 0;  // index into kF32Shapes, TileOrder
  int ns = 0, per_wave = 0, waves = 0, row_block = 0;
  int row_bytes = 0, lds_bytes = 0;
  std::vector<uint16_t> offs;  // [n_oblk][waves][n_rows rounded up to row_block][max(per_wave, 2)]
  std::vector<int32_t> sbase;  // [n_oblk][n_rows]
};

}  // namespace dd

struct dd_plan {
  dd_plan_desc desc{};
  std::vector<double> freqs;   // explicit frequencies (empty = uniform)
  std::vector<int32_t> shift;  // [n_dm][n_chan]
  int64_t n_out = 0;
  int32_t max_shift = 0;
  int64_t in_pitch_bytes = 0;
  dd::TileCfg fwd;             // forward tile shape
  int32_t span_fwd = 0;        // largest delay spread inside a forward DM block
  dd::IntTables itab;          // integer plans: forward kernel tables
  dd::FloatTables ftab_fwd;    // float plans: forward kernel tables
  dd::FloatTables ftab_adj;    // float plans: adjoint kernel tables
  // binding
  const void *d_tables = nullptr;
  int device = -1;
  bool bound = false;
};

namespace dd {

// Host plan helpers (plan.cpp).
dd_status build_shift_table(dd_plan &p);
int32_t max_dm_block_span(const dd_plan &p, int dm_block);
dd_status choose_forward_tiles(dd_plan &p);
// Rebuild the tables of one direction (0 forward, 1 adjoint) for compiled
// shape `shape` and TileOrder `order`.  DD_ERR_RANGE if the shape cannot hold
// the plan's delay spread; the plan is unchanged then.
dd_status set_tiles(dd_plan &p, int direction, int shape, int order);
int num_shapes(const dd_plan &p);
size_t table_bytes(const dd_plan &p);
// Byte offsets of the plan's current tables inside a table workspace of
// table_bytes(p) bytes.  Integer plans: [offs words][sbase int32] (direct-read
// shapes: the plain int32 shift table at 0).  Float plans: [forward offs]
// [forward sbase][adjoint offs][adjoint sbase].  Each part starts on 256 bytes.
struct TableLayout {
  size_t int_offs = 0, int_sbase = 0;
  size_t f_offs[2] = {0, 0}, f_sbase[2] = {0, 0};  // [forward, adjoint]
};
TableLayout table_layout(const dd_plan &p);
// Enqueue the copy of the plan's current tables into device memory `dst` (at
// least table_bytes(p) bytes) on `stream`.  Returns a hipError_t as int.
int copy_tables(const dd_plan &p, void *dst, void *stream);
// Enqueue the upload of the current tables into `ws` and mark the plan bound (api.cpp).
dd_status upload_tables(dd_plan &p, void *ws, void *stream);
dd_status hip_error(int e, const char *what);
// Apply tile choices recorded in the tuning cache file, if any (tune.cpp).
void apply_tune_cache(dd_plan &p);
// Upper bound of table_bytes over every shape set_tiles can choose.
size_t tune_table_bytes(const dd_plan &p);

// One beam of a batch, as the persistent kernel sees it.
struct BeamDesc {
  const uint8_t *x;
  const uint32_t *offs;
  const int32_t *sbase;
  float *out;
  int64_t pitch, n_samp, n_out, out_pitch;
  int64_t item_begin;  // first work item of this beam
  int32_t n_chan, n_dm, row_bytes, chan_block, tiles_t, tiles_d;
};

// Tables of the integer forward kernel for one staged shape; with fill false
// only the size checks run and t gets row_bytes / lds_bytes (no tables).
dd_status build_int_tables(const dd_plan &p, int ns, int dm_per_wave, int waves, int chan_block, int segs,
                           int lds_limit, IntTables *t, bool fill = true);

// Epilogue modes of the integer forward kernels for 16-bit input.  A sum of
// values up to 2^24 (binned 16-bit samples) is computed exactly from two
// 16-bit planes, the values' low and high halves: the low plane's launch keeps
// its exact 32-bit totals in the output buffer (kOutRawTotals), the high
// plane's launch reads them back and writes low + 2^16 * high, converted to
// float32 once (kOutCombineHigh).
enum OutMode { kOutFloat = 0, kOutRawTotals = 1, kOutCombineHigh = 2 };

// Kernel launchers (fwd_int.hip, kernels_f32.hip).  Return hipError_t as int.
// `tables` is the device copy of the plan's current tables (table_layout), the
// plan's bound workspace or any other copy.  `out_limit` > 0 computes only the
// first out_limit output samples of every output row (shorter launches for
// tile tuning); <= 0 computes all.  `out_mode` other than kOutFloat is valid
// for DD_U16 plans only.
int launch_forward_int(const dd_plan &p, const void *tables, const void *d_in, float *d_out, int64_t out_pitch,
                       void *stream, int64_t out_limit = 0, int out_mode = kOutFloat);
int launch_forward_f32(const dd_plan &p, const void *tables, const void *d_in, float *d_out, int64_t out_pitch,
                       void *stream, int64_t out_limit = 0);
// Float tile shapes compiled into the library: (ns, per_wave, waves, row_block).
extern const int kF32Shapes[][4];
extern const int kNumF32Shapes;
// Integer tile shapes compiled into the library: (ns, dm_per_wave, waves,
// chan_block, segs), in the order plans try them; segs > 0 marks the 8-bit
// phase-load staging form with copy rows of at most segs KiB.
extern const int kIntShapes[][5];
extern const int kNumIntShapes;
// Direct-read shapes (fwd_direct.hip): (16, dm_per_wave, waves, 0).  An integer
// plan's shape index s >= kNumIntShapes names kDirectShapes[s - kNumIntShapes];
// such a plan's tables are its plain shift table.
extern const int kDirectShapes[][4];
extern const int kNumDirectShapes;
inline const int *int_shape(int s) { return s < kNumIntShapes ? kIntShapes[s] : kDirectShapes[s - kNumIntShapes]; }
inline int int_shape_segs(int s) { return s < kNumIntShapes ? kIntShapes[s][4] : 0; }
// Staging slots of the phase-load form (its LDS ring depth).
constexpr int kPhaseSlots = 3;
inline bool is_direct(const TileCfg &t) { return t.chan_block == 0; }
int launch_forward_direct(const dd_plan &p, const void *tables, const void *d_in, float *d_out, int64_t out_pitch,
                          void *stream, int64_t out_limit = 0, int out_mode = kOutFloat);
int launch_adjoint(const dd_plan &p, const void *tables, const float *d_y, int64_t y_pitch, float *d_grad,
                   void *stream, int64_t out_limit = 0);

// Persistent batched forward: kernel entry, its launch geometry and the
// counter-reset kernel, for recording into a graph.
struct BatchLaunch {
  const void *reset_fn;
  const void *main_fn;
  int grid, block, lds_bytes;
};
int batch_kernels(int ns, int dm_per_wave, int waves, int chan_block, int segs, int dtype, int lds_bytes,
                  BatchLaunch *out);
// The same for a direct-read shape (fwd_direct.hip); its work items are time
// tiles of direct_tile_samples(dtype) outputs by DM blocks of waves x
// dm_per_wave rows, and a beam's table is its plain int32 shift table.
int batch_direct_kernels(int dm_per_wave, int waves, int dtype, BatchLaunch *out);
int direct_tile_samples(int dtype);

// Time binning (bin.hip): bytes per output element, and the launch.  The
// caller has validated every argument (sizes, alignment, factor 1..256).
int bin_out_bytes(int dtype);
int launch_bin(int dtype, const void *in, int64_t in_pitch, int n_chan, int64_t n_samp, int factor, void *out,
               int64_t out_pitch, void *stream);
// 16-bit input binned into low- and high-half uint16 planes (the high plane
// `hi_off` bytes after the low one in every output row), for exact binned sums.
int launch_bin_u16_split(const void *in, int64_t in_pitch, int n_chan, int64_t n_samp, int factor, void *out,
                         int64_t out_pitch, int64_t hi_off, void *stream);
// Corner turn (corner.hip), arguments validated by the caller.
int launch_corner_turn(int dtype, const void *in, int64_t in_pitch, int n_chan, int64_t n_samp, void *out,
                       int64_t out_pitch, void *stream);

}  // namespace dd
