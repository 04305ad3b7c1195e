// Float forward and adjoint dedispersion kernels for gfx950 (CDNA4, wave64).
//
// Both directions are the same shifted sum over staged rows:
//   forward  (Sec. 2, Eq. 3):      S(d, t)   = sum_c x(c, t + shift(c, d))
//   adjoint  (transpose of Eq. 3): g(c, tau) = sum_d y(d, tau - shift(c, d)),
//                                  zero where tau - shift falls outside [0, N_out)
// In general out(o, t) = sum_k X(k, t + sh(o, k)) with staged rows k (channels
// forward, DM rows adjoint), outputs o (DM rows forward, channels adjoint) and
// sh = shift (forward) or -shift (adjoint).
//
// A workgroup owns NW*R outputs by 64*NS samples.  Rows stream in blocks of CB
// through a ring of kRing LDS slots with direct buffer-to-LDS loads, kRing-1
// blocks ahead; each staged row starts at the block's smallest sh rounded down
// to 4 floats.  Buffer bounds checks turn every read outside a row (including
// the negative times of the adjoint) into zeros, which is exactly the
// indicator of the adjoint.  Floats are 4-byte granular, so every window is
// word aligned: lane i owns words i, i+64, ... of the window, so each LDS read
// is a contiguous, bank-conflict-free 256-byte wave access; no realignment.
//
// Float sums use a fixed order that depends only on the row index: rows in
// groups of 32 summed in order into a partial, then the partials in order.
// Results are bitwise independent of the tile shape; no atomics.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd_internal.h"
#include "tile_order.h"

namespace dd {
namespace {

constexpr int kBufferRsrcFlags = 0x00020000;  // raw (untyped) buffer access, word 3 of the descriptor
constexpr int kRing = 3;
// Load segments (1 KiB each) per block: at most min(kStageSegs, kMaxSegsPerWave * NW),
// checked on the host.  A wave has at most (kRing - 1) * kMaxSegsPerWave loads in flight.
constexpr int kStageSegs = 64;
constexpr int kMaxSegsPerWave = 16;

constexpr int max_loads_per_wave(int segs, int nw) {
  return (segs + nw - 1) / nw < kMaxSegsPerWave ? (segs + nw - 1) / nw : kMaxSegsPerWave;
}

typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void_t;

template <typename T>
__device__ __forceinline__ T scalar_load(const T *p, int64_t i) {
  return ((const __attribute__((address_space(4))) T *)p)[i];
}

__device__ __forceinline__ v4i_t make_rsrc(const void *base, int bytes) {
  const uint64_t a = (uint64_t)base;
  v4i_t r;
  r.x = (int)(uint32_t)a;
  r.y = (int)(uint32_t)(a >> 32);
  r.z = bytes;
  r.w = kBufferRsrcFlags;
  return r;
}

// 16 bytes per lane from buffer offset `voff` into LDS at lds_addr + 16 * lane
// (asm: the kernel waits for these loads itself, see fwd_int.hip).
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"  // m0 is reserved, but nothing else in these kernels uses it
__device__ __forceinline__ void dma16(const v4i_t &rs, uint32_t voff, uint32_t lds_addr) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tbuffer_load_dwordx4 %0, %2, 0 offen lds"
               :
               : "v"(voff), "s"(lds_addr), "s"(rs)
               : "memory", "m0");
}
#pragma clang diagnostic pop

__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

struct FArgs {
  const float *x;        // staged rows: [n_rows][row_pitch] floats
  const uint32_t *offs;  // [n_oblk][NW][n_rows rounded up to CB][max(R,2)/2]: uint16 LDS byte offsets, in pairs
  const int32_t *sbase;  // [n_oblk][n_rows]: first staged time of each row, relative to the tile start
  float *out;            // [n_outputs][out_pitch]
  int64_t row_pitch, out_pitch;
  int32_t n_rows, row_len;       // rows and valid floats per row
  int32_t n_outputs, out_len;    // outputs and valid samples per output
  int32_t row_bytes;             // LDS bytes of one staged row
};

// This wave's load segments of a block, the same for every block of a tile:
// segment s = wave + m*NW is 64 lanes x 16 bytes of row kk starting at chunk
// j0 (segs = ceil(row_bytes / 1 KiB) per row).  Segments past the block's
// last are padding loads: every wave issues exactly MAXT loads per block, so a
// fixed vmcnt wait is exact; padding loads read nothing (zero-size buffer) and
// land in the sink.
template <int MAXT>
struct DmaPlan {
  int kk[MAXT];            // row within the block (0 for padding)
  uint32_t lds_off[MAXT];  // byte offset of the segment inside a ring slot
  uint32_t voff[MAXT];     // this lane's byte offset inside the staged row
  bool ok[MAXT];           // a real segment (wave-uniform)
  bool lane_ok[MAXT];      // this lane's 16 bytes lie inside the row (always true for padding)
};

template <int NW, int CB, int MAXT>
__device__ __forceinline__ DmaPlan<MAXT> dma_plan(int row_bytes, int row_stride, int wave, int lane) {
  DmaPlan<MAXT> d;
  const int segs = (row_bytes + 1023) >> 10;
#pragma unroll
  for (int m = 0; m < MAXT; ++m) {
    const int s = wave + m * NW;
    d.ok[m] = s < CB * segs;
    const int kk = d.ok[m] ? s / segs : 0;
    const int j0 = d.ok[m] ? (s - kk * segs) << 6 : 0;
    d.kk[m] = kk;
    d.lds_off[m] = (uint32_t)(kk * row_stride + 16 * j0);
    d.voff[m] = 16u * (uint32_t)(j0 + lane);
    d.lane_ok[m] = !d.ok[m] || 16 * (j0 + lane) < row_bytes;
  }
  return d;
}

// Stage bases of the rows this wave loads for block `kb` (first row); scalar
// loads issued one block before stage_dma needs them.
template <int MAXT>
__device__ __forceinline__ void stage_bases(const FArgs &a, const int32_t *sb, int kb, const DmaPlan<MAXT> &d,
                                            int32_t (&base)[MAXT]) {
#pragma unroll
  for (int m = 0; m < MAXT; ++m) {
    const int k = __builtin_amdgcn_readfirstlane(min(kb + d.kk[m], a.n_rows - 1));
    base[m] = scalar_load(sb, k);
  }
}

// Issue this wave's loads of block `kb` into ring slot `slot` (rows `row_stride` apart).
template <int MAXT>
__device__ __forceinline__ void stage_dma(const FArgs &a, const DmaPlan<MAXT> &d, const int32_t (&base_in)[MAXT],
                                          int64_t t0, int kb, uint8_t *slot, uint8_t *sink) {
  const uint32_t slot_addr = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void_t *)slot);
  const uint32_t sink_addr = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void_t *)sink);
#pragma unroll
  for (int m = 0; m < MAXT; ++m) {
    const bool row_ok = d.ok[m] && kb + d.kk[m] < a.n_rows;  // wave-uniform
    const int k = __builtin_amdgcn_readfirstlane(min(kb + d.kk[m], a.n_rows - 1));
    const int32_t base = row_ok ? base_in[m] : 0;
    const v4i_t rs = make_rsrc(a.x + (int64_t)k * a.row_pitch, row_ok ? 4 * a.row_len : 0);
    // first staged float: time t0 + base (a multiple of 4, possibly negative for the adjoint:
    // the offset then wraps past the row and reads zeros)
    const uint32_t voff = 4u * (uint32_t)(t0 + base) + d.voff[m];
    const uint32_t lds_addr = d.ok[m] ? slot_addr + d.lds_off[m] : sink_addr;
    if (d.lane_ok[m]) dma16(rs, voff, lds_addr);
  }
}

template <int NS, int R, int NW, int CB>
__device__ __forceinline__ void f32_tile(uint8_t *lds, const FArgs &a, int oblk, int tblk) {
  constexpr int RP = R < 2 ? 2 : R;
  constexpr int NOW = RP / 2;
  constexpr int MAXT = max_loads_per_wave(kStageSegs, NW);
  static_assert(32 % CB == 0, "blocks must tile the groups of 32 rows");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = (int64_t)tblk * (64 * NS);
  const int rows_pad = (a.n_rows + CB - 1) / CB * CB;
  const uint32_t *woffs = a.offs + ((int64_t)oblk * NW + wave) * rows_pad * NOW;
  const int32_t *sb = a.sbase + (int64_t)oblk * a.n_rows;
  const int slot_bytes = CB * a.row_bytes;
  const int nblk = rows_pad / CB;

  float tot[R][NS], part[R][NS];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < NS; ++j) tot[r][j] = part[r][j] = 0.0f;

  uint8_t *sink = lds + kRing * slot_bytes;  // 1 KiB after the ring: target of the padding loads
  const DmaPlan<MAXT> dp = dma_plan<NW, CB, MAXT>(a.row_bytes, a.row_bytes, wave, lane);
  int32_t bases[MAXT];
#pragma unroll
  for (int k = 0; k < kRing - 1; ++k) {
    stage_bases<MAXT>(a, sb, k * CB, dp, bases);
    stage_dma<MAXT>(a, dp, bases, t0, k * CB, lds + k * slot_bytes, sink);
  }
  stage_bases<MAXT>(a, sb, (kRing - 1) * CB, dp, bases);
  uint32_t ow[CB * NOW];  // offsets of block 0; each iteration fetches the next block's
#pragma unroll
  for (int q = 0; q < CB * NOW; ++q) ow[q] = scalar_load(woffs, q);

  const uint8_t *lane_base = lds + 4 * lane;
  for (int b = 0; b < nblk; ++b) {
    // Block b's loads have landed (this wave's); after the barrier every
    // wave's have, and nobody reads the slot of block b-1 any more.
    wait_vmcnt<(kRing - 2) * MAXT>();
    lds_barrier();
    stage_dma<MAXT>(a, dp, bases, t0, (b + kRing - 1) * CB, lds + ((b + kRing - 1) % kRing) * slot_bytes,
                    sink);  // zeros past the end
    const uint8_t *blk = lane_base + (b % kRing) * slot_bytes;
    // Reads run one (row, output) pair ahead of the adds in a second register set.
    float wv[2][NS];
    auto read_pair = [&](int q, float (&dst)[NS]) {
      const int kk = q / R, r = q % R;
      const uint32_t e = (ow[kk * NOW + (r >> 1)] >> (16 * (r & 1))) & 0xFFFFu;
      const float *p = (const float *)(blk + kk * a.row_bytes + e);
#pragma unroll
      for (int j = 0; j < NS; ++j) dst[j] = p[64 * j];
    };
    read_pair(0, wv[0]);
#pragma unroll
    for (int q = 0; q < CB * R; ++q) {
      if (q + 1 < CB * R) read_pair(q + 1, wv[(q + 1) & 1]);
#pragma unroll
      for (int j = 0; j < NS; ++j) part[q % R][j] += wv[q & 1][j];
    }
    if (((b + 1) * CB) % 32 == 0 || b + 1 == nblk) {  // end of a group of 32 rows
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          tot[r][j] += part[r][j];
          part[r][j] = 0.0f;
        }
    }
    // Scalar loads for the next iteration (its offsets, the stage bases of the
    // block it stages), after this block's LDS reads: LDS and scalar loads
    // share one wait counter, so none of their waits lands in the summation.
    const int oi = __builtin_amdgcn_readfirstlane(min(b + 1, nblk - 1) * CB * NOW);
#pragma unroll
    for (int q = 0; q < CB * NOW; ++q) ow[q] = scalar_load(woffs, oi + q);
    stage_bases<MAXT>(a, sb, (b + kRing) * CB, dp, bases);
  }
  wait_vmcnt<0>();
  lds_barrier();

  // Word j of lane i is sample t0 + i + 64j: stores are contiguous across the wave.
  const int o0 = oblk * (NW * R) + wave * R;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int o = o0 + r;
    if (o >= a.n_outputs) break;
    float *orow = a.out + (int64_t)o * a.out_pitch;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int64_t t = t0 + lane + 64 * j;
      if (t < a.out_len) orow[t] = tot[r][j];
    }
  }
}

template <int NS, int R, int NW, int CB>
__global__ __launch_bounds__(NW * 64) void f32_kernel(FArgs a, int n_oblk, int n_tiles, int order) {
  extern __shared__ __align__(16) uint8_t lds[];
  int oblk, tblk;
  tile_of(blockIdx.x, n_oblk, n_tiles, order, oblk, tblk);
  f32_tile<NS, R, NW, CB>(lds, a, oblk, tblk);
}

#define DD_F32_SHAPES(X) \
  X(16, 2, 16, 8) X(16, 2, 16, 4) X(16, 1, 16, 4) X(16, 1, 16, 2) X(16, 1, 16, 1) X(16, 1, 4, 1) X(16, 1, 1, 1)

template <int NS, int R, int NW, int CB>
int launch_f32_shape(const FArgs &a, int lds_bytes, int order, hipStream_t st) {
  const int64_t tiles = (a.out_len + 64 * NS - 1) / (64 * NS);
  const int64_t n_oblk = (a.n_outputs + NW * R - 1) / (NW * R);
  if (tiles * n_oblk >= ((int64_t)1 << 31)) return (int)hipErrorInvalidConfiguration;
  const void *fn = (const void *)f32_kernel<NS, R, NW, CB>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return (int)e;
  hipLaunchKernelGGL((f32_kernel<NS, R, NW, CB>), dim3((unsigned)(tiles * n_oblk)), dim3(NW * 64), lds_bytes, st, a,
                     (int)n_oblk, (int)tiles, order);
  return (int)hipGetLastError();
}

int launch_f32(const FloatTables &t, FArgs a, int64_t out_limit, hipStream_t st) {
  if (out_limit > 0 && out_limit < a.out_len) a.out_len = (int32_t)out_limit;
#define DD_TRY(NS, R, NW, CB)                                               \
  if (t.ns == NS && t.per_wave == R && t.waves == NW && t.row_block == CB) \
    return launch_f32_shape<NS, R, NW, CB>(a, t.lds_bytes, t.order, st);
  DD_F32_SHAPES(DD_TRY)
#undef DD_TRY
  return (int)hipErrorInvalidValue;
}

}  // namespace

#define DD_ROW(NS, R, NW, CB) {NS, R, NW, CB},
const int kF32Shapes[][4] = {DD_F32_SHAPES(DD_ROW)};
#undef DD_ROW
const int kNumF32Shapes = (int)(sizeof(kF32Shapes) / sizeof(kF32Shapes[0]));

int launch_forward_f32(const dd_plan &p, const void *tables, const void *d_in, float *d_out, int64_t out_pitch,
                       void *stream, int64_t out_limit) {
  const FloatTables &t = p.ftab_fwd;
  const TableLayout L = table_layout(p);
  FArgs a;
  a.x = (const float *)d_in;
  a.offs = (const uint32_t *)((const uint8_t *)tables + L.f_offs[0]);
  a.sbase = (const int32_t *)((const uint8_t *)tables + L.f_sbase[0]);
  a.out = d_out;
  a.row_pitch = p.in_pitch_bytes / 4;
  a.out_pitch = out_pitch;
  a.n_rows = p.desc.n_chan;
  a.row_len = (int32_t)p.desc.n_samp;
  a.n_outputs = p.desc.n_dm;
  a.out_len = (int32_t)p.n_out;
  a.row_bytes = t.row_bytes;
  return launch_f32(t, a, out_limit, (hipStream_t)stream);
}

int launch_adjoint(const dd_plan &p, const void *tables, const float *d_y, int64_t y_pitch, float *d_grad,
                   void *stream, int64_t out_limit) {
  const FloatTables &t = p.ftab_adj;
  const TableLayout L = table_layout(p);
  FArgs a;
  a.x = d_y;
  a.offs = (const uint32_t *)((const uint8_t *)tables + L.f_offs[1]);
  a.sbase = (const int32_t *)((const uint8_t *)tables + L.f_sbase[1]);
  a.out = d_grad;
  a.row_pitch = y_pitch;
  a.out_pitch = p.in_pitch_bytes / 4;
  a.n_rows = p.desc.n_dm;
  a.row_len = (int32_t)p.n_out;
  a.n_outputs = p.desc.n_chan;
  a.out_len = (int32_t)p.desc.n_samp;
  a.row_bytes = t.row_bytes;
  return launch_f32(t, a, out_limit, (hipStream_t)stream);
}

}  // namespace dd
