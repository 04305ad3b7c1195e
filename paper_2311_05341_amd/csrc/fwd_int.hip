// Integer forward kernels (uint8 and packed uint4 input) for gfx950.
//
// Forward transform, Sec. 2, Eq. 3:  S(d, t) = sum_c x(c, t + shift(c, d)).
//
// Tiling.  A workgroup of NW waves owns NW*R consecutive DM rows (a "DM block")
// and 64*NS consecutive output samples (a "time tile"); wave w owns R of the
// rows and each lane NS consecutive samples of them, accumulated in registers.
// Channels are visited in blocks of `chan_block`: the rows of a channel block
// are staged in LDS once, starting at the block's first-DM delay rounded down
// to 16 bytes, and each staged sample then serves all NW*R DM rows of the
// workgroup (the data reuse of the shared-memory algorithm of Sec. 4.1).  Two
// LDS buffers alternate.
//
// Byte alignment.  LDS reads on gfx950 are fast only when naturally aligned,
// but a DM's delay starts its window at any byte.  Each staged row is therefore
// kept in four copies shifted by 0..3 bytes ("phases").  For a (channel, DM)
// pair with window offset o, a lane reads the copy of phase o % 4 from byte
// o - o % 4 on: whole, aligned 32-bit words, no realignment arithmetic.
//
// Exact arithmetic with two samples per add (the SIMD-within-a-word idea of
// Sec. 4.1).  For each 4-sample word w = [b0 b1 b2 b3] a lane adds
//     mix += w                       (all four bytes; carries cross byte lanes)
//     odd += [b1, 0, b3, 0]          (two 16-bit lanes, one v_perm)
// For <= 257 channels no 16-bit lane of `odd` overflows, and
//     mix - (odd << 8) = sum b0 + 2^16 * sum b2        (mod 2^32)
// recovers the even samples exactly.  Every 256 channels both are flushed into
// per-sample int32 totals, which stay below 2^24 and convert to float exactly.
//
// Staging runs two blocks ahead: global reads for block b+2 are issued into
// registers before block b is summed, and block b+1's phase copies are written
// after it, so one barrier per block suffices.
//
// Grid order: blockIdx.x runs over DM blocks, so the workgroups resident at any
// time share a few time tiles and read the same input rows through L2/MALL.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd_internal.h"

namespace dd {
namespace {

constexpr uint32_t kOddSel = 0x0C030C01u;  // v_perm: bytes 1 and 3 into bytes 0 and 2, zeros elsewhere

// Unpack 8 bytes of 4-bit samples (even sample in the low nibble) into 16 bytes.
__device__ __forceinline__ uint4 unpack_u4(uint2 p) {
  const uint32_t lo0 = p.x & 0x0F0F0F0Fu, hi0 = (p.x >> 4) & 0x0F0F0F0Fu;
  const uint32_t lo1 = p.y & 0x0F0F0F0Fu, hi1 = (p.y >> 4) & 0x0F0F0F0Fu;
  uint4 r;
  r.x = __builtin_amdgcn_perm(hi0, lo0, 0x05010400u);
  r.y = __builtin_amdgcn_perm(hi0, lo0, 0x07030602u);
  r.z = __builtin_amdgcn_perm(hi1, lo1, 0x05010400u);
  r.w = __builtin_amdgcn_perm(hi1, lo1, 0x07030602u);
  return r;
}

// Write phases 1..3 of one 16-byte chunk whose phase-0 words are w[0..3] and
// whose next word is w[4]; `dst` points at the chunk in phase 0.
__device__ __forceinline__ void write_phases(uint8_t *dst, int row_bytes, const uint32_t (&w)[5]) {
#pragma unroll
  for (int p = 1; p < 4; ++p) {
    uint4 v;
    v.x = __builtin_amdgcn_alignbyte(w[1], w[0], p);
    v.y = __builtin_amdgcn_alignbyte(w[2], w[1], p);
    v.z = __builtin_amdgcn_alignbyte(w[3], w[2], p);
    v.w = __builtin_amdgcn_alignbyte(w[4], w[3], p);
    *(uint4 *)(dst + p * row_bytes) = v;
  }
}

template <int NS, int R>
__device__ __forceinline__ void flush(uint32_t (&mix)[R][NS / 4], uint32_t (&odd)[R][NS / 4], uint32_t (&tot)[R][NS]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int k = 0; k < NS / 4; ++k) {
      const uint32_t od = odd[r][k];
      const uint32_t ev = mix[r][k] - (od << 8);
      tot[r][4 * k + 0] += ev & 0xFFFFu;
      tot[r][4 * k + 1] += od & 0xFFFFu;
      tot[r][4 * k + 2] += ev >> 16;
      tot[r][4 * k + 3] += od >> 16;
      mix[r][k] = 0;
      odd[r][k] = 0;
    }
  }
}

// Kernel arguments shared by the plain and the batched kernels.
struct IntArgs {
  const uint8_t *x;       // [n_chan][pitch] bytes
  const uint32_t *offs;   // [n_dblk][NW][n_chan][max(R,2)/2]: pairs of uint16 (shift - stage base)
  const int32_t *sbase;   // [n_dblk][n_chan]: stage base (first-DM shift rounded down to the unit)
  float *out;             // [n_dm][out_pitch]
  int64_t pitch, n_samp, n_out, out_pitch;
  int32_t n_chan, n_dm, row_bytes, chan_block;
};

// Staging of one channel block, in two halves: `load` issues the global reads
// into registers (one task = one 16-byte LDS chunk of a row, i.e. 16 samples,
// plus the first 4 samples of the next chunk), and `write` later stores the
// four byte-phase copies of every chunk.  Between the two the workgroup sums
// the previous block, which hides the global-memory latency.
template <int MAXT>
struct Held {
  uint32_t w[MAXT][5];
};

template <int NT, int MAXT, bool U4>
__device__ __forceinline__ void stage_load(const IntArgs &a, const int32_t *sb, int64_t t0, int cb, int nch,
                                           Held<MAXT> &h) {
  const int row_chunks = a.row_bytes >> 4;
#pragma unroll
  for (int k = 0; k < MAXT; ++k) {
    const int i = threadIdx.x + k * NT;
#pragma unroll
    for (int q = 0; q < 5; ++q) h.w[k][q] = 0;
    if (i < nch * row_chunks) {
      const int cc = i / row_chunks, j = i - cc * row_chunks;
      const int c = cb + cc;
      const int64_t g = t0 + sb[c] + 16 * (int64_t)j;  // first sample of the chunk (multiple of 16)
      const uint8_t *row = a.x + (int64_t)c * a.pitch;
      if (!U4) {
        if (g < a.n_samp) {
          const uint4 v = *(const uint4 *)(row + g);
          h.w[k][0] = v.x;
          h.w[k][1] = v.y;
          h.w[k][2] = v.z;
          h.w[k][3] = v.w;
        }
        if (g + 16 < a.n_samp) h.w[k][4] = *(const uint32_t *)(row + g + 16);
      } else {
        if (g < a.n_samp) {
          const uint2 v = *(const uint2 *)(row + (g >> 1));
          h.w[k][0] = v.x;
          h.w[k][1] = v.y;
        }
        if (g + 16 < a.n_samp) h.w[k][4] = *(const uint32_t *)(row + ((g + 16) >> 1));
      }
    }
  }
}

template <int NT, int MAXT, bool U4>
__device__ __forceinline__ void stage_write(const IntArgs &a, int nch, uint8_t *buf, const Held<MAXT> &h) {
  const int row_chunks = a.row_bytes >> 4;
#pragma unroll
  for (int k = 0; k < MAXT; ++k) {
    const int i = threadIdx.x + k * NT;
    if (i < nch * row_chunks) {
      const int cc = i / row_chunks, j = i - cc * row_chunks;
      uint8_t *p0 = buf + cc * 4 * a.row_bytes + 16 * j;
      uint32_t w[5];
      if (!U4) {
#pragma unroll
        for (int q = 0; q < 5; ++q) w[q] = h.w[k][q];
      } else {
        const uint4 v = unpack_u4(make_uint2(h.w[k][0], h.w[k][1]));
        const uint4 n = unpack_u4(make_uint2(h.w[k][4], 0u));
        w[0] = v.x;
        w[1] = v.y;
        w[2] = v.z;
        w[3] = v.w;
        w[4] = n.x;
      }
      *(uint4 *)p0 = make_uint4(w[0], w[1], w[2], w[3]);
      write_phases(p0, a.row_bytes, w);
    }
  }
}

// Staging tasks per block are at most kStageTasks (host keeps
// chan_block * row_bytes / 16 <= kStageTasks), i.e. kStageTasks / threads per thread.
constexpr int kStageTasks = 1024;

// One tile: DM block `dblk`, time tile `tblk`.  `lds` holds two buffers of
// chan_block * 4 * row_bytes bytes.
template <int NS, int R, int NW, bool U4>
__device__ __forceinline__ void fwd_int_tile(uint8_t *lds, const IntArgs &a, int dblk, int tblk) {
  constexpr int NT = NW * 64;
  constexpr int RP = R < 2 ? 2 : R;  // uint16 slots per channel in the offset table
  constexpr int NOW = RP / 2;        // uint32 words per channel
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = (int64_t)tblk * (64 * NS);
  const uint32_t *woffs = a.offs + ((int64_t)dblk * NW + wave) * a.n_chan * NOW;
  const int32_t *sb = a.sbase + (int64_t)dblk * a.n_chan;
  const int buf_bytes = a.chan_block * 4 * a.row_bytes;

  uint32_t tot[R][NS], mix[R][NS / 4], odd[R][NS / 4];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int j = 0; j < NS; ++j) tot[r][j] = 0;
#pragma unroll
    for (int k = 0; k < NS / 4; ++k) mix[r][k] = odd[r][k] = 0;
  }

  const int nblk = (a.n_chan + a.chan_block - 1) / a.chan_block;
  constexpr int MAXT = kStageTasks / NT;
  Held<MAXT> next, after;  // stages b+1 and b+2
  stage_load<NT, MAXT, U4>(a, sb, t0, 0, min(a.chan_block, a.n_chan), next);
  if (nblk > 1) stage_load<NT, MAXT, U4>(a, sb, t0, a.chan_block, min(a.chan_block, a.n_chan - a.chan_block), after);
  stage_write<NT, MAXT, U4>(a, min(a.chan_block, a.n_chan), lds, next);
  next = after;
  __syncthreads();

  const uint8_t *lane_base = lds + NS * lane;
  int since_flush = 0;
  for (int b = 0; b < nblk; ++b) {
    const int cb = b * a.chan_block;
    const int nch = min(a.chan_block, a.n_chan - cb);
    const int cur_off = (b & 1) * buf_bytes;
    if (b + 2 < nblk) {
      const int c2 = cb + 2 * a.chan_block;
      stage_load<NT, MAXT, U4>(a, sb, t0, c2, min(a.chan_block, a.n_chan - c2), after);
    }
    // Sum this block: every (channel, DM row) pair reads NS/4 aligned words of
    // the byte phase that puts its window on a word boundary.
    for (int cc = 0; cc < nch; ++cc) {
      uint32_t ow[NOW];
#pragma unroll
      for (int q = 0; q < NOW; ++q) ow[q] = woffs[(int64_t)(cb + cc) * NOW + q];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t o = (ow[r >> 1] >> (16 * (r & 1))) & 0xFFFFu;
        const uint32_t *p = (const uint32_t *)(lane_base + cur_off + (cc * 4 + (int)(o & 3u)) * a.row_bytes +
                                               (o & ~3u));
#pragma unroll
        for (int k = 0; k < NS / 4; ++k) {
          const uint32_t w = p[k];
          mix[r][k] += w;
          odd[r][k] += __builtin_amdgcn_perm(w, w, kOddSel);
        }
      }
    }
    since_flush += nch;
    const bool more = b + 1 < nblk;
    if (since_flush >= 256 || !more) {
      flush<NS, R>(mix, odd, tot);
      since_flush = 0;
    }
    if (more) {
      const int c1 = cb + a.chan_block;
      stage_write<NT, MAXT, U4>(a, min(a.chan_block, a.n_chan - c1), lds + ((b + 1) & 1) * buf_bytes, next);
      next = after;
    }
    __syncthreads();
  }

  const int64_t tl = t0 + (int64_t)NS * lane;
  const int d0 = dblk * (NW * R) + wave * R;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int d = d0 + r;
    if (d >= a.n_dm) break;
    float *orow = a.out + (int64_t)d * a.out_pitch;
#pragma unroll
    for (int j = 0; j < NS; j += 4) {
      const int64_t t = tl + j;
      if (t + 3 < a.n_out) {
        *(float4 *)(orow + t) = make_float4((float)tot[r][j], (float)tot[r][j + 1], (float)tot[r][j + 2],
                                            (float)tot[r][j + 3]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (t + i < a.n_out) orow[t + i] = (float)tot[r][j + i];
      }
    }
  }
}

// One workgroup per tile; grid = (DM blocks, time tiles).
template <int NS, int R, int NW, bool U4>
__global__ __launch_bounds__(NW * 64) void fwd_int_kernel(IntArgs a) {
  extern __shared__ __align__(16) uint8_t lds[];
  fwd_int_tile<NS, R, NW, U4>(lds, a, blockIdx.x, blockIdx.y);
}

__global__ void reset_counter_kernel(unsigned long long *counter) { *counter = 0ull; }

// Persistent batched forward kernel.  Workgroups repeatedly claim the next work
// item (beam, DM block, time tile) from a device counter; items are numbered
// beam by beam with the beams in decreasing cost order and, inside a beam,
// DM block fastest.  A workgroup returns at its first claim past the last
// item, so every wave reaches the exit.
template <int NS, int R, int NW, bool U4>
__global__ __launch_bounds__(NW * 64) void fwd_int_batched_kernel(const BeamDesc *__restrict__ beams, int n_beams,
                                                                   long long n_items,
                                                                   unsigned long long *__restrict__ counter) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ long long claimed;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) claimed = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const unsigned long long raw = (unsigned long long)claimed;
    const long long item = (long long)(((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(raw >> 32)) << 32) |
                                       (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)raw));
    if (item >= n_items) return;
    int lo = 0, hi = n_beams - 1;  // last beam whose item_begin <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (beams[mid].item_begin <= item) lo = mid; else hi = mid - 1;
    }
    const BeamDesc &b = beams[lo];
    const long long k = item - b.item_begin;
    const int tblk = (int)(k / b.tiles_d), dblk = (int)(k - (long long)tblk * b.tiles_d);
    IntArgs a;
    a.x = b.x;
    a.offs = b.offs;
    a.sbase = b.sbase;
    a.out = b.out;
    a.pitch = b.pitch;
    a.n_samp = b.n_samp;
    a.n_out = b.n_out;
    a.out_pitch = b.out_pitch;
    a.n_chan = b.n_chan;
    a.n_dm = b.n_dm;
    a.row_bytes = b.row_bytes;
    a.chan_block = b.chan_block;
    fwd_int_tile<NS, R, NW, U4>(lds, a, dblk, tblk);
  }
}

#define DD_INT_SHAPES(X) X(16, 2, 16) X(16, 4, 8) X(32, 2, 8) X(16, 1, 16) X(32, 1, 8)

template <int NS, int R, int NW>
int launch_int_shape(const dd_plan &p, const void *d_in, float *d_out, int64_t out_pitch, hipStream_t st) {
  const TileCfg &t = p.fwd;
  IntArgs a;
  a.x = (const uint8_t *)d_in;
  a.offs = (const uint32_t *)((const uint8_t *)p.d_tables + p.int_offs_off);
  a.sbase = (const int32_t *)((const uint8_t *)p.d_tables + p.int_sbase_off);
  a.out = d_out;
  a.pitch = p.in_pitch_bytes;
  a.n_samp = p.desc.n_samp;
  a.n_out = p.n_out;
  a.out_pitch = out_pitch;
  a.n_chan = p.desc.n_chan;
  a.n_dm = p.desc.n_dm;
  a.row_bytes = t.row_bytes;
  a.chan_block = t.chan_block;
  const int64_t tiles_t = (p.n_out + 64 * NS - 1) / (64 * NS);
  if (tiles_t > 65535) return (int)hipErrorInvalidConfiguration;
  dim3 grid((unsigned)((p.desc.n_dm + NW * R - 1) / (NW * R)), (unsigned)tiles_t);
  const void *fn = p.desc.dtype == DD_U4 ? (const void *)fwd_int_kernel<NS, R, NW, true>
                                         : (const void *)fwd_int_kernel<NS, R, NW, false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, t.lds_bytes);
  if (e != hipSuccess) return (int)e;
  if (p.desc.dtype == DD_U4)
    hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, true>), grid, dim3(NW * 64), t.lds_bytes, st, a);
  else
    hipLaunchKernelGGL((fwd_int_kernel<NS, R, NW, false>), grid, dim3(NW * 64), t.lds_bytes, st, a);
  return (int)hipGetLastError();
}

}  // namespace

const int kIntShapes[][3] = {{16, 2, 16}, {16, 4, 8}, {32, 2, 8}, {16, 1, 16}, {32, 1, 8}};
const int kNumIntShapes = 5;

int launch_forward_int(const dd_plan &p, const void *d_in, float *d_out, int64_t out_pitch, void *stream) {
  const TileCfg &t = p.fwd;
#define DD_TRY(NS, R, NW) \
  if (t.ns == NS && t.dm_per_wave == R && t.waves == NW) return launch_int_shape<NS, R, NW>(p, d_in, d_out, out_pitch, (hipStream_t)stream);
  DD_INT_SHAPES(DD_TRY)
#undef DD_TRY
  return (int)hipErrorInvalidValue;
}

int batch_kernels(int ns, int dm_per_wave, int waves, bool u4, int lds_bytes, BatchLaunch *out) {
  const void *fn = nullptr;
#define DD_TRY(NS, R, NW)                                                              \
  if (ns == NS && dm_per_wave == R && waves == NW)                                     \
    fn = u4 ? (const void *)fwd_int_batched_kernel<NS, R, NW, true>                     \
            : (const void *)fwd_int_batched_kernel<NS, R, NW, false>;
  DD_INT_SHAPES(DD_TRY)
#undef DD_TRY
  if (!fn) return (int)hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return (int)e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, waves * 64, lds_bytes);
  if (e != hipSuccess) return (int)e;
  int dev = 0, n_cu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  out->reset_fn = (const void *)reset_counter_kernel;
  out->main_fn = fn;
  out->grid = n_cu * (per_cu > 0 ? per_cu : 1);
  out->block = waves * 64;
  out->lds_bytes = lds_bytes;
  return 0;
}

}  // namespace dd
