// Forward and adjoint dedispersion kernels for gfx950 (CDNA4, wave64).
//
// Forward (Sec. 2, Eq. 3): S(d, t) = sum_c x(c, t + shift(c, d)).
// A workgroup owns a tile of (waves * R) DM rows by 64*NS output samples.  It
// walks the channels in blocks: each block's rows are staged into LDS once,
// starting at the tile's first-DM delay rounded down to a 16-byte chunk, and
// every staged sample then feeds all DM rows of the tile (the reuse the
// shared-memory algorithm of Sec. 4.1 is built on).  Each lane keeps NS
// consecutive output samples of R DM rows in registers.
//
// LDS reads on gfx950 are only fast when naturally aligned, while a DM's delay
// puts its window at an arbitrary byte offset.  So a lane always reads aligned
// 16-byte chunks and realigns in registers: the offset is wave-uniform (all
// lanes of a wave share the DM and channel), so the word part of it selects an
// unrolled variant and the byte part is an SGPR operand of v_alignbyte/v_perm.
//
// Exact integer accumulation with two samples per add (the SIMD-within-a-word
// idea of Sec. 4.1): for each 4-sample word w = [b0 b1 b2 b3] a lane adds
//   mix += w                    (all four bytes, carries mixing across bytes)
//   odd += [b1, 0, b3, 0]       (two 16-bit lanes)
// For up to 257 channels the 16-bit lanes of `odd` cannot overflow and
//   mix - (odd << 8) = b0_sum + 2^16 * b2_sum      (mod 2^32)
// recovers the even samples exactly, so every 256 channels the pair is
// flushed into per-sample int32 totals.  Totals stay below 2^24 and convert
// to float exactly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd_internal.h"

namespace dd {
namespace {

// v_perm selector taking bytes (b+1) and (b+3) of {hi:lo} into bytes 0 and 2
// and zeros (selector 0x0C) into bytes 1 and 3.
__device__ __forceinline__ uint32_t odd_selector(uint32_t b) {
  return 0x0C000C00u | ((b + 3u) << 16) | (b + 1u);
}

template <int NS, int WQ>
__device__ __forceinline__ void accumulate_u8(const uint32_t (&w)[4 * (NS / 16 + 1)], uint32_t br,
                                              uint32_t sel, uint32_t (&mix)[NS / 4],
                                              uint32_t (&odd)[NS / 4]) {
#pragma unroll
  for (int k = 0; k < NS / 4; ++k) {
    const uint32_t lo = w[WQ + k], hi = w[WQ + k + 1];
    mix[k] += __builtin_amdgcn_alignbyte(hi, lo, br);
    odd[k] += __builtin_amdgcn_perm(hi, lo, sel);
  }
}

template <int NS, int R>
__device__ __forceinline__ void flush_u8(uint32_t (&mix)[R][NS / 4], uint32_t (&odd)[R][NS / 4],
                                         uint32_t (&tot)[R][NS]) {
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

// One forward tile of the integer kernel (uint8 or packed uint4 input): DM rows
// [by*NW*R, by*NW*R + NW*R) by samples [bx*64*NS, bx*64*NS + 64*NS), all
// channels.  `lds` holds chan_block rows of row_bytes bytes.
template <int NS, int R, int NW, bool U4>
__device__ __forceinline__ void fwd_int_tile(
    uint8_t *lds, const uint8_t *__restrict__ x, int64_t pitch, int n_chan, int64_t n_samp,
    const int32_t *__restrict__ shift, int n_dm, int64_t n_out, float *__restrict__ out,
    int64_t out_pitch, int row_bytes, int chan_block, int bx, int by) {
  constexpr int NCH = NS / 16 + 1;     // aligned 16-byte chunks one lane reads
  constexpr int UNIT = U4 ? 32 : 16;   // staging alignment in samples (one 16-byte global chunk)
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = (int64_t)bx * (64 * NS);
  const int d_lo = by * (NW * R);
  const int32_t *s_lo = shift + (int64_t)d_lo * n_chan;
  const int32_t *srow[R];
#pragma unroll
  for (int r = 0; r < R; ++r) srow[r] = shift + (int64_t)min(d_lo + wave * R + r, n_dm - 1) * n_chan;

  uint32_t tot[R][NS], mix[R][NS / 4], odd[R][NS / 4];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int j = 0; j < NS; ++j) tot[r][j] = 0;
#pragma unroll
    for (int k = 0; k < NS / 4; ++k) mix[r][k] = odd[r][k] = 0;
  }

  const int row_chunks = row_bytes >> 4;
  int since_flush = 0;
  for (int cb = 0; cb < n_chan; cb += chan_block) {
    const int nch = min(chan_block, n_chan - cb);
    __syncthreads();
    // Stage rows cb..cb+nch-1: LDS byte i of row cc is sample g0 + i of channel cb+cc.
    for (int i = threadIdx.x; i < nch * row_chunks; i += NW * 64) {
      const int cc = i / row_chunks, j = i - cc * row_chunks;
      const int c = cb + cc;
      const int64_t g0 = (t0 + s_lo[c]) & ~(int64_t)(UNIT - 1);
      const int64_t g = g0 + 16 * (int64_t)j;  // first sample of this LDS chunk
      uint4 v = make_uint4(0, 0, 0, 0);
      if (g < n_samp) {
        if (!U4) {
          v = *(const uint4 *)(x + (int64_t)c * pitch + g);
        } else {
          v = unpack_u4(*(const uint2 *)(x + (int64_t)c * pitch + (g >> 1)));
        }
      }
      *(uint4 *)(lds + cc * row_bytes + 16 * j) = v;
    }
    __syncthreads();
    for (int cc = 0; cc < nch; ++cc) {
      const int c = cb + cc;
      const int32_t base = s_lo[c] & ~(UNIT - 1);
      const uint8_t *rowp = lds + cc * row_bytes + NS * lane;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t o = (uint32_t)(srow[r][c] - base);  // 0 .. span + UNIT - 1
        const uint4 *p = (const uint4 *)(rowp + (o & ~15u));
        uint32_t w[4 * NCH];
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
          const uint4 v = p[q];
          w[4 * q + 0] = v.x;
          w[4 * q + 1] = v.y;
          w[4 * q + 2] = v.z;
          w[4 * q + 3] = v.w;
        }
        const uint32_t br = o & 3u, sel = odd_selector(br);
        switch ((o >> 2) & 3u) {
          case 0: accumulate_u8<NS, 0>(w, br, sel, mix[r], odd[r]); break;
          case 1: accumulate_u8<NS, 1>(w, br, sel, mix[r], odd[r]); break;
          case 2: accumulate_u8<NS, 2>(w, br, sel, mix[r], odd[r]); break;
          default: accumulate_u8<NS, 3>(w, br, sel, mix[r], odd[r]); break;
        }
      }
    }
    since_flush += nch;
    if (since_flush >= 256 || cb + chan_block >= n_chan) {
      flush_u8<NS, R>(mix, odd, tot);
      since_flush = 0;
    }
  }

  const int64_t tl = t0 + (int64_t)NS * lane;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int d = d_lo + wave * R + r;
    if (d >= n_dm) break;
    float *orow = out + (int64_t)d * out_pitch;
#pragma unroll
    for (int j = 0; j < NS; j += 4) {
      const int64_t t = tl + j;
      if (t + 3 < n_out) {
        *(float4 *)(orow + t) = make_float4((float)tot[r][j], (float)tot[r][j + 1],
                                            (float)tot[r][j + 2], (float)tot[r][j + 3]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (t + i < n_out) orow[t + i] = (float)tot[r][j + i];
      }
    }
  }
}

// Integer forward kernel: one workgroup per tile.
// grid = (ceil(n_out / (64*NS)), ceil(n_dm / (NW*R))), block = NW*64.
template <int NS, int R, int NW, bool U4>
__global__ __launch_bounds__(NW * 64) void fwd_int_kernel(
    const uint8_t *__restrict__ x, int64_t pitch, int n_chan, int64_t n_samp,
    const int32_t *__restrict__ shift, int n_dm, int64_t n_out, float *__restrict__ out,
    int64_t out_pitch, int row_bytes, int chan_block) {
  extern __shared__ __align__(16) uint8_t lds[];
  fwd_int_tile<NS, R, NW, U4>(lds, x, pitch, n_chan, n_samp, shift, n_dm, n_out, out, out_pitch, row_bytes,
                              chan_block, blockIdx.x, blockIdx.y);
}

__global__ void reset_counter_kernel(unsigned long long *counter) { *counter = 0ull; }

// Persistent batched forward kernel.  Every workgroup repeatedly claims the
// next work item from a device counter (items are numbered beam by beam, the
// beams in decreasing cost order) and runs that beam's tile.  A workgroup stops
// at the first claim past the last item, so every wave reaches the exit.
template <int NS, int R, int NW, bool U4>
__global__ __launch_bounds__(NW * 64) void fwd_int_batched_kernel(
    const BeamDesc *__restrict__ beams, int n_beams, long long n_items,
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
    const int by = (int)(k / b.tiles_t), bx = (int)(k - (long long)by * b.tiles_t);
    fwd_int_tile<NS, R, NW, U4>(lds, b.x, b.pitch, b.n_chan, b.n_samp, b.shift, b.n_dm, b.n_out, b.out,
                                b.out_pitch, b.row_bytes, b.chan_block, bx, by);
  }
}

template <int NS, int WQ>
__device__ __forceinline__ void accumulate_f32(const float (&w)[NS + 4], float (&acc)[NS]) {
#pragma unroll
  for (int j = 0; j < NS; ++j) acc[j] += w[WQ + j];
}

// Float forward kernel.  Channels are summed in groups of 32 (global channel
// index / 32): inside a group in channel order into a partial sum, then the
// partial is added to the total in group order.  The order depends only on the
// channel index, so every tile shape gives the same bits.
template <int NS, int R, int NW>
__global__ __launch_bounds__(NW * 64) void fwd_f32_kernel(
    const float *__restrict__ x, int64_t pitch_elems, int n_chan, int64_t n_samp,
    const int32_t *__restrict__ shift, int n_dm, int64_t n_out, float *__restrict__ out,
    int64_t out_pitch, int row_bytes, int chan_block) {
  extern __shared__ __align__(16) uint8_t lds[];
  constexpr int NCH = NS / 4 + 1;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = (int64_t)blockIdx.x * (64 * NS);
  const int d_lo = blockIdx.y * (NW * R);
  const int32_t *s_lo = shift + (int64_t)d_lo * n_chan;
  const int32_t *srow[R];
#pragma unroll
  for (int r = 0; r < R; ++r) srow[r] = shift + (int64_t)min(d_lo + wave * R + r, n_dm - 1) * n_chan;

  float tot[R][NS], part[R][NS];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < NS; ++j) tot[r][j] = part[r][j] = 0.0f;

  const int row_chunks = row_bytes >> 4;
  const int row_floats = row_bytes >> 2;
  const float *ldsf = (const float *)lds;
  for (int cb = 0; cb < n_chan; cb += chan_block) {
    const int nch = min(chan_block, n_chan - cb);
    __syncthreads();
    for (int i = threadIdx.x; i < nch * row_chunks; i += NW * 64) {
      const int cc = i / row_chunks, j = i - cc * row_chunks;
      const int c = cb + cc;
      const int64_t g0 = (t0 + s_lo[c]) & ~(int64_t)3;
      const int64_t g = g0 + 4 * (int64_t)j;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (g < n_samp) v = *(const float4 *)(x + (int64_t)c * pitch_elems + g);
      *(float4 *)(lds + cc * row_bytes + 16 * j) = v;
    }
    __syncthreads();
    for (int cc = 0; cc < nch; ++cc) {
      const int c = cb + cc;
      const int32_t base = s_lo[c] & ~3;
      const float *rowp = ldsf + cc * row_floats + NS * lane;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t o = (uint32_t)(srow[r][c] - base);
        const float4 *p = (const float4 *)(rowp + (o & ~3u));
        float w[NS + 4];
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
          const float4 v = p[q];
          w[4 * q + 0] = v.x;
          w[4 * q + 1] = v.y;
          w[4 * q + 2] = v.z;
          w[4 * q + 3] = v.w;
        }
        switch (o & 3u) {
          case 0: accumulate_f32<NS, 0>(w, part[r]); break;
          case 1: accumulate_f32<NS, 1>(w, part[r]); break;
          case 2: accumulate_f32<NS, 2>(w, part[r]); break;
          default: accumulate_f32<NS, 3>(w, part[r]); break;
        }
      }
      if (((c + 1) & 31) == 0 || c + 1 == n_chan) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int j = 0; j < NS; ++j) {
            tot[r][j] += part[r][j];
            part[r][j] = 0.0f;
          }
      }
    }
  }

  const int64_t tl = t0 + (int64_t)NS * lane;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int d = d_lo + wave * R + r;
    if (d >= n_dm) break;
    float *orow = out + (int64_t)d * out_pitch;
#pragma unroll
    for (int j = 0; j < NS; j += 4) {
      const int64_t t = tl + j;
      if (t + 3 < n_out) {
        *(float4 *)(orow + t) = make_float4(tot[r][j], tot[r][j + 1], tot[r][j + 2], tot[r][j + 3]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (t + i < n_out) orow[t + i] = tot[r][j + i];
      }
    }
  }
}

// Adjoint kernel (transpose of Eq. 3, gather form):
//   g(c, tau) = sum_d [0 <= tau - shift(c,d) < n_out] y(d, tau - shift(c,d)).
// A workgroup owns (NW * R) channels by 64*NS samples of tau.  DM rows are
// staged DB at a time: row d holds y(d, u) for u from u0(d) = (tau0 - smax(d))
// rounded down to 4, where smax(d) is the largest delay of the workgroup's
// channels at DM d; samples outside [0, n_out) are staged as zeros, which
// implements the indicator.  DMs are summed in groups of 32 (global DM index
// / 32), in DM order inside a group, then group by group: tile-independent.
template <int NS, int R, int NW>
__global__ __launch_bounds__(NW * 64) void adj_f32_kernel(
    const float *__restrict__ y, int64_t y_pitch, int n_chan, int64_t n_samp,
    const int32_t *__restrict__ shift_t /* [n_chan][n_dm] */,
    const int32_t *__restrict__ smax /* [n_cblocks][n_dm] */, int n_dm, int64_t n_out,
    float *__restrict__ g, int64_t g_pitch_elems, int row_bytes, int dm_block) {
  extern __shared__ __align__(16) uint8_t lds[];
  constexpr int NCH = NS / 4 + 1;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t tau0 = (int64_t)blockIdx.x * (64 * NS);
  const int c_lo = blockIdx.y * (NW * R);
  const int32_t *smax_row = smax + (int64_t)blockIdx.y * n_dm;
  const int32_t *scol[R];
#pragma unroll
  for (int r = 0; r < R; ++r) scol[r] = shift_t + (int64_t)min(c_lo + wave * R + r, n_chan - 1) * n_dm;

  float tot[R][NS], part[R][NS];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < NS; ++j) tot[r][j] = part[r][j] = 0.0f;

  const int row_chunks = row_bytes >> 4;
  const int row_floats = row_bytes >> 2;
  const float *ldsf = (const float *)lds;
  for (int db = 0; db < n_dm; db += dm_block) {
    const int nd = min(dm_block, n_dm - db);
    __syncthreads();
    for (int i = threadIdx.x; i < nd * row_chunks; i += NW * 64) {
      const int dd = i / row_chunks, j = i - dd * row_chunks;
      const int d = db + dd;
      const int64_t u0 = (tau0 - smax_row[d]) & ~(int64_t)3;  // floor to a multiple of 4 (also < 0)
      const int64_t u = u0 + 4 * (int64_t)j;
      const float *yr = y + (int64_t)d * y_pitch;
      float4 v;
      if (u >= 0 && u + 3 < n_out) {
        v = *(const float4 *)(yr + u);
      } else {
        v.x = (u + 0 >= 0 && u + 0 < n_out) ? yr[u + 0] : 0.0f;
        v.y = (u + 1 >= 0 && u + 1 < n_out) ? yr[u + 1] : 0.0f;
        v.z = (u + 2 >= 0 && u + 2 < n_out) ? yr[u + 2] : 0.0f;
        v.w = (u + 3 >= 0 && u + 3 < n_out) ? yr[u + 3] : 0.0f;
      }
      *(float4 *)(lds + dd * row_bytes + 16 * j) = v;
    }
    __syncthreads();
    for (int dd = 0; dd < nd; ++dd) {
      const int d = db + dd;
      const int32_t sm = smax_row[d];
      // LDS index of y(d, tau0 - s + k) is k + (tau0 - s) - u0 = k + (sm - s) + ((tau0 - sm) & 3).
      const int32_t phase = (int32_t)((tau0 - sm) & 3);
      const float *rowp = ldsf + dd * row_floats + NS * lane;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t o = (uint32_t)(sm - scol[r][d] + phase);
        const float4 *p = (const float4 *)(rowp + (o & ~3u));
        float w[NS + 4];
#pragma unroll
        for (int q = 0; q < NCH; ++q) {
          const float4 v = p[q];
          w[4 * q + 0] = v.x;
          w[4 * q + 1] = v.y;
          w[4 * q + 2] = v.z;
          w[4 * q + 3] = v.w;
        }
        switch (o & 3u) {
          case 0: accumulate_f32<NS, 0>(w, part[r]); break;
          case 1: accumulate_f32<NS, 1>(w, part[r]); break;
          case 2: accumulate_f32<NS, 2>(w, part[r]); break;
          default: accumulate_f32<NS, 3>(w, part[r]); break;
        }
      }
      if (((d + 1) & 31) == 0 || d + 1 == n_dm) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int j = 0; j < NS; ++j) {
            tot[r][j] += part[r][j];
            part[r][j] = 0.0f;
          }
      }
    }
  }

  const int64_t tl = tau0 + (int64_t)NS * lane;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int c = c_lo + wave * R + r;
    if (c >= n_chan) break;
    float *grow = g + (int64_t)c * g_pitch_elems;
#pragma unroll
    for (int j = 0; j < NS; j += 4) {
      const int64_t t = tl + j;
      if (t + 3 < n_samp) {
        *(float4 *)(grow + t) = make_float4(tot[r][j], tot[r][j + 1], tot[r][j + 2], tot[r][j + 3]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (t + i < n_samp) grow[t + i] = tot[r][j + i];
      }
    }
  }
}

template <typename K>
static int set_lds(K kern, int bytes) {
  return (int)hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <int NS, int R, int NW>
static int launch_int(const dd_plan &p, const void *d_in, float *d_out, int64_t out_pitch, hipStream_t st) {
  const TileCfg &t = p.fwd;
  dim3 grid((unsigned)((p.n_out + 64 * NS - 1) / (64 * NS)), (unsigned)((p.desc.n_dm + NW * R - 1) / (NW * R)));
  if (p.desc.dtype == DD_U4) {
    auto k = fwd_int_kernel<NS, R, NW, true>;
    int e = set_lds(k, t.lds_bytes);
    if (e) return e;
    hipLaunchKernelGGL(k, grid, dim3(NW * 64), t.lds_bytes, st, (const uint8_t *)d_in, p.in_pitch_bytes,
                       p.desc.n_chan, p.desc.n_samp, p.d_shift, p.desc.n_dm, p.n_out, d_out, out_pitch,
                       t.row_bytes, t.chan_block);
  } else {
    auto k = fwd_int_kernel<NS, R, NW, false>;
    int e = set_lds(k, t.lds_bytes);
    if (e) return e;
    hipLaunchKernelGGL(k, grid, dim3(NW * 64), t.lds_bytes, st, (const uint8_t *)d_in, p.in_pitch_bytes,
                       p.desc.n_chan, p.desc.n_samp, p.d_shift, p.desc.n_dm, p.n_out, d_out, out_pitch,
                       t.row_bytes, t.chan_block);
  }
  return (int)hipGetLastError();
}

template <int NS, int R, int NW>
static int launch_f32(const dd_plan &p, const void *d_in, float *d_out, int64_t out_pitch, hipStream_t st) {
  const TileCfg &t = p.fwd;
  dim3 grid((unsigned)((p.n_out + 64 * NS - 1) / (64 * NS)), (unsigned)((p.desc.n_dm + NW * R - 1) / (NW * R)));
  auto k = fwd_f32_kernel<NS, R, NW>;
  int e = set_lds(k, t.lds_bytes);
  if (e) return e;
  hipLaunchKernelGGL(k, grid, dim3(NW * 64), t.lds_bytes, st, (const float *)d_in, p.in_pitch_bytes / 4,
                     p.desc.n_chan, p.desc.n_samp, p.d_shift, p.desc.n_dm, p.n_out, d_out, out_pitch,
                     t.row_bytes, t.chan_block);
  return (int)hipGetLastError();
}

}  // namespace

int launch_forward(const dd_plan &p, const void *d_in, float *d_out, int64_t out_pitch, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const TileCfg &t = p.fwd;
  if (p.desc.dtype == DD_F32) {
    if (t.ns == 16 && t.waves == 4) {
      switch (t.dm_per_wave) {
        case 4: return launch_f32<16, 4, 4>(p, d_in, d_out, out_pitch, st);
        case 2: return launch_f32<16, 2, 4>(p, d_in, d_out, out_pitch, st);
        case 1: return launch_f32<16, 1, 4>(p, d_in, d_out, out_pitch, st);
      }
    }
    if (t.ns == 16 && t.waves == 2 && t.dm_per_wave == 1) return launch_f32<16, 1, 2>(p, d_in, d_out, out_pitch, st);
    if (t.ns == 16 && t.waves == 1 && t.dm_per_wave == 1) return launch_f32<16, 1, 1>(p, d_in, d_out, out_pitch, st);
    return (int)hipErrorInvalidValue;
  }
  if (t.ns == 32 && t.waves == 4) {
    switch (t.dm_per_wave) {
      case 4: return launch_int<32, 4, 4>(p, d_in, d_out, out_pitch, st);
      case 2: return launch_int<32, 2, 4>(p, d_in, d_out, out_pitch, st);
      case 1: return launch_int<32, 1, 4>(p, d_in, d_out, out_pitch, st);
    }
  }
  if (t.ns == 32 && t.waves == 2 && t.dm_per_wave == 1) return launch_int<32, 1, 2>(p, d_in, d_out, out_pitch, st);
  if (t.ns == 32 && t.waves == 1 && t.dm_per_wave == 1) return launch_int<32, 1, 1>(p, d_in, d_out, out_pitch, st);
  return (int)hipErrorInvalidValue;
}

int launch_adjoint(const dd_plan &p, const float *d_y, int64_t y_pitch, float *d_grad, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  const TileCfg &t = p.adj;
  const int32_t *shift_t = p.d_shift + (size_t)p.desc.n_dm * p.desc.n_chan;
  const int32_t *smax = shift_t + (size_t)p.desc.n_dm * p.desc.n_chan;
  const int cpb = t.waves * t.dm_per_wave;  // channels per workgroup
  dim3 grid((unsigned)((p.desc.n_samp + 64 * t.ns - 1) / (64 * t.ns)), (unsigned)((p.desc.n_chan + cpb - 1) / cpb));
#define DD_ADJ(NS, R, NW)                                                                                   \
  if (t.ns == NS && t.dm_per_wave == R && t.waves == NW) {                                                   \
    auto k = adj_f32_kernel<NS, R, NW>;                                                                       \
    int e = set_lds(k, t.lds_bytes);                                                                          \
    if (e) return e;                                                                                          \
    hipLaunchKernelGGL(k, grid, dim3(NW * 64), t.lds_bytes, st, d_y, y_pitch, p.desc.n_chan,             \
                       p.desc.n_samp, shift_t, smax, p.desc.n_dm, p.n_out, d_grad, p.in_pitch_bytes / 4,     \
                       t.row_bytes, t.chan_block);                                                            \
    return (int)hipGetLastError();                                                                           \
  }
  DD_ADJ(16, 4, 4)
  DD_ADJ(16, 2, 4)
  DD_ADJ(16, 1, 4)
  DD_ADJ(16, 1, 2)
  DD_ADJ(16, 1, 1)
#undef DD_ADJ
  return (int)hipErrorInvalidValue;
}

int batch_kernels(int ns, int dm_per_wave, int waves, bool u4, int lds_bytes, BatchLaunch *out) {
  const void *fn = nullptr;
#define DD_BATCH(NS, R, NW)                                                             \
  if (ns == NS && dm_per_wave == R && waves == NW) {                                    \
    fn = u4 ? (const void *)fwd_int_batched_kernel<NS, R, NW, true>                      \
            : (const void *)fwd_int_batched_kernel<NS, R, NW, false>;                    \
  }
  DD_BATCH(32, 4, 4)
  DD_BATCH(32, 2, 4)
  DD_BATCH(32, 1, 4)
#undef DD_BATCH
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
