// Direct-read forward transform for integer input: the fallback for plans
// whose delay spread across a DM block is too wide for LDS staging to pay.
//
// The LDS kernel stages, per channel, the union of the windows of a block's
// DM rows: T + spread samples for T outputs.  When the delay grows by hundreds
// of samples per DM step (low frequencies, coarse steps) that union is mostly
// spread, each staged byte serves one or two DM rows, and building its byte
// phases costs more than it saves.  This kernel reads every (channel, DM)
// window straight from global memory instead and leaves the reuse between
// neighbouring DM rows, whose windows overlap, to the L1 and L2 caches (the
// cache-based variant of the paper's GPU implementation, Sec. 4; its results
// cite a slowdown of up to 4x for it).
//
// Windows start at any sample, but the loads stay 4-byte aligned: a lane
// loads the aligned words covering its 16-byte (8-bit input; 32-byte for
// 16-bit) window, takes the word after them from the next lane (a wave shift,
// DPP), and funnel-shifts them (v_alignbit, by a wave-uniform bit count) into
// the window's words.  Lane 63 has no next lane: it loads its window only for
// lane 62 and produces no output, so a wave covers 63 lanes' samples and every
// (channel, DM) window costs one vector load instruction per 16 bytes.  Each
// channel gets one raw buffer descriptor spanning its row pitch; a window's
// aligned delay offset is added to the per-lane offset, and the loads pass no
// scalar offset (which the hardware would not range-check): the bound is
// checked against the whole offset, so every byte past the row pitch reads as
// zero and no read can leave the input.  In the last time tile, where a lane's
// window may run past the row, the words are loaded one by one: a
// 4-byte-aligned word lies wholly inside or wholly outside the bound (both the
// pitch and the delay offset are multiples of 4 bytes), so the bound check
// never drops bytes a valid output needs.  The delays of 8 channels come with
// one scalar load per DM row, and the row pointer steps by the pitch: the
// kernel's scalar work per window is a few instructions.
//
// Accumulation is the same exact SIMD-in-word arithmetic as the LDS kernels:
// 8-bit words as mix/odd pairs flushed every 256 channels, 4-bit words as even
// nibbles (E) and the word shifted down a nibble (S) flushed every 16 channels,
// 16-bit words as mix and high halves.
//
// A workgroup covers NW * R DM rows x 63 * NS samples; wave w owns R rows, lane
// i < 63 samples NS*i .. NS*i + NS-1 of the tile (NS = 16, or 32 for 4-bit input).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dd_internal.h"
#include "tile_order.h"

namespace dd {
namespace {

constexpr uint32_t kOdd = 0x0C030C01u;  // v_perm: bytes 1 and 3 into bytes 0 and 2
constexpr int kRsrcWord3 = 0x00020000;  // raw (untyped) buffer access
constexpr int kUnroll = 2;              // channels whose loads are issued together
constexpr int kOutLanes = 63;           // lanes of a wave that produce output (lane 63 only loads)

struct DirectArgs {
  const uint8_t *x;      // [n_chan][pitch] bytes
  const int32_t *shift;  // [n_dm][n_chan]
  float *out;            // [n_dm][out_pitch]
  int64_t pitch, n_out, out_pitch;
  int32_t n_chan, n_dm;
  int32_t out_mode;  // an OutMode; other than kOutFloat for 16-bit input only
};

// Output of one exact total by OutMode (see fwd_int.hip): float32, the raw
// 32-bit total, or low (read back) + 2^16 * this total converted once.
__device__ __forceinline__ void store_total(float *o, uint32_t v, int mode) {
  if (mode == kOutRawTotals)
    *(uint32_t *)o = v;
  else if (mode == kOutCombineHigh)
    *o = (float)((double)*(const uint32_t *)o + 65536.0 * (double)v);
  else
    *o = (float)v;
}

// acc + byte M of w (zero-extended): one SDWA add.
template <int M>
__device__ __forceinline__ uint32_t add_byte(uint32_t acc, uint32_t w) {
  uint32_t r;
  if constexpr (M == 0)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
        : "=v"(r) : "v"(acc), "v"(w));
  else if constexpr (M == 1)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
        : "=v"(r) : "v"(acc), "v"(w));
  else if constexpr (M == 2)
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
        : "=v"(r) : "v"(acc), "v"(w));
  else
    asm("v_add_u32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
        : "=v"(r) : "v"(acc), "v"(w));
  return r;
}

template <typename T>
__device__ __forceinline__ T scalar_load(const T *p, int64_t i) {
  return ((const __attribute__((address_space(4))) T *)p)[i];
}

typedef int v4i __attribute__((ext_vector_type(4)));

template <int BITS>
constexpr int lane_samples() { return BITS == 4 ? 32 : 16; }

typedef int32_t v8i32 __attribute__((ext_vector_type(8), aligned(4)));  // rows of the delay table are only 4-byte aligned
constexpr int kDelayChunk = 8;  // channels whose delays one scalar load per row reads

// The sums of one wave's R rows over every channel (see the file comment): per
// chunk of 8 channels one scalar load per row reads their delays; per channel
// one buffer descriptor spans its row pitch (an empty one for the unrolled tail
// past the block's last channel, which reads zeros), and each window's aligned
// delay offset goes into the range-checked per-lane offset.  LAST loads the
// words one by one (the last time tile, where windows may run past the row).
template <int BITS, int R, bool LAST>
__device__ __forceinline__ void direct_channels(const DirectArgs &a, const int (&drow)[R], uint32_t vo,
                                                uint32_t (&tot)[R][lane_samples<BITS>()],
                                                uint32_t (&mix)[R][lane_samples<BITS>() * BITS / 32],
                                                uint32_t (&odd)[R][lane_samples<BITS>() * BITS / 32]) {
  constexpr int NS = lane_samples<BITS>();
  constexpr int WORDS = NS * BITS / 32;  // window words per lane (4, or 8 for 16-bit)
  // channels between exact flushes: 256 for bytes, 16 for nibbles (no byte lane of E above 255)
  constexpr int kFlush = BITS == 16 ? (1 << 30) : BITS == 4 ? 16 : 256;
  static_assert(kFlush % kDelayChunk == 0, "flush blocks hold whole delay chunks");
  const int32_t *srow[R];
#pragma unroll
  for (int r = 0; r < R; ++r) srow[r] = a.shift + (int64_t)drow[r] * a.n_chan;
  for (int cb = 0; cb < a.n_chan; cb += kFlush) {
    const int ce = min(cb + kFlush, a.n_chan);
    for (int c0 = cb; c0 < ce; c0 += kDelayChunk) {
      const int nc = min(kDelayChunk, ce - c0);  // wave-uniform
      // FULL: a whole chunk in straight-line code, so the next pair's loads can be issued
      // early.  Only for 2-row waves: with 4 rows the extra registers cost occupancy
      // (measured on 4096 ch u8 x 2^20, 120-190 MHz: 4 rows x 4 waves 110.2 ms with a
      // branch per channel pair against 134.8 ms straight; 2 x 8: 155.7 against 127.5).
      auto chunk = [&](auto full) {
        constexpr bool FULL = decltype(full)::value;
        int dl[R][kDelayChunk];
        if (FULL || nc == kDelayChunk) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const v8i32 v = *(const __attribute__((address_space(4))) v8i32 *)(srow[r] + c0);
#pragma unroll
            for (int q = 0; q < kDelayChunk; ++q) dl[r][q] = v[q];
          }
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int q = 0; q < kDelayChunk; ++q) dl[r][q] = scalar_load(srow[r], c0 + min(q, nc - 1));
        }
        const uint8_t *row = a.x + (int64_t)c0 * a.pitch;
#pragma unroll
        for (int q0 = 0; q0 < kDelayChunk; q0 += kUnroll) {
          if (!FULL && q0 >= nc) break;
          uint32_t raw[kUnroll][R][WORDS + 1];
          int sh[kUnroll][R];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const bool live = FULL || q0 + u < nc;  // wave-uniform
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void *)row, (short)0, live ? (int)a.pitch : 0, kRsrcWord3);
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const int64_t bit = (int64_t)dl[r][q0 + u] * BITS;  // bit offset of the delay
              const uint32_t off = vo + (uint32_t)(bit >> 5) * 4;  // aligned byte offset, range-checked
              sh[u][r] = (int)(bit & 31);
              if constexpr (!LAST) {
#pragma unroll
                for (int q = 0; q < WORDS / 4; ++q) {
                  const v4i v = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16 * q, 0, 0);
                  raw[u][r][4 * q] = v.x;
                  raw[u][r][4 * q + 1] = v.y;
                  raw[u][r][4 * q + 2] = v.z;
                  raw[u][r][4 * q + 3] = v.w;
                }
              } else {
#pragma unroll
                for (int q = 0; q < WORDS; ++q) raw[u][r][q] = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4 * q, 0, 0);
              }
            }
            if (live) row += a.pitch;
          }
          // The word after a lane's window is the next lane's first word (a wave shift, DPP);
          // lane 63 gets zero and its sums are never stored.
#pragma unroll
          for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r)  // wave_shl:1
              raw[u][r][WORDS] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)raw[u][r][0], 0x130, 0xF, 0xF, false);
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
#pragma unroll
              for (int k = 0; k < WORDS; ++k) {
                const uint32_t v = __builtin_amdgcn_alignbit(raw[u][r][k + 1], raw[u][r][k], sh[u][r]);
                if constexpr (BITS == 8) {
                  mix[r][k] += v;
                  odd[r][k] += __builtin_amdgcn_perm(v, v, kOdd);
                } else if constexpr (BITS == 16) {
                  mix[r][k] += v;
                  odd[r][k] += v >> 16;
                } else {  // nibbles: E = even nibbles in the byte lanes, S = the word shifted down a nibble
                  mix[r][k] += v & 0x0F0F0F0Fu;
                  odd[r][k] += v >> 4;
                }
              }
            }
          }
        }
      };
      if (R <= 2 && nc == kDelayChunk)
        chunk(std::true_type{});
      else
        chunk(std::false_type{});
    }
    // Flush the block of channels into the int32 totals.  Bytes:
    // mix - (odd << 8) = sum of bytes 0 + 2^16 * sum of bytes 2 (each sum < 2^16).
    if constexpr (BITS == 8) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < WORDS; ++k) {
          const uint32_t e = mix[r][k] - (odd[r][k] << 8), o = odd[r][k];
          tot[r][4 * k] += e & 0xFFFFu;
          tot[r][4 * k + 1] += o & 0xFFFFu;
          tot[r][4 * k + 2] += e >> 16;
          tot[r][4 * k + 3] += o >> 16;
          mix[r][k] = odd[r][k] = 0;
        }
    } else if constexpr (BITS == 4) {
      // word k holds samples 8k .. 8k+7: byte m of E is sample 8k + 2m, byte m of the odd-nibble
      // sums O = S - 16 * (E >> 8) is sample 8k + 2m + 1 (no byte lane above 255 after 16 channels)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < WORDS; ++k) {
          const uint32_t e = mix[r][k], o = odd[r][k] - ((e >> 4) & 0x0FFFFFF0u);
          uint32_t *t = tot[r] + 8 * k;
          t[0] = add_byte<0>(t[0], e);
          t[2] = add_byte<1>(t[2], e);
          t[4] = add_byte<2>(t[4], e);
          t[6] = add_byte<3>(t[6], e);
          t[1] = add_byte<0>(t[1], o);
          t[3] = add_byte<1>(t[3], o);
          t[5] = add_byte<2>(t[5], o);
          t[7] = add_byte<3>(t[7], o);
          mix[r][k] = odd[r][k] = 0;
        }
    }
  }
}

// One tile: DM block dblk (NW * R rows) x time tile tblk (63 * NS samples).
// No LDS and no barrier.
template <int BITS, int R, int NW>
__device__ __forceinline__ void direct_tile(const DirectArgs &a, int dblk, int tblk) {
  constexpr int NS = lane_samples<BITS>();
  constexpr int WORDS = NS * BITS / 32;  // window words per lane (4, or 8 for 16-bit)
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int d0 = (dblk * NW + w) * R;
  const int64_t t0 = (int64_t)tblk * kOutLanes * NS;
  const uint32_t vo = (uint32_t)((t0 + NS * lane) * BITS / 8);  // byte of the lane's first sample
  const bool last_tile = t0 + 64 * NS > a.n_out;                 // wave-uniform; lane 63's window too
  int drow[R];
#pragma unroll
  for (int r = 0; r < R; ++r) drow[r] = min(d0 + r, a.n_dm - 1);

  // Totals per row and sample.  8-bit: exact int32; 4-bit: likewise; 16-bit: the
  // word sums themselves (mix) and the high-half sums (hi), resolved at the end.
  uint32_t tot[R][NS];
  uint32_t mix[R][WORDS], odd[R][WORDS];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int k = 0; k < NS; ++k) tot[r][k] = 0;
#pragma unroll
    for (int k = 0; k < WORDS; ++k) mix[r][k] = odd[r][k] = 0;
  }
  if (last_tile)
    direct_channels<BITS, R, true>(a, drow, vo, tot, mix, odd);
  else
    direct_channels<BITS, R, false>(a, drow, vo, tot, mix, odd);
  if constexpr (BITS == 16) {
    // low samples: mix - (hi << 16) (mod 2^32), exact for up to 65537 channels
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k = 0; k < WORDS; ++k) {
        tot[r][2 * k] = mix[r][k] - (odd[r][k] << 16);
        tot[r][2 * k + 1] = odd[r][k];
      }
  }
  const int64_t tl = t0 + NS * lane;
  if (lane < kOutLanes) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (d0 + r >= a.n_dm) break;
      float *o = a.out + (int64_t)(d0 + r) * a.out_pitch + tl;
      if (BITS == 16 && a.out_mode != kOutFloat) {
        for (int k = 0; k < NS && tl + k < a.n_out; ++k) store_total(o + k, tot[r][k], a.out_mode);
      } else if (tl + NS <= a.n_out) {
#pragma unroll
        for (int k = 0; k < NS; k += 4)
          *(float4 *)(o + k) =
              make_float4((float)tot[r][k], (float)tot[r][k + 1], (float)tot[r][k + 2], (float)tot[r][k + 3]);
      } else {
        for (int k = 0; k < NS && tl + k < a.n_out; ++k) o[k] = (float)tot[r][k];
      }
    }
  }
}

template <int BITS, int R, int NW>
__global__ __launch_bounds__(NW * 64) void fwd_direct_kernel(DirectArgs a, int n_dblk, int n_tiles, int order) {
  int dblk, tblk;
  tile_of((int)blockIdx.x, n_dblk, n_tiles, order, dblk, tblk);
  direct_tile<BITS, R, NW>(a, dblk, tblk);
}

__global__ void reset_direct_counter_kernel(unsigned long long *counter) { *counter = 0ull; }

// Workgroup barrier for the claimed-item slot in LDS (the tiles themselves use
// no LDS; the tile's stores need not have completed).
__device__ __forceinline__ void claim_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Persistent batched direct-read kernel, the counterpart of the staged one in
// fwd_int.hip: workgroups claim (beam, DM block, time tile) work items from a
// device counter (beams in decreasing cost order, DM block fastest inside a
// beam); a beam's delay table is the plain int32 shift table (BeamDesc.offs).
// The claim of the next item is issued when an item starts and read when it
// ends.  A tile has no barrier of its own, so a second barrier after reading
// the claim keeps thread 0 from overwriting it before every wave has read it.
// A workgroup returns at its first claim past the last item: every wave
// reaches the exit.
// Waves per SIMD the batched kernel is held to.  Its claim state costs 8-12
// more VGPRs than the one-launch kernel; on the 8-wave shape for 4-bit samples
// that would leave one resident workgroup per CU instead of two (8 wide-spread
// beams, 1024-2048 ch x 2^18-2^19 at 120-190 MHz: 33.9 -> 27.2 ms when held to
// 4 waves).  The other shapes keep their occupancy as they are (16-bit ones
// held to 4 or 3 waves ran 11% and 8% slower).
template <int BITS, int NW>
constexpr int direct_batched_waves() {
  return NW == 8 && BITS == 4 ? 4 : 1;
}

template <int BITS, int R, int NW>
__global__ __launch_bounds__(NW * 64, (direct_batched_waves<BITS, NW>())) void fwd_direct_batched_kernel(
    const BeamDesc *__restrict__ beams, int n_beams, long long n_items, unsigned long long *__restrict__ counter) {
  __shared__ long long claimed;
  if (threadIdx.x == 0) claimed = (long long)atomicAdd(counter, 1ull);
  claim_barrier();
  long long item = claimed;
  int lo = 0;
  for (;;) {
    item = (long long)(((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)((unsigned long long)item >> 32))
                        << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)item));
    if (item >= n_items) return;
    unsigned long long next = 0;
    if (threadIdx.x == 0) next = atomicAdd(counter, 1ull);  // the following claim, read after this tile
    while (lo + 1 < n_beams && scalar_load(&beams[lo + 1].item_begin, 0) <= item) ++lo;
    const BeamDesc &b = beams[lo];
    const long long k = item - b.item_begin;
    const int tblk = (int)(k / b.tiles_d), dblk = (int)(k - (long long)tblk * b.tiles_d);
    DirectArgs a;
    a.x = b.x;
    a.shift = (const int32_t *)b.offs;
    a.out = b.out;
    a.pitch = b.pitch;
    a.n_out = b.n_out;
    a.out_pitch = b.out_pitch;
    a.n_chan = b.n_chan;
    a.n_dm = b.n_dm;
    a.out_mode = kOutFloat;
    direct_tile<BITS, R, NW>(a, dblk, tblk);
    if (threadIdx.x == 0) claimed = (long long)next;
    claim_barrier();  // publishes the claim
    item = claimed;
    claim_barrier();  // every wave has read it before thread 0 writes the next one
  }
}

// Compiled direct shapes: (samples per lane for 8-bit input, DM rows per wave, waves, 0).
#define DD_DIRECT_SHAPES(X) X(4, 4) X(2, 8)

template <int R, int NW>
int launch_direct_shape(const dd_plan &p, const void *tables, const void *d_in, float *d_out, int64_t out_pitch,
                        hipStream_t st, int64_t out_limit, int out_mode) {
  DirectArgs a;
  a.x = (const uint8_t *)d_in;
  a.shift = (const int32_t *)((const uint8_t *)tables + table_layout(p).int_offs);
  a.out = d_out;
  a.pitch = p.in_pitch_bytes;
  a.n_out = out_limit > 0 && out_limit < p.n_out ? out_limit : p.n_out;
  a.out_pitch = out_pitch;
  a.n_chan = p.desc.n_chan;
  a.n_dm = p.desc.n_dm;
  a.out_mode = out_mode;
  const int bits = p.desc.dtype == DD_U4 ? 4 : p.desc.dtype == DD_U16 ? 16 : 8;
  // every descriptor base row + (delay bytes rounded down to 4) must lie inside the row pitch
  if ((int64_t)p.max_shift * bits / 8 >= p.in_pitch_bytes) return (int)hipErrorInvalidValue;
  const int ns = bits == 4 ? 32 : 16;
  const int64_t tiles_t = (a.n_out + kOutLanes * ns - 1) / (kOutLanes * ns);
  const int64_t n_dblk = (a.n_dm + NW * R - 1) / (NW * R);
  if (tiles_t * n_dblk >= ((int64_t)1 << 31)) return (int)hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)(tiles_t * n_dblk)), block(NW * 64);
  if (bits == 4)
    hipLaunchKernelGGL((fwd_direct_kernel<4, R, NW>), grid, block, 0, st, a, (int)n_dblk, (int)tiles_t, p.fwd.order);
  else if (bits == 16)
    hipLaunchKernelGGL((fwd_direct_kernel<16, R, NW>), grid, block, 0, st, a, (int)n_dblk, (int)tiles_t, p.fwd.order);
  else
    hipLaunchKernelGGL((fwd_direct_kernel<8, R, NW>), grid, block, 0, st, a, (int)n_dblk, (int)tiles_t, p.fwd.order);
  return (int)hipGetLastError();
}

}  // namespace

#define DD_ROW(R, NW) {16, R, NW, 0},
const int kDirectShapes[][4] = {DD_DIRECT_SHAPES(DD_ROW)};
#undef DD_ROW
const int kNumDirectShapes = (int)(sizeof(kDirectShapes) / sizeof(kDirectShapes[0]));

int launch_forward_direct(const dd_plan &p, const void *tables, const void *d_in, float *d_out, int64_t out_pitch,
                          void *stream, int64_t out_limit, int out_mode) {
  const TileCfg &t = p.fwd;
#define DD_TRY(R, NW)                     \
  if (t.dm_per_wave == R && t.waves == NW) \
    return launch_direct_shape<R, NW>(p, tables, d_in, d_out, out_pitch, (hipStream_t)stream, out_limit, out_mode);
  DD_DIRECT_SHAPES(DD_TRY)
#undef DD_TRY
  return (int)hipErrorInvalidValue;
}

int direct_tile_samples(int dtype) {
  return kOutLanes * (dtype == DD_U4 ? lane_samples<4>() : dtype == DD_U16 ? lane_samples<16>() : lane_samples<8>());
}

int batch_direct_kernels(int dm_per_wave, int waves, int dtype, BatchLaunch *out) {
  const void *fn = nullptr;
#define DD_TRY(R, NW)                                                                                    \
  if (dm_per_wave == R && waves == NW)                                                                   \
    fn = dtype == DD_U4    ? (const void *)fwd_direct_batched_kernel<4, R, NW>                           \
         : dtype == DD_U16 ? (const void *)fwd_direct_batched_kernel<16, R, NW>                          \
                           : (const void *)fwd_direct_batched_kernel<8, R, NW>;
  DD_DIRECT_SHAPES(DD_TRY)
#undef DD_TRY
  if (!fn) return (int)hipErrorInvalidValue;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, waves * 64, 0);
  if (e != hipSuccess) return (int)e;
  int dev = 0, n_cu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  out->reset_fn = (const void *)reset_direct_counter_kernel;
  out->main_fn = fn;
  out->grid = n_cu * (per_cu > 0 ? per_cu : 1);
  out->block = waves * 64;
  out->lds_bytes = 0;
  return 0;
}

}  // namespace dd
