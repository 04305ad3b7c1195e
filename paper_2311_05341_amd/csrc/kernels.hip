// Float forward and adjoint dedispersion kernels for gfx950 (CDNA4, wave64).
//
// Forward (Sec. 2, Eq. 3): S(d, t) = sum_c x(c, t + shift(c, d)).  A
// workgroup owns (waves * R) DM rows by 64*NS output samples; channel blocks
// are staged in LDS starting at the tile's first-DM delay rounded down to 4
// floats, so every staged sample serves all the tile's DM rows (Sec. 4.1).
// Float rows are 4-byte granular, so a lane's window is always word aligned:
// it reads aligned 16-byte chunks and the wave-uniform word offset selects one
// of four unrolled variants.
//
// Float sums use a fixed order that depends only on the channel (forward) or
// DM (adjoint) index: groups of 32 summed in order, then the group sums in
// order.  Results are bitwise independent of the tile shape.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dd_internal.h"

namespace dd {
namespace {

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
  return launch_forward_int(p, d_in, d_out, out_pitch, stream);
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

}  // namespace dd
