// Time binning ("downsampling", applied before the transform for high-DM
// ranges in Secs. 5.2 and 5.3 and counted in the real-time factor of Sec. 5.5):
//
//     out(c, j) = sum_{i < F} x(c, j*F + i),   0 <= j < n_bins = n_samp / F.
//
// 8- and 4-bit input gives exact uint16 sums (F <= 256 keeps them below 2^16);
// 16-bit input gives float32 holding exact integer sums (below 2^24); float32
// input gives float32 sums in an order fixed by F.
//
// These are streaming kernels bound by HBM: every input byte of the whole bins
// is read once with 16-byte loads that are contiguous across a wave, every
// output written once.  A workgroup takes 256 * 4 consecutive units of one row
// (unit = one 16-byte input chunk, or one bin for the generic kernel); grid y
// walks the channel rows.
//
//   bin_chunk_kernel  F divides the samples of a chunk: one lane turns its
//                     chunk into whole bins (SWAR adds for 8- and 4-bit data).
//   bin_group_kernel  F a larger power of two: L = F / (samples per chunk)
//                     consecutive lanes each sum one chunk, then add across
//                     the group with cross-lane shuffles.
//   bin_any_kernel    any other F: one lane per bin, one sample at a time.
#include <hip/hip_runtime.h>

#include "dd_internal.h"

namespace dd {
namespace {

constexpr int kBinThreads = 256;
constexpr int kBinUnits = 4;  // units per thread

struct BinArgs {
  const uint8_t *in;
  int64_t in_pitch;  // bytes
  uint8_t *out;
  int64_t out_pitch;  // bytes
  int n_chan;
  int64_t n_bins;
  int64_t n_units;  // units of work per row (chunks, or bins for the generic kernel)
  int factor;
};

template <int DT>
struct BinTraits;
template <>
struct BinTraits<DD_U8> {
  static constexpr int kSamples = 16;  // samples per 16-byte chunk
  using Out = uint16_t;
};
template <>
struct BinTraits<DD_U4> {
  static constexpr int kSamples = 32;
  using Out = uint16_t;
};
template <>
struct BinTraits<DD_U16> {
  static constexpr int kSamples = 8;
  using Out = float;
};
template <>
struct BinTraits<DD_F32> {
  static constexpr int kSamples = 4;
  using Out = float;
};

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// Bins of F consecutive 8-bit samples held in bytes of w[0..3] (byte order =
// time order); each bin sum < 2^16.  Writes 16 / F uint16 results to o.
template <int F>
__device__ __forceinline__ void bins_of_bytes(const uint32_t (&w)[4], uint16_t *o) {
  if constexpr (F == 1) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t a = perm(w[k], w[k], 0x0C010C00u), b = perm(w[k], w[k], 0x0C030C02u);
      o[4 * k + 0] = (uint16_t)a;
      o[4 * k + 1] = (uint16_t)(a >> 16);
      o[4 * k + 2] = (uint16_t)b;
      o[4 * k + 3] = (uint16_t)(b >> 16);
    }
  } else {
    // pair sums as two 16-bit lanes per word: [x0 + x1, x2 + x3]
    uint32_t p[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = (w[k] & 0x00FF00FFu) + ((w[k] >> 8) & 0x00FF00FFu);
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = p[k] & 0xFFFFu;
      v[2 * k + 1] = p[k] >> 16;
    }
    constexpr int G = F / 2;  // pair sums per bin
#pragma unroll
    for (int b = 0; b < 8 / G; ++b) {
      uint32_t s = 0;
#pragma unroll
      for (int i = 0; i < G; ++i) s += v[b * G + i];
      o[b] = (uint16_t)s;
    }
  }
}

template <int DT, int F>
__device__ __forceinline__ void chunk_bins(uint4 c, typename BinTraits<DT>::Out *o) {
  const uint32_t w[4] = {c.x, c.y, c.z, c.w};
  if constexpr (DT == DD_U8) {
    bins_of_bytes<F>(w, o);
  } else if constexpr (DT == DD_U4) {
    // even samples in the low nibbles, odd in the high ones
    uint32_t e[4], d[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      e[k] = w[k] & 0x0F0F0F0Fu;
      d[k] = (w[k] >> 4) & 0x0F0F0F0Fu;
    }
    if constexpr (F == 1) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t q[4] = {perm(d[k], e[k], 0x0C040C00u), perm(d[k], e[k], 0x0C050C01u),
                               perm(d[k], e[k], 0x0C060C02u), perm(d[k], e[k], 0x0C070C03u)};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          o[8 * k + 2 * i] = (uint16_t)q[i];
          o[8 * k + 2 * i + 1] = (uint16_t)(q[i] >> 16);
        }
      }
    } else {
      uint32_t s[4];  // byte b of s[k] = the pair (2b, 2b+1) of word k, at most 30
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k] = e[k] + d[k];
      bins_of_bytes<F / 2>(s, o);
    }
  } else if constexpr (DT == DD_U16) {
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = w[k] & 0xFFFFu;
      v[2 * k + 1] = w[k] >> 16;
    }
#pragma unroll
    for (int b = 0; b < 8 / F; ++b) {
      uint32_t s = 0;
#pragma unroll
      for (int i = 0; i < F; ++i) s += v[b * F + i];
      o[b] = (float)s;
    }
  } else {
    const float v[4] = {__uint_as_float(c.x), __uint_as_float(c.y), __uint_as_float(c.z), __uint_as_float(c.w)};
#pragma unroll
    for (int b = 0; b < 4 / F; ++b) {
      float s = v[b * F];
#pragma unroll
      for (int i = 1; i < F; ++i) s += v[b * F + i];
      o[b] = s;
    }
  }
}

// Store n outputs (all when whole) of one chunk; `dst` is 2*sizeof(o) aligned
// when n_full outputs are stored as one vector.
template <typename T, int N>
__device__ __forceinline__ void store_bins(T *dst, const T *o, int n) {
  if (n >= N) {
    if constexpr (N * sizeof(T) % 16 == 0) {
#pragma unroll
      for (int i = 0; i < (int)(N * sizeof(T) / 16); ++i) {
        uint4 q;
        __builtin_memcpy(&q, (const uint8_t *)o + 16 * i, 16);
        ((uint4 *)dst)[i] = q;
      }
    } else if constexpr (N * sizeof(T) == 8) {
      uint2 q;
      __builtin_memcpy(&q, o, 8);
      *(uint2 *)dst = q;
    } else if constexpr (N * sizeof(T) == 4) {
      uint32_t q;
      __builtin_memcpy(&q, o, 4);
      *(uint32_t *)dst = q;
    } else {
      dst[0] = o[0];
    }
  } else {
    for (int i = 0; i < n; ++i) dst[i] = o[i];
  }
}

template <int DT, int F>
__global__ __launch_bounds__(kBinThreads) void bin_chunk_kernel(BinArgs a) {
  using Out = typename BinTraits<DT>::Out;
  constexpr int S = BinTraits<DT>::kSamples;
  constexpr int O = S / F;  // bins per chunk
  for (int c = blockIdx.y; c < a.n_chan; c += gridDim.y) {
    const uint4 *row = (const uint4 *)(a.in + (int64_t)c * a.in_pitch);
    Out *orow = (Out *)(a.out + (int64_t)c * a.out_pitch);
    const int64_t k0 = (int64_t)blockIdx.x * (kBinThreads * kBinUnits) + threadIdx.x;
    uint4 w[kBinUnits];
#pragma unroll
    for (int u = 0; u < kBinUnits; ++u) {
      const int64_t k = k0 + u * kBinThreads;
      if (k < a.n_units) w[u] = row[k];
    }
#pragma unroll
    for (int u = 0; u < kBinUnits; ++u) {
      const int64_t k = k0 + u * kBinThreads;
      if (k < a.n_units) {
        Out o[O];
        chunk_bins<DT, F>(w[u], o);
        const int64_t j0 = k * O;
        const int64_t left = a.n_bins - j0;
        store_bins<Out, O>(orow + j0, o, left < O ? (int)left : O);
      }
    }
  }
}

template <int DT>
__device__ __forceinline__ auto chunk_total(uint4 c) {
  if constexpr (DT == DD_U8) {
    uint32_t s = __builtin_amdgcn_sad_u8(c.x, 0u, 0u);
    s = __builtin_amdgcn_sad_u8(c.y, 0u, s);
    s = __builtin_amdgcn_sad_u8(c.z, 0u, s);
    return __builtin_amdgcn_sad_u8(c.w, 0u, s);
  } else if constexpr (DT == DD_U4) {
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) s = __builtin_amdgcn_sad_u8((w[k] & 0x0F0F0F0Fu) + ((w[k] >> 4) & 0x0F0F0F0Fu), 0u, s);
    return s;
  } else if constexpr (DT == DD_U16) {
    return (c.x & 0xFFFFu) + (c.x >> 16) + (c.y & 0xFFFFu) + (c.y >> 16) + (c.z & 0xFFFFu) + (c.z >> 16) +
           (c.w & 0xFFFFu) + (c.w >> 16);
  } else {
    return ((__uint_as_float(c.x) + __uint_as_float(c.y)) + __uint_as_float(c.z)) + __uint_as_float(c.w);
  }
}

template <int DT, int L>
__global__ __launch_bounds__(kBinThreads) void bin_group_kernel(BinArgs a) {
  using Out = typename BinTraits<DT>::Out;
  for (int c = blockIdx.y; c < a.n_chan; c += gridDim.y) {
    const uint4 *row = (const uint4 *)(a.in + (int64_t)c * a.in_pitch);
    Out *orow = (Out *)(a.out + (int64_t)c * a.out_pitch);
    const int64_t k0 = (int64_t)blockIdx.x * (kBinThreads * kBinUnits) + threadIdx.x;
    uint4 w[kBinUnits];
#pragma unroll
    for (int u = 0; u < kBinUnits; ++u) {
      const int64_t k = k0 + u * kBinThreads;
      w[u] = k < a.n_units ? row[k] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < kBinUnits; ++u) {
      // n_units is a multiple of L and groups are L-aligned: a group is wholly
      // in range or wholly out, and every lane takes part in the shuffles.
      const int64_t k = k0 + u * kBinThreads;
      auto s = chunk_total<DT>(w[u]);
#pragma unroll
      for (int m = L / 2; m >= 1; m >>= 1) s += __shfl_xor(s, m);
      if (k < a.n_units && (k & (L - 1)) == 0) orow[k / L] = (Out)s;
    }
  }
}

template <int DT>
__device__ __forceinline__ uint32_t int_sample(const uint8_t *row, int64_t t) {
  if constexpr (DT == DD_U8) return row[t];
  else if constexpr (DT == DD_U4) return (row[t >> 1] >> (4 * (t & 1))) & 15u;
  else return ((const uint16_t *)row)[t];
}

template <int DT>
__global__ __launch_bounds__(kBinThreads) void bin_any_kernel(BinArgs a) {
  using Out = typename BinTraits<DT>::Out;
  for (int c = blockIdx.y; c < a.n_chan; c += gridDim.y) {
    const uint8_t *row = a.in + (int64_t)c * a.in_pitch;
    Out *orow = (Out *)(a.out + (int64_t)c * a.out_pitch);
    const int64_t j0 = (int64_t)blockIdx.x * (kBinThreads * kBinUnits) + threadIdx.x;
    for (int u = 0; u < kBinUnits; ++u) {
      const int64_t j = j0 + u * kBinThreads;
      if (j >= a.n_bins) break;
      const int64_t t0 = j * a.factor;
      if constexpr (DT == DD_F32) {
        const float *r = (const float *)row;
        float s = r[t0];
        for (int i = 1; i < a.factor; ++i) s += r[t0 + i];
        orow[j] = s;
      } else {
        uint32_t s = 0;
        for (int i = 0; i < a.factor; ++i) s += int_sample<DT>(row, t0 + i);
        orow[j] = (Out)s;
      }
    }
  }
}

// 16-bit input binned into two uint16 planes: the low and high halves of
// every exact bin sum (below 2^24 for F <= 256, so the high half is at most
// 255).  The transform then sums each plane exactly in 32-bit integers and
// combines them once (OutMode in dd_internal.h).  Row c of the low plane is at
// out + c * out_pitch, of the high plane `hi_off` bytes further.  One lane per
// bin; the bin's 2F bytes are read as whole words where F allows.
__global__ __launch_bounds__(kBinThreads) void bin_u16_split_kernel(BinArgs a, int64_t hi_off) {
  const int f = a.factor;
  for (int c = blockIdx.y; c < a.n_chan; c += gridDim.y) {
    const uint8_t *row = a.in + (int64_t)c * a.in_pitch;
    uint16_t *lo = (uint16_t *)(a.out + (int64_t)c * a.out_pitch);
    uint16_t *hi = (uint16_t *)(a.out + (int64_t)c * a.out_pitch + hi_off);
    const int64_t j0 = (int64_t)blockIdx.x * (kBinThreads * kBinUnits) + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kBinUnits; ++u) {
      const int64_t j = j0 + u * kBinThreads;
      if (j >= a.n_bins) break;
      const uint8_t *b = row + 2 * j * f;  // 16-byte aligned when f % 8 == 0, 4-byte when f is even
      uint32_t s = 0;
      if (f % 8 == 0) {
        for (int i = 0; i < f; i += 8) {
          const uint4 w = *(const uint4 *)(b + 2 * i);
          s += (w.x & 0xFFFFu) + (w.x >> 16) + (w.y & 0xFFFFu) + (w.y >> 16) + (w.z & 0xFFFFu) + (w.z >> 16) +
               (w.w & 0xFFFFu) + (w.w >> 16);
        }
      } else if (f % 2 == 0) {
        for (int i = 0; i < f; i += 2) {
          const uint32_t w = *(const uint32_t *)(b + 2 * i);
          s += (w & 0xFFFFu) + (w >> 16);
        }
      } else {
        for (int i = 0; i < f; ++i) s += ((const uint16_t *)b)[i];
      }
      lo[j] = (uint16_t)s;
      hi[j] = (uint16_t)(s >> 16);
    }
  }
}

using BinKernel = void (*)(BinArgs);

template <int DT, int F>
constexpr BinKernel chunk_or_group() {
  constexpr int S = BinTraits<DT>::kSamples;
  if constexpr (F <= S) return bin_chunk_kernel<DT, F>;
  else return bin_group_kernel<DT, F / S>;
}

// Power-of-two factors 1..256 for one input type.
template <int DT>
BinKernel pick_pow2(int f, int *unit_samples) {
  *unit_samples = BinTraits<DT>::kSamples;
  switch (f) {
    case 1: return chunk_or_group<DT, 1>();
    case 2: return chunk_or_group<DT, 2>();
    case 4: return chunk_or_group<DT, 4>();
    case 8: return chunk_or_group<DT, 8>();
    case 16: return chunk_or_group<DT, 16>();
    case 32: return chunk_or_group<DT, 32>();
    case 64: return chunk_or_group<DT, 64>();
    case 128: return chunk_or_group<DT, 128>();
    case 256: return chunk_or_group<DT, 256>();
  }
  return nullptr;
}

}  // namespace

int bin_out_bytes(int dtype) { return dtype == DD_U8 || dtype == DD_U4 ? 2 : 4; }

int launch_bin(int dtype, const void *in, int64_t in_pitch, int n_chan, int64_t n_samp, int factor, void *out,
               int64_t out_pitch, void *stream) {
  BinArgs a;
  a.in = (const uint8_t *)in;
  a.in_pitch = in_pitch;
  a.out = (uint8_t *)out;
  a.out_pitch = out_pitch;
  a.n_chan = n_chan;
  a.n_bins = n_samp / factor;
  a.factor = factor;
  BinKernel k = nullptr;
  int unit = 0;
  if ((factor & (factor - 1)) == 0) {
    switch (dtype) {
      case DD_U8: k = pick_pow2<DD_U8>(factor, &unit); break;
      case DD_U4: k = pick_pow2<DD_U4>(factor, &unit); break;
      case DD_U16: k = pick_pow2<DD_U16>(factor, &unit); break;
      case DD_F32: k = pick_pow2<DD_F32>(factor, &unit); break;
    }
  }
  if (k) {
    // chunks covering the whole bins (chunk kernel), or exactly L chunks per bin
    a.n_units = factor <= unit ? (a.n_bins * factor + unit - 1) / unit : a.n_bins * (factor / unit);
  } else {
    switch (dtype) {
      case DD_U8: k = bin_any_kernel<DD_U8>; break;
      case DD_U4: k = bin_any_kernel<DD_U4>; break;
      case DD_U16: k = bin_any_kernel<DD_U16>; break;
      case DD_F32: k = bin_any_kernel<DD_F32>; break;
      default: return (int)hipErrorInvalidValue;
    }
    a.n_units = a.n_bins;
  }
  const int64_t per_block = (int64_t)kBinThreads * kBinUnits;
  const dim3 grid((unsigned)((a.n_units + per_block - 1) / per_block), (unsigned)(n_chan < 65535 ? n_chan : 65535));
  hipLaunchKernelGGL(k, grid, dim3(kBinThreads), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_bin_u16_split(const void *in, int64_t in_pitch, int n_chan, int64_t n_samp, int factor, void *out,
                         int64_t out_pitch, int64_t hi_off, void *stream) {
  BinArgs a;
  a.in = (const uint8_t *)in;
  a.in_pitch = in_pitch;
  a.out = (uint8_t *)out;
  a.out_pitch = out_pitch;
  a.n_chan = n_chan;
  a.n_bins = n_samp / factor;
  a.n_units = a.n_bins;
  a.factor = factor;
  const int64_t per_block = (int64_t)kBinThreads * kBinUnits;
  const dim3 grid((unsigned)((a.n_bins + per_block - 1) / per_block), (unsigned)(n_chan < 65535 ? n_chan : 65535));
  hipLaunchKernelGGL(bin_u16_split_kernel, grid, dim3(kBinThreads), 0, (hipStream_t)stream, a, hi_off);
  return (int)hipGetLastError();
}

}  // namespace dd
