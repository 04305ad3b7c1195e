// Corner turn of the input: time-major spectra in[t][c] (as telescopes write
// them) to the channel-major rows out[c][t] the transform reads (the input
// transpose of the pipelines in Sec. 5.3, counted in the real-time factor of
// Sec. 5.5).  For 4-bit data a spectrum packs channel pairs into a byte and an
// output row packs time pairs, the even index in the low nibble.
//
// An HBM-bound LDS-tiled transpose.  A workgroup of 256 lanes takes a tile of
// TC channels x TT samples: it reads the tile's TT spectrum segments of 256
// bytes with 16-byte loads (16 lanes per segment, 8 loads in flight per lane)
// into LDS rows padded by 16 bytes, then writes TC output segments of 128 bytes,
// each lane assembling 16-byte pieces of one channel row from LDS element reads
// (consecutive lanes take consecutive channels: conflict-free byte reads).
// Workgroups walk the channel tiles of one time tile consecutively, so the
// spectra are read as contiguous runs.
#include <hip/hip_runtime.h>

#include "dd_internal.h"

namespace dd {
namespace {

constexpr int kCtThreads = 256;

template <int DT>
struct CtGeom;
// TC channels, TT samples per tile; 256 input bytes per spectrum segment and 128
// output bytes per row segment for every type.
template <>
struct CtGeom<DD_U8> {
  static constexpr int TC = 256, TT = 128, ES = 1;
};
template <>
struct CtGeom<DD_U16> {
  static constexpr int TC = 128, TT = 64, ES = 2;
};
template <>
struct CtGeom<DD_F32> {
  static constexpr int TC = 64, TT = 32, ES = 4;
};
template <>
struct CtGeom<DD_U4> {
  static constexpr int TC = 256, TT = 256, ES = 0;  // half-byte elements
};

struct CtArgs {
  const uint8_t *in;
  int64_t in_pitch;  // bytes between spectra
  uint8_t *out;
  int64_t out_pitch;  // bytes between channel rows
  int n_chan;
  int64_t n_samp;
  int64_t in_row_bytes;   // bytes of one spectrum
  int64_t out_row_bytes;  // bytes of one channel row
  int n_ctiles;
};

template <int DT>
__global__ __launch_bounds__(kCtThreads) void corner_turn_kernel(CtArgs a) {
  using G = CtGeom<DT>;
  constexpr int kInSeg = DT == DD_U4 ? G::TC / 2 : G::TC * G::ES;   // bytes of a spectrum segment
  constexpr int kOutSeg = DT == DD_U4 ? G::TT / 2 : G::TT * G::ES;  // bytes of a row segment
  constexpr int kPitch = kInSeg + 16;                                // LDS row pitch
  constexpr int kInChunks = G::TT * (kInSeg / 16);
  constexpr int kOutChunks = G::TC * (kOutSeg / 16);
  static_assert(kInChunks % kCtThreads == 0 && kOutChunks % kCtThreads == 0, "tile shape");
  __shared__ __attribute__((aligned(16))) uint8_t tile[G::TT * kPitch];

  const int ct = (int)(blockIdx.x % (unsigned)a.n_ctiles);
  const int64_t tt = blockIdx.x / (unsigned)a.n_ctiles;
  const int64_t t0 = tt * G::TT;
  const int64_t b0 = (int64_t)ct * kInSeg;  // first byte of the tile in a spectrum
  const int c0 = ct * G::TC;

  // Read: chunk q covers bytes 16*(q % S) of spectrum t0 + q / S (S = chunks per segment).
  constexpr int S = kInSeg / 16;
  uint4 v[kInChunks / kCtThreads];
#pragma unroll
  for (int k = 0; k < kInChunks / kCtThreads; ++k) {
    const int q = threadIdx.x + k * kCtThreads;
    const int64_t t = t0 + q / S;
    const int64_t b = b0 + 16 * (q % S);
    // A chunk that starts inside the spectrum lies inside its 16-byte-multiple pitch.
    v[k] = (t < a.n_samp && b < a.in_row_bytes) ? *(const uint4 *)(a.in + t * a.in_pitch + b) : make_uint4(0, 0, 0, 0);
  }
#pragma unroll
  for (int k = 0; k < kInChunks / kCtThreads; ++k) {
    const int q = threadIdx.x + k * kCtThreads;
    *(uint4 *)(tile + (q / S) * kPitch + 16 * (q % S)) = v[k];
  }
  __syncthreads();

  // Write: chunk q is channel c0 + q % TC, output bytes 16*(q / TC) of the row segment.
#pragma unroll
  for (int k = 0; k < kOutChunks / kCtThreads; ++k) {
    const int q = threadIdx.x + k * kCtThreads;
    const int cl = q % G::TC;
    const int j = q / G::TC;
    const int c = c0 + cl;
    const int64_t ob = (t0 * (DT == DD_U4 ? 1 : G::ES)) / (DT == DD_U4 ? 2 : 1) + 16 * j;  // byte in the row
    if (c >= a.n_chan || ob >= a.out_row_bytes) continue;
    uint32_t w[4];
    if constexpr (DT == DD_U8) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint8_t *p = tile + (16 * j + 4 * i) * kPitch + cl;
        w[i] = (uint32_t)p[0] | ((uint32_t)p[kPitch] << 8) | ((uint32_t)p[2 * kPitch] << 16) |
               ((uint32_t)p[3 * kPitch] << 24);
      }
    } else if constexpr (DT == DD_U16) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint8_t *p = tile + (8 * j + 2 * i) * kPitch + 2 * cl;
        w[i] = (uint32_t)*(const uint16_t *)p | ((uint32_t)*(const uint16_t *)(p + kPitch) << 16);
      }
    } else if constexpr (DT == DD_F32) {
#pragma unroll
      for (int i = 0; i < 4; ++i) w[i] = *(const uint32_t *)(tile + (4 * j + i) * kPitch + 4 * cl);
    } else {
      // 32 samples: nibble cl of spectra 32j .. 32j+31
      const int sh = 4 * (cl & 1);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        uint32_t x = 0;
#pragma unroll
        for (int n = 0; n < 8; ++n) x |= (uint32_t)((tile[(32 * j + 8 * i + n) * kPitch + (cl >> 1)] >> sh) & 15u) << (4 * n);
        w[i] = x;
      }
    }
    uint8_t *dst = a.out + (int64_t)c * a.out_pitch + ob;
    if (ob + 16 <= a.out_row_bytes) {
      *(uint4 *)dst = make_uint4(w[0], w[1], w[2], w[3]);
    } else {  // the row's last, partial piece: only its own bytes
      const int n = (int)(a.out_row_bytes - ob);
      for (int i = 0; i < n; ++i) dst[i] = (uint8_t)(w[i >> 2] >> (8 * (i & 3)));
    }
  }
}

template <int DT>
int launch_ct(const CtArgs &a0, hipStream_t st) {
  using G = CtGeom<DT>;
  CtArgs a = a0;
  a.n_ctiles = (a.n_chan + G::TC - 1) / G::TC;
  const int64_t n_ttiles = (a.n_samp + G::TT - 1) / G::TT;
  const int64_t blocks = n_ttiles * a.n_ctiles;
  if (blocks > 0x7fffffff) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(corner_turn_kernel<DT>, dim3((unsigned)blocks), dim3(kCtThreads), 0, st, a);
  return (int)hipGetLastError();
}

}  // namespace

int launch_corner_turn(int dtype, const void *in, int64_t in_pitch, int n_chan, int64_t n_samp, void *out,
                       int64_t out_pitch, void *stream) {
  CtArgs a;
  a.in = (const uint8_t *)in;
  a.in_pitch = in_pitch;
  a.out = (uint8_t *)out;
  a.out_pitch = out_pitch;
  a.n_chan = n_chan;
  a.n_samp = n_samp;
  a.n_ctiles = 0;
  hipStream_t st = (hipStream_t)stream;
  switch (dtype) {
    case DD_U8:
      a.in_row_bytes = n_chan, a.out_row_bytes = n_samp;
      return launch_ct<DD_U8>(a, st);
    case DD_U16:
      a.in_row_bytes = 2 * (int64_t)n_chan, a.out_row_bytes = 2 * n_samp;
      return launch_ct<DD_U16>(a, st);
    case DD_F32:
      a.in_row_bytes = 4 * (int64_t)n_chan, a.out_row_bytes = 4 * n_samp;
      return launch_ct<DD_F32>(a, st);
    case DD_U4:
      a.in_row_bytes = ((int64_t)n_chan + 1) / 2, a.out_row_bytes = n_samp / 2;
      return launch_ct<DD_U4>(a, st);
  }
  return (int)hipErrorInvalidValue;
}

}  // namespace dd
