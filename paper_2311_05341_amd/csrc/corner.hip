// Corner turn of the input: time-major spectra in[t][c] (as telescopes write
// them) to the channel-major rows out[c][t] the transform reads (the input
// transpose of the pipelines in Sec. 5.3, counted in the real-time factor of
// Sec. 5.5).  For 4-bit data a spectrum packs channel pairs into a byte and an
// output row packs time pairs, the even index in the low nibble.
//
// An HBM-bound LDS-tiled transpose.  A workgroup of 256 lanes takes a tile of
// TC channels x TT samples: it reads the tile's TT spectrum segments of 256
// bytes with 16-byte loads (16 lanes per segment, several loads in flight per
// lane) into LDS, then writes TC output segments of 128 bytes.  Workgroups walk
// the channel tiles of one time tile consecutively, so the spectra are read as
// contiguous runs.
//
// 8-bit, 16-bit and float data (corner_turn_words_kernel): a lane takes one
// 32-bit column of the tile (4, 2 or 1 channels) over the samples of one
// 16-byte output piece, reads it as 32-bit words and transposes them in
// registers with v_perm (a 4x4 byte transpose is 8 v_perm).  The 8 lanes that
// share a column take its 8 output pieces, so every store instruction writes
// whole 128-byte runs of 8 rows.  The 16-byte column blocks of LDS row r are
// XOR-swizzled with the output piece r belongs to, which makes those reads
// conflict-free.  4-bit data (corner_turn_kernel) assemble each output piece
// from nibble reads.
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

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// ES-byte elements (1, 2 or 4).  Tile: 256 input bytes x 128 output bytes per row;
// 64 word columns x 8 output pieces = 512 units, two per lane.
template <int DT>
__global__ __launch_bounds__(kCtThreads) void corner_turn_words_kernel(CtArgs a) {
  using G = CtGeom<DT>;
  constexpr int ES = G::ES;
  constexpr int R = 16 / ES;   // samples per 16-byte output piece = LDS rows per piece
  constexpr int EPW = 4 / ES;  // channels per 32-bit word
  static_assert(G::TC * ES == 256 && G::TT == 8 * R, "tile shape");
  __shared__ __attribute__((aligned(16))) uint8_t tile[G::TT * 256];

  const int ct = (int)(blockIdx.x % (unsigned)a.n_ctiles);
  const int64_t t0 = (int64_t)(blockIdx.x / (unsigned)a.n_ctiles) * G::TT;
  const int64_t b0 = (int64_t)ct * 256;
  const int c0 = ct * G::TC;

  // Read the TT x 256-byte block; 16-byte block k of row r goes to block k ^ (r / R).
  constexpr int kLoads = G::TT * 16 / kCtThreads;
  uint4 v[kLoads];
#pragma unroll
  for (int s = 0; s < kLoads; ++s) {
    const int q = threadIdx.x + s * kCtThreads;
    const int64_t t = t0 + q / 16;
    const int64_t b = b0 + 16 * (q % 16);
    // A chunk that starts inside the spectrum lies inside its 16-byte-multiple pitch.
    v[s] = (t < a.n_samp && b < a.in_row_bytes) ? *(const uint4 *)(a.in + t * a.in_pitch + b) : make_uint4(0, 0, 0, 0);
  }
#pragma unroll
  for (int s = 0; s < kLoads; ++s) {
    const int q = threadIdx.x + s * kCtThreads;
    const int r = q / 16;
    *(uint4 *)(tile + r * 256 + 16 * ((q % 16) ^ (r / R))) = v[s];
  }
  __syncthreads();

#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int u = threadIdx.x + s * kCtThreads;
    const int j = u % 8;   // output piece: samples R*j .. R*j + R-1 of the tile
    const int w = u / 8;   // word column: channels EPW*w .. EPW*w + EPW-1 of the tile
    uint32_t d[R];
#pragma unroll
    for (int i = 0; i < R; ++i) d[i] = *(const uint32_t *)(tile + (R * j + i) * 256 + 16 * ((w / 4) ^ j) + 4 * (w % 4));
    uint32_t o[EPW][4];  // o[k] = the 16 output bytes of channel EPW*w + k
    if constexpr (ES == 1) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const uint32_t x0 = perm(d[4 * g + 1], d[4 * g], 0x05010400u), x1 = perm(d[4 * g + 1], d[4 * g], 0x07030602u);
        const uint32_t x2 = perm(d[4 * g + 3], d[4 * g + 2], 0x05010400u);
        const uint32_t x3 = perm(d[4 * g + 3], d[4 * g + 2], 0x07030602u);
        o[0][g] = perm(x2, x0, 0x05040100u);
        o[1][g] = perm(x2, x0, 0x07060302u);
        o[2][g] = perm(x3, x1, 0x05040100u);
        o[3][g] = perm(x3, x1, 0x07060302u);
      }
    } else if constexpr (ES == 2) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        o[0][g] = perm(d[2 * g + 1], d[2 * g], 0x05040100u);
        o[1][g] = perm(d[2 * g + 1], d[2 * g], 0x07060302u);
      }
    } else {
#pragma unroll
      for (int g = 0; g < 4; ++g) o[0][g] = d[g];
    }
    const int64_t ob = t0 * ES + 16 * j;  // byte of the row
    if (ob >= a.out_row_bytes) continue;
#pragma unroll
    for (int k = 0; k < EPW; ++k) {
      const int c = c0 + EPW * w + k;
      if (c >= a.n_chan) break;
      uint8_t *dst = a.out + (int64_t)c * a.out_pitch + ob;
      if (ob + 16 <= a.out_row_bytes) {
        *(uint4 *)dst = make_uint4(o[k][0], o[k][1], o[k][2], o[k][3]);
      } else {  // the row's last, partial piece: only its own bytes
        const int n = (int)(a.out_row_bytes - ob);
        for (int i = 0; i < n; ++i) dst[i] = (uint8_t)(o[k][i >> 2] >> (8 * (i & 3)));
      }
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
  if constexpr (DT == DD_U4)
    hipLaunchKernelGGL(corner_turn_kernel<DT>, dim3((unsigned)blocks), dim3(kCtThreads), 0, st, a);
  else
    hipLaunchKernelGGL(corner_turn_words_kernel<DT>, dim3((unsigned)blocks), dim3(kCtThreads), 0, st, a);
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
