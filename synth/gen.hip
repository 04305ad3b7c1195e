// GPU build of the synthetic-input generator (definition in gen_common.h).
// Used to fill large filterbanks directly in device memory; the CPU build in
// gen.c produces the same bytes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gen_common.h"

// One thread writes 16 consecutive samples (4 hashes) of one row.
__global__ void synth_u8_kernel(uint8_t *__restrict__ out, int n_chan, int64_t n_samp, int64_t pitch,
                                uint64_t seed, int64_t t_start, const uint8_t *__restrict__ table) {
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
  if (t >= n_samp) return;
  for (int c = blockIdx.y; c < n_chan; c += gridDim.y) {  // grid y holds at most 65535 rows
    const uint64_t base = synth_row_base(seed, c);
    uint8_t v[16];
    for (int k = 0; k < 16; ++k) {
      const int64_t g = t_start + t + k;
      const uint64_t h = synth_splitmix64(base + (uint64_t)(g >> 2));
      v[k] = table[(h >> (16 * (g & 3))) & 0xFFFF];
    }
    uint8_t *row = out + (int64_t)c * pitch;
    if (t + 16 <= n_samp && ((uintptr_t)(row + t) & 3) == 0) {
      uint32_t w[4];
      for (int q = 0; q < 4; ++q)
        w[q] = v[4 * q] | (v[4 * q + 1] << 8) | (v[4 * q + 2] << 16) | ((uint32_t)v[4 * q + 3] << 24);
      uint32_t *dst = (uint32_t *)(row + t);
      for (int q = 0; q < 4; ++q) dst[q] = w[q];
    } else {
      for (int k = 0; k < 16 && t + k < n_samp; ++k) row[t + k] = v[k];
    }
  }
}

// One thread writes 8 consecutive 16-bit samples (2 hashes) of one row.
__global__ void synth_u16_kernel(uint16_t *__restrict__ out, int n_chan, int64_t n_samp, int64_t pitch,
                                 uint64_t seed, int64_t t_start, const uint16_t *__restrict__ table) {
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8;
  if (t >= n_samp) return;
  for (int c = blockIdx.y; c < n_chan; c += gridDim.y) {
    const uint64_t base = synth_row_base(seed, c);
    uint16_t *row = out + (int64_t)c * pitch;
    for (int k = 0; k < 8 && t + k < n_samp; ++k) {
      const int64_t g = t_start + t + k;
      const uint64_t h = synth_splitmix64(base + (uint64_t)(g >> 2));
      row[t + k] = table[(h >> (16 * (g & 3))) & 0xFFFF];
    }
  }
}

__global__ void synth_u4_kernel(uint8_t *__restrict__ out, int n_chan, int64_t n_samp, int64_t pitch_bytes,
                                uint64_t seed, int64_t t_start) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8;  // first output byte
  if (i0 >= n_samp / 2) return;
  for (int c = blockIdx.y; c < n_chan; c += gridDim.y) {
    const uint64_t base = synth_row_base(seed, c);
    uint8_t *row = out + (int64_t)c * pitch_bytes;
    for (int64_t i = i0; i < i0 + 8 && i < n_samp / 2; ++i) {
      uint8_t b = 0;
      for (int k = 0; k < 2; ++k) {
        const int64_t g = t_start + 2 * i + k;
        const uint64_t h = synth_splitmix64(base + (uint64_t)(g >> 2));
        b |= (uint8_t)(((h >> (16 * (g & 3))) & 15u) << (4 * k));
      }
      row[i] = b;
    }
  }
}

extern "C" int synth_u8_table_gpu(uint8_t *d_out, int n_chan, int64_t n_samp, int64_t pitch, uint64_t seed,
                                  int64_t t_start, const uint8_t *d_table, void *stream) {
  if (n_chan <= 0 || n_samp <= 0) return (int)hipErrorInvalidValue;
  const int64_t per_row = (n_samp + 16 * 256 - 1) / (16 * 256);
  hipLaunchKernelGGL(synth_u8_kernel, dim3((unsigned)per_row, (unsigned)(n_chan < 65535 ? n_chan : 65535)), dim3(256), 0,
                     (hipStream_t)stream, d_out, n_chan, n_samp, pitch, seed, t_start, d_table);
  return (int)hipGetLastError();
}

extern "C" int synth_u16_table_gpu(uint16_t *d_out, int n_chan, int64_t n_samp, int64_t pitch, uint64_t seed,
                                   int64_t t_start, const uint16_t *d_table, void *stream) {
  if (n_chan <= 0 || n_samp <= 0 || pitch < n_samp) return (int)hipErrorInvalidValue;
  const int64_t per_row = (n_samp + 8 * 256 - 1) / (8 * 256);
  hipLaunchKernelGGL(synth_u16_kernel, dim3((unsigned)per_row, (unsigned)(n_chan < 65535 ? n_chan : 65535)), dim3(256), 0,
                     (hipStream_t)stream, d_out, n_chan, n_samp, pitch, seed, t_start, d_table);
  return (int)hipGetLastError();
}

extern "C" int synth_u4_packed_gpu(uint8_t *d_out, int n_chan, int64_t n_samp, int64_t pitch_bytes,
                                   uint64_t seed, int64_t t_start, void *stream) {
  if (n_chan <= 0 || n_samp <= 0 || (n_samp & 1) || (t_start & 1))
    return (int)hipErrorInvalidValue;
  const int64_t per_row = (n_samp / 2 + 8 * 256 - 1) / (8 * 256);
  hipLaunchKernelGGL(synth_u4_kernel, dim3((unsigned)per_row, (unsigned)(n_chan < 65535 ? n_chan : 65535)), dim3(256), 0,
                     (hipStream_t)stream, d_out, n_chan, n_samp, pitch_bytes, seed, t_start);
  return (int)hipGetLastError();
}
