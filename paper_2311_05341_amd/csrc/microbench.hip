// Microbenchmarks of the three rates that bound the dedispersion kernels on
// gfx950, measured on the machine the kernels run on instead of taken from a
// datasheet: the VALU issue rate of each integer add form the accumulate loops
// use, the LDS read bandwidth per access width and alignment (the quantity the
// shared-memory bandwidth analysis of Sec. 5.1 prices), and the HBM copy rate.
//
// Every kernel does a fixed, counted amount of work and writes one word per
// lane, so nothing is optimised away; the caller times the launch with HIP
// events and divides.  Built as its own library (libddmb.so): the transform
// library does not depend on it.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// ---------------------------------------------------------------------------
// VALU.  Each lane runs kChains independent dependency chains of one
// instruction form, kUnroll instructions per chain per loop trip; with several
// waves per SIMD the chains' latency is hidden and the loop measures issue
// rate.  The operand registers are loop-invariant values from the input.
constexpr int kChains = 8;
constexpr int kUnroll = 8;

enum ValuForm { kAddU32 = 0, kAdd3U32 = 1, kPkAddU16 = 2, kAddSdwa = 3, kPerm = 4, kSwarPair = 5 };

template <int FORM>
__device__ __forceinline__ void valu_step(uint32_t (&acc)[kChains], uint32_t a, uint32_t b) {
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    if constexpr (FORM == kAddU32) {
      asm volatile("v_add_u32 %0, %0, %1" : "+v"(acc[i]) : "v"(a));
    } else if constexpr (FORM == kAdd3U32) {
      asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(acc[i]) : "v"(a), "v"(b));
    } else if constexpr (FORM == kPkAddU16) {
      asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(acc[i]) : "v"(a));
    } else if constexpr (FORM == kAddSdwa) {
      asm volatile("v_add_u32_sdwa %0, %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_1"
                   : "+v"(acc[i])
                   : "v"(a));
    } else if constexpr (FORM == kPerm) {
      asm volatile("v_perm_b32 %0, %0, %1, %2" : "+v"(acc[i]) : "v"(a), "v"(b));
    }
  }
}

// The accumulate loop's own mix of instructions for one pair of channel words
// (8 sample-adds): two v_perm_b32 and two v_add3_u32.  kChains / 2 pairs of
// (mix, odd) accumulators.
__device__ __forceinline__ void swar_step(uint32_t (&acc)[kChains], uint32_t w1, uint32_t w2, uint32_t sel) {
#pragma unroll
  for (int i = 0; i < kChains; i += 2) {
    uint32_t p1, p2;
    asm volatile("v_perm_b32 %0, %1, %1, %2" : "=v"(p1) : "v"(w1), "v"(sel));
    asm volatile("v_perm_b32 %0, %1, %1, %2" : "=v"(p2) : "v"(w2), "v"(sel));
    asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(acc[i]) : "v"(w1), "v"(w2));
    asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(acc[i + 1]) : "v"(p1), "v"(p2));
  }
}

template <int FORM>
__global__ __launch_bounds__(256) void valu_kernel(const uint32_t *in, uint32_t *out, int iters) {
  const uint32_t a = in[threadIdx.x & 63], b = in[64 + (threadIdx.x & 63)];
  uint32_t acc[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) acc[i] = a + (uint32_t)i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if constexpr (FORM == kSwarPair)
        swar_step(acc, a, b, 0x0C030C01u);
      else
        valu_step<FORM>(acc, a, b);
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) s ^= acc[i];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// ---------------------------------------------------------------------------
// LDS reads.  A workgroup fills 48 KiB of LDS, then each wave reads it in a
// loop.  Trip i of wave w starts at byte misalign + ((w + 4 i) * 8 * S) mod
// 32 KiB, where S is the bytes one wave read covers (64 lanes x WIDTH), and
// issues kReads reads at S-byte steps from there: constant offsets, so no
// address arithmetic per read.  Lanes are contiguous (lane i at + i * WIDTH).
// Results fold into two registers per lane (v_add3_u32 for 8 and 16 bytes:
// at most one lane-op per 4 bytes read, below the LDS time per read).  The
// compiler pairs reads S bytes apart into one instruction: 4-byte reads issue as
// ds_read2st64_b32 (the accumulate loops' form), 8-byte ones as
// ds_read2st64_b64, 16-byte ones as ds_read_b128.
constexpr int kLdsBytes = 48 * 1024;
constexpr int kLdsSpan = 32 * 1024;
constexpr int kReads = 8;

__device__ __forceinline__ uint32_t fold3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

template <int WIDTH>
__global__ __launch_bounds__(256) void lds_kernel(uint32_t *out, int iters, int misalign) {
  __shared__ __align__(16) uint8_t lds[kLdsBytes];
  for (int i = threadIdx.x; i < kLdsBytes / 4; i += blockDim.x) ((uint32_t *)lds)[i] = (uint32_t)i * 2654435761u;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int S = 64 * WIDTH;  // bytes one wave read covers
  uint32_t acc0 = 0, acc1 = 0;
  uint32_t pos = (uint32_t)(wave * kReads * S);
  for (int it = 0; it < iters; ++it) {
    const uint8_t *base = lds + misalign + (pos & (kLdsSpan - 1));  // reads end below 32 KiB + 8 S + 15 <= 40 KiB + 15
#pragma unroll
    for (int r = 0; r < kReads; ++r) {
      const uint8_t *p = base + r * S;
      if constexpr (WIDTH == 4) {
        const uint32_t v = *((const uint32_t *)p + lane);
        if (r & 1)
          acc1 ^= v;
        else
          acc0 ^= v;
      } else if constexpr (WIDTH == 8) {
        const uint2 v = *((const uint2 *)p + lane);
        acc0 = fold3(acc0, v.x, v.y);
      } else {
        const uint4 v = *((const uint4 *)p + lane);
        acc0 = fold3(acc0, v.x, v.y);
        acc1 = fold3(acc1, v.z, v.w);
      }
    }
    pos += (uint32_t)(4 * kReads * S);
  }
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc0 ^ acc1;
}

// ---------------------------------------------------------------------------
// HBM copy: 16 bytes per lane per trip, grid-stride, n16 16-byte elements.
__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// Instruction forms of ddmb_valu: 0 v_add_u32, 1 v_add3_u32, 2 v_pk_add_u16,
// 3 v_add_u32 SDWA (high half), 4 v_perm_b32, 5 the 8-bit accumulate pair
// (2 v_perm_b32 + 2 v_add3_u32).
int ddmb_valu_instructions_per_lane(int form, int iters) {
  return iters * kUnroll * kChains * (form == kSwarPair ? 2 : 1);
}

// Launch `blocks` workgroups of 256 lanes; d_in holds 128 uint32, d_out
// blocks * 256 uint32.  Each lane issues ddmb_valu_instructions_per_lane(form, iters)
// instructions of the form.  Returns a hipError_t.
int ddmb_valu(int form, int blocks, int iters, const void *d_in, void *d_out, void *stream) {
  if (blocks <= 0 || iters <= 0 || !d_in || !d_out) return (int)hipErrorInvalidValue;
  const hipStream_t st = (hipStream_t)stream;
  const uint32_t *in = (const uint32_t *)d_in;
  uint32_t *out = (uint32_t *)d_out;
  switch (form) {
    case kAddU32: hipLaunchKernelGGL(valu_kernel<kAddU32>, dim3(blocks), dim3(256), 0, st, in, out, iters); break;
    case kAdd3U32: hipLaunchKernelGGL(valu_kernel<kAdd3U32>, dim3(blocks), dim3(256), 0, st, in, out, iters); break;
    case kPkAddU16: hipLaunchKernelGGL(valu_kernel<kPkAddU16>, dim3(blocks), dim3(256), 0, st, in, out, iters); break;
    case kAddSdwa: hipLaunchKernelGGL(valu_kernel<kAddSdwa>, dim3(blocks), dim3(256), 0, st, in, out, iters); break;
    case kPerm: hipLaunchKernelGGL(valu_kernel<kPerm>, dim3(blocks), dim3(256), 0, st, in, out, iters); break;
    case kSwarPair: hipLaunchKernelGGL(valu_kernel<kSwarPair>, dim3(blocks), dim3(256), 0, st, in, out, iters); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

// Bytes one lane reads from LDS in one ddmb_lds launch.
int ddmb_lds_bytes_per_lane(int width, int iters) { return iters * kReads * width; }

// LDS read kernel: width 4, 8 or 16 bytes per lane and read, starting
// `misalign` bytes (0..15) past a 16-byte boundary.  `blocks` workgroups of
// 256 lanes, d_out blocks * 256 uint32.
int ddmb_lds(int width, int misalign, int blocks, int iters, void *d_out, void *stream) {
  if (blocks <= 0 || iters <= 0 || !d_out || misalign < 0 || misalign > 15) return (int)hipErrorInvalidValue;
  const hipStream_t st = (hipStream_t)stream;
  uint32_t *out = (uint32_t *)d_out;
  if (width == 4)
    hipLaunchKernelGGL(lds_kernel<4>, dim3(blocks), dim3(256), 0, st, out, iters, misalign);
  else if (width == 8)
    hipLaunchKernelGGL(lds_kernel<8>, dim3(blocks), dim3(256), 0, st, out, iters, misalign);
  else if (width == 16)
    hipLaunchKernelGGL(lds_kernel<16>, dim3(blocks), dim3(256), 0, st, out, iters, misalign);
  else
    return (int)hipErrorInvalidValue;
  return (int)hipGetLastError();
}

// Copy `bytes` (a multiple of 16; both pointers 16-byte aligned) with `blocks`
// workgroups of 256 lanes.
int ddmb_copy(const void *d_src, void *d_dst, size_t bytes, int blocks, void *stream) {
  if (!d_src || !d_dst || (bytes & 15) || blocks <= 0 || ((uintptr_t)d_src & 15) || ((uintptr_t)d_dst & 15))
    return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const uint4 *)d_src,
                     (uint4 *)d_dst, bytes / 16);
  return (int)hipGetLastError();
}

}  // extern "C"
