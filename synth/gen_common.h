/*
 * Counter-based sample generator shared (as a definition) by the CPU and GPU
 * builds of the synthetic-input module.  It contains no dedispersion
 * arithmetic.
 *
 * Each 64-bit hash is SplitMix64's output function (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) applied to a
 * counter.  Channel c of a filterbank with seed s starts at counter
 * base(s, c) = splitmix64(s * 2^32 + c); time sample t takes 16 bits of
 * splitmix64(base + floor(t / 4)), bits 16*(t mod 4) .. 16*(t mod 4) + 15.
 * Any slice of any row can be generated independently.
 */
#ifndef SYNTH_GEN_COMMON_H
#define SYNTH_GEN_COMMON_H
#include <stdint.h>

#if defined(__HIPCC__)
#define SYNTH_FN __host__ __device__ static inline
#else
#define SYNTH_FN static inline
#endif

SYNTH_FN uint64_t synth_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

SYNTH_FN uint64_t synth_row_base(uint64_t seed, int64_t c) {
  return synth_splitmix64((seed << 32) + (uint64_t)c);
}

#endif
