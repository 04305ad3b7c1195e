/*
 * CPU build of the synthetic-input generator (definition in gen_common.h).
 * 8-bit Gaussian samples come from a 65536-entry quantile table built by the
 * Python front end; 4-bit samples are the low 4 bits of the 16-bit draw.
 */
#include <stdint.h>

#include "gen_common.h"

/* out[c*pitch + t] = table[draw(seed, c, t_start + t)] for t < n_samp. */
void synth_u8_table(uint8_t *out, int n_chan, int64_t n_samp, int64_t pitch, uint64_t seed,
                    int64_t t_start, const uint8_t *table) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < n_chan; ++c) {
    const uint64_t base = synth_row_base(seed, c);
    uint8_t *row = out + (int64_t)c * pitch;
    for (int64_t t = 0; t < n_samp; ++t) {
      const int64_t g = t_start + t;
      const uint64_t h = synth_splitmix64(base + (uint64_t)(g >> 2));
      row[t] = table[(h >> (16 * (g & 3))) & 0xFFFF];
    }
  }
}

/* 16-bit samples: out[c*pitch + t] = table[draw(seed, c, t_start + t)] (pitch in samples). */
void synth_u16_table(uint16_t *out, int n_chan, int64_t n_samp, int64_t pitch, uint64_t seed,
                     int64_t t_start, const uint16_t *table) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < n_chan; ++c) {
    const uint64_t base = synth_row_base(seed, c);
    uint16_t *row = out + (int64_t)c * pitch;
    for (int64_t t = 0; t < n_samp; ++t) {
      const int64_t g = t_start + t;
      const uint64_t h = synth_splitmix64(base + (uint64_t)(g >> 2));
      row[t] = table[(h >> (16 * (g & 3))) & 0xFFFF];
    }
  }
}

/* Packed 4-bit uniform samples: byte i of row c holds samples t_start + 2i
 * (low nibble) and t_start + 2i + 1 (high nibble); t_start and n_samp even. */
void synth_u4_packed(uint8_t *out, int n_chan, int64_t n_samp, int64_t pitch_bytes, uint64_t seed,
                     int64_t t_start) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < n_chan; ++c) {
    const uint64_t base = synth_row_base(seed, c);
    uint8_t *row = out + (int64_t)c * pitch_bytes;
    for (int64_t i = 0; i < n_samp / 2; ++i) {
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
