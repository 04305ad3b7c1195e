/*
 * The paper's tiled CPU algorithm (Sec. 3, Algorithm 2) for 8-bit input: a CPU
 * comparison for the GPU kernels, not a fallback -- nothing in the GPU path
 * calls it.
 *
 * Loop tiling as in Algorithm 2: threads take (time block of D_t samples, DM
 * block of D_dm trials) pairs; for each, the channels are walked in blocks of
 * D_f, and every DM row of the block adds the D_f delayed input rows into its
 * D_t partial sums.  Neighbouring DM rows read overlapping windows of the same
 * channel rows, so the block's input stays in cache (the temporal locality the
 * paper tiles for), and the D_t sums of one row are contiguous (the spatial
 * locality).  Differences: the per-block partial sums are 16-bit (at most 256
 * channels of 8-bit samples, so they cannot overflow), which lets the compiler
 * widen and add 16 or 32 samples per instruction, and are added into 32-bit
 * totals after each channel block; and the result is not divided by the
 * channel count (the GPU kernels and the oracle do not normalise either).
 * Results are exact integer sums converted once to float: identical to the
 * oracle's.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define DD_CPU_MAX_DF 256

/* Vector widths chosen at run time (AVX-512BW, AVX2 or plain x86-64). */
__attribute__((target_clones("arch=skylake-avx512", "avx2", "default")))
static void add_row_u8(uint16_t *restrict s, const uint8_t *restrict x, int n) {
  for (int t = 0; t < n; ++t) s[t] = (uint16_t)(s[t] + x[t]);
}

__attribute__((target_clones("arch=skylake-avx512", "avx2", "default")))
static void widen_add(int32_t *restrict tot, const uint16_t *restrict s, int n) {
  for (int t = 0; t < n; ++t) tot[t] += s[t];
}

/*
 * out[r][t] = sum_c x[c][t + shift[r][c]] for r < n_dm, t < n_out.
 *   x      [n_chan] rows of `pitch` bytes, samples 0 .. n_out + max shift - 1 read.
 *   shift  int32 [n_dm][n_chan], each in [0, n_samp - n_out].
 *   out    float32 [n_dm][out_pitch].
 *   d_t, d_dm, d_f  tile sizes (Algorithm 2's D_t, D_dm, D_f); d_f <= 256.
 * Returns 0, or -1 for bad arguments, -2 if out of memory.
 */
int dd_cpu_tiled_forward_u8(const uint8_t *x, int64_t pitch, int n_chan, const int32_t *shift, int n_dm,
                            int64_t n_out, float *out, int64_t out_pitch, int d_t, int d_dm, int d_f) {
  if (!x || !shift || !out || n_chan < 1 || n_dm < 1 || n_out < 1 || out_pitch < n_out) return -1;
  if (d_t < 1 || d_dm < 1 || d_f < 1 || d_f > DD_CPU_MAX_DF) return -1;
  const int64_t n_tb = (n_out + d_t - 1) / d_t;
  const int n_db = (n_dm + d_dm - 1) / d_dm;
  int err = 0;
#pragma omp parallel
  {
    int32_t *tot = (int32_t *)malloc(sizeof(int32_t) * (size_t)d_dm * (size_t)d_t);
    uint16_t *s16 = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)d_t);
    if (!tot || !s16) {
#pragma omp atomic write
      err = 1;
    }
#pragma omp for collapse(2) schedule(dynamic, 1)
    for (int64_t tb = 0; tb < n_tb; ++tb) {
      for (int db = 0; db < n_db; ++db) {
        if (!tot || !s16) continue;
        const int64_t i = tb * d_t;
        const int nt = (int)(n_out - i < d_t ? n_out - i : d_t);
        const int j0 = db * d_dm;
        const int nj = n_dm - j0 < d_dm ? n_dm - j0 : d_dm;
        memset(tot, 0, sizeof(int32_t) * (size_t)nj * (size_t)d_t);
        for (int kk = 0; kk < n_chan; kk += d_f) {
          const int ke = kk + d_f < n_chan ? kk + d_f : n_chan;
          for (int j = 0; j < nj; ++j) {
            const int32_t *sh = shift + (int64_t)(j0 + j) * n_chan;
            memset(s16, 0, sizeof(uint16_t) * (size_t)nt);
            for (int k = kk; k < ke; ++k) add_row_u8(s16, x + (int64_t)k * pitch + i + sh[k], nt);
            widen_add(tot + (size_t)j * d_t, s16, nt);
          }
        }
        for (int j = 0; j < nj; ++j) {
          float *o = out + (int64_t)(j0 + j) * out_pitch + i;
          const int32_t *tr = tot + (size_t)j * d_t;
          for (int t = 0; t < nt; ++t) o[t] = (float)tr[t];
        }
      }
    }
    free(tot);
    free(s16);
  }
  return err ? -2 : 0;
}
