/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU statement of brute-force incoherent
 * dedispersion, used to check the GPU library.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant with the GPU path.
 *
 * What it computes (Novotny et al., "Accelerating Dedispersion using
 * Many-Core Architectures"):
 *
 *   shift table   Sec. 1, Eq. 1 (cold-plasma law) with the per-channel form of
 *                 Sec. 4.1 (channel i at f_high - i*df), constant 4.148808e3
 *                 s MHz^2 cm^3 / pc, rounded half-up to whole samples.
 *   forward       Sec. 2, Eq. 3 and Algorithm 1:  S(d,t) = sum_c x(c, t + shift(c,d))
 *                 for t in [0, N_out), N_out = N_t - max shift, no normalisation.
 *   adjoint       The transpose of Eq. 3 in scatter form:
 *                 g(c, t + shift(c,d)) += y(d, t).
 *
 * Precision: the shift table is IEEE FP64 with no contraction (build with
 * -ffp-contract=off).  Integer input accumulates in int64, float input in
 * FP64; outputs are converted once at the end.
 *
 * Loops: DM rows outermost (OpenMP), channels in the middle, time innermost.
 * No blocking, fusion or reordering beyond that.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_KDM 4.148808e3 /* s MHz^2 cm^3 pc^-1 */

/* Frequency of channel c: an explicit list, else f_high - c*df (Sec. 4.1). */
static double chan_freq(int c, double f_high, double chan_bw, const double *freqs) {
  return freqs ? freqs[c] : f_high - (double)c * chan_bw;
}

/*
 * Integer shift table shift[d*n_chan + c] in samples (Eq. 1 divided by t_samp,
 * rounded half up).  DM_d = dm_start + d*dm_step, evaluated per d (no running
 * sum).  Returns 0, or -1 if a channel frequency is not positive or a shift
 * does not fit an int32.
 */
int oracle_shift_table(int n_chan, double f_high, double chan_bw, const double *freqs,
                       double t_samp, double dm_start, double dm_step, int n_dm,
                       int32_t *shift) {
  for (int c = 0; c < n_chan; ++c)
    if (!(chan_freq(c, f_high, chan_bw, freqs) > 0.0)) return -1;
  for (int d = 0; d < n_dm; ++d) {
    double dm = dm_start + (double)d * dm_step;
    for (int c = 0; c < n_chan; ++c) {
      double f = chan_freq(c, f_high, chan_bw, freqs);
      double k = 1.0 / (f * f) - 1.0 / (f_high * f_high);
      double delay_samples = ((dm * ORACLE_KDM) * k) / t_samp;
      double s = floor(delay_samples + 0.5);
      if (!(s >= -2147483648.0 && s <= 2147483647.0)) return -1;
      shift[(int64_t)d * n_chan + c] = (int32_t)s;
    }
  }
  return 0;
}

/* Input sample X(c, t) for the three input encodings. */
static inline int64_t x_u8(const uint8_t *x, int64_t pitch, int c, int64_t t) {
  return x[(int64_t)c * pitch + t];
}
/* 4-bit: two samples per byte, the even sample in the low nibble. */
static inline int64_t x_u4(const uint8_t *x, int64_t pitch_bytes, int c, int64_t t) {
  uint8_t b = x[(int64_t)c * pitch_bytes + (t >> 1)];
  return (t & 1) ? (b >> 4) : (b & 15);
}

/* 16-bit: little-endian unsigned samples, two bytes each (pitch in bytes). */
static inline int64_t x_u16(const uint8_t *x, int64_t pitch_bytes, int c, int64_t t) {
  const uint8_t *p = x + (int64_t)c * pitch_bytes + 2 * t;
  return (int64_t)p[0] | ((int64_t)p[1] << 8);
}

/* 32-bit: little-endian unsigned samples, four bytes each (pitch in bytes).
 * Time-binned 16-bit data holds sums of up to 256 such samples, which need
 * 24 bits. */
static inline int64_t x_u32(const uint8_t *x, int64_t pitch_bytes, int c, int64_t t) {
  const uint8_t *p = x + (int64_t)c * pitch_bytes + 4 * t;
  return (int64_t)p[0] | ((int64_t)p[1] << 8) | ((int64_t)p[2] << 16) | ((int64_t)p[3] << 24);
}

/* Every read x(c, t + shift) with t < n_out must stay inside [0, n_samp). */
static int shifts_in_range(const int32_t *shift, int n_chan, int n_dm, int64_t n_samp,
                           int64_t n_out) {
  if (n_out <= 0) return 0;
  for (int64_t i = 0; i < (int64_t)n_chan * n_dm; ++i)
    if (shift[i] < 0 || (int64_t)shift[i] + n_out > n_samp) return 0;
  return 1;
}

/*
 * Forward transform on a set of DM rows.  rows == NULL means all n_rows = n_dm
 * rows in order; otherwise out row r holds DM row rows[r].  out is
 * [n_rows][n_out] float, each int64 sum converted once to float (round to
 * nearest even; exact below 2^24).  dtype: 1 = u8, 2 = u4 (pitch in bytes),
 * 4 = u16, 5 = u32 (pitch in bytes); 3 = f32 uses oracle_forward_f32 instead.
 */
int oracle_forward_int(int dtype, const uint8_t *x, int64_t pitch, int n_chan, int64_t n_samp,
                       const int32_t *shift, int n_dm, int64_t n_out,
                       const int32_t *rows, int n_rows, float *out) {
  if (dtype != 1 && dtype != 2 && dtype != 4 && dtype != 5) return -1;
  if (!shifts_in_range(shift, n_chan, n_dm, n_samp, n_out)) return -1;
  int bad = 0;
#pragma omp parallel
  {
    int64_t *acc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_out > 0 ? n_out : 1));
    if (!acc) {
#pragma omp atomic write
      bad = 1;
    }
#pragma omp for schedule(dynamic, 1)
    for (int r = 0; r < n_rows; ++r) {
      if (!acc) continue;
      int d = rows ? rows[r] : r;
      if (d < 0 || d >= n_dm) {
#pragma omp atomic write
        bad = 1;
        continue;
      }
      memset(acc, 0, sizeof(int64_t) * (size_t)n_out);
      for (int c = 0; c < n_chan; ++c) {
        int64_t s = shift[(int64_t)d * n_chan + c];
        if (dtype == 1) {
          for (int64_t t = 0; t < n_out; ++t) acc[t] += x_u8(x, pitch, c, t + s);
        } else if (dtype == 2) {
          for (int64_t t = 0; t < n_out; ++t) acc[t] += x_u4(x, pitch, c, t + s);
        } else if (dtype == 4) {
          for (int64_t t = 0; t < n_out; ++t) acc[t] += x_u16(x, pitch, c, t + s);
        } else {
          for (int64_t t = 0; t < n_out; ++t) acc[t] += x_u32(x, pitch, c, t + s);
        }
      }
      for (int64_t t = 0; t < n_out; ++t) out[(int64_t)r * n_out + t] = (float)acc[t];
    }
    free(acc);
  }
  return bad ? -1 : 0;
}

/*
 * Corner turn of the input (the "transposing of the input data" that the
 * pipelines of Sec. 5.3 run before the transform and that the real-time factor
 * of Sec. 5.5 counts): time-major spectra in[t][c] (each time sample holds all
 * channels) to channel-major rows out[c][t], the layout Eq. 3 is evaluated on.
 * dtype 1 = u8, 3 = f32, 4 = u16 (little-endian): element copy.  dtype 2 = u4:
 * in a spectrum two channels share a byte (channel 2k in the low nibble), in an
 * output row two time samples (sample 2k in the low nibble); n_samp even.
 * Pitches in bytes.  Returns -1 on bad arguments.
 */
int oracle_corner_turn(int dtype, const uint8_t *in, int64_t in_pitch, int n_chan, int64_t n_samp, uint8_t *out,
                       int64_t out_pitch) {
  if (n_chan < 1 || n_samp < 1) return -1;
  if (dtype == 2) {
    if (n_samp % 2) return -1;
    if (in_pitch < (n_chan + 1) / 2 || out_pitch < n_samp / 2) return -1;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < n_chan; ++c) {
      for (int64_t t = 0; t < n_samp; t += 2) {
        const uint8_t b0 = in[t * in_pitch + c / 2], b1 = in[(t + 1) * in_pitch + c / 2];
        const int v0 = (c % 2) ? (b0 >> 4) : (b0 & 15);
        const int v1 = (c % 2) ? (b1 >> 4) : (b1 & 15);
        out[(int64_t)c * out_pitch + t / 2] = (uint8_t)(v0 | (v1 << 4));
      }
    }
    return 0;
  }
  const int es = dtype == 1 ? 1 : dtype == 4 ? 2 : dtype == 3 ? 4 : 0;
  if (!es || in_pitch < (int64_t)n_chan * es || out_pitch < n_samp * es) return -1;
#pragma omp parallel for schedule(static)
  for (int c = 0; c < n_chan; ++c)
    for (int64_t t = 0; t < n_samp; ++t)
      for (int b = 0; b < es; ++b) out[(int64_t)c * out_pitch + t * es + b] = in[t * in_pitch + (int64_t)c * es + b];
  return 0;
}

/*
 * Time binning, the "downsampling" that Secs. 5.2 and 5.3 apply before the
 * transform for high-DM ranges and that the real-time factor of Sec. 5.5
 * counts (downsampling by `factor`): xb(c, j) = sum_{i < factor} x(c, j*factor + i)
 * for j < n_samp / factor (a trailing partial bin is dropped).  Sums, not
 * means, like the transform itself (no normalisation).  Integer input
 * (dtype 1 = u8, 2 = u4, 4 = u16; pitch in bytes) -> int64 out[c][j];
 * out_pitch in elements.  Returns -1 on bad arguments.
 */
int oracle_bin_int(int dtype, const uint8_t *x, int64_t pitch, int n_chan, int64_t n_samp, int factor,
                   int64_t *out, int64_t out_pitch) {
  if ((dtype != 1 && dtype != 2 && dtype != 4) || factor < 1 || n_chan < 1 || n_samp < 0) return -1;
  const int64_t n_bins = n_samp / factor;
  if (out_pitch < n_bins) return -1;
#pragma omp parallel for schedule(static)
  for (int c = 0; c < n_chan; ++c) {
    for (int64_t j = 0; j < n_bins; ++j) {
      int64_t acc = 0;
      for (int i = 0; i < factor; ++i) {
        const int64_t t = j * factor + i;
        acc += dtype == 1 ? x_u8(x, pitch, c, t) : dtype == 2 ? x_u4(x, pitch, c, t) : x_u16(x, pitch, c, t);
      }
      out[(int64_t)c * out_pitch + j] = acc;
    }
  }
  return 0;
}

/* Float binning in FP64: out[c][j] = sum_{i < factor} x[c][j*factor + i]. */
int oracle_bin_f32(const float *x, int64_t pitch, int n_chan, int64_t n_samp, int factor, double *out,
                   int64_t out_pitch) {
  if (factor < 1 || n_chan < 1 || n_samp < 0) return -1;
  const int64_t n_bins = n_samp / factor;
  if (out_pitch < n_bins) return -1;
#pragma omp parallel for schedule(static)
  for (int c = 0; c < n_chan; ++c)
    for (int64_t j = 0; j < n_bins; ++j) {
      double acc = 0.0;
      for (int i = 0; i < factor; ++i) acc += (double)x[(int64_t)c * pitch + j * factor + i];
      out[(int64_t)c * out_pitch + j] = acc;
    }
  return 0;
}

/*
 * Forward transform for float input, in FP64.  out[r][t] is the FP64 sum and
 * abs_out (if not NULL) the FP64 sum of the absolute values of the same terms,
 * which scales the float tolerance.
 */
int oracle_forward_f32(const float *x, int64_t pitch, int n_chan, int64_t n_samp,
                       const int32_t *shift, int n_dm, int64_t n_out, const int32_t *rows,
                       int n_rows, double *out, double *abs_out) {
  if (!shifts_in_range(shift, n_chan, n_dm, n_samp, n_out)) return -1;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int r = 0; r < n_rows; ++r) {
    int d = rows ? rows[r] : r;
    if (d < 0 || d >= n_dm) {
#pragma omp atomic write
      bad = 1;
      continue;
    }
    double *o = out + (int64_t)r * n_out;
    double *a = abs_out ? abs_out + (int64_t)r * n_out : NULL;
    for (int64_t t = 0; t < n_out; ++t) o[t] = 0.0;
    if (a)
      for (int64_t t = 0; t < n_out; ++t) a[t] = 0.0;
    for (int c = 0; c < n_chan; ++c) {
      const float *row = x + (int64_t)c * pitch + shift[(int64_t)d * n_chan + c];
      for (int64_t t = 0; t < n_out; ++t) o[t] += (double)row[t];
      if (a)
        for (int64_t t = 0; t < n_out; ++t) a[t] += fabs((double)row[t]);
    }
  }
  return bad ? -1 : 0;
}

/*
 * Adjoint (transpose of Eq. 3) in scatter form, FP64: for every d, c and
 * t < n_out, g[c][t + shift(c,d)] += y[d][t].  g is [n_chan][n_samp] doubles
 * and is overwritten; entries that no output reads stay exactly 0.  Channels
 * are independent, so the channel loop is the parallel one.
 */
int oracle_adjoint_f64(const float *y, int64_t y_pitch, int n_chan, int64_t n_samp,
                       const int32_t *shift, int n_dm, int64_t n_out, double *g) {
  if (!shifts_in_range(shift, n_chan, n_dm, n_samp, n_out)) return -1;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < n_chan; ++c) {
    double *gr = g + (int64_t)c * n_samp;
    for (int64_t t = 0; t < n_samp; ++t) gr[t] = 0.0;
    for (int d = 0; d < n_dm; ++d) {
      int64_t s = shift[(int64_t)d * n_chan + c];
      const float *yr = y + (int64_t)d * y_pitch;
      for (int64_t t = 0; t < n_out; ++t) gr[t + s] += (double)yr[t];
    }
  }
  return bad ? -1 : 0;
}
