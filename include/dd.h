/*
 * dd.h -- C ABI of the MI355X (gfx950) brute-force incoherent dedispersion library.
 *
 * The transform (Novotny et al., "Accelerating Dedispersion using Many-Core
 * Architectures", Sec. 2, Eq. 3 and Algorithm 1) maps a channel-major
 * filterbank x(c, t) to the dedispersed plane
 *
 *     S(d, t) = sum_{c=0}^{N_ch-1} x(c, t + shift(c, d)),   0 <= t < N_out,
 *
 * with one output row per trial DM, DM_d = dm_start + d * dm_step (the fixed-step
 * plan of Sec. 5.1), no normalisation, and N_out = N_t - max_{c,d} shift(c, d).
 * The integer delay follows the cold-plasma law of Sec. 1, Eq. 1, with channel c
 * at f_high - c * df as in the per-channel coefficients of Sec. 4.1:
 *
 *     shift(c, d) = floor(DM_d * 4.148808e3 * (f_c^-2 - f_high^-2) / t_samp + 1/2)
 *
 * evaluated once on the host in IEEE FP64 in exactly that order (f in MHz,
 * t_samp in seconds).  The device only ever sees the integer table.
 *
 * Conventions for every function below:
 *   - The return value is a dd_status: DD_OK (0) or a negative error code.  No
 *     function throws, aborts or prints.  dd_last_error() returns a
 *     thread-local text describing the most recent failure on the calling thread.
 *   - "Device pointer" means memory the caller allocated on the current HIP
 *     device; the library never allocates, frees or synchronises device memory.
 *   - "stream" is a hipStream_t passed as void* (NULL = the default stream).  All
 *     execute calls are asynchronous on that stream; the caller keeps every
 *     buffer and the plan alive until the queued work has finished.
 *   - Argument and shape checks happen on the host before anything is enqueued;
 *     a failed check enqueues nothing.  Device faults surface at the caller's
 *     next synchronisation, as for any HIP call.
 */
#ifndef DD_H
#define DD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DD_OK = 0,
  DD_ERR_ARG = -1,       /* null pointer, non-positive size, unknown dtype, bad plan field */
  DD_ERR_TOO_SHORT = -2, /* n_samp <= largest shift: no complete output sample */
  DD_ERR_RANGE = -3,     /* channel frequency <= 0 or > f_high, negative DM, int32/size overflow */
  DD_ERR_ALIGN = -4,     /* a device pointer is not 16-byte aligned, or a pitch breaks 16-byte rows */
  DD_ERR_DTYPE = -5,     /* operation not defined for the plan's input type */
  DD_ERR_NOT_BOUND = -6, /* execute before dd_plan_bind / dd_batch_bind */
  DD_ERR_HIP = -7,       /* a HIP runtime call failed; dd_last_error() has its text */
  DD_ERR_NOMEM = -8      /* host allocation failed */
} dd_status;

/* Input sample encodings.  DD_U4 holds two samples per byte, the even time
 * sample in the low nibble. */
typedef enum { DD_U8 = 1, DD_U4 = 2, DD_F32 = 3 } dd_dtype;

/* Plan description (Sec. 2 problem statement; fixed-step DM plan of Sec. 5.1). */
typedef struct {
  int32_t n_chan;              /* number of channels N_ch > 0 */
  int64_t n_samp;              /* time samples per channel N_t > max shift; even for DD_U4 */
  int32_t dtype;               /* a dd_dtype */
  double f_high_mhz;           /* frequency of channel 0 (the top of the band), MHz, > 0 */
  double chan_bw_mhz;          /* channel spacing df >= 0: channel c at f_high - c*df */
  const double *chan_freq_mhz; /* optional explicit [n_chan] frequencies in (0, f_high];
                                  NULL = uniform spacing.  Copied by dd_plan_create. */
  double t_samp_s;             /* sampling time, seconds, > 0 */
  double dm_start;             /* first trial DM, pc cm^-3, >= 0 */
  double dm_step;              /* DM step, >= 0 */
  int32_t n_dm;                /* number of trial DMs > 0 */
  int64_t in_pitch_bytes;      /* bytes between consecutive channel rows of the input;
                                  0 = tightly packed rows.  Must be a multiple of 16. */
} dd_plan_desc;

/* What a plan needs and produces (filled by dd_plan_query). */
typedef struct {
  int64_t n_out;              /* valid output samples per DM row: n_samp - max_shift */
  int32_t max_shift;          /* largest entry of the shift table */
  int32_t n_dm, n_chan;
  int64_t in_pitch_bytes;     /* effective input row pitch */
  size_t dev_table_bytes;     /* device workspace dd_plan_bind needs (shift table + tiling tables) */
  const int32_t *host_shift;  /* the FP64-derived table, int32 [n_dm][n_chan]; owned by the plan */
  int32_t kernel_ns, kernel_dm_per_wave, kernel_waves, kernel_chan_block; /* chosen tile shape */
} dd_plan_info;

typedef struct dd_plan dd_plan;
typedef struct dd_batch dd_batch;

/*
 * Build a plan on the host: validate the description, evaluate the FP64 shift
 * table (Eq. 1 per channel and DM, rounded half up), derive N_out and the
 * per-DM-block delay spans that size the LDS staging, and choose a tile shape.
 * *out receives a new plan owned by the caller (free with dd_plan_destroy).
 * Errors: DD_ERR_ARG, DD_ERR_RANGE, DD_ERR_TOO_SHORT, DD_ERR_NOMEM.
 */
dd_status dd_plan_create(const dd_plan_desc *desc, dd_plan **out);

/* Release a plan.  Safe on NULL.  Queued work that uses it must have finished. */
void dd_plan_destroy(dd_plan *plan);

/* Fill *info with the plan's sizes and tables.  Errors: DD_ERR_ARG. */
dd_status dd_plan_query(const dd_plan *plan, dd_plan_info *info);

/*
 * Bind the plan to caller-owned device workspace of at least
 * info.dev_table_bytes bytes (16-byte aligned) on the current device, and
 * enqueue the upload of the plan's tables into it on `stream`.  The workspace
 * must stay allocated while the plan is used.  A plan can be re-bound.
 * Errors: DD_ERR_ARG, DD_ERR_ALIGN, DD_ERR_HIP.
 */
dd_status dd_plan_bind(dd_plan *plan, void *d_workspace, size_t bytes, void *stream);

/*
 * Forward transform (Eq. 3 / Algorithm 1) on `stream`.
 *   d_in   device pointer, [n_chan] rows of in_pitch_bytes; row c holds x(c, 0..n_samp-1)
 *          as uint8, packed uint4 or float32 per the plan's dtype.  16-byte aligned.
 *   d_out  device pointer, float32 [n_dm][out_pitch]; row d, columns 0..n_out-1 receive
 *          S(d, t).  Columns >= n_out are not written.  16-byte aligned.
 *   out_pitch  elements between output rows, >= n_out, multiple of 4.
 * Integer inputs accumulate exactly in int32 and are converted once to float32
 * (exact: every sum is below 2^24 for n_chan <= 65793).  Float input
 * accumulates in float32 in a fixed order: channels in groups of 32 summed in
 * order, then the group sums in order; the result does not depend on the tile shape.
 * Errors: DD_ERR_ARG, DD_ERR_ALIGN, DD_ERR_NOT_BOUND, DD_ERR_HIP.
 */
dd_status dd_execute(const dd_plan *plan, const void *d_in, float *d_out, int64_t out_pitch,
                     void *stream);

/*
 * Adjoint (transpose of Eq. 3, "re-dispersion") for DD_F32 plans, in gather form:
 *     g(c, tau) = sum_d [0 <= tau - shift(c,d) < n_out] * y(d, tau - shift(c,d)).
 *   d_y        device pointer, float32 [n_dm][y_pitch], columns 0..n_out-1 read.
 *   y_pitch    elements, >= n_out, multiple of 4.
 *   d_grad_in  device pointer, float32 [n_chan] rows of in_pitch_bytes; columns
 *              0..n_samp-1 of every row are overwritten (exact zeros where no
 *              output reads the sample).
 * No atomics; DMs are summed in a fixed order (groups of 32 in order), so the
 * result is deterministic and independent of the tile shape.
 * Errors: DD_ERR_DTYPE (integer plan), DD_ERR_ARG, DD_ERR_ALIGN, DD_ERR_NOT_BOUND, DD_ERR_HIP.
 */
dd_status dd_execute_adjoint(const dd_plan *plan, const float *d_y, int64_t y_pitch,
                             float *d_grad_in, void *stream);

/*
 * Batch of independent forward transforms ("beams"), each with its own plan
 * (channel count, length, DM plan), run as ONE persistent kernel launch that
 * pulls (beam, DM block, time tile) work items from a device counter, largest
 * items first.  The launch sequence is recorded once as a HIP graph and
 * replayed by every dd_execute_batched call.
 *
 * dd_batch_create: plans[0..n-1] must be DD_U8 or DD_U4 plans and outlive the
 *   batch.  Errors: DD_ERR_ARG, DD_ERR_DTYPE, DD_ERR_NOMEM.
 * dd_batch_workspace_bytes: device workspace dd_batch_bind needs.
 * dd_batch_bind: d_in[b], d_out[b], out_pitch[b] as for dd_execute of plan b;
 *   d_workspace holds the work list, descriptors, the beams' tables and the
 *   counter (>= dd_batch_workspace_bytes, 16-byte aligned).  Uploads on
 *   `stream` and records the graph; re-binding re-records it.
 *   Errors: DD_ERR_ARG, DD_ERR_ALIGN, DD_ERR_HIP.
 * dd_execute_batched: replay the graph on `stream`.  Errors: DD_ERR_NOT_BOUND, DD_ERR_HIP.
 */
dd_status dd_batch_create(const dd_plan *const *plans, int32_t n, dd_batch **out);
dd_status dd_batch_workspace_bytes(const dd_batch *batch, size_t *bytes);
dd_status dd_batch_bind(dd_batch *batch, const void *const *d_in, float *const *d_out,
                        const int64_t *out_pitch, void *d_workspace, size_t bytes, void *stream);
dd_status dd_execute_batched(dd_batch *batch, void *stream);
void dd_batch_destroy(dd_batch *batch);

/* Static text for a status code, and the calling thread's last error detail. */
const char *dd_status_string(dd_status status);
const char *dd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DD_H */
