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
 * sample in the low nibble.  DD_U16 holds unsigned 16-bit samples, low byte
 * first (the paper's three integer precisions, Sec. 5). */
typedef enum { DD_U8 = 1, DD_U4 = 2, DD_F32 = 3, DD_U16 = 4 } dd_dtype;

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
  int32_t kernel_ns, kernel_dm_per_wave, kernel_waves, kernel_chan_block; /* forward tile shape */
  int32_t kernel_order;       /* forward workgroup order (see dd_tiles) */
  size_t tune_ws_bytes;       /* device workspace dd_plan_autotune needs (tables of any shape) */
} dd_plan_info;

/* A tile choice for one direction of a plan.  A workgroup computes
 * waves * per_wave output rows (DM rows forward, channels adjoint) over 64 * ns
 * output samples, staging row_block input rows (channels forward, DM rows
 * adjoint) per LDS stage.  row_block 0 marks a direct-read shape of an integer
 * plan: no LDS staging, every (channel, DM) window read from the caches (for
 * wide delay spreads; a workgroup covers 63 * ns samples, 2 * 63 * ns for 4-bit
 * input). */
typedef struct {
  int32_t shape;  /* index of a shape compiled into the library for the plan's dtype */
  int32_t order;  /* workgroup order: 0 = time tiles fastest, 1 = each XCD takes whole time tiles,
                     2 = each XCD takes its time tiles for 4 output blocks at a time, 3 = each XCD
                     takes a contiguous run of time tiles, time tiles fastest */
  int32_t ns, per_wave, waves, row_block; /* the shape (output of dd_plan_get_tiles) */
  int32_t segs;   /* staging form of an integer shape (output): 0 = raw rows staged once, the
                     byte-phase copies built in LDS; > 0 = the phase copies loaded directly
                     (8-bit: four byte phases; 4-bit: the four even nibble phases, the odd
                     ones built in LDS; 16-bit: copies from bytes 0 and 2), each copy row in
                     at most segs 1 KiB loads */
} dd_tiles;

/* Result of dd_plan_autotune.  Times are per launch over the timed span. */
typedef struct {
  int32_t n_tried;           /* (shape, order) candidates timed */
  dd_tiles best;             /* fastest candidate, now the plan's choice */
  double best_ms;            /* its time */
  double default_ms;         /* time of the choice the plan had before tuning */
  int64_t timed_out_samples; /* output samples per row computed by each timed launch */
} dd_tune_report;

typedef struct dd_plan dd_plan;
typedef struct dd_batch dd_batch;

/*
 * Build a plan on the host: validate the description, evaluate the FP64 shift
 * table (Eq. 1 per channel and DM, rounded half up), derive N_out and the
 * per-DM-block delay spans that size the LDS staging, and choose a tile shape.
 * *out receives a new plan owned by the caller (free with dd_plan_destroy).
 * Limits, each refused with DD_ERR_RANGE: n_samp < 2^29; in_pitch_bytes < 2^31;
 * n_chan <= 65793 (DD_U8), 1118481 (DD_U4) or 65537 (DD_U16), so that integer
 * sums stay exact (see dd_execute); every shift fits int32; for DD_F32 plans a
 * delay spread that some compiled staging shape holds (integer plans fall back
 * to the direct-read shapes, which hold any spread).
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
 *          as uint8, packed uint4, uint16 or float32 per the plan's dtype.  16-byte aligned.
 *   d_out  device pointer, float32 [n_dm][out_pitch]; row d, columns 0..n_out-1 receive
 *          S(d, t).  Columns >= n_out are not written.  16-byte aligned.
 *   out_pitch  elements between output rows, >= n_out, multiple of 4.
 * Integer inputs accumulate exactly in 32-bit integers and are converted once
 * to float32: exact for 8- and 4-bit input (every sum is below 2^24 for
 * n_chan <= 65793 resp. 1118481); 16-bit sums (n_chan <= 65537) are exact
 * below 2^24 and rounded to nearest even above, as the conversion of the exact
 * sum would be.  Float input
 * accumulates in float32 in a fixed order: channels in groups of 32 summed in
 * order, then the group sums in order; the result does not depend on the tile shape.
 * Errors: DD_ERR_ARG, DD_ERR_ALIGN, DD_ERR_NOT_BOUND, DD_ERR_HIP.
 */
dd_status dd_execute(const dd_plan *plan, const void *d_in, float *d_out, int64_t out_pitch,
                     void *stream);

/*
 * dd_execute without a workspace, for callers that cannot allocate device
 * memory or bind one (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, result and errors as
 * dd_execute, but the plan need not be bound: on every call the plan's device
 * tables are copied (hipMemcpyAsync on `stream`) into a static device array of
 * DD_NOALLOC_TABLE_BYTES bytes inside the library, which every device the
 * library runs on holds until the process ends, and the forward kernels read
 * them there.  Nothing is allocated or freed.  Plans whose tables
 * (dev_table_bytes of dd_plan_query) exceed the array are refused with
 * DD_ERR_RANGE before anything is enqueued.  All calls on one device share the
 * array and it keeps only the last call's tables: calls on one device must not
 * overlap in time (one stream, or an explicit ordering between streams);
 * overlapping calls race on the tables.  Errors: those of dd_execute except
 * DD_ERR_NOT_BOUND, plus DD_ERR_RANGE.
 */
#define DD_NOALLOC_TABLE_BYTES ((size_t)32 << 20)
dd_status dd_execute_noalloc(const dd_plan *plan, const void *d_in, float *d_out, int64_t out_pitch,
                             void *stream);

/*
 * Adjoint (transpose of Eq. 3, "re-dispersion") for DD_F32 plans, in gather form:
 *     g(c, tau) = sum_d [0 <= tau - shift(c,d) < n_out] * y(d, tau - shift(c,d)).
 *   d_y        device pointer, float32 [n_dm][y_pitch], columns 0..n_out-1 read;
 *              4-byte aligned (a gradient tensor of any row length can be passed as is).
 *   y_pitch    elements, >= n_out (any value).
 *   d_grad_in  device pointer, float32 [n_chan] rows of in_pitch_bytes; columns
 *              0..n_samp-1 of every row are overwritten (exact zeros where no
 *              output reads the sample).
 * No atomics; DMs are summed in a fixed order (groups of 32 in order), so the
 * result is deterministic and independent of the tile shape.
 * Errors: DD_ERR_DTYPE (integer plan), DD_ERR_ARG, DD_ERR_ALIGN (d_y not 4-byte or d_grad
 * not 16-byte aligned), DD_ERR_NOT_BOUND, DD_ERR_HIP.
 */
dd_status dd_execute_adjoint(const dd_plan *plan, const float *d_y, int64_t y_pitch,
                             float *d_grad_in, void *stream);

/*
 * Tile shapes and their tuning.  The tile shape (output rows per workgroup,
 * samples per lane, input rows per LDS stage) and the workgroup order decide
 * speed only: results are bitwise identical for every choice (exact integer
 * sums; fixed-order float sums).  dd_plan_create picks the first compiled
 * shape that holds the plan's delay spread, 8-bit plans trying the phase-load
 * shapes first, in order 2 (16-bit plans take the 8-wave, 4-rows-per-wave,
 * 4-channel shape, phase-load form first, when two of its workgroups fit in
 * one CU's LDS); an 8- or 16-bit plan left with stages of at most 4 channels
 * (16-bit: other than that shape) takes the 4 rows x 4 waves direct-read shape
 * in order 1 (order 2 for 8-bit plans that fit only 1- or 2-channel stages);
 * 4-bit plans take the 2 rows x 8 waves direct-read shape in order 1 whatever
 * their spread; or the choice recorded for an identical plan in the tuning
 * cache (below).
 *
 * direction: 0 = forward; 1 = adjoint (DD_F32 plans only).
 *
 * dd_plan_shape_count: number of compiled shapes for the plan's dtype.
 * dd_plan_get_tiles: current choice for `direction`.
 * dd_plan_set_tiles: rebuild the plan's tables for compiled shape `shape` and
 *   workgroup order `order` (0 to 3).  DD_ERR_RANGE (plan unchanged) if the shape
 *   cannot stage the plan's delay spread.  On success the plan is unbound:
 *   query dev_table_bytes again and call dd_plan_bind before executing.
 * dd_plan_autotune: time every (shape, order) that holds the plan's spread and
 *   keep the fastest (the current choice stays unless another is at least 2%
 *   faster).  Each candidate runs on the caller's buffers over the first
 *   timed_out_samples output samples of every row (all of them for small plans;
 *   otherwise an eighth of the job, between 10^12 and 4*10^12 adds per launch),
 *   once to warm up and twice timed with HIP events on `stream`.  The call
 *   synchronises `stream`.
 *     forward: d_src is the input (as dd_execute), d_dst the output with
 *              `pitch` = out_pitch;
 *     adjoint: d_src is y with `pitch` = y_pitch, d_dst the gradient (as
 *              dd_execute_adjoint).
 *   d_dst's contents are unspecified afterwards.  d_ws (>= tune_ws_bytes of
 *   dd_plan_query, 16-byte aligned) receives each candidate's tables; on
 *   success the plan is bound to d_ws with the winner's tables.  If the
 *   environment variable DD_TUNE_CACHE names a file, the winner is appended to
 *   it (one text line per plan and direction) and later dd_plan_create calls
 *   for an identical plan description apply it.  *report may be NULL.
 *   Errors: DD_ERR_ARG, DD_ERR_ALIGN, DD_ERR_DTYPE, DD_ERR_HIP (plan unbound then).
 */
dd_status dd_plan_shape_count(const dd_plan *plan, int32_t *n);
dd_status dd_plan_get_tiles(const dd_plan *plan, int32_t direction, dd_tiles *tiles);
dd_status dd_plan_set_tiles(dd_plan *plan, int32_t direction, int32_t shape, int32_t order);
dd_status dd_plan_autotune(dd_plan *plan, int32_t direction, const void *d_src, float *d_dst, int64_t pitch,
                           void *d_ws, size_t ws_bytes, void *stream, dd_tune_report *report);

/*
 * Batch of independent forward transforms ("beams"), each with its own plan
 * (channel count, length, DM plan), run by persistent kernel launches that pull
 * (beam, DM block, time tile) work items from a device counter, largest items
 * first.  Every beam has a tile shape of its own, staged or direct-read; the
 * beams of one shape form a group, one persistent launch per group, the groups
 * independent of each other.  The launch sequence is recorded once as a HIP
 * graph and replayed by every dd_execute_batched call.  By default a beam runs
 * its plan's own forward tile shape (the plan's default, or what the plan was
 * set or tuned to), else (a staged shape whose LDS need falls in the 64 bytes
 * the persistent kernel keeps for itself) the first staged shape that holds the
 * beam (the phase-load shapes first), else the plan's default direct-read
 * shape; dd_batch_set_tiles puts every beam on one shape and dd_batch_autotune
 * chooses between these assignments.
 *
 * dd_batch_create: plans[0..n-1] must be integer plans (DD_U8, DD_U4 or DD_U16),
 *   all of one dtype, and outlive the batch.  Errors: DD_ERR_ARG, DD_ERR_DTYPE, DD_ERR_NOMEM.
 * dd_batch_workspace_bytes: device workspace dd_batch_bind needs (it does not depend on the shapes).
 * dd_batch_bind: d_in[b], d_out[b], out_pitch[b] as for dd_execute of plan b;
 *   d_workspace holds the group counters, the beam descriptors and the beams'
 *   tables (staged offsets, or the plain shift table for a direct-read shape;
 *   >= dd_batch_workspace_bytes, 16-byte aligned).  Uploads on
 *   `stream` and records the graph; re-binding re-records it.
 *   Errors: DD_ERR_ARG, DD_ERR_ALIGN, DD_ERR_HIP.
 * dd_execute_batched: replay the graph on `stream`.  Errors: DD_ERR_NOT_BOUND, DD_ERR_ARG (the
 *   current device is not the one the batch was bound on), DD_ERR_HIP.
 * dd_batch_get_tiles: the shape every beam runs (order is always 0: work items are claimed
 *   dynamically), or shape = -1 and all other fields 0 when the beams run different shapes.
 * dd_batch_get_beam_tiles: the shape beam `beam` (0..n-1, the order of dd_batch_create) runs.
 * dd_batch_set_tiles: put every beam on compiled shape `shape` (below dd_plan_shape_count of
 *   the beams' plans: staged or direct-read; DD_ERR_RANGE, batch unchanged, if a beam cannot
 *   be staged with it); unbinds the batch, which keeps its workspace size.
 * dd_batch_autotune: with the arguments of dd_batch_bind, time the current assignment, every
 *   beam at its default shape, and every staged shape with at least 32 DM rows per workgroup and
 *   every direct-read shape for all beams, each on the whole batch (one warm-up replay, one timed replay with HIP events on
 *   `stream`); keep the fastest (the current one stays unless another is at least 2% faster) and
 *   leave the batch bound with it.  Outputs are overwritten.  Synchronises `stream`.  *report may
 *   be NULL (best is as dd_batch_get_tiles; timed_out_samples is 0: whole replays are timed).
 *   Errors: as dd_batch_bind.
 */
dd_status dd_batch_create(const dd_plan *const *plans, int32_t n, dd_batch **out);
dd_status dd_batch_workspace_bytes(const dd_batch *batch, size_t *bytes);
dd_status dd_batch_bind(dd_batch *batch, const void *const *d_in, float *const *d_out,
                        const int64_t *out_pitch, void *d_workspace, size_t bytes, void *stream);
dd_status dd_execute_batched(dd_batch *batch, void *stream);
dd_status dd_batch_get_tiles(const dd_batch *batch, dd_tiles *tiles);
dd_status dd_batch_get_beam_tiles(const dd_batch *batch, int32_t beam, dd_tiles *tiles);
dd_status dd_batch_set_tiles(dd_batch *batch, int32_t shape);
dd_status dd_batch_autotune(dd_batch *batch, const void *const *d_in, float *const *d_out, const int64_t *out_pitch,
                            void *d_workspace, size_t bytes, void *stream, dd_tune_report *report);
void dd_batch_destroy(dd_batch *batch);

/*
 * Time binning ("downsampling"), which Secs. 5.2 and 5.3 apply to the input of
 * high-DM ranges and whose cost the real-time factor of Sec. 5.5 includes:
 *
 *     out(c, j) = sum_{i < factor} x(c, j*factor + i),   0 <= j < n_bins = n_samp / factor,
 *
 * sums without normalisation; a trailing partial bin is dropped.
 *   dtype      input encoding (a dd_dtype); the output encoding is
 *              dd_bin_out_dtype(dtype): DD_U8 and DD_U4 give exact uint16 sums,
 *              DD_U16 gives float32 holding the exact integer sums (below 2^24),
 *              DD_F32 gives float32 sums (float32 arithmetic, an order that
 *              depends only on `factor`).  (Surveys bin 16-bit input into
 *              split uint16 planes instead; see dd_survey_create.)
 *   d_in       device pointer, [n_chan] rows of in_pitch_bytes (>= one packed row,
 *              multiple of 16); samples 0..n_bins*factor-1 of each row are read.
 *   factor     1..256 (keeps every integer sum exact in its output type).
 *   d_out      device pointer, [n_chan] rows of out_pitch_bytes (>= n_bins output
 *              elements, multiple of 16); columns 0..n_bins-1 are written, nothing
 *              else.  Must not overlap d_in.
 * Both pointers 16-byte aligned.  Asynchronous on `stream`; allocates nothing.
 * Errors: DD_ERR_ARG, DD_ERR_TOO_SHORT (n_bins == 0), DD_ERR_ALIGN, DD_ERR_RANGE, DD_ERR_HIP.
 */
dd_status dd_bin_time(int32_t dtype, const void *d_in, int64_t in_pitch_bytes, int32_t n_chan, int64_t n_samp,
                      int32_t factor, void *d_out, int64_t out_pitch_bytes, void *stream);
/* Output encoding of dd_bin_time for an input encoding (0 for an unknown one). */
int32_t dd_bin_out_dtype(int32_t dtype);

/*
 * Corner turn of the input (the transposing of the input data that the
 * pipelines of Sec. 5.3 run before the transform and the real-time factor of
 * Sec. 5.5 includes): time-major spectra to channel-major rows,
 *
 *     out(c, t) = in(t, c),   0 <= c < n_chan, 0 <= t < n_samp.
 *
 *   dtype      DD_U8, DD_U16 or DD_F32 (element transpose), or DD_U4: a spectrum
 *              holds channel pairs per byte and an output row time pairs per byte,
 *              the even index in the low nibble (n_samp even).
 *   d_in       device pointer, [n_samp] spectra of in_pitch_bytes (>= the packed
 *              spectrum, multiple of 16).
 *   d_out      device pointer, [n_chan] rows of out_pitch_bytes (>= the packed row,
 *              multiple of 16); exactly the row bytes are written.  Must not overlap d_in.
 * Both 16-byte aligned.  Asynchronous on `stream`; allocates nothing.
 * Errors: DD_ERR_ARG, DD_ERR_ALIGN, DD_ERR_RANGE, DD_ERR_HIP.
 */
dd_status dd_corner_turn(int32_t dtype, const void *d_in, int64_t in_pitch_bytes, int32_t n_chan, int64_t n_samp,
                         void *d_out, int64_t out_pitch_bytes, void *stream);

/*
 * Multi-range DM plan ("survey"): several DM ranges, each with its own fixed
 * step and time-binning factor, over one filterbank (the plan of Table
 * tab:plans in Sec. 5.2; the binned high-DM ranges of Sec. 5.3).
 *
 * Range r is an ordinary plan over the input binned by bin_r: n_samp / bin_r
 * samples of t_samp * bin_r seconds in encoding dd_bin_out_dtype(dtype) (the
 * input itself when bin_r == 1), with DM_d = dm_start_r + d * dm_step_r.  Its
 * output is that plan's S(d, t), t counted in binned samples.  Ranges that
 * share a factor share one binned copy.  For DD_U16 input the binned copy
 * instead holds the exact bin sums (below 2^24) as two uint16 planes per row,
 * their low and their high halves, and the range's plan is a DD_U16 plan over
 * the low plane: dd_survey_execute sums both planes exactly in 32-bit integers
 * and writes the float32 of low + 2^16 * high, so every output of an integer
 * survey is the float32 of its exact integer sum (rounded once, to nearest
 * even, above 2^24).
 *
 * dd_survey_create: `base` gives the filterbank (n_chan, n_samp, dtype, band,
 *   t_samp_s, in_pitch_bytes); its DM fields are ignored.  ranges[0..n-1]:
 *   n_dm > 0, dm_step >= 0, dm_start >= 0, bin in 1..256.  flags: 0, or
 *   DD_SURVEY_TIME_MAJOR: the input is time-major spectra ([n_samp] spectra of
 *   base->in_pitch_bytes, as dd_corner_turn reads them); every execute first
 *   turns it into a channel-major copy in the workspace.  Errors as
 *   dd_plan_create for each range's plan, plus DD_ERR_ARG.
 * dd_survey_plan: the plan of range r, owned by the survey (query it for
 *   n_out; re-tiling it through dd_plan_set_tiles unbinds the survey).
 * dd_survey_workspace_bytes: device workspace dd_survey_bind needs: the binned
 *   copies plus every range's tables at their largest (so re-tiling or tuning
 *   a range never changes the layout).
 * dd_survey_bind: lay the workspace out (16-byte aligned, >= the size above)
 *   and enqueue the table uploads on `stream`.  Errors: DD_ERR_ARG, DD_ERR_ALIGN, DD_ERR_HIP.
 * dd_survey_autotune: bin the input, then dd_plan_autotune every range
 *   (forward) on its own input and d_out[r]; leaves the survey bound.  Synchronises `stream`.
 * dd_survey_execute: on `stream`, corner-turn the input (DD_SURVEY_TIME_MAJOR),
 *   bin it once per distinct factor > 1, then run every range's forward transform: d_out[r] is float32
 *   [n_dm_r][out_pitch[r]] as for dd_execute of range r's plan.
 *   Errors: DD_ERR_ARG, DD_ERR_ALIGN, DD_ERR_NOT_BOUND, DD_ERR_HIP.
 */
typedef struct {
  double dm_start; /* first trial DM of the range, pc cm^-3 */
  double dm_step;  /* DM step of the range */
  int32_t n_dm;    /* trial DMs in the range */
  int32_t bin;     /* time-binning factor applied to the input for this range, 1..256 */
} dd_range;

typedef struct dd_survey dd_survey;

#define DD_SURVEY_TIME_MAJOR 1

dd_status dd_survey_create(const dd_plan_desc *base, const dd_range *ranges, int32_t n_ranges, int32_t flags,
                           dd_survey **out);
dd_status dd_survey_plan(const dd_survey *survey, int32_t r, dd_plan **plan);
dd_status dd_survey_workspace_bytes(const dd_survey *survey, size_t *bytes);
dd_status dd_survey_bind(dd_survey *survey, void *d_workspace, size_t bytes, void *stream);
dd_status dd_survey_autotune(dd_survey *survey, const void *d_in, float *const *d_out, const int64_t *out_pitch,
                             void *stream);
dd_status dd_survey_execute(const dd_survey *survey, const void *d_in, float *const *d_out,
                            const int64_t *out_pitch, void *stream);
void dd_survey_destroy(dd_survey *survey);

/* Static text for a status code, and the calling thread's last error detail. */
const char *dd_status_string(dd_status status);
const char *dd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DD_H */
