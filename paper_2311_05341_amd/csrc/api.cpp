// C ABI entry points: argument checking, plan lifetime, table upload and
// kernel dispatch.  Declarations and contracts are in include/dd.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <new>
#include <string>

#include "dd_internal.h"

namespace dd {

static thread_local std::string g_last_error;

dd_status fail(dd_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

static dd_status hip_fail(int e, const char *what) {
  return fail(DD_ERR_HIP, std::string(what) + ": " + hipGetErrorString((hipError_t)e));
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

static int64_t packed_row_bytes(int dtype, int64_t n_samp) {
  if (dtype == DD_U4) return n_samp / 2;
  if (dtype == DD_U16) return n_samp * 2;
  if (dtype == DD_F32) return n_samp * 4;
  return n_samp;
}

dd_status hip_error(int e, const char *what) { return hip_fail(e, what); }

int copy_tables(const dd_plan &p, void *dst, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  uint8_t *base = (uint8_t *)dst;
  const TableLayout L = table_layout(p);
  hipError_t e = hipSuccess;
  if (p.desc.dtype != DD_F32 && is_direct(p.fwd)) {  // the direct kernel reads the plain shift table
    e = hipMemcpyAsync(base + L.int_offs, p.shift.data(), p.shift.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
  } else if (p.desc.dtype != DD_F32) {
    e = hipMemcpyAsync(base + L.int_offs, p.itab.offs.data(), p.itab.offs.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(base + L.int_sbase, p.itab.sbase.data(), p.itab.sbase.size() * 4, hipMemcpyHostToDevice, st);
  } else {
    const FloatTables *tabs[2] = {&p.ftab_fwd, &p.ftab_adj};
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
      e = hipMemcpyAsync(base + L.f_offs[k], tabs[k]->offs.data(), tabs[k]->offs.size() * 2, hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(base + L.f_sbase[k], tabs[k]->sbase.data(), tabs[k]->sbase.size() * 4,
                           hipMemcpyHostToDevice, st);
    }
  }
  return (int)e;
}

// Enqueue the upload of the plan's current tables into `ws` and mark the plan
// bound to it on the current device.
dd_status upload_tables(dd_plan &p, void *ws, void *stream) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const int ce = copy_tables(p, ws, stream);
  if (ce) return hip_fail(ce, "table upload");
  p.d_tables = ws;
  p.device = dev;
  p.bound = true;
  return DD_OK;
}

}  // namespace dd

using namespace dd;

extern "C" {

dd_status dd_plan_create(const dd_plan_desc *desc, dd_plan **out) {
  if (!desc || !out) return fail(DD_ERR_ARG, "null argument");
  *out = nullptr;
  const dd_plan_desc &d = *desc;
  if (d.n_chan <= 0 || d.n_dm <= 0 || d.n_samp <= 0) return fail(DD_ERR_ARG, "n_chan, n_dm and n_samp must be positive");
  if (d.dtype != DD_U8 && d.dtype != DD_U4 && d.dtype != DD_U16 && d.dtype != DD_F32)
    return fail(DD_ERR_ARG, "unknown dtype");
  if (d.dtype == DD_U4 && (d.n_samp & 1)) return fail(DD_ERR_ARG, "n_samp must be even for 4-bit input");
  if (!(d.t_samp_s > 0.0) || !isfinite(d.t_samp_s)) return fail(DD_ERR_ARG, "t_samp must be positive");
  if (!(d.f_high_mhz > 0.0) || !isfinite(d.f_high_mhz)) return fail(DD_ERR_RANGE, "f_high must be positive");
  if (!(d.chan_bw_mhz >= 0.0) || !isfinite(d.chan_bw_mhz)) return fail(DD_ERR_ARG, "chan_bw must be >= 0");
  if (!(d.dm_start >= 0.0) || !isfinite(d.dm_start)) return fail(DD_ERR_RANGE, "dm_start must be >= 0");
  if (!(d.dm_step >= 0.0) || !isfinite(d.dm_step)) return fail(DD_ERR_RANGE, "dm_step must be >= 0");
  if (d.n_samp >= ((int64_t)1 << 29)) return fail(DD_ERR_RANGE, "n_samp must be below 2^29");
  // Exactness of int32 accumulation and float output: every sum below 2^24.
  if (d.dtype == DD_U8 && d.n_chan > 65793) return fail(DD_ERR_RANGE, "more than 65793 8-bit channels cannot be summed exactly in float32");
  if (d.dtype == DD_U4 && d.n_chan > 1118481) return fail(DD_ERR_RANGE, "too many 4-bit channels for exact float32 output");
  // 16-bit: the per-sample 32-bit totals must not wrap: 65535 * n_chan < 2^32.
  if (d.dtype == DD_U16 && d.n_chan > 65537) return fail(DD_ERR_RANGE, "more than 65537 16-bit channels overflow 32-bit sums");
  const int64_t row = packed_row_bytes(d.dtype, d.n_samp);
  const int64_t pitch = d.in_pitch_bytes ? d.in_pitch_bytes : row;
  if (pitch < row) return fail(DD_ERR_ARG, "in_pitch_bytes smaller than one row");
  if (pitch % 16) return fail(DD_ERR_ALIGN, "input row pitch must be a multiple of 16 bytes");
  if (pitch >= ((int64_t)1 << 31)) return fail(DD_ERR_RANGE, "input rows must be shorter than 2^31 bytes");
  if ((double)d.n_dm * (double)d.n_chan * 12.0 > 9.0e18) return fail(DD_ERR_RANGE, "table size overflow");

  dd_plan *p = new (std::nothrow) dd_plan();
  if (!p) return fail(DD_ERR_NOMEM, "plan allocation failed");
  p->desc = d;
  p->in_pitch_bytes = pitch;
  if (d.chan_freq_mhz) {
    try {
      p->freqs.assign(d.chan_freq_mhz, d.chan_freq_mhz + d.n_chan);
    } catch (const std::bad_alloc &) {
      delete p;
      return fail(DD_ERR_NOMEM, "frequency table allocation failed");
    }
  }
  p->desc.chan_freq_mhz = nullptr;
  p->desc.in_pitch_bytes = pitch;
  dd_status st = build_shift_table(*p);
  if (st == DD_OK) st = choose_forward_tiles(*p);
  if (st == DD_OK) apply_tune_cache(*p);
  if (st != DD_OK) {
    delete p;
    return st;
  }
  *out = p;
  return DD_OK;
}

void dd_plan_destroy(dd_plan *plan) { delete plan; }

dd_status dd_plan_query(const dd_plan *p, dd_plan_info *info) {
  if (!p || !info) return fail(DD_ERR_ARG, "null argument");
  memset(info, 0, sizeof(*info));
  info->n_out = p->n_out;
  info->max_shift = p->max_shift;
  info->n_dm = p->desc.n_dm;
  info->n_chan = p->desc.n_chan;
  info->in_pitch_bytes = p->in_pitch_bytes;
  info->dev_table_bytes = table_bytes(*p);
  info->host_shift = p->shift.data();
  info->kernel_ns = p->fwd.ns;
  info->kernel_dm_per_wave = p->fwd.dm_per_wave;
  info->kernel_waves = p->fwd.waves;
  info->kernel_chan_block = p->fwd.chan_block;
  info->kernel_order = p->fwd.order;
  info->tune_ws_bytes = tune_table_bytes(*p);
  return DD_OK;
}

dd_status dd_plan_bind(dd_plan *p, void *ws, size_t bytes, void *stream) {
  if (!p || !ws) return fail(DD_ERR_ARG, "null argument");
  if (!aligned16(ws)) return fail(DD_ERR_ALIGN, "workspace must be 16-byte aligned");
  if (bytes < table_bytes(*p)) return fail(DD_ERR_ARG, "workspace smaller than dev_table_bytes");
  return upload_tables(*p, ws, stream);
}

static dd_status check_exec(const dd_plan *p) {
  if (!p) return fail(DD_ERR_ARG, "null plan");
  if (!p->bound) return fail(DD_ERR_NOT_BOUND, "plan is not bound to device workspace");
  int dev = -1;
  if (hipGetDevice(&dev) == hipSuccess && dev != p->device)
    return fail(DD_ERR_ARG, "plan is bound on another device");
  return DD_OK;
}

dd_status dd_execute(const dd_plan *p, const void *d_in, float *d_out, int64_t out_pitch, void *stream) {
  dd_status st = check_exec(p);
  if (st != DD_OK) return st;
  if (!d_in || !d_out) return fail(DD_ERR_ARG, "null buffer");
  if (!aligned16(d_in) || !aligned16(d_out)) return fail(DD_ERR_ALIGN, "buffers must be 16-byte aligned");
  if (out_pitch < p->n_out) return fail(DD_ERR_ARG, "out_pitch < n_out");
  if (out_pitch % 4) return fail(DD_ERR_ALIGN, "out_pitch must be a multiple of 4 elements");
  int e = p->desc.dtype == DD_F32 ? launch_forward_f32(*p, p->d_tables, d_in, d_out, out_pitch, stream)
                                  : launch_forward_int(*p, p->d_tables, d_in, d_out, out_pitch, stream);
  if (e) return hip_fail(e, "forward launch");
  return DD_OK;
}

dd_status dd_execute_adjoint(const dd_plan *p, const float *d_y, int64_t y_pitch, float *d_grad, void *stream) {
  if (p && p->desc.dtype != DD_F32) return fail(DD_ERR_DTYPE, "the adjoint is defined for float32 plans only");
  dd_status st = check_exec(p);
  if (st != DD_OK) return st;
  if (!d_y || !d_grad) return fail(DD_ERR_ARG, "null buffer");
  // y rows are staged by 16-byte loads from 4-byte-aligned row starts (every
  // dword range-checked against the row), so y only needs float alignment
  if (((uintptr_t)d_y & 3u) || !aligned16(d_grad))
    return fail(DD_ERR_ALIGN, "d_y must be 4-byte and d_grad 16-byte aligned");
  if (y_pitch < p->n_out) return fail(DD_ERR_ARG, "y_pitch < n_out");
  int e = launch_adjoint(*p, p->d_tables, d_y, y_pitch, d_grad, stream);
  if (e) return hip_fail(e, "adjoint launch");
  return DD_OK;
}

const char *dd_status_string(dd_status s) {
  switch (s) {
    case DD_OK: return "ok";
    case DD_ERR_ARG: return "invalid argument";
    case DD_ERR_TOO_SHORT: return "input shorter than the largest delay";
    case DD_ERR_RANGE: return "value out of range";
    case DD_ERR_ALIGN: return "misaligned pointer or pitch";
    case DD_ERR_DTYPE: return "operation not defined for this input type";
    case DD_ERR_NOT_BOUND: return "plan or batch not bound to device workspace";
    case DD_ERR_HIP: return "HIP runtime error";
    case DD_ERR_NOMEM: return "host allocation failed";
  }
  return "unknown status";
}

const char *dd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
