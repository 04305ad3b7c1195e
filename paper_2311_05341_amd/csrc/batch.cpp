// Batched forward: many beams, each with its own plan, in one persistent
// kernel launch recorded once as a HIP graph (counter reset, then the
// persistent kernel) and replayed by dd_execute_batched.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "dd_internal.h"

using namespace dd;

struct dd_batch {
  std::vector<const dd_plan *> plans;
  int dtype = 0;
  int shape = 0;                // index of the shared LDS shape in kIntShapes
  TileCfg tile;                 // shared tile shape (ns, dm_per_wave, waves)
  std::vector<IntTables> tables;  // per beam (original index), for the shared shape
  int lds_bytes = 0;
  std::vector<int> order;       // beams in decreasing per-item cost
  std::vector<BeamDesc> descs;  // in `order`
  long long n_items = 0;
  size_t table_off = 0, ws_bytes = 0;
  std::vector<size_t> table_offs, sbase_offs;  // per beam (original index)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool bound = false;
  int device = -1;
};

static const int kBatchLdsLimit = 160 * 1024 - 64;  // leaves room for the claimed-item slot

static size_t up256(size_t v) { return (v + 255) / 256 * 256; }

static void release_graph(dd_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Table bytes of one beam's plan under LDS shape k (offsets, stage bases), each
// rounded up to 256 bytes.
static void int_table_bytes(const dd_plan &p, const int *k, size_t *offs, size_t *sbase) {
  const int64_t nd = p.desc.n_dm, nc = p.desc.n_chan, dblk = (int64_t)k[1] * k[2];
  const int64_t n_dblk = (nd + dblk - 1) / dblk, rp = k[1] < 2 ? 2 : k[1], ncp = (nc + k[3] - 1) / k[3] * k[3];
  *offs = up256((size_t)(n_dblk * k[2] * ncp * rp) * sizeof(uint16_t));
  *sbase = up256((size_t)(n_dblk * nc) * sizeof(int32_t));
}

// Switch the batch to LDS shape s: every beam's tables, the launch geometry and
// the work list.  DD_ERR_RANGE (batch unchanged) if a beam cannot be staged.
static dd_status batch_set_shape(dd_batch *b, int s) {
  const int n = (int)b->plans.size();
  const int *k = kIntShapes[s];
  std::vector<IntTables> tabs(n);
  int lds = 0;
  for (int i = 0; i < n; ++i) {
    const dd_status st = build_int_tables(*b->plans[i], k[0], k[1], k[2], k[3], k[4], kBatchLdsLimit, &tabs[i]);
    if (st != DD_OK) return st;
    lds = std::max(lds, tabs[i].lds_bytes);
  }
  b->tables = std::move(tabs);
  b->shape = s;
  b->tile.ns = k[0];
  b->tile.dm_per_wave = k[1];
  b->tile.waves = k[2];
  b->tile.chan_block = k[3];
  b->tile.segs = k[4];
  b->lds_bytes = lds;
  const int dm_tile = k[1] * k[2], t_tile = 64 * k[0];
  b->descs.resize(n);
  long long items = 0;
  for (int q = 0; q < n; ++q) {
    const int i = b->order[q];
    const dd_plan &p = *b->plans[i];
    BeamDesc &d = b->descs[q];
    memset(&d, 0, sizeof(d));
    d.n_chan = p.desc.n_chan;
    d.n_dm = p.desc.n_dm;
    d.n_samp = p.desc.n_samp;
    d.n_out = p.n_out;
    d.pitch = p.in_pitch_bytes;
    d.row_bytes = b->tables[i].row_bytes;
    d.chan_block = b->tables[i].chan_block;
    d.tiles_t = (int)((p.n_out + t_tile - 1) / t_tile);
    d.tiles_d = (p.desc.n_dm + dm_tile - 1) / dm_tile;
    d.item_begin = items;
    items += (long long)d.tiles_t * d.tiles_d;
  }
  b->n_items = items;
  b->bound = false;
  return DD_OK;
}

extern "C" {

dd_status dd_batch_create(const dd_plan *const *plans, int32_t n, dd_batch **out) {
  if (!plans || !out || n <= 0) return fail(DD_ERR_ARG, "need at least one plan");
  *out = nullptr;
  dd_batch *b = new (std::nothrow) dd_batch();
  if (!b) return fail(DD_ERR_NOMEM, "batch allocation failed");
  b->dtype = plans[0] ? plans[0]->desc.dtype : 0;
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) { delete b; return fail(DD_ERR_ARG, "null plan in batch"); }
    if (plans[i]->desc.dtype != DD_U8 && plans[i]->desc.dtype != DD_U4 && plans[i]->desc.dtype != DD_U16) {
      delete b;
      return fail(DD_ERR_DTYPE, "batches take integer (8-, 4- or 16-bit) plans");
    }
    if (plans[i]->desc.dtype != b->dtype) { delete b; return fail(DD_ERR_DTYPE, "all beams of a batch share one dtype"); }
    b->plans.push_back(plans[i]);
  }
  // Work items: beams ordered by per-item cost (channels x DM rows per tile), largest first.
  b->order.resize(n);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) {
    return b->plans[a]->desc.n_chan > b->plans[c]->desc.n_chan;
  });
  // Workspace layout: counter, descriptors, then per beam room for its tables
  // under the largest compiled shape, so changing the shape never moves them.
  size_t off = up256(sizeof(unsigned long long)) + up256(sizeof(BeamDesc) * (size_t)n);
  b->table_off = off;
  b->table_offs.assign(n, 0);
  b->sbase_offs.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    size_t ob = 0, sbb = 0;
    for (int s = 0; s < kNumIntShapes; ++s) {
      size_t o, sb;
      int_table_bytes(*b->plans[i], kIntShapes[s], &o, &sb);
      ob = std::max(ob, o);
      sbb = std::max(sbb, sb);
    }
    b->table_offs[i] = off;
    off += ob;
    b->sbase_offs[i] = off;
    off += sbb;
  }
  b->ws_bytes = off;
  // One tile shape for all beams: the first compiled shape every beam can stage
  // (two workgroups' worth of LDS is not required: the kernel runs one per CU),
  // phase-load shapes first for 8-bit beams.
  dd_status st = DD_ERR_RANGE;
  for (int pass = 0; pass < 2 && st != DD_OK; ++pass)
    for (int s = 0; s < kNumIntShapes && st != DD_OK; ++s) {
      if ((kIntShapes[s][4] > 0) != (pass == 0)) continue;
      st = batch_set_shape(b, s);
      if (st == DD_ERR_NOMEM) { delete b; return st; }
    }
  if (st != DD_OK) { delete b; return fail(DD_ERR_RANGE, "a beam's delay spread exceeds the LDS staging capacity"); }
  *out = b;
  return DD_OK;
}

dd_status dd_batch_workspace_bytes(const dd_batch *b, size_t *bytes) {
  if (!b || !bytes) return fail(DD_ERR_ARG, "null argument");
  *bytes = b->ws_bytes;
  return DD_OK;
}

dd_status dd_batch_bind(dd_batch *b, const void *const *d_in, float *const *d_out, const int64_t *out_pitch,
                        void *ws, size_t bytes, void *stream) {
  if (!b || !d_in || !d_out || !out_pitch || !ws) return fail(DD_ERR_ARG, "null argument");
  if (((uintptr_t)ws & 15u) != 0) return fail(DD_ERR_ALIGN, "workspace must be 16-byte aligned");
  if (bytes < b->ws_bytes) return fail(DD_ERR_ARG, "workspace smaller than dd_batch_workspace_bytes");
  const int n = (int)b->plans.size();
  for (int i = 0; i < n; ++i) {
    if (!d_in[i] || !d_out[i]) return fail(DD_ERR_ARG, "null beam buffer");
    if (((uintptr_t)d_in[i] & 15u) || ((uintptr_t)d_out[i] & 15u)) return fail(DD_ERR_ALIGN, "beam buffers must be 16-byte aligned");
    if (out_pitch[i] < b->plans[i]->n_out || (out_pitch[i] & 3)) return fail(DD_ERR_ARG, "bad beam out_pitch");
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(DD_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  uint8_t *base = (uint8_t *)ws;
  for (int k = 0; k < n; ++k) {
    const int i = b->order[k];
    BeamDesc &d = b->descs[k];
    d.x = (const uint8_t *)d_in[i];
    d.out = d_out[i];
    d.out_pitch = out_pitch[i];
    d.offs = (const uint32_t *)(base + b->table_offs[i]);
    d.sbase = (const int32_t *)(base + b->sbase_offs[i]);
  }
  hipStream_t st = (hipStream_t)stream;
  e = hipMemcpyAsync(base + up256(sizeof(unsigned long long)), b->descs.data(), sizeof(BeamDesc) * n,
                     hipMemcpyHostToDevice, st);
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    e = hipMemcpyAsync(base + b->table_offs[i], b->tables[i].offs.data(), b->tables[i].offs.size() * 2,
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(base + b->sbase_offs[i], b->tables[i].sbase.data(), b->tables[i].sbase.size() * 4,
                         hipMemcpyHostToDevice, st);
  }
  if (e != hipSuccess) return fail(DD_ERR_HIP, std::string("batch upload: ") + hipGetErrorString(e));

  BatchLaunch L = {};
  int le = batch_kernels(b->tile.ns, b->tile.dm_per_wave, b->tile.waves, b->tile.chan_block, b->tile.segs, b->dtype,
                         b->lds_bytes, &L);
  if (le) return fail(DD_ERR_HIP, std::string("batch kernel setup: ") + hipGetErrorString((hipError_t)le));
  if (!L.reset_fn || !L.main_fn) return fail(DD_ERR_HIP, "batch kernel setup: missing kernel entry");
  release_graph(b);
  unsigned long long *counter = (unsigned long long *)base;
  const BeamDesc *descs = (const BeamDesc *)(base + up256(sizeof(unsigned long long)));
  int nb = n;
  long long items = b->n_items;
  void *reset_args[] = {&counter};
  void *main_args[] = {&descs, &nb, &items, &counter};
  hipGraphNode_t n_reset = nullptr, n_main = nullptr;
  hipKernelNodeParams kp;
  e = hipGraphCreate(&b->graph, 0);
  if (e == hipSuccess) {
    memset(&kp, 0, sizeof(kp));
    kp.func = (void *)L.reset_fn;
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(1);
    kp.sharedMemBytes = 0;
    kp.kernelParams = reset_args;
    e = hipGraphAddKernelNode(&n_reset, b->graph, nullptr, 0, &kp);
  }
  if (e == hipSuccess) {
    memset(&kp, 0, sizeof(kp));
    kp.func = (void *)L.main_fn;
    kp.gridDim = dim3(L.grid);
    kp.blockDim = dim3(L.block);
    kp.sharedMemBytes = L.lds_bytes;
    kp.kernelParams = main_args;
    e = hipGraphAddKernelNode(&n_main, b->graph, &n_reset, 1, &kp);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    release_graph(b);
    return fail(DD_ERR_HIP, std::string("graph build: ") + hipGetErrorString(e));
  }
  b->bound = true;
  b->device = dev;
  return DD_OK;
}

dd_status dd_execute_batched(dd_batch *b, void *stream) {
  if (!b) return fail(DD_ERR_ARG, "null batch");
  if (!b->bound || !b->exec) return fail(DD_ERR_NOT_BOUND, "batch is not bound");
  int dev = -1;
  if (hipGetDevice(&dev) == hipSuccess && dev != b->device) return fail(DD_ERR_ARG, "batch is bound on another device");
  hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(DD_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  return DD_OK;
}

dd_status dd_batch_get_tiles(const dd_batch *b, dd_tiles *t) {
  if (!b || !t) return fail(DD_ERR_ARG, "null argument");
  const int *k = kIntShapes[b->shape];
  t->shape = b->shape;
  t->order = 0;
  t->ns = k[0];
  t->per_wave = k[1];
  t->waves = k[2];
  t->row_block = k[3];
  t->segs = k[4];
  return DD_OK;
}

dd_status dd_batch_set_tiles(dd_batch *b, int32_t shape) {
  if (!b) return fail(DD_ERR_ARG, "null batch");
  if (shape < 0 || shape >= kNumIntShapes) return fail(DD_ERR_ARG, "no such staged tile shape");
  const dd_status st = batch_set_shape(b, shape);
  if (st == DD_ERR_RANGE) return fail(st, "a beam's delay spread does not fit this shape");
  return st;
}

dd_status dd_batch_autotune(dd_batch *b, const void *const *d_in, float *const *d_out, const int64_t *out_pitch,
                            void *ws, size_t bytes, void *stream, dd_tune_report *rep) {
  if (!b) return fail(DD_ERR_ARG, "null batch");
  const int orig = b->shape;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_error(he, "hipEventCreate");
  }
  // Bind shape s, replay once to warm up, then time one replay.
  auto time_shape = [&](int s, double *ms) -> dd_status {
    dd_status r = batch_set_shape(b, s);
    if (r != DD_OK) return r;
    r = dd_batch_bind(b, d_in, d_out, out_pitch, ws, bytes, stream);
    if (r != DD_OK) return r;
    hipError_t e = hipGraphLaunch(b->exec, st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) return hip_error(e, "batch tuning launch");
    *ms = t;
    return DD_OK;
  };
  double default_ms = 0.0, best_ms = 0.0;
  int best = orig, tried = 0;
  dd_status status = time_shape(orig, &default_ms);
  if (status == DD_OK) {
    best_ms = default_ms;
    tried = 1;
    // Candidates: shapes with at least 32 DM rows per workgroup (the smaller ones
    // only pay where the batch's own default already had to fall back to them).
    for (int s = 0; s < kNumIntShapes && status == DD_OK; ++s) {
      if (s == orig || kIntShapes[s][1] * kIntShapes[s][2] < 32) continue;
      double ms = 0.0;
      const dd_status ts = time_shape(s, &ms);
      if (ts == DD_ERR_RANGE) continue;
      if (ts != DD_OK) {
        status = ts;
        break;
      }
      ++tried;
      if (ms < best_ms) {
        best_ms = ms;
        best = s;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != DD_OK) {
    const std::string msg = dd_last_error();
    (void)hipStreamSynchronize(st);
    (void)batch_set_shape(b, orig);
    return fail(status, msg);
  }
  if (best_ms > 0.98 * default_ms) {  // within timing noise of the default: keep it
    best = orig;
    best_ms = default_ms;
  }
  status = batch_set_shape(b, best);
  if (status == DD_OK) status = dd_batch_bind(b, d_in, d_out, out_pitch, ws, bytes, stream);
  if (status == DD_OK) {
    const hipError_t se = hipStreamSynchronize(st);
    if (se != hipSuccess) status = hip_error(se, "hipStreamSynchronize");
  }
  if (status != DD_OK) return status;
  if (rep) {
    memset(rep, 0, sizeof(*rep));
    rep->n_tried = tried;
    dd_batch_get_tiles(b, &rep->best);
    rep->best_ms = best_ms;
    rep->default_ms = default_ms;
    rep->timed_out_samples = 0;
  }
  return DD_OK;
}

void dd_batch_destroy(dd_batch *b) {
  if (!b) return;
  release_graph(b);
  delete b;
}

}  // extern "C"
