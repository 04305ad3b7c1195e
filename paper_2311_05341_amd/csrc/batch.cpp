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
  // One tile shape for all beams: the first compiled shape every beam can stage
  // (two workgroups' worth of LDS is not required: the kernel runs one per CU).
  bool found = false;
  for (int s = 0; s < kNumIntShapes && !found; ++s) {
    b->tables.assign(n, IntTables());
    bool ok = true;
    int lds = 0;
    for (int i = 0; i < n && ok; ++i) {
      dd_status st = build_int_tables(*b->plans[i], kIntShapes[s][0], kIntShapes[s][1], kIntShapes[s][2],
                                      kIntShapes[s][3], kBatchLdsLimit, &b->tables[i]);
      if (st == DD_ERR_NOMEM) { delete b; return st; }
      ok = st == DD_OK;
      if (ok) lds = std::max(lds, b->tables[i].lds_bytes);
    }
    if (ok) {
      b->tile.ns = kIntShapes[s][0];
      b->tile.dm_per_wave = kIntShapes[s][1];
      b->tile.waves = kIntShapes[s][2];
      b->tile.chan_block = kIntShapes[s][3];
      b->lds_bytes = lds;
      found = true;
    }
  }
  if (!found) { delete b; return fail(DD_ERR_RANGE, "a beam's delay spread exceeds the LDS staging capacity"); }
  // Work items: beams ordered by per-item cost (channels x DM rows per tile), largest first.
  b->order.resize(n);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) {
    return b->plans[a]->desc.n_chan > b->plans[c]->desc.n_chan;
  });
  const int dm_tile = b->tile.waves * b->tile.dm_per_wave, t_tile = 64 * b->tile.ns;
  size_t off = up256(sizeof(unsigned long long)) + up256(sizeof(BeamDesc) * (size_t)n);
  b->table_off = off;
  b->table_offs.assign(n, 0);
  b->sbase_offs.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    b->table_offs[i] = off;
    off += up256(b->tables[i].offs.size() * sizeof(uint16_t));
    b->sbase_offs[i] = off;
    off += up256(b->tables[i].sbase.size() * sizeof(int32_t));
  }
  b->ws_bytes = off;
  b->descs.resize(n);
  long long items = 0;
  for (int k = 0; k < n; ++k) {
    const int i = b->order[k];
    const dd_plan &p = *b->plans[i];
    BeamDesc &d = b->descs[k];
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
  int le = batch_kernels(b->tile.ns, b->tile.dm_per_wave, b->tile.waves, b->tile.chan_block, b->dtype,
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
  hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(DD_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  return DD_OK;
}

void dd_batch_destroy(dd_batch *b) {
  if (!b) return;
  release_graph(b);
  delete b;
}

}  // extern "C"
