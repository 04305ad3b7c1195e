// Batched forward: many beams, each with its own plan, run by persistent
// kernel launches recorded once as a HIP graph and replayed by
// dd_execute_batched.  Each beam has a tile shape of its own, staged or
// direct-read; beams of one shape form a group, and each group is one
// persistent launch (counter reset, then the kernel claiming that group's work
// items), the groups independent nodes of the graph.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "dd_internal.h"

using namespace dd;

namespace {

// Beams sharing one tile shape and as many workgroups per CU as their LDS
// allows: one persistent launch.  (The launch's LDS is the largest of its
// beams', so beams of one staged shape whose LDS needs allow different numbers
// of resident workgroups are kept apart.)
struct BatchGroup {
  int shape = 0;                // plan shape index (staged below kNumIntShapes, direct-read above)
  int per_cu = 0;               // workgroups per CU its beams' LDS allows (0: direct-read, no LDS)
  int lds_bytes = 0;            // largest of its beams' LDS needs
  std::vector<int> beams;       // original beam indices, in decreasing per-item cost
  size_t desc_first = 0;        // index of its first descriptor in the workspace's descriptor array
  long long n_items = 0;
};

}  // namespace

struct dd_batch {
  std::vector<const dd_plan *> plans;
  int dtype = 0;
  std::vector<int> shape;         // per beam (original index): its shape
  std::vector<IntTables> tables;  // per beam (original index), for its shape (empty for direct-read)
  std::vector<int> order;         // beams in decreasing per-item cost
  std::vector<BatchGroup> groups;
  std::vector<BeamDesc> descs;    // group after group, each group's beams in cost order
  size_t ws_bytes = 0;
  std::vector<size_t> table_offs, sbase_offs;  // per beam (original index)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool bound = false;
  int device = -1;
};

static const int kBatchLdsLimit = 160 * 1024 - 64;  // leaves room for the claimed-item slot
static const int kMaxGroups = 64;

static size_t up256(size_t v) { return (v + 255) / 256 * 256; }

static bool direct_shape(int s) { return s >= kNumIntShapes; }
static int num_batch_shapes() { return kNumIntShapes + kNumDirectShapes; }

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
  const int64_t n_dblk = (nd + dblk - 1) / dblk, ew = int_entry_words(k[1], k[4]), ncp = (nc + k[3] - 1) / k[3] * k[3];
  *offs = up256((size_t)(n_dblk * k[2] * ncp * ew) * sizeof(uint32_t));
  *sbase = up256((size_t)(n_dblk * nc) * sizeof(int32_t));
}

// Workspace layout: one 256-byte counter slot per group (at most one per
// compiled shape and LDS occupancy class), the beam descriptors, then per beam
// room for its tables under the largest compiled staged shape or its plain
// int32 shift table (what a direct-read shape reads), so that no assignment of
// shapes moves anything.
static size_t counters_bytes() { return (size_t)kMaxGroups * 256; }
static size_t descs_offset() { return counters_bytes(); }

// Give beam i shape shapes[i], for every beam: tables, groups, work items.
// DD_ERR_RANGE (batch unchanged) if a beam cannot be staged with its shape.
static dd_status batch_assign(dd_batch *b, const std::vector<int> &shapes) {
  const int n = (int)b->plans.size();
  std::vector<IntTables> tabs(n);
  for (int i = 0; i < n; ++i) {
    const dd_plan &p = *b->plans[i];
    if (direct_shape(shapes[i])) {  // reads the plan's shift table; its descriptors stay inside the row pitch
      const int bits = p.desc.dtype == DD_U4 ? 4 : p.desc.dtype == DD_U16 ? 16 : 8;
      if ((int64_t)p.max_shift * bits / 8 >= p.in_pitch_bytes) return fail(DD_ERR_RANGE, "delay exceeds the row pitch");
      continue;
    }
    const int *k = kIntShapes[shapes[i]];
    const dd_status st = build_int_tables(p, k[0], k[1], k[2], k[3], k[4], kBatchLdsLimit, &tabs[i]);
    if (st != DD_OK) return st;
  }
  std::vector<BatchGroup> groups;
  for (int q = 0; q < n; ++q) {  // groups in order of their costliest beam
    const int i = b->order[q];
    // the staged kernel keeps 64 bytes of LDS of its own
    const int per_cu = direct_shape(shapes[i]) ? 0 : (kBatchLdsLimit + 64) / (tabs[i].lds_bytes + 64);
    auto g = std::find_if(groups.begin(), groups.end(),
                          [&](const BatchGroup &x) { return x.shape == shapes[i] && x.per_cu == per_cu; });
    if (g == groups.end()) {
      groups.emplace_back();
      g = groups.end() - 1;
      g->shape = shapes[i];
      g->per_cu = per_cu;
    }
    g->beams.push_back(i);
    g->lds_bytes = std::max(g->lds_bytes, tabs[i].lds_bytes);
  }
  if ((int)groups.size() > kMaxGroups) return fail(DD_ERR_RANGE, "too many distinct beam shapes in one batch");
  std::vector<BeamDesc> descs(n);
  size_t q = 0;
  for (BatchGroup &g : groups) {
    const int *k = int_shape(g.shape);
    const int dm_tile = k[1] * k[2], t_tile = direct_shape(g.shape) ? direct_tile_samples(b->dtype) : 64 * k[0];
    g.desc_first = q;
    long long items = 0;
    for (int i : g.beams) {
      const dd_plan &p = *b->plans[i];
      BeamDesc &d = descs[q++];
      memset(&d, 0, sizeof(d));
      d.n_chan = p.desc.n_chan;
      d.n_dm = p.desc.n_dm;
      d.n_samp = p.desc.n_samp;
      d.n_out = p.n_out;
      d.pitch = p.in_pitch_bytes;
      d.row_bytes = tabs[i].row_bytes;
      d.chan_block = tabs[i].chan_block;
      d.tiles_t = (int)((p.n_out + t_tile - 1) / t_tile);
      d.tiles_d = (p.desc.n_dm + dm_tile - 1) / dm_tile;
      d.item_begin = items;
      items += (long long)d.tiles_t * d.tiles_d;
    }
    g.n_items = items;
  }
  b->tables = std::move(tabs);
  b->groups = std::move(groups);
  b->descs = std::move(descs);
  b->shape = shapes;
  b->bound = false;
  return DD_OK;
}

// The shape a beam runs by default: its plan's own forward shape (its default,
// or what the plan was set or tuned to), staged or direct-read, else the first
// staged shape that holds it (phase-load shapes first), else the plan's
// default direct-read shape.
static int default_shape(const dd_plan &p) {
  if (is_direct(p.fwd) && direct_shape(p.fwd.shape)) return p.fwd.shape;
  if (!is_direct(p.fwd) && p.fwd.shape < kNumIntShapes) {
    IntTables t;
    const int *k = kIntShapes[p.fwd.shape];
    if (build_int_tables(p, k[0], k[1], k[2], k[3], k[4], kBatchLdsLimit, &t, false) == DD_OK) return p.fwd.shape;
  }
  for (int pass = 0; pass < 2; ++pass)
    for (int s = 0; s < kNumIntShapes; ++s) {
      if ((kIntShapes[s][4] > 0) != (pass == 0)) continue;
      IntTables t;
      const int *k = kIntShapes[s];
      if (build_int_tables(p, k[0], k[1], k[2], k[3], k[4], kBatchLdsLimit, &t, false) == DD_OK) return s;
    }
  return kNumIntShapes + (p.desc.dtype == DD_U4 ? 1 : 0);
}

static void fill_tiles(int s, dd_tiles *t) {
  const int *k = int_shape(s);
  t->shape = s;
  t->order = 0;
  t->ns = k[0];
  t->per_wave = k[1];
  t->waves = k[2];
  t->row_block = k[3];
  t->segs = k[4];
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
  size_t off = descs_offset() + up256(sizeof(BeamDesc) * (size_t)n);
  b->table_offs.assign(n, 0);
  b->sbase_offs.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    size_t ob = up256(b->plans[i]->shift.size() * sizeof(int32_t)), sbb = 0;
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
  std::vector<int> shapes(n);
  for (int i = 0; i < n; ++i) shapes[i] = default_shape(*b->plans[i]);
  const dd_status st = batch_assign(b, shapes);
  if (st != DD_OK) { delete b; return st; }
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
  for (const BatchGroup &g : b->groups)
    for (size_t k = 0; k < g.beams.size(); ++k) {
      const int i = g.beams[k];
      BeamDesc &d = b->descs[g.desc_first + k];
      d.x = (const uint8_t *)d_in[i];
      d.out = d_out[i];
      d.out_pitch = out_pitch[i];
      d.offs = (const uint32_t *)(base + b->table_offs[i]);
      d.sbase = (const int32_t *)(base + b->sbase_offs[i]);
    }
  hipStream_t st = (hipStream_t)stream;
  e = hipMemcpyAsync(base + descs_offset(), b->descs.data(), sizeof(BeamDesc) * n, hipMemcpyHostToDevice, st);
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    if (direct_shape(b->shape[i])) {
      const std::vector<int32_t> &sh = b->plans[i]->shift;
      e = hipMemcpyAsync(base + b->table_offs[i], sh.data(), sh.size() * 4, hipMemcpyHostToDevice, st);
      continue;
    }
    e = hipMemcpyAsync(base + b->table_offs[i], b->tables[i].offs.data(), b->tables[i].offs.size() * 4,
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(base + b->sbase_offs[i], b->tables[i].sbase.data(), b->tables[i].sbase.size() * 4,
                         hipMemcpyHostToDevice, st);
  }
  if (e != hipSuccess) return fail(DD_ERR_HIP, std::string("batch upload: ") + hipGetErrorString(e));

  // The graph: per group, a counter reset and then the group's persistent
  // kernel.  The groups do not depend on each other, so the runtime may run
  // them side by side (a group's workgroups then fill the CUs that another
  // group's tail leaves idle).  The node parameters are copied when the nodes
  // are added, so per-group argument storage only has to live until then.
  release_graph(b);
  e = hipGraphCreate(&b->graph, 0);
  for (size_t gi = 0; gi < b->groups.size() && e == hipSuccess; ++gi) {
    const BatchGroup &g = b->groups[gi];
    const int *k = int_shape(g.shape);
    BatchLaunch L = {};
    const int le = direct_shape(g.shape) ? batch_direct_kernels(k[1], k[2], b->dtype, &L)
                                         : batch_kernels(k[0], k[1], k[2], k[3], k[4], b->dtype, g.lds_bytes, &L);
    if (le) {
      release_graph(b);
      return fail(DD_ERR_HIP, std::string("batch kernel setup: ") + hipGetErrorString((hipError_t)le));
    }
    if (!L.reset_fn || !L.main_fn) {
      release_graph(b);
      return fail(DD_ERR_HIP, "batch kernel setup: missing kernel entry");
    }
    unsigned long long *counter = (unsigned long long *)(base + 256 * gi);
    const BeamDesc *descs = (const BeamDesc *)(base + descs_offset()) + g.desc_first;
    int nb = (int)g.beams.size();
    long long items = g.n_items;
    void *reset_args[] = {&counter};
    void *main_args[] = {&descs, &nb, &items, &counter};
    hipGraphNode_t n_reset = nullptr, n_main = nullptr;
    hipKernelNodeParams kp;
    memset(&kp, 0, sizeof(kp));
    kp.func = (void *)L.reset_fn;
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(1);
    kp.sharedMemBytes = 0;
    kp.kernelParams = reset_args;
    e = hipGraphAddKernelNode(&n_reset, b->graph, nullptr, 0, &kp);
    if (e != hipSuccess) break;
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
  memset(t, 0, sizeof(*t));
  if (std::all_of(b->shape.begin(), b->shape.end(), [&](int s) { return s == b->shape[0]; })) {
    fill_tiles(b->shape[0], t);
  } else {
    t->shape = -1;  // the beams run different shapes: see dd_batch_get_beam_tiles
  }
  return DD_OK;
}

dd_status dd_batch_get_beam_tiles(const dd_batch *b, int32_t beam, dd_tiles *t) {
  if (!b || !t) return fail(DD_ERR_ARG, "null argument");
  if (beam < 0 || beam >= (int)b->plans.size()) return fail(DD_ERR_ARG, "no such beam");
  fill_tiles(b->shape[beam], t);
  return DD_OK;
}

dd_status dd_batch_set_tiles(dd_batch *b, int32_t shape) {
  if (!b) return fail(DD_ERR_ARG, "null batch");
  if (shape < 0 || shape >= num_batch_shapes()) return fail(DD_ERR_ARG, "no such tile shape");
  const dd_status st = batch_assign(b, std::vector<int>(b->plans.size(), shape));
  if (st == DD_ERR_RANGE) return fail(st, "a beam's delay spread does not fit this shape");
  return st;
}

dd_status dd_batch_autotune(dd_batch *b, const void *const *d_in, float *const *d_out, const int64_t *out_pitch,
                            void *ws, size_t bytes, void *stream, dd_tune_report *rep) {
  if (!b) return fail(DD_ERR_ARG, "null batch");
  const std::vector<int> orig = b->shape;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_error(he, "hipEventCreate");
  }
  // Bind an assignment, replay once to warm up, then time one replay.
  auto time_assign = [&](const std::vector<int> &shapes, double *ms) -> dd_status {
    dd_status r = batch_assign(b, shapes);
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
  // Candidates: the current assignment, every beam at its default shape, and
  // every staged shape with at least 32 DM rows per workgroup, and every
  // direct-read shape, shared by all beams (smaller staged ones only pay where
  // a beam's default had to fall back to them).
  std::vector<std::vector<int>> cands;
  cands.push_back(orig);
  std::vector<int> defaults(orig.size());
  for (size_t i = 0; i < orig.size(); ++i) defaults[i] = default_shape(*b->plans[i]);
  if (defaults != orig) cands.push_back(defaults);
  for (int s = 0; s < num_batch_shapes(); ++s) {
    if (!direct_shape(s) && kIntShapes[s][1] * kIntShapes[s][2] < 32) continue;
    std::vector<int> all(orig.size(), s);
    if (all != orig && all != defaults) cands.push_back(all);
  }
  double default_ms = 0.0, best_ms = 0.0;
  size_t best = 0;
  int tried = 0;
  dd_status status = DD_OK;
  for (size_t c = 0; c < cands.size() && status == DD_OK; ++c) {
    double ms = 0.0;
    const dd_status ts = time_assign(cands[c], &ms);
    if (ts == DD_ERR_RANGE && c > 0) continue;
    if (ts != DD_OK) {
      status = ts;
      break;
    }
    ++tried;
    if (c == 0) {
      default_ms = best_ms = ms;
    } else if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != DD_OK) {
    const std::string msg = dd_last_error();
    (void)hipStreamSynchronize(st);
    (void)batch_assign(b, orig);
    return fail(status, msg);
  }
  if (best_ms > 0.98 * default_ms) {  // within timing noise of the current choice: keep it
    best = 0;
    best_ms = default_ms;
  }
  status = batch_assign(b, cands[best]);
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
