// dd_execute_noalloc: the forward transform of dd_execute for callers that
// cannot allocate device memory or bind a workspace (code under graph capture,
// tight serving loops, harnesses that forbid allocation).  The plan's device
// tables go into a file-scope device array instead of a bound workspace.
//
// The array is a HIP symbol: in host code its name is a host-side stand-in,
// not a device address.  Its device address is looked up once per device with
// hipGetSymbolAddress (on the first call made with that device current) and
// only that address is ever passed to copies and kernels.  Each device holds
// its own copy of the array until the process ends.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>

#include "dd_internal.h"

namespace dd {
namespace {

constexpr size_t kScratchBytes = DD_NOALLOC_TABLE_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return (int)e;
  if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!ptr) return (int)hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace
}  // namespace dd

using namespace dd;

extern "C" dd_status dd_execute_noalloc(const dd_plan *p, const void *d_in, float *d_out, int64_t out_pitch,
                                        void *stream) {
  if (!p) return fail(DD_ERR_ARG, "null plan");
  if (!d_in || !d_out) return fail(DD_ERR_ARG, "null buffer");
  if (((uintptr_t)d_in & 15u) || ((uintptr_t)d_out & 15u)) return fail(DD_ERR_ALIGN, "buffers must be 16-byte aligned");
  if (out_pitch < p->n_out) return fail(DD_ERR_ARG, "out_pitch < n_out");
  if (out_pitch % 4) return fail(DD_ERR_ALIGN, "out_pitch must be a multiple of 4 elements");
  const size_t need = table_bytes(*p);
  if (need > kScratchBytes)
    return fail(DD_ERR_RANGE, "plan tables need " + std::to_string(need) + " bytes, more than the " +
                                  std::to_string(kScratchBytes) + "-byte static table area of dd_execute_noalloc");
  void *tables = nullptr;
  int e = scratch_address(&tables);
  if (e) return hip_error(e, "hipGetSymbolAddress(scratch)");
  // The tables are rewritten on every call (the area keeps only the last
  // call's contents); the kernels read nothing else from it.
  e = copy_tables(*p, tables, stream);
  if (e) return hip_error(e, "table upload");
  e = p->desc.dtype == DD_F32 ? launch_forward_f32(*p, tables, d_in, d_out, out_pitch, stream)
                              : launch_forward_int(*p, tables, d_in, d_out, out_pitch, stream);
  if (e) return hip_error(e, "forward launch");
  return DD_OK;
}
