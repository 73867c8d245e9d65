// fld_step_static: one radiation step whose workspace is a device array of
// the library itself, for callers that cannot allocate device memory (code
// under stream capture, tight serving loops, harnesses that forbid
// hipMalloc).  Declared in include/fld.h.
//
// The array below is the workspace of every such call on a device.  In host
// code its name stands for a host-side shadow, not for device memory, so the
// device address is looked up once per device with hipGetSymbolAddress (with
// that device current) and only that address is ever handed to the engine and
// its kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fld.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // FLD_STATIC_SCRATCH_BYTES
static_assert(kScratchBytes == FLD_STATIC_SCRATCH_BYTES, "header and source agree");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// device address of this device's copy of the array (nullptr on failure)
void *scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" {

size_t fld_static_scratch_bytes(void) { return kScratchBytes; }

fld_status fld_step_static(const fld_grid *g, const fld_params *p,
                           void *hip_stream, double *E, const double *kappa,
                           const double *eta, double dt, double a, double adot,
                           fld_stats *stats) {
  if (!g || !p || !E || !kappa || !eta) return FLD_EINVAL;
  const size_t need = fld_workspace_bytes(g, p);
  if (need == 0) return FLD_EINVAL;
  if (need > kScratchBytes) return FLD_ENOMEM;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return FLD_EDEVICE;
  void *ws = scratch_ptr(dev);
  if (!ws) return FLD_EDEVICE;
  // launches one by one: no graph to instantiate, no capture stream to create
  fld_params q = *p;
  q.use_graph = 0;
  fld_handle *h = nullptr;
  fld_status st = fld_create(g, &q, hip_stream, ws, kScratchBytes, &h);
  if (st != FLD_OK) return st;
  st = fld_step(h, E, kappa, eta, dt, a, adot, stats);
  fld_status d = fld_destroy(h);
  return st != FLD_OK ? st : d;
}

}  // extern "C"
