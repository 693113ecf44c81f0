// wave_create_static: a context whose workspace is the library's own device
// memory, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The workspace is `scratch`, a file-scope device array of WAVE_STATIC_BYTES.
// Each GPU the library runs on holds its own copy until the process ends.
// In host code the array's name is only a stand-in for the symbol, so its
// device address is resolved once per device with hipGetSymbolAddress and
// only that address is used afterwards.
#include <mutex>

#include "wave.h"
#include "wave_internal.h"

namespace {

constexpr size_t kScratchBytes = WAVE_STATIC_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// The current device's scratch address (resolved on its first use there).
int scratch_on_current_device(int *device, void **ptr) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return WAVE_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return WAVE_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return WAVE_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *device = dev;
  *ptr = g_scratch_ptr[dev];
  return WAVE_OK;
}

}  // namespace

extern "C" {

int wave_create_static(const wave_params *p, const float *vel_dev, void *hip_stream, wave_t *out) {
  if (!p || !out || !vel_dev) return WAVE_EINVAL;
  *out = nullptr;
  if (p->graph_steps != 0) return WAVE_EINVAL;
  size_t need = 0;
  int rc = wave_workspace_bytes(p, &need);
  if (rc) return rc;
  if (need > kScratchBytes) return WAVE_ENOSPC;
  int dev = -1;
  void *ptr = nullptr;
  rc = scratch_on_current_device(&dev, &ptr);
  if (rc) return rc;
  return wave::create_static_ctx(p, vel_dev, ptr, kScratchBytes, hip_stream, out, dev);
}

}  // extern "C"
