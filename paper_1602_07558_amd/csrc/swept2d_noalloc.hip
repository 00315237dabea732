// swept2d_advance_noalloc: the swept advance for callers that cannot
// allocate device memory. Its panels (the pyramids' and bridges' sides that
// pass between the stage kernels) live in one file-scope device array of
// fixed size instead of per-handle allocations.
//
// In host code the array's name stands for a host-side shadow, not for a
// device address: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current), kept in g_ptr, and only
// that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/swept2d.h"
#include "engine.hpp"

namespace swept {
int set_error(int code, const char* fmt, ...);
int noalloc_advance(int nx, int ny, int nvars, int pde, int substeps, int prec, const double* params, int np,
                    int tile, void* dev_state, long long T, long long nsteps, hipStream_t stream, void* scratch,
                    size_t scratch_bytes);
}  // namespace swept

namespace {

constexpr size_t kScratchBytes = SWEPT2D_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Panel storage shared by every call on a device (each device holds its own
// copy until the process ends).
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices];  // device address of `scratch` on each device, or null

// Device address of `scratch` on the current device (looked up on the first
// call there), or null with the error recorded.
void* scratch_address(int* rc) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *rc = swept::set_error(SWEPT2D_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *rc = swept::set_error(SWEPT2D_EUNSUPPORTED, "device %d beyond the %d the static scratch tracks", dev,
                           kMaxDevices);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *rc = swept::set_error(SWEPT2D_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return nullptr;
    }
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" int swept2d_advance_noalloc(int nx, int ny, int nvars, int pde, int substeps, int prec,
                                       const double* params, int np, int tile, void* dev_state, long long T,
                                       long long nsteps, void* hip_stream) {
  int rc = 0;
  void* p = scratch_address(&rc);
  if (!p) return rc;
  hipStream_t s = (hip_stream == SWEPT2D_NULL_STREAM) ? nullptr : static_cast<hipStream_t>(hip_stream);
  return swept::noalloc_advance(nx, ny, nvars, pde, substeps, prec, params, np, tile, dev_state, T, nsteps, s, p,
                                kScratchBytes);
}
