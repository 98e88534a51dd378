// The pressure solve for callers that cannot allocate device memory
// (nfvm_mg_solve_device_noalloc): its reduction partials and scalars live in
// a fixed device array of this file instead of memory the library
// allocates.  Each device that runs the call holds its own copy of the array
// until the process ends; every call on a device shares it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "engine.hpp"

namespace {

// 2 MiB: the scalars plus the partials of about 87,000 workgroups, which
// covers the autotuned launches of grids up to the 1024 x 512 x 256 room.
constexpr size_t SCRATCH_DOUBLES = (size_t)1 << 18;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

// Device address of this device's copy of the array, looked up once per
// device with the device current.  (The host-side name of the array is not a
// device address.)
double* scratch_here() {
  int dev = 0;
  NFVM_CK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw nfvm::Error{NFVM_E_DEVICE, "device id out of range"};
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    NFVM_CK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw nfvm::Error{NFVM_E_DEVICE, "no device address for the solve scratch"};
    g_ptr[dev] = (double*)p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" nfvm_status nfvm_mg_solve_device_noalloc(nfvm_grid_t grid, const double* b_dev,
                                                    double* x_dev, double tol,
                                                    int32_t max_cycles, int32_t forced_cycles,
                                                    nfvm_step_stats* stats) {
  if (!grid || !b_dev || !x_dev) {
    nfvm::set_error("grid, b and x are required");
    return NFVM_E_INVAL;
  }
  try {
    double* s = scratch_here();
    nfvm_status st = NFVM_OK;
    grid->g->mg_solve_scratch(b_dev, x_dev, tol, max_cycles, forced_cycles, stats, &st, s,
                              SCRATCH_DOUBLES);
    if (st == NFVM_E_NOTCONV) nfvm::set_error("pressure solve reached max_cycles");
    if (st == NFVM_E_DIVERGED) nfvm::set_error("non-finite residual");
    return st;
  } catch (const nfvm::Error& e) {
    nfvm::set_error(e.msg);
    (void)hipGetLastError();  // (as every other entry point: no stale last error)
    return e.st;
  } catch (const std::exception& e) {
    nfvm::set_error(e.what());
    return NFVM_E_DEVICE;
  }
}
