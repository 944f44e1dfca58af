// lsr_energy_noalloc: the energy functional of caller-given nodal fields for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops).  The energy kernels' per-block partial sums, which
// lsr_energy keeps in a job's workspace, live here in a file-scope device
// array, one copy per device, whose address is taken once per device.
#include <mutex>

#include "lsr_job.h"

using namespace lsr;

namespace {

// Per-block partial sums of the energy kernels (every block writes its own
// slot on every call, so nothing needs clearing): 8 KiB per device.
constexpr size_t kScratchDoubles = ENERGY_BLOCKS;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, taken with that
// device current the first time it is asked for.
lsr_status scratch_ptr(double** out) {
  int dev = 0;
  LSR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LSR_E_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LSR_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return LSR_OK;
}

}  // namespace

extern "C" lsr_status lsr_energy_noalloc(const lsr_grid* grid, int32_t precision,
                                         const void* dev_phi, const double* dev_d, double p,
                                         int32_t R, double* dev_out, void* hip_stream) {
  lsr_status st = grid_ok(grid);
  if (st != LSR_OK) return st;
  if (precision != LSR_FP32 && precision != LSR_FP64)
    return fail(LSR_E_INVALID, "precision must be LSR_FP32 or LSR_FP64");
  if (!dev_phi || !dev_d || !dev_out) return fail(LSR_E_INVALID, "NULL argument");
  if (!(p > 0.0) || !isfinite(p)) return fail(LSR_E_INVALID, "p must be finite and > 0");
  if (R < 1 || R > 64) return fail(LSR_E_INVALID, "R must be in 1..64");
  double* partial = nullptr;
  st = scratch_ptr(&partial);
  if (st != LSR_OK) return st;
  lsr_grid g = *grid;
  if (g.dim == 2) {
    g.n[2] = 1;
    g.lo[2] = 0.0;
  }
  const DevGrid dg = make_devgrid(g);
  hipStream_t s = (hipStream_t)hip_stream;
  if (precision == LSR_FP64)
    LSR_HIP(launch_energy<double>(g.dim, dg, (const double*)dev_phi, dev_d, p, R, partial, dev_out,
                                  s));
  else
    LSR_HIP(launch_energy<float>(g.dim, dg, (const float*)dev_phi, dev_d, p, R, partial, dev_out,
                                 s));
  return LSR_OK;
}
