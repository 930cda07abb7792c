// The residual entry point for callers that cannot allocate device memory: the
// same kernels as msir_residual, with every scratch buffer carved from one
// file-scope device array per GPU instead of the handle's growable workspace.
//
// Host code never passes the array's name to a kernel or a copy: its device
// address on each GPU is taken once with hipGetSymbolAddress (with that device
// current) when the first handle on the device is created, and kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/msir.h"
#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr size_t kNoAllocDoubles = MSIR_NOALLOC_SCRATCH_BYTES / sizeof(double);
// [0, 32): the last-block counter (and padding to 256 bytes); then the buffers
constexpr size_t kCounterDoubles = 32;

static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
static double* g_scratch[kMaxDevices];
static std::once_flag g_once[kMaxDevices];
static int g_status[kMaxDevices];

__global__ void k_zero_counter(unsigned* counter) {
  if (threadIdx.x == 0) *counter = 0u;
}

// Called with `device` current (msir_create).  Records the array's address on this
// device and clears its counter; the result is kept for every later handle.
int noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return MSIR_ERR_HIP;
  std::call_once(g_once[device], [device]() {
    double* p = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      g_status[device] = MSIR_ERR_HIP;
      return;
    }
    k_zero_counter<<<1, 64>>>((unsigned*)p);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      g_status[device] = MSIR_ERR_HIP;
      return;
    }
    g_scratch[device] = p;
    g_status[device] = 0;
  });
  return g_status[device];
}

// r = b - A x in ur, s = ||r||_inf, rhat = fl_u(r / s) on the handle's stream with the
// per-device scratch array.  Returns MSIR_ERR_SIZE when the buffers for order n do not
// fit the array.
int residual_noalloc(Ctx& c, int n, const double* A, int lda, const double* x, const double* b, int ur, int u,
                     double* rhat, double* s_dev) {
  if (c.device < 0 || c.device >= kMaxDevices || !g_scratch[c.device]) return MSIR_ERR_HIP;
  if (c.sp) return MSIR_ERR_SIZE;
  const size_t need = residual_scratch_doubles(n, ur, false);
  if (kCounterDoubles + need > kNoAllocDoubles) return MSIR_ERR_SIZE;
  double* base = g_scratch[c.device];
  const GemvPlan g = gemv_plan(n, 0);
  const size_t part = (size_t)g.ns * n;
  const int rb = (n + 255) / 256;
  ResidWork w;
  w.counter = (unsigned*)base;
  double* q = base + kCounterDoubles;
  w.blockmax = q; q += 2 * (size_t)rb;
  w.rh = q; q += n;
  if (ur == P_DD) { w.rl = q; q += n; }
  w.ph = q; q += part;
  if (ur == P_DD) { w.pl = q; q += part; }
  // the counter must start at zero: a call cut short before its last block ran would
  // have left it set, so it is cleared by a kernel on the stream (no memset node)
  k_zero_counter<<<1, 64, 0, c.stream>>>(w.counter);
  HIP_CHECK(hipGetLastError());
  return residual_with(c, n, A, lda, x, b, ur, u, rhat, s_dev, false, w);
}

}  // namespace msir
