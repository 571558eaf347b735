// Single-LP launch of the LDS-resident workgroup solve (lpd_wgsolve.h).
#include <mutex>

#include "lpd_wgsolve.h"

namespace lpd {
namespace {

constexpr int kWgThreads = 512;

template <int NT>
__global__ void __launch_bounds__(NT) wg_solve_kernel(SolveArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  wg_solve<NT>(a, smem);
}

}  // namespace

size_t wg_lds_bytes(int64_t m, int64_t n) { return wg_layout(m, n).total; }

namespace {
// Per device, looked up once: the LDS a workgroup may use, and whether the
// kernel has been allowed all of it (small solves are launch-bound, so the
// attribute is not set again on every call).
constexpr int kMaxDev = 64;
std::once_flag g_lds_once[kMaxDev], g_attr_once[kMaxDev];
int g_lds[kMaxDev];
hipError_t g_attr[kMaxDev];
}  // namespace

size_t wg_lds_limit() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return 0;
  std::call_once(g_lds_once[dev], [dev] {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds = 0;
    g_lds[dev] = lds;
  });
  return (size_t)g_lds[dev];
}

hipError_t launch_wg_solve(const SolveArgs& a, hipStream_t stream) {
  const size_t lds = wg_lds_bytes(a.m, a.n);
  auto fn = wg_solve_kernel<kWgThreads>;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  const int limit = (int)wg_lds_limit();
  std::call_once(g_attr_once[dev], [fn, limit, dev] {
    g_attr[dev] = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, limit);
  });
  if (g_attr[dev] != hipSuccess) return g_attr[dev];
  if (lds > (size_t)limit) return hipErrorInvalidValue;
  fn<<<1, kWgThreads, lds, stream>>>(a);
  return hipGetLastError();
}

}  // namespace lpd
