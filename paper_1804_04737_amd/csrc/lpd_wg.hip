// Single-LP launch of the LDS-resident workgroup solve (lpd_wgsolve.h).
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

size_t wg_lds_limit() {
  int dev = 0, lds = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  return (size_t)lds;
}

hipError_t launch_wg_solve(const SolveArgs& a, hipStream_t stream) {
  const size_t lds = wg_lds_bytes(a.m, a.n);
  auto fn = wg_solve_kernel<kWgThreads>;
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  fn<<<1, kWgThreads, lds, stream>>>(a);
  return hipGetLastError();
}

}  // namespace lpd
