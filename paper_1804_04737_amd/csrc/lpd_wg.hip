// Single-LP launch of the LDS-resident workgroup solve (lpd_wgsolve.h).
#include <cstdlib>
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

// The same solve by a single wave: wave-level fences and the DPP arg-min
// instead of workgroup barriers.
__global__ void __launch_bounds__(kWave) wave_solve_kernel(SolveArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  lds_solve<WaveGroup>(a, smem);
}

typedef void (*WgKernel)(SolveArgs);

// Threads of the LDS solve, by tableau cells: 512 for tiny tableaux, 1024
// from kWideCells on (measured, us per solve with 256 / 512 / 1024 threads:
// 16 x 16 17.3 / 17.9 / 18.4, 32 x 32 17.4 / 14.5 / 14.4, 64 x 64
// 59.1 / 45.3 / 38.9, 90 x 90 90.8 / 62.1 / 53.8; a single wave is 3-4x
// slower from 32 x 32 on).
// LPD_WG_THREADS (64, 256, 512 or 1024) overrides it, for tuning.
constexpr int64_t kWideCells = 2000;
int wg_threads(int64_t cells) {
  static const int forced = [] {
    const char* e = getenv("LPD_WG_THREADS");
    const int t = e ? atoi(e) : 0;
    return (t == 64 || t == 256 || t == 512 || t == 1024) ? t : 0;
  }();
  if (forced) return forced;
  return cells >= kWideCells ? 1024 : kWgThreads;
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
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  const int limit = (int)wg_lds_limit();
  std::call_once(g_attr_once[dev], [limit, dev] {
    const WgKernel fns[] = {wg_solve_kernel<kWgThreads>, wg_solve_kernel<256>, wg_solve_kernel<1024>,
                            wave_solve_kernel};
    hipError_t r = hipSuccess;
    for (WgKernel f : fns)
      if (r == hipSuccess) r = hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, limit);
    g_attr[dev] = r;
  });
  if (g_attr[dev] != hipSuccess) return g_attr[dev];
  if (lds > (size_t)limit) return hipErrorInvalidValue;
  const int nt = wg_threads((a.m + 1) * (a.m + a.n + 1));
  if (nt == kWave) wave_solve_kernel<<<1, kWave, lds, stream>>>(a);
  else if (nt == 256) wg_solve_kernel<256><<<1, 256, lds, stream>>>(a);
  else if (nt == 1024) wg_solve_kernel<1024><<<1, 1024, lds, stream>>>(a);
  else wg_solve_kernel<kWgThreads><<<1, kWgThreads, lds, stream>>>(a);
  return hipGetLastError();
}

}  // namespace lpd
