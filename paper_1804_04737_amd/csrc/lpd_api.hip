// Host runtime behind the C ABI declared in include/lpdense.h: argument
// validation, schedule choice, stream-ordered workspace and kernel launches.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>

#include "lpd_kernels.h"
#include "lpdense.h"

namespace lpd {
namespace {

constexpr int kMaxDevices = 64;

// Per-device facts computed once (immutable afterwards).
struct DeviceInfo {
  bool ok = false;
  int ncu = 0;
};

std::once_flag g_once[kMaxDevices];
DeviceInfo g_info[kMaxDevices];

int device_info(DeviceInfo* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LPD_ERR_DEVICE;
  if (dev < 0 || dev >= kMaxDevices) return LPD_ERR_DEVICE;
  std::call_once(g_once[dev], [dev] {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return;
    if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) return;
    if (!p.cooperativeLaunch) return;
    // Keep freed workspace in the stream-ordered pool instead of returning it
    // to the driver after every solve.
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t threshold = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
    }
    g_info[dev].ncu = p.multiProcessorCount;
    g_info[dev].ok = true;
  });
  if (!g_info[dev].ok) return LPD_ERR_DEVICE;
  *out = g_info[dev];
  return LPD_SUCCESS;
}

// Largest m + n the kernels index with 32-bit row / column numbers.
constexpr int64_t kMaxDim = (int64_t(1) << 30);

int validate(const lpd_problem* prob, const lpd_outputs* out) {
  if (!prob || !out) return LPD_ERR_NULL_POINTER;
  if (prob->m < 1 || prob->n < 1) return LPD_ERR_INVALID_ARG;
  if (prob->m > kMaxDim || prob->n > kMaxDim || prob->m + prob->n + 1 > kMaxDim) return LPD_ERR_SIZE_OVERFLOW;
  if (!prob->A || !prob->b || !prob->c) return LPD_ERR_NULL_POINTER;
  if (!out->x || !out->obj || !out->status) return LPD_ERR_NULL_POINTER;
  if (out->trace_cap < 0) return LPD_ERR_INVALID_ARG;
  if (out->trace_cap > 0 && !out->trace) return LPD_ERR_NULL_POINTER;
  // (m+1)*(n+m+1) doubles must be addressable.
  const double cells = (double)(prob->m + 1) * (double)(prob->n + prob->m + 1);
  if (cells * 8.0 > 9.0e18) return LPD_ERR_SIZE_OVERFLOW;
  return LPD_SUCCESS;
}

int resolve_options(const lpd_problem* prob, const lpd_options* opt, SolveArgs* a, int* schedule,
                    int* grid_blocks) {
  double eps_d = LPD_DEFAULT_EPS, eps_p = LPD_DEFAULT_EPS;
  int64_t max_iter = 50 * (prob->m + prob->n);
  *schedule = LPD_SCHED_AUTO;
  *grid_blocks = 0;
  if (opt) {
    if (std::isnan(opt->eps_d) || std::isnan(opt->eps_p) || std::isinf(opt->eps_d) || std::isinf(opt->eps_p))
      return LPD_ERR_INVALID_ARG;
    if (opt->eps_d > 0) eps_d = opt->eps_d;
    if (opt->eps_p > 0) eps_p = opt->eps_p;
    if (opt->max_iter >= 0) max_iter = opt->max_iter;
    if (opt->schedule < LPD_SCHED_AUTO || opt->schedule > LPD_SCHED_GRID) return LPD_ERR_INVALID_ARG;
    if (opt->grid_blocks < 0) return LPD_ERR_INVALID_ARG;
    *schedule = opt->schedule;
    *grid_blocks = opt->grid_blocks;
  }
  a->eps_d = eps_d;
  a->eps_p = eps_p;
  a->max_iter = max_iter;
  return LPD_SUCCESS;
}

int hip_err(hipError_t e) {
  if (e == hipSuccess) return LPD_SUCCESS;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return LPD_ERR_OUT_OF_MEMORY;
  return LPD_ERR_HIP;
}

}  // namespace
}  // namespace lpd

using namespace lpd;

extern "C" {

int lp_solve_dense_ex(const lpd_problem* prob, const lpd_options* opt, const lpd_outputs* out,
                      hipStream_t stream) {
  int rc = validate(prob, out);
  if (rc != LPD_SUCCESS) return rc;
  DeviceInfo dev;
  rc = device_info(&dev);
  if (rc != LPD_SUCCESS) return rc;

  SolveArgs a{};
  a.m = prob->m;
  a.n = prob->n;
  a.A = prob->A;
  a.b = prob->b;
  a.c = prob->c;
  int schedule = 0, grid_blocks = 0;
  rc = resolve_options(prob, opt, &a, &schedule, &grid_blocks);
  if (rc != LPD_SUCCESS) return rc;
  a.x = out->x;
  a.obj = out->obj;
  a.status = out->status;
  a.y = out->y;
  a.iterations = out->iterations;
  a.trace = out->trace_cap > 0 ? out->trace : nullptr;
  a.trace_cap = out->trace_cap;
  a.basis_out = out->basis;
  a.tableau_out = out->tableau;
  if (out->phase_cap < 0 || (out->phase_cap > 0 && !out->phase_ticks)) return LPD_ERR_INVALID_ARG;
  a.phase_ticks = out->phase_cap > 0 ? out->phase_ticks : nullptr;
  a.phase_cap = out->phase_cap;

  const bool fits_lds = wg_lds_bytes(a.m, a.n) <= wg_lds_limit();
  if (schedule == LPD_SCHED_WORKGROUP && !fits_lds) return LPD_ERR_TOO_LARGE;
  if (schedule == LPD_SCHED_WORKGROUP || (schedule == LPD_SCHED_AUTO && fits_lds))
    return hip_err(launch_wg_solve(a, stream));

  const int maxb = grid_max_blocks(a.m, a.n, 0);
  if (maxb <= 0) return LPD_ERR_TOO_LARGE;
  int nb = grid_blocks > 0 ? grid_blocks : dev.ncu;
  if (nb > maxb) nb = maxb;
  const GridLayout L = grid_layout(a.m, a.n, nb);
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && L.total > total_b) return LPD_ERR_OUT_OF_MEMORY;
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, L.total, stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return hip_err(e);
  }
  e = launch_grid_solve(a, ws, nb, 0, stream);
  const hipError_t ef = hipFreeAsync(ws, stream);
  if (e != hipSuccess) return hip_err(e);
  return hip_err(ef);
}

int lp_solve_dense(int64_t m, int64_t n, const double* A, const double* b, const double* c, double* x,
                   double* obj, int32_t* status, hipStream_t stream) {
  lpd_problem p{m, n, A, b, c};
  lpd_outputs o{};
  o.x = x;
  o.obj = obj;
  o.status = status;
  return lp_solve_dense_ex(&p, nullptr, &o, stream);
}

uint64_t lpd_workspace_bytes(int64_t m, int64_t n) {
  if (m < 1 || n < 1 || m > kMaxDim || n > kMaxDim) return 0;
  if (wg_lds_bytes(m, n) <= wg_lds_limit()) return 0;
  DeviceInfo dev;
  const int nb = device_info(&dev) == LPD_SUCCESS ? dev.ncu : 256;
  return grid_layout(m, n, nb).total;
}

const char* lpd_error_string(int code) {
  switch (code) {
    case LPD_SUCCESS: return "success";
    case LPD_ERR_INVALID_ARG: return "invalid argument";
    case LPD_ERR_NULL_POINTER: return "null pointer";
    case LPD_ERR_SIZE_OVERFLOW: return "size overflow";
    case LPD_ERR_OUT_OF_MEMORY: return "out of device memory";
    case LPD_ERR_HIP: return "HIP runtime error";
    case LPD_ERR_DEVICE: return "no usable gfx950 device";
    case LPD_ERR_TOO_LARGE: return "problem too large for this schedule or budget";
    case LPD_ERR_NOT_FOUND: return "not found";
    default: return "unknown";
  }
}

const char* lpd_status_string(int32_t s) {
  switch (s) {
    case LPD_OPTIMAL: return "OPTIMAL";
    case LPD_UNBOUNDED: return "UNBOUNDED";
    case LPD_ITERATION_LIMIT: return "ITERATION_LIMIT";
    case LPD_INFEASIBLE_START: return "INFEASIBLE_START";
    case LPD_NUMERICAL: return "NUMERICAL";
    case LPD_DEVICE_TIMEOUT: return "DEVICE_TIMEOUT";
    default: return "unknown";
  }
}

int lpd_version(void) { return 100; }

}  // extern "C"
