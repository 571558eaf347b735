// Host runtime behind the C ABI declared in include/lpdense.h: argument
// validation, schedule choice, stream-ordered workspace and kernel launches.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <atomic>
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "lpd_batch.h"
#include "lpd_kernels.h"
#include "lpdense.h"

// Workspace of lp_solve_dense_noalloc: a file-scope device array, one copy
// per device, held until the process ends.  In host code its name is not a
// device address: the library passes kernels the address that
// hipGetSymbolAddress returns for the current device.  Every call on a device
// shares that device's copy.
constexpr uint64_t kScratchMax = 128ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchMax];

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

// Devices whose default memory pool the library set to keep freed
// workspace (bit d: device d), and the teardown that undoes it at process
// exit: it runs before the HIP runtime's own teardown (registered after the
// runtime started), synchronises the device, restores the pool's release
// threshold and returns what the pool still holds.
std::atomic<uint64_t> g_pool_devices{0};
std::once_flag g_exit_once;

void release_pools_at_exit() {
  const uint64_t mask = g_pool_devices.exchange(0);
  for (int d = 0; d < kMaxDevices; ++d) {
    if (!((mask >> d) & 1u)) continue;
    if (hipSetDevice(d) != hipSuccess) continue;
    (void)hipDeviceSynchronize();
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, d) == hipSuccess) {
      uint64_t threshold = 0;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold);
      (void)hipMemPoolTrimTo(pool, 0);
    }
  }
  (void)hipGetLastError();
}

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
    // to the device driver after every solve.
    keep_freed_pool_memory(dev);
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
    if (opt->schedule < LPD_SCHED_AUTO || opt->schedule > LPD_SCHED_GRID_CONDENSED_PAIRED) return LPD_ERR_INVALID_ARG;
    if (opt->grid_blocks < 0) return LPD_ERR_INVALID_ARG;
    if (opt->watchdog_us > (INT64_MAX / 100)) return LPD_ERR_INVALID_ARG;
    *schedule = opt->schedule;
    *grid_blocks = opt->grid_blocks;
    // 100 ticks of the device's real-time clock per microsecond.
    a->watchdog = opt->watchdog_us < 0 ? -1 : opt->watchdog_us * 100;
  }
  a->eps_d = eps_d;
  a->eps_p = eps_p;
  a->max_iter = max_iter;
  return LPD_SUCCESS;
}

// Batch schedule parameters from the autotune table (written by
// paper_1804_04737_amd/autotune.py next to the library, or the file named by
// LPD_AUTOTUNE_FILE); built-in defaults when there is none.  Read once.
struct Tuning {
  int team_size = 0;                    // 0: size teams per LP
  int64_t team_min_bytes = 2 << 20;
  int64_t team_bytes_per_wg = 2 << 20;
  int wave_slots = 0;                   // 0: no wave-per-instance class
};

const Tuning& tuning() {
  static std::once_flag once;
  static Tuning t;
  std::call_once(once, [] {
    std::string path;
    if (const char* e = std::getenv("LPD_AUTOTUNE_FILE")) {
      path = e;
    } else {
      Dl_info info;
      if (dladdr(reinterpret_cast<void*>(&lp_solve_batch), &info) && info.dli_fname) {
        path = info.dli_fname;
        const size_t slash = path.rfind('/');
        path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/autotune.json";
      }
    }
    std::ifstream f(path);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    auto num = [&](const char* key, int64_t dflt) -> int64_t {
      size_t p = s.find(std::string("\"") + key + "\"");
      if (p == std::string::npos) return dflt;
      p = s.find(':', p);
      if (p == std::string::npos) return dflt;
      char* end = nullptr;
      const long long v = std::strtoll(s.c_str() + p + 1, &end, 10);
      return end == s.c_str() + p + 1 ? dflt : (int64_t)v;
    };
    const int64_t ts = num("team_size", t.team_size);
    if (ts >= 0 && ts <= 1024) t.team_size = (int)ts;
    t.team_min_bytes = num("team_min_bytes", t.team_min_bytes);
    const int64_t bw = num("team_bytes_per_wg", t.team_bytes_per_wg);
    if (bw > 0) t.team_bytes_per_wg = bw;
    const int64_t ws = num("wave_slots", t.wave_slots);
    if (ws >= 0 && ws <= 16) t.wave_slots = (int)ws;
  });
  return t;
}

int hip_err(hipError_t e) {
  if (e == hipSuccess) return LPD_SUCCESS;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return LPD_ERR_OUT_OF_MEMORY;
  return LPD_ERR_HIP;
}

// One batched launch over the LPs `idx` (indices into the caller's arrays).
int run_batch(BatchPlan& P, const std::vector<int32_t>& idx, const int64_t* m, const int64_t* n,
              const double* A_pack, const int64_t* A_off, const double* b_pack, const int64_t* b_off,
              const double* c_pack, const int64_t* c_off, double* x_pack, const int64_t* x_off, double* obj,
              int32_t* status, int64_t* iterations, double eps_d, double eps_p, int64_t max_iter,
              hipStream_t stream) {
  const int32_t count = (int32_t)idx.size();
  std::vector<BatchItem> items((size_t)count);
  for (int32_t j = 0; j < count; ++j) {
    const int32_t i = idx[(size_t)j];
    SolveArgs& a = items[(size_t)j].a;
    a.m = m[i];
    a.n = n[i];
    a.A = A_pack + A_off[i];
    a.b = b_pack + b_off[i];
    a.c = c_pack + c_off[i];
    a.eps_d = eps_d;
    a.eps_p = eps_p;
    a.max_iter = max_iter >= 0 ? max_iter : 50 * (m[i] + n[i]);
    a.x = x_pack + x_off[i];
    a.obj = obj + i;
    a.status = status + i;
    a.iterations = iterations ? iterations + i : nullptr;
    items[(size_t)j].klass = P.klass[(size_t)j];
    items[(size_t)j].tclass = P.tclass[(size_t)j];
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && P.total > total_b) return LPD_ERR_OUT_OF_MEMORY;
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, P.total, stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return hip_err(e);
  }
  e = launch_batch(P, items, ws, stream);
  const hipError_t ef = hipFreeAsync(ws, stream);
  if (e != hipSuccess) return hip_err(e);
  return hip_err(ef);
}


// Device address of `scratch` on each device (null until looked up).
std::once_flag g_scratch_once[kMaxDevices];
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (null if the lookup failed).
void* scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::call_once(g_scratch_once[dev], [dev] {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[dev] = ptr;
    else (void)hipGetLastError();
  });
  return g_scratch_ptr[dev];
}

// Index arrays of a start from a given basic tableau, laid out as
// [basis (m) | pos (ncols) | lab (n + 1) | colof (ncols)] (lab and colof for
// the condensed tableau only, n = ncols - m), built on the host and copied
// to the device in front of the solve.  The host copy is released by a host
// function enqueued after the copy, so the call stays asynchronous.
struct StartIndex {
  std::vector<int32_t> v;
  int64_t off_pos = 0, off_lab = 0, off_colof = 0;
};

void release_start_index(void* p) { delete static_cast<StartIndex*>(p); }

StartIndex* start_index(int64_t m, int64_t ncols, const int64_t* basis0, bool condensed) {
  const int64_t n = ncols - m;
  auto* s = new StartIndex;
  s->off_pos = m;
  s->off_lab = m + ncols;
  s->off_colof = s->off_lab + (condensed ? n + 1 : 0);
  s->v.assign((size_t)(s->off_colof + (condensed ? ncols : 0)), -1);
  for (int64_t i = 0; i < m; ++i) {
    s->v[(size_t)i] = (int32_t)basis0[i];
    s->v[(size_t)(s->off_pos + basis0[i])] = (int32_t)i;
  }
  if (condensed) {
    int64_t c = 0;
    for (int64_t j = 0; j < ncols; ++j)
      if (s->v[(size_t)(s->off_pos + j)] < 0) {
        s->v[(size_t)(s->off_lab + c)] = (int32_t)j;
        s->v[(size_t)(s->off_colof + j)] = (int32_t)c;
        ++c;
      }
  }
  return s;
}

// Copies a start's index arrays to `dev` (stream-ordered) and points the
// solve's arguments at them; takes ownership of `si`.
hipError_t upload_start_index(StartIndex* si, int32_t* dev, SolveArgs& a, bool condensed, hipStream_t stream) {
  hipError_t e = hipMemcpyAsync(dev, si->v.data(), si->v.size() * 4, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipLaunchHostFunc(stream, release_start_index, si);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(stream);
    delete si;
    return e;
  }
  a.basis0 = dev;
  a.pos0 = dev + si->off_pos;
  a.lab0 = condensed ? dev + si->off_lab : nullptr;
  a.colof0 = condensed ? dev + si->off_colof : nullptr;
  return hipSuccess;
}

// Grid size when the caller names none: one workgroup per 160 KiB of stored
// tableau, in multiples of 8 (one per XCD each), at least 64 and at most one
// per compute unit.  Below about 40 MiB a sweep is short, and the per-pivot
// barrier costs more with each added workgroup than the added bandwidth
// saves (measured from 4 to 70 MiB; a count off a multiple of 8 was slower).
int default_grid_blocks(int64_t m, int64_t n, bool condensed, int ncu) {
  const double bytes = 8.0 * (double)(m + 1) * (double)((condensed ? n : n + m) + 1);
  const double want = 8.0 * std::floor(bytes / (160.0 * 1024.0) / 8.0);
  return (int)std::max(std::min(want, (double)ncu), (double)std::min(64, ncu));
}

// Runs the solve described by `a` (inputs, options and outputs set) on
// `schedule`.  The workspace is allocated stream-ordered on `stream`, or
// (noalloc) taken from `scratch` (kScratchMax bytes, no allocation at all:
// sizes beyond it are rejected).  `basis0` (host, m entries) starts from the
// tableau a.T0 instead of Table 1.
int run_solve(SolveArgs& a, int schedule, int grid_blocks, bool noalloc, const int64_t* basis0,
              hipStream_t stream) {
  DeviceInfo dev;
  int rc = device_info(&dev);
  if (rc != LPD_SUCCESS) return rc;
  const int64_t ncols = a.m + a.n;
  const bool fits_lds = wg_lds_bytes(a.m, a.n) <= wg_lds_limit();
  if (schedule == LPD_SCHED_WORKGROUP && !fits_lds) return LPD_ERR_TOO_LARGE;
  if (schedule == LPD_SCHED_WORKGROUP || (schedule == LPD_SCHED_AUTO && fits_lds)) {
    if (!basis0) return hip_err(launch_wg_solve(a, stream));
    StartIndex* si = start_index(a.m, ncols, basis0, false);
    void* meta = nullptr;
    hipError_t e = hipMallocAsync(&meta, si->v.size() * 4, stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      delete si;
      return hip_err(e);
    }
    e = upload_start_index(si, static_cast<int32_t*>(meta), a, false, stream);
    if (e == hipSuccess) e = launch_wg_solve(a, stream);
    const hipError_t ef = hipFreeAsync(meta, stream);
    return hip_err(e != hipSuccess ? e : ef);
  }

  // A tableau with no nonbasic column has nothing to store condensed: the
  // full-tableau schedules give the same results.
  bool condensed = schedule == LPD_SCHED_GRID_CONDENSED || schedule == LPD_SCHED_GRID_CONDENSED_PAIRED;
  const bool paired = schedule == LPD_SCHED_GRID_PAIRED || schedule == LPD_SCHED_GRID_CONDENSED_PAIRED;
  if (a.n == 0) condensed = false;
  const int maxb = grid_max_blocks(a.m, a.n, 0, condensed, paired);
  if (maxb <= 0) return LPD_ERR_TOO_LARGE;
  int nb = grid_blocks > 0 ? grid_blocks : default_grid_blocks(a.m, a.n, condensed, dev.ncu);
  if (nb > maxb) nb = maxb;
  const GridLayout L = grid_layout(a.m, a.n, nb, condensed, paired);
  if (noalloc) {
    if (basis0) return LPD_ERR_INVALID_ARG;
    if (L.total > kScratchMax) return LPD_ERR_TOO_LARGE;
    void* ws = scratch_ptr();
    if (!ws) return LPD_ERR_HIP;
    return hip_err(launch_grid_solve(a, ws, nb, 0, stream, condensed, paired));
  }
  StartIndex* si = basis0 ? start_index(a.m, ncols, basis0, condensed) : nullptr;
  const uint64_t meta_bytes = si ? (uint64_t)si->v.size() * 4 : 0;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && L.total + meta_bytes > total_b) {
    delete si;
    return LPD_ERR_OUT_OF_MEMORY;
  }
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, L.total + meta_bytes, stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete si;
    return hip_err(e);
  }
  if (si)
    e = upload_start_index(si, reinterpret_cast<int32_t*>(static_cast<unsigned char*>(ws) + L.total), a, condensed,
                           stream);
  if (e == hipSuccess) e = launch_grid_solve(a, ws, nb, 0, stream, condensed, paired);
  const hipError_t ef = hipFreeAsync(ws, stream);
  if (e != hipSuccess) return hip_err(e);
  return hip_err(ef);
}

// Outputs of a solve into its kernel arguments (validated by the caller).
int bind_outputs(const lpd_outputs* out, SolveArgs* a) {
  a->x = out->x;
  a->obj = out->obj;
  a->status = out->status;
  a->y = out->y;
  a->iterations = out->iterations;
  a->trace = out->trace_cap > 0 ? out->trace : nullptr;
  a->trace_cap = out->trace_cap;
  a->basis_out = out->basis;
  a->tableau_out = out->tableau;
  if (out->phase_cap < 0 || (out->phase_cap > 0 && !out->phase_ticks)) return LPD_ERR_INVALID_ARG;
  a->phase_ticks = out->phase_cap > 0 ? out->phase_ticks : nullptr;
  a->phase_cap = out->phase_cap;
  return LPD_SUCCESS;
}

// lp_solve_dense_ex (noalloc: lp_solve_dense_noalloc).
int solve_dense(const lpd_problem* prob, const lpd_options* opt, const lpd_outputs* out, hipStream_t stream,
                bool noalloc) {
  int rc = validate(prob, out);
  if (rc != LPD_SUCCESS) return rc;
  SolveArgs a{};
  a.m = prob->m;
  a.n = prob->n;
  a.A = prob->A;
  a.b = prob->b;
  a.c = prob->c;
  int schedule = 0, grid_blocks = 0;
  rc = resolve_options(prob, opt, &a, &schedule, &grid_blocks);  // no HIP call before this
  if (rc != LPD_SUCCESS) return rc;
  rc = bind_outputs(out, &a);
  if (rc != LPD_SUCCESS) return rc;
  return run_solve(a, schedule, grid_blocks, noalloc, nullptr, stream);
}

}  // namespace

void keep_freed_pool_memory(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) != hipSuccess) return;
  uint64_t threshold = UINT64_MAX;
  if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &threshold) != hipSuccess) return;
  g_pool_devices.fetch_or(uint64_t(1) << device);
  std::call_once(g_exit_once, [] { std::atexit(release_pools_at_exit); });
}

BatchKnobs tuned_batch_knobs() {
  BatchKnobs k;
  k.team_size = tuning().team_size;
  k.team_min_bytes = tuning().team_min_bytes;
  k.team_bytes_per_wg = tuning().team_bytes_per_wg;
  k.wave_slots = tuning().wave_slots;
  return k;
}

}  // namespace lpd

using namespace lpd;

extern "C" {

int lp_solve_dense_ex(const lpd_problem* prob, const lpd_options* opt, const lpd_outputs* out,
                      hipStream_t stream) {
  return solve_dense(prob, opt, out, stream, false);
}

int lp_solve_dense_noalloc(const lpd_problem* prob, const lpd_options* opt, const lpd_outputs* out,
                           hipStream_t stream) {
  return solve_dense(prob, opt, out, stream, true);
}

int lp_solve_tableau(int64_t m, int64_t ncols, const double* T0, const int64_t* basis0, const lpd_options* opt,
                     const lpd_outputs* out, hipStream_t stream) {
  if (!out) return LPD_ERR_NULL_POINTER;
  if (m < 1 || ncols < m) return LPD_ERR_INVALID_ARG;
  if (m > kMaxDim || ncols + 1 > kMaxDim) return LPD_ERR_SIZE_OVERFLOW;
  if ((double)(m + 1) * (double)(ncols + 1) * 8.0 > 9.0e18) return LPD_ERR_SIZE_OVERFLOW;
  if (!T0 || !basis0 || !out->x || !out->obj || !out->status) return LPD_ERR_NULL_POINTER;
  if (out->y) return LPD_ERR_INVALID_ARG;
  if (out->trace_cap < 0) return LPD_ERR_INVALID_ARG;
  if (out->trace_cap > 0 && !out->trace) return LPD_ERR_NULL_POINTER;
  std::vector<char> seen((size_t)ncols, 0);
  for (int64_t i = 0; i < m; ++i) {
    if (basis0[i] < 0 || basis0[i] >= ncols || seen[(size_t)basis0[i]]) return LPD_ERR_INVALID_ARG;
    seen[(size_t)basis0[i]] = 1;
  }
  const lpd_problem shape{m, ncols - m, nullptr, nullptr, nullptr};
  SolveArgs a{};
  a.m = m;
  a.n = ncols - m;
  a.T0 = T0;
  a.x_count = ncols;
  int schedule = 0, grid_blocks = 0;
  int rc = resolve_options(&shape, opt, &a, &schedule, &grid_blocks);  // default cap 50 * ncols
  if (rc != LPD_SUCCESS) return rc;
  rc = bind_outputs(out, &a);
  if (rc != LPD_SUCCESS) return rc;
  return run_solve(a, schedule, grid_blocks, false, basis0, stream);
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

int lp_solve_batch(int32_t count, const int64_t* m, const int64_t* n, const double* A_pack, const int64_t* A_off,
                   const double* b_pack, const int64_t* b_off, const double* c_pack, const int64_t* c_off,
                   double* x_pack, const int64_t* x_off, double* obj, int32_t* status,
                   const lpd_batch_options* opt, hipStream_t stream) {
  if (count < 1) return LPD_ERR_INVALID_ARG;
  if (!m || !n || !A_pack || !A_off || !b_pack || !b_off || !c_pack || !c_off || !x_pack || !x_off || !obj ||
      !status)
    return LPD_ERR_NULL_POINTER;
  for (int32_t i = 0; i < count; ++i) {
    if (m[i] < 1 || n[i] < 1) return LPD_ERR_INVALID_ARG;
    if (m[i] > kMaxDim || n[i] > kMaxDim || m[i] + n[i] + 1 > kMaxDim) return LPD_ERR_SIZE_OVERFLOW;
    if (A_off[i] < 0 || b_off[i] < 0 || c_off[i] < 0 || x_off[i] < 0) return LPD_ERR_INVALID_ARG;
  }
  DeviceInfo dev;
  int rc = device_info(&dev);
  if (rc != LPD_SUCCESS) return rc;

  double eps_d = LPD_DEFAULT_EPS, eps_p = LPD_DEFAULT_EPS;
  int64_t max_iter = -1, team_min = 0, per_wg = 0;
  int team_size = 0, nblocks = dev.ncu, wave_slots = 0;
  bool condensed = true;
  int64_t* iterations = nullptr;
  if (opt) {
    if (std::isnan(opt->eps_d) || std::isnan(opt->eps_p) || std::isinf(opt->eps_d) || std::isinf(opt->eps_p))
      return LPD_ERR_INVALID_ARG;
    if (opt->eps_d > 0) eps_d = opt->eps_d;
    if (opt->eps_p > 0) eps_p = opt->eps_p;
    max_iter = opt->max_iter;
    if (opt->team_size < 0 || opt->grid_blocks < 0) return LPD_ERR_INVALID_ARG;
    if (opt->team_bytes_per_wg < 0) return LPD_ERR_INVALID_ARG;
    team_size = opt->team_size;
    team_min = opt->team_min_bytes;
    per_wg = opt->team_bytes_per_wg;
    if (opt->grid_blocks > 0) nblocks = opt->grid_blocks;
    iterations = opt->iterations;
    if (opt->wave_slots > 16) return LPD_ERR_INVALID_ARG;
    wave_slots = opt->wave_slots;
    condensed = opt->full_tableau == 0;
  }
  // Unset knobs (0) come from the autotune table.  A team size > 0 fixes the
  // size; else a given team_bytes_per_wg asks for per-LP sizing; else the
  // table decides both.
  BatchKnobs knobs;
  if (team_size > 0) {
    knobs.team_size = team_size;
  } else if (per_wg > 0) {
    knobs.team_size = 0;
    knobs.team_bytes_per_wg = per_wg;
  } else {
    knobs.team_size = tuning().team_size;
    knobs.team_bytes_per_wg = tuning().team_bytes_per_wg;
  }
  knobs.team_min_bytes = team_min != 0 ? team_min : tuning().team_min_bytes;
  knobs.wave_slots = wave_slots > 0 ? wave_slots : (wave_slots < 0 ? 0 : tuning().wave_slots);
  knobs.condensed = condensed;

  // LPs the batch kernel cannot place (pivot row longer than the LDS holds)
  // are solved after the batch, one at a time on the grid schedule with two
  // pivots per sweep and column panels (a batch is not resumed, so the
  // paired schedule applies), on the same stream: the same results as in the
  // batch.
  const size_t lds_total = (size_t)batch_lds_total();
  std::vector<int32_t> in_batch, alone;
  for (int32_t i = 0; i < count; ++i)
    (batch_can_place(m[i], n[i], condensed, lds_total) ? in_batch : alone).push_back(i);
  const int32_t nbat = (int32_t)in_batch.size();
  std::vector<int64_t> mb((size_t)nbat), nbv((size_t)nbat);
  for (int32_t j = 0; j < nbat; ++j) {
    mb[(size_t)j] = m[in_batch[(size_t)j]];
    nbv[(size_t)j] = n[in_batch[(size_t)j]];
  }
  if (nbat > 0) {
    BatchPlan P = plan_batch(nbat, mb.data(), nbv.data(), knobs, nblocks);
    if (!P.ok) return LPD_ERR_TOO_LARGE;
    const int maxb = batch_max_blocks(P.lds_bytes, P.condensed);
    if (maxb <= 0) return LPD_ERR_TOO_LARGE;
    if (nblocks > maxb) P = plan_batch(nbat, mb.data(), nbv.data(), knobs, maxb);
    rc = run_batch(P, in_batch, m, n, A_pack, A_off, b_pack, b_off, c_pack, c_off, x_pack, x_off, obj, status,
                   iterations, eps_d, eps_p, max_iter, stream);
    if (rc != LPD_SUCCESS) return rc;
  }
  for (int32_t i : alone) {
    lpd_problem pr{m[i], n[i], A_pack + A_off[i], b_pack + b_off[i], c_pack + c_off[i]};
    lpd_options o{};
    o.eps_d = eps_d;
    o.eps_p = eps_p;
    o.max_iter = max_iter;
    o.schedule = condensed ? LPD_SCHED_GRID_CONDENSED_PAIRED : LPD_SCHED_GRID_PAIRED;
    o.grid_blocks = opt ? opt->grid_blocks : 0;
    lpd_outputs out{};
    out.x = x_pack + x_off[i];
    out.obj = obj + i;
    out.status = status + i;
    out.iterations = iterations ? iterations + i : nullptr;
    rc = lp_solve_dense_ex(&pr, &o, &out, stream);
    if (rc != LPD_SUCCESS) return rc;
  }
  return LPD_SUCCESS;
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
    case LPD_INFEASIBLE: return "INFEASIBLE";
    default: return "unknown";
  }
}

int lpd_version(void) { return 100; }

}  // extern "C"
