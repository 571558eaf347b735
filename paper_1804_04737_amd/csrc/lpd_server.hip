// Serving runtime: continuous batching of dense LPs on one GPU.
//
// Requests arrive from any host thread (lpd_server_submit).  A worker thread
// owns one HIP stream and repeats epochs:
//   1. admission: waiting requests, in arrival order, become resident while
//      their device footprint fits in the memory budget; their A, b, c are
//      copied to HBM and their solve state starts at "not started";
//   2. one batched launch over every resident LP (lpd_batch.hip): each LP
//      advances by at most `pivots_per_epoch` pivots and keeps its tableau and
//      scalars in HBM between epochs (LPs small enough for LDS finish in one
//      epoch);
//   3. statuses come back; finished LPs copy x, obj, pivots to the caller's
//      host buffers, their memory returns to the budget and a completion with
//      host timestamps is queued for lpd_server_poll.
// A request that arrives while others run is admitted in the next epoch, so
// work from different requests overlaps on the device.  Every LP performs
// exactly the pivots of its own lp_solve_dense call, so its result is
// bit-identical alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "lpd_batch.h"
#include "lpdense.h"

namespace lpd {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id = 0;
  int64_t m = 0, n = 0;
  const double *A = nullptr, *b = nullptr, *c = nullptr;  // caller's host arrays
  double* x_out = nullptr;                                  // caller's host buffer (n)
  double t_arrive = 0, t_admit = 0;
  uint64_t footprint = 0;
  bool has_ws = false;  // footprint includes a grid-walk workspace
  // device side (resident requests)
  int32_t slot = -1;
  unsigned char* dmem = nullptr;  // inputs, x, then the workspace
  double *dA = nullptr, *db = nullptr, *dc = nullptr, *dx = nullptr;
  unsigned char* dws = nullptr;
};

// Device copy of A, b, c and x of an m x n request.
uint64_t input_bytes(int64_t m, int64_t n) { return (uint64_t)round_up(8 * (m * n + m + n + n), 256); }

// Device bytes a resident request holds: inputs, x and (for LPs that do not
// fit in LDS) its grid-walk workspace.
uint64_t footprint_of(int64_t m, int64_t n, bool lds) {
  return input_bytes(m, n) + (lds ? 0 : grid_layout(m, n, 1).total);
}

}  // namespace
}  // namespace lpd

using namespace lpd;

struct lpd_server {
  int device = 0;
  uint64_t budget = 0;
  lpd_server_options opt{};
  BatchKnobs knobs;
  hipStream_t stream = nullptr;
  // Slot tables (device): status, objective, pivots and solve state of each
  // resident LP, with pinned host mirrors.
  int32_t* d_status = nullptr;
  double* d_obj = nullptr;
  int64_t* d_iter = nullptr;
  SolveState* d_state = nullptr;
  int32_t* h_status = nullptr;
  double* h_obj = nullptr;
  int64_t* h_iter = nullptr;
  SolveState* h_state = nullptr;
  int32_t nslots = 0;
  int nblocks = 0;
  size_t lds_limit = 0;
  // Batch descriptor buffer, grown as needed (worker only).
  void* meta = nullptr;
  uint64_t meta_bytes = 0;

  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> pending;
  std::vector<lpd_completion> done;
  bool stop = false;
  int64_t next_id = 1;
  uint64_t used = 0;          // footprint of admitted requests (under mu)
  lpd_server_stats stats{};   // under mu
  // worker-only state
  std::vector<Request> resident;
  std::vector<int32_t> free_slots;
  std::thread worker;
  Clock::time_point t0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  void run();
  void epoch();
  void release(Request& r);
  void complete(Request& r, int32_t status, double obj, int64_t iters);
};

void lpd_server::complete(Request& r, int32_t status, double obj, int64_t iters) {
  lpd_completion cpl{};
  cpl.id = r.id;
  cpl.status = status;
  cpl.obj = obj;
  cpl.iterations = iters;
  cpl.m = r.m;
  cpl.n = r.n;
  cpl.x = r.x_out;
  cpl.t_arrive = r.t_arrive;
  cpl.t_admit = r.t_admit;
  cpl.t_done = now();
  std::lock_guard<std::mutex> g(mu);
  done.push_back(cpl);
  stats.completed += 1;
}

void lpd_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    std::vector<Request> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !pending.empty() || !resident.empty(); });
      if (stop && pending.empty() && resident.empty()) return;
      // Admission in arrival order while the budget and the slot table allow.
      while (!pending.empty() && (int32_t)(resident.size() + admit.size()) < nslots) {
        Request& r = pending.front();
        if (used + r.footprint > budget) break;
        r.t_admit = now();
        used += r.footprint;
        stats.peak_bytes = std::max<uint64_t>(stats.peak_bytes, used);
        admit.push_back(r);
        pending.pop_front();
      }
      stats.resident = (int64_t)(resident.size() + admit.size());
      stats.waiting = (int64_t)pending.size();
    }
    for (Request& r : admit) {
      hipError_t e = hipMallocAsync((void**)&r.dmem, r.footprint, stream);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        release(r);
        complete(r, e == hipErrorOutOfMemory ? LPD_ERR_OUT_OF_MEMORY : LPD_ERR_HIP, 0.0, 0);
        continue;
      }
      r.slot = free_slots.back();
      free_slots.pop_back();
      r.dA = reinterpret_cast<double*>(r.dmem);
      r.db = r.dA + r.m * r.n;
      r.dc = r.db + r.m;
      r.dx = r.dc + r.n;
      r.dws = r.dmem + input_bytes(r.m, r.n);
      (void)hipMemcpyAsync(r.dA, r.A, 8 * (size_t)(r.m * r.n), hipMemcpyHostToDevice, stream);
      (void)hipMemcpyAsync(r.db, r.b, 8 * (size_t)r.m, hipMemcpyHostToDevice, stream);
      (void)hipMemcpyAsync(r.dc, r.c, 8 * (size_t)r.n, hipMemcpyHostToDevice, stream);
      // Fresh slot: status "running", solve not started.
      h_status[r.slot] = -1;
      h_state[r.slot] = SolveState{};
      (void)hipMemcpyAsync(d_status + r.slot, h_status + r.slot, 4, hipMemcpyHostToDevice, stream);
      (void)hipMemcpyAsync(d_state + r.slot, h_state + r.slot, sizeof(SolveState), hipMemcpyHostToDevice, stream);
      resident.push_back(r);
    }
    if (!resident.empty()) epoch();
  }
}

void lpd_server::release(Request& r) {
  if (r.dmem) (void)hipFreeAsync(r.dmem, stream);
  r.dmem = nullptr;
  if (r.slot >= 0) free_slots.push_back(r.slot);
  r.slot = -1;
  std::lock_guard<std::mutex> g(mu);
  used -= r.footprint;
}

void lpd_server::epoch() {
  const int32_t count = (int32_t)resident.size();
  std::vector<int64_t> m((size_t)count), n((size_t)count);
  for (int32_t i = 0; i < count; ++i) {
    m[(size_t)i] = resident[(size_t)i].m;
    n[(size_t)i] = resident[(size_t)i].n;
  }
  BatchPlan P = plan_batch(count, m.data(), n.data(), knobs, nblocks);
  hipError_t e = P.ok ? hipSuccess : hipErrorInvalidValue;
  if (e == hipSuccess) {
    const int maxb = batch_max_blocks(P.lds_bytes);
    if (maxb <= 0) e = hipErrorInvalidValue;
    else if (nblocks > maxb) P = plan_batch(count, m.data(), n.data(), knobs, maxb);
  }
  std::vector<BatchItem> items((size_t)count);
  for (int32_t i = 0; i < count && e == hipSuccess; ++i) {
    Request& r = resident[(size_t)i];
    BatchItem& it = items[(size_t)i];
    it = BatchItem{};
    SolveArgs& a = it.a;
    a.m = r.m;
    a.n = r.n;
    a.A = r.dA;
    a.b = r.db;
    a.c = r.dc;
    a.eps_d = opt.eps_d;
    a.eps_p = opt.eps_p;
    a.max_iter = opt.max_iter > 0 ? opt.max_iter : 50 * (r.m + r.n);
    a.x = r.dx;
    a.obj = d_obj + r.slot;
    a.status = d_status + r.slot;
    a.iterations = d_iter + r.slot;
    a.state = d_state + r.slot;
    a.pivot_budget = opt.pivots_per_epoch;
    it.klass = P.klass[(size_t)i];
    it.tclass = P.tclass[(size_t)i];
    it.ws = r.dws;
    // The planner's LDS test is the one submit used; never launch an LP
    // without the workspace its class walks over.
    if (it.klass != kClassLds && !r.has_ws) e = hipErrorInvalidValue;
  }
  if (e == hipSuccess && P.total > meta_bytes) {
    if (meta) (void)hipFreeAsync(meta, stream);
    meta = nullptr;
    meta_bytes = 0;
    e = hipMallocAsync(&meta, P.total, stream);
    if (e == hipSuccess) meta_bytes = P.total;
  }
  if (e == hipSuccess) e = launch_batch(P, items, meta, stream);
  if (e != hipSuccess) (void)hipGetLastError();
  // Statuses, objectives and pivot counts of every slot in one copy each.
  (void)hipMemcpyAsync(h_status, d_status, 4 * (size_t)nslots, hipMemcpyDeviceToHost, stream);
  (void)hipMemcpyAsync(h_obj, d_obj, 8 * (size_t)nslots, hipMemcpyDeviceToHost, stream);
  (void)hipMemcpyAsync(h_iter, d_iter, 8 * (size_t)nslots, hipMemcpyDeviceToHost, stream);
  const hipError_t es = hipStreamSynchronize(stream);
  if (e == hipSuccess) e = es;
  {
    std::lock_guard<std::mutex> g(mu);
    stats.epochs += 1;
  }
  std::vector<Request> still, fin;
  for (Request& r : resident) {
    const int32_t st = e == hipSuccess ? h_status[r.slot] : (int32_t)LPD_ERR_HIP;
    if (st == -1) {
      still.push_back(r);
    } else {
      if (st >= 0) (void)hipMemcpyAsync(r.x_out, r.dx, 8 * (size_t)r.n, hipMemcpyDeviceToHost, stream);
      fin.push_back(r);
    }
  }
  if (!fin.empty()) (void)hipStreamSynchronize(stream);
  for (Request& r : fin) {
    const int32_t st = e == hipSuccess ? h_status[r.slot] : (int32_t)LPD_ERR_HIP;
    const double obj = h_obj[r.slot];
    const int64_t iters = h_iter[r.slot];
    release(r);
    complete(r, st, obj, iters);
  }
  resident.swap(still);
}

extern "C" {

lpd_server* lpd_server_create(int device, uint64_t budget_bytes, const lpd_server_options* opt) {
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return nullptr;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess || std::strncmp(p.gcnArchName, "gfx950", 6) != 0)
    return nullptr;
  if (hipSetDevice(device) != hipSuccess) return nullptr;
  if (opt && (std::isnan(opt->eps_d) || std::isnan(opt->eps_p))) return nullptr;
  lpd_server* s = new lpd_server();
  s->device = device;
  s->budget = budget_bytes;
  if (opt) s->opt = *opt;
  if (!(s->opt.eps_d > 0)) s->opt.eps_d = LPD_DEFAULT_EPS;
  if (!(s->opt.eps_p > 0)) s->opt.eps_p = LPD_DEFAULT_EPS;
  if (s->opt.pivots_per_epoch <= 0) s->opt.pivots_per_epoch = 32;
  if (s->opt.max_resident <= 0) s->opt.max_resident = 4096;
  const BatchKnobs tuned = tuned_batch_knobs();
  s->knobs.team_size = 0;  // teams sized per LP
  s->knobs.team_min_bytes = s->opt.team_min_bytes != 0 ? s->opt.team_min_bytes : tuned.team_min_bytes;
  s->knobs.team_bytes_per_wg = s->opt.team_bytes_per_wg > 0 ? s->opt.team_bytes_per_wg : tuned.team_bytes_per_wg;
  s->knobs.own_workspaces = true;
  s->nslots = s->opt.max_resident;
  s->nblocks = p.multiProcessorCount;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) lds = 0;
  s->lds_limit = (size_t)lds;
  // Keep freed pool memory reserved: admissions and departures allocate and
  // free stream-ordered all the time.
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
    uint64_t keep = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  const size_t ns = (size_t)s->nslots;
  bool ok = hipStreamCreate(&s->stream) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->d_status, 4 * ns) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->d_obj, 8 * ns) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->d_iter, 8 * ns) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->d_state, sizeof(SolveState) * ns) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&s->h_status, 4 * ns, 0) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&s->h_obj, 8 * ns, 0) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&s->h_iter, 8 * ns, 0) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&s->h_state, sizeof(SolveState) * ns, 0) == hipSuccess;
  (void)hipSetDevice(prev);
  if (!ok) {
    (void)hipGetLastError();
    lpd_server_destroy(s);
    return nullptr;
  }
  for (int32_t i = s->nslots - 1; i >= 0; --i) s->free_slots.push_back(i);
  s->t0 = Clock::now();
  s->worker = std::thread([s] { s->run(); });
  return s;
}

int64_t lpd_server_submit(lpd_server* s, int64_t m, int64_t n, const double* A, const double* b, const double* c,
                          double* x_out) {
  if (!s) return LPD_ERR_NOT_FOUND;
  if (m < 1 || n < 1) return LPD_ERR_INVALID_ARG;
  if (!A || !b || !c || !x_out) return LPD_ERR_NULL_POINTER;
  if (m > (1 << 30) || n > (1 << 30) || m + n + 1 > (1 << 30)) return LPD_ERR_SIZE_OVERFLOW;
  // Same LDS test as the batch planner.
  const bool lds = wg_lds_bytes(m, n) + 256 <= s->lds_limit;
  const uint64_t f = footprint_of(m, n, lds);
  if (f > s->budget) return LPD_ERR_TOO_LARGE;
  Request r;
  r.m = m;
  r.n = n;
  r.A = A;
  r.b = b;
  r.c = c;
  r.x_out = x_out;
  r.footprint = f;
  r.has_ws = !lds;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return LPD_ERR_NOT_FOUND;
    r.id = s->next_id++;
    r.t_arrive = s->now();
    s->pending.push_back(r);
    s->stats.submitted += 1;
  }
  s->cv.notify_one();
  return r.id;
}

int lpd_server_poll(lpd_server* s, lpd_completion* out, int max) {
  if (!s || (!out && max > 0) || max < 0) return LPD_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  const int k = (int)std::min<size_t>((size_t)max, s->done.size());
  for (int i = 0; i < k; ++i) out[i] = s->done[(size_t)i];
  s->done.erase(s->done.begin(), s->done.begin() + k);
  return k;
}

int lpd_server_get_stats(lpd_server* s, lpd_server_stats* out) {
  if (!s || !out) return LPD_ERR_NULL_POINTER;
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->stats;
  out->used_bytes = s->used;
  out->budget_bytes = s->budget;
  return LPD_SUCCESS;
}

void lpd_server_destroy(lpd_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->device);
  if (s->stream) {
    if (s->meta) (void)hipFreeAsync(s->meta, s->stream);
    (void)hipStreamSynchronize(s->stream);
  }
  (void)hipFree(s->d_status);
  (void)hipFree(s->d_obj);
  (void)hipFree(s->d_iter);
  (void)hipFree(s->d_state);
  (void)hipHostFree(s->h_status);
  (void)hipHostFree(s->h_obj);
  (void)hipHostFree(s->h_iter);
  (void)hipHostFree(s->h_state);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  (void)hipSetDevice(prev);
  delete s;
}

}  // extern "C"
