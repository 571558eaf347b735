// Serving runtime: continuous batching of dense LPs on one GPU.
//
// Requests arrive from any host thread (lpd_server_submit).  A worker thread
// drives two HIP streams (both at the default priority) in a pipeline:
//   admission  waiting requests, in arrival order, become resident while their
//              device footprint fits in what the budget has left; their A, b,
//              c go to HBM on the copy stream while the current epoch runs;
//   epoch      one batched launch (lpd_batch.hip) over every resident LP on
//              the compute stream: each LP advances by a bounded number of
//              pivots and keeps its tableau and scalars in HBM between epochs
//              (LPs small enough for LDS finish within one epoch).
//              Workgroups are shared out in proportion to the tableau bytes
//              of the resident LPs, one team per LP, and each LP's pivot
//              budget is sized so that every workgroup streams about the same
//              bytes per epoch: all of them advance together and finish the
//              epoch at about the same time;
//   retire     statuses come back; finished LPs copy x to the caller's host
//              buffer on a third stream while the next epoch already runs,
//              then their memory returns to the budget and a completion with
//              host timestamps is queued for lpd_server_poll.
// Requests admitted during epoch E join epoch E+1 (the compute stream waits
// for their copies), so work from different requests overlaps on the device.
// Every LP performs exactly the pivots of its own lp_solve_dense call, so its
// result is bit-identical alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
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
  bool wide = false;    // pivot row longer than the LDS: own grid launch each epoch
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
uint64_t footprint_of(int64_t m, int64_t n, bool lds, bool condensed) {
  return input_bytes(m, n) + (lds ? 0 : grid_layout(m, n, 1, condensed).total);
}

// Smallest tableau share a workgroup gets under share sizing: below this the
// per-pivot barrier costs more than the workgroup's part of the sweep.
constexpr int64_t kShareMinBytesPerWg = 256 << 10;

}  // namespace
}  // namespace lpd

using namespace lpd;

struct lpd_server {
  int device = 0;
  uint64_t budget = 0;
  lpd_server_options opt{};
  BatchKnobs knobs;
  hipStream_t stream = nullptr;       // compute: epochs, result copies, frees
  hipStream_t copy_stream = nullptr;  // admission: allocations and input copies
  hipStream_t res_stream = nullptr;   // results: x of finished LPs back to the host
  hipEvent_t ev_staged = nullptr;     // end of the last admission round's copies
  hipEvent_t ev_xdone = nullptr;      // end of the retiring LPs' x copies
  hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr;  // around the epoch launch
  // Slot tables (device): status, objective, pivots and solve state of each
  // resident LP, with pinned host mirrors.  init_status / init_state are
  // pinned constants (-1, not started) that fresh slots are copied from.
  int32_t* d_status = nullptr;
  double* d_obj = nullptr;
  int64_t* d_iter = nullptr;
  SolveState* d_state = nullptr;
  int32_t* h_status = nullptr;
  double* h_obj = nullptr;
  int64_t* h_iter = nullptr;
  int32_t* init_status = nullptr;
  SolveState* init_state = nullptr;
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
  std::vector<Request> resident, staged;
  std::vector<Request> retiring;  // finished in the last epoch, x on its way
  std::vector<int32_t> retiring_status;
  std::vector<double> retiring_obj;
  std::vector<int64_t> retiring_iter;
  std::vector<int32_t> free_slots;
  bool in_flight = false;
  hipError_t epoch_err = hipSuccess;
  std::thread worker;
  Clock::time_point t0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  void run();
  void admit();
  void launch_epoch();
  void retire_epoch();
  void finish_retiring();
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

void lpd_server::release(Request& r) {
  if (r.dmem) (void)hipFreeAsync(r.dmem, stream);
  r.dmem = nullptr;
  if (r.slot >= 0) free_slots.push_back(r.slot);
  r.slot = -1;
  std::lock_guard<std::mutex> g(mu);
  used -= r.footprint;
}

void lpd_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      if (!in_flight && resident.empty() && staged.empty() && retiring.empty())
        cv.wait(lk, [&] { return stop || !pending.empty(); });
      if (stop && pending.empty() && !in_flight && resident.empty() && staged.empty() && retiring.empty()) return;
    }
    admit();  // its copies overlap the epoch in flight
    if (in_flight) retire_epoch();
    if (!staged.empty()) {
      (void)hipStreamWaitEvent(stream, ev_staged, 0);
      for (Request& r : staged) resident.push_back(r);
      staged.clear();
    }
    if (!resident.empty()) launch_epoch();
    finish_retiring();  // while the new epoch runs
  }
}

// Admission in arrival order while the budget and the slot table allow; the
// admitted requests' inputs go to HBM on the copy stream.
void lpd_server::admit() {
  std::vector<Request> batch;
  {
    std::lock_guard<std::mutex> g(mu);
    uint64_t round_bytes = 0;
    while (!pending.empty() && batch.size() < free_slots.size()) {
      Request& r = pending.front();
      if (used + r.footprint > budget) break;
      // Bounded copy work per step, so that retiring and relaunching are not
      // held up behind a burst of admissions.
      const uint64_t in = 8 * (uint64_t)(r.m * r.n + r.m + r.n);
      if (!batch.empty() && round_bytes + in > (uint64_t)opt.admit_bytes_per_round) break;
      round_bytes += in;
      r.t_admit = now();
      used += r.footprint;
      stats.peak_bytes = std::max<uint64_t>(stats.peak_bytes, used);
      batch.push_back(r);
      pending.pop_front();
    }
    stats.resident = (int64_t)(resident.size() + staged.size() + batch.size());
    stats.waiting = (int64_t)pending.size();
  }
  if (batch.empty()) return;
  const Clock::time_point h0 = Clock::now();
  uint64_t bytes = 0;
  for (Request& r : batch) {
    hipError_t e = hipMallocAsync((void**)&r.dmem, r.footprint, copy_stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      r.dmem = nullptr;
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
    (void)hipMemcpyAsync(r.dA, r.A, 8 * (size_t)(r.m * r.n), hipMemcpyHostToDevice, copy_stream);
    (void)hipMemcpyAsync(r.db, r.b, 8 * (size_t)r.m, hipMemcpyHostToDevice, copy_stream);
    (void)hipMemcpyAsync(r.dc, r.c, 8 * (size_t)r.n, hipMemcpyHostToDevice, copy_stream);
    (void)hipMemcpyAsync(d_status + r.slot, init_status + r.slot, 4, hipMemcpyHostToDevice, copy_stream);
    (void)hipMemcpyAsync(d_state + r.slot, init_state + r.slot, sizeof(SolveState), hipMemcpyHostToDevice,
                         copy_stream);
    bytes += 8 * (uint64_t)(r.m * r.n + r.m + r.n);
    staged.push_back(r);
  }
  (void)hipEventRecord(ev_staged, copy_stream);
  std::lock_guard<std::mutex> g(mu);
  stats.admit_host_seconds += std::chrono::duration<double>(Clock::now() - h0).count();
  stats.copy_bytes += bytes;
}

void lpd_server::launch_epoch() {
  // LPs the batch kernel can place go into one batched launch; wide ones
  // (pivot row longer than the LDS holds) each get a grid launch of their own
  // after it, with column panels, resumable like the batch's team LPs.
  std::vector<int32_t> in_batch, wide;
  for (int32_t i = 0; i < (int32_t)resident.size(); ++i) (resident[(size_t)i].wide ? wide : in_batch).push_back(i);
  const int32_t count = (int32_t)in_batch.size();
  std::vector<int64_t> m((size_t)count), n((size_t)count);
  for (int32_t j = 0; j < count; ++j) {
    m[(size_t)j] = resident[(size_t)in_batch[(size_t)j]].m;
    n[(size_t)j] = resident[(size_t)in_batch[(size_t)j]].n;
  }
  hipError_t e = hipSuccess;
  BatchPlan P;
  if (count > 0) {
    P = plan_batch(count, m.data(), n.data(), knobs, nblocks, lds_limit);
    if (!P.ok) e = hipErrorInvalidValue;
    if (e == hipSuccess) {
      const int maxb = batch_max_blocks(P.lds_bytes, P.condensed);
      if (maxb <= 0) e = hipErrorInvalidValue;
      else if (nblocks > maxb) P = plan_batch(count, m.data(), n.data(), knobs, maxb, lds_limit);
    }
  }
  auto args_of = [&](const Request& r) {
    SolveArgs a{};
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
    return a;
  };
  // Pivots per epoch: a pivot streams the tableau twice (read, write), split
  // over the workgroups the LP runs on.
  auto budget_of = [&](const Request& r, double wgs) {
    if (opt.pivots_per_epoch > 0) return (int64_t)opt.pivots_per_epoch;
    const double k = (double)opt.epoch_bytes_per_wg * wgs / (2.0 * stored_bytes(r.m, r.n, knobs.condensed));
    return (int64_t)std::max(1.0, std::min(k, 1e9));
  };
  std::vector<BatchItem> items((size_t)count);
  for (int32_t j = 0; j < count && e == hipSuccess; ++j) {
    const Request& r = resident[(size_t)in_batch[(size_t)j]];
    BatchItem& it = items[(size_t)j];
    it = BatchItem{};
    it.a = args_of(r);
    it.klass = P.klass[(size_t)j];
    it.tclass = P.tclass[(size_t)j];
    it.a.pivot_budget = budget_of(r, it.klass == kClassTeam ? (double)P.cls_size[it.tclass] : 1.0);
    it.ws = r.dws;
    // The planner's LDS test is the one submit used; never launch an LP
    // without the workspace its class walks over.
    if (it.klass != kClassLds && it.klass != kClassWave && !r.has_ws) e = hipErrorInvalidValue;
  }
  if (e == hipSuccess && count > 0 && P.total > meta_bytes) {
    if (meta) (void)hipFreeAsync(meta, stream);
    meta = nullptr;
    meta_bytes = 0;
    e = hipMallocAsync(&meta, P.total, stream);
    if (e == hipSuccess) meta_bytes = P.total;
  }
  (void)hipEventRecord(ev_k0, stream);
  if (e == hipSuccess && count > 0) e = launch_batch(P, items, meta, stream);
  for (int32_t i : wide) {
    if (e != hipSuccess) break;
    const Request& r = resident[(size_t)i];
    SolveArgs a = args_of(r);
    const int nb = std::min(nblocks, grid_max_blocks(r.m, r.n, 0, knobs.condensed));
    if (nb <= 0 || !r.has_ws) {
      e = hipErrorInvalidValue;
      break;
    }
    a.pivot_budget = budget_of(r, (double)nb);
    e = launch_grid_solve(a, r.dws, nb, 0, stream, knobs.condensed);
  }
  (void)hipEventRecord(ev_k1, stream);
  if (e != hipSuccess) (void)hipGetLastError();
  // Statuses, objectives and pivot counts of every slot in one copy each.
  (void)hipMemcpyAsync(h_status, d_status, 4 * (size_t)nslots, hipMemcpyDeviceToHost, stream);
  (void)hipMemcpyAsync(h_obj, d_obj, 8 * (size_t)nslots, hipMemcpyDeviceToHost, stream);
  (void)hipMemcpyAsync(h_iter, d_iter, 8 * (size_t)nslots, hipMemcpyDeviceToHost, stream);
  epoch_err = e;
  in_flight = true;
}

void lpd_server::retire_epoch() {
  in_flight = false;
  hipError_t e = epoch_err;
  const hipError_t es = hipStreamSynchronize(stream);
  if (e == hipSuccess) e = es;
  float ms = 0.f;
  const bool timed = e == hipSuccess && hipEventElapsedTime(&ms, ev_k0, ev_k1) == hipSuccess;
  {
    std::lock_guard<std::mutex> g(mu);
    stats.epochs += 1;
    if (timed) stats.kernel_seconds += ms * 1e-3;
  }
  // Finished LPs: their x goes back on the result stream (the epoch that
  // wrote it is complete), and they are completed once it has arrived, after
  // the next epoch has been launched.  Their slot-table entries are read now:
  // the next epoch's copies overwrite the host mirrors.
  std::vector<Request> still;
  for (Request& r : resident) {
    const int32_t st = e == hipSuccess ? h_status[r.slot] : (int32_t)LPD_ERR_HIP;
    if (st == -1) {
      still.push_back(r);
    } else {
      if (st >= 0) (void)hipMemcpyAsync(r.x_out, r.dx, 8 * (size_t)r.n, hipMemcpyDeviceToHost, res_stream);
      retiring.push_back(r);
      retiring_status.push_back(st);
      retiring_obj.push_back(h_obj[r.slot]);
      retiring_iter.push_back(h_iter[r.slot]);
    }
  }
  if (!retiring.empty()) (void)hipEventRecord(ev_xdone, res_stream);
  resident.swap(still);
}

void lpd_server::finish_retiring() {
  if (retiring.empty()) return;
  (void)hipEventSynchronize(ev_xdone);
  // Their memory is freed on the compute stream after the x copies (and
  // after the epoch just launched, which does not touch it).
  (void)hipStreamWaitEvent(stream, ev_xdone, 0);
  for (size_t k = 0; k < retiring.size(); ++k) {
    Request& r = retiring[k];
    release(r);
    complete(r, retiring_status[k], retiring_obj[k], retiring_iter[k]);
  }
  retiring.clear();
  retiring_status.clear();
  retiring_obj.clear();
  retiring_iter.clear();
}

extern "C" {

lpd_server* lpd_server_create(int device, uint64_t budget_bytes, const lpd_server_options* opt) {
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return nullptr;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess || std::strncmp(p.gcnArchName, "gfx950", 6) != 0)
    return nullptr;
  if (opt && (std::isnan(opt->eps_d) || std::isnan(opt->eps_p))) return nullptr;
  if (hipSetDevice(device) != hipSuccess) return nullptr;
  lpd_server* s = new lpd_server();
  s->device = device;
  s->budget = budget_bytes;
  if (opt) s->opt = *opt;
  if (!(s->opt.eps_d > 0)) s->opt.eps_d = LPD_DEFAULT_EPS;
  if (!(s->opt.eps_p > 0)) s->opt.eps_p = LPD_DEFAULT_EPS;
  if (s->opt.pivots_per_epoch < 0) s->opt.pivots_per_epoch = 0;
  if (s->opt.epoch_bytes_per_wg <= 0) s->opt.epoch_bytes_per_wg = 256ll << 20;
  if (s->opt.admit_bytes_per_round <= 0) s->opt.admit_bytes_per_round = 512ll << 20;
  if (s->opt.max_resident <= 0) s->opt.max_resident = 4096;
  s->knobs.team_size = 0;
  s->knobs.share = true;
  s->knobs.share_min_bytes_per_wg = s->opt.team_bytes_per_wg > 0 ? s->opt.team_bytes_per_wg : kShareMinBytesPerWg;
  // Default threshold: any LP that could fill a team of two.
  s->knobs.team_min_bytes = s->opt.team_min_bytes != 0 ? s->opt.team_min_bytes : 2 * s->knobs.share_min_bytes_per_wg;
  s->knobs.own_workspaces = true;
  s->knobs.wave_slots = tuned_batch_knobs().wave_slots;
  s->knobs.condensed = s->opt.full_tableau == 0;
  s->nslots = s->opt.max_resident;
  s->nblocks = p.multiProcessorCount;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) lds = 0;
  s->lds_limit = (size_t)lds;
  // Keep freed pool memory reserved: admissions and departures allocate and
  // free stream-ordered all the time.
  keep_freed_pool_memory(device);
  const size_t ns = (size_t)s->nslots;
  bool ok = hipStreamCreate(&s->stream) == hipSuccess;
  ok = ok && hipStreamCreate(&s->copy_stream) == hipSuccess;
  ok = ok && hipStreamCreate(&s->res_stream) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&s->ev_staged, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&s->ev_xdone, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreate(&s->ev_k0) == hipSuccess;
  ok = ok && hipEventCreate(&s->ev_k1) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->d_status, 4 * ns) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->d_obj, 8 * ns) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->d_iter, 8 * ns) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->d_state, sizeof(SolveState) * ns) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&s->h_status, 4 * ns, 0) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&s->h_obj, 8 * ns, 0) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&s->h_iter, 8 * ns, 0) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&s->init_status, 4 * ns, 0) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&s->init_state, sizeof(SolveState) * ns, 0) == hipSuccess;
  (void)hipSetDevice(prev);
  if (!ok) {
    (void)hipGetLastError();
    lpd_server_destroy(s);
    return nullptr;
  }
  for (size_t i = 0; i < ns; ++i) {
    s->init_status[i] = -1;
    s->init_state[i] = SolveState{};
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
  // Same LDS tests as the batch planner: an LP it cannot place runs as a
  // grid launch of its own each epoch.
  const bool wide = !batch_can_place(m, n, s->knobs.condensed, s->lds_limit);
  const bool lds = !wide && wg_lds_bytes(m, n) + 256 <= s->lds_limit;
  // A wide LP's workspace has barrier slots for a launch on every CU.
  const uint64_t f = wide ? input_bytes(m, n) + grid_layout(m, n, s->nblocks, s->knobs.condensed).total
                          : footprint_of(m, n, lds, s->knobs.condensed);
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
  r.wide = wide;
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
  if (s->copy_stream) (void)hipStreamSynchronize(s->copy_stream);
  if (s->res_stream) (void)hipStreamSynchronize(s->res_stream);
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
  (void)hipHostFree(s->init_status);
  (void)hipHostFree(s->init_state);
  for (hipEvent_t ev : {s->ev_staged, s->ev_xdone, s->ev_k0, s->ev_k1})
    if (ev) (void)hipEventDestroy(ev);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  if (s->res_stream) (void)hipStreamDestroy(s->res_stream);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  (void)hipSetDevice(prev);
  delete s;
}

}  // extern "C"
