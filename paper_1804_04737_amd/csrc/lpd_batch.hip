// Batched solve of many independent dense LPs in one persistent launch.
//
// Every LP is solved by exactly the algorithm of the single-LP paths
// (lpd_team.h, lpd_wgsolve.h), so its result is bit-identical to its own
// lp_solve_dense call.  The launch is cooperative (all workgroups resident):
//
//   phase 1  workgroups form teams of S; each team pops the next large LP
//            (tableau >= team_min_bytes) from a big-first queue and solves it
//            with the team-scoped reduction barrier;
//   phase 2  when the large queue is empty, every workgroup pops small LPs
//            one at a time: LDS-resident if the tableau fits in LDS, else the
//            one-workgroup grid walk over its private workspace in HBM.
//
// Queue heads are device-scope atomic counters; a team's pop is broadcast to
// its members through the team barrier, which also guarantees that every
// member has finished reading the previous LP before the next one is built in
// the shared workspace.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lpd_batch.h"
#include "lpd_team.h"
#include "lpd_wgsolve.h"

namespace lpd {
namespace {

constexpr int kBT = 1024;  // threads per workgroup

__global__ void __launch_bounds__(kBT) batch_kernel(BatchWork bw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int32_t s_idx;
  const int b = blockIdx.x, S = bw.team_size;
  uint32_t epoch = 0;

  // ---- phase 1: teams on the large LPs
  const int team = S > 0 ? b / S : 0;
  if (S > 0 && team < bw.n_teams) {
    const Team tm{b % S, S, bw.slots + (size_t)team * 2 * S, &epoch};
    unsigned char* ws = bw.team_ws + (size_t)team * bw.team_ws_stride;
    for (;;) {
      Cand c = cand_none();
      if (tm.rank == 0) {
        if (threadIdx.x == 0) s_idx = (int32_t)atomicAdd(&bw.counters[0], 1u);
        __syncthreads();
        c.v = 0.0;
        c.i = s_idx;
      }
      // Broadcast the leader's pick; also fences the previous LP of the team.
      const Cand got = grid_reduce(tm, c, ++epoch, reinterpret_cast<Cand*>(smem));
      if ((got.flags & kFlagTimeout) || got.i >= bw.n_team) break;
      const BatchItem& it = bw.items[bw.team_list[__builtin_amdgcn_readfirstlane(got.i)]];
      const GridLayout L = grid_layout(it.a.m, it.a.n, S);
      GridWork w = make_grid_work(L, it.a.m, ws);
      w.cap_cap = bw.cap_cap;
      w.lds_vecs = bw.lds_vecs;
      team_solve<kBT, 0>(it.a, w, tm, smem);
    }
  }

  // ---- phase 2: one workgroup per small LP
  const Team solo{0, 1, nullptr, &epoch};
  unsigned char* ws = bw.wg_ws ? bw.wg_ws + (size_t)b * bw.wg_ws_stride : nullptr;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_idx = (int32_t)atomicAdd(&bw.counters[8], 1u);
    __syncthreads();
    const int32_t idx = __builtin_amdgcn_readfirstlane(s_idx);
    if (idx >= bw.n_single) break;
    const BatchItem& it = bw.items[bw.single_list[idx]];
    if (it.klass == kClassLds) {
      wg_solve<kBT>(it.a, smem);
    } else {
      const GridLayout L = grid_layout(it.a.m, it.a.n, 1);
      GridWork w = make_grid_work(L, it.a.m, ws);
      w.cap_cap = bw.cap_cap;
      w.lds_vecs = bw.lds_vecs;
      team_solve<kBT, 0>(it.a, w, solo, smem);
    }
  }
}

__global__ void batch_clear_kernel(uint32_t* counters, BarrierSlot* slots, int nslots) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2) counters[i * 8] = 0u;
  if (i < nslots) slots[i].epoch = 0u;
}

int lds_limit_bytes() {
  int dev = 0, lds = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  return lds;
}

}  // namespace

BatchPlan plan_batch(int32_t count, const int64_t* m, const int64_t* n, int team_size, int64_t team_min_bytes,
                     int nblocks) {
  BatchPlan P;
  P.nblocks = nblocks;
  // Static LDS of the kernel (s_idx) plus alignment slack stays outside the dynamic budget.
  const size_t limit = (size_t)std::max(0, lds_limit_bytes() - 256);
  std::vector<std::pair<double, int32_t>> team, single;
  int64_t max_vw = 1;
  size_t lds_wg = 0;
  for (int32_t i = 0; i < count; ++i) {
    const double R = (double)m[i] + 1, W = (double)(n[i] + m[i] + 1);
    const double bytes = R * W * 8.0;
    const double work = bytes * (double)(m[i] + n[i]);  // proxy: tableau size x pivot-count scale
    const size_t lds_i = wg_lds_bytes(m[i], n[i]);
    int32_t klass;
    if (lds_i <= limit) {
      klass = kClassLds;
      lds_wg = std::max(lds_wg, lds_i);
    } else if (team_size > 1 && team_min_bytes >= 0 && bytes >= (double)team_min_bytes) {
      klass = kClassTeam;
    } else {
      klass = kClassSingle;
    }
    P.klass.push_back(klass);
    if (klass != kClassLds) max_vw = std::max<int64_t>(max_vw, (n[i] + m[i] + 1) / 2);
    (klass == kClassTeam ? team : single).push_back({-work, i});
  }
  std::stable_sort(team.begin(), team.end());
  std::stable_sort(single.begin(), single.end());
  for (auto& t : team) P.team_list.push_back(t.second);
  for (auto& s : single) P.single_list.push_back(s.second);
  P.team_size = team.empty() ? 0 : std::max(1, std::min(team_size, nblocks));
  P.n_teams = P.team_size ? nblocks / P.team_size : 0;

  // LDS: the grid walk needs the pivot row of the widest non-LDS LP plus a
  // capture list; the LDS-resident LPs need their whole tableau.
  const size_t base = kScratchBytes + (size_t)max_vw * 16 + 16;
  P.ok = base <= limit;
  P.lds_vecs = (int32_t)max_vw;
  P.cap_cap = P.ok ? (int32_t)std::min<size_t>(kCapMax, (limit - base) / kCapEntryBytes) : 0;
  P.lds_bytes = std::max(lds_wg, base + (size_t)P.cap_cap * kCapEntryBytes);

  // Workspaces: one per team (largest team LP), one per workgroup (largest single LP in HBM).
  uint64_t team_ws = 0, wg_ws = 0;
  for (int32_t i : P.team_list) team_ws = std::max<uint64_t>(team_ws, grid_layout(m[i], n[i], P.team_size).total);
  for (int32_t i : P.single_list)
    if (P.klass[i] == kClassSingle) wg_ws = std::max<uint64_t>(wg_ws, grid_layout(m[i], n[i], 1).total);
  P.team_ws_stride = team_ws;
  P.wg_ws_stride = wg_ws;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off += (uint64_t)round_up((int64_t)bytes, 256);
    return o;
  };
  P.off_items = take((uint64_t)count * sizeof(BatchItem));
  P.off_lists = take((uint64_t)(P.team_list.size() + P.single_list.size()) * 4 + 4);
  P.off_counters = take(64);
  P.off_slots = take((uint64_t)P.n_teams * 2 * std::max(P.team_size, 1) * sizeof(BarrierSlot));
  P.off_team_ws = take((uint64_t)P.n_teams * team_ws);
  P.off_wg_ws = take((uint64_t)nblocks * wg_ws);
  P.total = off;
  return P;
}

hipError_t launch_batch(const BatchPlan& P, const std::vector<BatchItem>& items, void* workspace,
                        hipStream_t stream) {
  unsigned char* base = static_cast<unsigned char*>(workspace);
  // Descriptor table and queues: one host-to-device copy (pageable source;
  // the runtime stages it before returning).
  std::vector<unsigned char> host(P.off_counters);
  std::memcpy(host.data() + P.off_items, items.data(), items.size() * sizeof(BatchItem));
  int32_t* lists = reinterpret_cast<int32_t*>(host.data() + P.off_lists);
  std::copy(P.team_list.begin(), P.team_list.end(), lists);
  std::copy(P.single_list.begin(), P.single_list.end(), lists + P.team_list.size());
  hipError_t e = hipMemcpyAsync(base, host.data(), host.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;

  BatchWork bw{};
  bw.items = reinterpret_cast<const BatchItem*>(base + P.off_items);
  bw.team_list = reinterpret_cast<const int32_t*>(base + P.off_lists);
  bw.n_team = (int32_t)P.team_list.size();
  bw.single_list = bw.team_list + P.team_list.size();
  bw.n_single = (int32_t)P.single_list.size();
  bw.counters = reinterpret_cast<uint32_t*>(base + P.off_counters);
  bw.slots = reinterpret_cast<BarrierSlot*>(base + P.off_slots);
  bw.team_ws = base + P.off_team_ws;
  bw.team_ws_stride = P.team_ws_stride;
  bw.wg_ws = P.wg_ws_stride ? base + P.off_wg_ws : nullptr;
  bw.wg_ws_stride = P.wg_ws_stride;
  bw.team_size = P.team_size;
  bw.n_teams = P.n_teams;
  bw.cap_cap = P.cap_cap;
  bw.lds_vecs = P.lds_vecs;

  const int nslots = P.n_teams * 2 * std::max(P.team_size, 1);
  batch_clear_kernel<<<(std::max(nslots, 2) + 255) / 256, 256, 0, stream>>>(bw.counters, bw.slots, nslots);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_bytes);
  if (e != hipSuccess) return e;
  void* params[] = {&bw};
  return hipLaunchCooperativeKernel((const void*)batch_kernel, dim3(P.nblocks), dim3(kBT), params,
                                    (unsigned)P.lds_bytes, stream);
}

int batch_max_blocks(size_t lds_bytes) {
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipFuncSetAttribute((const void*)batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) !=
      hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel, kBT, lds_bytes) != hipSuccess) return 0;
  return per_cu * ncu;
}

}  // namespace lpd
