// Batched solve of many independent dense LPs in one persistent launch.
//
// Every LP is solved by exactly the algorithm of the single-LP paths
// (lpd_team.h, lpd_wgsolve.h), so its result is bit-identical to its own
// lp_solve_dense call.  The launch is cooperative (all workgroups resident):
//
//   phase 1  the workgroups of team class c form teams of size_c; each team
//            pops the next LP of its class from a big-first queue and solves
//            it with the team-scoped reduction barrier (classes group LPs of
//            similar size: larger LPs get larger teams);
//   phase 2  when its class queue is empty (or it belongs to no class), a
//            workgroup pops small LPs one at a time: LDS-resident if the
//            tableau fits in LDS, else the one-workgroup grid walk over HBM.
//
// Queue heads are device-scope atomic counters; a team's pop is broadcast to
// its members through the team barrier, which also guarantees that every
// member has finished reading the previous LP before the next one is built in
// the shared workspace.  LPs that carry a SolveState may stop after a pivot
// budget and resume in a later launch (the serving runtime uses this).
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

// One tiny LP on one wave.  Kept out of line (pointer arguments only), so its
// registers do not add to those of the team and workgroup phases.
__device__ __noinline__ void wave_solve_one(const SolveArgs* a, unsigned char* slice) {
  lds_solve<WaveGroup>(*a, slice);
}

template <bool CD>
__global__ void __launch_bounds__(kBT) batch_kernel(BatchWork bw) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int32_t s_idx;
  const int b = blockIdx.x;
  uint32_t epoch = 0;

  // ---- phase 1: teams of this workgroup's class on the large LPs
  int c = -1;
  for (int q = 0; q < bw.n_classes; ++q)
    if (b >= bw.cls[q].base && b < bw.cls[q].base + bw.cls[q].n_teams * bw.cls[q].size) c = q;
  if (c >= 0) {
    const TeamClass& tc = bw.cls[c];
    const int team = (b - tc.base) / tc.size;
    const Team tm{(b - tc.base) % tc.size, tc.size, tc.slots + (size_t)team * 2 * tc.size, &epoch};
    for (;;) {
      Cand pick = cand_none();
      if (tm.rank == 0) {
        if (threadIdx.x == 0) s_idx = (int32_t)atomicAdd(&bw.counters[8 * c], 1u);
        __syncthreads();
        pick.v = 0.0;
        pick.i = s_idx;
      }
      // Broadcast the leader's pick; also fences the previous LP of the team.
      const Cand got = grid_reduce(tm, pick, ++epoch, reinterpret_cast<Cand*>(smem));
      const int32_t idx = __builtin_amdgcn_readfirstlane(got.i);
      if ((got.flags & kFlagTimeout) || idx >= tc.n_items) break;
      const BatchItem& it = bw.items[tc.list[idx]];
      unsigned char* ws = it.ws ? it.ws : tc.ws + (size_t)team * tc.ws_stride;
      GridWork w = make_grid_work(grid_layout(it.a.m, it.a.n, tc.size, CD), it.a.m, ws);
      w.cap_cap = bw.cap_cap;
      w.lds_vecs = bw.lds_vecs;
      // Temporal tableau loads (ld_tab): the LPs in flight at once fit in the
      // memory-side cache (measured 7.8 % more LPs/s on the batch of 1024).
      team_solve<kBT, 0, CD, true, false, false, true>(it.a, w, tm, smem);
    }
  }

  // ---- phase 2: one workgroup per small LP
  const Team solo{0, 1, nullptr, &epoch};
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_idx = (int32_t)atomicAdd(&bw.counters[8 * kMaxTeamClasses], 1u);
    __syncthreads();
    const int32_t idx = __builtin_amdgcn_readfirstlane(s_idx);
    if (idx >= bw.n_single) break;
    const BatchItem& it = bw.items[bw.single_list[idx]];
    if (it.klass == kClassLds) {
      wg_solve<kBT>(it.a, smem);
    } else {
      unsigned char* ws = it.ws ? it.ws : bw.wg_ws + (size_t)b * bw.wg_ws_stride;
      GridWork w = make_grid_work(grid_layout(it.a.m, it.a.n, 1, CD), it.a.m, ws);
      w.cap_cap = bw.cap_cap;
      w.lds_vecs = bw.lds_vecs;
      team_solve<kBT, 0, CD, false, false, false, true>(it.a, w, solo, smem);
    }
  }

  // ---- phase 3: one wave per tiny LP, each wave on its own LDS slice (the
  // last phase-2 barrier guarantees nobody still reads the shared LDS).
  const int wv = threadIdx.x / kWave;
  if (wv < bw.wave_slots) {
    unsigned char* slice = smem + (size_t)wv * bw.wave_slice;
    for (;;) {
      int32_t idx = 0;
      if ((threadIdx.x & (kWave - 1)) == 0)
        idx = (int32_t)atomicAdd(&bw.counters[8 * (kMaxTeamClasses + 1)], 1u);
      idx = __builtin_amdgcn_readfirstlane(idx);
      if (idx >= bw.n_wave) break;
      wave_solve_one(&bw.items[bw.wave_list[idx]].a, slice);
    }
  }
}

__global__ void batch_clear_kernel(uint32_t* counters, BarrierSlot* slots, int nslots) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= kMaxTeamClasses + 1) counters[i * 8] = 0u;
  if (i < nslots) slots[i].epoch = 0u;
}

int lds_limit_bytes() {
  int dev = 0, lds = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  return lds;
}

int pow2_floor(int64_t x) {
  int p = 1;
  while ((int64_t)p * 2 <= x) p *= 2;
  return p;
}

}  // namespace

BatchPlan plan_batch(int32_t count, const int64_t* m, const int64_t* n, const BatchKnobs& K, int nblocks,
                     size_t lds_per_block) {
  BatchPlan P;
  P.nblocks = nblocks;
  P.condensed = K.condensed;
  const bool cd = K.condensed;
  // Static LDS of the kernel (s_idx) plus alignment slack stays outside the dynamic budget.
  const int lds_total = lds_per_block ? (int)lds_per_block : lds_limit_bytes();
  const size_t limit = (size_t)std::max(0, lds_total - 256);
  P.klass.assign((size_t)count, kClassSingle);
  P.tclass.assign((size_t)count, -1);
  std::vector<int> want((size_t)count, 0);
  std::vector<double> work((size_t)count);
  std::vector<std::pair<double, int32_t>> single;
  int64_t max_vw = 1;
  size_t lds_wg = 0;
  double w_single = 0.0;
  double share_total = 0.0;  // tableau bytes of the LPs that do not fit in LDS
  if (K.share)
    for (int32_t i = 0; i < count; ++i)
      if (wg_lds_bytes(m[i], n[i]) > limit) share_total += stored_bytes(m[i], n[i], cd);
  // Wave-per-instance slices: the whole LDS split evenly (16-byte aligned).
  const int slots = std::max(0, std::min(K.wave_slots, kBT / kWave));
  const size_t slice = slots > 0 ? (limit / (size_t)slots) & ~size_t(15) : 0;
  std::vector<std::pair<double, int32_t>> wave;
  for (int32_t i = 0; i < count; ++i) {
    const double bytes = stored_bytes(m[i], n[i], cd);
    work[(size_t)i] = bytes * (double)(m[i] + n[i]);  // proxy: tableau size x pivot-count scale
    const size_t lds_i = wg_lds_bytes(m[i], n[i]);
    if (slots > 0 && lds_i <= slice) {
      P.klass[(size_t)i] = kClassWave;
      wave.push_back({-work[(size_t)i], i});
      continue;
    }
    if (lds_i <= limit) {
      P.klass[(size_t)i] = kClassLds;
      lds_wg = std::max(lds_wg, lds_i);
    } else {
      max_vw = std::max<int64_t>(max_vw, grid_layout(m[i], n[i], 1, cd).vw);
      if (K.team_min_bytes >= 0 && bytes >= (double)K.team_min_bytes) {
        int s = 0;
        if (K.team_size > 0) {
          s = K.team_size;
        } else if (K.share) {
          const double cap = K.share_min_bytes_per_wg > 0 ? bytes / (double)K.share_min_bytes_per_wg : 1e18;
          s = pow2_floor((int64_t)std::min(cap, (double)nblocks * bytes / share_total));
        } else if (K.team_bytes_per_wg > 0) {
          s = pow2_floor((int64_t)(bytes / (double)K.team_bytes_per_wg));
        }
        s = std::min(s, nblocks);
        if (s >= 2) {
          P.klass[(size_t)i] = kClassTeam;
          want[(size_t)i] = s;
        }
      }
    }
    if (P.klass[(size_t)i] != kClassTeam) {
      single.push_back({-work[(size_t)i], i});
      w_single += work[(size_t)i];
    }
  }
  // Team classes: the distinct wanted sizes, largest first; beyond
  // kMaxTeamClasses the smaller sizes join the smallest kept class.
  std::vector<int> sizes;
  for (int s : want)
    if (s >= 2 && std::find(sizes.begin(), sizes.end(), s) == sizes.end()) sizes.push_back(s);
  std::sort(sizes.rbegin(), sizes.rend());
  // At most kMaxTeamClasses classes, and few enough that every class keeps a
  // team of two or more when the grid is small (the shrink loop below ends).
  const int max_classes = std::min(kMaxTeamClasses, nblocks / 2);
  if ((int)sizes.size() > max_classes) sizes.resize((size_t)std::max(0, max_classes));
  if (sizes.empty())
    for (int32_t i = 0; i < count; ++i)
      if (P.klass[(size_t)i] == kClassTeam) {
        P.klass[(size_t)i] = kClassSingle;
        single.push_back({-work[(size_t)i], i});
        w_single += work[(size_t)i];
      }
  P.n_classes = (int)sizes.size();
  std::vector<std::pair<double, int32_t>> cl[kMaxTeamClasses];
  double wc[kMaxTeamClasses] = {};
  for (int32_t i = 0; i < count; ++i) {
    if (P.klass[(size_t)i] != kClassTeam) continue;
    int c = P.n_classes - 1;
    for (int q = 0; q < P.n_classes; ++q)
      if (sizes[(size_t)q] == want[(size_t)i]) c = q;
    P.tclass[(size_t)i] = c;
    cl[c].push_back({-work[(size_t)i], i});
    wc[c] += work[(size_t)i];
  }
  double w_all = w_single;
  for (int c = 0; c < P.n_classes; ++c) w_all += wc[c];
  // Workgroups per class in proportion to its work (at least one team, at
  // most one team per LP); the rest starts on the one-workgroup queue.
  int used = 0;
  for (int c = 0; c < P.n_classes; ++c) {
    int s = sizes[(size_t)c];
    int g = (int)(nblocks * (wc[c] / std::max(w_all, 1.0)));
    if (K.share) g = (int)cl[c].size() * s;  // one team per LP
    g = std::max(s, g / s * s);
    g = std::min<int>(g, (int)cl[c].size() * s);
    P.cls_size[c] = s;
    P.cls_teams[c] = g / s;
    used += g;
  }
  while (used > nblocks) {  // shrink the class with the most workgroups
    int big = 0;
    for (int c = 1; c < P.n_classes; ++c)
      if (P.cls_teams[c] * P.cls_size[c] > P.cls_teams[big] * P.cls_size[big]) big = c;
    if (P.cls_teams[big] > 1) {
      --P.cls_teams[big];
      used -= P.cls_size[big];
    } else if (P.cls_size[big] > 2) {
      used -= P.cls_size[big] / 2;
      P.cls_size[big] /= 2;
    } else {
      break;  // every class is down to one team of two: n_classes * 2 <= nblocks
    }
  }
  int base = 0;
  for (int c = 0; c < P.n_classes; ++c) {
    P.cls_base[c] = base;
    base += P.cls_teams[c] * P.cls_size[c];
    std::stable_sort(cl[c].begin(), cl[c].end());
    for (auto& e : cl[c]) P.cls_list[c].push_back(e.second);
  }
  std::stable_sort(single.begin(), single.end());
  for (auto& e : single) P.single_list.push_back(e.second);
  std::stable_sort(wave.begin(), wave.end());
  for (auto& e : wave) P.wave_list.push_back(e.second);
  if (!P.wave_list.empty()) {
    P.wave_slots = slots;
    P.wave_slice = (uint32_t)slice;
  }

  // LDS: the grid walk needs the pivot row of the widest non-LDS LP plus a
  // capture list; the LDS-resident LPs need their whole tableau.
  const size_t lbase = kScratchBytes + (size_t)max_vw * 16 + 16;
  P.ok = lbase <= limit;
  P.lds_vecs = (int32_t)max_vw;
  P.cap_cap = P.ok ? (int32_t)std::min<size_t>(kCapMax, (limit - lbase) / kCapEntryBytes) : 0;
  P.lds_bytes = std::max(lds_wg, lbase + (size_t)P.cap_cap * kCapEntryBytes);
  if (P.wave_slots > 0) P.lds_bytes = std::max(P.lds_bytes, (size_t)P.wave_slots * P.wave_slice);

  // Shared workspaces unless every LP brings its own.
  uint64_t team_ws_total = 0, nslots = 0;
  for (int c = 0; c < P.n_classes; ++c) {
    uint64_t s = 0;
    if (!K.own_workspaces)
      for (int32_t i : P.cls_list[c]) s = std::max<uint64_t>(s, grid_layout(m[i], n[i], 1, cd).total);
    P.cls_ws_stride[c] = s;
    team_ws_total += (uint64_t)P.cls_teams[c] * s;
    nslots += (uint64_t)P.cls_teams[c] * 2 * P.cls_size[c];
  }
  if (!K.own_workspaces)
    for (int32_t i : P.single_list)
      if (P.klass[(size_t)i] == kClassSingle)
        P.wg_ws_stride = std::max<uint64_t>(P.wg_ws_stride, grid_layout(m[i], n[i], 1, cd).total);
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off += (uint64_t)round_up((int64_t)bytes, 256);
    return o;
  };
  P.off_items = take((uint64_t)count * sizeof(BatchItem));
  P.off_lists = take((uint64_t)count * 4 + 4);
  P.off_counters = take(32 * (kMaxTeamClasses + 2) + 32);
  P.off_slots = take(nslots * sizeof(BarrierSlot));
  P.off_team_ws = take(team_ws_total);
  P.off_wg_ws = take((uint64_t)nblocks * P.wg_ws_stride);
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
  BatchWork bw{};
  bw.items = reinterpret_cast<const BatchItem*>(base + P.off_items);
  const int32_t* dlists = reinterpret_cast<const int32_t*>(base + P.off_lists);
  size_t at = 0;
  BarrierSlot* slots = reinterpret_cast<BarrierSlot*>(base + P.off_slots);
  unsigned char* tws = base + P.off_team_ws;
  bw.n_classes = P.n_classes;
  for (int c = 0; c < P.n_classes; ++c) {
    TeamClass& tc = bw.cls[c];
    tc.size = P.cls_size[c];
    tc.base = P.cls_base[c];
    tc.n_teams = P.cls_teams[c];
    tc.n_items = (int32_t)P.cls_list[c].size();
    std::copy(P.cls_list[c].begin(), P.cls_list[c].end(), lists + at);
    tc.list = dlists + at;
    at += P.cls_list[c].size();
    tc.ws = P.cls_ws_stride[c] ? tws : nullptr;
    tc.ws_stride = P.cls_ws_stride[c];
    tws += (size_t)tc.n_teams * tc.ws_stride;
    tc.slots = slots;
    slots += (size_t)tc.n_teams * 2 * tc.size;
  }
  std::copy(P.single_list.begin(), P.single_list.end(), lists + at);
  bw.single_list = dlists + at;
  bw.n_single = (int32_t)P.single_list.size();
  at += P.single_list.size();
  std::copy(P.wave_list.begin(), P.wave_list.end(), lists + at);
  bw.wave_list = dlists + at;
  bw.n_wave = (int32_t)P.wave_list.size();
  bw.wave_slots = P.wave_slots;
  bw.wave_slice = P.wave_slice;
  bw.counters = reinterpret_cast<uint32_t*>(base + P.off_counters);
  bw.wg_ws = P.wg_ws_stride ? base + P.off_wg_ws : nullptr;
  bw.wg_ws_stride = P.wg_ws_stride;
  bw.cap_cap = P.cap_cap;
  bw.lds_vecs = P.lds_vecs;
  hipError_t e = hipMemcpyAsync(base, host.data(), host.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return e;

  const int nslots = (int)(slots - reinterpret_cast<BarrierSlot*>(base + P.off_slots));
  batch_clear_kernel<<<(std::max(nslots, kMaxTeamClasses + 2) + 255) / 256, 256, 0, stream>>>(
      bw.counters, reinterpret_cast<BarrierSlot*>(base + P.off_slots), nslots);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const void* fn = P.condensed ? (const void*)batch_kernel<true> : (const void*)batch_kernel<false>;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_bytes);
  if (e != hipSuccess) return e;
  void* params[] = {&bw};
  return hipLaunchCooperativeKernel(fn, dim3(P.nblocks), dim3(kBT), params,
                                    (unsigned)P.lds_bytes, stream);
}

int batch_lds_total() { return lds_limit_bytes(); }

bool batch_can_place(int64_t m, int64_t n, bool condensed, size_t lds_total) {
  // Same budget as plan_batch: the kernel's static LDS and alignment slack
  // stay outside it.
  const size_t limit = lds_total > 256 ? lds_total - 256 : 0;
  if (wg_lds_bytes(m, n) <= limit) return true;
  return kScratchBytes + (size_t)grid_layout(m, n, 1, condensed).vw * 16 + 16 <= limit;
}

int batch_max_blocks(size_t lds_bytes, bool condensed) {
  const void* fn = condensed ? (const void*)batch_kernel<true> : (const void*)batch_kernel<false>;
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes) !=
      hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBT, lds_bytes) != hipSuccess) return 0;
  return per_cu * ncu;
}

}  // namespace lpd
