// Host/device types of the batched solve (lpd_batch.hip).
#pragma once

#include <vector>

#include "lpd_kernels.h"

namespace lpd {

// How one LP of a batch is solved.
enum : int32_t {
  kClassLds = 0,     // one workgroup, tableau in LDS
  kClassSingle = 1,  // one workgroup, grid walk over a private HBM workspace
  kClassTeam = 2     // a team of workgroups, grid walk over the team's workspace
};

struct BatchItem {
  SolveArgs a;
  int32_t klass;
  int32_t pad;
};

// Device view of a batch (all pointers into one workspace allocation).
struct BatchWork {
  const BatchItem* items;
  const int32_t* team_list;    // LP indices of the team queue, big first
  int32_t n_team;
  const int32_t* single_list;  // LP indices of the one-workgroup queue, big first
  int32_t n_single;
  uint32_t* counters;          // queue heads: [0] team queue, [8] one-workgroup queue
  BarrierSlot* slots;          // n_teams * 2 * team_size
  unsigned char* team_ws;
  uint64_t team_ws_stride;
  unsigned char* wg_ws;
  uint64_t wg_ws_stride;
  int32_t team_size, n_teams;
  int32_t cap_cap, lds_vecs;
};

// Host plan: classes, queue orders, LDS and workspace sizes.
struct BatchPlan {
  bool ok = false;
  int nblocks = 0, team_size = 0, n_teams = 0;
  int32_t cap_cap = 0, lds_vecs = 0;
  size_t lds_bytes = 0;
  std::vector<int32_t> klass, team_list, single_list;
  uint64_t team_ws_stride = 0, wg_ws_stride = 0;
  uint64_t off_items = 0, off_lists = 0, off_counters = 0, off_slots = 0, off_team_ws = 0, off_wg_ws = 0;
  uint64_t total = 0;
};

BatchPlan plan_batch(int32_t count, const int64_t* m, const int64_t* n, int team_size, int64_t team_min_bytes,
                     int nblocks);
hipError_t launch_batch(const BatchPlan& P, const std::vector<BatchItem>& items, void* workspace,
                        hipStream_t stream);
int batch_max_blocks(size_t lds_bytes);

}  // namespace lpd
