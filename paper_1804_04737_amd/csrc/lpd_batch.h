// Host/device types of the batched solve (lpd_batch.hip), shared with the
// serving runtime (lpd_server.hip).
#pragma once

#include <vector>

#include "lpd_kernels.h"

namespace lpd {

// How one LP of a batch is solved.
enum : int32_t {
  kClassLds = 0,     // one workgroup, tableau in LDS (always runs to the end)
  kClassSingle = 1,  // one workgroup, grid walk over an HBM workspace
  kClassTeam = 2,    // a team of workgroups, grid walk over an HBM workspace
  kClassWave = 3     // one wave, tableau in the wave's slice of LDS (runs to the end)
};

constexpr int kMaxTeamClasses = 4;

struct BatchItem {
  SolveArgs a;
  int32_t klass;
  int32_t tclass;     // team class index (kClassTeam only)
  unsigned char* ws;  // the LP's own workspace, or null for the batch's shared ones
};

// Workgroups [base, base + n_teams * size) form teams of `size` that share
// one queue of LPs.
struct TeamClass {
  int32_t size, base, n_teams, n_items;
  const int32_t* list;  // LP indices, big first
  unsigned char* ws;    // per-team workspaces (null when every LP brings its own)
  uint64_t ws_stride;
  BarrierSlot* slots;   // n_teams * 2 * size
};

// Device view of a batch (pointers into one workspace allocation).
struct BatchWork {
  const BatchItem* items;
  TeamClass cls[kMaxTeamClasses];
  int32_t n_classes;
  uint32_t* counters;          // queue heads: [8 c] team class c, [8 kMaxTeamClasses] singles,
                               // [8 (kMaxTeamClasses + 1)] one-wave LPs
  const int32_t* single_list;  // LP indices of the one-workgroup queue, big first
  int32_t n_single;
  const int32_t* wave_list;    // LP indices of the one-wave queue, big first
  int32_t n_wave;
  int32_t wave_slots;          // waves per workgroup that take one-wave LPs
  uint32_t wave_slice;         // LDS bytes of each such wave
  unsigned char* wg_ws;        // per-workgroup workspaces (null when not needed)
  uint64_t wg_ws_stride;
  int32_t cap_cap, lds_vecs;
};

// Scheduling knobs of a batch.
struct BatchKnobs {
  int team_size = 0;               // > 0: one fixed team size; 0: sized per LP
  int64_t team_min_bytes = 0;      // tableau bytes from which an LP gets a team (< 0: never)
  int64_t team_bytes_per_wg = 0;   // per-LP team sizing: tableau bytes per workgroup
  bool own_workspaces = false;     // every non-LDS LP brings its own workspace (BatchItem::ws)
  // Share sizing (team_size 0 only): every non-LDS LP gets workgroups in
  // proportion to its tableau bytes, at most one per share_min_bytes_per_wg,
  // one team per LP, so that all of them advance at once (epochs of the
  // serving runtime, where each LP does a bounded number of pivots).
  bool share = false;
  int64_t share_min_bytes_per_wg = 0;
  // Wave-per-instance: > 0 splits each workgroup's LDS into this many slices;
  // an LP whose LDS tableau fits in one slice is solved by a single wave.
  int wave_slots = 0;
  // Large LPs on the condensed tableau (nonbasic columns only; same bits).
  bool condensed = false;
};

// Host plan: classes, queue orders, LDS and workspace sizes.
struct BatchPlan {
  bool ok = false;
  int nblocks = 0;
  int n_classes = 0;
  int cls_size[kMaxTeamClasses] = {}, cls_base[kMaxTeamClasses] = {}, cls_teams[kMaxTeamClasses] = {};
  std::vector<int32_t> cls_list[kMaxTeamClasses];
  uint64_t cls_ws_stride[kMaxTeamClasses] = {};
  int32_t cap_cap = 0, lds_vecs = 0;
  size_t lds_bytes = 0;
  std::vector<int32_t> klass, tclass, single_list, wave_list;
  int32_t wave_slots = 0;
  uint32_t wave_slice = 0;
  bool condensed = false;
  uint64_t wg_ws_stride = 0;
  uint64_t off_items = 0, off_lists = 0, off_counters = 0, off_slots = 0, off_team_ws = 0, off_wg_ws = 0;
  uint64_t total = 0;
};

// lds_per_block: LDS bytes a workgroup may use (0: ask the current device).
BatchPlan plan_batch(int32_t count, const int64_t* m, const int64_t* n, const BatchKnobs& knobs, int nblocks,
                     size_t lds_per_block = 0);
// Copies the descriptor table and starts the cooperative launch (items[i].klass
// / tclass must come from the plan).
hipError_t launch_batch(const BatchPlan& P, const std::vector<BatchItem>& items, void* workspace,
                        hipStream_t stream);
int batch_max_blocks(size_t lds_bytes, bool condensed = false);
// Knobs from the autotune table (built-in defaults when there is none).
BatchKnobs tuned_batch_knobs();
// Keeps freed stream-ordered workspace in `device`'s default memory pool
// (release threshold raised), and registers once the process-exit teardown
// that synchronises the device, restores the threshold and trims the pool.
void keep_freed_pool_memory(int device);
// LDS per workgroup (bytes) of the current device, as the planner uses it.
int batch_lds_total();
// Whether the batch kernel can place an LP (lds_total: the device's LDS per
// workgroup): its tableau fits in the planner's LDS budget, or, walked over
// HBM, its pivot row does beside the reduction scratch (the batch kernel has
// no column panels).
bool batch_can_place(int64_t m, int64_t n, bool condensed, size_t lds_total);
// Tableau bytes of an m x n LP and the bytes one grid-walk workspace needs.
inline double tableau_bytes(int64_t m, int64_t n) { return ((double)m + 1) * (double)(n + m + 1) * 8.0; }
// Bytes of the tableau a grid walk stores and streams: the full one, or only
// the n nonbasic columns on the condensed tableau.
inline double stored_bytes(int64_t m, int64_t n, bool condensed) {
  return ((double)m + 1) * (double)(condensed ? n + 1 : n + m + 1) * 8.0;
}

}  // namespace lpd
