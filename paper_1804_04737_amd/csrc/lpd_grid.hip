// Single-LP persistent cooperative-grid solve: one team made of every
// workgroup of the launch (the algorithm is in lpd_team.h).
#include <algorithm>
#include <cstdlib>

#include "lpd_team.h"

namespace lpd {
namespace {

template <int NT, int MAP, bool CD = false, bool PN = false, bool FU = false, bool TL = false>
__global__ void __launch_bounds__(NT) grid_solve_kernel(SolveArgs a, GridWork w) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  uint32_t epoch = 0;
  const Team tm{(int)blockIdx.x, (int)gridDim.x, w.slots, &epoch};
  team_solve<NT, MAP, CD, true, PN, FU, TL>(a, w, tm, smem);
}

// Clears the barrier slots of a fresh workspace (stream-ordered, no memset node).
__global__ void clear_slots_kernel(BarrierSlot* s, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s[i].epoch = 0u;
}

constexpr int kNT = 1024;

// Kernel variants (thread mapping); index 0 is the default.
typedef void (*GridKernel)(SolveArgs, GridWork);
constexpr GridKernel kVariants[] = {grid_solve_kernel<kNT, 0>, grid_solve_kernel<kNT, 1>};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
// Condensed tableau (nonbasic columns only).
constexpr GridKernel kCondensed = grid_solve_kernel<kNT, 0, true>;
// Pivot rows longer than the LDS holds: the sweep runs over column panels.
constexpr GridKernel kPanelled = grid_solve_kernel<kNT, 0, false, true>;
constexpr GridKernel kPanelledCondensed = grid_solve_kernel<kNT, 0, true, true>;
// Two pivots per sweep (two rows per column panel), full and condensed tableau.
constexpr GridKernel kPaired = grid_solve_kernel<kNT, 0, false, true, true>;
constexpr GridKernel kPairedCondensed = grid_solve_kernel<kNT, 0, true, true, true>;
// The same with plain (temporal) tableau loads, for tableaux that stay
// resident in the memory-side cache between sweeps.
constexpr GridKernel kTemporal = grid_solve_kernel<kNT, 0, false, false, false, true>;
constexpr GridKernel kTemporalCondensed = grid_solve_kernel<kNT, 0, true, false, false, true>;
constexpr GridKernel kTemporalPaired = grid_solve_kernel<kNT, 0, false, true, true, true>;
constexpr GridKernel kTemporalPairedCondensed = grid_solve_kernel<kNT, 0, true, true, true, true>;

// LPD_GRID_VARIANT (tuning / diagnostics) picks the thread mapping; 0 by default.
int variant_index(int64_t) {
  const char* e = getenv("LPD_GRID_VARIANT");
  const int x = e ? atoi(e) : 0;
  return (x >= 0 && x < kNumVariants) ? x : 0;
}

// Largest stored tableau (constraint rows, bytes) swept with temporal loads:
// 288 MiB, or LPD_TEMPORAL_MAX_MB (tuning and tests; 0 turns them off), read
// at every launch.
uint64_t temporal_max_bytes() {
  const char* e = getenv("LPD_TEMPORAL_MAX_MB");
  const long x = e ? atol(e) : 288;
  return (uint64_t)(x > 0 ? x : 0) << 20;
}

GridKernel pick_kernel(const GridLayout& L, int64_t m, bool condensed, bool panelled, bool paired = false) {
  const bool tl = variant_index(L.vw) == 0 && (uint64_t)m * (uint64_t)L.ld * 8 <= temporal_max_bytes();
  if (paired) {
    if (tl) return condensed ? kTemporalPairedCondensed : kTemporalPaired;
    return condensed ? kPairedCondensed : kPaired;
  }
  if (panelled) return condensed ? kPanelledCondensed : kPanelled;
  if (tl) return condensed ? kTemporalCondensed : kTemporal;
  return condensed ? kCondensed : kVariants[variant_index(L.vw)];
}

int lds_limit() {
  int dev = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  return lds_max;
}

// LDS plan of the grid kernel: reduction scratch, the normalised pivot row
// (vw 16-byte vectors) and a capture list of up to kCapMax entries, shrunk to
// what the LDS leaves.  A pivot row that does not fit with a full capture
// list is held one panel at a time: *vecs (the LDS row buffer, in vectors)
// is then below vw, a multiple of 64, with room for a full capture list.
// Returns 0 if even that does not fit.
size_t lds_plan(int64_t m, int64_t n, int32_t* cap, int32_t* vecs, bool condensed, bool paired = false) {
  const int64_t vw = grid_layout(m, n, 1, condensed).vw;
  const size_t limit = (size_t)lds_limit();
  const size_t fixed = kScratchBytes + 16;
  const size_t full_cap = (size_t)kCapMax * kCapEntryBytes;
  size_t c;
  int64_t v;
  if (paired) {
    // Two rows per panel: *vecs = 2 x the panel width (a multiple of 64).
    if (limit < fixed + full_cap + 2 * 64 * 16) return 0;
    const int64_t pw = std::min<int64_t>(round_up(vw, 64), (int64_t)((limit - fixed - full_cap) / 32) / 64 * 64);
    *cap = kCapMax;
    *vecs = (int32_t)(2 * pw);
    return fixed + (size_t)(2 * pw) * 16 + full_cap;
  }
  if (fixed + (size_t)vw * 16 + full_cap <= limit) {
    v = vw;
    c = kCapMax;
  } else if (fixed + (size_t)vw * 16 <= limit && (limit - fixed - (size_t)vw * 16) / kCapEntryBytes >= 256) {
    // The whole row fits with a shorter capture list (overflow is handled).
    v = vw;
    c = std::min<size_t>(kCapMax, (limit - fixed - (size_t)vw * 16) / kCapEntryBytes);
  } else {
    if (limit < fixed + full_cap + 64 * 16) return 0;
    v = (int64_t)((limit - fixed - full_cap) / 16) / 64 * 64;
    c = kCapMax;
  }
  *cap = (int32_t)c;
  *vecs = (int32_t)v;
  return fixed + (size_t)v * 16 + c * kCapEntryBytes;
}

}  // namespace

size_t grid_lds_bytes(int64_t m, int64_t n, int /*nthreads*/, bool condensed) {
  int32_t cap = 0, vecs = 0;
  return lds_plan(m, n, &cap, &vecs, condensed);
}

int grid_max_blocks(int64_t m, int64_t n, int nthreads, bool condensed, bool paired) {
  (void)nthreads;
  int32_t cap = 0, vecs = 0;
  const size_t lds = lds_plan(m, n, &cap, &vecs, condensed, paired);
  if (lds == 0) return 0;
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const GridLayout L = grid_layout(m, n, 1, condensed, paired);
  auto fn = pick_kernel(L, m, condensed, vecs < L.vw, paired);
  if (hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kNT, lds) != hipSuccess) return 0;
  return per_cu * ncu;
}

hipError_t launch_grid_solve(const SolveArgs& a, void* workspace, int nblocks, int nthreads,
                             hipStream_t stream, bool condensed, bool paired) {
  (void)nthreads;
  // Two pivots per sweep: not resumable.
  if (paired && a.state) return hipErrorInvalidValue;
  const GridLayout L = grid_layout(a.m, a.n, nblocks, condensed, paired);
  GridWork w = make_grid_work(L, a.m, workspace);
  const size_t lds = lds_plan(a.m, a.n, &w.cap_cap, &w.lds_vecs, condensed, paired);
  if (lds == 0) return hipErrorInvalidValue;

  const int nslots = 2 * nblocks;
  clear_slots_kernel<<<(nslots + 255) / 256, 256, 0, stream>>>(w.slots, nslots);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  auto fn = pick_kernel(L, a.m, condensed, w.lds_vecs < L.vw, paired);
  e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  SolveArgs args = a;
  void* params[] = {&args, &w};
  return hipLaunchCooperativeKernel((const void*)fn, dim3(nblocks), dim3(kNT), params, (unsigned)lds, stream);
}

}  // namespace lpd
