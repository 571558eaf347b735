// Kernel parameter blocks and launch entry points shared between the host
// runtime (lpd_api.hip) and the kernels (lpd_grid.hip, lpd_wg.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpd {

// Where a resumable solve stands between launches (device memory, one per LP).
struct SolveState {
  int32_t phase;   // 0: not started, 1: suspended between pivots, 2: finished
  int32_t k, l, lprev;
  double g, p;
  int64_t iter;
  int32_t kc, kprev;  // condensed tableau: stored column of k; entering variable of the last pivot
};

// Inputs, options and outputs of one LP solve as the kernels see them.
struct SolveArgs {
  int64_t m, n;
  const double* A;
  const double* b;
  const double* c;
  double eps_d, eps_p;
  int64_t max_iter;
  // outputs (device; optional ones may be null)
  double* x;
  double* obj;
  int32_t* status;
  double* y;
  int64_t* iterations;
  int32_t* trace;
  int64_t trace_cap;
  int64_t* basis_out;
  double* tableau_out;
  uint64_t* phase_ticks;
  int64_t phase_cap;
  // Resumable solves (grid walk only): state kept in device memory between
  // launches, and the most pivots one launch may do (< 0: no limit).  The
  // budget is ignored when state is null.
  SolveState* state;
  int64_t pivot_budget;
  // Start from a given basic tableau instead of building Table 1 from A, b,
  // c (T0 null: Table 1).  With ncols = n + m variable columns, T0 is
  // (m+1) x (ncols+1) row-major, RHS last, objective row last; basis0[i] is
  // the variable of row i and pos0[j] the row of variable j (-1 if
  // nonbasic).  Condensed tableau: lab0[c] (n + 1 entries, the last unused)
  // is the variable held in stored column c, the nonbasic variables in
  // increasing order, and colof0[j] the stored column of variable j (-1 if
  // basic).
  const double* T0;
  const int32_t* basis0;
  const int32_t* pos0;
  const int32_t* lab0;
  const int32_t* colof0;
  int64_t x_count;  // entries of x written by the read-out (0: n)
  // Bound of every barrier wait of a multi-workgroup team, in ticks of the
  // 100 MHz real-time clock: 0 the default (10 s), < 0 none (each wait
  // gives up at once, for tests of the timeout path).
  int64_t watchdog;
};

// Reduction-barrier slot: one per workgroup and per epoch parity, 128 B apart.
struct alignas(128) BarrierSlot {
  double v;
  double aux;
  int32_t i;
  int32_t flags;
  uint32_t epoch;
  uint32_t pad0;
  uint64_t t_arrive;  // device real-time clock at arrival (diagnostics)
  uint64_t t_pub;     // ... after the release that precedes publication (diagnostics)
  uint32_t pad[20];
};
static_assert(sizeof(BarrierSlot) == 128, "slot must fill one 128 B line");

// Chunk-ticket counters of the update sweep's dynamic part: kTicketCounters
// counters, each in its own block of kTicketStride uint32 (4 KiB), each with
// one word per pivot parity (128 B apart).
constexpr int kTicketCounters = 2;
constexpr int kTicketStride = 1024;

// Device workspace of the persistent grid solve (all pointers into one allocation).
struct GridWork {
  int64_t ld;      // row stride of T in doubles (multiple of 32)
  int64_t vw;      // 16-byte vectors per row that carry data: ceil((n+m)/2)
  double* T;       // m x ld, constraint rows, columns 0..n+m-1 (RHS kept apart)
  double* obj[2];  // objective row (ld doubles), double-buffered by pivot parity
  double* pr[2];   // normalised pivot row of the last pivot (ld doubles), by parity
  double* pcol[2]; // column of the entering variable, rows 0..m-1, by parity
  double* rhs[2];  // right-hand side, rows 0..m (row m = objective value), by parity
  int32_t* basis;  // m: basic variable of each row
  int32_t* pos;    // n+m: row of each basic variable, -1 if nonbasic
  // Condensed tableau only (T holds the n nonbasic columns):
  int32_t* lab;    // n: variable held by each stored column
  int32_t* col_of; // n+m: stored column of each nonbasic variable, -1 if basic
  uint32_t* tickets;   // sweep chunk tickets: counter h of pivot parity q at [h * kTicketStride + 32 q]
  BarrierSlot* slots; // 2 * nblocks
  // Two pivots per sweep only: the normalised pivot row of the pair's first
  // pivot (ld doubles) and the entering column of its second pivot after the
  // first update (m doubles), each workgroup writing one slice of each; and a
  // private copy of that row per workgroup (priv_stride doubles each), used
  // where the row is longer than the LDS.
  double* prt;
  double* pap;
  double* priv;
  int64_t priv_stride;
  int32_t cap_cap;     // capacity of the LDS capture list (entries)
  int32_t lds_vecs;    // capacity of the LDS pivot-row buffer (16-byte vectors; < vw: column panels)
};

// Sizes of the grid workspace pieces (bytes, each rounded to 256).
struct GridLayout {
  int64_t ld, vw;
  uint64_t off_T, off_obj, off_pr, off_pcol, off_rhs, off_basis, off_pos, off_lab, off_colof, off_tickets,
      off_pair, off_priv, off_slots, total;
};

__host__ __device__ inline int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// Workspace of one team solve of an m x n LP by `nblocks` workgroups.  The
// full tableau stores the n+m columns of Table 1; the condensed one only the
// n columns of the nonbasic variables (the basic ones are unit columns).
// `paired` (two pivots per sweep) adds one row and one column, and one row
// per workgroup.
__host__ __device__ inline GridLayout grid_layout(int64_t m, int64_t n, int nblocks, bool condensed = false,
                                                 bool paired = false) {
  GridLayout L{};
  L.vw = condensed ? (n + 1) / 2 : (n + m + 1) / 2;
  L.ld = round_up(2 * L.vw, 32);
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off += (uint64_t)round_up((int64_t)bytes, 256);
    return o;
  };
  L.off_T = take((uint64_t)m * L.ld * 8);
  L.off_obj = take(2ull * L.ld * 8);
  L.off_pr = take(2ull * L.ld * 8);
  L.off_pcol = take(2ull * (uint64_t)m * 8);
  L.off_rhs = take(2ull * (uint64_t)(m + 1) * 8);
  L.off_basis = take((uint64_t)m * 4);
  L.off_pos = take((uint64_t)(n + m) * 4);
  L.off_lab = take(condensed ? (uint64_t)(n + 1) * 4 : 0);  // n + 1: read in pairs
  L.off_colof = take(condensed ? (uint64_t)(n + m) * 4 : 0);
  L.off_tickets = take((uint64_t)kTicketCounters * kTicketStride * 4);  // one 4 KiB block per counter
  L.off_pair = take(paired ? (uint64_t)(L.ld + round_up(m, 32)) * 8 : 0);
  L.off_priv = take(paired ? (uint64_t)nblocks * (uint64_t)L.ld * 8 : 0);
  L.off_slots = take(2ull * nblocks * sizeof(BarrierSlot));
  L.total = off;
  return L;
}

// Pointers of a GridWork carved out of `workspace` by layout L (LDS fields unset).
__host__ __device__ inline GridWork make_grid_work(const GridLayout& L, int64_t m, void* workspace) {
  unsigned char* base = static_cast<unsigned char*>(workspace);
  GridWork w{};
  w.ld = L.ld;
  w.vw = L.vw;
  w.T = reinterpret_cast<double*>(base + L.off_T);
  for (int q = 0; q < 2; ++q) {
    w.obj[q] = reinterpret_cast<double*>(base + L.off_obj) + q * L.ld;
    w.pr[q] = reinterpret_cast<double*>(base + L.off_pr) + q * L.ld;
    w.pcol[q] = reinterpret_cast<double*>(base + L.off_pcol) + q * m;
    w.rhs[q] = reinterpret_cast<double*>(base + L.off_rhs) + q * (m + 1);
  }
  w.basis = reinterpret_cast<int32_t*>(base + L.off_basis);
  w.pos = reinterpret_cast<int32_t*>(base + L.off_pos);
  w.lab = reinterpret_cast<int32_t*>(base + L.off_lab);
  w.col_of = reinterpret_cast<int32_t*>(base + L.off_colof);
  w.tickets = reinterpret_cast<uint32_t*>(base + L.off_tickets);
  w.prt = reinterpret_cast<double*>(base + L.off_pair);
  w.pap = w.prt + L.ld;
  w.priv = reinterpret_cast<double*>(base + L.off_priv);
  w.priv_stride = L.ld;
  w.slots = reinterpret_cast<BarrierSlot*>(base + L.off_slots);
  return w;
}

// Host-side launchers (return hipError_t of the launch).
hipError_t launch_grid_solve(const SolveArgs& a, void* workspace, int nblocks, int nthreads,
                             hipStream_t stream, bool condensed = false, bool paired = false);
// Largest grid the persistent kernel can run co-resident with `nthreads` per block
// and the LDS a given tableau width needs (0 if it cannot run at all).
int grid_max_blocks(int64_t m, int64_t n, int nthreads, bool condensed = false, bool paired = false);
// LDS bytes the grid kernel needs for an n+m wide tableau.
size_t grid_lds_bytes(int64_t m, int64_t n, int nthreads, bool condensed = false);

// Single-workgroup solve with the tableau resident in LDS.
size_t wg_lds_bytes(int64_t m, int64_t n);
size_t wg_lds_limit();
hipError_t launch_wg_solve(const SolveArgs& a, hipStream_t stream);

}  // namespace lpd
