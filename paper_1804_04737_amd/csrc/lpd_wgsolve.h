// Solve of one small dense LP whose whole tableau fits in LDS, by one
// workgroup or by one wave.
//
// The (m+1) x (n+m+1) tableau of Table 1 (Coutinho et al., Section 2) is
// built in LDS and the group runs Steps 2-5 in a loop with group-level
// synchronisation only; the result leaves LDS once, at the end.  Same arithmetic
// contract as the grid path: IEEE division for the pivot row, one fma per
// eliminated element, lexicographic (value, index) arg-minima.
#pragma once

#include <type_traits>

#include "lpd_device.h"
#include "lpd_kernels.h"

namespace lpd {

// Small control block in LDS: the pivot the group's leading wave chose, or
// the status that ends the solve.
struct WgCtrl {
  double p;
  int32_t k, l, status, pad;
};

// LDS: the tableau with rows padded to an even number of doubles (16-byte
// aligned rows, so that the update moves two columns per access; the pad
// column holds zero and is never read as data), then the entering column,
// the basis, one partial arg-min per wave (any NT <= 1024) and the control
// block.
constexpr int kWgWaves = 1024 / kWave;

__host__ __device__ inline int64_t wg_ldw(int64_t W) { return (W + 1) & ~int64_t(1); }

struct WgLayout {
  size_t off_T, off_pcol, off_basis, off_scratch, off_ctrl, total;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline WgLayout wg_layout(int64_t m, int64_t n) {
  const size_t R = (size_t)m + 1, ldw = (size_t)wg_ldw(n + m + 1);
  WgLayout L;
  L.off_T = 0;
  L.off_pcol = align16(R * ldw * 8);
  L.off_basis = L.off_pcol + align16(R * 8);
  L.off_scratch = L.off_basis + align16((size_t)m * 4);
  L.off_ctrl = L.off_scratch + kWgWaves * sizeof(Cand);
  L.total = L.off_ctrl + sizeof(WgCtrl);
  return L;
}

// Thread groups that can run the LDS solve: a whole workgroup of NT threads,
// or one wave on its own slice of the workgroup's LDS (several small LPs per
// workgroup, one per wave).  Wave 0 of the group takes the decisions.
template <int NT>
struct BlockGroup {
  static constexpr int kThreads = NT;
  __device__ static int rank() { return threadIdx.x; }
  // LDS writes before, reads after.
  __device__ static void sync() { __syncthreads(); }
  // Global stores before complete before those after.
  __device__ static void order_global() { __syncthreads(); }
};

struct WaveGroup {
  static constexpr int kThreads = kWave;
  __device__ static int rank() { return threadIdx.x & (kWave - 1); }
  // A wave's LDS accesses execute in order: only the compiler needs fencing.
  __device__ static void sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __device__ static void order_global() {
    __builtin_amdgcn_s_waitcnt(0);
    sync();
  }
};

// Wave arg-min for the LDS solve, equal to the lexicographic (value, index)
// arg-min on candidates that are never NaN: the least value (v_min), then
// the least index among the lanes that hold a value equal to it, then the
// payload of the lowest such lane.  All lanes must be active; every lane
// gets the result.  ROWS16: only lanes 0-15 hold candidates (the others
// must hold cand_none), and the reduction stays within the first row of 16.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_min_d(double v) {
  int2 q = __builtin_bit_cast(int2, v);
  q.x = __builtin_amdgcn_update_dpp(q.x, q.x, CTRL, ROW_MASK, 0xF, false);
  q.y = __builtin_amdgcn_update_dpp(q.y, q.y, CTRL, ROW_MASK, 0xF, false);
  return __builtin_fmin(v, __builtin_bit_cast(double, q));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int32_t dpp_min_i(int32_t x) {
  return min(x, __builtin_amdgcn_update_dpp(x, x, CTRL, ROW_MASK, 0xF, false));
}

template <bool ROWS16>
__device__ __forceinline__ Cand wave_argmin(const Cand& c) {
  constexpr int kLast = ROWS16 ? 15 : 63;
  double v = c.v;
  v = dpp_min_d<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v = dpp_min_d<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v = dpp_min_d<0x141, 0xF>(v);  // row_half_mirror
  v = dpp_min_d<0x140, 0xF>(v);  // row_mirror
  if (!ROWS16) {
    v = dpp_min_d<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_min_d<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  }
  const double vmin = readlane_d(v, kLast);
  int32_t i = c.v == vmin ? c.i : kNoIndex;
  i = dpp_min_i<0xB1, 0xF>(i);
  i = dpp_min_i<0x4E, 0xF>(i);
  i = dpp_min_i<0x141, 0xF>(i);
  i = dpp_min_i<0x140, 0xF>(i);
  if (!ROWS16) {
    i = dpp_min_i<0x142, 0xA>(i);
    i = dpp_min_i<0x143, 0xC>(i);
  }
  Cand r;
  r.i = __builtin_amdgcn_readlane(i, kLast);
  const uint64_t hit = __ballot(c.i == r.i && c.v == vmin);
  const int lane = hit ? (int)__builtin_ctzll(hit) : 0;
  r.v = readlane_d(c.v, lane);
  r.aux = readlane_d(c.aux, lane);
  r.flags = 0;
  if (__ballot(c.flags & kFlagNonFinite)) r.flags |= kFlagNonFinite;
  if (__ballot(c.flags & kFlagNegativeB)) r.flags |= kFlagNegativeB;
  return r;
}

// Elements per thread and batch in the flat walks over the tableau: their
// loads are all issued before the first one is used.
constexpr int kWgBatch = 4;

// Position (row, column) of a flat tableau index, advanced by the group size
// with a carry, so that the walks need no division per element.
struct WgCursor {
  int32_t i, j;
  __device__ void step(int32_t di, int32_t dj, int32_t W) {
    i += di;
    j += dj;
    if (j >= W) {
      j -= W;
      ++i;
    }
  }
};

// Per pivot: (1) every wave reduces the pricing offers its threads made on
// the objective row into its partial; (2) after a barrier, wave 0 combines
// the partials into the entering column k (Step 2), gathers column k into
// pcol and runs the ratio test (Step 3), and publishes the pivot (or the
// status) in the control block; (3) after a barrier, the group divides row
// l by the pivot (Step 4); (4) after a barrier, every thread eliminates
// column k from its share of the other rows (Step 5) and prices its share
// of the updated objective row for the next pivot.  Three workgroup
// barriers per pivot; the decisions take one wave and no cross-wave
// reduction.
template <class Grp>
__device__ void lds_solve(const SolveArgs& a, unsigned char* smem) {
  constexpr int NT = Grp::kThreads;
  constexpr int U = kWgBatch;
  const int32_t m = (int32_t)a.m, n = (int32_t)a.n, ncols = n + m, W = ncols + 1, R = m + 1;
  const int32_t ldw = (int32_t)wg_ldw(W), hw = ldw / 2, RL = R * ldw, RH = R * hw;
  const WgLayout L = wg_layout(m, n);
  double* T = reinterpret_cast<double*>(smem + L.off_T);
  double* pcol = reinterpret_cast<double*>(smem + L.off_pcol);
  int32_t* basis = reinterpret_cast<int32_t*>(smem + L.off_basis);
  Cand* part = reinterpret_cast<Cand*>(smem + L.off_scratch);
  WgCtrl* ctrl = reinterpret_cast<WgCtrl*>(smem + L.off_ctrl);
  const int tid = Grp::rank(), lane = tid & (kWave - 1), wave = tid / kWave;
  constexpr int nw = NT / kWave;
  // Flat walks: thread tid takes elements tid, tid + NT, ... of the row-major
  // R x ldw tableau (Step 1), or pairs of columns tid, tid + NT, ... of the
  // R x ldw/2 pairs (Step 5).
  const int32_t di = NT / ldw, dj = NT % ldw, pdi = NT / hw, pdj = NT % hw;
  const WgCursor first{tid / ldw, tid % ldw}, pfirst{tid / hw, tid % hw};
  const int32_t full_batches = RH / (U * NT), tail_slots = (RH - full_batches * U * NT + NT - 1) / NT;
  double* Tm = T + (size_t)m * ldw;

  // Step 1: Table 1 layout, RHS in column W-1, objective row last; or (T0)
  // a given basic tableau of that layout, its right-hand side unchecked.
  // With it, the pricing offers of the initial objective row.
  Cand pc = cand_none();
  {
    const double* dummy = a.T0 ? a.T0 : a.b;
    WgCursor cur = first;
    for (int32_t e0 = tid; e0 < RL; e0 += U * NT) {
      // Every lane loads (from the first entry of T0, else of b, where the
      // entry is a constant, the pad or past the end), so that the batch's
      // loads are issued back to back.  T0 comes without b.
      double v[U], k[U];
      bool ld[U];
      int32_t ri[U], cj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t e = e0 + u * NT, i = cur.i, j = cur.j;
        ri[u] = i;
        cj[u] = j;
        cur.step(di, dj, ldw);
        const double* src = dummy;
        ld[u] = e < RL && j < W;
        k[u] = 0.0;
        if (a.T0) src = a.T0 + (int64_t)i * W + j;
        else if (i < m) {
          if (j < n) src = a.A + (int64_t)i * n + j;
          else if (j == ncols) src = a.b + i;
          else ld[u] = false, k[u] = (j - n == i) ? 1.0 : 0.0;
        } else if (j < n) src = a.c + j;
        else ld[u] = false;
        if (!ld[u]) src = dummy;
        v[u] = *src;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t e = e0 + u * NT;
        if (e >= RL) continue;
        double x = ld[u] ? v[u] : k[u];
        if (!a.T0 && ri[u] == m && cj[u] < n) x = -x;
        if (!is_finite(x)) pc.flags |= kFlagNonFinite;
        if (!a.T0 && ri[u] < m && cj[u] == ncols && x < 0.0) pc.flags |= kFlagNegativeB;
        if (ri[u] == m && cj[u] < ncols && !__builtin_isnan(x)) cand_offer(pc, x, cj[u], 0.0);
        T[e] = x;
      }
    }
  }
  for (int32_t i = tid; i < m; i += NT) basis[i] = a.T0 ? a.basis0[i] : n + i;

  int32_t status = -1;
  int64_t iter = 0;
  for (;;) {
    // (1) This wave's partial of the pricing offers (and of the flags).
    if (__ballot(pc.i != kNoIndex || pc.flags != 0)) pc = wave_argmin<false>(pc);
    if (lane == 0) part[wave] = pc;
    Grp::sync();

    // (2) Wave 0: Steps 2 and 3, then the control block.
    if (wave == 0) {
      WgCtrl cb{0.0, 0, 0, -1, 0};
      Cand q = lane < nw ? part[lane] : cand_none();
      q = wave_argmin<true>(q);
      if (iter == 0 && (q.flags & kFlagNegativeB) && !(q.flags & kFlagNonFinite)) cb.status = kInfeasibleStart;
      else if (q.flags & kFlagNonFinite) cb.status = kNumerical;
      else if (q.v >= -a.eps_d) cb.status = kOptimal;
      else if (iter == a.max_iter) cb.status = kIterLimit;
      if (cb.status < 0) {
        const int32_t k = q.i;
        Cand rc = cand_none();
        for (int32_t i0 = lane; i0 < R; i0 += U * kWave) {
          double aik[U], rhs[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int32_t i = min(i0 + u * kWave, m);
            aik[u] = T[(size_t)i * ldw + k];
            rhs[u] = T[(size_t)i * ldw + W - 1];
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int32_t i = i0 + u * kWave;
            if (i >= R) continue;
            pcol[i] = aik[u];
            if (i < m) {
              if (!is_finite(aik[u]) || !is_finite(rhs[u])) rc.flags |= kFlagNonFinite;
              if (aik[u] > a.eps_p) cand_offer(rc, rhs[u] / aik[u], i, aik[u]);
            }
          }
        }
        rc = wave_argmin<false>(rc);
        if (rc.flags & kFlagNonFinite) cb.status = kNumerical;
        else if (rc.i == kNoIndex) cb.status = kUnbounded;
        else cb = WgCtrl{rc.aux, k, rc.i, -1, 0};
      }
      if (lane == 0) {
        *ctrl = cb;
        if (cb.status < 0) {
          basis[cb.l] = cb.k;
          if (iter < a.trace_cap && a.trace) {
            a.trace[2 * iter] = cb.k;
            a.trace[2 * iter + 1] = cb.l;
          }
        }
      }
    }
    Grp::sync();
    const WgCtrl cb = *ctrl;
    status = __builtin_amdgcn_readfirstlane(cb.status);
    if (status >= 0) break;
    const int32_t l = __builtin_amdgcn_readfirstlane(cb.l);
    const double p = __builtin_bit_cast(double, uniform_u64(__builtin_bit_cast(uint64_t, cb.p)));

    // (3) Step 4: divide the pivot row by the pivot.
    double* Tl = T + (size_t)l * ldw;
    for (int32_t j = tid; j < W; j += NT) Tl[j] = Tl[j] / p;
    Grp::sync();

    // (4) Step 5: eliminate column k from every other row (objective row
    // too), and price this thread's share of the updated objective row.
    pc = cand_none();
    const dbl2* Tl2 = reinterpret_cast<const dbl2*>(Tl);
    dbl2* T2 = reinterpret_cast<dbl2*>(T);
    WgCursor cur = pfirst;
    // One batch of UB slots (pairs p0, p0 + NT, ...), all loads issued
    // first.  TAIL: some slots may lie past the end (they load a valid pair
    // and store nothing); otherwise every slot is in range.
    auto batch = [&](int32_t p0, auto ub, auto tail) {
      constexpr int UB = decltype(ub)::value;
      constexpr bool TAIL = decltype(tail)::value;
      dbl2 t[UB], r[UB];
      double f[UB];
      int32_t ri[UB], cj[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        ri[u] = cur.i;
        cj[u] = cur.j;
        cur.step(pdi, pdj, hw);
        t[u] = T2[TAIL ? min(p0 + u * NT, RH - 1) : p0 + u * NT];
        r[u] = Tl2[cj[u]];
        f[u] = pcol[TAIL ? min(ri[u], m) : ri[u]];
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        dbl2 v;
        v.x = __builtin_fma(-f[u], r[u].x, t[u].x);
        v.y = __builtin_fma(-f[u], r[u].y, t[u].y);
        if ((TAIL && p0 + u * NT >= RH) || ri[u] == l) continue;
        T2[p0 + u * NT] = v;
        if (ri[u] == m) {
          const int32_t j = 2 * cj[u];
          if (j < ncols) {
            if (!is_finite(v.x)) pc.flags |= kFlagNonFinite;
            if (!__builtin_isnan(v.x)) cand_offer(pc, v.x, j, 0.0);
          }
          if (j + 1 < ncols) {
            if (!is_finite(v.y)) pc.flags |= kFlagNonFinite;
            if (!__builtin_isnan(v.y)) cand_offer(pc, v.y, j + 1, 0.0);
          }
        }
      }
    };
    using no_tail = std::integral_constant<bool, false>;
    using is_tail = std::integral_constant<bool, true>;
    // Full batches (every thread's U slots in range), then one batch of as
    // many slots as the rest needs, so that no thread walks a batch of
    // empty slots.
    int32_t p0 = tid;
    for (int32_t bb = full_batches; bb > 0; --bb, p0 += U * NT) batch(p0, std::integral_constant<int, U>(), no_tail());
    static_assert(U == 4, "the tail batch covers 1 to 4 slots");
    switch (tail_slots) {
      case 1: batch(p0, std::integral_constant<int, 1>(), is_tail()); break;
      case 2: batch(p0, std::integral_constant<int, 2>(), is_tail()); break;
      case 3: batch(p0, std::integral_constant<int, 3>(), is_tail()); break;
      case 4: batch(p0, std::integral_constant<int, 4>(), is_tail()); break;
      default: break;
    }
    ++iter;
  }

  // Read-out: x from the basic rows' RHS, objective value, duals.
  const int32_t nx = a.x_count > 0 ? (int32_t)a.x_count : n;
  for (int32_t j = tid; j < nx; j += NT) a.x[j] = 0.0;
  Grp::order_global();
  for (int32_t i = tid; i < m; i += NT) {
    const int32_t bv = basis[i];
    if (bv < nx) a.x[bv] = T[(size_t)i * ldw + W - 1];
    if (a.y) a.y[i] = Tm[n + i];
    if (a.basis_out) a.basis_out[i] = bv;
  }
  if (a.tableau_out) {
    WgCursor cur = first;  // over R x ldw; the pad column is not written out
    for (int32_t e = tid; e < RL; e += NT) {
      if (cur.j < W) a.tableau_out[(int64_t)cur.i * W + cur.j] = T[e];
      cur.step(di, dj, ldw);
    }
  }
  if (tid == 0) {
    *a.obj = Tm[W - 1];
    *a.status = status;
    if (a.iterations) *a.iterations = iter;
  }
}

template <int NT>
__device__ void wg_solve(const SolveArgs& a, unsigned char* smem) {
  lds_solve<BlockGroup<NT>>(a, smem);
}


}  // namespace lpd
