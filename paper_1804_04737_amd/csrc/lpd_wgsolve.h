// Solve of one small dense LP whose whole tableau fits in LDS, by one
// workgroup or by one wave.
//
// The (m+1) x (n+m+1) tableau of Table 1 (Coutinho et al., Section 2) is
// built in LDS and the group runs Steps 2-5 in a loop with group-level
// synchronisation only; the result leaves LDS once, at the end.  Same arithmetic
// contract as the grid path: IEEE division for the pivot row, one fma per
// eliminated element, lexicographic (value, index) arg-minima.
#pragma once

#include "lpd_device.h"
#include "lpd_kernels.h"

namespace lpd {

constexpr int kWgScratch = 1024 / kWave + 1;  // block-reduction scratch entries (any NT <= 1024)

struct WgLayout {
  size_t off_T, off_pcol, off_basis, off_scratch, total;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline WgLayout wg_layout(int64_t m, int64_t n) {
  const size_t R = (size_t)m + 1, W = (size_t)(n + m + 1);
  WgLayout L;
  L.off_T = 0;
  L.off_pcol = align16(R * W * 8);
  L.off_basis = L.off_pcol + align16(R * 8);
  L.off_scratch = L.off_basis + align16((size_t)m * 4);
  L.total = L.off_scratch + kWgScratch * sizeof(Cand);
  return L;
}

// Thread groups that can run the LDS solve: a whole workgroup of NT threads,
// or one wave on its own slice of the workgroup's LDS (several small LPs per
// workgroup, one per wave).
template <int NT>
struct BlockGroup {
  static constexpr int kThreads = NT;
  __device__ static int rank() { return threadIdx.x; }
  // LDS writes before, reads after.
  __device__ static void sync() { __syncthreads(); }
  // Arg-min over the group; also orders the LDS writes made before it.
  __device__ static Cand reduce(Cand c, Cand* scratch) { return block_reduce(c, scratch); }
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
  __device__ static Cand reduce(Cand c, Cand*) {
    sync();
    return wave_reduce(c);
  }
  __device__ static void order_global() {
    __builtin_amdgcn_s_waitcnt(0);
    sync();
  }
};

template <class Grp>
__device__ void lds_solve(const SolveArgs& a, unsigned char* smem) {
  constexpr int NT = Grp::kThreads;
  const int32_t m = (int32_t)a.m, n = (int32_t)a.n, ncols = n + m, W = ncols + 1, R = m + 1;
  const WgLayout L = wg_layout(m, n);
  double* T = reinterpret_cast<double*>(smem + L.off_T);
  double* pcol = reinterpret_cast<double*>(smem + L.off_pcol);
  int32_t* basis = reinterpret_cast<int32_t*>(smem + L.off_basis);
  Cand* scratch = reinterpret_cast<Cand*>(smem + L.off_scratch);
  const int tid = Grp::rank(), lane = tid & (kWave - 1), wave = tid / kWave, nw = NT / kWave;

  // Step 1: Table 1 layout, RHS in column W-1, objective row last; or (T0)
  // a given basic tableau of that layout, its right-hand side unchecked.
  int32_t flags = 0;
  for (int32_t i = wave; i < R; i += nw) {
    double* Ti = T + (size_t)i * W;
    for (int32_t j = lane; j < W; j += kWave) {
      double v;
      if (a.T0) {
        v = a.T0[(int64_t)i * W + j];
      } else if (i < m) {
        if (j < n) v = a.A[(int64_t)i * n + j];
        else if (j < ncols) v = (j - n == i) ? 1.0 : 0.0;
        else {
          v = a.b[i];
          if (v < 0.0) flags |= kFlagNegativeB;
        }
      } else {
        v = j < n ? -a.c[j] : 0.0;
      }
      if (!is_finite(v)) flags |= kFlagNonFinite;
      Ti[j] = v;
    }
  }
  for (int32_t i = tid; i < m; i += NT) basis[i] = a.T0 ? a.basis0[i] : n + i;
  Cand fc = cand_none();
  fc.flags = flags;
  fc = Grp::reduce(fc, scratch);

  int32_t status = -1;
  if (fc.flags & kFlagNonFinite) status = kNumerical;
  else if (fc.flags & kFlagNegativeB) status = kInfeasibleStart;

  int64_t iter = 0;
  double* Tm = T + (size_t)m * W;
  while (status < 0) {
    // Step 2: most negative reduced cost, lowest index on ties.
    Cand pc = cand_none();
    for (int32_t j = tid; j < ncols; j += NT) {
      const double v = Tm[j];
      if (!is_finite(v)) pc.flags |= kFlagNonFinite;
      if (!__builtin_isnan(v)) cand_offer(pc, v, j, 0.0);
    }
    pc = Grp::reduce(pc, scratch);
    if (pc.flags & kFlagNonFinite) { status = kNumerical; break; }
    if (pc.v >= -a.eps_d) { status = kOptimal; break; }
    if (iter == a.max_iter) { status = kIterLimit; break; }
    const int32_t k = pc.i;

    // Step 3: min ratio over rows with T[i,k] > eps_p, lowest row on ties.
    Cand rc = cand_none();
    for (int32_t i = tid; i < R; i += NT) {
      const double aik = T[(size_t)i * W + k];
      pcol[i] = aik;
      if (i < m) {
        const double r = T[(size_t)i * W + W - 1];
        if (!is_finite(aik) || !is_finite(r)) rc.flags |= kFlagNonFinite;
        if (aik > a.eps_p) cand_offer(rc, r / aik, i, aik);
      }
    }
    rc = Grp::reduce(rc, scratch);  // orders the pcol writes too
    if (rc.flags & kFlagNonFinite) { status = kNumerical; break; }
    if (rc.i == kNoIndex) { status = kUnbounded; break; }
    const int32_t l = rc.i;
    const double p = rc.aux;

    // Step 4: divide the pivot row by the pivot.
    double* Tl = T + (size_t)l * W;
    for (int32_t j = tid; j < W; j += NT) Tl[j] = Tl[j] / p;
    Grp::sync();

    // Step 5: eliminate column k from every other row (objective row too).
    for (int32_t i = wave; i < R; i += nw) {
      if (i == l) continue;
      double* Ti = T + (size_t)i * W;
      const double f = pcol[i];
      for (int32_t j = lane; j < W; j += kWave) Ti[j] = __builtin_fma(-f, Tl[j], Ti[j]);
    }
    if (tid == 0) {
      basis[l] = k;
      if (iter < a.trace_cap && a.trace) {
        a.trace[2 * iter] = k;
        a.trace[2 * iter + 1] = l;
      }
    }
    ++iter;
    Grp::sync();
  }

  // Read-out: x from the basic rows' RHS, objective value, duals.
  const int32_t nx = a.x_count > 0 ? (int32_t)a.x_count : n;
  for (int32_t j = tid; j < nx; j += NT) a.x[j] = 0.0;
  Grp::order_global();
  for (int32_t i = tid; i < m; i += NT) {
    const int32_t bv = basis[i];
    if (bv < nx) a.x[bv] = T[(size_t)i * W + W - 1];
    if (a.y) a.y[i] = Tm[n + i];
    if (a.basis_out) a.basis_out[i] = bv;
  }
  if (a.tableau_out)
    for (int32_t e = tid; e < R * W; e += NT) a.tableau_out[e] = T[e];
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
