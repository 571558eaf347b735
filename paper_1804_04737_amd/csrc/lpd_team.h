// Team-parameterised dense-tableau solve (gfx950): the persistent-grid
// algorithm run by a team of co-resident workgroups.  One LP on the whole GPU
// is a team of every workgroup (lpd_grid.hip); a batch runs many teams, each
// on its own LP (lpd_batch.hip).
//
// The whole simplex loop of Coutinho et al. (Section 2, Steps 1-5, iterated
// as in Section 3) runs on the device with one team-wide synchronisation per
// pivot:
//
//   P_t  (every workgroup, redundantly)  read the current pivot row l_t and
//        the objective row; divide the pivot row by the pivot (Step 4) into
//        LDS; update the objective row (Step 5 for row m) and price it
//        (Step 2 of the next pivot) -> k_{t+1}, g_{t+1}.  Each workgroup
//        publishes one slice of the new objective row and pivot row.
//   Q_t  (all workgroups, flat grid-stride over constraint rows x 16-byte
//        vectors)  T[i,:] <- fma(-f_i, r, T[i,:]) for i != l_t (Step 5),
//        streamed once with 128-bit loads (non-temporal, or temporal on
//        tableaux the memory-side cache holds) and non-temporal stores.  The
//        thread that meets element (i, k_{t+1}) forms the new entering-column
//        entry and right-hand side of row i and appends them to an LDS list;
//        after the sweep the workgroup forms the ratios (Step 3 of the next
//        pivot) and their lexicographic minimum.
//   R_t  reduction barrier: every workgroup publishes its ratio candidate,
//        waits for all others and reduces them -> l_{t+1}.
//
// Layout in HBM: constraint rows 0..m-1 of the tableau, row-major, stride
// `ld` (multiple of 32 doubles); the objective row, the right-hand side and
// the entering column live in separate double-buffered vectors so that every
// workgroup can read the previous pivot's values while the new ones are
// written.  The row that was pivot row at t-1 is not rewritten during Q_{t-1}
// (others are still reading it in P_{t-1}); its current content is the
// normalised pivot row kept in `pr`, and Q_t writes it back.
#pragma once

#include "lpd_device.h"
#include "lpd_kernels.h"

namespace lpd {

// A team of co-resident workgroups solving one LP together.
struct Team {
  int rank;            // this workgroup's index in the team
  int size;            // workgroups in the team
  BarrierSlot* slots;  // 2 * size reduction-barrier slots (epoch parity x rank)
  uint32_t* epoch;     // barrier epoch; grows across every solve the team runs
};

constexpr int kCandScratch = 32;  // LDS entries for block reductions (>= 1024/64 + 1)
constexpr uint64_t kWatchdogTicks = 1000000000ull;  // 10 s of the 100 MHz real-time clock
constexpr int kTicks = 8;         // phase_ticks entries per pivot
constexpr int kCapMax = 1024;     // LDS capture-list entries (entering-column elements per workgroup)
constexpr size_t kScratchBytes = kCandScratch * sizeof(Cand);
constexpr size_t kCapEntryBytes = 8 + 8 + 4;  // new column entry, new RHS, row
constexpr int kChunkSteps = 2;                 // dynamic sweep chunk: 2 x NT vectors
constexpr int kChunkStepsPaired = 3;           // ... with two pivots per sweep
constexpr int kChunkStepsTL = 4;               // ... with one pivot per sweep and temporal loads
constexpr int kPairCountWord = 64;             // ticket region word counting arrivals at the pair's barrier
constexpr int64_t kStaticSteps = 16;           // static grid steps before the dynamic part
constexpr int64_t kDynMinSteps = 48;           // sweeps shorter than this are all static
constexpr int64_t kStaticStepsPairedTL = 8;    // the same for two pivots per sweep with
constexpr int64_t kDynMinStepsPairedTL = 16;   // temporal loads (ld_tab)

// Tableau workspaces are always device global memory.  Saying so lets the
// compiler use global (not flat) loads and stores even where the pointer was
// itself loaded from memory (batch descriptors).
typedef __attribute__((address_space(1))) dbl2 gdbl2;
__device__ __forceinline__ void st_stream(dbl2* p, dbl2 v) { __builtin_nontemporal_store(v, (gdbl2*)p); }
// Tableau loads of the sweep: non-temporal, or (TL) plain loads.  Plain loads
// keep a tableau of up to about the memory-side cache's 256 MiB resident in
// it from one sweep to the next; on an in-place 128-bit RMW stream they ran
// at 6.9 TB/s against 6.4-6.6 TB/s non-temporal from 128 to 288 MB, and
// below the non-temporal ones from 320 MB up.
template <bool TL>
__device__ __forceinline__ dbl2 ld_tab(const dbl2* p) {
  if constexpr (TL) return *(const gdbl2*)p;
  else return __builtin_nontemporal_load((const gdbl2*)p);
}

// Plain loads and stores of workspace vectors, through global pointers.
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ double gld(const double* p) { return *(const gdouble*)p; }
__device__ __forceinline__ void gst(double* p, double v) { *(gdouble*)p = v; }
__device__ __forceinline__ dbl2 gld2(const dbl2* p) { return *(const gdbl2*)p; }
__device__ __forceinline__ void gst2(dbl2* p, dbl2 v) { *(gdbl2*)p = v; }

// Gives a wave-uniform value a scalar register of its own.  Fields of the
// kernel's argument block are otherwise loaded as wide register tuples, and
// the register allocator spills and reloads such a tuple as a whole, also
// inside the sweep where one field of it is needed.  (Where the value was
// loaded into vector registers, e.g. from a batch descriptor, the first
// lane's copy is taken: the callers pass values that every lane agrees on.)
template <class T>
__device__ __forceinline__ T own_sreg(T v) {
  static_assert(sizeof(T) % 4 == 0, "32-bit words only");
  uint32_t wd[sizeof(T) / 4];
  __builtin_memcpy(wd, &v, sizeof(T));
  for (unsigned q = 0; q < sizeof(T) / 4; ++q) wd[q] = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)wd[q]);
  __builtin_memcpy(&v, wd, sizeof(T));
  asm("" : "+s"(v));
  return v;
}

// Bound of a barrier wait in ticks of the 100 MHz real-time clock, from a
// solve's watchdog option: 0 the default, > 0 that many ticks, < 0 none at
// all (every wait gives up at once: a test of the timeout path).
__device__ __forceinline__ int64_t wait_budget(int64_t watchdog) {
  return watchdog == 0 ? (int64_t)kWatchdogTicks : watchdog;
}

// Grid-wide lexicographic arg-min that doubles as the barrier.
// `c` is this workgroup's reduced candidate (identical in all its threads).
// Every workgroup returns the same global result.  A wait that exceeds
// `budget` ticks (wait_budget; < 0: every wait) gives up and flags
// kFlagTimeout instead of hanging.
__device__ Cand grid_reduce(const Team& tm, Cand c, uint32_t epoch, Cand* scratch,
                            bool diag = false, uint64_t* tk = nullptr, int64_t budget = kWatchdogTicks) {
  const int nb = tm.size;
  if (nb == 1) {
    // A one-workgroup team shares nothing across CUs: a workgroup barrier is
    // enough for its own global-memory traffic.
    __syncthreads();
    return c;
  }
  BarrierSlot* slots = tm.slots;
  // All of this wave's memory operations (tableau stores included) complete
  // before the workgroup barrier; thread 0's agent-scope release then makes
  // them visible to the other XCDs' caches before the slot is published.
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  BarrierSlot* buf = slots + (size_t)(epoch & 1u) * nb;
  if (threadIdx.x == 0) {
    BarrierSlot* s = buf + tm.rank;
    s->v = c.v;
    s->aux = c.aux;
    s->i = c.i;
    s->flags = c.flags;
    if (diag) s->t_arrive = __builtin_amdgcn_s_memrealtime();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (diag) {
      // Diagnostics: time after the release, made visible by a second release.
      s->t_pub = __builtin_amdgcn_s_memrealtime();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __hip_atomic_store(&s->epoch, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // Wave 0 alone polls every slot, acquires and reduces the candidates; the
  // other waves wait at one workgroup barrier for the result.  (Measured
  // against four polling waves and a block reduction: 1024 x 8192 3-4 %
  // faster, 4096^2 0.5-1.6 %, 8192^2 unchanged.)
  Cand* const result = scratch + (kCandScratch - 1);  // not used by block_reduce
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    Cand got = cand_none();
    if (budget < 0) got.flags |= kFlagTimeout;  // no wait at all
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (int s = lane; s < nb && budget >= 0; s += kWave) {
      // Epochs only grow; a slot written for a later epoch also counts as
      // arrived (its payload lives in the other parity buffer).
      while ((int32_t)(__hip_atomic_load(&buf[s].epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - epoch) < 0) {
        __builtin_amdgcn_s_sleep(1);
        // Watchdog: a barrier that has not completed after `budget` ticks of
        // the 100 MHz real-time counter reports a timeout instead of waiting
        // forever.
        if (__builtin_amdgcn_s_memrealtime() - t0 > (uint64_t)budget) {
          got.flags |= kFlagTimeout;
          break;
        }
      }
    }
    // One agent-scope acquire per workgroup, after every slot has been seen
    // and before any payload is read: it invalidates this CU's L1 and the
    // XCD's L2, which the other waves share; they read nothing written by
    // other workgroups before the workgroup barrier below.
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (tk && lane == 0) tk[5] = __builtin_amdgcn_s_memrealtime();
    uint64_t ta = 0, tp = 0;
    for (int s = lane; s < nb; s += kWave) {
      Cand o;
      o.v = buf[s].v;
      o.aux = buf[s].aux;
      o.i = buf[s].i;
      o.flags = buf[s].flags;
      got = cand_merge(got, o);
      if (tk) {
        ta = max(ta, buf[s].t_arrive);
        tp = max(tp, buf[s].t_pub);
      }
    }
    if (tk) {
      // Diagnostics only: latest arrival and latest publication over all workgroups.
      for (int msk = kWave / 2; msk > 0; msk >>= 1) {
        ta = max(ta, __builtin_bit_cast(uint64_t, shfl_xor_d(__builtin_bit_cast(double, ta), msk)));
        tp = max(tp, __builtin_bit_cast(uint64_t, shfl_xor_d(__builtin_bit_cast(double, tp), msk)));
      }
      if (lane == 0 && ta) {
        __hip_atomic_fetch_max(tk + 3, ta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_max(tk + 4, tp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    got = wave_reduce(got);
    if (lane == 0) *result = got;
  }
  __syncthreads();
  // The result is the same in every lane: make that explicit (scalar registers).
  Cand r = *result;
  r.v = __builtin_bit_cast(double, uniform_u64(__builtin_bit_cast(uint64_t, r.v)));
  r.aux = __builtin_bit_cast(double, uniform_u64(__builtin_bit_cast(uint64_t, r.aux)));
  r.i = __builtin_amdgcn_readfirstlane(r.i);
  r.flags = __builtin_amdgcn_readfirstlane(r.flags);
  if (tk && threadIdx.x == 0) tk[6] = __builtin_amdgcn_s_memrealtime();
  return r;
}

// Offer objective-row entry j (value v) to the pricing arg-min.
__device__ __forceinline__ void price_offer(Cand& c, double v, int64_t j, int64_t ncols) {
  if (j < ncols) {
    if (!is_finite(v)) c.flags |= kFlagNonFinite;
    if (!__builtin_isnan(v)) cand_offer(c, v, (int32_t)j, 0.0);
  }
}

// Condensed tableau: stored column `col` holds variable `label`; ties are
// broken by the label (as on the full tableau), the column is the payload.
__device__ __forceinline__ void price_offer_cd(Cand& c, double v, int32_t label, int32_t col, int32_t sc) {
  if (col < sc) {
    if (!is_finite(v)) c.flags |= kFlagNonFinite;
    if (!__builtin_isnan(v)) cand_offer(c, v, label, (double)col);
  }
}

// Ratio-test contribution of row i with new entering-column value `a` and
// new right-hand side `r` (Step 3 of the next pivot).
__device__ __forceinline__ void ratio_offer(Cand& c, double a, double r, int32_t i, double eps_p) {
  if (!is_finite(a) || !is_finite(r)) c.flags |= kFlagNonFinite;
  if (a > eps_p) cand_offer(c, r / a, i, a);
}

// MAP selects how (workgroup, thread) maps onto the flat grid-stride walk:
//   0: workgroup b owns NT consecutive vectors per sweep step;
//   1: each workgroup is split into NT/256 sub-groups of 256 threads that act
//      as workgroups b, b + nb, b + 2 nb, ... (4 KiB pieces per sweep step).
// CD selects the condensed tableau: T holds only the n columns of the
// nonbasic variables (lab[c]: variable of stored column c).  A pivot on
// (l, k) turns k's column into the leaving variable's: its entries are what
// the full tableau computes for the unit column e_l, fma(-f_i, RN(1/p), +0)
// and RN(1/p) in row l, so every value equals the full tableau's bit for bit.
// basis[l] changes one pivot late (all workgroups read basis[] while the
// leader would otherwise write it): the row of the previous pivot holds kprev.
// DYN = false compiles the dynamic sweep out (for callers whose teams are
// always one workgroup, which never use it).
// PN = true is for pivot rows longer than the LDS holds (w.lds_vecs < vw):
// the sweep runs over column panels of w.lds_vecs vectors, panel after
// panel, and a workgroup forms the panel of the normalised pivot row it
// needs from the pivot row itself (same division as in P, so the same bits).
// FU = true (with PN, either tableau, not resumable) does two pivots per sweep
// where it can: the P phase also prices the objective row after the first
// pivot, forms the entering column of the second after the first update and
// its ratio test, and the second normalised row; the sweep then applies both
// updates to each element, fma(-a'_i, r2, fma(-f_i, r1, T)), the roundings of
// two sweeps.  A pair takes one pivot where the second would not be made
// (a status after the first, or the iteration cap).  Each workgroup publishes
// a slice of the first normalised row and of the second multiplier column;
// a counter barrier after the column gather makes them visible before any
// sweep starts (the sweep also rewrites row l and column k1, which P reads).
// TL selects the sweep's tableau loads (ld_tab).
template <int NT, int MAP, bool CD = false, bool DYN = true, bool PN = false, bool FU = false, bool TL = false>
__device__ void team_solve(const SolveArgs& a, const GridWork& w, const Team& tm, unsigned char* smem) {
  static_assert(!FU || PN, "two pivots per sweep: column panels");
  Cand* scratch = reinterpret_cast<Cand*>(smem);
  dbl2* prow = reinterpret_cast<dbl2*>(smem + kScratchBytes);
  // Capture list: elements of the entering column met during the sweep.
  unsigned char* capb = smem + kScratchBytes + (size_t)w.lds_vecs * 16;
  double* cap_a = reinterpret_cast<double*>(capb);
  double* cap_r = cap_a + w.cap_cap;
  int32_t* cap_i = reinterpret_cast<int32_t*>(cap_r + w.cap_cap);
  int32_t* cap_count = cap_i + w.cap_cap;
  uint32_t* s_tk = reinterpret_cast<uint32_t*>(cap_count + 1);  // 2 ticket broadcast slots
  if (threadIdx.x == 0) *cap_count = 0;

  const int nb = tm.size, tid = threadIdx.x;
  const bool leader = tm.rank == 0;
  const int32_t m = own_sreg((int32_t)a.m), n = own_sreg((int32_t)a.n), ncols = n + m;
  const int32_t sc = CD ? n : ncols;  // stored (priced) columns
  const int64_t ld = own_sreg(w.ld);
  const int32_t vw = own_sreg((int32_t)w.vw);
  const int32_t cap_cap = own_sreg(w.cap_cap);
  double* const Tm = own_sreg(w.T);  // constraint rows of the tableau
  const int64_t G = (int64_t)nb * NT;
  const int64_t gid = MAP == 0 ? (int64_t)tm.rank * NT + tid
                               : ((int64_t)(tid / 256) * nb + tm.rank) * 256 + (tid & 255);
  // Flat grid-stride walk over (row, vector): start and step in (row, vec) form.
  const int32_t i_start = (int32_t)(gid / vw), v_start = (int32_t)(gid % vw);
  const int32_t step_q = (int32_t)(G / vw), step_r = (int32_t)(G % vw);
  // Slice of the objective / pivot rows this workgroup publishes each pivot.
  const int32_t pub_v0 = (int32_t)((int64_t)vw * tm.rank / nb);
  const int32_t pub_v1 = (int32_t)((int64_t)vw * (tm.rank + 1) / nb);
  uint32_t& epoch = *tm.epoch;
  // Dynamic split of each sweep: the first kStaticSteps grid steps (flat
  // index below e_static) follow the static grid-stride walk, which covers
  // the latency of the first tickets; the rest, in chunks of kChunkSteps x
  // NT vectors, go to whichever workgroup of the team asks next (atomic
  // ticket counters), so that workgroups that run slower leave work to
  // faster ones up to the end of the sweep.  Measured at 8192 x 8192 on 256
  // workgroups: with one counter, 3-step chunks beat 2 (that counter's
  // atomics become the limit) and 4..8 (coarser balance); two counters make
  // 2-step chunks the best.
  const int64_t e_total = (int64_t)m * vw;
  const int64_t steps_total = (e_total + G - 1) / G;
  // The dynamic part costs a few microseconds per pivot (ticket broadcasts,
  // the last chunk's latency); it only pays off on long sweeps.  Two pivots
  // per sweep on a cache-resident tableau gain from it from 16 steps on
  // (2048 x 8192: 44.4 -> 41.5 ms); one pivot per sweep there does not.
  constexpr bool kPairTL = FU && TL;
  const bool dyn = DYN && nb > 1 && steps_total >= (kPairTL ? kDynMinStepsPairedTL : kDynMinSteps);
  const int64_t e_static = dyn ? min((int64_t)(kPairTL ? kStaticStepsPairedTL : kStaticSteps) * G, e_total) : e_total;
  // Two pivots per sweep do twice the work per element: longer chunks there;
  // and a cache-resident tableau streams faster: longer chunks there too
  // (4 steps: 3072 x 6144 108.9 -> 106.8 ms, the 1024-LP batch -0.8 %; 8
  // steps lost 6 % at 4096^2).
  constexpr int kCS = FU ? kChunkStepsPaired : TL ? kChunkStepsTL : kChunkSteps;
  const int64_t chunk = (int64_t)kCS * NT;
  // Panels (PN): as few as the LDS allows, of nearly equal width in whole
  // 128-byte lines (npan - 1 panels of pvw vectors and a last one of
  // pw_last; unequal panels leave one ticket counter's workgroups changing
  // panels at the end of the sweep); a chunk never straddles two panels.
  const int32_t pvw_max = PN ? (FU ? w.lds_vecs / 2 : w.lds_vecs) : vw;  // FU: two rows per panel
  const int32_t npan = PN ? (vw + pvw_max - 1) / pvw_max : 1;
  const int32_t pvw = PN ? min(pvw_max, (int32_t)round_up((vw + npan - 1) / npan, 8)) : vw;
  const int32_t pw_last = vw - (npan - 1) * pvw;
  const int64_t cpp = ((int64_t)m * pvw + chunk - 1) / chunk;  // chunks per full panel
  const uint32_t n_chunks =
      PN ? (uint32_t)((int64_t)(npan - 1) * cpp + ((int64_t)m * pw_last + chunk - 1) / chunk)
         : (dyn ? (uint32_t)((e_total - e_static + chunk - 1) / chunk) : 0u);
  const int64_t n_static = e_static > gid ? (e_static - gid - 1) / G + 1 : 0;
  const int32_t dq_q = (int32_t)(NT / vw), dq_r = (int32_t)(NT % vw);

  int32_t status = -1;
  int64_t iter = 0;
  int32_t lprev = -1;  // pivot row of the last pivot done (-1: none)
  int32_t fpar = 0;    // parity of the current objective / rhs buffers
  int32_t k = -1, l = -1;
  int32_t kc = -1, kprev = -1;  // stored column of k; k of the previous pivot
  double g = 0.0, p = 1.0;
  // A resumable solve that was suspended between pivots picks up where it
  // stopped: the tableau and vectors are in the workspace, the scalars here.
  const bool resume = a.state != nullptr && a.state->phase == 1;
  if (resume) {
    k = a.state->k;
    l = a.state->l;
    lprev = a.state->lprev;
    g = a.state->g;
    p = a.state->p;
    iter = a.state->iter;
    kc = a.state->kc;
    kprev = a.state->kprev;
    fpar = (int32_t)(iter & 1);
  } else {
    // ---------------- Step 1: initial tableau ----------------
    // Table 1 from A, b, c, or (T0) a given basic tableau copied as it is
    // (condensed: its nonbasic columns), with its right-hand side unchecked.
    int32_t flags = 0;
    const double* const T0 = a.T0;
    const int64_t W0 = (int64_t)ncols + 1;  // row length of T0
    {
      int32_t i = i_start, v = v_start;
      while (i < m) {
        const int32_t j0 = 2 * v, j1 = 2 * v + 1;
        dbl2 t;
        if (T0) {
          const double* Ti = T0 + (int64_t)i * W0;
          if (CD) {
            t.x = j0 < n ? Ti[a.lab0[j0]] : 0.0;
            t.y = j1 < n ? Ti[a.lab0[j1]] : 0.0;
          } else {
            t.x = j0 < ncols ? Ti[j0] : 0.0;
            t.y = j1 < ncols ? Ti[j1] : 0.0;
          }
        } else {
          const double* Ai = a.A + (int64_t)i * n;
          t.x = j0 < n ? Ai[j0] : (!CD && j0 == n + i ? 1.0 : 0.0);
          t.y = j1 < n ? Ai[j1] : (!CD && j1 == n + i ? 1.0 : 0.0);
        }
        if (!is_finite(t.x) || !is_finite(t.y)) flags |= kFlagNonFinite;
        st_stream(reinterpret_cast<dbl2*>(w.T + (int64_t)i * ld) + v, t);
        v += step_r;
        i += step_q;
        if (v >= vw) { v -= vw; ++i; }
      }
    }
    for (int64_t v = gid; v < vw; v += G) {
      const int64_t j0 = 2 * v, j1 = 2 * v + 1;
      dbl2 o;
      if (T0) {
        const double* Tobj = T0 + (int64_t)m * W0;
        o.x = j0 < sc ? Tobj[CD ? a.lab0[j0] : j0] : 0.0;
        o.y = j1 < sc ? Tobj[CD ? a.lab0[j1] : j1] : 0.0;
      } else {
        o.x = j0 < n ? -a.c[j0] : 0.0;
        o.y = j1 < n ? -a.c[j1] : 0.0;
      }
      if (!is_finite(o.x) || !is_finite(o.y)) flags |= kFlagNonFinite;
      reinterpret_cast<dbl2*>(w.obj[0])[v] = o;
    }
    for (int64_t i = gid; i <= m; i += G) {
      double bi = 0.0;
      if (T0) {
        bi = T0[i * W0 + ncols];
        if (!is_finite(bi)) flags |= kFlagNonFinite;
        if (i < m) w.basis[i] = a.basis0[i];
      } else if (i < m) {
        bi = a.b[i];
        if (!is_finite(bi)) flags |= kFlagNonFinite;
        if (bi < 0.0) flags |= kFlagNegativeB;
        w.basis[i] = (int32_t)(n + i);
      }
      w.rhs[0][i] = bi;
    }
    for (int64_t j = gid; j < ncols; j += G) {
      if (T0) {
        w.pos[j] = a.pos0[j];
        if (CD) {
          w.col_of[j] = a.colof0[j];
          if (j < n) w.lab[j] = a.lab0[j];
        }
      } else {
        w.pos[j] = j < n ? -1 : (int32_t)(j - n);
        if (CD) {
          w.col_of[j] = j < n ? (int32_t)j : -1;
          if (j < n) w.lab[j] = (int32_t)j;
        }
      }
    }

    // Ticket counters reset (counter h to its first chunk, h) whatever the
    // team size: a resumable solve may be continued by a larger team in a
    // later launch.
    if (leader && tid == 0) {
      for (int h = 0; h < kTicketCounters; ++h) {
        __hip_atomic_store(w.tickets + h * kTicketStride, (uint32_t)h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(w.tickets + h * kTicketStride + 32, (uint32_t)h, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
      if (FU) __hip_atomic_store(w.tickets + kPairCountWord, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    {
      Cand f0 = cand_none();
      f0.flags = flags;
      f0 = block_reduce(f0, scratch);
      const Cand gf = grid_reduce(tm, f0, ++epoch, scratch, false, nullptr, wait_budget(a.watchdog));
      if (gf.flags & kFlagTimeout) status = kDeviceTimeout;
      else if (gf.flags & kFlagNonFinite) status = kNumerical;
      else if (gf.flags & kFlagNegativeB) status = kInfeasibleStart;
    }

    // ---------------- Step 2 on the initial objective row ----------------
    if (status < 0) {
      Cand pc = cand_none();
      const dbl2* o = reinterpret_cast<const dbl2*>(w.obj[0]);
      for (int32_t v = tid; v < vw; v += NT) {
        const dbl2 ov = o[v];
        if constexpr (CD) {
          // Ties go to the lowest variable label (stored column c holds
          // variable c in Table 1).
          const int2 lb = *reinterpret_cast<const int2*>(w.lab + 2 * v);
          price_offer_cd(pc, ov.x, lb.x, 2 * v, sc);
          price_offer_cd(pc, ov.y, lb.y, 2 * v + 1, sc);
        } else {
          price_offer(pc, ov.x, 2 * (int64_t)v, sc);
          price_offer(pc, ov.y, 2 * (int64_t)v + 1, sc);
        }
      }
      pc = block_reduce(pc, scratch);
      if (pc.flags & kFlagNonFinite) status = kNumerical;
      else if (pc.v >= -a.eps_d) status = kOptimal;
      else if (a.max_iter == 0) status = kIterLimit;
      k = pc.i;
      kc = CD ? (int32_t)pc.aux : pc.i;
      g = pc.v;
    }
    // ---------------- Step 3 on the initial tableau ----------------
    if (status < 0) {
      Cand rc = cand_none();
      for (int64_t i = gid; i < m; i += G) {
        const double aik = w.T[i * ld + kc];
        const double r = w.rhs[0][i];
        w.pcol[0][i] = aik;
        ratio_offer(rc, aik, r, (int32_t)i, a.eps_p);
      }
      rc = block_reduce(rc, scratch);
      const Cand gr = grid_reduce(tm, rc, ++epoch, scratch, false, nullptr, wait_budget(a.watchdog));
      if (gr.flags & kFlagTimeout) status = kDeviceTimeout;
      else if (gr.flags & kFlagNonFinite) status = kNumerical;
      else if (gr.i == kNoIndex) status = kUnbounded;
      l = gr.i;
      p = gr.aux;
    }
  }

  // ---------------- pivot loop ----------------
  const bool ticks = leader && a.phase_ticks != nullptr;
  int64_t done_here = 0;  // pivots done by this call
  int64_t rnd = iter;     // sweeps done (FU: buffers alternate per sweep, not per pivot)
  while (status < 0) {
    const int64_t rp = FU ? rnd : iter;  // parity of this sweep's buffers
    if (a.state && a.pivot_budget >= 0 && done_here == a.pivot_budget) break;  // suspend
    ++done_here;
    uint64_t* tk = (ticks && iter < a.phase_cap) ? a.phase_ticks + kTicks * iter : nullptr;
    if (tk && tid == 0) {
      tk[0] = __builtin_amdgcn_s_memrealtime();
      // Entries 3 and 4 are maxima over every workgroup (atomic max after
      // the barrier has seen this workgroup's arrival): start them at zero.
      tk[3] = 0;
      tk[4] = 0;
    }
    // The previous pivot's ticket counters are idle until the next pivot
    // (every workgroup passed the last barrier after its final ticket): reset
    // them.
    if (dyn && leader && tid == 0)
      for (int h = 0; h < kTicketCounters; ++h)
        __hip_atomic_store(w.tickets + h * kTicketStride + 32 * ((rp + 1) & 1), (uint32_t)h, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    const int cur = (int)(rp & 1), nxt = cur ^ 1;
    double* obj_nxt = w.obj[nxt];
    const double* rhs_cur = own_sreg(w.rhs[cur]);
    double* rhs_nxt = own_sreg(w.rhs[nxt]);
    const double* pcol_cur = own_sreg(w.pcol[cur]);
    double* pcol_nxt = own_sreg(w.pcol[nxt]);
    double* pr_cur = w.pr[cur];
    const dbl2* pr_prev = own_sreg(reinterpret_cast<const dbl2*>(w.pr[nxt]));

    // ---- P_t: Step 4 (pivot row / pivot, into LDS), Step 5 on the objective
    // row, Step 2 for the next pivot.  Row l's current content is the
    // normalised row of the previous pivot if l was pivot row then.
    const dbl2* rowl = (l == lprev) ? pr_prev : reinterpret_cast<const dbl2*>(w.T + (int64_t)l * ld);
    Cand pc = cand_none();
    const double prhs = gld(rhs_cur + l) / p;
    // Condensed: the variable leaving the basis (row l), which takes over
    // stored column kc.
    // (Two pivots per sweep write the basis after the pair's barrier, so it
    // is current here; one pivot per sweep writes it one pivot late.)
    const int32_t vleave = CD ? ((!FU && l == lprev) ? kprev : w.basis[l]) : 0;
    // Objective row after this pivot, entry v; also stages r_v in LDS.
    auto p_update = [&](int32_t v, dbl2 t, dbl2 o) -> dbl2 {
      dbl2 r, on;
      if constexpr (CD) {
        const bool x_k = 2 * v == kc, y_k = 2 * v + 1 == kc;
        r.x = x_k ? 1.0 / p : t.x / p;
        r.y = y_k ? 1.0 / p : t.y / p;
        on.x = __builtin_fma(-g, r.x, x_k ? 0.0 : o.x);
        on.y = __builtin_fma(-g, r.y, y_k ? 0.0 : o.y);
      } else {
        r.x = t.x / p;
        r.y = t.y / p;
        on.x = __builtin_fma(-g, r.x, o.x);
        on.y = __builtin_fma(-g, r.y, o.y);
      }
      if constexpr (!PN) prow[v] = r;
      // Each workgroup publishes one slice of the new rows (all copies agree).
      if (v >= pub_v0 && v < pub_v1) {
        gst2(reinterpret_cast<dbl2*>(obj_nxt) + v, on);
        gst2(reinterpret_cast<dbl2*>(pr_cur) + v, r);
      }
      if constexpr (CD) {
        const int2 lb = *reinterpret_cast<const int2*>(w.lab + 2 * v);
        price_offer_cd(pc, on.x, 2 * v == kc ? vleave : lb.x, 2 * v, sc);
        price_offer_cd(pc, on.y, 2 * v + 1 == kc ? vleave : lb.y, 2 * v + 1, sc);
      } else {
        price_offer(pc, on.x, 2 * (int64_t)v, ncols);
        price_offer(pc, on.y, 2 * (int64_t)v + 1, ncols);
      }
      return on;
    };
    const dbl2* obj_cur = reinterpret_cast<const dbl2*>(w.obj[cur]);
    // Two pivots per sweep (FU): the pair's second pivot (k1, l1), its
    // pivot p1, normalised right-hand side prhs1, the first update's
    // multiplier of row l1 (fl1) and that row before the pair (rowl1).
    // Condensed: k1's stored column kc1 and the variable leaving row l1.
    bool two = false;
    int32_t l1 = -1, k1 = -1, kc1 = -1, vleave1 = -1;
    double p1 = 1.0, prhs1 = 0.0, fl1 = 0.0;
    const dbl2* rowl1 = rowl;
    dbl2* const prt = FU ? own_sreg(reinterpret_cast<dbl2*>(w.prt)) : nullptr;
    double* const pap = FU ? own_sreg(w.pap) : nullptr;
    // FU: this workgroup's own copy of r_t for its later passes, in LDS when
    // the row fits (until the sweep loads a panel over it), else in its
    // private region.
    const bool rt_lds = vw <= w.lds_vecs;
    dbl2* const priv_rt = FU ? reinterpret_cast<dbl2*>(w.priv + (int64_t)tm.rank * w.priv_stride) : nullptr;
    auto keep_rt = [&](int32_t v, dbl2 r) {
      if (rt_lds) prow[v] = r;
      else gst2(priv_rt + v, r);
    };
    auto kept_rt = [&](int32_t v) -> dbl2 { return rt_lds ? prow[v] : gld2(priv_rt + v); };
    // FU with one panel: both rows of the pair fit side by side in LDS, r_t
    // at [0, vw) from pass 1 and r1 at [pvw, pvw + vw) from pass 3 (the same
    // bits as the panel load), so the sweep starts with its panel loaded.
    const bool one_panel = FU && npan == 1 && rt_lds;
    if constexpr (FU) {
      // Pass 1: first pivot's normalised row (kept, and this workgroup's
      // slice published) and the objective row after it, priced for k1.
      Cand pc1 = cand_none();
      for (int32_t v0 = tid; v0 < vw; v0 += 4 * NT) {
        dbl2 t[4], o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int32_t v = v0 + q * NT;
          if (v < vw) {
            t[q] = gld2(rowl + v);
            o[q] = gld2(obj_cur + v);
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int32_t v = v0 + q * NT;
          if (v < vw) {
            // Condensed: stored column kc becomes the leaving variable's
            // (unit column e_l before the pivot), as in one pivot's P.
            const bool x_k = CD && 2 * v == kc, y_k = CD && 2 * v + 1 == kc;
            dbl2 r, on;
            r.x = x_k ? 1.0 / p : t[q].x / p;
            r.y = y_k ? 1.0 / p : t[q].y / p;
            on.x = __builtin_fma(-g, r.x, x_k ? 0.0 : o[q].x);
            on.y = __builtin_fma(-g, r.y, y_k ? 0.0 : o[q].y);
            keep_rt(v, r);
            if (v >= pub_v0 && v < pub_v1) gst2(prt + v, r);
            if constexpr (CD) {
              const int2 lb = *reinterpret_cast<const int2*>(w.lab + 2 * v);
              price_offer_cd(pc1, on.x, x_k ? vleave : lb.x, 2 * v, sc);
              price_offer_cd(pc1, on.y, y_k ? vleave : lb.y, 2 * v + 1, sc);
            } else {
              price_offer(pc1, on.x, 2 * (int64_t)v, ncols);
              price_offer(pc1, on.y, 2 * (int64_t)v + 1, ncols);
            }
          }
        }
      }
      pc1 = block_reduce(pc1, scratch);  // also orders the kept row's writes
      k1 = pc1.i;
      kc1 = CD ? (int32_t)pc1.aux : pc1.i;
      const double g1 = pc1.v;
      // (Condensed: the leaving variable's reduced cost after the first
      // pivot, -g/p, is positive, so kc1 != kc whenever k1 is taken.)
      two = !(pc1.flags & kFlagNonFinite) && !(g1 >= -a.eps_d) && iter + 2 <= a.max_iter && (!CD || kc1 != kc);
      if (two) {
        // Entering column k1 and right-hand side after the first pivot, and
        // the second pivot's ratio test (Step 3), for every row.
        const dbl2 rk = kept_rt(kc1 >> 1);
        const double rt_k1 = (kc1 & 1) ? rk.y : rk.x;
        // This workgroup publishes rows [pa0, pa1) of the column.
        const int32_t pa0 = (int32_t)((int64_t)m * tm.rank / nb), pa1 = (int32_t)((int64_t)m * (tm.rank + 1) / nb);
        const double eps_p = a.eps_p;
        Cand rc1 = cand_none();
        for (int32_t i = tid; i < m; i += NT) {
          double ap, rhp;
          if (i == l) {
            ap = rt_k1;
            rhp = prhs;
          } else {
            const double f = gld(pcol_cur + i);
            const double* rowi = (i == lprev) ? reinterpret_cast<const double*>(pr_prev) : Tm + (int64_t)i * ld;
            ap = __builtin_fma(-f, rt_k1, gld(rowi + kc1));
            rhp = __builtin_fma(-f, prhs, gld(rhs_cur + i));
          }
          if (i >= pa0 && i < pa1) gst(pap + i, ap);
          ratio_offer(rc1, ap, rhp, i, eps_p);
        }
        rc1 = block_reduce(rc1, scratch);
        if (rc1.i == kNoIndex || (rc1.flags & kFlagNonFinite)) {
          two = false;
        } else {
          l1 = rc1.i;
          p1 = rc1.aux;
          fl1 = l1 == l ? 0.0 : gld(pcol_cur + l1);
          const double rhp1 = l1 == l ? prhs : __builtin_fma(-fl1, prhs, gld(rhs_cur + l1));
          prhs1 = rhp1 / p1;
          rowl1 = (l1 == lprev) ? pr_prev : reinterpret_cast<const dbl2*>(Tm + (int64_t)l1 * ld);
          if constexpr (CD) vleave1 = l1 == l ? k : w.basis[l1];
        }
      }
      // Arrival at the pair's publication barrier: this workgroup's slices of
      // r_t and of the column after the first pivot are written back, and
      // its reads of row l and column k1, which the sweep rewrites, have
      // returned.  No sweep starts before every workgroup has arrived; the
      // third pass below overlaps the wait.
      if (nb > 1) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tid == 0) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_fetch_add(w.tickets + kPairCountWord, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      if (two) {
        // Pass 3: the second normalised row (row l1 after the first update,
        // divided by p1) and the objective row after both pivots, priced for
        // the next pair; this workgroup's slices of both are published.
        const double g1c = g1;
        Cand pc2 = cand_none();
        for (int32_t v = tid; v < vw; v += NT) {
          const dbl2 rt = kept_rt(v);
          const dbl2 o = gld2(obj_cur + v);
          // Condensed: columns kc and kc1 hold the leaving variables' unit
          // columns before their pivots.
          const bool x_k = CD && 2 * v == kc, y_k = CD && 2 * v + 1 == kc;
          const bool x_k1 = CD && 2 * v == kc1, y_k1 = CD && 2 * v + 1 == kc1;
          dbl2 on, x, r1, on2;
          on.x = __builtin_fma(-g, rt.x, x_k ? 0.0 : o.x);
          on.y = __builtin_fma(-g, rt.y, y_k ? 0.0 : o.y);
          if (l1 == l) {
            x = rt;
          } else {
            const dbl2 t1 = gld2(rowl1 + v);
            x.x = __builtin_fma(-fl1, rt.x, x_k ? 0.0 : t1.x);
            x.y = __builtin_fma(-fl1, rt.y, y_k ? 0.0 : t1.y);
          }
          r1.x = x_k1 ? 1.0 / p1 : x.x / p1;
          r1.y = y_k1 ? 1.0 / p1 : x.y / p1;
          on2.x = __builtin_fma(-g1c, r1.x, x_k1 ? 0.0 : on.x);
          on2.y = __builtin_fma(-g1c, r1.y, y_k1 ? 0.0 : on.y);
          if (v >= pub_v0 && v < pub_v1) {
            gst2(reinterpret_cast<dbl2*>(obj_nxt) + v, on2);
            gst2(reinterpret_cast<dbl2*>(pr_cur) + v, r1);
          }
          if (one_panel) prow[pvw + v] = r1;  // the sweep's only panel, second row
          if constexpr (CD) {
            const int2 lb = *reinterpret_cast<const int2*>(w.lab + 2 * v);
            price_offer_cd(pc2, on2.x, x_k1 ? vleave1 : (x_k ? vleave : lb.x), 2 * v, sc);
            price_offer_cd(pc2, on2.y, y_k1 ? vleave1 : (y_k ? vleave : lb.y), 2 * v + 1, sc);
          } else {
            price_offer(pc2, on2.x, 2 * (int64_t)v, ncols);
            price_offer(pc2, on2.y, 2 * (int64_t)v + 1, ncols);
          }
        }
        if (leader && tid == 0) {
          const double z1 = __builtin_fma(-g, prhs, gld(rhs_cur + m));
          gst(rhs_nxt + m, __builtin_fma(-g1c, prhs1, z1));
          if constexpr (!CD) {  // condensed: after the pair's barrier
            const int32_t leaving = w.basis[l];
            w.pos[leaving] = -1;
            w.pos[k] = l;
            w.basis[l] = k;
            const int32_t leaving1 = w.basis[l1];
            w.pos[leaving1] = -1;
            w.pos[k1] = l1;
            w.basis[l1] = k1;
          }
          if (a.trace) {
            if (iter < a.trace_cap) {
              a.trace[2 * iter] = k;
              a.trace[2 * iter + 1] = l;
            }
            if (iter + 1 < a.trace_cap) {
              a.trace[2 * iter + 2] = k1;
              a.trace[2 * iter + 3] = l1;
            }
          }
        }
        pc = block_reduce(pc2, scratch);
      } else {
        // One pivot this sweep: publish this workgroup's slices of the
        // objective row after it and of its normalised row.
        for (int32_t v = pub_v0 + tid; v < pub_v1; v += NT) {
          const dbl2 rt = kept_rt(v);
          const dbl2 o = gld2(obj_cur + v);
          const bool x_k = CD && 2 * v == kc, y_k = CD && 2 * v + 1 == kc;
          dbl2 on;
          on.x = __builtin_fma(-g, rt.x, x_k ? 0.0 : o.x);
          on.y = __builtin_fma(-g, rt.y, y_k ? 0.0 : o.y);
          gst2(reinterpret_cast<dbl2*>(obj_nxt) + v, on);
          gst2(reinterpret_cast<dbl2*>(pr_cur) + v, rt);
        }
        if (leader && tid == 0) {
          gst(rhs_nxt + m, __builtin_fma(-g, prhs, gld(rhs_cur + m)));
          if constexpr (!CD) {  // condensed: after the pair's barrier
            const int32_t leaving = w.basis[l];
            w.pos[leaving] = -1;
            w.pos[k] = l;
            w.basis[l] = k;
          }
          if (iter < a.trace_cap && a.trace) {
            a.trace[2 * iter] = k;
            a.trace[2 * iter + 1] = l;
          }
        }
        pc = pc1;
      }
    } else {
      for (int32_t v0 = tid; v0 < vw; v0 += 4 * NT) {
        dbl2 t[4], o[4];
  #pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int32_t v = v0 + q * NT;
          if (v < vw) {
            t[q] = gld2(rowl + v);
            o[q] = gld2(obj_cur + v);
          }
        }
  #pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int32_t v = v0 + q * NT;
          if (v < vw) (void)p_update(v, t[q], o[q]);
        }
      }
      if (leader && tid == 0) {
        gst(rhs_nxt + m, __builtin_fma(-g, prhs, gld(rhs_cur + m)));
        if constexpr (CD) {
          if (lprev >= 0) w.basis[lprev] = kprev;  // the previous pivot's change, one pivot late
          w.pos[vleave] = -1;
          w.pos[k] = l;
          w.lab[kc] = vleave;
          w.col_of[vleave] = kc;
          w.col_of[k] = -1;
        } else {
          const int32_t leaving = w.basis[l];
          w.pos[leaving] = -1;
          w.pos[k] = l;
          w.basis[l] = k;
        }
        if (iter < a.trace_cap && a.trace) {
          a.trace[2 * iter] = k;
          a.trace[2 * iter + 1] = l;
        }
      }
      pc = block_reduce(pc, scratch);  // also orders the LDS writes of prow
    }
    if (tk && tid == 0) tk[1] = __builtin_amdgcn_s_memrealtime();
    const int32_t kn = pc.i;                                  // entering variable of the next pivot
    const int32_t kcn = CD ? (int32_t)pc.aux : pc.i;          // ... and its stored column
    const double gn = pc.v;
    const int32_t pflags = pc.flags;

    // ---- Q_t: Step 5 on every constraint row, fused with Step 3 for k_{t+1}.
    Cand rc = cand_none();
    if constexpr (FU) {
      // Wait until every workgroup has arrived (after its column gather),
      // then acquire their slices; a bounded wait like the barrier's.
      if (nb > 1) {
        if (tid == 0) {
          const uint32_t target = (uint32_t)nb * (uint32_t)(rnd + 1);
          const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
          const int64_t budget = wait_budget(a.watchdog);
          if (budget < 0) rc.flags |= kFlagTimeout;
          while (budget >= 0 &&
                 (int32_t)(__hip_atomic_load(w.tickets + kPairCountWord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                           target) < 0) {
            __builtin_amdgcn_s_sleep(1);
            if (__builtin_amdgcn_s_memrealtime() - t0 > (uint64_t)budget) {
              rc.flags |= kFlagTimeout;
              break;
            }
          }
          // One acquire per workgroup: it invalidates the XCD's L2 and this
          // CU's L1, which the other waves share after the barrier.  (An
          // acquire in every wave costs the sweep ~25 us at 8192 x 8192.)
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
      }
      if (tk && tid == 0) tk[7] = __builtin_amdgcn_s_memrealtime();
      if constexpr (CD) {
        // Condensed: basis, positions and column labels of the sweep's
        // pivots.  Every workgroup has read the basis and priced with the
        // labels of this round (all arrived), and the third pass overrides
        // the labels of columns kc and kc1.
        if (leader && tid == 0) {
          w.pos[vleave] = -1;
          w.pos[k] = l;
          w.basis[l] = k;
          w.lab[kc] = vleave;
          w.col_of[vleave] = kc;
          w.col_of[k] = -1;
          if (two) {
            w.pos[vleave1] = -1;
            w.pos[k1] = l1;
            w.basis[l1] = k1;
            w.lab[kc1] = vleave1;
            w.col_of[vleave1] = kc1;
            w.col_of[k1] = -1;
          }
        }
      }
    }
    {
      const int32_t kv = kcn >> 1, kh = kcn & 1;
      // Condensed: stored column kc becomes the leaving variable's column,
      // whose full-tableau entries before the pivot are 0 off row l.
      const int32_t kcv = kc >> 1, kch = kc & 1;
      const int32_t kc1v = (FU && CD) ? kc1 >> 1 : -1, kc1h = kc1 & 1;  // FU, condensed: the second pivot's column
      const double eps_p = own_sreg(a.eps_p);
      const int64_t ldv = ld / 2;  // row stride in 16-byte vectors
      // One element (i, v) of the dynamic part: the same work as one step of
      // the static walk below.
      int32_t pv0 = 0;  // first vector of the panel in LDS (PN)
      // FU: the row multipliers of the pair (f_i, a'_i) are kept from this
      // thread's previous element while the row stays the same.
      int32_t ci = -1;
      double cf = 0.0, cap2 = 0.0;
      auto element = [&](int32_t i, int32_t v) {
        const dbl2* rowp = reinterpret_cast<const dbl2*>(Tm) + (int64_t)i * ldv;
        double f;
        if constexpr (FU) {
          if (i != ci) {
            ci = i;
            cf = gld(pcol_cur + i);
            if (two) cap2 = gld(pap + i);
          }
          f = cf;
        } else {
          f = gld(pcol_cur + i);
        }
        const bool cap = (v == kv);
        double rh = 0.0;
        if (cap) rh = gld(rhs_cur + i);
        const dbl2* src = (i == lprev) ? pr_prev : rowp;
        dbl2 t;
        if (i != l) t = ld_tab<TL>(src + v);
        if (CD && v == kcv) {
          if (kch) t.y = 0.0;
          else t.x = 0.0;
        }
        const dbl2 r = prow[PN ? v - pv0 : v];
        dbl2 nv;
        if (i == l) {
          nv = r;
        } else {
          nv.x = __builtin_fma(-f, r.x, t.x);
          nv.y = __builtin_fma(-f, r.y, t.y);
        }
        double ap = 0.0;  // FU: the second pivot's multiplier of row i
        if constexpr (FU) {
          if (two) {
            ap = cap2;
            const dbl2 r2 = prow[pvw + v - pv0];
            if (CD && v == kc1v) {  // the second leaving variable's unit column
              if (kc1h) nv.y = 0.0;
              else nv.x = 0.0;
            }
            if (i == l1) {
              nv = r2;
            } else {
              nv.x = __builtin_fma(-ap, r2.x, nv.x);
              nv.y = __builtin_fma(-ap, r2.y, nv.y);
            }
          }
        }
        if (cap) {
          const double an = kh ? nv.y : nv.x;
          double rn = (i == l) ? prhs : __builtin_fma(-f, prhs, rh);
          if constexpr (FU) {
            if (two) rn = (i == l1) ? prhs1 : __builtin_fma(-ap, prhs1, rn);
          }
          gst(pcol_nxt + i, an);
          gst(rhs_nxt + i, rn);
          const int32_t slot = cap_cap ? atomicAdd(cap_count, 1) : 0;
          if (slot < cap_cap) {
            cap_a[slot] = an;
            cap_r[slot] = rn;
            cap_i[slot] = i;
          } else {
            ratio_offer(rc, an, rn, i, eps_p);
          }
        }
        // The pivot row of the sweep's last pivot is kept in pr_cur (written
        // back by the next sweep).
        if (i != (FU && two ? l1 : l)) st_stream(const_cast<dbl2*>(rowp) + v, nv);
      };
      // Ticket counters: counter h holds the next chunk it hands out and
      // steps by K (K = kTicketCounters): chunks h, h + K, h + 2K, ...  Each
      // counter has its own 4 KiB block, so one counter's atomics do not
      // bound the whole sweep.  A workgroup asks the first counter, from its
      // home counter on, that has not run dry for it.  Thread 0 keeps a queue
      // of two tickets: both are requested before the static walk, and a new
      // one after this thread's first element of each chunk.  Tickets are
      // used in the order they were requested; as one thread's requests to
      // one counter are ordered, a ticket past the end means every later
      // ticket of that counter is too.  (This pivot's counters were reset a
      // pivot ago.)
      uint32_t* ctr0 = w.tickets + 32 * (rp & 1);
      const int home = tm.rank & (kTicketCounters - 1);
      uint32_t dry = 0;  // bit h: counter h has run dry (thread 0)
      auto request = [&]() -> uint32_t {
        int h = home;
        for (int j = 0; j < kTicketCounters && ((dry >> h) & 1u); ++j) h = (h + 1) & (kTicketCounters - 1);
        return __hip_atomic_fetch_add(ctr0 + h * kTicketStride, (uint32_t)kTicketCounters, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
      };
      uint32_t tq0 = 0, tq1 = 0;  // ticket queue, oldest first (thread 0)
      if (dyn && tid == 0) {
        tq0 = request();
        tq1 = request();
      }
      if constexpr (PN) {
        // Panel-major sweep.  Chunk c: panel pp = c / cpp (the last panel
        // takes the rest), elements [lc * chunk, (lc + 1) * chunk) of the
        // panel's m x pw block in row-major order.  Chunks come from the
        // tickets on long sweeps, else in the static order rank, rank + nb, ...
        constexpr uint32_t kAllDry = (1u << kTicketCounters) - 1u;
        // First chunk of counter h's share: whole panels when the panels
        // divide evenly between the counters, else an even split.
        auto share_lo = [&](uint32_t h) -> uint32_t {
          if (h >= (uint32_t)kTicketCounters) return n_chunks;
          if (npan % kTicketCounters == 0) return (uint32_t)((int64_t)h * (npan / kTicketCounters) * cpp);
          const uint32_t per = (n_chunks + kTicketCounters - 1) / kTicketCounters;
          return min(n_chunks, h * per);
        };
        int32_t loaded = one_panel ? 0 : -1;  // (pv0 = 0)
        uint32_t jst = 0;
        for (int par = 0;; par ^= 1) {
          uint32_t c;
          if (dyn) {
            if (tid == 0) {
              uint32_t cn = n_chunks;
              while (dry != kAllDry) {
                const uint32_t t = tq0;
                tq0 = tq1;
                {
                  // Counter h hands out a contiguous share of the chunks
                  // (ticket j: chunk h * per + j), so the workgroups of
                  // different counters work in different panels and do
                  // not all change panels at once.
                  const uint32_t h = t % (uint32_t)kTicketCounters, j = t / (uint32_t)kTicketCounters;
                  const uint32_t lo = share_lo(h), hi = share_lo(h + 1);
                  if (lo + j < hi) {
                    cn = lo + j;
                    break;
                  }
                }
                dry |= 1u << (t % (uint32_t)kTicketCounters);
                if (dry != kAllDry) tq1 = request();
              }
              s_tk[par] = cn;
            }
            __syncthreads();
            c = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)s_tk[par]);
          } else {
            c = (uint32_t)tm.rank + jst * (uint32_t)nb;
            ++jst;
          }
          if (c >= n_chunks) break;
          const int32_t pp = (int64_t)c < (int64_t)(npan - 1) * cpp ? (int32_t)(c / cpp) : npan - 1;
          const int64_t lc = (int64_t)c - (int64_t)pp * cpp;
          const int32_t pw = pp < npan - 1 ? pvw : pw_last;
          if (pp != loaded) {
            // Normalised pivot row, vectors [pp * pvw, pp * pvw + pw), into
            // LDS.  Row l is read-only during the sweep (as in P).
            __syncthreads();
            pv0 = pp * pvw;
            for (int32_t u = tid; u < pw; u += NT) {
              const int32_t vq = pv0 + u;
              dbl2 r;
              if constexpr (FU) {
                // Both normalised rows of the pair (as in P: same bits); r_t
                // as the workgroups published it.  Row l1 is not rewritten
                // by this sweep.
                r = gld2(prt + vq);
                if (two) {
                  const bool x_k = CD && 2 * vq == kc, y_k = CD && 2 * vq + 1 == kc;
                  const bool x_k1 = CD && 2 * vq == kc1, y_k1 = CD && 2 * vq + 1 == kc1;
                  dbl2 x;
                  if (l1 == l) {
                    x = r;
                  } else {
                    const dbl2 t1 = gld2(rowl1 + vq);
                    x.x = __builtin_fma(-fl1, r.x, x_k ? 0.0 : t1.x);
                    x.y = __builtin_fma(-fl1, r.y, y_k ? 0.0 : t1.y);
                  }
                  dbl2 r1;
                  r1.x = x_k1 ? 1.0 / p1 : x.x / p1;
                  r1.y = y_k1 ? 1.0 / p1 : x.y / p1;
                  prow[pvw + u] = r1;
                }
              } else {
                const dbl2 tr = gld2(rowl + vq);
                if constexpr (CD) {
                  r.x = 2 * vq == kc ? 1.0 / p : tr.x / p;
                  r.y = 2 * vq + 1 == kc ? 1.0 / p : tr.y / p;
                } else {
                  r.x = tr.x / p;
                  r.y = tr.y / p;
                }
              }
              prow[u] = r;
            }
            __syncthreads();
            loaded = pp;
          }
          const int64_t e0 = lc * chunk + tid;
          int32_t ii = (int32_t)(e0 / pw), vv = (int32_t)(e0 % pw);
          const int32_t pq = NT / pw, pr = NT % pw;
          for (int qq = 0; qq < kCS; ++qq) {
            if (ii < m) element(ii, pv0 + vv);
            if (dyn && qq == 0 && tid == 0) tq1 = request();
            vv += pr;
            ii += pq;
            if (vv >= pw) {
              vv -= pw;
              ++ii;
            }
          }
        }
      } else {
        int32_t i = i_start, v = v_start;
        const dbl2* rowp = reinterpret_cast<const dbl2*>(Tm) + (int64_t)i * ldv;
        const int64_t row_step = (int64_t)step_q * ldv;
        for (int64_t q = 0; q < n_static; ++q) {
          const double f = gld(pcol_cur + i);
          const bool cap = (v == kv);
          double rh = 0.0;
          if (cap) rh = gld(rhs_cur + i);
          const dbl2* src = (i == lprev) ? pr_prev : rowp;
          dbl2 t;
          if (i != l) t = ld_tab<TL>(src + v);
          if (CD && v == kcv) {
            if (kch) t.y = 0.0;
            else t.x = 0.0;
          }
          const dbl2 r = prow[v];
          dbl2 nv;
          if (i == l) {
            nv = r;
          } else {
            nv.x = __builtin_fma(-f, r.x, t.x);
            nv.y = __builtin_fma(-f, r.y, t.y);
          }
          // The capture runs before this element's store is issued: waiting on
          // its operands must not also wait for the store to complete.
          if (cap) {
            // New entering-column entry and right-hand side of row i; the ratio
            // itself is formed after the sweep by the whole workgroup.
            const double an = kh ? nv.y : nv.x;
            const double rn = (i == l) ? prhs : __builtin_fma(-f, prhs, rh);
            gst(pcol_nxt + i, an);
            gst(rhs_nxt + i, rn);
            const int32_t slot = cap_cap ? atomicAdd(cap_count, 1) : 0;
            if (slot < cap_cap) {
              cap_a[slot] = an;
              cap_r[slot] = rn;
              cap_i[slot] = i;
            } else {
              ratio_offer(rc, an, rn, i, eps_p);
            }
          }
          if (i != l) st_stream(const_cast<dbl2*>(rowp) + v, nv);
          v += step_r;
          i += step_q;
          rowp += row_step;
          if (v >= vw) {
            v -= vw;
            ++i;
            rowp += ldv;
          }
        }
        if (dyn) {
          // Dynamic part of the sweep.  Chunk c covers flat elements
          // e_static + c * chunk + [0, chunk); thread tid takes every NT-th.
          // Thread 0 takes the oldest ticket and broadcasts it through one of
          // two LDS slots (the next write cannot overtake a slow reader).  A
          // ticket past the end marks its counter dry and is replaced, until a
          // valid one comes or every counter is dry: then the ticket still in
          // flight is past the end too.
          constexpr uint32_t kAllDry = (1u << kTicketCounters) - 1u;
          for (int par = 0;; par ^= 1) {
            if (tid == 0) {
              uint32_t c = n_chunks;
              while (dry != kAllDry) {
                const uint32_t t = tq0;
                tq0 = tq1;
                if (t < n_chunks) {
                  c = t;
                  break;
                }
                dry |= 1u << (t % (uint32_t)kTicketCounters);
                if (dry != kAllDry) tq1 = request();
              }
              s_tk[par] = c;
            }
            __syncthreads();
            const uint32_t c = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)s_tk[par]);
            if (c >= n_chunks) break;
            const int64_t e0 = e_static + (int64_t)c * chunk + tid;
            int32_t ii = (int32_t)(e0 / vw), vv = (int32_t)(e0 % vw);
            for (int qq = 0; qq < kCS; ++qq) {
              if (ii < m) element(ii, vv);
              if (qq == 0 && tid == 0) tq1 = request();
              vv += dq_r;
              ii += dq_q;
              if (vv >= vw) {
                vv -= vw;
                ++ii;
              }
            }
          }
        }
      }
      __syncthreads();
      const int32_t ncap = min(*cap_count, cap_cap);
      for (int32_t e = tid; e < ncap; e += NT) ratio_offer(rc, cap_a[e], cap_r[e], cap_i[e], eps_p);
    }
    rc = block_reduce(rc, scratch);
    if (tid == 0) *cap_count = 0;
    if (tk && tid == 0) tk[2] = __builtin_amdgcn_s_memrealtime();
    const Cand gr = grid_reduce(tm, rc, ++epoch, scratch, a.phase_ticks != nullptr, tk, wait_budget(a.watchdog));

    // ---- loop control (identical decision in every workgroup)
    if constexpr (FU) {
      iter += two ? 2 : 1;
      lprev = two ? l1 : l;
      ++rnd;
      fpar = (int)(rnd & 1);
    } else {
      ++iter;
      lprev = l;
      fpar = (int)(iter & 1);
    }
    kprev = k;
    if (gr.flags & kFlagTimeout) status = kDeviceTimeout;
    else if (pflags & kFlagNonFinite) status = kNumerical;
    else if (gn >= -a.eps_d) status = kOptimal;
    else if (iter == a.max_iter) status = kIterLimit;
    else if (gr.flags & kFlagNonFinite) status = kNumerical;
    else if (gr.i == kNoIndex) status = kUnbounded;
    k = kn;
    kc = kcn;
    g = gn;
    l = gr.i;
    p = gr.aux;
  }

  if (status < 0) {
    // Suspended: keep the scalars for the next call (all workgroups agree).
    if (leader && tid == 0)
      for (int h = 0; h < kTicketCounters; ++h)
        __hip_atomic_store(w.tickets + h * kTicketStride + 32 * ((iter + 1) & 1), (uint32_t)h, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    if (CD && leader && tid == 0 && lprev >= 0) w.basis[lprev] = kprev;
    if (leader && tid == 0) {
      a.state->phase = 1;
      a.state->kc = kc;
      a.state->kprev = kprev;
      a.state->k = k;
      a.state->l = l;
      a.state->lprev = lprev;
      a.state->g = g;
      a.state->p = p;
      a.state->iter = iter;
    }
    return;
  }
  if (a.state && leader && tid == 0) a.state->phase = 2;
  if (status == kDeviceTimeout) {
    // Some workgroup gave up waiting: the workspace may be incomplete (even
    // the index arrays of Step 1), so nothing is read back but the status.
    if (leader && tid == 0) *a.status = status;
    return;
  }

  // ---------------- solution read-out ----------------
  const double* rhs_f = w.rhs[fpar];
  const double* obj_f = w.obj[fpar];
  const double* pr_last = w.pr[fpar ^ 1];  // normalised row of the last pivot
  const int64_t nx = a.x_count > 0 ? a.x_count : n;
  for (int64_t j = gid; j < nx; j += G) {
    const int32_t r = w.pos[j];
    a.x[j] = r >= 0 ? rhs_f[r] : 0.0;
  }
  if (a.y)
    for (int64_t i = gid; i < m; i += G) {
      // A basic variable's objective-row entry is +0 in the full tableau.
      const int32_t col = CD ? w.col_of[n + i] : (int32_t)(n + i);
      a.y[i] = col >= 0 ? obj_f[col] : 0.0;
    }
  if (a.basis_out)
    for (int64_t i = gid; i < m; i += G) a.basis_out[i] = (CD && !FU && i == lprev) ? kprev : w.basis[i];
  if (a.tableau_out) {
    const int64_t W = (int64_t)ncols + 1;
    for (int64_t e = gid; e < (int64_t)(m + 1) * W; e += G) {
      const int64_t i = e / W, j = e - i * W;
      double val;
      const int32_t col = (!CD || j == ncols) ? (int32_t)j : w.col_of[j];
      if (j == ncols) val = rhs_f[i];
      else if (col < 0) val = (i == w.pos[j]) ? 1.0 : 0.0;  // basic: unit column
      else if (i == m) val = obj_f[col];
      else if (i == lprev) val = pr_last[col];
      else val = w.T[i * ld + col];
      a.tableau_out[e] = val;
    }
  }
  if (leader && tid == 0) {
    *a.obj = rhs_f[m];
    *a.status = status;
    if (a.iterations) *a.iterations = iter;
  }
}


}  // namespace lpd
