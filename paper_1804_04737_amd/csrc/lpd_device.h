// Device-side building blocks shared by the lpdense kernels (gfx950, wave64).
//
// Arithmetic contract of the pivot (Coutinho et al., Section 2, Steps 2-5):
//  * FP64, round to nearest even, no fast-math, denormals kept;
//  * the pivot row is divided by the pivot with IEEE division (never a
//    reciprocal multiply);
//  * every other element is updated with exactly one fused multiply-add,
//    fma(-f_i, r_j, T[i,j]), and no other operation is contracted (the
//    library is built with -ffp-contract=off and calls __builtin_fma);
//  * arg-minima are lexicographic on (value, index), which is associative and
//    commutative, so any reduction tree picks the same winner; NaN values are
//    never candidates (they are flagged instead).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpd {

constexpr int kWave = 64;
constexpr int32_t kNoIndex = 0x7fffffff;

// Status codes written to the device status output (mirror of lpd_status).
enum : int32_t { kOptimal = 0, kUnbounded = 1, kIterLimit = 2, kInfeasibleStart = 3, kNumerical = 4,
                 kDeviceTimeout = 5 };

// Flag bits carried by partial results.
enum : int32_t { kFlagNonFinite = 1, kFlagNegativeB = 2, kFlagTimeout = 4 };

typedef double dbl2 __attribute__((ext_vector_type(2)));

// (value, index) strictly better than (v2, i2) in lexicographic order.
__device__ __forceinline__ bool lex_less(double v1, int32_t i1, double v2, int32_t i2) {
  return v1 < v2 || (v1 == v2 && i1 < i2);
}

__device__ __forceinline__ bool is_finite(double v) { return __builtin_isfinite(v); }

// Candidate record of an arg-min: value, index, an extra payload carried with
// the winner (the pivot element for the ratio test) and OR-ed flags.
struct Cand {
  double v;
  double aux;
  int32_t i;
  int32_t flags;
};

__device__ __forceinline__ Cand cand_none() { return Cand{__builtin_inf(), 0.0, kNoIndex, 0}; }

__device__ __forceinline__ void cand_offer(Cand& c, double v, int32_t i, double aux) {
  if (lex_less(v, i, c.v, c.i)) {
    c.v = v;
    c.i = i;
    c.aux = aux;
  }
}

__device__ __forceinline__ Cand cand_merge(const Cand& a, const Cand& b) {
  Cand r = lex_less(b.v, b.i, a.v, a.i) ? b : a;
  r.flags = a.flags | b.flags;
  return r;
}

__device__ __forceinline__ double shfl_xor_d(double v, int m) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __shfl_xor(p.x, m, kWave);
  p.y = __shfl_xor(p.y, m, kWave);
  return __builtin_bit_cast(double, p);
}

// ---- wave / workgroup arg-min ------------------------------------------------
// Cross-lane moves use DPP (data-parallel primitives of the VALU) instead of
// LDS permutes: quad permutations, row mirrors and the row broadcasts of the
// gfx9 family carry (value, index) towards lane 63 in six steps.

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(x, x, CTRL, ROW_MASK, 0xF, false);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void dpp_step(double& v, int32_t& i) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = dpp_i<CTRL, ROW_MASK>(p.x);
  p.y = dpp_i<CTRL, ROW_MASK>(p.y);
  const double ov = __builtin_bit_cast(double, p);
  const int32_t oi = dpp_i<CTRL, ROW_MASK>(i);
  if (lex_less(ov, oi, v, i)) {
    v = ov;
    i = oi;
  }
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_readlane(p.x, lane);
  p.y = __builtin_amdgcn_readlane(p.y, lane);
  return __builtin_bit_cast(double, p);
}

// Wave-wide lexicographic arg-min; all lanes must be active.  Every lane gets
// the result (the payload `aux` of the winning lane, flags OR-ed).
__device__ __forceinline__ Cand wave_reduce(Cand c) {
  double v = c.v;
  int32_t i = c.i;
  dpp_step<0xB1, 0xF>(v, i);   // quad_perm [1,0,3,2]
  dpp_step<0x4E, 0xF>(v, i);   // quad_perm [2,3,0,1]
  dpp_step<0x141, 0xF>(v, i);  // row_half_mirror
  dpp_step<0x140, 0xF>(v, i);  // row_mirror
  dpp_step<0x142, 0xA>(v, i);  // row_bcast:15 into rows 1 and 3
  dpp_step<0x143, 0xC>(v, i);  // row_bcast:31 into rows 2 and 3
  Cand r;
  r.v = readlane_d(v, 63);
  r.i = __builtin_amdgcn_readlane(i, 63);
  // Payload of the winner: the lowest lane holding exactly (r.v, r.i).
  const uint64_t hit = __ballot(c.i == r.i && c.v == r.v);
  const int lane = hit ? (int)__builtin_ctzll(hit) : 0;
  r.aux = readlane_d(c.aux, lane);
  r.flags = 0;
  if (__ballot(c.flags & kFlagNonFinite)) r.flags |= kFlagNonFinite;
  if (__ballot(c.flags & kFlagNegativeB)) r.flags |= kFlagNegativeB;
  if (__ballot(c.flags & kFlagTimeout)) r.flags |= kFlagTimeout;
  return r;
}

// Block-wide arg-min; every thread gets the result.  `scratch` holds at least
// blockDim.x / 64 + 1 entries of LDS.  Contains two __syncthreads().
__device__ __forceinline__ Cand block_reduce(Cand c, Cand* scratch) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
  c = wave_reduce(c);
  if (lane == 0) scratch[w] = c;
  __syncthreads();
  if (w == 0) {
    Cand d = lane < nw ? scratch[lane] : cand_none();
    d = wave_reduce(d);
    if (lane == 0) scratch[nw] = d;
  }
  __syncthreads();
  // The result is the same in every lane: make that explicit (scalar registers).
  Cand r = scratch[nw];
  r.v = __builtin_bit_cast(double, uniform_u64(__builtin_bit_cast(uint64_t, r.v)));
  r.aux = __builtin_bit_cast(double, uniform_u64(__builtin_bit_cast(uint64_t, r.aux)));
  r.i = __builtin_amdgcn_readfirstlane(r.i);
  r.flags = __builtin_amdgcn_readfirstlane(r.flags);
  return r;
}

}  // namespace lpd
