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

__device__ __forceinline__ Cand wave_reduce(Cand c) {
#pragma unroll
  for (int m = kWave / 2; m > 0; m >>= 1) {
    Cand o;
    o.v = shfl_xor_d(c.v, m);
    o.aux = shfl_xor_d(c.aux, m);
    o.i = __shfl_xor(c.i, m, kWave);
    o.flags = __shfl_xor(c.flags, m, kWave);
    c = cand_merge(c, o);
  }
  return c;
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
    if (lane >= nw) d.flags = 0;
    d = wave_reduce(d);
    if (lane == 0) scratch[nw] = d;
  }
  __syncthreads();
  return scratch[nw];
}

}  // namespace lpd
