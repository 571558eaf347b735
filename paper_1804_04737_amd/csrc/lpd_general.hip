// Two-phase solve of a general LP -- rows <=, = or >= with right-hand sides
// of any sign -- on the pivot kernels of lp_solve_dense_ex (Section 2 states
// the problem with equality rows; the paper's experiments start from the
// slack basis of <= rows with b >= 0, which phase I provides in general).
//
// Phase I LP, canonical form (max c1^T x1, A1 x1 <= b1, x1 >= 0, b1 >= 0):
//   row i scaled by sigma_i = +-1 so that its right-hand side is >= 0;
//   a row that then reads ">=" gets a surplus column (-1) and, like every
//   "=" row, an artificial variable as its (implicit) slack: the slack basis
//   is then feasible.  c1 = sum of the artificial rows of A1, so that
//   c1^T x1 = sum(b1 over artificial rows) - sum(artificials): the LP is
//   feasible iff phase I reaches that sum.
// Phase II LP, canonical form again, whose slack basis is phase I's final
// basis: structural columns = phase I's nonbasic non-artificial variables,
// taken from phase I's final tableau; costs c_N - A_N^T c_B; an artificial
// still basic (at level zero) gets a mirrored row -row <= 0 so that it stays
// zero.  Every reduction below is one sequential sum in a fixed order, so
// the results are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "lpdense.h"

namespace lpd {
namespace {

constexpr int kTB = 256;

__global__ void build_phase1_kernel(int64_t m, int64_t n, int64_t n1, const double* A, const double* b,
                                    const int8_t* sigma, const int32_t* surcol, double* A1, double* b1) {
  const int64_t e = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (e < m * n1) {
    const int64_t i = e / n1, j = e - i * n1;
    double v;
    if (j < n) v = sigma[i] > 0 ? A[i * n + j] : -A[i * n + j];
    else v = (j - n == surcol[i]) ? -1.0 : 0.0;
    A1[e] = v;
  }
  if (e < m) b1[e] = fabs(b[e]);  // sigma_i b_i >= 0 by the choice of sigma_i
}

// c1_j = sum over artificial rows i (in row order) of A1[i][j].
__global__ void artificial_row_sum_kernel(int64_t m, int64_t n1, const double* A1, const int8_t* art, double* c1) {
  const int64_t j = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (j >= n1) return;
  double acc = 0.0;
  for (int64_t i = 0; i < m; ++i)
    if (art[i]) acc = acc + A1[i * n1 + j];
  c1[j] = acc;
}

// Phase II data from phase I's final tableau T1 ((m+1) x W1, Table 1 layout):
// A2[i][t] = T1[src(i)][N[t]] (mirrored rows negated), b2[i] = max(rhs, +0),
// and 0 for rows whose basic variable is an artificial.
__global__ void build_phase2_kernel(int64_t m, int64_t W1, int64_t n2, int64_t n_extra, const double* T1,
                                    const int32_t* N, const int32_t* extra_rows, const int8_t* zero_rhs,
                                    double* A2, double* b2) {
  const int64_t m2 = m + n_extra;
  const int64_t e = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (e < m2 * n2) {
    const int64_t i = e / n2, t = e - i * n2;
    const int64_t src = i < m ? i : extra_rows[i - m];
    const double v = T1[src * W1 + N[t]];
    A2[e] = i < m ? v : -v;
  }
  if (e < m2) {
    double r = 0.0;
    if (e < m && !zero_rhs[e]) {
      const double t = T1[e * W1 + W1 - 1];
      r = t > 0.0 ? t : 0.0;
    }
    b2[e] = r;
  }
}

// c2_t = cN_t - sum_i cB_i A2[i][t] over the m original rows, in row order.
__global__ void reduced_cost_kernel(int64_t m, int64_t n2, const double* A2, const double* cB, const double* cN,
                                    double* c2) {
  const int64_t t = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (t >= n2) return;
  double acc = 0.0;
  for (int64_t i = 0; i < m; ++i) acc = acc + cB[i] * A2[i * n2 + t];
  c2[t] = cN[t] - acc;
}

// x of the original variables: a phase II structural takes its phase II
// value; a variable basic in phase I's basis (row i) takes row i's slack at
// the phase II optimum, b2_i - sum_t A2[i][t] x2_t (in column order).
__global__ void recover_kernel(int64_t m, int64_t n, int64_t n2, const double* A2, const double* b2,
                               const double* x2, const int32_t* N, const int32_t* basis1, double* x) {
  const int64_t t = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (t < n2 && N[t] < n) x[N[t]] = x2[t];
  if (t < m && basis1[t] < n) {
    double acc = 0.0;
    for (int64_t u = 0; u < n2; ++u) acc = acc + A2[t * n2 + u] * x2[u];
    x[basis1[t]] = b2[t] - acc;
  }
}

// obj = sum_j c_j x_j in index order (one thread: the order is the definition).
__global__ void objective_kernel(int64_t n, const double* c, const double* x, double* obj) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double acc = 0.0;
#pragma unroll 8
  for (int64_t j = 0; j < n; ++j) acc = acc + c[j] * x[j];
  *obj = acc;
}

// x = the first n entries of a phase I / direct solution.
__global__ void copy_kernel(int64_t n, const double* src, double* dst) {
  const int64_t j = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (j < n) dst[j] = src[j];
}

unsigned blocks_for(int64_t count) { return (unsigned)((count + kTB - 1) / kTB); }

int hip_code(hipError_t e) {
  if (e == hipSuccess) return LPD_SUCCESS;
  (void)hipGetLastError();
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return LPD_ERR_OUT_OF_MEMORY;
  return LPD_ERR_HIP;
}

// Stream-ordered device buffers freed together at the end.
struct Arena {
  hipStream_t s;
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;
  template <class T>
  T* get(size_t count) {
    void* p = nullptr;
    if (err == hipSuccess) err = hipMallocAsync(&p, count * sizeof(T) + 16, s);
    if (err != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  ~Arena() {
    for (void* p : ptrs) (void)hipFreeAsync(p, s);
    (void)hipStreamSynchronize(s);
  }
};

}  // namespace
}  // namespace lpd

using namespace lpd;

extern "C" int lp_solve_general(int64_t m, int64_t n, const double* A, const double* b, const double* c,
                                const int8_t* sense, const lpd_options* opt, double* x, double* obj,
                                int32_t* status, int64_t* iterations, hipStream_t stream) {
  if (m < 1 || n < 1) return LPD_ERR_INVALID_ARG;
  if (!A || !b || !c || !x || !obj || !status) return LPD_ERR_NULL_POINTER;
  if (m > (int64_t(1) << 28) || n > (int64_t(1) << 28)) return LPD_ERR_SIZE_OVERFLOW;
  if (sense)
    for (int64_t i = 0; i < m; ++i)
      if (sense[i] != LPD_ROW_LE && sense[i] != LPD_ROW_EQ && sense[i] != LPD_ROW_GE) return LPD_ERR_INVALID_ARG;
  lpd_options o{};
  if (opt) o = *opt;

  std::vector<double> hb((size_t)m), hc((size_t)n);
  hipError_t e = hipMemcpyAsync(hb.data(), b, 8 * (size_t)m, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), c, 8 * (size_t)n, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_code(e);

  // Row plan.
  std::vector<int8_t> sigma((size_t)m), art((size_t)m);
  std::vector<int32_t> surcol((size_t)m, -1);
  int32_t q = 0;
  for (int64_t i = 0; i < m; ++i) {
    const int s = sense ? sense[i] : LPD_ROW_LE;
    const double bi = hb[(size_t)i];
    if (s == LPD_ROW_LE) {
      const bool neg = bi < 0.0;
      sigma[(size_t)i] = neg ? -1 : 1;
      art[(size_t)i] = neg;
      if (neg) surcol[(size_t)i] = q++;
    } else if (s == LPD_ROW_GE) {
      const bool pos = bi > 0.0;  // b <= 0: -A_i x <= -b_i is already a slack row
      sigma[(size_t)i] = pos ? 1 : -1;
      art[(size_t)i] = pos;
      if (pos) surcol[(size_t)i] = q++;
    } else {
      sigma[(size_t)i] = bi < 0.0 ? -1 : 1;
      art[(size_t)i] = 1;
    }
  }
  const int64_t n1 = n + q;
  int64_t n_art = 0;
  double sum_b_art = 0.0;
  for (int64_t i = 0; i < m; ++i)
    if (art[(size_t)i]) {
      ++n_art;
      sum_b_art = sum_b_art + std::fabs(hb[(size_t)i]);
    }

  Arena ar{stream};
  int8_t* d_sigma = ar.get<int8_t>((size_t)m);
  int8_t* d_art = ar.get<int8_t>((size_t)m);
  int32_t* d_surcol = ar.get<int32_t>((size_t)m);
  double* A1 = ar.get<double>((size_t)(m * n1));
  double* b1 = ar.get<double>((size_t)m);
  double* c1 = ar.get<double>((size_t)n1);
  double* x1 = ar.get<double>((size_t)n1);
  double* obj1 = ar.get<double>(1);
  int32_t* st1 = ar.get<int32_t>(1);
  int64_t* it1 = ar.get<int64_t>(1);
  int64_t* basis1 = ar.get<int64_t>((size_t)m);
  const int64_t W1 = n1 + m + 1;
  double* T1 = n_art > 0 ? ar.get<double>((size_t)((m + 1) * W1)) : nullptr;
  if (ar.err != hipSuccess) return hip_code(ar.err);
  (void)hipMemcpyAsync(d_sigma, sigma.data(), (size_t)m, hipMemcpyHostToDevice, stream);
  (void)hipMemcpyAsync(d_art, art.data(), (size_t)m, hipMemcpyHostToDevice, stream);
  (void)hipMemcpyAsync(d_surcol, surcol.data(), 4 * (size_t)m, hipMemcpyHostToDevice, stream);
  build_phase1_kernel<<<blocks_for(std::max(m * n1, m)), kTB, 0, stream>>>(m, n, n1, A, b, d_sigma, d_surcol, A1,
                                                                            b1);
  if (n_art > 0) {
    artificial_row_sum_kernel<<<blocks_for(n1), kTB, 0, stream>>>(m, n1, A1, d_art, c1);
  } else {
    // No artificial row: the scaled LP is canonical already; one solve with c.
    (void)hipMemcpyAsync(c1, c, 8 * (size_t)n, hipMemcpyDeviceToDevice, stream);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return hip_code(e);

  lpd_problem p1{m, n1, A1, b1, c1};
  lpd_outputs out1{};
  out1.x = x1;
  out1.obj = obj1;
  out1.status = st1;
  out1.iterations = it1;
  out1.basis = basis1;
  out1.tableau = T1;
  int rc = lp_solve_dense_ex(&p1, &o, &out1, stream);
  if (rc != LPD_SUCCESS) return rc;

  int32_t h_st1 = 0;
  int64_t h_it1 = 0;
  double h_obj1 = 0.0;
  std::vector<int64_t> h_basis((size_t)m);
  (void)hipMemcpyAsync(&h_st1, st1, 4, hipMemcpyDeviceToHost, stream);
  (void)hipMemcpyAsync(&h_it1, it1, 8, hipMemcpyDeviceToHost, stream);
  (void)hipMemcpyAsync(&h_obj1, obj1, 8, hipMemcpyDeviceToHost, stream);
  (void)hipMemcpyAsync(h_basis.data(), basis1, 8 * (size_t)m, hipMemcpyDeviceToHost, stream);
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_code(e);

  int32_t h_status = h_st1;
  int64_t h_iters = h_it1;
  const bool feasible =
      h_st1 == LPD_OPTIMAL && (n_art == 0 || h_obj1 >= sum_b_art - 1e-9 * std::max(1.0, sum_b_art));
  if (n_art == 0 || h_st1 != LPD_OPTIMAL || !feasible) {
    // Done after one solve: the direct answer, or phase I's point with its status.
    if (h_st1 == LPD_OPTIMAL && !feasible) h_status = LPD_INFEASIBLE;
    copy_kernel<<<blocks_for(n), kTB, 0, stream>>>(n, x1, x);
  } else {
    // Phase II layout from phase I's basis.
    std::vector<int8_t> basic((size_t)(n1 + m), 0);
    for (int64_t i = 0; i < m; ++i) basic[(size_t)h_basis[(size_t)i]] = 1;
    std::vector<int32_t> N, extra;
    std::vector<int8_t> zero_rhs((size_t)m, 0);
    for (int64_t v = 0; v < n1 + m; ++v) {
      const bool is_art = v >= n1 && art[(size_t)(v - n1)];
      if (!basic[(size_t)v] && !is_art) N.push_back((int32_t)v);
    }
    std::vector<double> cB((size_t)m), cN(N.size());
    std::vector<int32_t> b1v((size_t)m);
    for (int64_t i = 0; i < m; ++i) {
      const int64_t v = h_basis[(size_t)i];
      b1v[(size_t)i] = (int32_t)v;
      cB[(size_t)i] = v < n ? hc[(size_t)v] : 0.0;
      if (v >= n1 && art[(size_t)(v - n1)]) {  // artificial left basic, at level zero
        extra.push_back((int32_t)i);
        zero_rhs[(size_t)i] = 1;
      }
    }
    for (size_t t = 0; t < N.size(); ++t) cN[t] = N[t] < n ? hc[(size_t)N[t]] : 0.0;
    const int64_t n2 = (int64_t)N.size(), m2 = m + (int64_t)extra.size();

    int32_t* d_N = ar.get<int32_t>(N.size() + 1);
    int32_t* d_extra = ar.get<int32_t>(extra.size() + 1);
    int8_t* d_zero = ar.get<int8_t>((size_t)m);
    int32_t* d_b1v = ar.get<int32_t>((size_t)m);
    double* d_cB = ar.get<double>((size_t)m);
    double* d_cN = ar.get<double>(N.size() + 1);
    double* A2 = ar.get<double>((size_t)(m2 * std::max<int64_t>(n2, 1)));
    double* b2 = ar.get<double>((size_t)m2);
    double* c2 = ar.get<double>((size_t)std::max<int64_t>(n2, 1));
    double* x2 = ar.get<double>((size_t)std::max<int64_t>(n2, 1));
    double* obj2 = ar.get<double>(1);
    int32_t* st2 = ar.get<int32_t>(1);
    int64_t* it2 = ar.get<int64_t>(1);
    if (ar.err != hipSuccess) return hip_code(ar.err);
    if (n2) (void)hipMemcpyAsync(d_N, N.data(), 4 * N.size(), hipMemcpyHostToDevice, stream);
    if (!extra.empty()) (void)hipMemcpyAsync(d_extra, extra.data(), 4 * extra.size(), hipMemcpyHostToDevice, stream);
    (void)hipMemcpyAsync(d_zero, zero_rhs.data(), (size_t)m, hipMemcpyHostToDevice, stream);
    (void)hipMemcpyAsync(d_b1v, b1v.data(), 4 * (size_t)m, hipMemcpyHostToDevice, stream);
    (void)hipMemcpyAsync(d_cB, cB.data(), 8 * (size_t)m, hipMemcpyHostToDevice, stream);
    if (n2) (void)hipMemcpyAsync(d_cN, cN.data(), 8 * N.size(), hipMemcpyHostToDevice, stream);
    build_phase2_kernel<<<blocks_for(std::max(m2 * n2, m2)), kTB, 0, stream>>>(
        m, W1, n2, (int64_t)extra.size(), T1, d_N, d_extra, d_zero, A2, b2);
    int32_t h_st2 = LPD_OPTIMAL;
    int64_t h_it2 = 0;
    if (n2 > 0) {
      reduced_cost_kernel<<<blocks_for(n2), kTB, 0, stream>>>(m, n2, A2, d_cB, d_cN, c2);
      e = hipGetLastError();
      if (e != hipSuccess) return hip_code(e);
      lpd_problem p2{m2, n2, A2, b2, c2};
      lpd_outputs out2{};
      out2.x = x2;
      out2.obj = obj2;
      out2.status = st2;
      out2.iterations = it2;
      rc = lp_solve_dense_ex(&p2, &o, &out2, stream);
      if (rc != LPD_SUCCESS) return rc;
      (void)hipMemcpyAsync(&h_st2, st2, 4, hipMemcpyDeviceToHost, stream);
      (void)hipMemcpyAsync(&h_it2, it2, 8, hipMemcpyDeviceToHost, stream);
    }
    recover_kernel<<<blocks_for(std::max(n2, m)), kTB, 0, stream>>>(m, n, n2, A2, b2, x2, d_N, d_b1v, x);
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_code(e);
    h_status = h_st2;
    h_iters = h_it1 + h_it2;
  }
  objective_kernel<<<1, 1, 0, stream>>>(n, c, x, obj);
  (void)hipMemcpyAsync(status, &h_status, 4, hipMemcpyHostToDevice, stream);
  if (iterations) (void)hipMemcpyAsync(iterations, &h_iters, 8, hipMemcpyHostToDevice, stream);
  e = hipGetLastError();
  const hipError_t es = hipStreamSynchronize(stream);  // host sources above must outlive the copies
  if (e == hipSuccess) e = es;
  return hip_code(e);
}
