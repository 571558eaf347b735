// Two-phase solve of a general LP -- rows <=, = or >= with right-hand sides
// of any sign -- on the pivot kernels (Section 2 states the problem with
// equality rows; its Steps 1-5 start from the slack basis of <= rows with
// b >= 0).  The textbook two-phase method, every pivot in the kernels of
// lp_solve_tableau:
//
//   rows      row i times sigma_i = -1 when b_i < 0, or b_i = 0 on a >= row,
//             so that every right-hand side is >= 0;
//   phase I   Table 1's layout [sigma A | -S | I | sigma b] (S: one surplus
//             column per row that now reads >=; I: each row's slack, or an
//             artificial variable on >= and = rows), objective +1 in the
//             artificial columns with those basic columns eliminated
//             (maximise minus the sum of the artificials); Steps 2-5;
//   feasible  iff phase I's optimum >= -1e-9 max(1, sum of the artificial
//             rows' right-hand sides);
//   drive-out each artificial still basic, rows in order, leaves by a pivot
//             on the lowest non-artificial column with |entry| > eps_p; a
//             row without one is redundant;
//   phase II  artificial columns and redundant rows deleted, objective row
//             [-c | 0 | 0] with the basic columns eliminated; Steps 2-5.
//
// Every elimination of the objective row is Step 5's fused multiply-add, one
// row after the other in row order, so the results are reproducible bit for
// bit.  The host decides what depends on phase I's outcome (which rows are
// redundant, the phase II layout) between synchronisations of the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "lpd_device.h"
#include "lpdense.h"

namespace lpd {
namespace {

constexpr int kTB = 256;
constexpr int kSelectThreads = 1024;

unsigned blocks_for(int64_t count) { return (unsigned)((count + kTB - 1) / kTB); }

// Phase I constraint rows, (m x W1) of the (m+1) x W1 tableau:
// [sigma_i A_i | -1 in row i's surplus column | 1 in column n1 + i | sigma_i b_i].
__global__ void phase1_rows_kernel(int64_t m, int64_t n, int64_t n1, const double* A, const double* b,
                                   const int8_t* sigma, const int32_t* surcol, double* T) {
  const int64_t W1 = n1 + m + 1;
  const int64_t e = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (e >= m * W1) return;
  const int64_t i = e / W1, j = e - i * W1;
  const bool neg = sigma[i] < 0;
  double v;
  if (j < n) v = neg ? -A[i * n + j] : A[i * n + j];
  else if (j < n1) v = (j - n == surcol[i]) ? -1.0 : 0.0;
  else if (j < n1 + m) v = (j - n1 == i) ? 1.0 : 0.0;
  else v = neg ? -b[i] : b[i];
  T[e] = v;
}

// Phase I objective row: +1 in the artificial columns, then for each
// artificial row in order (its basic column holds +1 in the objective row
// when it comes) the elimination fma(-1, T[i][j], .) of Step 5.
__global__ void phase1_objective_kernel(int64_t m, int64_t n1, const int8_t* art, double* T) {
  const int64_t W1 = n1 + m + 1;
  const int64_t j = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (j >= W1) return;
  double acc = (j >= n1 && j < n1 + m && art[j - n1]) ? 1.0 : 0.0;
  for (int64_t i = 0; i < m; ++i)
    if (art[i]) acc = __builtin_fma(-1.0, T[i * W1 + j], acc);
  T[m * W1 + j] = acc;
}

// Drive-out, step 1 (one workgroup): in row `row` of the phase I tableau,
// the lowest non-artificial column k with |T[row][k]| > eps_p.  If there is
// one: the pivot row T[row][:] / T[row][k] (IEEE division) into prow, the
// pivot column T[:][k] (objective row included) into pcol, and k into
// *sel; else *sel = -1 (a redundant row).
__global__ void __launch_bounds__(kSelectThreads)
    driveout_select_kernel(int64_t m, int64_t n1, const int8_t* art, const double* T, int64_t row, double eps_p,
                           double* prow, double* pcol, int32_t* sel) {
  __shared__ Cand scratch[kSelectThreads / kWave + 1];
  const int64_t ncols = n1 + m, W1 = ncols + 1;
  const double* Tr = T + row * W1;
  Cand c = cand_none();
  for (int64_t j = threadIdx.x; j < ncols; j += blockDim.x) {
    const bool artificial = j >= n1 && art[j - n1];
    if (!artificial && __builtin_fabs(Tr[j]) > eps_p) cand_offer(c, 0.0, (int32_t)j, 0.0);
  }
  c = block_reduce(c, scratch);
  if (c.i == kNoIndex) {
    if (threadIdx.x == 0) *sel = -1;
    return;
  }
  const int64_t k = c.i;
  const double p = Tr[k];
  for (int64_t j = threadIdx.x; j < W1; j += blockDim.x) prow[j] = Tr[j] / p;
  for (int64_t i = threadIdx.x; i <= m; i += blockDim.x) pcol[i] = T[i * W1 + k];
  if (threadIdx.x == 0) *sel = (int32_t)k;
}

// Drive-out, step 2: Steps 4-5 of that pivot over the whole tableau (the
// pivot column was captured before any row changes).
__global__ void driveout_apply_kernel(int64_t m, int64_t W1, double* T, int64_t row, const double* prow,
                                      const double* pcol, const int32_t* sel) {
  if (*sel < 0) return;
  const int64_t e = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (e >= (m + 1) * W1) return;
  const int64_t i = e / W1, j = e - i * W1;
  T[e] = i == row ? prow[j] : __builtin_fma(-pcol[i], prow[j], T[e]);
}

// Phase II constraint rows: the kept rows and columns (the RHS last) of the
// phase I tableau after the drive-out.
__global__ void phase2_rows_kernel(int64_t m2, int64_t W2, int64_t W1, const double* T1, const int32_t* rows,
                                   const int32_t* cols, double* T2) {
  const int64_t e = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (e >= m2 * W2) return;
  const int64_t i = e / W2, j = e - i * W2;
  T2[e] = T1[(int64_t)rows[i] * W1 + cols[j]];
}

// Phase II objective row: [-c | 0 | 0], then for each row in order with
// f_i != 0 the elimination fma(-f_i, T2[i][j], .) of Step 5, f_i being the
// objective-row entry of row i's basic column when row i comes: -c of a
// basic original variable, 0 otherwise (the earlier rows are 0 in that
// column, so it is unchanged until then).
__global__ void phase2_objective_kernel(int64_t m2, int64_t W2, int64_t n, const double* c, const double* f,
                                        double* T2) {
  const int64_t j = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (j >= W2) return;
  double acc = j < n ? -c[j] : 0.0;
  for (int64_t i = 0; i < m2; ++i)
    if (f[i] != 0.0) acc = __builtin_fma(-f[i], T2[i * W2 + j], acc);
  T2[m2 * W2 + j] = acc;
}

// Phase II with no constraint row left (every row redundant): Steps 2-3 on
// the objective row alone -- optimal if no reduced cost is below -eps_d, else
// unbounded (no row for the ratio test), or the iteration cap if it is 0.
__global__ void __launch_bounds__(kSelectThreads)
    no_rows_kernel(int64_t W2, const double* objrow, double eps_d, int64_t max_iter, int32_t* status) {
  __shared__ Cand scratch[kSelectThreads / kWave + 1];
  Cand c = cand_none();
  for (int64_t j = threadIdx.x; j < W2; j += blockDim.x) {
    const double v = objrow[j];
    if (!is_finite(v)) c.flags |= kFlagNonFinite;
    if (j < W2 - 1 && !__builtin_isnan(v)) cand_offer(c, v, (int32_t)j, 0.0);
  }
  c = block_reduce(c, scratch);
  if (threadIdx.x != 0) return;
  if (c.flags & kFlagNonFinite) *status = kNumerical;
  else if (c.v >= -eps_d) *status = kOptimal;
  else if (max_iter == 0) *status = kIterLimit;
  else *status = kUnbounded;
}

// obj = sum_j c_j x_j in index order (one thread: the order is the definition).
__global__ void objective_kernel(int64_t n, const double* c, const double* x, double* obj) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double acc = 0.0;
  for (int64_t j = 0; j < n; ++j) acc = acc + c[j] * x[j];
  *obj = acc;
}

// The n original variables' values: the first n entries of a phase's x.
__global__ void copy_kernel(int64_t n, const double* src, double* dst) {
  const int64_t j = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (j < n) dst[j] = src[j];
}

__global__ void zero_kernel(int64_t n, double* dst) {
  const int64_t j = (int64_t)blockIdx.x * kTB + threadIdx.x;
  if (j < n) dst[j] = 0.0;
}

// Final status and pivot count: phase II's status and pivots plus `before`.
__global__ void finish_kernel(const int32_t* st2, const int64_t* it2, int64_t before, int32_t* status,
                              int64_t* iterations) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  *status = *st2;
  if (iterations) *iterations = before + (it2 ? *it2 : 0);
}

int hip_code(hipError_t e) {
  if (e == hipSuccess) return LPD_SUCCESS;
  (void)hipGetLastError();
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return LPD_ERR_OUT_OF_MEMORY;
  return LPD_ERR_HIP;
}

// Stream-ordered device buffers, freed together when the call returns (after
// the stream has drained: the host arrays copied from live until then).
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
  if (o.max_iter < 0) o.max_iter = 50 * (m + n);  // per phase
  if (std::isnan(o.eps_p) || std::isinf(o.eps_p)) return LPD_ERR_INVALID_ARG;
  const double eps_p = o.eps_p > 0 ? o.eps_p : LPD_DEFAULT_EPS;

  Arena ar{stream};
  std::vector<double> hb((size_t)m), hc((size_t)n);
  hipError_t e = hipMemcpyAsync(hb.data(), b, 8 * (size_t)m, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), c, 8 * (size_t)n, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_code(e);

  // Rows: sigma, the sense after scaling, surplus columns, artificials.
  std::vector<int8_t> sigma((size_t)m), art((size_t)m);
  std::vector<int32_t> surcol((size_t)m, -1);
  int32_t q = 0;
  for (int64_t i = 0; i < m; ++i) {
    const int s = sense ? sense[i] : LPD_ROW_LE;
    const double bi = hb[(size_t)i];
    const bool flip = bi < 0.0 || (bi == 0.0 && s == LPD_ROW_GE);
    sigma[(size_t)i] = flip ? -1 : 1;
    const int scaled = !flip ? s : (s == LPD_ROW_LE ? LPD_ROW_GE : (s == LPD_ROW_GE ? LPD_ROW_LE : LPD_ROW_EQ));
    art[(size_t)i] = scaled != LPD_ROW_LE;
    if (scaled == LPD_ROW_GE) surcol[(size_t)i] = q++;
  }
  const int64_t n1 = n + q, ncols1 = n1 + m, W1 = ncols1 + 1;
  double sum_b_art = 0.0;
  for (int64_t i = 0; i < m; ++i)
    if (art[(size_t)i]) sum_b_art = sum_b_art + (sigma[(size_t)i] < 0 ? -hb[(size_t)i] : hb[(size_t)i]);

  int8_t* d_sigma = ar.get<int8_t>((size_t)m);
  int8_t* d_art = ar.get<int8_t>((size_t)m);
  int32_t* d_surcol = ar.get<int32_t>((size_t)m);
  double* T1 = ar.get<double>((size_t)((m + 1) * W1));
  double* T1f = ar.get<double>((size_t)((m + 1) * W1));
  double* x1 = ar.get<double>((size_t)ncols1);
  double* obj1 = ar.get<double>(1);
  int32_t* st1 = ar.get<int32_t>(1);
  int64_t* it1 = ar.get<int64_t>(1);
  int64_t* basis1 = ar.get<int64_t>((size_t)m);
  if (ar.err != hipSuccess) return hip_code(ar.err);
  e = hipMemcpyAsync(d_sigma, sigma.data(), (size_t)m, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_art, art.data(), (size_t)m, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_surcol, surcol.data(), 4 * (size_t)m, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_code(e);
  phase1_rows_kernel<<<blocks_for(m * W1), kTB, 0, stream>>>(m, n, n1, A, b, d_sigma, d_surcol, T1);
  phase1_objective_kernel<<<blocks_for(W1), kTB, 0, stream>>>(m, n1, d_art, T1);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_code(e);

  // Phase I.
  std::vector<int64_t> hbasis((size_t)m);
  for (int64_t i = 0; i < m; ++i) hbasis[(size_t)i] = n1 + i;
  lpd_outputs out1{};
  out1.x = x1;
  out1.obj = obj1;
  out1.status = st1;
  out1.iterations = it1;
  out1.basis = basis1;
  out1.tableau = T1f;
  int rc = lp_solve_tableau(m, ncols1, T1, hbasis.data(), &o, &out1, stream);
  if (rc != LPD_SUCCESS) return rc;
  int32_t h_st1 = 0;
  int64_t h_it1 = 0;
  double h_obj1 = 0.0;
  e = hipMemcpyAsync(&h_st1, st1, 4, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&h_it1, it1, 8, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&h_obj1, obj1, 8, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(hbasis.data(), basis1, 8 * (size_t)m, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_code(e);

  const bool feasible = h_st1 == LPD_OPTIMAL && h_obj1 >= -1e-9 * std::max(1.0, sum_b_art);
  int32_t h_status = 0;
  if (!feasible) {
    // No phase II: phase I's point, its status (or INFEASIBLE), c^T x.
    h_status = h_st1 == LPD_OPTIMAL ? LPD_INFEASIBLE : h_st1;
    copy_kernel<<<blocks_for(n), kTB, 0, stream>>>(n, x1, x);
    objective_kernel<<<1, 1, 0, stream>>>(n, c, x, obj);
    e = hipMemcpyAsync(status, &h_status, 4, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && iterations) e = hipMemcpyAsync(iterations, &h_it1, 8, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);  // the host sources outlive the copies
    return hip_code(e);
  }

  // Drive-out of the artificial variables still basic, rows in order.
  auto is_art_col = [&](int64_t j) { return j >= n1 && art[(size_t)(j - n1)]; };
  std::vector<int64_t> cand_rows;
  for (int64_t i = 0; i < m; ++i)
    if (is_art_col(hbasis[(size_t)i])) cand_rows.push_back(i);
  std::vector<int32_t> sel(cand_rows.size() + 1, -1);
  if (!cand_rows.empty()) {
    double* prow = ar.get<double>((size_t)W1);
    double* pcol = ar.get<double>((size_t)(m + 1));
    int32_t* d_sel = ar.get<int32_t>(cand_rows.size());
    if (ar.err != hipSuccess) return hip_code(ar.err);
    for (size_t t = 0; t < cand_rows.size(); ++t) {
      driveout_select_kernel<<<1, kSelectThreads, 0, stream>>>(m, n1, d_art, T1f, cand_rows[t], eps_p, prow, pcol,
                                                               d_sel + t);
      driveout_apply_kernel<<<blocks_for((m + 1) * W1), kTB, 0, stream>>>(m, W1, T1f, cand_rows[t], prow, pcol,
                                                                          d_sel + t);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(sel.data(), d_sel, 4 * cand_rows.size(), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_code(e);
  }
  int64_t n_drive = 0;
  std::vector<char> redundant((size_t)m, 0);
  for (size_t t = 0; t < cand_rows.size(); ++t) {
    if (sel[t] >= 0) {
      hbasis[(size_t)cand_rows[t]] = sel[t];
      ++n_drive;
    } else {
      redundant[(size_t)cand_rows[t]] = 1;
    }
  }

  // Phase II layout: kept rows and (non-artificial) columns, the RHS last.
  std::vector<int32_t> rows, cols, where((size_t)ncols1, -1);
  for (int64_t i = 0; i < m; ++i)
    if (!redundant[(size_t)i]) rows.push_back((int32_t)i);
  for (int64_t j = 0; j < ncols1; ++j)
    if (!is_art_col(j)) {
      where[(size_t)j] = (int32_t)cols.size();
      cols.push_back((int32_t)j);
    }
  cols.push_back((int32_t)ncols1);
  const int64_t m2 = (int64_t)rows.size(), W2 = (int64_t)cols.size(), ncols2 = W2 - 1;
  std::vector<int64_t> basis2((size_t)m2);
  std::vector<double> f((size_t)std::max<int64_t>(m2, 1), 0.0);
  for (int64_t r = 0; r < m2; ++r) {
    const int64_t v = hbasis[(size_t)rows[(size_t)r]];
    basis2[(size_t)r] = where[(size_t)v];
    f[(size_t)r] = v < n ? -hc[(size_t)v] : 0.0;
  }
  int32_t* d_rows = ar.get<int32_t>(rows.size() + 1);
  int32_t* d_cols = ar.get<int32_t>(cols.size());
  double* d_f = ar.get<double>(f.size());
  double* T2 = ar.get<double>((size_t)((m2 + 1) * W2));
  double* x2 = ar.get<double>((size_t)ncols2);
  double* obj2 = ar.get<double>(1);
  int32_t* st2 = ar.get<int32_t>(1);
  int64_t* it2 = ar.get<int64_t>(1);
  if (ar.err != hipSuccess) return hip_code(ar.err);
  e = hipSuccess;
  if (m2 > 0) e = hipMemcpyAsync(d_rows, rows.data(), 4 * rows.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_cols, cols.data(), 4 * cols.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_f, f.data(), 8 * f.size(), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_code(e);
  if (m2 > 0) phase2_rows_kernel<<<blocks_for(m2 * W2), kTB, 0, stream>>>(m2, W2, W1, T1f, d_rows, d_cols, T2);
  phase2_objective_kernel<<<blocks_for(W2), kTB, 0, stream>>>(m2, W2, n, c, d_f, T2);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_code(e);

  // Phase II.
  if (m2 == 0) {
    no_rows_kernel<<<1, kSelectThreads, 0, stream>>>(W2, T2, o.eps_d > 0 ? o.eps_d : LPD_DEFAULT_EPS, o.max_iter,
                                                     st2);
    zero_kernel<<<blocks_for(n), kTB, 0, stream>>>(n, x);
    e = hipMemcpyAsync(obj, T2 + (W2 - 1), 8, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hip_code(e);
    finish_kernel<<<1, 1, 0, stream>>>(st2, nullptr, h_it1 + n_drive, status, iterations);
  } else {
    lpd_outputs out2{};
    out2.x = x2;
    out2.obj = obj2;
    out2.status = st2;
    out2.iterations = it2;
    rc = lp_solve_tableau(m2, ncols2, T2, basis2.data(), &o, &out2, stream);
    if (rc != LPD_SUCCESS) return rc;
    copy_kernel<<<blocks_for(n), kTB, 0, stream>>>(n, x2, x);  // the first n columns are x's
    e = hipMemcpyAsync(obj, obj2, 8, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return hip_code(e);
    finish_kernel<<<1, 1, 0, stream>>>(st2, it2, h_it1 + n_drive, status, iterations);
  }
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return hip_code(e);
}
