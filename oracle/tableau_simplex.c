/*
 * Reference oracle: plain, slow FP64 dense-tableau simplex on the CPU.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header or constant with the HIP
 * library.
 *
 * What it computes (Coutinho, Lins e Silva, Aloise, Xavier-de-Souza,
 * "A Scalable Shared-Memory Parallel Simplex for Large-Scale Linear
 * Programming", Section 2):
 *
 *   maximize c^T x  subject to  A x <= b,  x >= 0,  with b >= 0,
 *
 * solved by the standard (full-tableau) simplex method from the slack basis:
 *   Step 1  build the initial tableau of Table 1: constraint rows
 *           [A_i | e_i | b_i], objective row [-c | 0 | 0] last;
 *   Step 2  pick the entering column k among the negative reduced costs of
 *           the objective row (most negative one), stop if none;
 *   Step 3  ratio test rho_i = b_i / a_ik over the positive a_ik, leaving row
 *           l = argmin rho_i; unbounded if there is no positive a_ik;
 *   Step 4  divide the pivot row by the pivot a_lk;
 *   Step 5  row_i <- row_i - a_ik * row_l for every other row, the objective
 *           row included.
 * Section 3 (the parallel scheme) repeats Steps 2-5 in a loop until the
 * objective row has no negative entry; that loop is taken here, serially.
 *
 * Readings where the paper is silent (all shared with the GPU library by
 * specification, not by code):
 *  - pricing runs over every non-RHS column j in [0, n+m) (slack columns can
 *    acquire negative reduced costs after a pivot);
 *  - ties in pricing and in the ratio test go to the lowest index;
 *  - optimal iff min_j T[m,j] >= -eps_d; eligible ratio rows have
 *    T[i,k] > eps_p; unbounded iff no row is eligible;
 *  - the stored right-hand side is used unclamped;
 *  - the pivot row is divided first (IEEE division), then every other row is
 *    updated with one fused multiply-add per element,
 *    T[i,j] <- fma(-f_i, r_j, T[i,j]), f_i = T[i,k] read before row i changes;
 *  - loop order per iteration: price -> (optimal?) -> (iteration cap?) ->
 *    ratio test -> (unbounded?) -> pivot;
 *  - non-finite input, or a non-finite value met by the pricing scan or the
 *    ratio test, ends the solve with status NUMERICAL; a negative b_i ends it
 *    with INFEASIBLE_START (no pivot), since Step 1's slack basis needs b>=0.
 *
 * Besides the solve from Table 1 (oracle_solve), the file offers the same
 * Steps 2-5 from any basic tableau (oracle_solve_tableau), one pivot on a
 * given element (oracle_pivot: Steps 4-5 alone) and the elimination of the
 * basic columns from the objective row (oracle_price_out: Step 5 applied to
 * the objective row with each basic row as pivot row).  The two-phase method
 * for general LPs (oracle/general.py) is composed of these.
 *
 * Build: gcc -O3 -mavx2 -std=c11 -mfma -ffp-contract=off -fno-math-errno -shared -fPIC
 * (-ffp-contract=off: the only fused operation is the explicit fma() call.)
 * Built with -fopenmp as well, Step 5 runs its rows in parallel threads; the
 * rows are independent, so every value is the same as in the serial build.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define ORC_OPTIMAL 0
#define ORC_UNBOUNDED 1
#define ORC_ITERATION_LIMIT 2
#define ORC_INFEASIBLE_START 3
#define ORC_NUMERICAL 4

#define ORC_ERR_ARG (-1)
#define ORC_ERR_NOMEM (-2)

/* Row-major tableau element (i, j); ld = W = n + m + 1 (no padding). */
#define TAB(T, ld, i, j) ((T)[(size_t)(i) * (size_t)(ld) + (size_t)(j)])

/* Step 1 (Table 1): rows 0..m-1 are [A_i | e_i | b_i], row m is [-c | 0 | 0]. */
static void build_initial_tableau(int64_t m, int64_t n, const double *A,
                                  const double *b, const double *c, double *T) {
    const int64_t W = n + m + 1;
    memset(T, 0, sizeof(double) * (size_t)(m + 1) * (size_t)W);
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) TAB(T, W, i, j) = A[i * n + j];
        TAB(T, W, i, n + i) = 1.0;
        TAB(T, W, i, W - 1) = b[i];
    }
    for (int64_t j = 0; j < n; ++j) TAB(T, W, m, j) = -c[j];
}

/* Solution read from the final tableau: x_j is the RHS of the row whose basic
 * variable is j (0 if j is nonbasic); z is the objective row's RHS; the dual
 * y_i is the objective-row entry of slack column n+i. */
static void extract(int64_t m, int64_t n, const double *T, const int64_t *basis,
                    double *x, double *obj, double *y) {
    const int64_t W = n + m + 1;
    if (x) {
        for (int64_t j = 0; j < n; ++j) x[j] = 0.0;
        for (int64_t i = 0; i < m; ++i)
            if (basis[i] < n) x[basis[i]] = TAB(T, W, i, W - 1);
    }
    if (obj) *obj = TAB(T, W, m, W - 1);
    if (y)
        for (int64_t i = 0; i < m; ++i) y[i] = TAB(T, W, m, n + i);
}

/* Steps 4-5 for the pivot element (l, k): divide row l by T[l,k], then
 * eliminate column k from every other row of the R-row tableau, the
 * objective row included; the multiplier is read before the row changes. */
static void pivot_on(int64_t R, int64_t W, double *T, int64_t l, int64_t k) {
    /* Step 4: divide the pivot row by the pivot element. */
    const double p = TAB(T, W, l, k);
    for (int64_t j = 0; j < W; ++j) TAB(T, W, l, j) = TAB(T, W, l, j) / p;

    /* Step 5: eliminate column k from every other row, objective row
     * included; the multiplier is read before the row is changed. */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < R; ++i) {
        if (i == l) continue;
        const double f = TAB(T, W, i, k);
        for (int64_t j = 0; j < W; ++j)
            TAB(T, W, i, j) = fma(-f, TAB(T, W, l, j), TAB(T, W, i, j));
    }
}

/* Steps 2-5 repeated (Section 3's loop) on the tableau T of m constraint
 * rows and the objective row m, with ncols variable columns and the RHS in
 * column ncols; basis[i] is the variable of row i.  Stops at a status;
 * returns it and leaves the final tableau and basis in place. */
static int iterate(int64_t m, int64_t ncols, double *T, int64_t *basis, double eps_d,
                   double eps_p, int64_t max_iter, int64_t *iters, int32_t *trace,
                   int64_t trace_cap) {
    const int64_t R = m + 1, W = ncols + 1;
    int status = -1;
    int64_t iter = 0;
    while (status < 0) {
        /* Step 2: entering column = most negative reduced cost, lowest index
         * on ties (strict < in a left-to-right scan). */
        int64_t k = -1;
        double best = INFINITY;
        int bad = 0;
        for (int64_t j = 0; j < ncols; ++j) {
            const double v = TAB(T, W, m, j);
            if (!isfinite(v)) bad = 1;
            if (v < best) {
                best = v;
                k = j;
            }
        }
        if (bad || k < 0) {
            status = ORC_NUMERICAL;
            break;
        }
        if (best >= -eps_d) {
            status = ORC_OPTIMAL;
            break;
        }
        if (iter == max_iter) {
            status = ORC_ITERATION_LIMIT;
            break;
        }

        /* Step 3: min-ratio test over the rows with a positive entry in
         * column k; lowest row index on ties. */
        int64_t l = -1;
        double best_rho = INFINITY;
        for (int64_t i = 0; i < m; ++i) {
            const double a = TAB(T, W, i, k), r = TAB(T, W, i, W - 1);
            if (!isfinite(a) || !isfinite(r)) bad = 1;
            if (a > eps_p) {
                const double rho = r / a;
                if (l < 0 || rho < best_rho) {
                    best_rho = rho;
                    l = i;
                }
            }
        }
        if (bad) {
            status = ORC_NUMERICAL;
            break;
        }
        if (l < 0) {
            status = ORC_UNBOUNDED;
            break;
        }

        /* Steps 4-5. */
        pivot_on(R, W, T, l, k);

        basis[l] = k;
        if (trace && iter < trace_cap) {
            trace[2 * iter] = (int32_t)k;
            trace[2 * iter + 1] = (int32_t)l;
        }
        ++iter;
    }
    if (iters) *iters = iter;
    return status;
}

/*
 * oracle_solve: solve one LP; see the header comment for the rules.
 *   A      m*n row-major, b length m, c length n (host memory, read only)
 *   eps_d  optimality tolerance, eps_p ratio-test pivot tolerance
 *   max_iter  cap on the number of pivots (>= 0)
 * Optional outputs (NULL to skip):
 *   x (n), obj (1), y (m), iters (1), basis_out (m, int64),
 *   trace (2*trace_cap int32: entering column k then leaving row l per pivot),
 *   tableau_out ((m+1)*(n+m+1) row-major, the final tableau).
 * Returns the status (0..4) or a negative error code.
 */
int oracle_solve(int64_t m, int64_t n, const double *A, const double *b,
                 const double *c, double eps_d, double eps_p, int64_t max_iter,
                 double *x, double *obj, double *y, int64_t *iters,
                 int64_t *basis_out, int32_t *trace, int64_t trace_cap,
                 double *tableau_out) {
    if (m < 1 || n < 1 || !A || !b || !c || max_iter < 0) return ORC_ERR_ARG;
    const int64_t R = m + 1, W = n + m + 1;
    double *T = (double *)malloc(sizeof(double) * (size_t)R * (size_t)W);
    int64_t *basis = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    if (!T || !basis) {
        free(T);
        free(basis);
        return ORC_ERR_NOMEM;
    }

    /* Step 1. */
    build_initial_tableau(m, n, A, b, c, T);
    for (int64_t i = 0; i < m; ++i) basis[i] = n + i;

    int status = -1;
    int64_t iter = 0;

    /* Preconditions of the slack starting basis. */
    for (int64_t e = 0; e < m * n && status < 0; ++e)
        if (!isfinite(A[e])) status = ORC_NUMERICAL;
    for (int64_t i = 0; i < m && status < 0; ++i)
        if (!isfinite(b[i])) status = ORC_NUMERICAL;
    for (int64_t j = 0; j < n && status < 0; ++j)
        if (!isfinite(c[j])) status = ORC_NUMERICAL;
    for (int64_t i = 0; i < m && status < 0; ++i)
        if (b[i] < 0.0) status = ORC_INFEASIBLE_START;

    if (status < 0)
        status = iterate(m, n + m, T, basis, eps_d, eps_p, max_iter, &iter, trace, trace_cap);

    extract(m, n, T, basis, x, obj, y);
    if (iters) *iters = iter;
    if (basis_out) memcpy(basis_out, basis, sizeof(int64_t) * (size_t)m);
    if (tableau_out) memcpy(tableau_out, T, sizeof(double) * (size_t)R * (size_t)W);
    free(T);
    free(basis);
    return status;
}

/*
 * oracle_solve_tableau: Steps 2-5 from a given basic tableau instead of
 * Table 1, in place.
 *   m      constraint rows (>= 0); the objective row is row m
 *   ncols  variable columns (>= 1); the RHS is column ncols, so T is
 *          (m+1) x (ncols+1) row-major
 *   basis  m entries: the variable (column) of each row, whose column must
 *          be the unit vector of that row with a zero objective-row entry;
 *          updated in place
 * The right-hand side is used as stored.  A non-finite entry anywhere in T
 * gives NUMERICAL before any pivot.  iters and trace as in oracle_solve.
 * Returns the status or a negative error code.
 */
int oracle_solve_tableau(int64_t m, int64_t ncols, double *T, int64_t *basis, double eps_d,
                         double eps_p, int64_t max_iter, int64_t *iters, int32_t *trace,
                         int64_t trace_cap) {
    if (m < 0 || ncols < 1 || !T || (m > 0 && !basis) || max_iter < 0) return ORC_ERR_ARG;
    const int64_t W = ncols + 1;
    for (int64_t e = 0; e < (m + 1) * W; ++e)
        if (!isfinite(T[e])) {
            if (iters) *iters = 0;
            return ORC_NUMERICAL;
        }
    return iterate(m, ncols, T, basis, eps_d, eps_p, max_iter, iters, trace, trace_cap);
}

/* oracle_pivot: Steps 4-5 alone, on the element (l, k) of the
 * (m+1) x (ncols+1) tableau T (any nonzero T[l,k], either sign), in place. */
int oracle_pivot(int64_t m, int64_t ncols, double *T, int64_t l, int64_t k) {
    if (m < 1 || ncols < 1 || !T || l < 0 || l >= m || k < 0 || k >= ncols) return ORC_ERR_ARG;
    pivot_on(m + 1, ncols + 1, T, l, k);
    return 0;
}

/* oracle_price_out: makes the objective row (row m) zero in every basic
 * column, as Step 5 does when a column enters: for each row i in ascending
 * order, with f the objective-row entry of basis[i]'s column, if f != 0 the
 * objective row becomes fma(-f, row i, objective row), element by element
 * over all ncols+1 columns (row i holds 1 in that column). */
int oracle_price_out(int64_t m, int64_t ncols, double *T, const int64_t *basis) {
    if (m < 0 || ncols < 1 || !T || (m > 0 && !basis)) return ORC_ERR_ARG;
    const int64_t W = ncols + 1;
    for (int64_t i = 0; i < m; ++i) {
        const double g = TAB(T, W, m, basis[i]);
        if (g == 0.0) continue;
        for (int64_t j = 0; j < W; ++j) TAB(T, W, m, j) = fma(-g, TAB(T, W, i, j), TAB(T, W, m, j));
    }
    return 0;
}

/* oracle_threads: with the OpenMP build, sets the number of threads Step 5
 * uses (n > 0); returns the number it will use (1 in the serial build). */
int oracle_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
