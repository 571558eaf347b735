/*
 * lpdense: dense-tableau simplex for AMD Instinct MI355X (gfx950), C ABI.
 *
 * Problem (Coutinho et al., Section 2, eq. 1 in canonical <= form):
 *
 *     maximize  c^T x   subject to  A x <= b,  x >= 0,   with b >= 0,
 *
 * solved by the standard simplex method on the full (m+1) x (n+m+1) tableau
 * of Table 1 (constraint rows [A_i | e_i | b_i], objective row [-c | 0 | 0]),
 * starting from the slack basis.  One pivot (Section 2, Steps 2-5) is:
 *   Step 2  Dantzig pricing: entering column k = the lowest index j < n+m
 *           minimising the objective-row entry T[m,j]; optimal when
 *           T[m,k] >= -eps_d.
 *   Step 3  ratio test over rows i < m with T[i,k] > eps_p:
 *           rho_i = T[i,rhs] / T[i,k]; leaving row l = lowest i minimising
 *           rho_i; no eligible row means the LP is unbounded.
 *   Step 4  pivot row r = T[l,:] / T[l,k] (IEEE division).
 *   Step 5  every other row, objective row included:
 *           T[i,j] <- fma(-T[i,k], r_j, T[i,j]) (multiplier read before the
 *           row changes; one rounding per element).
 * Loop order per iteration: price -> optimal? -> iteration cap? -> ratio
 * test -> unbounded? -> pivot.  Non-finite input, or a non-finite value seen
 * by the pricing scan or by the ratio test, gives LPD_NUMERICAL; a negative
 * b_i gives LPD_INFEASIBLE_START before any pivot (the slack basis of
 * Section 2 needs b >= 0).  Every result is deterministic: for the same
 * inputs and options the outputs are bitwise identical on every call, for
 * every schedule, grid size and batch composition.
 *
 * Memory and ownership.  Unless a comment says "host", every pointer argument
 * is a DEVICE pointer on the current HIP device, and the caller owns it.
 * Matrices are row-major with leading dimension equal to their column count.
 * All solve calls are stream-ordered and asynchronous: they validate their
 * arguments on the host, enqueue work on `stream` and return; outputs are
 * valid once `stream` has completed, and the caller keeps every buffer alive
 * until then.  Workspace is allocated and freed stream-ordered on `stream`
 * (hipMallocAsync / hipFreeAsync) and belongs to the library.
 *
 * Errors.  A negative return value (lpd_error) means nothing was enqueued and
 * no output was written.  Data-dependent outcomes are not errors: they are
 * the lpd_status value written to the device-side `status` output.  On any
 * status other than LPD_OPTIMAL, x / obj / y describe the last basis reached.
 *
 * Thread safety: calls on distinct streams may run concurrently; the library
 * keeps no mutable global state apart from per-device launch limits that are
 * computed once.
 *
 * Processes: the grid schedules, lp_solve_batch and the server launch
 * cooperatively (every workgroup co-resident).  Use one process per device
 * for them: a second process's grid launch was seen to fail with
 * LPD_ERR_HIP once another process had launched cooperatively on the same
 * device.
 */
#ifndef LPDENSE_H
#define LPDENSE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Outcome of a solve, written to the device `status` output (int32). */
typedef enum lpd_status {
    LPD_OPTIMAL = 0,          /* no reduced cost below -eps_d */
    LPD_UNBOUNDED = 1,        /* entering column has no entry > eps_p */
    LPD_ITERATION_LIMIT = 2,  /* max_iter pivots done, not yet optimal */
    LPD_INFEASIBLE_START = 3, /* some b_i < 0: slack basis infeasible */
    LPD_NUMERICAL = 4,        /* NaN/Inf in the input or met while pivoting */
    LPD_DEVICE_TIMEOUT = 5,   /* a barrier wait of the persistent grid kernel did not
                                 complete within its watchdog time (lpd_options.watchdog_us,
                                 default 10 s): every workgroup gave up and the kernel
                                 returned.  Only `status` is valid then; x, obj, y,
                                 iterations, trace, basis and tableau are undefined.  Not
                                 expected in normal use. */
    LPD_INFEASIBLE = 6        /* lp_solve_general only: phase I ends with artificial
                                 variables left positive, no feasible point */
} lpd_status;

/* Synchronous argument / launch errors (negative return values). */
typedef enum lpd_error {
    LPD_SUCCESS = 0,
    LPD_ERR_INVALID_ARG = -1,   /* m < 1, n < 1, bad option value */
    LPD_ERR_NULL_POINTER = -2,  /* a required pointer is NULL */
    LPD_ERR_SIZE_OVERFLOW = -3, /* sizes overflow the index types */
    LPD_ERR_OUT_OF_MEMORY = -4, /* workspace does not fit on the device */
    LPD_ERR_HIP = -5,           /* a HIP runtime call or launch failed */
    LPD_ERR_DEVICE = -6,        /* no usable gfx950 device is current */
    LPD_ERR_TOO_LARGE = -7,     /* request exceeds a configured budget */
    LPD_ERR_NOT_FOUND = -8      /* unknown handle or request id */
} lpd_error;

/* Defaults used when an option is left at 0 / negative. */
#define LPD_DEFAULT_EPS 1e-9
/* Default iteration cap: 50 * (m + n). */

/* Schedules for the single-LP solve. */
typedef enum lpd_schedule {
    LPD_SCHED_AUTO = 0,       /* library picks (workgroup if the tableau fits in LDS) */
    LPD_SCHED_WORKGROUP = 1,  /* one workgroup runs the whole pivot loop */
    LPD_SCHED_GRID = 2,       /* persistent cooperative grid, one grid barrier per pivot */
    LPD_SCHED_GRID_CONDENSED = 3, /* the grid schedule on the condensed tableau: only the n
                                    columns of the nonbasic variables are stored and updated
                                    (the m basic columns of the full tableau are unit columns).
                                    Every output, the reconstructed full tableau included, is
                                    bitwise identical to the other schedules; a pivot moves
                                    16 (m+1)(n+1) bytes instead of 16 (m+1)(n+m+1) */
    LPD_SCHED_GRID_PAIRED = 4, /* the grid schedule with two pivots per sweep of the full
                                 tableau: the second pivot's entering column, ratio test and
                                 normalised row are formed before the sweep, which then applies
                                 both rank-1 updates to each element (the same roundings as two
                                 sweeps: every output is bitwise identical to the other
                                 schedules), moving about 8 (m+1)(n+m+1) bytes per pivot */
    LPD_SCHED_GRID_CONDENSED_PAIRED = 5 /* two pivots per sweep of the condensed tableau: both
                                           savings together, about 8 (m+1)(n+1) bytes per
                                           pivot, every output bitwise identical */
} lpd_schedule;

/*
 * lp_solve_dense: solve one LP with default options.
 *   m, n    number of constraints / structural variables (>= 1, host values)
 *   A       m*n row-major, b length m, c length n               (device, in)
 *   x       length n (out); obj, status: one double / one int32  (device, out)
 *   stream  HIP stream the work is enqueued on (0 = null stream)
 * Returns LPD_SUCCESS or a negative lpd_error.
 */
int lp_solve_dense(int64_t m, int64_t n, const double *A, const double *b, const double *c,
                   double *x, double *obj, int32_t *status, hipStream_t stream);

/* Problem description for lp_solve_dense_ex (all device pointers). */
typedef struct lpd_problem {
    int64_t m, n;
    const double *A; /* m*n row-major */
    const double *b; /* m */
    const double *c; /* n */
} lpd_problem;

/* Options (host struct; zero-initialise for defaults). */
typedef struct lpd_options {
    double eps_d;      /* optimality tolerance (<= 0: 1e-9) */
    double eps_p;      /* ratio-test pivot tolerance (<= 0: 1e-9) */
    int64_t max_iter;  /* pivot cap (< 0: 50*(m+n); 0 allowed) */
    int32_t schedule;  /* lpd_schedule */
    int32_t grid_blocks; /* grid schedule: workgroups to launch (0: one per 160 KiB of stored tableau,
                            in multiples of 8, at least 64 and at most one per CU; always capped
                            by co-residency) */
    int64_t watchdog_us; /* grid schedules: bound of every barrier wait in microseconds, after which
                            the solve gives up with LPD_DEVICE_TIMEOUT (0: 10 s; < 0: no wait at
                            all, every barrier gives up at once -- for tests of that path) */
} lpd_options;

/* Outputs (device pointers; NULL skips an optional output). */
typedef struct lpd_outputs {
    double *x;           /* n, required */
    double *obj;         /* 1, required */
    int32_t *status;     /* 1, required (lpd_status) */
    double *y;           /* m, optional: duals T[m, n+i] of the final tableau */
    int64_t *iterations; /* 1, optional: pivots performed */
    int32_t *trace;      /* 2*trace_cap, optional: (k, l) of each pivot, in order */
    int64_t trace_cap;   /* capacity of trace in pivots */
    int64_t *basis;      /* m, optional: basic variable of each row (0..n+m-1) */
    double *tableau;     /* (m+1)*(n+m+1), optional: final tableau, Table 1 layout */
    uint64_t *phase_ticks; /* 8*phase_cap, optional (grid schedules only, diagnostics):
                              readings of the device's 100 MHz real-time clock, one
                              entry of 8 per sweep, at the index of the sweep's first
                              pivot: [0] sweep start, [1] pricing done, [2] workgroup
                              0's update share done, [3] latest arrival of any
                              workgroup at the sweep's barrier, [4] latest publication
                              after its release fence, [5] workgroup 0 saw every
                              arrival, [6] barrier reduction done, [7] (two pivots per
                              sweep only) end of the wait at the pair's publication
                              barrier.  Entries [0]-[6] of every sweep are written
                              ([3] and [4] zeroed by workgroup 0, then raised to the
                              maximum), so they need no initialisation; [7] on the
                              one-pivot schedules, and the whole entry of a sweep's
                              second pivot on the paired ones, are left untouched.
                              Untouched on the workgroup schedule. */
    int64_t phase_cap;     /* capacity of phase_ticks in pivots */
} lpd_outputs;

/* The same struct under the name lpd_result. */
typedef lpd_outputs lpd_result;

/*
 * lp_solve_dense_ex: solve one LP with options and optional outputs.
 * `prob`, `opt` and `out` are host structs read during the call; `opt` may be
 * NULL for defaults.  Same semantics, errors and ownership as lp_solve_dense.
 * Sizes: LPD_SCHED_WORKGROUP needs the whole tableau in one workgroup's LDS
 * (else LPD_ERR_TOO_LARGE); the grid schedules take any size whose workspace
 * (about 8 (m+1)(n+m+1) bytes, or 8 (m+1)(n+1) condensed) fits in device
 * memory (else LPD_ERR_OUT_OF_MEMORY): a pivot row longer than the LDS holds
 * is swept in column panels, with the same results.  The two paired
 * schedules add one row and one column of the tableau, and one row per
 * workgroup (m + (nblocks + 1) (n + m + 1) doubles, n + 1 condensed).
 */
int lp_solve_dense_ex(const lpd_problem *prob, const lpd_options *opt, const lpd_outputs *out,
                      hipStream_t stream);

/*
 * lp_solve_dense_noalloc: lp_solve_dense_ex for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results (bitwise), errors and
 * stream ordering as lp_solve_dense_ex, but no allocation of any kind: the
 * grid schedules take their workspace from a fixed 128 MiB device array
 * that the library holds on every device it runs on until the process ends
 * (looked up on the first call on each device).  A problem whose workspace
 * (lpd_workspace_bytes, or the paired schedules' larger one) exceeds 128 MiB
 * returns LPD_ERR_TOO_LARGE with nothing enqueued: about m = n = 2,800 on the
 * full tableau, m = n = 4,000 on the condensed one.  LPs whose tableau fits
 * in LDS need no workspace and have no size limit beyond lp_solve_dense_ex's.
 * Every call on a device uses the same array: calls whose work overlaps on
 * one device (different streams, or other host threads) race and corrupt
 * each other's results; serialise them, e.g. on one stream.  The array
 * keeps the last call's contents; the kernels reset what must start at zero.
 */
int lp_solve_dense_noalloc(const lpd_problem *prob, const lpd_options *opt, const lpd_outputs *out,
                           hipStream_t stream);

/* Options of a batched solve (host struct; zero-initialise for defaults). */
typedef struct lpd_batch_options {
    double eps_d;            /* as lpd_options, for every LP (<= 0: 1e-9) */
    double eps_p;
    int64_t max_iter;        /* per LP; < 0: 50*(m_i+n_i); 0 allowed */
    int32_t team_size;       /* workgroups per team for large LPs: > 1 one fixed size for
                                all of them, 1 no teams, 0 sized per LP if
                                team_bytes_per_wg > 0, else the autotune table's choice
                                (built-in default: sized per LP) */
    int32_t grid_blocks;     /* workgroups of the launch (0: one per CU) */
    int64_t team_min_bytes;  /* tableau bytes from which an LP is solved by a team
                                (0: autotune table; < 0: never) */
    int64_t *iterations;     /* device, count entries, optional: pivots of each LP */
    int64_t team_bytes_per_wg; /* per-LP sizing: an LP of B tableau bytes gets a team of
                                  the largest power of two <= B / team_bytes_per_wg
                                  workgroups, capped by the grid (0: autotune table) */
    int32_t wave_slots;      /* wave-per-instance: each workgroup's LDS is split into this
                                many slices (<= 16) and an LP whose LDS tableau fits in one
                                slice is solved by a single wave (0: autotune table, whose
                                built-in default is off; < 0: off) */
    int32_t full_tableau;    /* 0: LPs solved by a grid walk (team or one workgroup) store
                                the condensed tableau (LPD_SCHED_GRID_CONDENSED: the same
                                bits, fewer bytes per pivot); nonzero: the full tableau */
} lpd_batch_options;

/*
 * lp_solve_batch: solve `count` independent LPs (max c_i^T x s.t. A_i x <= b_i,
 * x >= 0) in one persistent launch.  Each LP follows exactly the rules of
 * lp_solve_dense and its x / obj / status are bit-identical to what
 * lp_solve_dense returns for it alone, for any batch composition and order.
 *   count              number of LPs (>= 1)
 *   m, n               host arrays of count sizes (each >= 1)
 *   A_pack, b_pack,    device arrays holding every LP's A (row-major, m_i*n_i),
 *   c_pack               b (m_i) and c (n_i) back to back
 *   A_off, b_off,      host arrays of count element offsets into the packs
 *   c_off
 *   x_pack, x_off      device output pack and host offsets (n_i entries each)
 *   obj, status        device outputs, count entries each
 *   opt                may be NULL (defaults)
 * LPs whose tableau fits in a wave's slice of LDS (wave_slots) are solved by
 * one wave each; others whose tableau fits in LDS by one workgroup in LDS;
 * larger ones by one workgroup over HBM, or by a team of workgroups if the
 * tableau is at least team_min_bytes.  Large LPs are started first.  An LP
 * whose pivot row (n + m + 1 doubles, n + 1 condensed) does not fit in LDS
 * beside the reduction scratch (about 20,000 doubles on gfx950) is solved
 * after the batched launch, alone on the grid schedule with two pivots per
 * sweep (as lp_solve_dense_ex, same results), on the same stream.  Returns
 * LPD_SUCCESS or a negative lpd_error; asynchronous and stream-ordered like
 * lp_solve_dense.  Host arrays are only read during the call.
 */
int lp_solve_batch(int32_t count, const int64_t *m, const int64_t *n, const double *A_pack,
                   const int64_t *A_off, const double *b_pack, const int64_t *b_off, const double *c_pack,
                   const int64_t *c_off, double *x_pack, const int64_t *x_off, double *obj, int32_t *status,
                   const lpd_batch_options *opt, hipStream_t stream);

/*
 * Serving runtime (continuous batching).  A server owns one HIP stream on
 * `device` and a worker thread.  LPs submitted from any host thread wait in
 * arrival order; one is admitted (made resident in HBM) as soon as its
 * footprint fits in what the budget has left and a resident slot is free.
 * Admission never lets the footprints of resident LPs exceed the budget.
 * The worker repeats epochs: admit what fits, then run one batched launch
 * (the schedule of lp_solve_batch) in which every resident LP advances by at
 * most `pivots_per_epoch` pivots, its tableau staying in HBM between epochs
 * (an LP whose tableau fits in LDS is solved to the end within one epoch;
 * an LP whose pivot row is longer than lp_solve_batch can batch gets a grid
 * launch of its own in each epoch, after the batched one).
 * LPs that finished leave, their memory returns to the budget and their
 * completion is queued.  Requests that arrive while others run therefore
 * share the device with them.  Each LP performs exactly the pivots of its own
 * lp_solve_dense call, so x / obj / status / iterations are bit-identical to
 * a solve of it alone, whatever else is resident.
 *
 * Inputs of requests admitted while an epoch runs are copied on a second
 * stream and join the next epoch.
 *
 * Footprint of an m x n request: every device byte it holds while resident,
 * the tableau workspace (8 (m+1)(n+1) bytes on the condensed tableau,
 * 8 (m+1)(n+m+1) on the full one, rows padded to 32 doubles) plus a copy of
 * A, b, c and x.  LPs whose tableau fits in LDS need no
 * tableau workspace.
 */
typedef struct lpd_server lpd_server;

/* Server options (host struct; zero-initialise for defaults). */
typedef struct lpd_server_options {
    double eps_d;              /* as lpd_options (<= 0: 1e-9) */
    double eps_p;
    int64_t max_iter;          /* per LP (0 or < 0: 50*(m+n)) */
    int64_t pivots_per_epoch;  /* pivots each resident LP may do per launch; <= 0: sized
                                  per LP so that every workgroup streams about
                                  epoch_bytes_per_wg tableau bytes per launch */
    int32_t max_resident;      /* most LPs resident at once (<= 0: 4096) */
    int32_t full_tableau;      /* as lpd_batch_options (0: condensed tableau) */
    int64_t team_min_bytes;    /* tableau bytes from which an LP may get a team
                                  (0: twice team_bytes_per_wg; < 0: never) */
    int64_t team_bytes_per_wg; /* least tableau bytes per workgroup of a team (<= 0:
                                  256 KiB); workgroups are shared out in proportion to
                                  the tableau bytes of the resident LPs */
    int64_t epoch_bytes_per_wg; /* see pivots_per_epoch (<= 0: 256 MiB) */
    int64_t admit_bytes_per_round; /* input bytes copied per admission step at most
                                      (at least one request; <= 0: 512 MiB) */
} lpd_server_options;

/* One finished request, as returned by lpd_server_poll. */
typedef struct lpd_completion {
    int64_t id;          /* value lpd_server_submit returned */
    int32_t status;      /* lpd_status, or a negative lpd_error if the request failed
                            (e.g. LPD_ERR_OUT_OF_MEMORY, LPD_ERR_HIP) */
    int32_t reserved;
    double obj;          /* objective value c^T x */
    int64_t iterations;  /* pivots performed */
    int64_t m, n;
    double *x;           /* the caller's x_out buffer, now holding x (host) */
    double t_arrive;     /* seconds since server creation: submit returned ... */
    double t_admit;      /* ... admitted to the device ... */
    double t_done;       /* ... result in x_out and completion queued */
} lpd_completion;

/* Counters of a server (host struct). */
typedef struct lpd_server_stats {
    int64_t submitted, completed, epochs;
    int64_t resident, waiting;  /* at the last admission step */
    uint64_t used_bytes;        /* footprint of the resident LPs now */
    uint64_t peak_bytes;        /* largest used_bytes ever reached */
    uint64_t budget_bytes;
    uint64_t copy_bytes;        /* input bytes copied to the device so far */
    double kernel_seconds;      /* device time of the epoch launches (HIP events) */
    double admit_host_seconds;  /* worker time spent issuing admission copies */
} lpd_server_stats;

/* Creates a server on HIP device `device` with a footprint budget in bytes.
 * `opt` may be NULL.  Returns NULL if the device is not a usable gfx950 or a
 * device allocation fails. */
lpd_server *lpd_server_create(int device, uint64_t budget_bytes, const lpd_server_options *opt);

/* Queues one LP.  A, b, c (m*n row-major, m, n) and x_out (n) are HOST
 * arrays owned by the caller; they must stay valid, and A, b, c unchanged,
 * until the completion of this request has been returned by lpd_server_poll.
 * Returns the request id (> 0), or a negative lpd_error: LPD_ERR_INVALID_ARG
 * (m or n < 1), LPD_ERR_NULL_POINTER, LPD_ERR_SIZE_OVERFLOW,
 * LPD_ERR_TOO_LARGE (footprint above the whole budget), LPD_ERR_NOT_FOUND
 * (null or stopping server).  Thread-safe. */
int64_t lpd_server_submit(lpd_server *server, int64_t m, int64_t n, const double *A, const double *b,
                          const double *c, double *x_out);

/* Moves up to `max` completions, oldest first, into `out` (host array) and
 * returns how many; never blocks.  Thread-safe. */
int lpd_server_poll(lpd_server *server, lpd_completion *out, int max);

/* Copies the server's counters into `out` (host).  Thread-safe. */
int lpd_server_get_stats(lpd_server *server, lpd_server_stats *out);

/* Finishes every submitted request (their completions are then dropped),
 * stops the worker and frees the server. */
void lpd_server_destroy(lpd_server *server);

/*
 * lp_solve_tableau: Steps 2-5 (Section 2, iterated as in Section 3) from a
 * given basic tableau instead of Table 1: a warm start from any basis, and
 * the building block of lp_solve_general's two phases.
 *   m       constraint rows (>= 1, host)
 *   ncols   variable columns (>= m, host).  The tableau has m + 1 rows, the
 *           last being the objective row in Table 1's sign convention
 *           (reduced costs, minimised by pricing; its RHS is the objective
 *           value), and ncols + 1 columns, the last being the RHS.
 *   T0      (m+1) x (ncols+1) row-major (device, read only; not modified)
 *   basis0  HOST array of m column indices, the basic variable of each row:
 *           distinct and in [0, ncols) (else LPD_ERR_INVALID_ARG, nothing
 *           enqueued); read during the call only.  Each one's column must be
 *           the unit vector of its row with objective-row entry 0 (not
 *           checked: the caller states a basic tableau).
 *   opt     as lp_solve_dense_ex; the default iteration cap is 50 ncols
 *   out     x: ncols entries, the value of every column's variable (its
 *           row's RHS if basic, else 0); obj: the objective row's final RHS;
 *           status, iterations, trace ((k, l) with k a column of T0), basis
 *           (m), tableau ((m+1) x (ncols+1)), phase_ticks: as in
 *           lp_solve_dense_ex; y must be NULL (LPD_ERR_INVALID_ARG).
 * The right-hand side is used as stored, with no sign check (a start that is
 * not primal feasible is the caller's choice).  A non-finite entry anywhere
 * in T0 gives LPD_NUMERICAL with no pivot.  Every schedule applies: on the
 * condensed ones the stored columns are the nonbasic ones in increasing
 * order, pricing ties still go to the lowest column of T0, and all outputs
 * are bitwise those of the full tableau.  Asynchronous and stream-ordered
 * like lp_solve_dense_ex (the index arrays derived from basis0 are copied to
 * the device on `stream`).
 */
int lp_solve_tableau(int64_t m, int64_t ncols, const double *T0, const int64_t *basis0,
                     const lpd_options *opt, const lpd_outputs *out, hipStream_t stream);

/*
 * General LPs (two-phase method).  Section 2 states the problem with rows
 * A x = b and treats the canonical <= form with b >= 0, where the slack basis
 * is a feasible start.  lp_solve_general accepts rows of any sense and
 * right-hand sides of any sign:
 *
 *     maximize c^T x  subject to  A_i x (<=, =, >=) b_i,  x >= 0,
 *
 * by the textbook two-phase method on the pivot kernels (lp_solve_tableau):
 *  1. Row i is multiplied by -1 when b_i < 0, or when b_i = 0 and the row
 *     reads >=, so that every right-hand side is >= 0.
 *  2. Columns, in Table 1's layout: the n variables; one surplus column (-1)
 *     per row that now reads >=, in row order; one column per row holding
 *     the variable that starts basic there: its slack (<= rows) or an
 *     artificial variable (>= and = rows); the RHS.
 *  3. Phase I maximises minus the sum of the artificial variables: the
 *     objective row is +1 in the artificial columns, those basic columns
 *     then eliminated from it (Step 5 on the objective row, rows in order).
 *     Steps 2-5 run to a status.
 *  4. The LP is feasible iff phase I ends optimal at a value >= -1e-9 *
 *     max(1, sum of the artificial rows' right-hand sides); else the status
 *     is LPD_INFEASIBLE.
 *  5. Each artificial variable still basic (rows in order) is driven out by
 *     a pivot (Steps 4-5) on the lowest non-artificial column whose entry in
 *     its row exceeds eps_p in magnitude; a row with none is redundant.
 *  6. Phase II: the artificial columns and the redundant rows are deleted,
 *     the objective row becomes [-c | 0 | 0] with the basic columns
 *     eliminated from it, and Steps 2-5 run to a status.
 *  7. x_j is the RHS of x_j's row if basic, else 0; obj is the objective
 *     row's RHS.  When phase II is not reached, x is phase I's and obj =
 *     sum_j c_j x_j in index order.
 *
 *   m, n        sizes (host)
 *   A, b, c     device arrays, as lp_solve_dense (b of any sign)
 *   sense       host array of m lpd_row_sense values, or NULL for all <=
 *   opt         may be NULL; schedule, eps and max_iter apply to each phase
 *               (default cap 50 (m + n) per phase)
 *   x, obj, status  device outputs (x: n entries)
 *   iterations  optional device output: pivots of phase I, of the drive-out
 *               and of phase II
 * Unlike the other solve calls this one synchronises `stream`: the layout of
 * phase II depends on phase I's basis.  Returns LPD_SUCCESS or an lpd_error.
 */
typedef enum lpd_row_sense {
    LPD_ROW_LE = 0,
    LPD_ROW_EQ = 1,
    LPD_ROW_GE = 2
} lpd_row_sense;

int lp_solve_general(int64_t m, int64_t n, const double *A, const double *b, const double *c,
                     const int8_t *sense, const lpd_options *opt, double *x, double *obj,
                     int32_t *status, int64_t *iterations, hipStream_t stream);

/* Device workspace (bytes) a single solve of an m x n LP allocates on the
 * default schedule (0 when the tableau fits in one workgroup's LDS).  The
 * paired schedules take (nblocks + 1) (n + m + 1) + m more doubles (see
 * lp_solve_dense_ex). */
uint64_t lpd_workspace_bytes(int64_t m, int64_t n);

/* Static strings for an lpd_error / lpd_status code ("unknown" otherwise). */
const char *lpd_error_string(int code);
const char *lpd_status_string(int32_t status);

/* Library version as major*10000 + minor*100 + patch. */
int lpd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LPDENSE_H */
