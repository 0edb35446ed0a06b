/*
 * pdcs.h -- C ABI of the MI355X (gfx950) PDCS linear-programming solver.
 *
 * Problem solved (Section 1.1, eq. prob_cp, with box-bounded variables):
 *
 *     min  c^T x   s.t.  (G x - h)_i  = 0   for i <  m_zero      (zero cone)
 *                        (G x - h)_i >= 0   for the next rows     (nonnegative cone)
 *                        (G x - h)_B in K_soc for each second-order-cone block B,
 *                                   then in K_exp and in K_exp* for the exponential
 *                                   and dual-exponential blocks of 3 rows, the last
 *                                   rows (pdcs_problem_create_conic / _cones)
 *                        l <= x <= u                            (box, +-inf allowed)
 *
 * with its dual (eq. dual_conic): max h^T y + l^T lam+ - u^T lam-, lam = c - G^T y,
 * y in K_d = R^m_zero x R+^... x K_soc x ... x K_exp* x ... x K_exp x ... (the dual
 * cone of each row block; the second-order cone is self-dual).
 * The method is "PDCS with preconditioning" (Section 2.6): diagonal rescaling,
 * then the restarted, line-searched, reflected-Halpern PDHG loop of Algorithm 1
 * (Function 2 for the step size, Section 2.2 for the reflection parameter,
 * Section 2.3 / Algorithm 3 for restarts, Section 2.5 for the primal weight),
 * then unscaling.  Every step of the loop runs in HIP kernels on the GPU.
 *
 * Conventions
 *  - Every function returns an int status: PDCS_OK (0) or a negative PDCS_ERR_*.
 *    Solver outcomes are NOT errors; they are the exit codes of the paper's
 *    exit-code table (Section 3), reported in pdcs_info.exit_code.
 *  - Host input arrays are copied during the call; the caller keeps ownership.
 *  - Handles (problem, result, batch, mlp) are owned by the library until the
 *    matching *_destroy call.  A handle must not be used from two threads at once.
 *  - +-infinity bounds are IEEE infinities.  NaN anywhere in the data is an error.
 *  - "stream" arguments are a hipStream_t passed as void*.  The device-pointer
 *    calls (pdcs_problem_spmv, pdcs_mlp_*) are enqueued on that stream, NULL
 *    meaning the HIP null stream, which is ordered with the caller's work on
 *    blocking streams (e.g. PyTorch's default stream).  Solve calls run on the
 *    library's own stream and are synchronous: they return with results on host.
 *  - pdcs_last_error() returns a static string describing the last failure of
 *    the calling thread.
 */
#ifndef PDCS_H
#define PDCS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define PDCS_OK               0
#define PDCS_ERR_INVALID_ARG (-1)  /* null pointer, malformed CSR, NaN, l > u, bad sizes */
#define PDCS_ERR_UNSUPPORTED (-2)  /* a request this library does not implement        */
#define PDCS_ERR_OOM         (-3)  /* device or host allocation failed                  */
#define PDCS_ERR_HIP         (-4)  /* a HIP runtime call failed                          */
#define PDCS_ERR_SIZE        (-5)  /* problem too large for 32-bit device indexing       */
#define PDCS_ERR_STATE       (-6)  /* handle used in a state that does not allow the call */

/* ---- exit codes: exit-code table of Section 3 --------------------------- */
#define PDCS_EXIT_OPTIMAL                   0
#define PDCS_EXIT_MAX_ITER                  1
#define PDCS_EXIT_PRIMAL_INFEASIBLE_LOW_ACC 2
#define PDCS_EXIT_PRIMAL_INFEASIBLE_HIGH_ACC 3
#define PDCS_EXIT_DUAL_INFEASIBLE_LOW_ACC   4
#define PDCS_EXIT_DUAL_INFEASIBLE_HIGH_ACC  5
#define PDCS_EXIT_TIME_LIMIT                6
#define PDCS_EXIT_CONTINUE                  7
#define PDCS_EXIT_NUMERICAL_ERROR           8

/* ---- candidate rule ("method" option of Section 3) ---------------------- */
#define PDCS_METHOD_AUTO    0   /* smaller normalized duality gap (Section 2.3) */
#define PDCS_METHOD_AVERAGE 1   /* eta-weighted average of the interval          */
#define PDCS_METHOD_HALPERN 2   /* latest PDHG output                            */

/* ---- precision ---------------------------------------------------------- */
#define PDCS_PRECISION_FP64  0  /* FP64 values and iterates throughout              */
#define PDCS_PRECISION_MIXED 1  /* FP32 values, iterates and SpMV; FP64 reductions,
                                   scalars, restart decisions, termination checks
                                   (FP64 values) and an FP64 polish phase           */

typedef struct pdcs_problem_s* pdcs_problem;
typedef struct pdcs_result_s*  pdcs_result;
typedef struct pdcs_batch_s*   pdcs_batch;
typedef struct pdcs_mlp_s*     pdcs_mlp;

/* Solver options.  Defaults (pdcs_options_default) follow the option list of
 * Section 3 where the paper gives one. All fields are 8 bytes wide. */
typedef struct {
  double  rel_tol;            /* 1e-6: eq. PDCS_terminate_tolerance_rel                */
  double  abs_tol;            /* 1e-6: eq. PDCS_terminate_tolerance_abs                */
  double  time_limit;         /* 1000 s: exit code 6                                  */
  int64_t max_iter;           /* trial budget (every PDHG trial counts): exit code 1   */
  int64_t use_preconditioner; /* 1: diagonal rescaling (Section 2.6)                   */
  int64_t ruiz_iters;         /* 10 Ruiz passes (the paper does not fix the scaling)   */
  int64_t l2_pass;            /* 1: one sqrt-L2-norm pass after Ruiz                    */
  int64_t method;             /* PDCS_METHOD_*                                        */
  int64_t check_every;        /* 64: restart/termination check after every accepted
                                 trial whose trial count is a multiple of this         */
  int64_t precision;          /* PDCS_PRECISION_*                                     */
  int64_t stall_checks;       /* 512; mixed: switch to FP64 after this many checks
                                 without a 10% improvement of the relative KKT error
                                 once that error is below 100 * rel_tol, or after 8x
                                 this many checks without a new lowest error at any
                                 level (0: never)                                     */
  double  polish_switch_tol;  /* mixed: switch to FP64 once rel. KKT <= this (0: off)  */
  double  bisect_rel_eps;     /* 1e-6: relative bracket width of the gap bisection     */
  int64_t use_graph;          /* 1: replay each chunk of iterations as a hipGraph      */
  int64_t verbose;            /* 0: silent; 1: a line per print_freq trials for
                                 instance 0 (on stderr); 2: a line per check           */
  int64_t keep_state;         /* 1: keep the internal iterates for pdcs_result_state   */
  int64_t time_kernels;       /* 1: launch without graphs and time every launch of the
                                 SpMV-with-dual-step kernel with HIP events           */
  int64_t probe_passes;       /* 7: multisection passes per restart check (16 t each)  */
  int64_t trace_trials;       /* record the scalars of the first this-many trials      */
  int64_t compact;            /* 1: a batch of >= 8 LPs rebuilds its schedules over the
                                 still-active instances each time half of them have
                                 finished (results are identical either way)          */
  int64_t use_kkt_restart;    /* 0; 1: candidates are compared and the restart rules
                                 evaluated on KKT_omega instead of the normalized
                                 duality gap (Section 2.3, option use_kkt_restart)    */
  int64_t use_duality_gap_restart; /* 1: the normalized duality gap is the restart
                                 metric (with the KKT_omega fallback of Section 2.3);
                                 0: KKT_omega is, and the gap is not computed.
                                 use_kkt_restart = 1 also selects KKT_omega          */
  int64_t kkt_restart_freq;   /* trials between checks while KKT_omega is the metric;
                                 0 (default): check_every                             */
  int64_t duality_gap_restart_freq; /* trials between checks while the gap is the
                                 metric; 0 (default): check_every                     */
  int64_t print_freq;         /* verbose = 1: one progress line per this many trials
                                 (2000, as in the option list of Section 3)           */
  /* Infeasibility tolerances of the option list of Section 3 (exit codes 2-5).
   * Each test runs at every check that does not terminate, on the rays
   * r_x = Proj(D2 (x_hat - x_start)) and r_y = Proj(D1 (y_hat - y_start)): the
   * displacement of the PDHG output from the projected start point, unscaled and
   * projected onto the recession cone of the box and onto K_d.  With
   * lam = -G^T r_y and f = h^T r_y + sum_{l finite} l lam+ - sum_{u finite} u lam-:
   *   ratio_p = ||lam - Proj_Lambda(lam)||_2 / f,
   *   ratio_d = ||G r_x - Proj_{K_d*}(G r_x)||_2 / (-c^T r_x),
   * each +inf unless its denominator exceeds the rounding bound gamma_N = Nu/(1-Nu)
   * of its own sum times the sum of its terms' magnitudes.  High accuracy: exit
   * 3 (5) when ratio_p (ratio_d) < the tolerance.  Low accuracy: exit 2 (4)
   * once ratio_p (ratio_d) was below the tolerance at 3 consecutive checks at
   * which the dual objective (the negated primal objective) of the PDHG output
   * rose strictly.  0 switches a test off.                                          */
  double  eps_primal_infeasible_low_acc;   /* 1e-12 */
  double  eps_dual_infeasible_low_acc;     /* 1e-12 */
  double  eps_primal_infeasible_high_acc;  /* 1e-16 */
  double  eps_dual_infeasible_high_acc;    /* 1e-16 */
  int64_t reserved[4];
} pdcs_options;

/* Per-solve information (result fields of Section 3 plus counters). */
typedef struct {
  int64_t exit_code;          /* PDCS_EXIT_*                                          */
  int64_t iters;              /* trials (accepted + rejected), the paper's k-bar       */
  int64_t accepted_iters;
  int64_t restarts;
  int64_t checks;
  int64_t fp64_iters;         /* trials run in FP64 (all of them in FP64 mode)         */
  double  pobj, dobj;         /* c^T x and the dual objective at the returned point    */
  double  abs_p, abs_d, abs_gap;   /* infinity-norm errors, unscaled (Section 3)       */
  double  rel_p, rel_d, rel_gap;
  double  time_sec;           /* solve time: scaling + iterations + unscaling          */
  double  omega;              /* final primal weight                                  */
  double  eta_hat;            /* final step-size estimate                             */
  double  spmv_avg_ms;        /* time_kernels: mean duration of the SpMV+dual kernel   */
  int64_t spmv_launches;      /* time_kernels: number of launches timed                */
  double  reserved[4];
} pdcs_info;

/* Scalars of the internal state of a finished solve, in the rescaled space. */
typedef struct {
  double  omega, omega0, eta_hat, eta, beta, sum_eta;
  int64_t kbar, k, t, accepted;
  int64_t precision;          /* precision the iterates were in at exit               */
  double  rho_cur, rho_avg;   /* normalized duality gaps of the two restart candidates
                                 at the last check (Section 2.3)                      */
  double  r_cur, r_avg;       /* their radii ||z_c - z_anchor||_N                      */
  int64_t chosen;             /* candidate taken at the last check: 0 current, 1 average */
  double  ratio_p, ratio_d;   /* infeasibility ratios of the last check (see
                                 pdcs_options; NaN when the tests did not run)        */
  int64_t trend_p, trend_d;   /* consecutive checks passing the low-accuracy tests   */
} pdcs_state_scalars;

void        pdcs_options_default(pdcs_options* opts);
const char* pdcs_status_string(int exit_code);
const char* pdcs_last_error(void);
/* Number of visible GPUs (0 when none); never fails. */
int         pdcs_device_count(void);

/* ---- problems ----------------------------------------------------------
 * pdcs_problem_create: upload one LP (Section 1.1, eq. prob_cp, LP case).
 *   m, n       : rows and columns of G (m >= 0, n >= 1)
 *   m_zero     : rows [0, m_zero) are equalities, [m_zero, m) are ">=" rows
 *   row_ptr    : int64[m+1], nondecreasing, row_ptr[0] = 0, row_ptr[m] = nnz < 2^31
 *   col_idx    : int32[nnz], in [0, n), strictly increasing within a row
 *   val        : double[nnz], finite
 *   h          : double[m], finite;  c: double[n], finite
 *   l, u       : double[n], l <= u, l < +inf, u > -inf (NULL l means 0, NULL u means +inf)
 * All arrays are host memory, copied to the device; the transposed CSR is
 * built during the call.  Errors: PDCS_ERR_INVALID_ARG, PDCS_ERR_SIZE,
 * PDCS_ERR_OOM, PDCS_ERR_HIP.
 */
int  pdcs_problem_create(int64_t m, int64_t n, int64_t m_zero,
                         const int64_t* row_ptr, const int32_t* col_idx, const double* val,
                         const double* h, const double* c, const double* l, const double* u,
                         pdcs_problem* out);
/* pdcs_problem_create_conic: as pdcs_problem_create, with second-order-cone
 * row blocks (the socG option of Section 3): after the m_zero zero-cone rows
 * and the nonnegative-cone rows come n_soc blocks, block q holding the next
 * soc_dims[q] rows, with (G x - h)_block = (t, w) in K_soc = {||w|| <= t}
 * (Section 1.1, eq. prob_cp); the dual rows y_block lie in K_soc too (the cone
 * is self-dual).  After the diagonal rescaling a block's cones are
 * diag(D1) K_soc and diag(1/D1) K_soc, projected onto by a one-dimensional
 * root find (Section 2.6).  soc_dims is a host array of n_soc dimensions >= 1
 * with m_zero + sum(soc_dims) <= m, copied.  Problems with cone blocks always
 * take the band layout.  Errors: PDCS_ERR_INVALID_ARG as pdcs_problem_create,
 * and for a bad block list. */
int  pdcs_problem_create_conic(int64_t m, int64_t n, int64_t m_zero, int64_t n_soc,
                               const int64_t* soc_dims, const int64_t* row_ptr,
                               const int32_t* col_idx, const double* val,
                               const double* h, const double* c, const double* l,
                               const double* u, pdcs_problem* out);
/* pdcs_problem_create_cones: as pdcs_problem_create_conic, with exponential-
 * and dual-exponential-cone row blocks (the expG and dual_expG options of
 * Section 3) after the second-order-cone blocks: n_exp blocks of 3 rows with
 * (G x - h)_block = (x, y, z) in K_exp = closure {y > 0, y e^(x / y) <= z},
 * then n_dexp blocks of 3 rows in the dual cone K_exp* = closure
 * {(u, v, w): u < 0, -u e^(v / u) <= e w}, the last rows of the problem
 * (Section 1.1, eq. prob_cp).  The dual rows y_block lie in the dual cone of
 * each block (K_exp* for an exponential block, K_exp for a dual one); after
 * the diagonal rescaling a block's cones are diag(D1) K and diag(1/D1) K*,
 * projected onto by a one-dimensional root find (Section 2.6).  Needs
 * m_zero + sum(soc_dims) + 3 (n_exp + n_dexp) <= m; n_soc = 0 with soc_dims
 * null is allowed.  Problems with cone blocks always take the band layout
 * (pdcs_problem_set_layout does not change that).  Errors: as
 * pdcs_problem_create_conic. */
int  pdcs_problem_create_cones(int64_t m, int64_t n, int64_t m_zero, int64_t n_soc,
                               const int64_t* soc_dims, int64_t n_exp, int64_t n_dexp,
                               const int64_t* row_ptr, const int32_t* col_idx, const double* val,
                               const double* h, const double* c, const double* l,
                               const double* u, pdcs_problem* out);
/* pdcs_project_cone: the solver's projection onto a rescaled cone (Section
 * 2.6), for count vectors of dimension dim: out_q = Proj onto diag(f_q) K of
 * v_q, with K = K_soc = {(t, w): ||w|| <= t} (cone 0, any dim >= 1), K_exp
 * (cone 1, dim 3) or K_exp* (cone 2, dim 3).  v, f and out are host arrays of
 * dim * count doubles (vector q at [q dim, q dim + dim)), f > 0 and v finite;
 * the call copies them to the device, runs one wavefront per vector on the
 * current device (the device function the solver calls at its cone rows)
 * and copies the result back (synchronous).  count * dim <= 2^28.  kernel_ms
 * (host, may be null) receives the kernel's duration from HIP events around
 * its launch.  Errors: PDCS_ERR_INVALID_ARG, PDCS_ERR_SIZE, PDCS_ERR_OOM,
 * PDCS_ERR_HIP. */
int  pdcs_project_cone(int64_t cone, int64_t dim, int64_t count, const double* v, const double* f,
                       double* out, double* kernel_ms);
void pdcs_problem_destroy(pdcs_problem p);
int  pdcs_problem_dims(pdcs_problem p, int64_t* m, int64_t* n, int64_t* nnz);

/* pdcs_problem_spmv: one product with the UNSCALED matrix on device memory.
 *   transpose = 0: out[m] = G in[n];  transpose = 1: out[n] = G^T in[m].
 *   precision = PDCS_PRECISION_FP64: in/out are double*, FP64 values;
 *   precision = PDCS_PRECISION_MIXED: in/out are float*, FP32 values (row
 *               layout: FP64 accumulation; band layout: FP32 accumulation per
 *               window, FP64 sum of the window partials).
 * in_dev / out_dev are device pointers owned by the caller; the kernel is the
 * one the solver uses for its trial products under the problem's current
 * layout (pdcs_problem_set_layout), launched on `stream` and not synchronized;
 * the band layout also writes its own partial-sum buffer, so calls on one
 * problem must not overlap.  Errors: PDCS_ERR_INVALID_ARG. */
int  pdcs_problem_spmv(pdcs_problem p, int64_t transpose, int64_t precision,
                       const void* in_dev, void* out_dev, void* stream);

/* pdcs_problem_spmv_noalloc: pdcs_problem_spmv for callers that cannot
 * allocate device memory (code under HIP stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * pdcs_problem_spmv; the call allocates nothing, host or device.
 *   - The band layout's window partial sums go to a file-scope device array
 *     of 64 MiB (one per GPU, held until the process ends) instead of the
 *     problem's own buffer.  A product that needs more (P windows x R output
 *     rows x 4 B in FP32, x 8 B in FP64) fails with PDCS_ERR_SIZE.  The row
 *     layout uses no partial sums.
 *   - Every call on one GPU shares that array, which keeps the last call's
 *     contents: calls that overlap on one GPU race (use one stream, or order
 *     them).  Nothing in it needs clearing: each call overwrites every
 *     partial sum it reads.
 *   - The problem's device must be the current device (PDCS_ERR_INVALID_ARG
 *     otherwise).  The first call on a device resolves the array's address;
 *     make that call outside stream capture.
 * Errors: PDCS_ERR_INVALID_ARG, PDCS_ERR_SIZE, PDCS_ERR_HIP. */
int  pdcs_problem_spmv_noalloc(pdcs_problem p, int64_t transpose, int64_t precision,
                               const void* in_dev, void* out_dev, void* stream);

/* pdcs_problem_set_layout: storage of the matrix for the two SpMVs of every
 * trial of a single problem.
 *   PDCS_LAYOUT_ROWS : CSR row blocks, fused with the dual / dual-slack steps;
 *   PDCS_LAYOUT_BANDS: band tiles: row bands x gathered-index windows, entries
 *                      sorted by gathered index and summed per row in LDS, then
 *                      one partial sum per window combined by the epilogues;
 *   PDCS_LAYOUT_WORKGROUP: CSR row blocks, with every chunk of trials between
 *                      two restart checks run by one kernel that gives each
 *                      instance one workgroup: the passes of a trial are
 *                      separated by workgroup barriers instead of kernel
 *                      launches (latency-bound small instances);
 *   PDCS_LAYOUT_AUTO : bands for problems (and batches, see
 *                      pdcs_batch_set_layout) with at least 2^22 nonzeros,
 *                      the workgroup layout when every instance (iterates,
 *                      data and both CSR copies, FP64) fits in the LDS of one
 *                      workgroup (about 120 KiB: e.g. 200 rows, 500 columns,
 *                      2500 nonzeros) and has no cone blocks, else rows.
 *                      Instances that fit run their trials out of LDS; forced,
 *                      the layout works on global memory for larger ones.
 * All layouts compute the same products up to rounding order; rows and
 * workgroup produce bit-identical iterates.  Building the band tiles takes host
 * time proportional to nnz log nnz and 20 bytes of device memory per nonzero of
 * each of G and G^T.  Cone blocks always take the band layout.
 * Errors: PDCS_ERR_INVALID_ARG for an unknown layout. */
#define PDCS_LAYOUT_AUTO  0
#define PDCS_LAYOUT_ROWS  1
#define PDCS_LAYOUT_BANDS 2
#define PDCS_LAYOUT_WORKGROUP 3
int  pdcs_problem_set_layout(pdcs_problem p, int64_t layout);

/* pdcs_problem_set_band_schedule: shape of the band tiles of the band layout.
 *   rows      : tallest band height, a power of two in [256, 8192] (default 8192);
 *   min_tiles : the height is halved (not below 256) while fewer band-tiles
 *               (bands x gathered-index windows) would result, so that the
 *               256 CUs get work (default 384; 1 keeps `rows`);
 *   entry_cap : in a batch, bands are cut to at most about this many entries
 *               per window and instance, in [1024, 2^24] (default 32768).
 * The layout is rebuilt on the host (time proportional to nnz log nnz).
 * Products are the same up to rounding order.  Errors: PDCS_ERR_INVALID_ARG.
 * pdcs_problem_band_schedule reads the settings back; *built_rows receives the
 * band height the current layout of G uses and *windows its number of
 * gathered-index windows (both 0 when the band layout is not in use); any
 * pointer may be NULL. */
int  pdcs_problem_set_band_schedule(pdcs_problem p, int64_t rows, int64_t min_tiles, int64_t entry_cap);
int  pdcs_problem_band_schedule(pdcs_problem p, int64_t* rows, int64_t* min_tiles, int64_t* entry_cap,
                                int64_t* built_rows, int64_t* windows);

/* ---- single solve ------------------------------------------------------
 * pdcs_solve: Algorithm 4 (rescale, Algorithm 1, unscale) on one problem.
 *   x0 / y0 : optional host warm start (double[n] / double[m]); NULL = zero
 *             (projected onto the box and the dual cone).
 *   out     : receives a result handle (also on non-optimal exits).
 * Errors: PDCS_ERR_INVALID_ARG, PDCS_ERR_OOM, PDCS_ERR_HIP. */
int  pdcs_solve(pdcs_problem p, const pdcs_options* opts, const double* x0, const double* y0,
                void* stream, pdcs_result* out);

/* pdcs_solve_device: pdcs_solve with the warm start in device memory, e.g. the
 * output of the warm-start network (pdcs_mlp_forward) without a trip through
 * the host.  x0_dev / y0_dev: NULL or device arrays of n / m values, FP64
 * (warm_dtype = PDCS_PRECISION_FP64) or FP32 (PDCS_PRECISION_MIXED), unscaled,
 * owned by the caller and only read.  The solver's stream waits for the work
 * already enqueued on `stream` (NULL: the HIP null stream) before it reads
 * them; the call is synchronous like pdcs_solve.  A NaN in the warm start
 * ends the solve with exit code 8 (numerical error).
 * Errors: PDCS_ERR_INVALID_ARG, PDCS_ERR_OOM, PDCS_ERR_HIP. */
int  pdcs_solve_device(pdcs_problem p, const pdcs_options* opts, const void* x0_dev, const void* y0_dev,
                       int64_t warm_dtype, void* stream, pdcs_result* out);

int  pdcs_result_info(pdcs_result r, pdcs_info* out);
/* Device-pointer results (the fields of Section 3 without a host copy): copy
 * instance r's primal x (n), dual y (m) or dual slack c - G^T y (n), FP64, into
 * the caller's device buffer of exactly that length, enqueued on `stream`
 * (NULL: the HIP null stream) and not synchronized.  The result handle must
 * stay alive until the copy has run.  Errors: PDCS_ERR_INVALID_ARG (null
 * pointers, length mismatch), PDCS_ERR_HIP. */
int  pdcs_result_primal_device(pdcs_result r, double* x_dev, int64_t n, void* stream);
int  pdcs_result_dual_device(pdcs_result r, double* y_dev, int64_t m, void* stream);
int  pdcs_result_slack_device(pdcs_result r, double* lam_dev, int64_t n, void* stream);
/* Copy results of instance 0 (single solves) to host buffers of exactly the
 * given length (mismatch: PDCS_ERR_INVALID_ARG). x: primal, y: dual,
 * lam: dual slack c - G^T y (the "slack" field of Section 3). */
int  pdcs_result_primal(pdcs_result r, double* x, int64_t n);
int  pdcs_result_dual(pdcs_result r, double* y, int64_t m);
int  pdcs_result_slack(pdcs_result r, double* lam, int64_t n);
/* Diagonal scaling used (G_hat = D1 G D2, eq. rescaled_prob). */
int  pdcs_result_scaling(pdcs_result r, double* D1, int64_t m, double* D2, int64_t n);
/* Internal iterate state at exit, rescaled space, FP64 copies: Halpern iterate
 * (x, y), last PDHG output (x_hat, y_hat), anchor (x_a, y_a).  Any pointer may
 * be NULL.  Lengths are the problem's n (x-like) and m (y-like). */
int  pdcs_result_state(pdcs_result r, pdcs_state_scalars* s, double* x, double* y,
                       double* x_hat, double* y_hat, double* x_a, double* y_a);
/* Rescaled products G^T y_hat and G x_hat of the last trial (keep_state solves):
 * double[n] and double[m]; either pointer may be NULL. */
int  pdcs_result_products(pdcs_result r, double* gty_hat, double* gx_hat);
/* Scalars of the first trace_trials trials of instance 0 (16 doubles per trial:
 * kbar, eta, eta_bar, ||dx||^2, ||dy||^2, dy^T G dx, accepted, eta', beta, k
 * before the trial, then c^T x_hat, h^T y_hat, sum l lam+, sum u lam-,
 * err_p^2, err_d^2 of the rescaled problem; NaN where a rejected trial has no
 * value); *count receives the number of rows written.  Requires
 * trace_trials > 0 in the solve's options. */
int  pdcs_result_trace(pdcs_result r, double* out, int64_t max_trials, int64_t* count);
void pdcs_result_destroy(pdcs_result r);

/* ---- batched solves ----------------------------------------------------
 * pdcs_batch_create: pack `count` problems block-diagonally into one device
 * structure; every kernel of the iteration then runs once over all instances,
 * each with its own scalars (step size, primal weight, restart state, exit
 * code).  The problems are only read during the call. */
int  pdcs_batch_create(int64_t count, const pdcs_problem* probs, pdcs_batch* out);
/* Solve all instances; results[i] receives instance i's result handle.
 * x0s / y0s: NULL or arrays of `count` host pointers (each may be NULL). */
int  pdcs_batch_solve(pdcs_batch b, const pdcs_options* opts, const double* const* x0s,
                      const double* const* y0s, void* stream, pdcs_result* results);
/* As pdcs_batch_solve with device warm starts: x0s_dev / y0s_dev are NULL or
 * host arrays of `count` DEVICE pointers (each may be NULL), instance i's
 * pointing to n_i / m_i values of warm_dtype (PDCS_PRECISION_FP64: double,
 * PDCS_PRECISION_MIXED: float), e.g. rows of one [count x (n + m)] network
 * output.  Ordering and errors as pdcs_solve_device. */
int  pdcs_batch_solve_device(pdcs_batch b, const pdcs_options* opts, const void* const* x0s_dev,
                             const void* const* y0s_dev, int64_t warm_dtype, void* stream,
                             pdcs_result* results);
/* Autotune this batch's SpMV schedules: times candidates with HIP events and
 * keeps the fastest.  Row blocks (pdcs_batch_schedule; the layout of small
 * batches and of a band batch's tail after compaction) are tuned first; with
 * band tiles, band height, tile minimum and per-window entry cap
 * (pdcs_batch_band_schedule) are then tuned on the trial product G x_hat, each
 * candidate rebuilding the band layouts on the host.  Candidates beyond
 * time_budget_ms are skipped (<= 0: 2000 ms); the current schedules are always
 * among those timed. */
int  pdcs_batch_autotune(pdcs_batch b, double time_budget_ms);
/* Current schedule: iter_max (row-group iterations per wavefront tile),
 * block_nnz (nonzeros per workgroup), vec_per_block (elements per workgroup). */
int  pdcs_batch_schedule(pdcs_batch b, int64_t* iter_max, int64_t* block_nnz,
                         int64_t* vec_per_block);
int  pdcs_batch_set_schedule(pdcs_batch b, int64_t iter_max, int64_t block_nnz,
                             int64_t vec_per_block);
/* pdcs_batch_set_layout: as pdcs_problem_set_layout, for every instance of the
 * batch (each instance gets its own bands and gathered-index windows).
 * Errors: PDCS_ERR_INVALID_ARG. */
int  pdcs_batch_set_layout(pdcs_batch b, int64_t layout);
/* As pdcs_problem_set_band_schedule / pdcs_problem_band_schedule for a batch. */
int  pdcs_batch_set_band_schedule(pdcs_batch b, int64_t rows, int64_t min_tiles, int64_t entry_cap);
int  pdcs_batch_band_schedule(pdcs_batch b, int64_t* rows, int64_t* min_tiles, int64_t* entry_cap,
                              int64_t* built_rows, int64_t* windows);
void pdcs_batch_destroy(pdcs_batch b);

/* ---- warm-start MLP ----------------------------------------------------
 * 3-layer perceptron v = W3 relu(W2 relu(W1 u + b1) + b2) + b3 with BF16
 * weights (FP32 master copy) and FP32 accumulation on MFMA units.  Inputs and
 * outputs are device float32 row-major [batch x d].  pdcs_mlp_create: sizes in
 * [1, 2^26] for d_in and d_out, [1, 8192] for width, and fewer than 2^30
 * entries in each weight matrix (width x d_in, width x d_out); Glorot-uniform
 * weights from `seed`, zero biases.  Errors: PDCS_ERR_INVALID_ARG,
 * PDCS_ERR_OOM, PDCS_ERR_HIP. */
int  pdcs_mlp_create(int64_t d_in, int64_t width, int64_t d_out, uint64_t seed, pdcs_mlp* out);
int  pdcs_mlp_forward(pdcs_mlp net, const float* in_dev, float* out_dev, int64_t batch,
                      void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the mean
 * squared error, enqueued on `stream`.  The weight updates run inside the
 * weight-gradient products.  With loss_out non-NULL the call waits for the
 * step and *loss_out (host) receives the loss of the batch before the step;
 * with loss_out NULL it returns at once (the step runs asynchronously on
 * `stream`; in_dev and target_dev must stay valid until it has run). */
int  pdcs_mlp_train_step(pdcs_mlp net, const float* in_dev, const float* target_dev,
                         int64_t batch, float lr, float* loss_out, void* stream);
/* Read back one activation of the last forward, gradient or training call as
 * host float[count], count = batch x features: which = 0 the network input as
 * the first product sees it (standardized, BF16), 1 / 2 the hidden layers
 * after ReLU (BF16), 3 the loss gradient dL/dv (BF16), 4 / 5 the ReLU-masked
 * gradients dL/dz2 / dL/dz1 (BF16).  3-5 exist only after a gradient or
 * training call.  BF16 values are widened exactly.  The call waits for the
 * device to be idle.  Errors: PDCS_ERR_INVALID_ARG. */
int  pdcs_mlp_activation(pdcs_mlp net, int64_t which, float* host_out, int64_t count);
/* Gradients of the MSE loss at the current weights without updating them, as
 * FP32 device arrays laid out like the weights (W1[width x d_in], b1[width],
 * W2[width x width], b2[width], W3[d_out x width], b3[d_out]). */
int  pdcs_mlp_gradients(pdcs_mlp net, const float* in_dev, const float* target_dev,
                        int64_t batch, float* grad_dev, float* loss_out, void* stream);
/* Feature standardization, host float arrays: the network sees
 * (u - in_mean) / in_scale (d_in features) and its raw output z is returned by
 * pdcs_mlp_forward as z * out_scale + out_mean (d_out features); training
 * targets are standardized the same way, so the loss is the MSE in
 * standardized units.  A NULL mean/scale pair means identity for that side
 * (the default).  Scales must be finite and > 0.  Copied; the call waits for
 * the device to be idle.  Errors: PDCS_ERR_INVALID_ARG. */
int  pdcs_mlp_set_normalization(pdcs_mlp net, const float* in_mean, const float* in_scale,
                                const float* out_mean, const float* out_scale);
int  pdcs_mlp_num_params(pdcs_mlp net, int64_t* count);
/* Read or write the FP32 master weights (host float[num_params], same layout
 * as the gradients).  Writing also refreshes the BF16 copies. */
int  pdcs_mlp_get_params(pdcs_mlp net, float* params_host);
int  pdcs_mlp_set_params(pdcs_mlp net, const float* params_host);
void pdcs_mlp_destroy(pdcs_mlp net);

#ifdef __cplusplus
}
#endif
#endif /* PDCS_H */
