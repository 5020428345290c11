/*
 * dpdlp.h -- C ABI of the single-GPU (MI355X, gfx950) restarted
 * reflected-Halpern PDHG linear-programming solver (the PDLP family, as
 * distributed by D-PDLP, arXiv 2601.07628).
 *
 * Problem (Sec. 2.1, problem (1)):
 *     min  c^T x   s.t.   con_lo <= A x <= con_hi,   var_lo <= x <= var_hi
 * with A given in CSR.  An '=' row has con_lo == con_hi, a '>=' row has
 * con_hi == +inf, a '<=' row has con_lo == -inf; IEEE +-inf are the only
 * infinities.  The dual variable y follows the sign convention
 * L(x, y) = c^T x - y^T A x - p(-y; con_lo, con_hi): y >= 0 on '>=' rows,
 * y <= 0 on '<=' rows, y = 0 on free rows (the sets Y_i of Sec. 2.1).
 *
 * Every call returns an int: DPDLP_OK (0) or a negative DPDLP_E_* code, with
 * a message in dpdlp_last_error().  Not converging is not an error: it is
 * reported in dpdlp_result.status.  All pointers are plain host or device
 * pointers as stated per argument; "stream" is a hipStream_t passed as void*
 * (NULL = the null stream).  One problem handle is used by one host thread
 * and one stream at a time.
 */
#ifndef DPDLP_H
#define DPDLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define DPDLP_OK               0
#define DPDLP_E_INVALID_ARG   -1   /* a NULL pointer, a size out of range      */
#define DPDLP_E_BAD_CSR       -2   /* row_ptr not monotone, column out of      */
                                   /* range, duplicate (i,j), non-finite value */
#define DPDLP_E_BAD_BOUNDS    -3   /* lo > hi, NaN, lo = +inf or hi = -inf     */
#define DPDLP_E_HIP           -4   /* a HIP runtime call failed                */
#define DPDLP_E_OOM           -5   /* device memory exhausted                  */
#define DPDLP_E_NOT_SUPPORTED -6   /* a feature not built / wrong device       */

/* ---- solve status (dpdlp_result.status) -------------------------------- */
#define DPDLP_RUNNING          0
#define DPDLP_CONVERGED        1   /* max(r_primal, r_dual, r_gap) <= eps      */
#define DPDLP_ITER_LIMIT       2
#define DPDLP_TIME_LIMIT       3
#define DPDLP_NUMERICAL        4   /* a NaN/Inf appeared in the iterate        */

/* Where the pointers of a call live.  Every call that takes a memory kind
 * (in its arguments or in dpdlp_csr_lp) rejects any other value with
 * DPDLP_E_INVALID_ARG before it reads a pointer.                          */
#define DPDLP_MEM_HOST         0
#define DPDLP_MEM_DEVICE       1

#define DPDLP_FP64             0
#define DPDLP_FP32_MIXED       1

/* Input LP in CSR.  int32 indices: nnz < 2^31 (App. E.2 prices 4-byte
 * indices).  Column indices may be unsorted inside a row; duplicates are
 * rejected.  mem_kind says whether every pointer is host or device memory.
 * The caller keeps ownership; dpdlp_problem_create deep-copies.           */
typedef struct dpdlp_csr_lp {
    int32_t m, n;                 /* rows, columns; both >= 1            */
    const int32_t *row_ptr;       /* [m+1], row_ptr[0] = 0, monotone     */
    const int32_t *col_idx;       /* [nnz], nnz = row_ptr[m]             */
    const double *val;            /* [nnz]                               */
    const double *c;              /* [n]                                 */
    const double *con_lo, *con_hi;/* [m]                                 */
    const double *var_lo, *var_hi;/* [n]                                 */
    int32_t mem_kind;             /* DPDLP_MEM_HOST or DPDLP_MEM_DEVICE  */
} dpdlp_csr_lp;

/* Solver parameters; dpdlp_params_default() fills the defaults given here.
 * The paper fixes none of the constants except the block size B = 256 of
 * the block-wise permutation (Sec. 4.2); the rest follow PDLP practice.   */
typedef struct dpdlp_params {
    double eps;               /* 1e-8: relative KKT tolerance (App. B.4)     */
    int64_t max_iters;        /* 100000                                      */
    double time_limit;        /* seconds, <= 0: none                         */
    int32_t check_period;     /* K = 64: KKT/restart check every K (App. D)  */
    int32_t ruiz_iters;       /* 10 Ruiz infinity-norm passes                */
    double gamma;             /* 1.0: reflection of the Halpern step (App. A)*/
    double beta_suf, beta_nec, beta_art;   /* 0.2, 0.8, 0.36 (App. B.2)     */
    double kp, ki, kd;        /* 0.99, 0.01, 0.0: PID gains (App. B.3)       */
    double eta;               /* > 0: fixed step; 0: eta_safety/sigma_max(A~)*/
    double omega0;            /* > 0: fixed initial primal weight; 0: ||c~||/||b~|| */
    double eta_safety;        /* 0.998                                       */
    int32_t power_max_iters;  /* 5000: steps of each of the two sigma_max(A~) */
                              /* estimates (Golub-Kahan-Lanczos bidiagonal- */
                              /* ization from two seeded starts, the larger */
                              /* kept)                                      */
    int32_t use_pc;           /* 1: one Pock-Chambolle pass after Ruiz       */
    double power_tol;         /* 1e-6: an estimate stops when it grew by at  */
                              /* most this (relative) over 8 steps          */
    double pc_alpha;          /* 1.0                                         */
    int32_t perm_block;       /* 256: block size of the block-wise random    */
                              /* permutation (Sec. 4.2); 0: no permutation   */
    int32_t tile_nnz;         /* nonzeros per workgroup tile (Sec. 4.3 at CU */
                              /* granularity), max 2048; 0 = automatic: the  */
                              /* power of two in [256, 2048] nearest to      */
                              /* nnz / 800 on a log scale (about 800 tiles   */
                              /* per step, within one round of 5 resident    */
                              /* workgroups on each of the 256 CUs)          */
    uint64_t perm_seed;       /* seed of the block permutation               */
    int32_t precision;        /* DPDLP_FP64 or DPDLP_FP32_MIXED              */
    int32_t xcd_remap;        /* 1: map consecutive tiles onto one XCD        */
    double fp32_switch_tol;   /* FP32 -> FP64 switch when KKT <= this (1e-6); */
                              /* the KKT is always evaluated in FP64, so an  */
                              /* FP32 iterate with KKT <= eps ends the solve */
    int32_t fp32_stall_checks;/* ... or no 2x KKT improvement in this many checks (64), */
                              /* or divergence (fp32_diverge below); FP64   */
                              /* resumes as a fresh epoch at the last check */
                              /* point, after a divergence at the FP32      */
                              /* phase's best one with its primal weight    */
    int32_t gather_slices;    /* -1 (default): automatic; 0: off; S (multiple */
                              /* of 8, <= 64): cut the gathered dimension of */
                              /* each fused step into S contiguous slices of */
                              /* equal nonzero counts, slice s on XCD s % 8, */
                              /* partial sums added per segment in slice     */
                              /* order (the 2-D partition of Sec. 3.1 across */
                              /* the 8 XCDs).  Automatic slices a step when  */
                              /* its gathered vector exceeds 4 MB, when the  */
                              /* gathers of one XCD's resident tiles (160    */
                              /* consecutive tiles) touch more than 2 MB of  */
                              /* it (128-byte lines of 8-byte entries, in    */
                              /* both precisions), and when its partial      */
                              /* sums, one per (segment, slice) with         */
                              /* nonzeros at 20 bytes                        */
                              /* each, cost less than its 12 bytes per       */
                              /* nonzero: S = 16 when 8 slices would exceed  */
                              /* 2 MB each (in the iterate's precision) and  */
                              /* each gathered element is read >= 4 times    */
                              /* per pass, else 8                            */
    int32_t use_graphs;       /* 1: replay the check_period - 1 iterations    */
                              /* between two checks as one HIP graph (off    */
                              /* while dpdlp_profile_enable is on)           */
    int32_t perm_order;       /* 0: the block-wise random permutation alone; */
                              /* bit 0 (rows) / bit 1 (columns): hot-first, */
                              /* that order stably sorted by decreasing     */
                              /* nonzero count, so the most gathered entries */
                              /* of y / x share cache lines; automatic      */
                              /* slicing then leaves that gather unsliced   */
                              /* (equal index ranges would put most         */
                              /* nonzeros in one slice); values above 3 are  */
                              /* rejected                                   */
    int32_t gather_sort;      /* sliced steps: store each tile's nonzeros     */
                              /* sorted by gathered index (products go back  */
                              /* to their segment order in LDS) -1           */
                              /* (default): where that cuts the cache lines  */
                              /* one wave's gathers touch by >= 25%; 0: off; */
                              /* 1: always                                   */
    double fp32_diverge;      /* FP32 -> FP64 switch when the KKT exceeds    */
                              /* this multiple of the FP32 phase's best (10; */
                              /* 0: off)                                    */
} dpdlp_params;

typedef struct dpdlp_result {
    int32_t status;           /* DPDLP_CONVERGED, ... */
    int32_t restarts;
    int64_t iters;            /* PDHG iterations run (FP32 + FP64)           */
    int64_t fp32_iters;       /* iterations run in FP32 (mixed mode)         */
    double r_primal, r_dual, r_gap;   /* at the last check (App. B.4)        */
    double obj_primal, obj_dual;
    double omega, eta, sigma_max;
    double setup_seconds, solve_seconds;
    int32_t power_iters, n_checks;    /* Lanczos steps of the sigma_max estimate; checks */
    int32_t slices_primal, slices_dual;   /* gather slices of each fused step as built    */
                                          /* (0: unsliced)                              */
} dpdlp_result;

/* Scalars of the iteration state, for checkpoint / resume and parity tests. */
typedef struct dpdlp_state {
    double omega, r0, r_prev, pid_int, pid_prev;
    int64_t k, t;             /* epoch iteration, total iteration            */
    int32_t pid_started, restarts, status, n_checks;
    double r_primal, r_dual, r_gap, obj_primal, obj_dual, r_fixed_point;
} dpdlp_state;

/* One record per check (restart-decision log). restart: 0 none,
 * 1 sufficient, 2 necessary, 3 artificial decay (App. B.2).               */
typedef struct dpdlp_log_rec {
    int64_t t, k;
    double r, r0, r_primal, r_dual, r_gap, omega;
    int32_t restart, pad;
} dpdlp_log_rec;

typedef struct dpdlp_problem dpdlp_problem;

/* Default parameters (values above). */
void dpdlp_params_default(dpdlp_params *p);

/* Ingest and prepare a problem on the current HIP device, on `stream`:
 * validate (host), block-wise random permutation of rows and columns
 * (Sec. 4.2), CSC build (App. E.3 keeps both formats), nonzero-aware
 * workgroup tiles (Sec. 4.3), Ruiz + Pock-Chambolle rescaling, sigma_max(A~)
 * by Lanczos bidiagonalization for eta, and the initial primal weight.  *out receives a handle
 * that owns every device buffer; free it with dpdlp_problem_destroy.
 * Errors: INVALID_ARG, BAD_CSR, BAD_BOUNDS, HIP, OOM.                     */
int dpdlp_problem_create(const dpdlp_csr_lp *lp, const dpdlp_params *params,
                         void *stream, dpdlp_problem **out);
int dpdlp_problem_destroy(dpdlp_problem *prob);

/* Replace the objective and bounds of a prepared problem by those of another
 * member of the same family (same A): c [n], con_lo/con_hi [m], var_lo/var_hi
 * [n]; any may be NULL to keep the current values.  The matrix scaling,
 * tiles and step size are kept; the scaled vectors, the norms and omega0 are
 * recomputed.  The next dpdlp_iterate starts from a fresh dpdlp_init.
 * Errors: BAD_BOUNDS (as dpdlp_validate), HIP.                            */
int dpdlp_problem_update_data(dpdlp_problem *prob, const double *c, const double *con_lo,
                              const double *con_hi, const double *var_lo,
                              const double *var_hi, int32_t mem_kind, void *stream);

/* Change the run-time parameters of a prepared problem: eps, max_iters,
 * time_limit, check_period, gamma, beta_*, kp/ki/kd, xcd_remap, use_graphs
 * and the FP32 switch rule.  The other fields (scaling, step size, permutation, tiles,
 * precision) are fixed at creation and ignored here.  Errors: INVALID_ARG. */
int dpdlp_set_params(dpdlp_problem *prob, const dpdlp_params *params);

/* Diagonal quadratic objective (Sec. 6): the problem becomes
 *     min c^T x + x^T Q x / 2,  Q = diag(q),  under the same constraints.
 * q[n] (host or device per mem_kind, original column order, every entry
 * finite and >= 0) is copied; NULL returns to the LP.  The primal step
 * becomes the closed-form minimiser over the box of the separable
 * subproblem, xh = clamp((x - tau (c - A^T y)) / (1 + tau q), l, u) in the
 * scaled space (scaled Q = D_c Q D_c); the KKT adds Q x to the dual
 * residual, x^T Q x / 2 to the primal objective and takes it off the dual
 * objective.  Scaling, step size and primal weight stay those of the LP
 * part.  Call before dpdlp_init / dpdlp_solve (a later call takes effect
 * from the next iteration).  In DPDLP_FP32_MIXED mode the FP32 phase uses
 * an FP32 copy of the scaled diag(Q); the checks use the FP64 one.
 * INVALID_ARG for a negative or non-finite entry or a bad mem_kind.       */
int dpdlp_set_objective_diag(dpdlp_problem *prob, const double *q, int32_t mem_kind,
                             void *stream);

/* Start from (x0, y0) (original space; NULL = zeros): the point is scaled,
 * clamped into X and projected onto Y, and becomes the epoch anchor.  The
 * pointers are host or device per mem_kind.                              */
int dpdlp_init(dpdlp_problem *prob, const double *x0, const double *y0,
               int32_t mem_kind, void *stream);

/* Continue the restarted Halpern PDHG loop (Algorithm 1 at one device;
 * App. A-B) for at most n_iters iterations, stopping early on convergence,
 * the time limit, or max_iters in total.  Checks run every check_period
 * iterations and at the first iteration of each epoch.                    */
int dpdlp_iterate(dpdlp_problem *prob, int64_t n_iters, void *stream);

/* Full solve: dpdlp_init + dpdlp_iterate(max_iters) + output.  x_out [n] and
 * y_out [m] (may be NULL) receive T(z) of the last iteration in the original
 * space and order.  Pointers are host or device per mem_kind.  info may be
 * NULL.                                                                  */
int dpdlp_solve(dpdlp_problem *prob, const double *x0, const double *y0,
                double *x_out, double *y_out, int32_t mem_kind,
                dpdlp_result *info, void *stream);

/* Result of the work done so far, and the current primal/dual point T(z)
 * in the original space and order (x_out/y_out may be NULL).              */
int dpdlp_get_result(dpdlp_problem *prob, double *x_out, double *y_out,
                     int32_t mem_kind, dpdlp_result *info, void *stream);

/* Export / import the full iteration state in the SCALED space, original
 * order: the Halpern iterate (x, y), the epoch anchor (xa, ya), the last
 * T(z) (xh, yh), plus the scalars.  Any array pointer may be NULL on export.
 * Host or device per mem_kind.  Import then dpdlp_iterate continues exactly
 * as an uninterrupted run would.                                          */
int dpdlp_state_export(dpdlp_problem *prob, dpdlp_state *st, double *x, double *y,
                       double *xa, double *ya, double *xh, double *yh,
                       int32_t mem_kind, void *stream);
int dpdlp_state_import(dpdlp_problem *prob, const dpdlp_state *st, const double *x,
                       const double *y, const double *xa, const double *ya,
                       const double *xh, const double *yh, int32_t mem_kind,
                       void *stream);

/* Copy out the restart-decision log (up to cap records, oldest first);
 * *count receives the number of records available.                       */
int dpdlp_get_log(dpdlp_problem *prob, dpdlp_log_rec *recs, int32_t cap, int32_t *count);

/* Products with the SCALED matrix A~ in the original order: out = A~ in
 * (transpose = 0; in [n], out [m]) or A~^T in (transpose = 1).  Device
 * pointers.  Used by tests and the standalone SpMV bandwidth benchmark.   */
int dpdlp_spmv(dpdlp_problem *prob, int32_t transpose, const double *in, double *out,
               void *stream);

/* KKT of the original problem at an original-space point (x, y) with primal
 * step tau (tau <= 0: the current eta/omega) (App. B.4).  out5 (host):
 * r_primal, r_dual, r_gap, obj_primal, obj_dual.  x, y per mem_kind; with
 * x = y = NULL the point is the current start point of dpdlp_init (after
 * its clamping into X and projection onto Y).                             */
int dpdlp_kkt(dpdlp_problem *prob, const double *x, const double *y, double tau,
              int32_t mem_kind, double *out5, void *stream);

/* KKT error without allocation, for callers that cannot call hipMalloc
 * (code under HIP graph capture, tight serving loops).  It needs no
 * problem handle: the LP (or the diagonal QP of dpdlp_set_objective_diag
 * when q != NULL) is given in CSR by lp (lp->mem_kind must be
 * DPDLP_MEM_DEVICE) together with its CSC copy (col_ptr [n+1], row_idx
 * [nnz], val_csc [nnz]; the same matrix, any row order inside a column).
 * Every pointer is device memory: x [n], y [m], col_scale [n] or NULL,
 * q [n] or NULL, and out5 (5 doubles: r_primal, r_dual, r_gap, primal and
 * dual objective, as dpdlp_kkt).  The primal step of column j in the dual
 * residual is tau * col_scale[j]^2 (col_scale = NULL: tau), so with D_c from
 * dpdlp_get_scaling and tau = eta / omega the result is the solver's own
 * termination measure at (x, y), the one dpdlp_kkt reports.
 * The call is asynchronous on `stream` and allocates nothing: its partial
 * sums live in a fixed 3.7 MB device array that each GPU holds until the
 * process ends, which bounds m and n to [1, 16777216] (INVALID_ARG beyond).
 * Calls that overlap on one GPU share that array and race.  INVALID_ARG for
 * NULL pointers, host memory, sizes out of range or tau <= 0; HIP for a
 * launch failure.                                                        */
int dpdlp_kkt_noalloc(const dpdlp_csr_lp *lp, const int32_t *col_ptr, const int32_t *row_idx,
                      const double *val_csc, const double *col_scale, const double *q,
                      const double *x, const double *y, double tau, double *out5,
                      void *stream);

/* Scaling vectors D_r [m], D_c [n] (A~ = D_r A D_c) in the original order,
 * eta, sigma_max and omega0 (host pointers; any may be NULL).             */
int dpdlp_get_scaling(dpdlp_problem *prob, double *dr, double *dc, double *eta,
                      double *sigma_max, double *omega0, void *stream);

/* Random-gather rate probe: the ceiling for the gathers of the XCD-sliced
 * fused steps (Sec. 3.1's partition of the gathered vector, one slice per
 * XCD).  Gathers n_gathers entries of a device vector of n_vec elements
 * (precision DPDLP_FP64: double, DPDLP_FP32_MIXED: float) at uniform random
 * indices, 2048 per workgroup of 256 threads as in one tile, each
 * workgroup's indices inside one of `slices` equal slices of the vector
 * (slice s on XCD s % 8, an XCD's slices one after another), and sums them
 * per thread.  *avg_ms receives the mean time of one pass over `reps`
 * timed launches (HIP events on `stream`, after one warm-up launch);
 * *gathers_per_s (may be NULL) n_gathers divided by it.  The indices come
 * from a splitmix64 stream started at `seed`.  The call allocates and
 * frees its own device buffers (4 n_gathers + n_vec elements) and
 * synchronizes.  INVALID_ARG unless slices is a multiple of 8 up to 64,
 * slices <= n_vec < 2^31, 1 <= n_gathers < 2^31 and reps >= 1; OOM or HIP
 * on a device failure.                                                    */
int dpdlp_time_gather(int64_t n_vec, int32_t slices, int64_t n_gathers, int32_t precision,
                      int32_t reps, uint64_t seed, void *stream, double *avg_ms,
                      double *gathers_per_s);

/* Time one kernel class over `reps` launches on `stream` with HIP events:
 * which = 0 fused primal step, 1 fused dual step, 2 CSR SpMV, 3 CSC SpMV.
 * *avg_ms receives the mean duration; *bytes the algorithmic bytes moved per
 * launch (matrix stream + vector reads and writes, gathered vectors once).
 * Advances no solver state (the steps run on scratch copies of x and y).  */
int dpdlp_time_kernel(dpdlp_problem *prob, int32_t which, int32_t reps, void *stream,
                      double *avg_ms, double *bytes);

/* Per-kernel timing with HIP events recorded on the solver's stream around
 * every launch of dpdlp_iterate.  enable = 1 clears the totals and starts
 * recording; 0 stops.  dpdlp_get_profile fills, per kernel class c
 * (0 fused primal step, 1 fused dual step, 2 CSR check pass, 3 CSC check
 * pass, 4 control kernel, 5-7 unused), the summed milliseconds, the launch
 * count and the algorithmic bytes one launch moves (matrix stream once,
 * every vector read or written once, gathered vectors once).  Arrays have 8
 * entries (host); any may be NULL.                                        */
int dpdlp_profile_enable(dpdlp_problem *prob, int32_t enable);
int dpdlp_get_profile(dpdlp_problem *prob, double *total_ms, int64_t *launches,
                      double *bytes_per_launch);

/* ---- learned warm start --------------------------------------------------
 * Not in the paper (which starts from a given (x0, y0), Algorithm 1 input):
 * a bipartite message-passing network on the row/column graph of the scaled
 * matrix A~ of a prepared problem predicts a start point for problems of the
 * same family (same A and variable bounds; other c and row bounds).
 *   inputs  column j: [c~_j, c~_j - c~ref_j, x~ref_j, has_lo, has_hi,
 *                      lo~_j or 0, hi~_j or 0, 1, 0 x 8]   (x~ = x / D_c)
 *           row i:    [b~_i, b~_i - b~ref_i, y~ref_i, is_eq, has_lo, has_hi,
 *                      0, 1, 0 x 8]  (y~ = y / D_r; b = finite lower bound,
 *                      else finite upper bound, else 0; c~ = D_c c, b~ = D_r b)
 *   network H_c0 = relu(X_c W_cin), H_r0 = relu(X_r W_rin); per layer
 *           H_r = relu([H_r, A~ H_c] W_r), H_c = relu([H_c, A~^T H_r] W_c)
 *           (BF16 activations and weights, FP32 accumulation on the MFMA
 *           units); x~0 = x~ref + H_c w_x, y~0 = y~ref + H_r w_y.
 *   params  one FP32 vector: W_cin [16x128], W_rin [16x128], then per layer
 *           W_c [256x128], W_r [256x128] (row-major, input feature major),
 *           then w_x [128], w_y [128].
 *   loss    mean((x~0 - x~*)^2) + mean((y~0 - y~*)^2).
 * Vectors are in the original order and space; pointers per mem_kind.     */
typedef struct dpdlp_gnn dpdlp_gnn;

/* Network with `layers` message-passing layers on prob's graph (prob must
 * outlive it).  Parameters start at zero: set them with dpdlp_gnn_set_params. */
int dpdlp_gnn_create(dpdlp_problem *prob, int32_t layers, void *stream, dpdlp_gnn **out);
int dpdlp_gnn_destroy(dpdlp_gnn *gnn);
int64_t dpdlp_gnn_num_params(dpdlp_gnn *gnn);
/* Host FP32 parameter vector (count = dpdlp_gnn_num_params); resets Adam.  */
int dpdlp_gnn_set_params(dpdlp_gnn *gnn, const float *params, int64_t count, void *stream);
/* Copy the FP32 parameters and the last gradient to host (either may be NULL). */
int dpdlp_gnn_get_params(dpdlp_gnn *gnn, float *params, float *grads, int64_t count,
                         void *stream);
/* Family reference: c_ref [n], b_ref [m] (per-row b as above), and the
 * reference solution x_ref [n], y_ref [m] (original space).               */
int dpdlp_gnn_set_reference(dpdlp_gnn *gnn, const double *c_ref, const double *b_ref,
                            const double *x_ref, const double *y_ref, int32_t mem_kind,
                            void *stream);
/* The instance whose start point is predicted: c [n], con_lo/con_hi [m].   */
int dpdlp_gnn_set_instance(dpdlp_gnn *gnn, const double *c, const double *con_lo,
                           const double *con_hi, int32_t mem_kind, void *stream);
/* Predicted start point in the original space (x0 [n], y0 [m]; may be NULL). */
int dpdlp_gnn_forward(dpdlp_gnn *gnn, double *x0, double *y0, int32_t mem_kind, void *stream);
/* Forward + backward against a target solution (original space); the
 * gradient stays on the device for dpdlp_gnn_adam_step; loss2 (host, may be
 * NULL) receives the two mean squared errors (columns, rows).              */
int dpdlp_gnn_backward(dpdlp_gnn *gnn, const double *x_target, const double *y_target,
                       int32_t mem_kind, double *loss2, void *stream);
/* One Adam step on the FP32 master weights (bias-corrected), refreshing the
 * BF16 copies used by the forward pass.                                   */
int dpdlp_gnn_adam_step(dpdlp_gnn *gnn, double lr, double beta1, double beta2, double eps,
                        void *stream);
/* The network's MFMA GEMM kernel alone (tests): C [M x Nc] FP32 (row stride
 * ldc) = A [M x K] B [K x Nc] with BF16 bit patterns, A(i,k) at
 * A[i*a_rs + k*a_cs], B(k,j) at B[k*b_rs + j*b_cs].  Device pointers.    */
int dpdlp_gnn_gemm_test(const uint16_t *A, long a_rs, long a_cs, const uint16_t *B, long b_rs,
                        long b_cs, float *C, long ldc, int32_t M, int32_t Nc, int32_t K,
                        void *stream);

/* ---- host-only preprocessing, callable without a GPU -------------------- */

/* Validate a host CSR LP; 0 or BAD_CSR / BAD_BOUNDS / INVALID_ARG.        */
int dpdlp_validate(const dpdlp_csr_lp *lp);

/* Block-wise random permutation (Sec. 4.2): split [0, count) into blocks of
 * `block` (last one partial), shuffle the blocks with a seeded Fisher-Yates
 * (splitmix64 stream), keep the order inside each block.  perm[new] = old.
 * block <= 0 gives the identity.                                          */
int dpdlp_block_permutation(int32_t count, int32_t block, uint64_t seed, int32_t *perm);

/* Nonzero-aware tiles over segment pointers seg_ptr[nseg+1] (Sec. 4.3 at
 * workgroup granularity): consecutive segments are packed while the tile
 * holds <= tile_nnz nonzeros and <= 1024 segments; a segment longer than
 * tile_nnz is split into pieces of tile_nnz.  tiles[8*i .. 8*i+7] =
 * {seg_begin, seg_end, nnz_begin, nnz_end, width_log2, piece, npieces, 0}.
 * Call with tiles = NULL to get the count in *ntiles, then again with room
 * for that many.                                                          */
int dpdlp_build_tiles(const int32_t *seg_ptr, int32_t nseg, int32_t tile_nnz,
                      int32_t *tiles, int32_t *ntiles);

/* Row bounds of the problem statement's Ax (=, >=, <=) b form (Sec. 2):
 * row_type[i] 0 '=' gives lo = hi = b[i]; 1 '>=' gives lo = b[i], hi = +inf;
 * 2 '<=' gives lo = -inf, hi = b[i].  Host arrays of length m, written into
 * the caller's con_lo / con_hi.  INVALID_ARG for NULL pointers, m < 0, an
 * unknown type or a non-finite b[i] (nothing is written then).            */
int dpdlp_row_bounds(int32_t m, const double *b, const int32_t *row_type, double *con_lo,
                     double *con_hi);

/* ---- cost model of the distributed method (host only) ------------------- */

/* Constants of the per-iteration cost model (Sec. 3.3; App. E.1 and E.3):
 * bandwidths in bytes/s, latency in seconds, traffic coefficients in bytes. */
typedef struct dpdlp_cost_params {
    double b_mem;             /* effective HBM bandwidth of one device       */
    double b_net;             /* effective interconnect bandwidth            */
    double beta_sync;         /* latency of one single-hop collective        */
    double n_hop;             /* mean hop count between devices              */
    double c_spmv;            /* bytes per nonzero per iteration (24: FP64   */
                              /* value + INT32 index, read in CSR and CSC)   */
    double c_vec;             /* bytes per vector element per iteration (90) */
    double c_net;             /* bytes per all-reduced element (8, FP64)     */
} dpdlp_cost_params;

/* MI355X defaults: b_mem 8.0e12 (HBM3E peak), b_net 153.6e9 (one xGMI link:
 * a ring moves over one link per hop), beta_sync 10e-6 and n_hop 1 (the
 * paper's single-node values), c_spmv 24, c_vec 90, c_net 8.               */
void dpdlp_cost_params_default(dpdlp_cost_params *p);

/* Modelled time of one iteration on an R x C device grid (Sec. 3.3, the
 * four terms derived in App. E.2), in seconds: out[0] matrix stream
 * c_spmv nnz / (b_mem R C); out[1] vector traffic c_vec (n/C + m/R) / b_mem;
 * out[2] ring all-reduce payload c_net (n R + m C - (m + n)) / (R C b_net);
 * out[3] latency n_hop beta_sync ([R > 1] + [C > 1]); out[4] the sum.
 * out has room for 5 doubles.  INVALID_ARG for negative sizes, R or C < 1,
 * NULL pointers, or non-positive / non-finite bandwidths.                 */
int dpdlp_cost_step(int64_t m, int64_t n, int64_t nnz, int32_t R, int32_t C,
                    const dpdlp_cost_params *p, double *out);

/* Grid for ndev devices (Sec. 4.1): the factor pair R x C = ndev whose
 * aspect ratio R / C is closest to m / n, closeness measured as a ratio,
 * |log(R/C) - log(m/n)| (the reading that reproduces every grid of the
 * worked examples in App. E.4); ties (equal up to 1e-12) take the
 * smaller R.  INVALID_ARG for
 * m, n or ndev < 1 or NULL outputs.                                       */
int dpdlp_grid_select(int64_t m, int64_t n, int32_t ndev, int32_t *R, int32_t *C);

/* Automatic device count (Sec. 5.1): for each candidate count (counts,
 * ncounts > 0, e.g. {1, 2, 4, 8}) take its grid from dpdlp_grid_select and
 * its modelled time from dpdlp_cost_step; return the count with the least
 * time (ties: the smaller count), its grid, and that time in *t_step (may
 * be NULL).  INVALID_ARG for bad sizes, a count < 1 or NULL outputs.       */
int dpdlp_auto_devices(int64_t m, int64_t n, int64_t nnz, const int32_t *counts,
                       int32_t ncounts, const dpdlp_cost_params *p, int32_t *ndev,
                       int32_t *R, int32_t *C, double *t_step);

/* Messages. */
const char *dpdlp_status_string(int32_t status);
const char *dpdlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DPDLP_H */
