/*
 * schurilu.h -- C ABI of libschurilu: block-Jacobi and two-level (additive
 * Schur-complement) ILU preconditioners with flexible GMRES, as hand-written
 * HIP kernels for AMD Instinct MI355X (gfx950).
 *
 * Method: Xu, Li, Osei-Kuffuor, "A Two-level GPU-Accelerated Incomplete LU
 * Preconditioner for General Sparse Linear Systems", arXiv 2303.08881.
 *
 * Conventions for every call
 *  - Matrices are CSR with int64 row pointers, int32 column indices sorted
 *    strictly ascending inside each row, FP64 values, and a stored diagonal.
 *  - Pointers named d_* are device pointers (HIP device memory, e.g. the
 *    data_ptr() of a torch CUDA/HIP tensor); pointers named h_* are host.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *  - Return value: 0 on success, ILU_NOT_CONVERGED (> 0) from fgmres_solve
 *    when the iteration limit was reached, a negative ILU_ERR_* code on error.
 *    ilu_last_error() then returns a message (thread-local, valid until the
 *    next call from the same thread).
 *  - Nothing here falls back to a CPU path: without a usable gfx950 device
 *    every call that computes returns ILU_ERR_HIP.
 */
#ifndef SCHURILU_H
#define SCHURILU_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define ILU_OK 0
#define ILU_NOT_CONVERGED 1
#define ILU_ERR_INVALID_ARG (-1)
#define ILU_ERR_CSR (-2)        /* unsorted / duplicate / out-of-range column, missing diagonal */
#define ILU_ERR_ZERO_PIVOT (-3) /* zero or non-finite pivot; row (original numbering) in the message */
#define ILU_ERR_OOM (-4)
#define ILU_ERR_HIP (-5)
#define ILU_ERR_BREAKDOWN (-6)  /* NaN/Inf inside the Krylov iteration */
#define ILU_ERR_CAPACITY (-7)   /* an ILUT working row outgrew the kernel's on-chip buffer */
#define ILU_ERR_TIMEOUT (-8)    /* a bounded dependency wait expired (internal error) */

/* ---- option values ---- */
#define ILU_METHOD_BJ 0    /* block Jacobi: Section 2.1, algorithm "Block Jacobi ILU on GPU" */
#define ILU_METHOD_SCHUR 1 /* additive two-level: algorithm "Additive block ILU solve",
                              Section 3.2, algorithm "Additive SCHUR-ILU on GPU"          */
#define ILU_METHOD_RAP 2   /* multiplicative two-level: Section 2.2.3, algorithm
                              "Two-level multiplicative solve"; Section 3.3, eqs.
                              (20)-(29), algorithm "Multiplicative RAP-ILU on GPU"       */
#define ILU_FACT_ILU0 0    /* ILU(0) on the pattern of the block                    */
#define ILU_FACT_MILU0 1   /* modified ILU(0): dropped fill added to the diagonal,
                              Section 2.3 eq. (16)                                  */
#define ILU_FACT_ILUT 2    /* threshold ILU with a per-part fill limit              */
#define ILU_PIVOT_ERROR 0
#define ILU_PIVOT_PERTURB 1
#define ILU_TRSV_AUTO 0    /* pick per triangular factor (see trsv_mode)       */
#define ILU_TRSV_LEVELS 1  /* level-scheduled across workgroups, sync-free     */
#define ILU_TRSV_BLOCK 2   /* one workgroup per subdomain, barrier per level   */
#define ILU_PREC_F64 0     /* triangular factors stored and solved in FP64      */
#define ILU_PREC_F32 1     /* stored in FP32, solved in FP32                     */
#define ILU_PREC_F16 2     /* stored in FP16 (scaled per row), solved in FP32    */
#define ILU_ARNOLDI_AUTO 0     /* one launch per Arnoldi step when the vectors fit          */
#define ILU_ARNOLDI_PER_PASS 1 /* one launch per Gram-Schmidt pass                             */

typedef struct {
  int64_t n;               /* rows = columns */
  int64_t nnz;             /* row_ptr[n] */
  const int64_t *d_row_ptr; /* n+1, device */
  const int32_t *d_col;    /* nnz, device */
  const double *d_val;     /* nnz, device */
} ilu_csr_t;

/*
 * Options.  Defaults (ilu_default_options): BJ, ILU(0) everywhere, 3 inner
 * GMRES steps (the paper's default, Section 4.1), no drop, pivot errors,
 * automatic solve mode, FP64 factors, one-launch Arnoldi steps.
 *  interior_fact  factor of each subdomain block A_i (BJ), or of the interior
 *                 rows plus the partial elimination of the interface rows
 *                 (SCHUR, eq. (17));
 *                 RAP: the factor of each whole block A_i (interior and
 *                 interface rows), whose (1,1), (2,1), (1,2) and (2,2) blocks
 *                 give L_B U_B, W~, Z~ and L_S U_S (eq. (20)); MILU(0) makes
 *                 the coarse preconditioner keep RAP 1 = L_S U_S 1;
 *  interface_fact SCHUR only: factor of each local Schur complement S~_i,
 *                 whose triangular factors precondition the reduced system
 *                 (eq. (18)-(19));
 *  smooth_fact    RAP only: factor of the smoother, a second block-Jacobi
 *                 factorization of every A_i (ILU(0) in the paper);
 *  droptol, lfil  ILUT: an entry w_j of row i is dropped when
 *                 |w_j| < droptol * ||a_i||_2; at most lfil entries are kept
 *                 in the L part and in the U part of each row (the Schur part
 *                 of a partially eliminated row counts as its U part); the
 *                 diagonal is always kept.  lfil < 0 means no limit (only for
 *                 n <= 8192).
 *  inner_iters    SCHUR, RAP: GMRES steps on the reduced system per apply;
 *                 0 applies the local Schur factors once (block Jacobi on S).
 *  inner_rtol     SCHUR, RAP: stop the inner GMRES once its residual estimate is
 *                 <= inner_rtol times the norm of its right-hand side.
 *  pivot_mode     ILU_PIVOT_ERROR: a zero pivot fails setup with
 *                 ILU_ERR_ZERO_PIVOT.  ILU_PIVOT_PERTURB: a pivot with
 *                 |u_ii| < pivot_tol * max_j |a_ij| is replaced by
 *                 +-pivot_tol * max_j |a_ij| (sign of u_ii, + for 0).
 *  trsv_mode      execution of the triangular solves (results agree to
 *                 rounding: the block-local solve splits long rows over a few
 *                 lanes and multiplies by the reciprocal of the diagonal):
 *                 ILU_TRSV_BLOCK solves each subdomain in one workgroup
 *                 (chosen by AUTO when every factor has at most 16384 levels
 *                 and a subdomain has at most 2^20 rows or at most 1024 rows
 *                 per level on average); ILU_TRSV_LEVELS spreads every level
 *                 over the whole GPU with sync-free level counters.
 *  factor_prec    storage precision of the triangular factors that the
 *                 preconditioner solves with (L_B, U_B, L_S, U_S and their
 *                 diagonals; the factorization itself is FP64, and the W rows
 *                 and Z columns stay FP64 in both solve modes).
 *                 ILU_PREC_F32 rounds them to FP32 once at setup and runs the
 *                 triangular solves in FP32; ILU_PREC_F16 stores each entry
 *                 divided by the largest magnitude of its row, in FP16, with
 *                 the row scale in FP32, and solves in FP32.  Right-hand sides
 *                 and results of the solves stay FP64 vectors, and so does
 *                 everything else (W, C_off, SpMV, Arnoldi, Givens, the
 *                 convergence test): the outer FGMRES, which allows a varying
 *                 preconditioner, corrects the lower-precision apply.
 *  arnoldi_mode   how the modified Gram-Schmidt of each Arnoldi step runs, in
 *                 fgmres_solve and in the reduced-system GMRES of ilu_apply
 *                 (results agree to the grouping of the dot-product sums):
 *                 ILU_ARNOLDI_AUTO takes one launch per step (every pass of
 *                 the step inside it, the new direction held on chip, the
 *                 workgroups waiting for each other's partial sums between
 *                 the passes) when the vectors fit it (even length, up to
 *                 2^21 rows on a 256-CU device), and one launch per pass
 *                 otherwise; ILU_ARNOLDI_PER_PASS always takes one launch per
 *                 pass.  Such a launch needs all its workgroups resident at
 *                 once: solves that run at the same time on one device
 *                 (several streams) should use ILU_ARNOLDI_PER_PASS, as the
 *                 request server does for its handles.
 *  block_split    workgroups per subdomain in the block-local L_B and U_B
 *                 solves (results are identical for every value): 1 gives
 *                 each subdomain one workgroup; K >= 2 (at most 64) splits
 *                 its rows into K consecutive ranges, one workgroup each,
 *                 which solve their levels side by side and pass the values
 *                 that a later range needs from an earlier one through
 *                 device memory.  The solve stays unsplit when a range's
 *                 level would need more than 64 such values, a range would
 *                 span more than 4096 levels, or a level of a range would be
 *                 wider than 384 threads.
 *                 0 (auto) takes one range per 24,576 rows of a subdomain,
 *                 at least 2 for subdomains of 32,768 rows or more, at most
 *                 16, while the ranges of all subdomains fit the CUs.  The
 *                 solves of one handle must not run at the same time (they
 *                 share the exchange buffers).
 */
typedef struct {
  int32_t method;
  int32_t interior_fact;
  int32_t interface_fact;
  double droptol;
  int32_t lfil;
  int32_t inner_iters;
  double inner_rtol;
  int32_t pivot_mode;
  double pivot_tol;
  int32_t trsv_mode;
  int32_t factor_prec;
  int32_t smooth_fact;
  int32_t arnoldi_mode;
  int32_t block_split;
} ilu_options_t;

typedef struct {
  int32_t iterations;   /* outer Arnoldi steps summed over restart cycles */
  int32_t converged;    /* 1 if ||b - A x|| <= rtol ||b|| at exit           */
  double final_relres;  /* true relative residual at exit                   */
  double setup_ms;      /* time of the ilu_setup that built P (device events) */
  double solve_ms;      /* time of this fgmres_solve                         */
} ilu_result_t;

typedef struct ilu_precond ilu_precond_t;

/* Fill *opt with the defaults listed above. */
void ilu_default_options(ilu_options_t *opt);

/*
 * ilu_setup -- build the preconditioner P of A (the setup procedures of the
 * algorithms named at ILU_METHOD_*), entirely on the device.  RAP also keeps
 * a copy of A (its coarse operator multiplies by A) and builds the smoother's
 * factors as a second block-Jacobi preconditioner inside P.
 *  A        device CSR (validated on the device: ILU_ERR_CSR on bad input).
 *  d_part   device int32[n], subdomain of each row (0 <= part < nparts), or
 *           NULL for a single subdomain.  Rows coupled to another subdomain
 *           in either direction become interface rows (Section 2.2.1); each
 *           subdomain is ordered interior-first in its original row order.
 *  nparts   >= 1.
 *  opt      options (host struct), NULL for the defaults.
 *  stream   stream for all setup work; the call returns after the stream has
 *           finished it (errors are then known).
 *  P        out: handle owning all device memory of the preconditioner.
 *           A and d_part may be freed once ilu_setup returns.
 */
int ilu_setup(const ilu_csr_t *A, const int32_t *d_part, int32_t nparts, const ilu_options_t *opt,
              void *stream, ilu_precond_t **P);

/*
 * ilu_apply -- z = M^{-1} r (device vectors of length n, original numbering),
 * asynchronous on `stream`.  BJ: gather, L solve, U solve, scatter (Section
 * 3.1).  SCHUR: f' = L_B^-1 f, g' = g - W f', inner GMRES on the reduced
 * system, u = U_B^-1 (f' - Z y), scatter (Section 3.2).  RAP: x = the
 * smoother's block-Jacobi solve of r; g = R (r - A x); v from the inner GMRES
 * on (L_S U_S)^-1 R A P v = (L_S U_S)^-1 g; z = x + P v (Section 3.3).  r and
 * z must not alias.  Not re-entrant per handle (the workspace lives in P).
 */
int ilu_apply(ilu_precond_t *P, const double *d_r, double *d_z, void *stream);

/*
 * ilu_rap_matvec -- out = R A P v with R = (-W~ L_B^-1, I) and
 * P = (-U_B^-1 Z~; I) left unformed (Section 3.3, eqs. (21) and (28)): one
 * U_B solve with the Z~ columns, one product with A, one L_B solve with the
 * W~ rows.  Only for a RAP handle (ILU_ERR_INVALID_ARG otherwise).  d_v and
 * d_out: device vectors of length n_S in the interface numbering (interface
 * row i is original row perm[n_B + i], see ilu_export code 0); they must not
 * alias.  Asynchronous on `stream`; shares P's workspace like ilu_apply.
 */
int ilu_rap_matvec(ilu_precond_t *P, const double *d_v, double *d_out, void *stream);

/*
 * fgmres_solve -- right-preconditioned flexible GMRES(restart) for A x = b
 * (Section 4.1).  d_x holds x0 on entry and the iterate on exit.  Stops when
 * the Givens residual estimate reaches rtol*||b|| and the true residual
 * confirms it, or after maxit Arnoldi steps.  Synchronises `stream`.
 * res may be NULL.  h_hist, if not NULL, receives maxit+1 doubles: the
 * relative residual estimate after each step (entry 0 = initial).
 */
int fgmres_solve(const ilu_csr_t *A, ilu_precond_t *P, const double *d_b, double *d_x, double rtol,
                 int32_t restart, int32_t maxit, void *stream, ilu_result_t *res, double *h_hist);

/*
 * fgmres_solve_noalloc -- fgmres_solve for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, arithmetic and results
 * as fgmres_solve (x bit for bit), but the Krylov workspace -- the basis V,
 * the preconditioned directions Z, the residual, the Hessenberg and Givens
 * scalars and the reduction partials, (2 restart + 2) n doubles plus a few KB
 * -- lives in one fixed 64 MiB device array per GPU, held from the library's
 * load until the process ends, and no call allocates (no hipMalloc, hipFree,
 * host-pinned allocation or HIP event).  Each step's residual estimate is
 * read back synchronously.  P must come from ilu_setup (which allocates its
 * own buffers), and kernel timing must be off.  Errors: ILU_ERR_CAPACITY
 * when the workspace exceeds the array (for example restart 50 allows
 * n <= 82,000), ILU_ERR_INVALID_ARG as fgmres_solve.  res->solve_ms is host
 * time.  All calls on one GPU share its array: calls that overlap in time on
 * one device (several host threads or streams) race and give undefined
 * results.
 */
int fgmres_solve_noalloc(const ilu_csr_t *A, ilu_precond_t *P, const double *d_b, double *d_x, double rtol,
                         int32_t restart, int32_t maxit, void *stream, ilu_result_t *res, double *h_hist);

/* y = A x (device, FP64, each row summed in column order with fma). */
int csr_spmv(const ilu_csr_t *A, const double *d_x, double *d_y, void *stream);

/* Release every device allocation of P (after waiting for the device to
 * finish with them).  NULL is accepted.  The library keeps released device
 * blocks in a per-device cache and hands them to later allocations of at
 * most their size and at least half of it, so repeated setups of one problem
 * call neither hipMalloc nor hipFree. */
void ilu_destroy(ilu_precond_t *P);

/* Free every cached device block (all devices) back to the HIP runtime, and
 * the HIP events kept for kernel timing.  Blocks still owned by a live
 * preconditioner are not affected.  An allocation that fails also empties
 * the cache before it gives up.  A process should destroy its handles and
 * call this before it exits: a HIP call made from a finaliser that runs
 * after the runtime's own exit handlers is undefined. */
void ilu_memory_trim(void);

/* Message for the last error of the calling thread. */
const char *ilu_last_error(void);

/*
 * ilu_export -- copy an internal array to host memory for inspection.
 * If h_buf is NULL only *len (element count) is set.  Otherwise *len must be
 * >= the element count on entry.  Codes (element types in brackets):
 *   0 perm [int32 n] new->old, 1 iperm [int32 n], 2 interface flag [uint8 n],
 *   3 offsets [int64 2*nparts+2]: interior starts, then interface starts,
 *   CSR blocks at base+0 row_ptr [int64], +1 col [int32], +2 val [double]:
 *   10 L_B, 13 U_B (interior cols), 17 Z (interface cols, permuted numbering),
 *   20 W (interface rows, interior cols), 23 L_S, 26 U_S (interface numbering),
 *   30 C_off (interface rows, other subdomains' interface columns);
 *   16 diag of U_B [double n_B], 29 diag of U_S [double n_S];
 *   40..43 level of each row of L_B, U_B, L_S, U_S [int32];
 *   44 schedule of the L_B, U_B, L_S, U_S solves [int32 22]: for each, 1 if
 *      solved block-locally (one workgroup per subdomain), lanes per row,
 *      entries per lane, threads per workgroup; then 1 if L_S and U_S run as
 *      one launch, a bit mask of the block-local solves that run without the
 *      slow-row and wide-level checks (bit k for solve k: no slow row, every
 *      level within the workgroup), the factor storage precision, and the
 *      workgroups of the block-local L_S and U_S solves (one per subdomain,
 *      or one per connected component of L_S + U_S when a subdomain has a
 *      few; 0 when they are not block-local), and the workgroups per
 *      subdomain of the block-local L_B and U_B solves (block_split; 0 when
 *      they are not block-local).
 */
int ilu_export(ilu_precond_t *P, int32_t what, void *h_buf, int64_t *len);

/*
 * Kernel timing (a profiling aid for benchmarks; process-global, not
 * thread-safe).  ilu_kernel_timing(classes) times the kernel classes whose
 * bits are set in `classes` (bit k = class k below, ILU_K_ALL = every class,
 * 0 = off): each of their launches is bracketed by HIP events on the stream
 * it is launched on, and durations are resolved at the next host
 * synchronisation.  The events add a little time to every launch they
 * bracket, so time only the classes you need.  ilu_kernel_stats returns, for
 * one kernel class, the summed duration, the number of launches and the
 * summed algorithmic bytes (each stored entry, row pointer, right-hand side
 * and solution element counted once per launch).  reset != 0 clears it.
 */
#define ILU_K_TRSV_LB 0  /* forward solve with L_B, rows of W included (one extra level) */
#define ILU_K_TRSV_UB 1  /* backward solve with U_B, Z columns included           */
#define ILU_K_TRSV_LS 2  /* forward solve with the local Schur factors L_S (with  */
                         /* U_S when both run in one launch; bytes of both)      */
#define ILU_K_TRSV_US 3  /* backward solve with U_S                               */
#define ILU_K_SPMV 4     /* y = A x in the outer Krylov loop                      */
#define ILU_K_SPMV_COFF 5 /* C_off y in the reduced-system operator              */
#define ILU_K_MGS 6      /* outer Gram-Schmidt: a step's launch, or one pass's     */
#define ILU_K_COUNT 7
#define ILU_K_ALL ((1 << ILU_K_COUNT) - 1)
void ilu_kernel_timing(int32_t classes);
int ilu_kernel_stats(int32_t kind, double *total_ms, int64_t *launches, double *bytes, int32_t reset);

/*
 * ---- Batched systems (one persistent launch) ----
 * Many independent systems A_k x_k = b_k, each preconditioned by its own
 * ILU(0) and solved by right-preconditioned GMRES(m) to its own relative
 * tolerance: the block-Jacobi view of Section 3.1 with every block a system
 * of its own (own right-hand side, own convergence).  One workgroup takes
 * one system whole, largest first; the ILU(0) factorization (Section 2.3) and
 * the GMRES iterations of every system run in a single kernel launch, which
 * needs no host synchronisation and can be captured in a HIP graph.
 *
 * The batch is given as one block-diagonal CSR: the rows of system k are
 * [h_sys_row[k], h_sys_row[k+1]) and its columns must lie in the same range
 * (global numbering).  Limits, checked at setup (ILU_ERR_CAPACITY): at most
 * 16 entries per row and 4 strictly below (and above) the diagonal, at most
 * 1024 levels per triangular factor of a system, and each dependency of a
 * triangular row at most 2048 positions behind the end of the row's level
 * in level order (any 2D/3D stencil of side <= 1000 qualifies).
 */
typedef struct ilu_batch ilu_batch_t;

/*
 * ilu_batch_setup -- analyse the pattern of the batch once: validate it, the
 * levels of A's strict lower and upper parts in every system (as the
 * single-system setup does, one segment per system), the level-sorted
 * positions of both triangular solves, and the largest-first system order.
 * The pattern is copied; values are passed to each solve.  restart: the
 * largest GMRES restart that later solves may use (1..32), sizing the Krylov
 * basis ((restart + 1) n doubles).  Synchronises `stream`.
 */
int ilu_batch_setup(const ilu_csr_t *A, const int64_t *h_sys_row, int32_t nsys, int32_t restart, void *stream,
                    ilu_batch_t **B);

/*
 * ilu_batch_solve -- enqueue one persistent launch on `stream` (no host
 * synchronisation, no allocation): for every system, the ILU(0) factors of
 * the values d_val (nnz doubles on the setup's pattern), then GMRES(restart)
 * from the initial guess in d_x (n doubles, overwritten by the solution) for
 * the right-hand side d_b until ||b_k - A_k x_k|| <= rtol ||b_k|| or maxit
 * Arnoldi steps.  Read the per-system outcome with ilu_batch_results.
 */
int ilu_batch_solve(ilu_batch_t *B, const double *d_val, const double *d_b, double *d_x, double rtol,
                    int32_t restart, int32_t maxit, void *stream);

/*
 * ilu_batch_results -- synchronise `stream` and copy, per system: the
 * iteration count (Arnoldi steps over all cycles), the true relative residual
 * at exit, and the status (0 converged, ILU_NOT_CONVERGED, ILU_ERR_ZERO_PIVOT
 * or ILU_ERR_BREAKDOWN).  Any pointer may be NULL.
 */
int ilu_batch_results(ilu_batch_t *B, int32_t *h_iters, double *h_relres, int32_t *h_status, void *stream);

/*
 * ilu_batch_schedule -- launch shape of later solves: levels of at most
 * `merge` rows (0..64) run on one wavefront with a wavefront barrier instead
 * of a workgroup barrier; `wpc` workgroups per CU stay resident (1 up to what
 * the kernel's resources allow); `threads` per workgroup, 256 or 512 (a
 * system's vector passes stream twice the data at once with 512).  merge and
 * wpc change no arithmetic: results are bit-identical for every merge and
 * wpc.  The thread count changes the order in which a workgroup sums its dot
 * products, so results for 256 and 512 threads agree to rounding.
 */
int ilu_batch_schedule(ilu_batch_t *B, int32_t merge, int32_t wpc, int32_t threads);

/*
 * ilu_batch_tune -- the autotuner: run one full solve per candidate schedule
 * (threads in {256, 512}, merge in {0, 16, 32, 64}, every feasible wpc),
 * each from the initial guess in d_x, timed with device events, and keep the
 * fastest.  d_x holds the initial guess again on return.  Out: the chosen
 * merge, wpc, threads and its time (ms).
 */
int ilu_batch_tune(ilu_batch_t *B, const double *d_val, const double *d_b, double *d_x, double rtol,
                   int32_t restart, int32_t maxit, void *stream, int32_t *h_merge, int32_t *h_wpc,
                   int32_t *h_threads, double *h_ms);

/*
 * ilu_batch_capture / ilu_batch_replay -- capture one ilu_batch_solve with
 * these arguments into a HIP graph kept in B (stream must not be the default
 * stream), and launch that graph on `stream`.  A replay reads the values,
 * right-hand sides and initial guess found at those addresses when it runs.
 */
int ilu_batch_capture(ilu_batch_t *B, const double *d_val, const double *d_b, double *d_x, double rtol,
                      int32_t restart, int32_t maxit, void *stream);
int ilu_batch_replay(ilu_batch_t *B, void *stream);

/*
 * ilu_batch_export -- for parity tests: 0 the factor values of the last
 * solve on A's pattern [double nnz] (strict lower part L, diagonal and
 * strict upper part of U), 1 the level of each row in L [int32 n], 2 in U
 * [int32 n], 3 the schedule [int32 5]: entries per row and triangle, merge,
 * workgroups per CU, grid, threads per workgroup.  Same buffer protocol as
 * ilu_export.
 */
int ilu_batch_export(ilu_batch_t *B, int32_t what, void *h_buf, int64_t *len);

void ilu_batch_destroy(ilu_batch_t *B);

/*
 * ---- Serving: continuous batching of solve requests ----
 * A server owns `slots` worker threads on the current device, each with its
 * own stream, and a cache of preconditioners keyed by a caller-chosen matrix
 * id.  A request is one solve A x = b (fgmres_solve with the server's
 * options); for an id already resident the setup is skipped.  Requests that
 * arrive while others run start as soon as a slot is free and the device
 * bytes they need fit into the budget beside the resident factors and the
 * other running requests; idle factors are evicted least-recently-used first
 * to make room.  Two requests for one id never run at once (a handle is not
 * re-entrant): the later one waits.  Each request issues the same kernels as
 * a lone call would, so its result does not depend on the mix.
 */
typedef struct ilu_server ilu_server_t;

typedef struct {
  int64_t ticket;
  int64_t matrix_id;
  int32_t status;       /* the solve's return code: 0, ILU_NOT_CONVERGED or ILU_ERR_*      */
  int32_t iterations;
  double final_relres;
  int32_t cache_hit;    /* 1: the factors of matrix_id were resident                      */
  int32_t slot;         /* worker that ran it (-1: rejected before running)               */
  double submit_us;     /* host steady clock, microseconds since ilu_server_create        */
  double start_us;
  double done_us;
  double setup_ms;      /* device time of the setup (0 on a cache hit)                    */
  double solve_ms;      /* device time of the solve                                      */
} ilu_request_t;

/* slots in [1, 64]; budget_bytes: device bytes that resident factors and
 * running requests may hold together; opt: options of every setup (NULL =
 * defaults).  Threads start at once; the calling thread's device is used. */
int ilu_server_create(int32_t slots, int64_t budget_bytes, const ilu_options_t *opt, ilu_server_t **S);

/*
 * Queue one solve.  A: the matrix (device CSR) when matrix_id is not resident,
 * else ignored (may be NULL; a request for an unknown id without A completes
 * with ILU_ERR_INVALID_ARG).  d_part/nparts as in ilu_setup (used only when
 * the setup runs).  d_b, d_x: device vectors of the matrix's size, x0 in and
 * the solution out.  A, d_part, d_b and d_x must stay valid until the request
 * has completed.  *ticket receives the request's ticket (0, 1, ... in
 * submission order).  Returns at once.
 */
int ilu_server_submit(ilu_server_t *S, int64_t matrix_id, const ilu_csr_t *A, const int32_t *d_part, int32_t nparts,
                      const double *d_b, double *d_x, double rtol, int32_t restart, int32_t maxit, int64_t *ticket);

/* Block until the request `ticket` has completed (ticket < 0: the next one to
 * complete, in completion order) and copy its record to *out; the ticket is
 * then collected.  If the request failed (out->status < 0) ilu_last_error()
 * holds its message.  Returns ILU_ERR_INVALID_ARG for an unknown or already
 * collected ticket, or when nothing is outstanding. */
int ilu_server_wait(ilu_server_t *S, int64_t ticket, ilu_request_t *out);

/* Counters, first `count` of: [0] bytes held (resident factors + running
 * reservations), [1] peak of [0], [2] resident matrices, [3] cache hits,
 * [4] misses, [5] evictions, [6] queued requests, [7] running requests,
 * [8] budget. */
int ilu_server_stats(ilu_server_t *S, int64_t *h_stats, int32_t count);

/* Finish every queued request, stop the workers and free all resident
 * factors.  Records not collected are dropped. */
void ilu_server_destroy(ilu_server_t *S);

/* Sizes: n, n_B (interior rows), n_S (interface rows), nparts. */
int ilu_info(ilu_precond_t *P, int64_t *n, int64_t *nB, int64_t *nS, int32_t *nparts);

#ifdef __cplusplus
}
#endif
#endif
