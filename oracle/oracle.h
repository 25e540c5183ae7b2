/*
 * oracle.h -- plain, sequential FP64 CPU oracle for the block-Jacobi and
 * two-level (additive Schur-complement) ILU preconditioners with FGMRES.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path: only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no source with the GPU library.
 *
 * Everything is double precision, host memory, one thread.  Floating-point
 * contraction is disabled at build time (-ffp-contract=off) and every fused
 * multiply-add is an explicit fma(), so the order of every rounding is the
 * one written in oracle.c.
 *
 * Paper: Xu, Li, Osei-Kuffuor, "A Two-level GPU-Accelerated Incomplete LU
 * Preconditioner for General Sparse Linear Systems" (arXiv 2303.08881).
 */
#ifndef SCHURILU_ORACLE_H
#define SCHURILU_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_NOT_CONVERGED = 1,
  ORC_ERR_INVALID_ARG = -1,
  ORC_ERR_CSR = -2,
  ORC_ERR_ZERO_PIVOT = -3,
  ORC_ERR_OOM = -4,
  ORC_ERR_BREAKDOWN = -6
};

enum { ORC_BJ = 0, ORC_SCHUR = 1, ORC_RAP = 2 };
enum { ORC_ILU0 = 0, ORC_MILU0 = 1, ORC_ILUT = 2 };
enum { ORC_PIVOT_ERROR = 0, ORC_PIVOT_PERTURB = 1 };

typedef struct {
  int64_t n;
  const int64_t *row_ptr; /* n+1 */
  const int32_t *col;     /* row_ptr[n], ascending, unique per row */
  const double *val;
} orc_csr;

typedef struct {
  int32_t method;         /* ORC_BJ or ORC_SCHUR */
  int32_t interior_fact;  /* factor of the subdomain blocks (interior rows, and the
                             partial elimination of interface rows) */
  int32_t interface_fact; /* SCHUR only: factor of each local Schur complement */
  double droptol;         /* ILUT relative drop tolerance tau */
  int32_t lfil;           /* ILUT: max kept entries per part of a row */
  int32_t inner_iters;    /* SCHUR: GMRES steps on the reduced system */
  double inner_rtol;      /* SCHUR: early exit of the inner GMRES (0 = never) */
  int32_t pivot_mode;
  double pivot_tol;
  int32_t smooth_fact;    /* RAP only: factor of the smoother (ILU(0) in the paper); the coarse
                             factors R, P and L_S U_S come from interior_fact */
} orc_options;

typedef struct {
  int32_t iterations;  /* total outer Arnoldi steps over all restart cycles */
  int32_t converged;
  double final_relres; /* true ||b - A x|| / ||b|| at exit */
} orc_result;

typedef struct orc_precond orc_precond;

/* ---- building blocks (exposed for pins) ---- */
int orc_validate(const orc_csr *A);
int orc_classify(const orc_csr *A, const int32_t *part, int32_t nparts, uint8_t *is_iface);
int orc_permutation(int64_t n, const int32_t *part, int32_t nparts, const uint8_t *is_iface,
                    int32_t *perm, int32_t *iperm, int64_t *offsets /* 2*nparts+2 */);
void orc_spmv(const orc_csr *A, const double *x, double *y);
void orc_residual(const orc_csr *A, const double *b, const double *x, double *r);
/* level of each row: lower=1 -> dependencies are columns in [lo, r); lower=0 -> (r, hi) */
void orc_levels(int64_t n, const int64_t *rp, const int32_t *ci, int lower, int64_t lo,
                int64_t hi, int32_t *level);

/*
 * Factor the rows of M in order.  Rows r < nfull eliminate every column
 * k < r (a full ILU row); rows r >= nfull eliminate only k < nfull (a
 * partial ILU row, leaving a Schur-complement row).  Returns a handle to
 * the factor; read it with orc_fact_get, free with orc_fact_free.
 */
typedef struct orc_fact orc_fact;
int orc_factor(const orc_csr *M, int64_t nfull, int32_t method, double droptol, int32_t lfil,
               int32_t pivot_mode, double pivot_tol, orc_fact **out, int64_t *bad_row);
/* part: 0 = L (cols < min(r, nfull)), 1 = U (full rows, cols > r),
 *       2 = R (partial rows: remainder, cols >= nfull, diagonal included);
 * field: 0 row_ptr (int64, n+1), 1 col (int32), 2 val (double); D via part 3 field 2. */
int orc_fact_get(const orc_fact *F, int part, int field, const void **ptr, int64_t *len);
void orc_fact_free(orc_fact *F);

/* ---- preconditioner ---- */
int orc_setup(const orc_csr *A, const int32_t *part, int32_t nparts, const orc_options *opt,
              orc_precond **P, int64_t *bad_row);
void orc_apply(orc_precond *P, const double *r, double *z);
/* RAP only: out = R A P v for an interface vector v (local interface numbering),
 * unformed: -U_B^{-1} Z v, one SpMV with A, L_B^{-1} and W (exposed for pins). */
void orc_rap_matvec(orc_precond *P, const double *v, double *out);
int orc_fgmres(const orc_csr *A, orc_precond *P, const double *b, double *x, double rtol,
               int32_t restart, int32_t maxit, orc_result *res, double *hist /* maxit+1 or NULL */);
/* GMRES(m) right preconditioned with a fixed M: Arnoldi on A M^{-1}, only V
 * kept, x += M^{-1} (V c) at the end of each cycle (the batched systems). */
int orc_gmres(const orc_csr *A, orc_precond *P, const double *b, double *x, double rtol, int32_t restart,
              int32_t maxit, orc_result *res, double *hist /* maxit+1 or NULL */);
void orc_free(orc_precond *P);
/* Internal arrays for parity tests; see the ORC_X_* codes. */
int orc_export(const orc_precond *P, int32_t what, const void **ptr, int64_t *len);

enum {
  ORC_X_PERM = 0,     /* int32[n]  new -> old */
  ORC_X_IPERM = 1,    /* int32[n]  old -> new */
  ORC_X_IFACE = 2,    /* uint8[n]  interface flag, original numbering */
  ORC_X_OFFSETS = 3,  /* int64[2*nparts+2]: interior starts (nparts+1), interface starts (nparts+1) */
  ORC_X_LB = 10,      /* +0 row_ptr, +1 col, +2 val; interior rows, cols < row      */
  ORC_X_UB = 13,      /* interior rows, n_B > cols > row                              */
  ORC_X_DB = 16,      /* double[n_B] diagonal of U_B                                  */
  ORC_X_Z = 17,       /* interior rows, interface cols (global permuted numbering)    */
  ORC_X_W = 20,       /* interface rows (local 0..n_S), interior cols                 */
  ORC_X_LS = 23,      /* interface rows, interface cols (local), cols < row           */
  ORC_X_US = 26,      /* interface rows, local cols > row                             */
  ORC_X_DS = 29,      /* double[n_S]                                                  */
  ORC_X_COFF = 30,    /* interface rows, local cols in other subdomains               */
  ORC_X_LEV_LB = 40,  /* int32[n_B] */
  ORC_X_LEV_UB = 41,  /* int32[n_B] */
  ORC_X_LEV_LS = 42,  /* int32[n_S] */
  ORC_X_LEV_US = 43,  /* int32[n_S] */
  ORC_X_STILDE = 50   /* SCHUR: +0/+1/+2 the local Schur complements (interface rows) */
};

#ifdef __cplusplus
}
#endif
#endif
