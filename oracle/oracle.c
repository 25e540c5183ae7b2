/*
 * oracle.c -- plain sequential FP64 oracle (TEST INFRASTRUCTURE ONLY; see
 * oracle.h).  Written from the paper, section by section:
 *
 *   Section 2 (eq. (2)-(3))      p-way row partition, local systems A_i
 *   Section 2.2.1, Fig. 1         interior / interface labelling and the
 *                                 reordering to [[B, F], [E, C]]
 *   Section 2.2.2, algorithm      additive two-level solve
 *   "Additive block ILU solve"
 *   Section 2.3, eq. (11)-(16)    MILU: dropped fill compensated on the diagonal
 *   Section 3.1, algorithm        block-Jacobi ILU setup / solve
 *   "Block Jacobi ILU on GPU"
 *   Section 3.2, eq. (17)         partial ILU: L_B, U_B, W = E U_B^-1,
 *                                 Z = L_B^-1 F and the Schur rows in one pass
 *   Section 3.2 (one-solve form)  f' = L_B^-1 f, g' = g - W f', S y = g',
 *                                 u = U_B^-1 (f' - Z y)
 *   Section 3.2, eq. (18)-(19)    reduced system preconditioned by the local
 *                                 Schur factors, solved by a few GMRES steps
 *   Section 4.1                   right-preconditioned flexible GMRES(m)
 *   Section 2.2.3, algorithm      multiplicative two-level solve: smoother,
 *   "Two-level multiplicative     restriction R, coarse correction with
 *   solve"                        S = R A P, interpolation P
 *   Section 3.3, eq. (20)-(29)    R = (-W L_B^-1, I), P = (-U_B^-1 Z; I) from
 *                                 the (M)ILU(0) factors of each A_i, RAP
 *                                 unformed, L_S U_S as its preconditioner
 *
 * Where the paper is silent this file reads it as follows:
 *  - a row is an interface row when it is coupled to another subdomain in
 *    either direction (the pattern is symmetrised), so E and F are block
 *    diagonal;
 *  - each subdomain keeps its rows in their original order, interior rows
 *    first; globally all interiors (subdomain-major), then all interfaces;
 *  - ILUT: tau_i = droptol * ||a_i||_2 (norm of the original row, summed in
 *    column order); an L entry below tau_i is dropped when it is reached as
 *    a pivot, other entries after the elimination; at most lfil entries are
 *    kept in the L part and, separately, in the U part (the Schur part of a
 *    partially eliminated row counts as its U part), ranked by |v|
 *    descending, then column ascending; the diagonal is always kept;
 *  - the interface factor of the two-level method is taken of the Schur
 *    rows left by the partial factorization, and preconditions the reduced
 *    system as in eq. (18)-(19);
 *  - the inner GMRES starts from zero and takes a fixed number of steps
 *    (stopping early only on breakdown or an optional relative tolerance);
 *    zero steps means one application of the interface factors;
 *  - pivots: a zero or non-finite pivot is an error unless perturbation is
 *    asked for, which replaces |u_ii| < tol * max_j |a_ij| by
 *    +-tol * max_j |a_ij| (sign of u_ii, + for 0);
 *  - FGMRES: modified Gram-Schmidt, Givens rotations with
 *    r = sqrt(fma(a, a, b*b)), convergence on |g_{j+1}| <= rtol ||b||
 *    confirmed by the true residual, iterations counted over restarts.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* growable row-wise storage                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n;    /* rows appended so far */
  int64_t *rp;  /* n+1 (capacity rows_cap+1) */
  int32_t *ci;
  double *v;
  int64_t cap, rows_cap;
} rows_t;

static int rows_init(rows_t *R, int64_t nrows) {
  memset(R, 0, sizeof(*R));
  R->rows_cap = nrows;
  R->rp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nrows + 1));
  if (!R->rp) return ORC_ERR_OOM;
  R->rp[0] = 0;
  if (nrows > 0) R->rp[1] = 0; /* end of the (empty) open row */
  R->cap = 16;
  R->ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)R->cap);
  R->v = (double *)malloc(sizeof(double) * (size_t)R->cap);
  return (R->ci && R->v) ? ORC_OK : ORC_ERR_OOM;
}

static void rows_free(rows_t *R) {
  free(R->rp);
  free(R->ci);
  free(R->v);
  memset(R, 0, sizeof(*R));
}

/* append to the open row R->n, whose end is kept in rp[n+1] */
static int rows_push(rows_t *R, int32_t c, double v) {
  int64_t at = R->rp[R->n + 1];
  if (at + 1 > R->cap) {
    int64_t nc = R->cap * 2;
    int32_t *ci = (int32_t *)realloc(R->ci, sizeof(int32_t) * (size_t)nc);
    if (!ci) return ORC_ERR_OOM;
    R->ci = ci;
    double *vv = (double *)realloc(R->v, sizeof(double) * (size_t)nc);
    if (!vv) return ORC_ERR_OOM;
    R->v = vv;
    R->cap = nc;
  }
  R->ci[at] = c;
  R->v[at] = v;
  R->rp[R->n + 1] = at + 1;
  return ORC_OK;
}

/* close the open row and open the next one (empty) */
static void rows_end(rows_t *R) {
  R->n++;
  if (R->n < R->rows_cap) R->rp[R->n + 1] = R->rp[R->n];
}

/* ------------------------------------------------------------------------ */
/* validation, interface classification, permutation (Section 2.2.1)        */
/* ------------------------------------------------------------------------ */
int orc_validate(const orc_csr *A) {
  if (!A || A->n < 0) return ORC_ERR_INVALID_ARG;
  if (A->n == 0) return ORC_OK;
  if (!A->row_ptr || !A->col || !A->val) return ORC_ERR_INVALID_ARG;
  if (A->row_ptr[0] != 0) return ORC_ERR_CSR;
  for (int64_t i = 0; i < A->n; i++) {
    int64_t b = A->row_ptr[i], e = A->row_ptr[i + 1];
    if (e < b) return ORC_ERR_CSR;
    int diag = 0;
    for (int64_t p = b; p < e; p++) {
      int32_t c = A->col[p];
      if (c < 0 || c >= A->n) return ORC_ERR_CSR;
      if (p > b && A->col[p - 1] >= c) return ORC_ERR_CSR; /* unsorted or duplicate */
      if (c == i) diag = 1;
    }
    if (!diag) return ORC_ERR_CSR;
  }
  return ORC_OK;
}

/* Row i is an interface (exterior) row when it is coupled to a row of another
 * subdomain in either direction: some a_ij != 0 or a_ji != 0 with
 * part[j] != part[i].  Using both directions keeps E and F block diagonal for
 * nonsymmetric patterns. */
int orc_classify(const orc_csr *A, const int32_t *part, int32_t nparts, uint8_t *is_iface) {
  for (int64_t i = 0; i < A->n; i++) {
    if (part[i] < 0 || part[i] >= nparts) return ORC_ERR_INVALID_ARG;
    is_iface[i] = 0;
  }
  for (int64_t i = 0; i < A->n; i++)
    for (int64_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; p++) {
      int32_t j = A->col[p];
      if (part[j] != part[i]) {
        is_iface[i] = 1;
        is_iface[j] = 1;
      }
    }
  return ORC_OK;
}

/* Interior rows first, subdomain by subdomain, then interface rows subdomain
 * by subdomain; original order is kept inside each group.  perm maps new ->
 * old, iperm old -> new.  offsets[0..nparts] are the interior starts (the
 * last one is n_B), offsets[nparts+1 .. 2*nparts+1] the interface starts
 * (the first is n_B, the last n). */
int orc_permutation(int64_t n, const int32_t *part, int32_t nparts, const uint8_t *is_iface,
                    int32_t *perm, int32_t *iperm, int64_t *offsets) {
  int64_t *cnt = (int64_t *)calloc((size_t)(2 * nparts), sizeof(int64_t));
  if (!cnt) return ORC_ERR_OOM;
  for (int64_t i = 0; i < n; i++) cnt[(is_iface[i] ? nparts : 0) + part[i]]++;
  int64_t acc = 0;
  for (int32_t k = 0; k < 2 * nparts; k++) {
    int64_t c = cnt[k];
    cnt[k] = acc;
    acc += c;
  }
  for (int32_t s = 0; s < nparts; s++) offsets[s] = cnt[s];
  offsets[nparts] = (nparts > 0) ? cnt[nparts] : n;
  for (int32_t s = 0; s < nparts; s++) offsets[nparts + 1 + s] = cnt[nparts + s];
  offsets[2 * nparts + 1] = n;
  if (nparts == 0) offsets[0] = n;
  for (int64_t i = 0; i < n; i++) {
    int64_t at = cnt[(is_iface[i] ? nparts : 0) + part[i]]++;
    perm[at] = (int32_t)i;
    iperm[i] = (int32_t)at;
  }
  free(cnt);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* SpMV, residual, triangular solves, vector kernels                        */
/* ------------------------------------------------------------------------ */
void orc_spmv(const orc_csr *A, const double *x, double *y) {
  for (int64_t i = 0; i < A->n; i++) {
    double s = 0.0;
    for (int64_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; p++) s = fma(A->val[p], x[A->col[p]], s);
    y[i] = s;
  }
}

void orc_residual(const orc_csr *A, const double *b, const double *x, double *r) {
  for (int64_t i = 0; i < A->n; i++) {
    double s = b[i];
    for (int64_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; p++) s = fma(-A->val[p], x[A->col[p]], s);
    r[i] = s;
  }
}

static double dot(int64_t n, const double *x, const double *y) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s = fma(x[i], y[i], s);
  return s;
}

static double nrm2(int64_t n, const double *x) { return sqrt(dot(n, x, x)); }

/* x = L^{-1} b, L unit lower triangular given by its strict part (rows in
 * order, columns ascending).  b and x may alias. */
static void trsv_lower_unit(const rows_t *L, const double *b, double *x) {
  for (int64_t i = 0; i < L->n; i++) {
    double s = b[i];
    for (int64_t p = L->rp[i]; p < L->rp[i + 1]; p++) s = fma(-L->v[p], x[L->ci[p]], s);
    x[i] = s;
  }
}

/* x = U^{-1} b, U given by its strict upper part (columns ascending) and its
 * diagonal d; the sum runs in column order, then one true division. */
static void trsv_upper(const rows_t *U, const double *d, const double *b, double *x) {
  for (int64_t i = U->n - 1; i >= 0; i--) {
    double s = b[i];
    for (int64_t p = U->rp[i]; p < U->rp[i + 1]; p++) s = fma(-U->v[p], x[U->ci[p]], s);
    x[i] = s / d[i];
  }
}

void orc_levels(int64_t n, const int64_t *rp, const int32_t *ci, int lower, int64_t lo, int64_t hi,
                int32_t *level) {
  if (lower) {
    for (int64_t i = 0; i < n; i++) {
      int32_t l = 0;
      for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
        int64_t c = ci[p];
        if (c >= lo && c < i && level[c] + 1 > l) l = level[c] + 1;
      }
      level[i] = l;
    }
  } else {
    for (int64_t i = n - 1; i >= 0; i--) {
      int32_t l = 0;
      for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
        int64_t c = ci[p];
        if (c > i && c < hi && level[c] + 1 > l) l = level[c] + 1;
      }
      level[i] = l;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* row-wise factorization: ILU(0), MILU(0), ILUT, full or partial           */
/* ------------------------------------------------------------------------ */
struct orc_fact {
  int64_t n, nfull;
  rows_t L, U, R;
  double *D;
};

typedef struct {
  int32_t *a;
  int64_t n;
} heap_t; /* binary min-heap of column indices */

static void heap_push(heap_t *h, int32_t x) {
  int64_t i = h->n++;
  h->a[i] = x;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h->a[p] <= h->a[i]) break;
    int32_t t = h->a[p];
    h->a[p] = h->a[i];
    h->a[i] = t;
    i = p;
  }
}

static int32_t heap_pop(heap_t *h) {
  int32_t top = h->a[0];
  h->a[0] = h->a[--h->n];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < h->n && h->a[l] < h->a[m]) m = l;
    if (r < h->n && h->a[r] < h->a[m]) m = r;
    if (m == i) break;
    int32_t t = h->a[m];
    h->a[m] = h->a[i];
    h->a[i] = t;
    i = m;
  }
  return top;
}

typedef struct {
  double mag;
  int32_t col;
  double val;
} cand_t;

static int cmp_keep(const void *pa, const void *pb) { /* |v| descending, then column ascending */
  const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
  if (a->mag > b->mag) return -1;
  if (a->mag < b->mag) return 1;
  return (a->col > b->col) - (a->col < b->col);
}

static int cmp_col(const void *pa, const void *pb) {
  const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
  return (a->col > b->col) - (a->col < b->col);
}

static int cmp_i32(const void *pa, const void *pb) {
  int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
  return (a > b) - (a < b);
}

/* keep the lfil largest candidates (all when lfil < 0), output sorted by column */
static int emit_part(rows_t *R, cand_t *c, int64_t m, int32_t lfil) {
  if (lfil >= 0 && m > lfil) {
    qsort(c, (size_t)m, sizeof(cand_t), cmp_keep);
    m = lfil;
    qsort(c, (size_t)m, sizeof(cand_t), cmp_col);
  }
  for (int64_t k = 0; k < m; k++)
    if (rows_push(R, c[k].col, c[k].val)) return ORC_ERR_OOM;
  return ORC_OK;
}

int orc_factor(const orc_csr *M, int64_t nfull, int32_t method, double droptol, int32_t lfil,
               int32_t pivot_mode, double pivot_tol, orc_fact **out, int64_t *bad_row) {
  const int64_t n = M->n;
  const int ilut = (method == ORC_ILUT), milu = (method == ORC_MILU0);
  int rc = ORC_OK;
  if (nfull < 0 || nfull > n) return ORC_ERR_INVALID_ARG;
  orc_fact *F = (orc_fact *)calloc(1, sizeof(orc_fact));
  double *w = (double *)calloc((size_t)(n + 1), sizeof(double));
  uint8_t *state = (uint8_t *)calloc((size_t)(n + 1), 1); /* 0 absent, 1 present, 2 dropped */
  int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n + 1));
  heap_t heap = {(int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1)), 0};
  if (!F || !w || !state || !list || !cand || !heap.a) {
    rc = ORC_ERR_OOM;
    goto done;
  }
  F->n = n;
  F->nfull = nfull;
  F->D = (double *)calloc((size_t)(nfull + 1), sizeof(double));
  if (!F->D || rows_init(&F->L, n) || rows_init(&F->U, nfull) || rows_init(&F->R, n - nfull)) {
    rc = ORC_ERR_OOM;
    goto done;
  }

  for (int64_t r = 0; r < n; r++) {
    const int64_t lim = (r < nfull) ? r : nfull; /* eliminate columns k < lim */
    int64_t len = 0;
    double nrm2sq = 0.0, rowinf = 0.0;
    for (int64_t p = M->row_ptr[r]; p < M->row_ptr[r + 1]; p++) {
      int32_t c = M->col[p];
      double a = M->val[p];
      w[c] = a;
      state[c] = 1;
      list[len++] = c;
      nrm2sq = fma(a, a, nrm2sq);
      if (fabs(a) > rowinf) rowinf = fabs(a);
      if (c < lim) heap_push(&heap, c);
    }
    const double tau = droptol * sqrt(nrm2sq);
    double drop = 0.0;

    while (heap.n > 0) {
      const int32_t k = heap_pop(&heap);
      const double wk = w[k] / F->D[k];
      if (ilut && fabs(wk) < tau) { /* small multiplier: drop it, no elimination */
        w[k] = 0.0;
        state[k] = 2;
        continue;
      }
      w[k] = wk;
      for (int64_t p = F->U.rp[k]; p < F->U.rp[k + 1]; p++) {
        const int32_t j = F->U.ci[p];
        const double ukj = F->U.v[p];
        if (state[j] == 1) {
          w[j] = fma(-wk, ukj, w[j]);
        } else if (ilut) { /* new fill-in */
          state[j] = 1;
          w[j] = fma(-wk, ukj, 0.0);
          list[len++] = j;
          if (j < lim) heap_push(&heap, j);
        } else if (milu) { /* fill outside the pattern: remember it for the diagonal */
          drop = fma(-wk, ukj, drop);
        }
      }
    }
    qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);

    if (r < nfull) { /* full row: L | d | U */
      double d = w[r];
      if (milu) d = d + drop;
      if (pivot_mode == ORC_PIVOT_PERTURB) {
        double thr = pivot_tol * rowinf;
        if (fabs(d) < thr) d = (d < 0.0) ? -thr : thr;
      }
      if (d == 0.0 || !isfinite(d)) {
        if (bad_row) *bad_row = r;
        rc = ORC_ERR_ZERO_PIVOT;
        goto done;
      }
      F->D[r] = d;
      int64_t m = 0;
      for (int64_t q = 0; q < len; q++) {
        int32_t c = list[q];
        if (c < r && state[c] == 1) cand[m++] = (cand_t){fabs(w[c]), c, w[c]};
      }
      if ((rc = emit_part(&F->L, cand, m, ilut ? lfil : -1))) goto done;
      rows_end(&F->L);
      m = 0;
      for (int64_t q = 0; q < len; q++) {
        int32_t c = list[q];
        if (c > r && state[c] == 1 && !(ilut && fabs(w[c]) < tau)) cand[m++] = (cand_t){fabs(w[c]), c, w[c]};
      }
      if ((rc = emit_part(&F->U, cand, m, ilut ? lfil : -1))) goto done;
      rows_end(&F->U);
    } else { /* partial row: L (cols < nfull) | Schur remainder R */
      if (milu) w[r] = w[r] + drop;
      int64_t m = 0;
      for (int64_t q = 0; q < len; q++) {
        int32_t c = list[q];
        if (c < nfull && state[c] == 1) cand[m++] = (cand_t){fabs(w[c]), c, w[c]};
      }
      if ((rc = emit_part(&F->L, cand, m, ilut ? lfil : -1))) goto done;
      rows_end(&F->L);
      m = 0;
      for (int64_t q = 0; q < len; q++) {
        int32_t c = list[q];
        if (c >= nfull && c != r && state[c] == 1 && !(ilut && fabs(w[c]) < tau))
          cand[m++] = (cand_t){fabs(w[c]), c, w[c]};
      }
      if (ilut && lfil >= 0 && m > lfil) {
        qsort(cand, (size_t)m, sizeof(cand_t), cmp_keep);
        m = lfil;
      }
      cand[m++] = (cand_t){fabs(w[r]), (int32_t)r, w[r]}; /* the diagonal is always kept */
      qsort(cand, (size_t)m, sizeof(cand_t), cmp_col);
      for (int64_t k = 0; k < m; k++)
        if (rows_push(&F->R, cand[k].col, cand[k].val)) {
          rc = ORC_ERR_OOM;
          goto done;
        }
      rows_end(&F->R);
    }
    for (int64_t q = 0; q < len; q++) {
      w[list[q]] = 0.0;
      state[list[q]] = 0;
    }
  }

done:
  free(w);
  free(state);
  free(list);
  free(cand);
  free(heap.a);
  if (rc != ORC_OK && F) {
    orc_fact_free(F);
    F = NULL;
  }
  *out = F;
  return rc;
}

int orc_fact_get(const orc_fact *F, int part, int field, const void **ptr, int64_t *len) {
  const rows_t *R = part == 0 ? &F->L : part == 1 ? &F->U : part == 2 ? &F->R : NULL;
  if (part == 3) {
    *ptr = F->D;
    *len = F->nfull;
    return ORC_OK;
  }
  if (!R) return ORC_ERR_INVALID_ARG;
  if (field == 0) {
    *ptr = R->rp;
    *len = R->n + 1;
  } else if (field == 1) {
    *ptr = R->ci;
    *len = R->rp[R->n];
  } else {
    *ptr = R->v;
    *len = R->rp[R->n];
  }
  return ORC_OK;
}

void orc_fact_free(orc_fact *F) {
  if (!F) return;
  rows_free(&F->L);
  rows_free(&F->U);
  rows_free(&F->R);
  free(F->D);
  free(F);
}

/* ------------------------------------------------------------------------ */
/* preconditioner                                                            */
/* ------------------------------------------------------------------------ */
struct orc_precond {
  int64_t n, nB, nS;
  int32_t nparts;
  orc_options opt;
  int32_t *perm, *iperm;
  uint8_t *iface;
  int64_t *offsets;
  rows_t LB, UB, Z, W, LS, US, Coff, St;
  double *DB, *DS;
  int32_t *lev_lb, *lev_ub, *lev_ls, *lev_us;
  /* apply workspace */
  double *f, *g, *t, *y;
  /* inner GMRES workspace */
  double *V, *H, *cs, *sn, *gg, *c;
  double *w1, *w2;
  /* RAP: the smoother, the matrix, and work vectors */
  orc_precond *smoother;
  orc_csr A;
  double *ru, *rw, *rx;
};

typedef struct {
  int32_t c;
  double v;
} ent_t;

static int cmp_ent(const void *pa, const void *pb) {
  const ent_t *a = (const ent_t *)pa, *b = (const ent_t *)pb;
  return (a->c > b->c) - (a->c < b->c);
}

/* append rows [r0, r1) of R whose columns fall in [c0, c1), shifted by -shift */
static int copy_rows(rows_t *dst, const rows_t *src, int64_t r0, int64_t r1, int64_t c0, int64_t c1,
                     int64_t shift) {
  for (int64_t r = r0; r < r1; r++) {
    for (int64_t p = src->rp[r]; p < src->rp[r + 1]; p++) {
      int64_t c = src->ci[p];
      if (c >= c0 && c < c1)
        if (rows_push(dst, (int32_t)(c - shift), src->v[p])) return ORC_ERR_OOM;
    }
    rows_end(dst);
  }
  return ORC_OK;
}

void orc_free(orc_precond *P) {
  if (!P) return;
  free(P->perm);
  free(P->iperm);
  free(P->iface);
  free(P->offsets);
  rows_free(&P->LB);
  rows_free(&P->UB);
  rows_free(&P->Z);
  rows_free(&P->W);
  rows_free(&P->LS);
  rows_free(&P->US);
  rows_free(&P->Coff);
  rows_free(&P->St);
  free(P->DB);
  free(P->DS);
  free(P->lev_lb);
  free(P->lev_ub);
  free(P->lev_ls);
  free(P->lev_us);
  free(P->f);
  free(P->g);
  free(P->t);
  free(P->y);
  free(P->V);
  free(P->H);
  free(P->cs);
  free(P->sn);
  free(P->gg);
  free(P->c);
  free(P->w1);
  free(P->w2);
  orc_free(P->smoother);
  free(P->ru);
  free(P->rw);
  free(P->rx);
  free(P);
}

int orc_setup(const orc_csr *A, const int32_t *part_in, int32_t nparts, const orc_options *opt,
              orc_precond **out, int64_t *bad_row) {
  *out = NULL;
  int rc = orc_validate(A);
  if (rc) return rc;
  if (!opt || nparts < 1 || (opt->method != ORC_BJ && opt->method != ORC_SCHUR && opt->method != ORC_RAP))
    return ORC_ERR_INVALID_ARG;
  if (opt->method != ORC_BJ && opt->inner_iters < 0) return ORC_ERR_INVALID_ARG;
  const int64_t n = A->n;
  orc_precond *P = (orc_precond *)calloc(1, sizeof(orc_precond));
  if (!P) return ORC_ERR_OOM;
  P->n = n;
  P->nparts = nparts;
  P->opt = *opt;
  int32_t *part = (int32_t *)calloc((size_t)(n + 1), sizeof(int32_t));
  P->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  P->iperm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  P->iface = (uint8_t *)malloc((size_t)(n + 1));
  P->offsets = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * nparts + 2));
  orc_fact *F = NULL, *G = NULL;
  rows_t Ah, St;
  memset(&Ah, 0, sizeof(Ah));
  memset(&St, 0, sizeof(St));
  if (!part || !P->perm || !P->iperm || !P->iface || !P->offsets) {
    rc = ORC_ERR_OOM;
    goto fail;
  }
  if (part_in) memcpy(part, part_in, sizeof(int32_t) * (size_t)n);
  if ((rc = orc_classify(A, part, nparts, P->iface))) goto fail;
  if ((rc = orc_permutation(n, part, nparts, P->iface, P->perm, P->iperm, P->offsets))) goto fail;
  const int64_t nB = P->offsets[nparts], nS = n - nB;
  P->nB = nB;
  P->nS = nS;

  /* permuted intra-subdomain matrix and the cross-subdomain coupling C_off */
  if ((rc = rows_init(&Ah, n)) || (rc = rows_init(&P->Coff, nS))) goto fail;
  {
    ent_t *buf = (ent_t *)malloc(sizeof(ent_t) * (size_t)(n + 1));
    ent_t *bufo = (ent_t *)malloc(sizeof(ent_t) * (size_t)(n + 1));
    if (!buf || !bufo) {
      free(buf);
      free(bufo);
      rc = ORC_ERR_OOM;
      goto fail;
    }
    for (int64_t r = 0; r < n; r++) {
      int32_t i = P->perm[r];
      int64_t m = 0, mo = 0;
      for (int64_t p = A->row_ptr[i]; p < A->row_ptr[i + 1]; p++) {
        int32_t j = A->col[p];
        if (part[j] == part[i])
          buf[m++] = (ent_t){P->iperm[j], A->val[p]};
        else
          bufo[mo++] = (ent_t){(int32_t)(P->iperm[j] - nB), A->val[p]};
      }
      qsort(buf, (size_t)m, sizeof(ent_t), cmp_ent);
      for (int64_t k = 0; k < m; k++) rows_push(&Ah, buf[k].c, buf[k].v);
      rows_end(&Ah);
      if (r >= nB) {
        qsort(bufo, (size_t)mo, sizeof(ent_t), cmp_ent);
        for (int64_t k = 0; k < mo; k++) rows_push(&P->Coff, bufo[k].c, bufo[k].v);
        rows_end(&P->Coff);
      }
    }
    free(buf);
    free(bufo);
  }

  const orc_csr Mh = {n, Ah.rp, Ah.ci, Ah.v};
  const int schur = (opt->method == ORC_SCHUR);
  if ((rc = orc_factor(&Mh, schur ? nB : n, opt->interior_fact, opt->droptol, opt->lfil, opt->pivot_mode,
                       opt->pivot_tol, &F, bad_row)))
    goto fail;

  if ((rc = rows_init(&P->LB, nB)) || (rc = rows_init(&P->UB, nB)) || (rc = rows_init(&P->Z, nB)) ||
      (rc = rows_init(&P->W, nS)) || (rc = rows_init(&P->LS, nS)) || (rc = rows_init(&P->US, nS)))
    goto fail;
  P->DB = (double *)malloc(sizeof(double) * (size_t)(nB + 1));
  P->DS = (double *)malloc(sizeof(double) * (size_t)(nS + 1));
  if (!P->DB || !P->DS) {
    rc = ORC_ERR_OOM;
    goto fail;
  }
  copy_rows(&P->LB, &F->L, 0, nB, 0, nB, 0);
  copy_rows(&P->UB, &F->U, 0, nB, 0, nB, 0);
  copy_rows(&P->Z, &F->U, 0, nB, nB, n, 0);
  memcpy(P->DB, F->D, sizeof(double) * (size_t)nB);
  copy_rows(&P->W, &F->L, nB, n, 0, nB, 0);
  if (!schur) { /* block Jacobi: the full factor of each A_i */
    copy_rows(&P->LS, &F->L, nB, n, nB, n, nB);
    /* U rows of interface rows live at F->U rows nB..n */
    copy_rows(&P->US, &F->U, nB, n, nB, n, nB);
    memcpy(P->DS, F->D + nB, sizeof(double) * (size_t)nS);
  } else { /* two-level: factor the local Schur complements */
    if ((rc = rows_init(&St, nS))) goto fail;
    copy_rows(&St, &F->R, 0, nS, nB, n, nB);
    const orc_csr Sm = {nS, St.rp, St.ci, St.v};
    int64_t bad = -1;
    rc = orc_factor(&Sm, nS, opt->interface_fact, opt->droptol, opt->lfil, opt->pivot_mode, opt->pivot_tol, &G,
                    &bad);
    if (rc) {
      if (bad_row) *bad_row = bad >= 0 ? bad + nB : -1;
      goto fail;
    }
    copy_rows(&P->LS, &G->L, 0, nS, 0, nS, 0);
    copy_rows(&P->US, &G->U, 0, nS, 0, nS, 0);
    memcpy(P->DS, G->D, sizeof(double) * (size_t)nS);
    P->St = St;
    memset(&St, 0, sizeof(St));
  }

  P->lev_lb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nB + 1));
  P->lev_ub = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nB + 1));
  P->lev_ls = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nS + 1));
  P->lev_us = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nS + 1));
  if (!P->lev_lb || !P->lev_ub || !P->lev_ls || !P->lev_us) {
    rc = ORC_ERR_OOM;
    goto fail;
  }
  orc_levels(nB, P->LB.rp, P->LB.ci, 1, 0, nB, P->lev_lb);
  orc_levels(nB, P->UB.rp, P->UB.ci, 0, 0, nB, P->lev_ub);
  orc_levels(nS, P->LS.rp, P->LS.ci, 1, 0, nS, P->lev_ls);
  orc_levels(nS, P->US.rp, P->US.ci, 0, 0, nS, P->lev_us);

  {
    const int64_t k = opt->method != ORC_BJ ? opt->inner_iters : 0;
    P->f = (double *)malloc(sizeof(double) * (size_t)(nB + 1));
    P->g = (double *)malloc(sizeof(double) * (size_t)(nS + 1));
    P->t = (double *)malloc(sizeof(double) * (size_t)(nS + 1));
    P->y = (double *)malloc(sizeof(double) * (size_t)(nS + 1));
    P->V = (double *)malloc(sizeof(double) * (size_t)((k + 1) * nS + 1));
    P->H = (double *)calloc((size_t)((k + 1) * (k + 1) + 1), sizeof(double));
    P->cs = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    P->sn = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    P->gg = (double *)malloc(sizeof(double) * (size_t)(k + 2));
    P->c = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    P->w1 = (double *)malloc(sizeof(double) * (size_t)(nS + 1));
    P->w2 = (double *)malloc(sizeof(double) * (size_t)(nS + 1));
    if (!P->f || !P->g || !P->t || !P->y || !P->V || !P->H || !P->cs || !P->sn || !P->gg || !P->c || !P->w1 ||
        !P->w2) {
      rc = ORC_ERR_OOM;
      goto fail;
    }
  }
  if (opt->method == ORC_RAP) {
    /* the multiplicative method: the factors above (block-Jacobi form of each
     * A_i with interior_fact) give L_B, U_B, W, Z, L_S and U_S; the smoother is
     * a second block-Jacobi factorization with smooth_fact */
    orc_options so = *opt;
    so.method = ORC_BJ;
    so.interior_fact = opt->smooth_fact;
    if ((rc = orc_setup(A, part_in, nparts, &so, &P->smoother, bad_row))) goto fail;
    P->A = *A;
    P->ru = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    P->rw = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    P->rx = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!P->ru || !P->rw || !P->rx) {
      rc = ORC_ERR_OOM;
      goto fail;
    }
  }
  orc_fact_free(F);
  orc_fact_free(G);
  rows_free(&Ah);
  free(part);
  *out = P;
  return ORC_OK;
fail:
  orc_fact_free(F);
  orc_fact_free(G);
  rows_free(&Ah);
  rows_free(&St);
  free(part);
  orc_free(P);
  return rc;
}

/* x = (L_S U_S)^{-1} b on the interface unknowns (local Schur factors) */
static void schur_factor_solve(orc_precond *P, const double *b, double *x) {
  trsv_lower_unit(&P->LS, b, P->t);
  trsv_upper(&P->US, P->DS, P->t, x);
}

/* y = v + D^{-1} C_off v: the operator of the block-Jacobi preconditioned
 * reduced system, eq. (18)-(19) */
static void reduced_matvec(orc_precond *P, const double *v, double *y) {
  const rows_t *C = &P->Coff;
  for (int64_t i = 0; i < P->nS; i++) {
    double s = 0.0;
    for (int64_t p = C->rp[i]; p < C->rp[i + 1]; p++) s = fma(C->v[p], v[C->ci[p]], s);
    P->w1[i] = s;
  }
  schur_factor_solve(P, P->w1, P->w2);
  for (int64_t i = 0; i < P->nS; i++) y[i] = v[i] + P->w2[i];
}

/* Givens rotation zeroing b against a: r = sqrt(a^2 + b^2), c = a/r, s = b/r */
static void givens(double a, double b, double *c, double *s, double *r) {
  double rr = sqrt(fma(a, a, b * b));
  *r = rr;
  *c = a / rr;
  *s = b / rr;
}

/* out = R A P v for an interface vector v: P v = (-U_B^{-1} Z v; v), one
 * product with A in the original numbering, then R w = w_S - W L_B^{-1} w_B
 * (Section 3.3, eq. (21) and (28)); R, P and RAP stay unformed. */
void orc_rap_matvec(orc_precond *P, const double *v, double *out) {
  const int64_t n = P->n, nB = P->nB, nS = P->nS;
  double *t = P->f, *u = P->ru, *w = P->rw;
  for (int64_t i = 0; i < nB; i++) { /* t = -Z v */
    double s = 0.0;
    for (int64_t p = P->Z.rp[i]; p < P->Z.rp[i + 1]; p++) s = fma(-P->Z.v[p], v[P->Z.ci[p] - nB], s);
    t[i] = s;
  }
  trsv_upper(&P->UB, P->DB, t, t); /* y_B = -U_B^{-1} Z v */
  for (int64_t i = 0; i < nB; i++) u[P->perm[i]] = t[i];
  for (int64_t i = 0; i < nS; i++) u[P->perm[nB + i]] = v[i];
  orc_spmv(&P->A, u, w);
  for (int64_t i = 0; i < nB; i++) t[i] = w[P->perm[i]];
  trsv_lower_unit(&P->LB, t, t);
  for (int64_t i = 0; i < nS; i++) {
    double s = w[P->perm[nB + i]];
    for (int64_t p = P->W.rp[i]; p < P->W.rp[i + 1]; p++) s = fma(-P->W.v[p], t[P->W.ci[p]], s);
    out[i] = s;
  }
  (void)n;
}

/* the reduced operator of the multiplicative method, preconditioned by the
 * local Schur factors: y = (L_S U_S)^{-1} R A P v */
static void rap_op(orc_precond *P, const double *v, double *y) {
  orc_rap_matvec(P, v, P->w1);
  schur_factor_solve(P, P->w1, y);
}

/* y = v + D^{-1} C_off v for the additive method */
static void schur_op(orc_precond *P, const double *v, double *y) { reduced_matvec(P, v, y); }

/* k steps of GMRES (zero initial guess, modified Gram-Schmidt, Givens) on the
 * left-preconditioned reduced system op(y) = D^{-1} g': op is
 * I + D^{-1} C_off for the additive method (eq. (18)) and D^{-1} R A P for the
 * multiplicative one.  Stops early only on an exact breakdown or when
 * |g_{j+1}| <= inner_rtol * ||rhs||. */
static void inner_gmres(orc_precond *P, const double *gp, double *y,
                        void (*op)(orc_precond *, const double *, double *)) {
  const int64_t nS = P->nS;
  const int32_t k = P->opt.inner_iters;
  double *V = P->V, *H = P->H;
  const int64_t ldh = k + 1;
  schur_factor_solve(P, gp, V); /* rhs = D^{-1} g', kept in V[0] */
  double beta = nrm2(nS, V);
  for (int64_t i = 0; i < nS; i++) y[i] = 0.0;
  if (beta == 0.0 || k == 0) {
    if (k == 0) /* zero steps: fall back to the block-Jacobi solve */
      for (int64_t i = 0; i < nS; i++) y[i] = V[i];
    return;
  }
  for (int64_t i = 0; i < nS; i++) V[i] = V[i] / beta;
  P->gg[0] = beta;
  int32_t m = 0;
  for (int32_t j = 0; j < k; j++) {
    double *w = V + (int64_t)(j + 1) * nS;
    op(P, V + (int64_t)j * nS, w);
    for (int32_t i = 0; i <= j; i++) {
      double h = dot(nS, w, V + (int64_t)i * nS);
      H[i + ldh * j] = h;
      const double *vi = V + (int64_t)i * nS;
      for (int64_t l = 0; l < nS; l++) w[l] = fma(-h, vi[l], w[l]);
    }
    double hn = nrm2(nS, w);
    H[(j + 1) + ldh * j] = hn;
    for (int32_t i = 0; i < j; i++) {
      double a = H[i + ldh * j], b = H[(i + 1) + ldh * j];
      H[i + ldh * j] = fma(P->cs[i], a, P->sn[i] * b);
      H[(i + 1) + ldh * j] = fma(-P->sn[i], a, P->cs[i] * b);
    }
    double r;
    givens(H[j + ldh * j], H[(j + 1) + ldh * j], &P->cs[j], &P->sn[j], &r);
    H[j + ldh * j] = r;
    H[(j + 1) + ldh * j] = 0.0;
    P->gg[j + 1] = -P->sn[j] * P->gg[j];
    P->gg[j] = P->cs[j] * P->gg[j];
    m = j + 1;
    if (hn == 0.0) break;
    for (int64_t l = 0; l < nS; l++) w[l] = w[l] / hn;
    if (fabs(P->gg[j + 1]) <= P->opt.inner_rtol * beta) break;
  }
  for (int32_t i = m - 1; i >= 0; i--) { /* back substitution R c = g */
    double s = P->gg[i];
    for (int32_t l = i + 1; l < m; l++) s = fma(-H[i + ldh * l], P->c[l], s);
    P->c[i] = s / H[i + ldh * i];
  }
  for (int32_t i = 0; i < m; i++) {
    const double *vi = V + (int64_t)i * nS;
    for (int64_t l = 0; l < nS; l++) y[l] = fma(P->c[i], vi[l], y[l]);
  }
}

/* Multiplicative two-level solve (algorithm "Two-level multiplicative solve";
 * the GPU form of Section 3.3):
 * x = smoother(r); res = r - A x; the restriction g = res_S - W L_B^{-1} res_B;
 * v from k GMRES steps on (L_S U_S)^{-1} R A P v = (L_S U_S)^{-1} g; then the
 * interpolation z = x + P v = x + (-U_B^{-1} Z v; v). */
static void rap_apply(orc_precond *P, const double *r, double *z) {
  const int64_t n = P->n, nB = P->nB, nS = P->nS;
  double *f = P->f, *g = P->g, *y = P->y, *x = P->rx, *res = P->rw;
  orc_apply(P->smoother, r, x);
  orc_residual(&P->A, r, x, res);
  for (int64_t i = 0; i < nB; i++) f[i] = res[P->perm[i]];
  trsv_lower_unit(&P->LB, f, f);
  for (int64_t i = 0; i < nS; i++) {
    double s = res[P->perm[nB + i]];
    for (int64_t p = P->W.rp[i]; p < P->W.rp[i + 1]; p++) s = fma(-P->W.v[p], f[P->W.ci[p]], s);
    g[i] = s;
  }
  inner_gmres(P, g, y, rap_op);
  for (int64_t i = 0; i < nB; i++) { /* f = -Z v */
    double s = 0.0;
    for (int64_t p = P->Z.rp[i]; p < P->Z.rp[i + 1]; p++) s = fma(-P->Z.v[p], y[P->Z.ci[p] - nB], s);
    f[i] = s;
  }
  trsv_upper(&P->UB, P->DB, f, f);
  for (int64_t i = 0; i < nB; i++) z[P->perm[i]] = x[P->perm[i]] + f[i];
  for (int64_t i = 0; i < nS; i++) z[P->perm[nB + i]] = x[P->perm[nB + i]] + y[i];
  (void)n;
}

void orc_apply(orc_precond *P, const double *r, double *z) {
  const int64_t nB = P->nB, nS = P->nS;
  double *f = P->f, *g = P->g, *y = P->y;
  if (P->opt.method == ORC_RAP) {
    rap_apply(P, r, z);
    return;
  }
  for (int64_t i = 0; i < nB; i++) f[i] = r[P->perm[i]];
  for (int64_t i = 0; i < nS; i++) g[i] = r[P->perm[nB + i]];
  trsv_lower_unit(&P->LB, f, f); /* f' = L_B^{-1} f */
  for (int64_t i = 0; i < nS; i++) { /* g' = g - W f' */
    double s = g[i];
    for (int64_t p = P->W.rp[i]; p < P->W.rp[i + 1]; p++) s = fma(-P->W.v[p], f[P->W.ci[p]], s);
    g[i] = s;
  }
  if (P->opt.method == ORC_SCHUR)
    inner_gmres(P, g, y, schur_op);
  else
    schur_factor_solve(P, g, y);
  for (int64_t i = 0; i < nB; i++) { /* f'' = f' - Z y */
    double s = f[i];
    for (int64_t p = P->Z.rp[i]; p < P->Z.rp[i + 1]; p++) s = fma(-P->Z.v[p], y[P->Z.ci[p] - nB], s);
    f[i] = s;
  }
  trsv_upper(&P->UB, P->DB, f, f); /* u = U_B^{-1} f'' */
  for (int64_t i = 0; i < nB; i++) z[P->perm[i]] = f[i];
  for (int64_t i = 0; i < nS; i++) z[P->perm[nB + i]] = y[i];
}

int orc_export(const orc_precond *P, int32_t what, const void **ptr, int64_t *len) {
  const rows_t *R = NULL;
  int base = 0;
  switch (what) {
    case ORC_X_PERM: *ptr = P->perm; *len = P->n; return ORC_OK;
    case ORC_X_IPERM: *ptr = P->iperm; *len = P->n; return ORC_OK;
    case ORC_X_IFACE: *ptr = P->iface; *len = P->n; return ORC_OK;
    case ORC_X_OFFSETS: *ptr = P->offsets; *len = 2 * P->nparts + 2; return ORC_OK;
    case ORC_X_DB: *ptr = P->DB; *len = P->nB; return ORC_OK;
    case ORC_X_DS: *ptr = P->DS; *len = P->nS; return ORC_OK;
    case ORC_X_LEV_LB: *ptr = P->lev_lb; *len = P->nB; return ORC_OK;
    case ORC_X_LEV_UB: *ptr = P->lev_ub; *len = P->nB; return ORC_OK;
    case ORC_X_LEV_LS: *ptr = P->lev_ls; *len = P->nS; return ORC_OK;
    case ORC_X_LEV_US: *ptr = P->lev_us; *len = P->nS; return ORC_OK;
    default: break;
  }
  if (what >= ORC_X_LB && what < ORC_X_LB + 3) { R = &P->LB; base = ORC_X_LB; }
  else if (what >= ORC_X_UB && what < ORC_X_UB + 3) { R = &P->UB; base = ORC_X_UB; }
  else if (what >= ORC_X_Z && what < ORC_X_Z + 3) { R = &P->Z; base = ORC_X_Z; }
  else if (what >= ORC_X_W && what < ORC_X_W + 3) { R = &P->W; base = ORC_X_W; }
  else if (what >= ORC_X_LS && what < ORC_X_LS + 3) { R = &P->LS; base = ORC_X_LS; }
  else if (what >= ORC_X_US && what < ORC_X_US + 3) { R = &P->US; base = ORC_X_US; }
  else if (what >= ORC_X_COFF && what < ORC_X_COFF + 3) { R = &P->Coff; base = ORC_X_COFF; }
  else if (what >= ORC_X_STILDE && what < ORC_X_STILDE + 3) { R = &P->St; base = ORC_X_STILDE; }
  if (!R) return ORC_ERR_INVALID_ARG;
  if (!R->rp) { *ptr = NULL; *len = 0; return ORC_OK; }
  switch (what - base) {
    case 0: *ptr = R->rp; *len = R->n + 1; break;
    case 1: *ptr = R->ci; *len = R->rp[R->n]; break;
    default: *ptr = R->v; *len = R->rp[R->n]; break;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* flexible GMRES(m), right preconditioned                                   */
/* ------------------------------------------------------------------------ */
int orc_fgmres(const orc_csr *A, orc_precond *P, const double *b, double *x, double rtol, int32_t restart,
               int32_t maxit, orc_result *res, double *hist) {
  const int64_t n = A->n;
  if (restart < 1 || maxit < 0 || rtol < 0) return ORC_ERR_INVALID_ARG;
  const int32_t m = restart;
  double *V = (double *)malloc(sizeof(double) * (size_t)((m + 1) * n + 1));
  double *Zb = (double *)malloc(sizeof(double) * (size_t)(m * n + 1));
  double *H = (double *)calloc((size_t)((m + 1) * (m + 1)), sizeof(double));
  double *cs = (double *)malloc(sizeof(double) * (size_t)(m + 1));
  double *sn = (double *)malloc(sizeof(double) * (size_t)(m + 1));
  double *g = (double *)malloc(sizeof(double) * (size_t)(m + 2));
  double *c = (double *)malloc(sizeof(double) * (size_t)(m + 1));
  double *r = (double *)malloc(sizeof(double) * (size_t)(n + 1));
  int rc = ORC_OK;
  if (!V || !Zb || !H || !cs || !sn || !g || !c || !r) {
    rc = ORC_ERR_OOM;
    goto out;
  }
  const int64_t ldh = m + 1;
  const double bnorm = nrm2(n, b);
  int32_t its = 0;
  int converged = 0;
  double relres = 0.0;
  if (bnorm == 0.0) {
    for (int64_t i = 0; i < n; i++) x[i] = 0.0;
    converged = 1;
    if (hist) hist[0] = 0.0;
    goto finish;
  }
  orc_residual(A, b, x, r);
  double beta = nrm2(n, r);
  relres = beta / bnorm;
  if (hist) hist[0] = relres;
  if (!isfinite(beta)) {
    rc = ORC_ERR_BREAKDOWN;
    goto out;
  }
  if (beta <= rtol * bnorm) {
    converged = 1;
    goto finish;
  }
  while (its < maxit) {
    for (int64_t i = 0; i < n; i++) V[i] = r[i] / beta;
    g[0] = beta;
    int32_t jm = 0;
    int stop = 0;
    for (int32_t j = 0; j < m && !stop; j++) {
      double *zj = Zb + (int64_t)j * n;
      double *w = V + (int64_t)(j + 1) * n;
      orc_apply(P, V + (int64_t)j * n, zj);
      orc_spmv(A, zj, w);
      for (int32_t i = 0; i <= j; i++) {
        double h = dot(n, w, V + (int64_t)i * n);
        H[i + ldh * j] = h;
        const double *vi = V + (int64_t)i * n;
        for (int64_t l = 0; l < n; l++) w[l] = fma(-h, vi[l], w[l]);
      }
      double hn = nrm2(n, w);
      H[(j + 1) + ldh * j] = hn;
      for (int32_t i = 0; i < j; i++) {
        double a = H[i + ldh * j], bb = H[(i + 1) + ldh * j];
        H[i + ldh * j] = fma(cs[i], a, sn[i] * bb);
        H[(i + 1) + ldh * j] = fma(-sn[i], a, cs[i] * bb);
      }
      double rr;
      givens(H[j + ldh * j], H[(j + 1) + ldh * j], &cs[j], &sn[j], &rr);
      H[j + ldh * j] = rr;
      H[(j + 1) + ldh * j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      its++;
      jm = j + 1;
      if (!isfinite(hn) || !isfinite(g[j + 1])) {
        rc = ORC_ERR_BREAKDOWN;
        goto out;
      }
      if (hist) hist[its] = fabs(g[j + 1]) / bnorm;
      if (hn == 0.0) stop = 1;
      else
        for (int64_t l = 0; l < n; l++) w[l] = w[l] / hn;
      if (fabs(g[j + 1]) <= rtol * bnorm || its >= maxit) stop = 1;
    }
    for (int32_t i = jm - 1; i >= 0; i--) {
      double s = g[i];
      for (int32_t l = i + 1; l < jm; l++) s = fma(-H[i + ldh * l], c[l], s);
      c[i] = s / H[i + ldh * i];
    }
    for (int32_t i = 0; i < jm; i++) {
      const double *zi = Zb + (int64_t)i * n;
      for (int64_t l = 0; l < n; l++) x[l] = fma(c[i], zi[l], x[l]);
    }
    orc_residual(A, b, x, r);
    beta = nrm2(n, r);
    relres = beta / bnorm;
    if (!isfinite(beta)) {
      rc = ORC_ERR_BREAKDOWN;
      goto out;
    }
    if (beta <= rtol * bnorm) {
      converged = 1;
      break;
    }
  }
finish:
  if (res) {
    res->iterations = its;
    res->converged = converged;
    res->final_relres = relres;
  }
  rc = converged ? ORC_OK : ORC_NOT_CONVERGED;
out:
  free(V);
  free(Zb);
  free(H);
  free(cs);
  free(sn);
  free(g);
  free(c);
  free(r);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* GMRES(m), right preconditioned, with a fixed preconditioner               */
/* ------------------------------------------------------------------------ */
/* The batched systems use plain GMRES: the Arnoldi process runs on A M^{-1}
 * (w = A (M^{-1} v_j)), only the basis V is kept, and at the end of a cycle
 * the correction is x += M^{-1} (V c) -- one more preconditioner solve per
 * cycle instead of m stored preconditioned vectors.  Orthogonalization,
 * rotations, the convergence test and the iteration count are those of the
 * flexible variant above. */
int orc_gmres(const orc_csr *A, orc_precond *P, const double *b, double *x, double rtol, int32_t restart,
              int32_t maxit, orc_result *res, double *hist) {
  const int64_t n = A->n;
  if (restart < 1 || maxit < 0 || rtol < 0) return ORC_ERR_INVALID_ARG;
  const int32_t m = restart;
  double *V = (double *)malloc(sizeof(double) * (size_t)((m + 1) * n + 1));
  double *H = (double *)calloc((size_t)((m + 1) * (m + 1)), sizeof(double));
  double *cs = (double *)malloc(sizeof(double) * (size_t)(m + 1));
  double *sn = (double *)malloc(sizeof(double) * (size_t)(m + 1));
  double *g = (double *)malloc(sizeof(double) * (size_t)(m + 2));
  double *c = (double *)malloc(sizeof(double) * (size_t)(m + 1));
  double *r = (double *)malloc(sizeof(double) * (size_t)(n + 1));
  double *z = (double *)malloc(sizeof(double) * (size_t)(n + 1));
  double *u = (double *)malloc(sizeof(double) * (size_t)(n + 1));
  int rc = ORC_OK;
  if (!V || !H || !cs || !sn || !g || !c || !r || !z || !u) {
    rc = ORC_ERR_OOM;
    goto out;
  }
  const int64_t ldh = m + 1;
  const double bnorm = nrm2(n, b);
  int32_t its = 0;
  int converged = 0;
  double relres = 0.0;
  if (bnorm == 0.0) {
    for (int64_t i = 0; i < n; i++) x[i] = 0.0;
    converged = 1;
    if (hist) hist[0] = 0.0;
    goto finish;
  }
  orc_residual(A, b, x, r);
  double beta = nrm2(n, r);
  relres = beta / bnorm;
  if (hist) hist[0] = relres;
  if (!isfinite(beta)) {
    rc = ORC_ERR_BREAKDOWN;
    goto out;
  }
  if (beta <= rtol * bnorm) {
    converged = 1;
    goto finish;
  }
  while (its < maxit) {
    for (int64_t i = 0; i < n; i++) V[i] = r[i] / beta;
    g[0] = beta;
    int32_t jm = 0;
    int stop = 0;
    for (int32_t j = 0; j < m && !stop; j++) {
      double *w = V + (int64_t)(j + 1) * n;
      orc_apply(P, V + (int64_t)j * n, z); /* z = M^{-1} v_j */
      orc_spmv(A, z, w);                   /* w = A z */
      for (int32_t i = 0; i <= j; i++) {
        double h = dot(n, w, V + (int64_t)i * n);
        H[i + ldh * j] = h;
        const double *vi = V + (int64_t)i * n;
        for (int64_t l = 0; l < n; l++) w[l] = fma(-h, vi[l], w[l]);
      }
      double hn = nrm2(n, w);
      H[(j + 1) + ldh * j] = hn;
      for (int32_t i = 0; i < j; i++) {
        double a = H[i + ldh * j], bb = H[(i + 1) + ldh * j];
        H[i + ldh * j] = fma(cs[i], a, sn[i] * bb);
        H[(i + 1) + ldh * j] = fma(-sn[i], a, cs[i] * bb);
      }
      double rr;
      givens(H[j + ldh * j], H[(j + 1) + ldh * j], &cs[j], &sn[j], &rr);
      H[j + ldh * j] = rr;
      H[(j + 1) + ldh * j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      its++;
      jm = j + 1;
      if (!isfinite(hn) || !isfinite(g[j + 1])) {
        rc = ORC_ERR_BREAKDOWN;
        goto out;
      }
      if (hist) hist[its] = fabs(g[j + 1]) / bnorm;
      if (hn == 0.0) stop = 1;
      else
        for (int64_t l = 0; l < n; l++) w[l] = w[l] / hn;
      if (fabs(g[j + 1]) <= rtol * bnorm || its >= maxit) stop = 1;
    }
    for (int32_t i = jm - 1; i >= 0; i--) {
      double s = g[i];
      for (int32_t l = i + 1; l < jm; l++) s = fma(-H[i + ldh * l], c[l], s);
      c[i] = s / H[i + ldh * i];
    }
    for (int64_t l = 0; l < n; l++) u[l] = 0.0; /* u = V c, then x += M^{-1} u */
    for (int32_t i = 0; i < jm; i++) {
      const double *vi = V + (int64_t)i * n;
      for (int64_t l = 0; l < n; l++) u[l] = fma(c[i], vi[l], u[l]);
    }
    orc_apply(P, u, z);
    for (int64_t l = 0; l < n; l++) x[l] = x[l] + z[l];
    orc_residual(A, b, x, r);
    beta = nrm2(n, r);
    relres = beta / bnorm;
    if (!isfinite(beta)) {
      rc = ORC_ERR_BREAKDOWN;
      goto out;
    }
    if (beta <= rtol * bnorm) {
      converged = 1;
      break;
    }
  }
finish:
  if (res) {
    res->iterations = its;
    res->converged = converged;
    res->final_relres = relres;
  }
  rc = converged ? ORC_OK : ORC_NOT_CONVERGED;
out:
  free(V);
  free(H);
  free(cs);
  free(sn);
  free(g);
  free(c);
  free(r);
  free(z);
  free(u);
  return rc;
}
