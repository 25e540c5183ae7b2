// launch.hpp -- host-side launchers of the gfx950 kernels (internal interface
// between the kernel translation units and the runtime in capi.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct ilu_precond;

namespace silu {

int check_launch(const char *what);  // records a HIP launch error, returns ILU_ERR_HIP or 0

// ---- capi.cpp: runtime services for the serving engine (serve.cpp) ----
int api_fail(int code, const char *fmt, ...);  // sets ilu_last_error of this thread, returns code
int64_t precond_bytes(const ::ilu_precond *P);   // device bytes held by a handle (factors, schedules, workspaces)
// destroy a handle with no work queued on its blocks (its streams were
// synchronised), without the device-wide wait of ilu_destroy
void precond_destroy_idle(::ilu_precond *P);
int dev_alloc(void **p, size_t bytes);  // from the library's device block cache
void dev_free(void *p);

// ---- prims.hip ----
// out[0..n] = exclusive scan of in[0..n-1], out[n] = total (out may not alias in)
int scan_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp, size_t tmp_bytes, hipStream_t s);
size_t scan_tmp_bytes(int64_t n);
// stable LSD radix sort of (key, val) by key (keys < 2^key_bits); results in key_out/val_out
int radix_sort(const uint32_t *key_in, const int32_t *val_in, uint32_t *key_out, int32_t *val_out, int64_t n,
               int key_bits, void *tmp, size_t tmp_bytes, hipStream_t s);
size_t radix_tmp_bytes(int64_t n);
int histogram_keys(const uint32_t *key, int64_t n, int64_t nbins, int64_t *counts, hipStream_t s);
int fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
int fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);
int fill_f64(double *p, double v, int64_t n, hipStream_t s);
int iota_i32(int32_t *p, int64_t n, hipStream_t s);
int max_i32(const int32_t *p, int64_t n, int32_t *d_out, hipStream_t s);

// ---- setup.hip ----
int launch_validate(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nnz, const int32_t *part, int32_t nparts,
                    void *status, hipStream_t s);
int launch_classify(const int64_t *rp, const int32_t *ci, int64_t n, const int32_t *part, uint8_t *iface,
                    hipStream_t s);
int launch_perm_keys(int64_t n, const int32_t *part, int32_t nparts, const uint8_t *iface, uint32_t *key,
                     int32_t *val, hipStream_t s);
int launch_inverse_perm(int64_t n, const int32_t *perm, int32_t *iperm, hipStream_t s);
int launch_extract_counts(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nB, const int32_t *part,
                          const int32_t *perm, int64_t *cnt_intra, int64_t *cnt_cross, hipStream_t s);
int launch_extract_fill(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, int64_t nB,
                        const int32_t *part, const int32_t *perm, const int32_t *iperm, const int64_t *rp_intra,
                        int32_t *ci_intra, double *v_intra, const int64_t *rp_cross, int32_t *ci_cross,
                        double *v_cross, hipStream_t s);

// ---- factor.hip ----
struct FactLaunch {
  const int64_t *rp;
  const int32_t *ci;
  const double *v;
  int64_t n, nfull;
  int32_t method;
  double droptol;
  int32_t lfil;
  int32_t pivot_mode;
  double pivot_tol;
  int64_t nchunks;
  const int32_t *chunks;        // int2 {first row, rows} per chunk, stream after stream
  int64_t nstreams, ninit;      // streams; the first ninit get the workgroups at the start
  const int64_t *stream_chunk;  // [nstreams+1]
  unsigned int *ticket;         // [nstreams], zeroed
  const int64_t *Lrp;
  int32_t *Lc;
  double *Lv;
  int32_t *Llen;
  const int64_t *Urp;
  int32_t *Uc;
  double *Uv;
  int32_t *Ulen;
  const int64_t *Rrp;
  int32_t *Rc;
  double *Rv;
  int32_t *Rlen;
  double *D;
  int *done;
  int epoch;
  void *status;
  int64_t grid;  // workgroups, all resident (factor_resident_groups), >= ninit
};
int factor_resident_groups(int num_cu);
// histograms (2 x 32 buckets, zeroed) of log2 of each row's second-nearest and farthest lower (upper)
// neighbour distance
int launch_gap_hist(const int64_t *rp, const int32_t *ci, int64_t n, bool upper, unsigned long long *hist,
                    hipStream_t s);
int launch_fact_caps(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nfull, int32_t method, int32_t lfil,
                     int64_t *Lcap, int64_t *Ucap, int64_t *Rcap, hipStream_t s);
int launch_factor_rows(const FactLaunch &f, hipStream_t s);
// ILU(0) / MILU(0) of rows rows[0 .. cnt) of one level of the lower pattern
// over the interior columns (every earlier level already factored; partial
// rows, r >= nfull, take interior pivots only): the same factors as
// launch_factor_rows
int launch_factor_level(const FactLaunch &f, const int32_t *rows, int64_t cnt, hipStream_t s);
// *out = max(*out, longest of rows [0, n))
int launch_row_len_max(const int64_t *rp, int64_t n, int *out, hipStream_t s);
int launch_compact_rows(int64_t nrows, const int64_t *cap_rp, const int32_t *len, const int32_t *sc,
                        const double *sv, const int64_t *out_rp, int32_t *oc, double *ov, int64_t col_lo,
                        int64_t col_hi, int64_t shift, hipStream_t s);
int launch_count_rows(int64_t nrows, const int64_t *cap_rp, const int32_t *len, const int32_t *sc, int64_t col_lo,
                      int64_t col_hi, int64_t *cnt, hipStream_t s);
constexpr int FACT_WAVES = 2;         // waves per factorization workgroup (rows of a chunk interleaved over them)
constexpr int FACT_PART_B_CHUNK = 4;  // rows per chunk of a partial factorization's interface rows

constexpr int LEVEL_CHUNK_MAX = 256;  // rows per chunk of the level sweep
constexpr int LEVEL_WAVES = 2;        // waves per level-sweep workgroup, taking a chunk's rows in turn
// Level sweep over a stream schedule (build_streams); done[] zeroed, grid
// workgroups all resident (levels_resident_groups) and >= ninit.
int levels_resident_groups(int num_cu);
// levels of rows [row0, n) of a lower factor whose dependencies (columns in [lo, hi), below the row) are known
int launch_rows_level(const int64_t *rp, const int32_t *ci, int64_t row0, int64_t n, int64_t lo, int64_t hi,
                      int32_t *level, hipStream_t s);
int launch_levels_stream(const int64_t *rp, const int32_t *ci, bool lower, int64_t lo, int64_t hi,
                         const int32_t *chunks, int64_t nstreams, int64_t ninit, const int64_t *stream_chunk,
                         unsigned int *ticket, int32_t *level, int *done, void *status, int64_t grid, hipStream_t s);
// chunk table of a level-ordered row list: level_ptr[nlev+1] -> chunks of <= 64 rows
int launch_level_chunk_counts(const int64_t *level_ptr, int64_t nlev, int64_t *cnt, hipStream_t s);
int launch_level_chunks(const int64_t *level_ptr, int64_t nlev, const int64_t *chunk_base, int32_t *chunk_start,
                        int32_t *chunk_level, hipStream_t s);
int launch_levels_to_keys(const int32_t *level, int64_t n, uint32_t *key, int32_t *val, hipStream_t s);

// ---- trsv.hip ----
struct TrsvLaunch {
  int64_t nrows;           // rows in this solve
  const int32_t *rows;     // level-ordered row ids (nrows)
  const int32_t *chunk_start;  // [nchunks+1]
  const int32_t *chunk_level;  // [nchunks]
  int64_t nchunks;
  const int64_t *level_ptr;  // [nlev+1]
  unsigned long long *level_done;  // [nlev] cumulative counters
  unsigned long long epoch;
  unsigned long long *ticket;
  unsigned long long ticket_base;
  const int64_t *rp;
  const int32_t *ci;
  const double *v;
  const double *diag;      // NULL -> unit diagonal
  int64_t split_col;       // upper solves: columns >= split_col are processed first (Z part)
  const double *b;         // right-hand side base (block-local: in position order)
  const int32_t *b_map;    // rhs index = b_map ? b_map[row] : row (global solve)
  double *x;               // solution, indexed by row; columns index x too
                           // (block-local: the output vector, see out_map)
  double *scatter_out;     // optional: scatter_out[scatter_map[row]] = x
  const int32_t *scatter_map;
  void *status;
  int64_t max_waves;
  int role;  // 0 L_B|W, 1 U_B|Z, 2 L_S, 3 U_S
  // block-local schedule (launch_trsv_block)
  int64_t nblk;
  int64_t nlev_blk;
  const int32_t *blk_rows;     // rows sorted by (block, level)
  const int32_t *blk_lev_ptr;  // [nblk * nlev_blk + 1]
  // block-local storage (launch_trsv_lds): fixed-stride dependency entries
  const void *lds_c;       // (nrows + 1) * G * E 16-bit window slots, one word of E per lane
  const void *lds_v;       // (nrows + 1) * G * E values in the storage precision, in planes of one
                           // word (16 bytes or E values) per lane
  const int32_t *lds_rec;  // int4 per position (+ dummy): {row or ~row, output index, diagonal}
  const int32_t *out_map;  // row -> index of its solution in x (the output index of its position)
  int32_t lds_g;           // lanes per row: 1 (E = 2, 4), or 1, 2, 4, 8 (E = 8)
  int32_t lds_e;           // entries per lane: 2, 4 or 8
  int32_t lds_bt;          // threads per workgroup (multiple of 64, <= 512)
  int32_t lds_fast;        // no slow row, every level within bt / G rows: the solve skips both checks
  // storage precision of the factor values (0 FP64, 1 FP32, 2 FP16 scaled per
  // row), both modes; the level-scheduled solve reads v_lp, diag_lp and
  // scale_lp instead of v and diag when it is not 0
  int32_t prec;
  const void *v_lp;
  const float *diag_lp;
  const float *scale_lp;
  int64_t f64_row = INT64_MAX;  // level-scheduled lower solve: rows from here on (W) stay FP64
  // block split over several workgroups (launch_trsv_lds_split; nblk counts
  // the parts): exchange slots, the exports ({position, slot}) and imports by
  // (part, level), their number, and the start-order ticket
  double *xv = nullptr;
  const int32_t *xe = nullptr;
  const int32_t *elp = nullptr;
  const int32_t *ilp = nullptr;
  const int32_t *lrange = nullptr;  // int2 per part: first level, number of levels
  int64_t xlevels = 0;              // the most levels of any part
  int64_t nimp = 0;
  unsigned long long *xticket = nullptr;
};
int launch_trsv(const TrsvLaunch &t, hipStream_t s);
// FP32 / FP16 copies of a factor's values (and FP32 diagonal) for the
// level-scheduled solve; prec 1 FP32, 2 FP16 divided by the largest
// magnitude of the row's entries in columns < col_lim (scale[n] receives it)
int launch_lowp_factor(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, int64_t col_lim, int prec,
                       void *out, float *scale, const double *diag, float *diag_out, hipStream_t s);
int launch_trsv_lds(const TrsvLaunch &t, hipStream_t s);
// the block-local L_S and U_S solves of each subdomain in one launch, when
// both have the same lane shape (trsv_lds_pair_ok)
bool trsv_lds_pair_ok(const TrsvLaunch &lo, const TrsvLaunch &up);
int launch_trsv_lds_pair(const TrsvLaunch &lo, const TrsvLaunch &up, hipStream_t s);
// y[q] = x[map[q]]
int launch_gather(const double *x, const int32_t *map, int64_t n, double *y, hipStream_t s);
int launch_gather_i32(const int32_t *x, const int32_t *map, int64_t n, int32_t *y, hipStream_t s);
// a CSR with rows reordered (new row q = old row row0 + rows[q]) and columns c -> cmap[c - col_off]:
// the row lengths, then (orp from their scan) the entries in their old order
int launch_csr_perm_len(const int64_t *rp, int64_t row0, const int32_t *rows, int64_t nrows, int64_t *len,
                        hipStream_t s);
int launch_csr_perm_ent(const int64_t *rp, const int32_t *ci, const double *v, int64_t row0, const int32_t *rows,
                        int64_t nrows, const int32_t *cmap, int64_t col_off, const int64_t *orp, int32_t *oci,
                        double *ov, hipStream_t s);
// n rows of a unit lower factor whose dependencies are all solved (columns in
// x's order): out[i] = b[bmap[i]] - sum_j l_ij x_j in column order
int launch_rows_lower(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *b,
                      const int32_t *bmap, const double *x, double *out, hipStream_t s);
// out[q] = f[fmap[q]] - sum_j Z_qj y_j, in column order (f NULL: out = -Z y)
int launch_upper_rhs(const int32_t *fmap, int64_t n, const double *f, const int64_t *rp, const int32_t *ci,
                     const double *v, const double *y, double *out, hipStream_t s);
// z[mb[q]] = u[q] (q < nb), z[ms[q]] = y[q] (q < ns); with add non-NULL,
// z[t] = add[t] + (that value)
int launch_finish(const double *u, const int32_t *mb, int64_t nb, const double *y, const int32_t *ms, int64_t ns,
                  const double *add, double *z, hipStream_t s);
// block-local storage: pos[rows[q]] = q, the longest dependency row and the
// widest level (maxent, maxw must be zeroed), then the fixed-stride fill
int launch_lds_prepare(const int32_t *rows, const int64_t *rp, const int32_t *ci, int64_t n, int64_t split,
                       const int32_t *lev_ptr, int64_t nseg, int32_t *pos, int32_t *maxent, int32_t *maxw,
                       hipStream_t s);
int launch_lds_fill(const int32_t *rows, const int64_t *rp, const int32_t *ci, const double *v, const double *diag,
                    int64_t n, int64_t split, const int32_t *pos, const int32_t *lev_ptr, int64_t nseg, int G, int E,
                    int prec, const int32_t *omap, uint16_t *oc, void *ov, int32_t *rec, int *any_slow,
                    const int32_t *part, const int32_t *xrow, int32_t K1, const int32_t *ilp, int64_t nlev,
                    hipStream_t s);
// ---- block-local solve split over several workgroups per block (trsv_split.hip) ----
constexpr int SPLIT_LEVELS = 4096;  // levels of one part of a split solve (its pointers are held in LDS)
// the split solve (TrsvLaunch with xv, xidx, ilp, nimp, xticket; check-free factors only)
int launch_trsv_lds_split(const TrsvLaunch &t, hipStream_t s);
// part of each of n rows: K equal ranges of its block (starts bs[0..nblk]),
// numbered from the block's end for a backward solve
int launch_split_parts(const int64_t *bs, int32_t nblk, int64_t n, int32_t K, bool backward, int32_t *part,
                       hipStream_t s);
// per row: dependencies (columns < split) on rows of other parts
int launch_cross_count(const int64_t *rp, const int32_t *ci, int64_t n, int64_t split, const int32_t *part,
                       int64_t *cnt, hipStream_t s);
// one record per such dependency: source row, importing part * nlev + level
int launch_cross_emit(const int64_t *rp, const int32_t *ci, int64_t n, int64_t split, const int32_t *part,
                      const int32_t *level, int64_t nlev, const int64_t *off, uint32_t *src, int32_t *key,
                      hipStream_t s);
// on records sorted by (source, key): head flags (one import per source and
// importing part); bad[1] a source not in an earlier part
int launch_cross_heads(const uint32_t *src, const int32_t *key, int64_t m, const int32_t *part, int64_t nlev,
                       int64_t *head, int32_t *bad, hipStream_t s);
int launch_cross_compact(const uint32_t *src, const int32_t *key, int64_t m, const int64_t *head, const int64_t *rank,
                         uint32_t *isrc, uint32_t *ikey, hipStream_t s);
// xrow[source row * K1 + importing part - part of the row - 1] = import index
// (xrow preset to -1; K1 = parts per subdomain - 1)
int launch_cross_slots(const int32_t *isrc, const uint32_t *ikey, int64_t nimp, const int32_t *part, int64_t nlev,
                       int32_t K1, int32_t *xrow, hipStream_t s);
// bad[2]: an import out of its part's LDS ring when read; bad[3]: more than
// 64 imports needed by one level of one part
int launch_cross_check(const int64_t *rp, const int32_t *ci, int64_t n, int64_t split, const int32_t *part,
                       const int32_t *level, int64_t nlev, const int32_t *xrow, int32_t K1, const int32_t *ilp,
                       int32_t *bad, hipStream_t s);
int launch_cross_width(const int32_t *ilp, int64_t nkeys, int32_t *bad, hipStream_t s);
// lowest and highest level of each part's rows (lmin preset to INT32_MAX, lmax to -1)
int launch_part_levels(const int32_t *part, const int32_t *level, int64_t n, int32_t *lmin, int32_t *lmax,
                       hipStream_t s);
// the n words of the exchange array set to "not written"
int launch_fill_unset(double *xv, int64_t n, hipStream_t s);
// exports, one per import gi (source row isrc[gi]): key part * nlev + level
// of the source row, value gi
int launch_export_keys(const int32_t *isrc, int64_t nimp, const int32_t *part, const int32_t *level, int64_t nlev,
                       uint32_t *key, int32_t *val, hipStream_t s);
// xe[e] = {position of the source row, slot} for exports sorted by key
// (egi: their import indices), and the idle entry xe[nimp] = {0, 0}
int launch_export_fill(const int32_t *egi, const int32_t *isrc, const int32_t *pos, int64_t nimp, int32_t *xe,
                       hipStream_t s);
// block id of each row from ascending block starts (s1 below split, s2 from split on; s2 may be NULL)
int launch_row_blocks(int64_t nrows, int32_t nblk, const int64_t *s1, const int64_t *s2, int64_t split, int32_t *blk,
                      hipStream_t s);
int launch_block_level_keys(const int32_t *level, const int32_t *blk, int64_t n, int64_t nlev, uint32_t *key,
                            int32_t *val, hipStream_t s);
// Connected components of the union of two patterns on rows [0, n) (edges
// (r, c) with c in [0, n); rp2 may be NULL): root[i] = the smallest row of
// i's component, isroot[i] = 1 for those rows (lab: n words of scratch).
int launch_cc_label(const int64_t *rp1, const int32_t *ci1, const int64_t *rp2, const int32_t *ci2, int64_t n,
                    int32_t *lab, int32_t *root, int64_t *isroot, hipStream_t s);
// comp[i] = rank[root[i]] (rank: exclusive scan of isroot)
int launch_cc_number(const int32_t *root, const int64_t *rank, int64_t n, int32_t *comp, hipStream_t s);
int launch_i64_to_i32(const int64_t *in, int32_t *out, int64_t n, hipStream_t s);

// ---- batch.hip ----
constexpr int BATCH_THREADS = 256;  // default threads per workgroup of the batched solve (256 or 512)
constexpr int BATCH_RING = 2048;    // solution ring of a batched triangular solve (positions)
constexpr int BATCH_MMAX = 32;      // largest restart of the batched GMRES
constexpr int BATCH_LEVMAX = 1024;  // levels per triangular factor of one batched system
constexpr int BATCH_RMAX = 16;      // entries per row of a batched system
struct BatchLaunch {
  int32_t nsys;
  const int64_t *sys_row;
  const int32_t *order;
  const int32_t *nlevL, *nlevU, *levL, *levU;
  const uint8_t *wide;
  const int64_t *rp;
  const int32_t *ci;
  const double *av;
  const int64_t *dpos;
  double *lu;
  const int32_t *Lrow, *Urow, *Lout;
  const uint32_t *Lslot, *Uslot;
  const int64_t *Lsrc, *Usrc;
  double *Lval, *Uval, *Udiag;
  const double *b;
  double *x;
  double *V, *y, *u, *z, *t;
  double rtol;
  int m, maxit, merge, E, bt;
  int64_t grid;
  unsigned int *ticket;
  int32_t *iters, *status;
  double *relres;
};
// reset of the ticket counter, then the persistent factor + solve kernel
int launch_batch_solve(const BatchLaunch &L, hipStream_t s);
int batch_resident_groups(int num_cu, int E, int bt);  // bt: 256 or 512 threads per workgroup
int launch_row_sys(const int64_t *sys_row, int32_t nsys, int32_t *row_sys, hipStream_t s);
// out[q] = upos[lrows[q]] - (first row of that row's system): where the lower solve writes each solution
int launch_batch_lout(const int32_t *lrows, const int32_t *upos, const int64_t *sys_row, const int32_t *row_sys,
                      int64_t n, int32_t *out, hipStream_t s);
int launch_batch_levels(const int32_t *blk_lev_ptr, int64_t nlev_all, const int64_t *sys_row, int32_t nsys,
                        int levmax1, int32_t *levrel, int32_t *nlev, uint8_t *wide, bool or_wide, hipStream_t s);
int launch_batch_fill(const int32_t *pos_rows, int64_t n, const int64_t *sys_row, const int32_t *row_sys,
                      const int32_t *inv_pos, const int32_t *lev_of, const int32_t *levrel, int levmax1,
                      const int64_t *rp, const int32_t *ci, bool upper, int E, int32_t *prow, uint32_t *pslot,
                      int64_t *psrc, int64_t *dpos, int32_t *err, hipStream_t s);

// ---- krylov.hip ----
// kernel instance of a product, so that profilers report the outer matrix and
// the reduced system's coupling apart
enum SpmvTag { SPMV_A = 0, SPMV_COFF = 1, SPMV_USER = 2 };
int launch_spmv(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *x, double *y,
                hipStream_t s, SpmvTag tag = SPMV_USER);
int launch_residual(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *b,
                    const double *x, double *r, hipStream_t s);
constexpr int RED_BLOCKS = 512;  // most blocks (and partials) of the deterministic reductions
int launch_dot_partial(const double *x, const double *y, int64_t n, double *partials, hipStream_t s);
// w -= h v_prev with h = sum(partials_prev) (also stored to *h_out), then the
// partial dot of the new w with v_next (with w itself when v_next is NULL)
int launch_mgs_step(double *w, const double *v_prev, const double *partials_prev, double *h_out,
                    const double *v_next, int64_t n, double *partials_next, const int *stop, hipStream_t s);
// *out = sqrt(sum of the partials a pass over vectors of length n wrote)
int launch_reduce_final(const double *partials, int64_t n, double *out, hipStream_t s);
int launch_scale_copy(const double *x, const double *alpha_num, const double *alpha_den, double *y, int64_t n,
                      const int *stop, hipStream_t s);  // y = x / (*den), skipped if *den == 0
int launch_copy(const double *x, double *y, int64_t n, hipStream_t s);
// z[i] = x[i] + z[i]
int launch_add(const double *x, double *z, int64_t n, hipStream_t s);
int launch_scatter(const double *x, const int32_t *map, int64_t n, double *z, hipStream_t s);
// Givens step of Hessenberg column j (norm h_{j+1,j} = sqrt of the summed
// partials; skipped when *stop is set) and w = w / h_{j+1,j} (skipped when it
// is 0).  npart: number of norm partials (0: red_blocks(n), a per-pass
// reduction's).
int launch_givens_scale(double *H, int ldh, double *cs, double *sn, double *g, int j, const double *pnorm, int *stop,
                        int *nsteps, double *est, double *hn_out, const double *tol_ref, double rtol, double *w,
                        int64_t n, hipStream_t s, int npart = 0);
// the same with w kept apart (wt): v = wt / ||wt||, and y = C v for the next
// step (C in CSR), in one launch
int launch_givens_scale_spmv(double *H, int ldh, double *cs, double *sn, double *g, int j, const double *pnorm,
                             int *stop, int *nsteps, double *est, double *hn_out, const double *tol_ref, double rtol,
                             const double *wt, double *v, int64_t n, const int64_t *rp, const int32_t *ci,
                             const double *cv, double *y, hipStream_t s, int npart = 0);
// The orthogonalisation of Arnoldi step j in one launch: w (or a + b when a
// is given, stored to w) minus its MGS projections on v_0..v_j (v_i at
// V + i n), h_i to hcol[i], and the partials of <w, w> in pnorm (out->npart
// of them, at most RED_BLOCKS).  slots holds arnoldi_slots(passes) words
// (passes >= j + 1), all reset by launch_arnoldi_reset before the first
// launch; *launches counts the launches since then (advanced here).
// out->done is false (and nothing is launched) when the shape does not fit
// the kernel (odd n, unaligned vectors, n beyond its registers) or the grid
// does not fit on the device: the caller then runs the passes.
struct ArnoldiOut {
  bool done = false;
  double *pnorm = nullptr;
  int npart = 0;
};
int64_t arnoldi_slots(int passes);
int launch_arnoldi_reset(unsigned long long *slots, int passes, hipStream_t s);
int launch_arnoldi(double *w, const double *a, const double *b, const double *V, int64_t n, int j, double *hcol,
                   unsigned long long *slots, int passes, unsigned long long *launches, double *pnorm, int num_cu,
                   void *status, ArnoldiOut *out, hipStream_t s);
// whether launch_arnoldi can take these vectors (the device may still refuse the grid)
bool arnoldi_fits(int64_t n, const void *w, const void *a, const void *b, const void *V, int num_cu);
// w = a + b and the partials of <w, v>
int launch_sum_dot(double *w, const double *a, const double *b, const double *v, int64_t n, double *partials,
                   hipStream_t s);
int launch_backsolve(const double *H, int ldh, const double *g, const int *nsteps, double *c, hipStream_t s);
int launch_combine(double *y, const double *V, int64_t ldv, const double *c, const int *nsteps, int64_t n,
                   bool accumulate, hipStream_t s);
int launch_init_krylov(double *g, const double *beta, int *stop, int *nsteps, hipStream_t s);

}  // namespace silu
