// trsv.hip -- level-scheduled sparse triangular solves (Section 3.1: rows of
// one level are solved together), one launch per solve, no host round trips.
//
// Lower, unit diagonal:  x_r = b_r - sum_j l_rj x_j
// Upper:                 x_r = (b_r - sum_{j >= split} z_rj x_j - sum_{j < split} u_rj x_j) / d_r
// Each row is one lane and sums its entries sequentially in column order with
// fma (the columns >= split -- the Z block of the two-level solve, Section 3.2
// -- first), then divides once: the same rounding order as the sequential
// definition.
//
// Scheduling: rows are listed level by level; a wave takes, by atomic ticket,
// a chunk of <= 64 rows of one level.  Before computing, the chunk waits until
// the cumulative completion counter of the previous level reaches
// epoch * size(previous level); since every chunk of a level itself waited
// for the level before, this implies all earlier levels are complete.
// Counters are cumulative across calls (epoch = call number), so nothing is
// reset between solves.  Waits are bounded.
#include "common.hpp"
#include "launch.hpp"

namespace silu {
// (k_trsv: cross-workgroup level-scheduled variant; k_trsv_lds: one
// workgroup per subdomain on a level-ordered copy of the factor)

struct TrsvArgs {
  const int32_t *rows;
  const int32_t *chunk_start;
  const int32_t *chunk_level;
  int64_t nchunks;
  const int64_t *level_ptr;
  unsigned long long *level_done;
  unsigned long long epoch;
  unsigned long long *ticket;
  unsigned long long ticket_base;
  const int64_t *rp;
  const int32_t *ci;
  const double *v;
  const double *diag;
  int64_t split_col;
  const double *b;
  const int32_t *b_map;
  double *x;
  double *scatter_out;
  const int32_t *scatter_map;
  Status *st;
};

// ROLE only names the instantiation (0: L_B and W rows, 1: U_B with Z,
// 2: L_S, 3: U_S) so profilers report the four solves separately.
template <int ROLE>
__global__ void __launch_bounds__(WAVE) k_trsv(TrsvArgs a) {
  const int lane = lane_id();
  for (;;) {
    const unsigned long long t = wave_ticket(a.ticket) - a.ticket_base;
    if (t >= (unsigned long long)a.nchunks) return;
    const int32_t c0 = a.chunk_start[t], c1 = a.chunk_start[t + 1];
    const int32_t lev = a.chunk_level[t];
    const int32_t q = c0 + lane;
    const bool valid = q < c1;
    const int32_t r = valid ? a.rows[q] : 0;
    int64_t rb = 0, re = 0;
    double rhs = 0.0;
    if (valid) {
      rb = a.rp[r];
      re = a.rp[r + 1];
      rhs = a.b[a.b_map ? a.b_map[r] : r];
    }
    if (lev > 0) {
      bool ok = true;
      if (lane == 0) {
        const unsigned long long need = a.epoch * (unsigned long long)(a.level_ptr[lev] - a.level_ptr[lev - 1]);
        ok = wait_ctr_ge(&a.level_done[lev - 1], need, a.st, r);
      }
      if (!uniform_i32((int)ok)) return;
      fence_acquire();
    }
    if (valid) {
      double s = rhs;
      if (a.diag) {
        for (int64_t p = rb; p < re; p++) {
          const int32_t c = a.ci[p];
          if (c >= a.split_col) s = fma(-a.v[p], a.x[c], s);
        }
        for (int64_t p = rb; p < re; p++) {
          const int32_t c = a.ci[p];
          if (c < a.split_col) s = fma(-a.v[p], a.x[c], s);
        }
        s = s / a.diag[r];
      } else {
        for (int64_t p = rb; p < re; p++) s = fma(-a.v[p], a.x[a.ci[p]], s);
      }
      a.x[r] = s;
      if (a.scatter_out) a.scatter_out[a.scatter_map[r]] = s;
    }
    __syncthreads();
    if (lane == 0)
      __hip_atomic_fetch_add(&a.level_done[lev], (unsigned long long)(c1 - c0), __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Block-local variant: the subdomains are independent, so each block of rows
// (one subdomain) is solved by one workgroup that walks the block's levels
// with a workgroup barrier between consecutive non-empty levels.  Rows are
// listed block-major, level-minor; lev_ptr[b * nlev + l] .. [.. + 1] delimits
// the rows of level l in block b.  No cross-workgroup communication at all.
// ---------------------------------------------------------------------------
constexpr int BT = 256;          // threads per block-local solve
constexpr int BT_LDS_LEVELS = 16384;

// ---------------------------------------------------------------------------
// Block-local solve on a level-ordered copy of the factor.  Inside block b the
// rows are stored in solve order (level by level) and every dependency column
// is renumbered to its position in that order, so one level's rows and
// entries are contiguous in memory (coalesced streaming).
//
// Software pipeline: each thread owns at most one row of each level.  The
// metadata of its row (one 16-byte record, entry count, diagonal) is loaded
// six levels ahead, the right-hand side and the first PK entries (16-byte
// vector loads; rows are padded to a multiple of 4 entries) four levels
// ahead, into register sets that rotate by unrolling the level loop four
// times (copying a set would wait for its loads).  Every pipeline load is
// unconditional with a valid address, so the number of memory operations
// between a load and its use is fixed and the in-order vmcnt waits that the
// compiler inserts before level l do not wait for later levels' loads (the
// counter tracks at most 63 operations per wave, which sets the depth).
// Rows with more than PK entries, with a dependency older than the LDS window,
// or past the first BT rows of a level, are recomputed on a slow path.  The solution of
// the last XWIN positions is kept in an LDS ring: a dependency at position
// c >= q1 - XWIN (q1 = end of the current level) is read from LDS, older ones
// from the level-ordered global copy x_lo.  Columns outside the solve (the Z
// block of the U_B solve) are not part of the copy: that correction runs
// first as its own pass (k_ext_correct), as in the sequential definition.
// ---------------------------------------------------------------------------
constexpr int XWIN = 8192;

struct LdsTrsvArgs {
  const int4 *meta;        // position -> {row, rhs index, scatter index, first entry}
  const int32_t *nent;     // position -> entry count (entries padded per row to a multiple of 4)
  const int32_t *lev_ptr;  // [nblk * nlev + 1] positions
  int32_t nlev;
  int32_t npos;            // positions (rows) of the whole schedule, >= 1
  const int32_t *ci;       // dependency positions, 16-byte aligned rows
  const double *v;
  const double *diag;      // by position (diagonal roles only)
  const double *b;
  double *x_lo;            // solution by position; BT more slots receive idle lanes' stores
  double *x;               // solution by row
  double *scatter_out;     // scatter roles only
};

// Software pipeline over levels (see the notes above k_trsv_lds).
template <int PK>
struct Row {
  int32_t r, si, n;
  double d, rhs;
  int32_t c[PK];
  double w[PK];
};
struct Meta {
  int4 m;  // r, ri, si, e0
  int32_t n;
  double d;
};

template <bool DIAG>
__device__ __forceinline__ void load_meta(const LdsTrsvArgs &a, const int32_t *lp, int32_t l, Meta &M) {
  const int32_t q = lp[l] + (int32_t)threadIdx.x;
  const bool ok = q < lp[l + 1];
  const int32_t qc = ok ? q : a.npos - 1;
  M.m = a.meta[qc];
  const int32_t n = a.nent[qc];
  M.n = ok ? n : 0;
  if (DIAG) M.d = a.diag[qc];
}

template <int PK, bool DIAG, bool SCAT>
__device__ __forceinline__ void load_row(const LdsTrsvArgs &a, const Meta &M, Row<PK> &R) {
  R.r = M.m.x;
  R.si = M.m.z;
  R.n = M.n;
  R.d = DIAG ? M.d : 1.0;
  R.rhs = a.b[M.m.y];
  const int4 *c4 = reinterpret_cast<const int4 *>(a.ci + M.m.w);
  const double2 *v2 = reinterpret_cast<const double2 *>(a.v + M.m.w);
#pragma unroll
  for (int k = 0; k < PK / 4; k++) {
    const int4 c = c4[k];
    R.c[4 * k] = c.x;
    R.c[4 * k + 1] = c.y;
    R.c[4 * k + 2] = c.z;
    R.c[4 * k + 3] = c.w;
  }
#pragma unroll
  for (int k = 0; k < PK / 2; k++) {
    const double2 w = v2[k];
    R.w[2 * k] = w.x;
    R.w[2 * k + 1] = w.y;
  }
}

template <bool DIAG>
__device__ __forceinline__ double slow_row(const LdsTrsvArgs &a, const double *win, int32_t q, int32_t wlo) {
  const int4 m = a.meta[q];
  double s = a.b[m.y];
  const int32_t n = a.nent[q];
  for (int32_t k = 0; k < n; k++) {
    const int32_t c = a.ci[m.w + k];
    const double xv = c >= wlo ? win[c & (XWIN - 1)] : a.x_lo[c];
    s = fma(-a.v[m.w + k], xv, s);
  }
  if (DIAG) s = s / a.diag[q];
  return s;
}

template <int PK, bool DIAG, bool SCAT>
__device__ __forceinline__ void level_step(const LdsTrsvArgs &a, double *win, const int32_t *lp, int32_t l,
                                           Row<PK> &R, Meta &M) {
  const int32_t q0 = lp[l], q1 = lp[l + 1];
  if (q0 != q1) {  // uniform
    const int32_t wlo = q1 - XWIN;
    const int32_t q = q0 + (int32_t)threadIdx.x;
    const bool mine = q < q1;
    double xv[PK];
    bool slow = R.n > PK;
#pragma unroll
    for (int k = 0; k < PK; k++) {
      xv[k] = win[R.c[k] & (XWIN - 1)];
      slow |= (k < R.n) && R.c[k] < wlo;
    }
    double s = R.rhs;
#pragma unroll
    for (int k = 0; k < PK; k++) {
      const double t = fma(-R.w[k], xv[k], s);
      s = (k < R.n) ? t : s;
    }
    if (DIAG) s = s / R.d;
    if (mine && slow) s = slow_row<DIAG>(a, win, q, wlo);
    if (mine) win[q & (XWIN - 1)] = s;
    a.x_lo[mine ? q : a.npos + (int32_t)threadIdx.x] = s;
    if (mine) {
      a.x[R.r] = s;
      if (SCAT) a.scatter_out[R.si] = s;
    }
    for (int32_t qq = q0 + BT + (int32_t)threadIdx.x; qq < q1; qq += BT) {  // rows past the first BT
      const double s2 = slow_row<DIAG>(a, win, qq, wlo);
      const int4 m = a.meta[qq];
      win[qq & (XWIN - 1)] = s2;
      a.x_lo[qq] = s2;
      a.x[m.x] = s2;
      if (SCAT) a.scatter_out[m.z] = s2;
    }
    __syncthreads();
  }
  load_row<PK, DIAG, SCAT>(a, M, R);  // level l + 4
  load_meta<DIAG>(a, lp, l + 6, M);
}

template <int PK, bool DIAG, bool SCAT>
__global__ void __launch_bounds__(BT) k_trsv_lds(LdsTrsvArgs a) {
  __shared__ double win[XWIN];
  __shared__ int32_t lp[BT_LDS_LEVELS + 8];
  const int64_t base = (int64_t)blockIdx.x * a.nlev;
  const int32_t tid = (int32_t)threadIdx.x;
  const int32_t nlev = a.nlev;
  for (int l = tid; l <= nlev; l += BT) lp[l] = a.lev_ptr[base + l];
  __syncthreads();
  if (tid < 7) lp[nlev + 1 + tid] = lp[nlev];  // empty levels past the end
  __syncthreads();
  Row<PK> R0, R1, R2, R3;
  Meta M0, M1;
  load_meta<DIAG>(a, lp, 0, M0);
  load_row<PK, DIAG, SCAT>(a, M0, R0);
  load_meta<DIAG>(a, lp, 1, M1);
  load_row<PK, DIAG, SCAT>(a, M1, R1);
  load_meta<DIAG>(a, lp, 2, M0);
  load_row<PK, DIAG, SCAT>(a, M0, R2);
  load_meta<DIAG>(a, lp, 3, M1);
  load_row<PK, DIAG, SCAT>(a, M1, R3);
  load_meta<DIAG>(a, lp, 4, M0);
  load_meta<DIAG>(a, lp, 5, M1);
  // eight levels per iteration: the compiler tracks outstanding loads exactly
  // inside straight-line code but drains them at a loop back-edge
  for (int32_t l = 0; l < nlev; l += 8) {
    level_step<PK, DIAG, SCAT>(a, win, lp, l, R0, M0);
    if (l + 1 >= nlev) break;
    level_step<PK, DIAG, SCAT>(a, win, lp, l + 1, R1, M1);
    if (l + 2 >= nlev) break;
    level_step<PK, DIAG, SCAT>(a, win, lp, l + 2, R2, M0);
    if (l + 3 >= nlev) break;
    level_step<PK, DIAG, SCAT>(a, win, lp, l + 3, R3, M1);
    if (l + 4 >= nlev) break;
    level_step<PK, DIAG, SCAT>(a, win, lp, l + 4, R0, M0);
    if (l + 5 >= nlev) break;
    level_step<PK, DIAG, SCAT>(a, win, lp, l + 5, R1, M1);
    if (l + 6 >= nlev) break;
    level_step<PK, DIAG, SCAT>(a, win, lp, l + 6, R2, M0);
    if (l + 7 >= nlev) break;
    level_step<PK, DIAG, SCAT>(a, win, lp, l + 7, R3, M1);
  }
}

int launch_trsv_lds(const TrsvLaunch &t, hipStream_t s) {
  if (t.nblk == 0 || t.nrows == 0) return 0;
  if (t.nlev_blk > BT_LDS_LEVELS) return ILU_ERR_INVALID_ARG;
  LdsTrsvArgs a;
  a.meta = reinterpret_cast<const int4 *>(t.lo_meta);
  a.nent = t.lo_nent;
  a.lev_ptr = t.blk_lev_ptr;
  a.nlev = (int32_t)t.nlev_blk;
  a.npos = (int32_t)t.nrows;
  a.ci = t.lo_ci;
  a.v = t.lo_v;
  a.diag = t.lo_diag;
  a.b = t.b;
  a.x_lo = t.lo_x;
  a.x = t.x;
  a.scatter_out = t.scatter_out;
  const unsigned g = (unsigned)t.nblk;
  // row lengths decide the register copy: 4 entries for short rows, 20 otherwise
  const bool wide = t.lo_maxent > 4;
  switch (t.role) {
    case 0:
      if (wide) k_trsv_lds<20, false, false><<<g, BT, 0, s>>>(a);
      else k_trsv_lds<4, false, false><<<g, BT, 0, s>>>(a);
      break;
    case 1:
      if (wide) k_trsv_lds<20, true, true><<<g, BT, 0, s>>>(a);
      else k_trsv_lds<4, true, true><<<g, BT, 0, s>>>(a);
      break;
    case 2:
      if (wide) k_trsv_lds<20, false, false><<<g, BT, 0, s>>>(a);
      else k_trsv_lds<4, false, false><<<g, BT, 0, s>>>(a);
      break;
    default:
      if (wide) k_trsv_lds<20, true, false><<<g, BT, 0, s>>>(a);
      else k_trsv_lds<4, true, false><<<g, BT, 0, s>>>(a);
      break;
  }
  return check_launch("trsv_lds");
}

// ---- construction of the level-ordered copy ----
__global__ void k_pos_of_row(const int32_t *rows, int64_t n, int32_t *pos) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) pos[rows[q]] = (int32_t)q;
}

// dependency entries (columns < split) of the row at position q, padded to a
// multiple of 4 so every row starts 16-byte aligned
__global__ void k_lo_counts(const int32_t *rows, const int64_t *rp, const int32_t *ci, int64_t n, int64_t split,
                            int64_t *cnt, int32_t *nent) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  int64_t k = 0;
  for (int64_t p = rp[rows[q]]; p < rp[rows[q] + 1]; p++) k += ci[p] < split;
  nent[q] = (int32_t)k;
  cnt[q] = (k + 3) & ~(int64_t)3;
}

// entries of the row at position q in column order, renumbered to positions;
// columns >= split are left out; padding entries are zero
__global__ void k_lo_fill(const int32_t *rows, const int64_t *rp, const int32_t *ci, const double *v,
                          const double *diag, int64_t n, int64_t split, const int32_t *pos, const int64_t *orp,
                          int32_t *oci, double *ov, double *odiag, const int32_t *rhs_map, const int32_t *sct_map,
                          int4 *meta) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int32_t r = rows[q];
  int64_t o = orp[q];
  for (int64_t p = rp[r]; p < rp[r + 1]; p++)
    if (ci[p] < split) {
      oci[o] = pos[ci[p]];
      ov[o++] = v[p];
    }
  for (; o < orp[q + 1]; o++) {
    oci[o] = 0;
    ov[o] = 0.0;
  }
  if (diag) odiag[q] = diag[r];
  meta[q] = make_int4(r, rhs_map ? rhs_map[r] : r, sct_map ? sct_map[r] : 0, (int32_t)orp[q]);
}

__global__ void k_max_i32_simple(const int32_t *p, int64_t n, int32_t *out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) atomicMax(out, p[i]);
}

int launch_level_order_copy(const int32_t *rows, const int64_t *rp, const int32_t *ci, const double *v,
                            const double *diag, int64_t n, int64_t split, int32_t *pos, int64_t *cnt, int32_t *nent,
                            const int64_t *orp, int32_t *oci, double *ov, double *odiag, const int32_t *rhs_map,
                            const int32_t *sct_map, int32_t *meta, int32_t *maxent, int stage, hipStream_t s) {
  if (n == 0) return 0;
  const unsigned g = (unsigned)((n + 255) / 256);
  if (stage == 0) {
    k_pos_of_row<<<g, 256, 0, s>>>(rows, n, pos);
    k_lo_counts<<<g, 256, 0, s>>>(rows, rp, ci, n, split, cnt, nent);
    k_max_i32_simple<<<g, 256, 0, s>>>(nent, n, maxent);
  } else {
    k_lo_fill<<<g, 256, 0, s>>>(rows, rp, ci, v, diag, n, split, pos, orp, oci, ov, odiag, rhs_map, sct_map,
                                reinterpret_cast<int4 *>(meta));
  }
  return check_launch("level_order_copy");
}

// x[i] -= sum_j E_ij y_j over the rows of E (columns in y's numbering),
// sequentially in column order: the f'' = f' - Z y step of the two-level solve
__global__ void k_ext_correct(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, int64_t col_off,
                              const double *y, double *x) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = rp[i], e = rp[i + 1];
  if (b == e) return;
  double s = x[i];
  for (int64_t p = b; p < e; p++) s = fma(-v[p], y[ci[p] - col_off], s);
  x[i] = s;
}

int launch_ext_correct(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, int64_t col_off,
                       const double *y, double *x, hipStream_t s) {
  if (n == 0) return 0;
  k_ext_correct<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, v, n, col_off, y, x);
  return check_launch("ext_correct");
}

int launch_trsv(const TrsvLaunch &t, hipStream_t s) {
  if (t.nchunks == 0) return 0;
  TrsvArgs a;
  a.rows = t.rows;
  a.chunk_start = t.chunk_start;
  a.chunk_level = t.chunk_level;
  a.nchunks = t.nchunks;
  a.level_ptr = t.level_ptr;
  a.level_done = t.level_done;
  a.epoch = t.epoch;
  a.ticket = t.ticket;
  a.ticket_base = t.ticket_base;
  a.rp = t.rp;
  a.ci = t.ci;
  a.v = t.v;
  a.diag = t.diag;
  a.split_col = t.split_col;
  a.b = t.b;
  a.b_map = t.b_map;
  a.x = t.x;
  a.scatter_out = t.scatter_out;
  a.scatter_map = t.scatter_map;
  a.st = (Status *)t.status;
  const int64_t grid = t.nchunks < t.max_waves ? t.nchunks : t.max_waves;
  switch (t.role) {
    case 0: k_trsv<0><<<(unsigned)grid, WAVE, 0, s>>>(a); break;
    case 1: k_trsv<1><<<(unsigned)grid, WAVE, 0, s>>>(a); break;
    case 2: k_trsv<2><<<(unsigned)grid, WAVE, 0, s>>>(a); break;
    default: k_trsv<3><<<(unsigned)grid, WAVE, 0, s>>>(a); break;
  }
  return check_launch("trsv");
}

}  // namespace silu
