// trsv.hip -- level-scheduled sparse triangular solves (Section 3.1: rows of
// one level are solved together), one launch per solve, no host round trips.
//
// Lower, unit diagonal:  x_r = b_r - sum_j l_rj x_j
// Upper:                 x_r = (b_r - sum_{j >= split} z_rj x_j - sum_{j < split} u_rj x_j) / d_r
// Each row is one lane and sums its entries sequentially in column order with
// fma (the columns >= split -- the Z block of the two-level solve, Section 3.2
// -- first), then divides once: the same rounding order as the sequential
// definition.  With factors stored in FP32 the same steps run in FP32; with
// FP16 storage (each entry divided by its row's largest magnitude) the scaled
// entries are summed in FP32 and the sum, times the row scale, is subtracted
// from the right-hand side.  Vectors stay FP64.
//
// Scheduling: rows are listed level by level; a wave takes, by atomic ticket,
// a chunk of <= 64 rows of one level.  Before computing, the chunk waits until
// the cumulative completion counter of the previous level reaches
// epoch * size(previous level); since every chunk of a level itself waited
// for the level before, this implies all earlier levels are complete.
// Counters are cumulative across calls (epoch = call number), so nothing is
// reset between solves.  Waits are bounded.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"
#include "trsv_lds.hpp"

namespace silu {

// (k_trsv: cross-workgroup level-scheduled variant; k_trsv_lds: one
// workgroup per subdomain, software-pipelined, further below)

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
  const void *v_lp;       // factor values in FP32 or FP16 (P > 0)
  const float *diag_lp;   // FP32 diagonal (P > 0)
  const float *scale_lp;  // FP16: per-row scale of the stored values
  int64_t f64_row;        // P > 0: rows from here on (the W rows) are solved in FP64
};

// value p of the factor in the solve's arithmetic: FP64, FP32, or the FP16
// value (entry / row scale) as FP32
template <int P>
__device__ __forceinline__ auto trsv_val(const TrsvArgs &a, int64_t p) {
  if constexpr (P == 0)
    return a.v[p];
  else if constexpr (P == 1)
    return static_cast<const float *>(a.v_lp)[p];
  else
    return (float)__builtin_bit_cast(_Float16, static_cast<const uint16_t *>(a.v_lp)[p]);
}

// ROLE only names the instantiation (0: L_B and W rows, 1: U_B with Z,
// 2: L_S, 3: U_S) so profilers report the four solves separately.
template <int ROLE, int P>
__global__ void __launch_bounds__(WAVE) k_trsv(TrsvArgs a) {
  using A = typename std::conditional<P == 0, double, float>::type;
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
      const bool diag = P == 0 ? a.diag != nullptr : a.diag_lp != nullptr;
      // The Z block of an upper solve (columns >= split) is applied first, in
      // FP64 whatever the storage precision: only the triangular factors
      // themselves are stored in lower precision.
      double rz = rhs;
      if (diag)
        for (int64_t p = rb; p < re; p++) {
          const int32_t c = a.ci[p];
          if (c >= a.split_col) rz = fma(-a.v[p], a.x[c], rz);
        }
      A s;
      if (P != 0 && r >= a.f64_row) {
        // rows of W (below the last triangular row of a lower solve) stay
        // FP64 in every storage precision
        double t = rz;
        for (int64_t p = rb; p < re; p++) t = fma(-a.v[p], a.x[a.ci[p]], t);
        s = (A)t;
      } else {
        // FP16 storage: the scaled entries are summed first, then the sum
        // times the row scale is subtracted from the right-hand side
        s = P == 2 ? A(0) : (A)rz;
        const A sg = P == 2 ? A(1) : A(-1);
        for (int64_t p = rb; p < re; p++) {
          const int32_t c = a.ci[p];
          if (!diag || c < a.split_col) s = fma_t(sg * trsv_val<P>(a, p), (A)a.x[c], s);
        }
        if constexpr (P == 2) s = fma_t(-a.scale_lp[r], s, (A)rz);
      }
      if (diag) {
        if constexpr (P == 0)
          s = s / a.diag[r];
        else
          s = s / a.diag_lp[r];
      }
      a.x[r] = (double)s;
      if (a.scatter_out) a.scatter_out[a.scatter_map[r]] = (double)s;
    }
    __syncthreads();
    if (lane == 0)
      __hip_atomic_fetch_add(&a.level_done[lev], (unsigned long long)(c1 - c0), __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int G, int E, bool DIAG, int P, bool FAST>
__global__ void __launch_bounds__(BT_MAX) k_trsv_lds(LdsTrsvArgs a) {
  __shared__ typename Acc<P>::T win[XWIN + 1];  // slot XWIN stays 0: the target of padding entries
  __shared__ int32_t lp[BT_LDS_LEVELS + 2 * LOOK_MAX + 2];
  block_solve<G, E, DIAG, P, FAST>(a, win, lp);
}

// The same solve with up to 1024 threads, for one-lane rows (E <= 4): levels
// of up to 1024 rows stay on the pipelined path instead of the slow one.  Four
// waves per SIMD leave 128 registers per lane, so 4-entry rows keep a 5-level
// (FP64) or 7-level (FP32, FP16) pipeline, without register spills; the 16
// waves of a workgroup hide latency among themselves.
template <int E, int P>
constexpr int look_wide() {
  return E == 4 ? (P == 0 ? 5 : 7) : look_of<E, P>();
}
template <int E, bool DIAG, int P, bool FAST>
__global__ void __launch_bounds__(BT_WIDE) k_trsv_lds_wide(LdsTrsvArgs a) {
  __shared__ typename Acc<P>::T win[XWIN + 1];
  __shared__ int32_t lp[BT_LDS_LEVELS + 2 * LOOK_MAX + 2];
  block_solve<1, E, DIAG, P, FAST, look_wide<E, P>()>(a, win, lp);
}

// L_S then U_S of each subdomain in one launch (both with the same lane
// shape): U_S reads the solution that this workgroup's L_S wrote before the
// barrier between the two.
template <int G, int E, int P, bool FAST>
__global__ void __launch_bounds__(BT_MAX) k_trsv_lds_pair(LdsTrsvArgs lo, LdsTrsvArgs up) {
  __shared__ typename Acc<P>::T win[XWIN + 1];
  __shared__ int32_t lp[BT_LDS_LEVELS + 2 * LOOK_MAX + 2];
  block_solve<G, E, false, P, FAST>(lo, win, lp);
  __syncthreads();
  block_solve<G, E, true, P, FAST>(up, win, lp);
}

template <bool DIAG, int P, bool FAST>
static void launch_ge_p(int G, int E, unsigned grid, unsigned bt, const LdsTrsvArgs &a, hipStream_t s) {
  if (bt > (unsigned)BT_MAX) {  // lds_args admits this for G = 1, E <= 4 only
    if (E == 2)
      k_trsv_lds_wide<2, DIAG, P, FAST><<<grid, bt, 0, s>>>(a);
    else
      k_trsv_lds_wide<4, DIAG, P, FAST><<<grid, bt, 0, s>>>(a);
    return;
  }
  if (E == 2) {
    k_trsv_lds<1, 2, DIAG, P, FAST><<<grid, bt, 0, s>>>(a);
    return;
  }
  if (E == 4) {
    k_trsv_lds<1, 4, DIAG, P, FAST><<<grid, bt, 0, s>>>(a);
    return;
  }
  switch (G) {
    case 1: k_trsv_lds<1, 8, DIAG, P, FAST><<<grid, bt, 0, s>>>(a); break;
    case 2: k_trsv_lds<2, 8, DIAG, P, FAST><<<grid, bt, 0, s>>>(a); break;
    case 4: k_trsv_lds<4, 8, DIAG, P, FAST><<<grid, bt, 0, s>>>(a); break;
    default: k_trsv_lds<8, 8, DIAG, P, FAST><<<grid, bt, 0, s>>>(a); break;
  }
}

template <bool DIAG, bool FAST>
static void launch_ge_f(int G, int E, int prec, unsigned grid, unsigned bt, const LdsTrsvArgs &a, hipStream_t s) {
  if (prec == 1)
    launch_ge_p<DIAG, 1, FAST>(G, E, grid, bt, a, s);
  else if (prec == 2)
    launch_ge_p<DIAG, 2, FAST>(G, E, grid, bt, a, s);
  else
    launch_ge_p<DIAG, 0, FAST>(G, E, grid, bt, a, s);
}
template <bool DIAG>
static void launch_ge(int G, int E, int prec, bool fast, unsigned grid, unsigned bt, const LdsTrsvArgs &a,
                      hipStream_t s) {
  if (fast)
    launch_ge_f<DIAG, true>(G, E, prec, grid, bt, a, s);
  else
    launch_ge_f<DIAG, false>(G, E, prec, grid, bt, a, s);
}

template <int P, bool FAST>
static void launch_pair_pf(int G, int E, unsigned g, unsigned bt, const LdsTrsvArgs &a, const LdsTrsvArgs &b,
                           hipStream_t s) {
  if (E == 2)
    k_trsv_lds_pair<1, 2, P, FAST><<<g, bt, 0, s>>>(a, b);
  else if (E == 4)
    k_trsv_lds_pair<1, 4, P, FAST><<<g, bt, 0, s>>>(a, b);
  else if (G == 1)
    k_trsv_lds_pair<1, 8, P, FAST><<<g, bt, 0, s>>>(a, b);
  else if (G == 2)
    k_trsv_lds_pair<2, 8, P, FAST><<<g, bt, 0, s>>>(a, b);
  else if (G == 4)
    k_trsv_lds_pair<4, 8, P, FAST><<<g, bt, 0, s>>>(a, b);
  else
    k_trsv_lds_pair<8, 8, P, FAST><<<g, bt, 0, s>>>(a, b);
}
template <int P>
static void launch_pair_p(int G, int E, bool fast, unsigned g, unsigned bt, const LdsTrsvArgs &a,
                          const LdsTrsvArgs &b, hipStream_t s) {
  if (fast)
    launch_pair_pf<P, true>(G, E, g, bt, a, b, s);
  else
    launch_pair_pf<P, false>(G, E, g, bt, a, b, s);
}

static bool lds_args(const TrsvLaunch &t, LdsTrsvArgs &a) {
  const bool ge_ok = ((t.lds_e == 2 || t.lds_e == 4) && t.lds_g == 1) ||
                     (t.lds_e == 8 && (t.lds_g == 1 || t.lds_g == 2 || t.lds_g == 4 || t.lds_g == 8));
  const int bt_cap = (t.lds_g == 1 && t.lds_e <= 4) ? BT_WIDE : BT_MAX;
  if (t.nlev_blk > BT_LDS_LEVELS || t.lds_bt < 64 || t.lds_bt > bt_cap || t.lds_bt % 64 != 0 || !ge_ok ||
      !t.b || !t.x || !t.out_map)
    return false;
  a.ent_c = t.lds_c;
  a.ent_v = t.lds_v;
  a.nent = (uint32_t)((t.nrows + 1) * t.lds_g);
  a.rec = reinterpret_cast<const int4 *>(t.lds_rec);
  a.lev_ptr = t.blk_lev_ptr;
  a.nlev = (int32_t)t.nlev_blk;
  a.npos = (int32_t)t.nrows;
  a.rp = t.rp;
  a.ci = t.ci;
  a.v = t.v;
  a.split = t.split_col;
  a.b = t.b;
  a.out = t.x;
  a.omap = t.out_map;
  a.bt = t.lds_bt;
  return true;
}

int launch_trsv_lds(const TrsvLaunch &t, hipStream_t s) {
  if (t.nblk == 0 || t.nrows == 0) return 0;
  LdsTrsvArgs a;
  if (!lds_args(t, a)) return ILU_ERR_INVALID_ARG;
  const unsigned g = (unsigned)t.nblk, bt = (unsigned)t.lds_bt;
  if (t.diag)
    launch_ge<true>(t.lds_g, t.lds_e, t.prec, t.lds_fast != 0, g, bt, a, s);
  else
    launch_ge<false>(t.lds_g, t.lds_e, t.prec, t.lds_fast != 0, g, bt, a, s);
  return check_launch("trsv_lds");
}

bool trsv_lds_pair_ok(const TrsvLaunch &lo, const TrsvLaunch &up) {
  return lo.nblk == up.nblk && lo.nblk > 0 && lo.nrows > 0 && up.nrows > 0 && lo.lds_g == up.lds_g &&
         lo.lds_e == up.lds_e && lo.prec == up.prec && !lo.diag && up.diag && lo.lds_bt <= BT_MAX &&
         up.lds_bt <= BT_MAX;
}

int launch_trsv_lds_pair(const TrsvLaunch &lo, const TrsvLaunch &up, hipStream_t s) {
  LdsTrsvArgs a, b;
  if (!trsv_lds_pair_ok(lo, up) || !lds_args(lo, a) || !lds_args(up, b)) return ILU_ERR_INVALID_ARG;
  // one block size for both solves: each covers its own widest level
  a.bt = b.bt = std::max(a.bt, b.bt);
  const unsigned g = (unsigned)lo.nblk, bt = (unsigned)a.bt;
  const bool fast = lo.lds_fast && up.lds_fast;
  if (lo.prec == 1)
    launch_pair_p<1>(lo.lds_g, lo.lds_e, fast, g, bt, a, b, s);
  else if (lo.prec == 2)
    launch_pair_p<2>(lo.lds_g, lo.lds_e, fast, g, bt, a, b, s);
  else
    launch_pair_p<0>(lo.lds_g, lo.lds_e, fast, g, bt, a, b, s);
  return check_launch("trsv_lds_pair");
}

// ---- construction of the block-local storage ----
__global__ void k_pos_of_row(const int32_t *rows, int64_t n, int32_t *pos) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) pos[rows[q]] = (int32_t)q;
}

// dependency entries (columns < split) of the row at each position; maximum
// (one atomic per wave)
__global__ void k_lds_counts(const int32_t *rows, const int64_t *rp, const int32_t *ci, int64_t n, int64_t split,
                             int32_t *maxent) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int32_t k = 0;
  if (q < n)
    for (int64_t p = rp[rows[q]]; p < rp[rows[q] + 1]; p++) k += ci[p] < split;
  k = wave_max_int(k);
  if (lane_id() == 0) atomicMax(maxent, k);
}

// widest level of any block
__global__ void k_max_width(const int32_t *lev_ptr, int64_t nseg, int32_t *out) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < nseg) atomicMax(out, lev_ptr[k + 1] - lev_ptr[k]);
}

// Fill one position q (q == n: the dummy position).  lev_ptr is searched for
// the end of q's level, which bounds what the LDS window still holds.  The
// output index of position q is omap[rows[q]].  With part (a block split
// over workgroups), a dependency on a row of another part names the LDS
// ring slot of its import: xrow[column * K1 + part of the row - part of the
// column - 1] is the import's index, counted from the first import of the
// row's part, ilp[part * nlev].
__global__ void k_lds_fill(const int32_t *rows, const int64_t *rp, const int32_t *ci, const double *v,
                           const double *diag, int64_t n, int64_t split, const int32_t *pos, const int32_t *lev_ptr,
                           int64_t nseg, int G, int E, int prec, const int32_t *omap, uint16_t *oc, void *ov,
                           int4 *rec, int *any_slow, const int32_t *part, const int32_t *xrow, int32_t K1,
                           const int32_t *ilp, int64_t nlev) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q > n) return;
  const int64_t cap = (int64_t)G * E, nent = (n + 1) * G;
  // entry k of position q belongs to lane e = q G + k / E as its entry kk =
  // k % E.  A lane's E window slots (16 bits each) form one word, lanes
  // consecutive; its values form words of vpw values, and each load of the
  // solve reads one plane of such words for consecutive lanes, so the planes
  // are stored one after the other
  const int vsize = prec == 0 ? 8 : prec == 1 ? 4 : 2;
  const int64_t vpw = E < 16 / vsize ? E : 16 / vsize;
  auto at_c = [&](int64_t k) { return (q * G + k / E) * E + k % E; };
  auto put_v = [&](int64_t k, double x) {
    const int64_t e = q * G + k / E, kk = k % E;
    const int64_t at = ((kk / vpw) * nent + e) * vpw + kk % vpw;
    if (prec == 0)
      static_cast<double *>(ov)[at] = x;
    else if (prec == 1)
      static_cast<float *>(ov)[at] = (float)x;
    else
      static_cast<uint16_t *>(ov)[at] = __builtin_bit_cast(uint16_t, (_Float16)(float)x);
  };
  int64_t k = 0;
  if (q == n) {
    for (; k < cap; k++) {
      oc[at_c(k)] = XWIN;
      put_v(k, 0.0);
    }
    rec[q] = prec == 0 ? make_int4(0, 0, __double2loint(1.0), __double2hiint(1.0))
                       : make_int4(0, 0, __float_as_int(1.0f), __float_as_int(1.0f));
    return;
  }
  const int32_t r = rows[q];
  // FP16 storage: the entries divided by the largest magnitude of the row
  double scale = 1.0;
  if (prec == 2) {
    double m = 0.0;
    for (int64_t p = rp[r]; p < rp[r + 1]; p++)
      if (ci[p] < split) m = fmax(m, fabs(v[p]));
    if (m > 0.0) scale = (double)(float)m;
  }
  int32_t mind = 0x7fffffff;
  const int32_t ibase = part ? ilp[(int64_t)part[r] * nlev] : 0;
  for (int64_t p = rp[r]; p < rp[r + 1]; p++)
    if (ci[p] < split) {
      const int32_t c = ci[p];
      int32_t slot;
      if (part && part[c] != part[r]) {
        slot = XWIN + 1 + ((xrow[(int64_t)c * K1 + (part[r] - part[c] - 1)] - ibase) & (IWIN - 1));
      } else {
        const int32_t pc = pos[c];
        mind = min(mind, pc);
        slot = pc & (XWIN - 1);
      }
      if (k < cap) {
        oc[at_c(k)] = (uint16_t)slot;
        put_v(k, prec == 2 ? v[p] / scale : v[p]);
      }
      k++;
    }
  const bool too_long = k > cap;
  for (; k < cap; k++) {
    oc[at_c(k)] = XWIN;
    put_v(k, 0.0);
  }
  // end of q's level: the first segment boundary above q
  int64_t lo = 0, hi = nseg;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (lev_ptr[mid + 1] <= q)
      lo = mid + 1;
    else
      hi = mid;
  }
  const int32_t lend = lev_ptr[lo + 1];
  const bool slow = too_long || (int64_t)mind < (int64_t)lend - XWIN;
  if (slow) atomicOr(any_slow, 1);
  // the reciprocal of the diagonal: the solve multiplies by it (one multiply on
  // every level's dependent chain instead of a division)
  const double d = diag ? 1.0 / diag[r] : 1.0;
  const int32_t rr = slow ? ~r : r;
  rec[q] = prec == 0 ? make_int4(rr, omap[r], __double2loint(d), __double2hiint(d))
                     : make_int4(rr, omap[r], __float_as_int((float)d), __float_as_int((float)scale));
}

// Factor values of the level-scheduled solve in FP32, or in FP16 divided by
// the row's largest magnitude (the scale, rounded to FP32, is stored per row);
// the diagonal (if any) in FP32.  One thread per row.
__global__ void k_lowp_factor(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, int64_t col_lim,
                              int prec, void *out, float *scale, const double *diag, float *diag_out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  double sc = 1.0;
  if (prec == 2) {
    double m = 0.0;
    for (int64_t p = rp[r]; p < rp[r + 1]; p++)
      if (ci[p] < col_lim) m = fmax(m, fabs(v[p]));
    if (m > 0.0) sc = (double)(float)m;
    scale[r] = (float)sc;
  }
  for (int64_t p = rp[r]; p < rp[r + 1]; p++) {
    if (prec == 1)
      static_cast<float *>(out)[p] = (float)v[p];
    else
      static_cast<uint16_t *>(out)[p] = __builtin_bit_cast(uint16_t, (_Float16)(float)(v[p] / sc));
  }
  if (diag) diag_out[r] = (float)diag[r];
}

int launch_lowp_factor(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, int64_t col_lim, int prec,
                       void *out, float *scale, const double *diag, float *diag_out, hipStream_t s) {
  if (n == 0) return 0;
  k_lowp_factor<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, v, n, col_lim, prec, out, scale, diag, diag_out);
  return check_launch("lowp_factor");
}

int launch_lds_prepare(const int32_t *rows, const int64_t *rp, const int32_t *ci, int64_t n, int64_t split,
                       const int32_t *lev_ptr, int64_t nseg, int32_t *pos, int32_t *maxent, int32_t *maxw,
                       hipStream_t s) {
  if (n == 0) return 0;
  const unsigned g = (unsigned)((n + 255) / 256);
  k_pos_of_row<<<g, 256, 0, s>>>(rows, n, pos);
  k_lds_counts<<<g, 256, 0, s>>>(rows, rp, ci, n, split, maxent);
  k_max_width<<<(unsigned)((nseg + 255) / 256), 256, 0, s>>>(lev_ptr, nseg, maxw);
  return check_launch("lds_prepare");
}

int launch_lds_fill(const int32_t *rows, const int64_t *rp, const int32_t *ci, const double *v, const double *diag,
                    int64_t n, int64_t split, const int32_t *pos, const int32_t *lev_ptr, int64_t nseg, int G, int E,
                    int prec, const int32_t *omap, uint16_t *oc, void *ov, int32_t *rec, int *any_slow,
                    const int32_t *part, const int32_t *xrow, int32_t K1, const int32_t *ilp, int64_t nlev,
                    hipStream_t s) {
  k_lds_fill<<<(unsigned)((n + 1 + 255) / 256), 256, 0, s>>>(rows, rp, ci, v, diag, n, split, pos, lev_ptr, nseg, G, E,
                                                              prec, omap, oc, ov, reinterpret_cast<int4 *>(rec),
                                                              any_slow, part, xrow, K1, ilp, nlev);
  return check_launch("lds_fill");
}

// ---- orders of the block-local solves (setup) ----
// y[q] = x[map[q]] for index vectors
__global__ void k_gather_i32(const int32_t *x, const int32_t *map, int64_t n, int32_t *y) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) y[q] = x[map[q]];
}

int launch_gather_i32(const int32_t *x, const int32_t *map, int64_t n, int32_t *y, hipStream_t s) {
  if (n == 0) return 0;
  k_gather_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, map, n, y);
  return check_launch("gather_i32");
}

// A CSR with its rows reordered (new row q = old row row0 + rows[q]) and each
// column c replaced by cmap[c - col_off]; the entries of a row keep their
// order.  First the row lengths, then (after a scan) the entries.
__global__ void k_csr_perm_len(const int64_t *rp, int64_t row0, const int32_t *rows, int64_t nrows, int64_t *len) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nrows) return;
  const int64_t r = row0 + rows[q];
  len[q] = rp[r + 1] - rp[r];
}
__global__ void k_csr_perm_ent(const int64_t *rp, const int32_t *ci, const double *v, int64_t row0,
                               const int32_t *rows, int64_t nrows, const int32_t *cmap, int64_t col_off,
                               const int64_t *orp, int32_t *oci, double *ov) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nrows) return;
  const int64_t r = row0 + rows[q];
  int64_t o = orp[q];
  for (int64_t p = rp[r]; p < rp[r + 1]; p++, o++) {
    oci[o] = cmap[ci[p] - col_off];
    ov[o] = v[p];
  }
}

int launch_csr_perm_len(const int64_t *rp, int64_t row0, const int32_t *rows, int64_t nrows, int64_t *len,
                        hipStream_t s) {
  if (nrows == 0) return 0;
  k_csr_perm_len<<<(unsigned)((nrows + 255) / 256), 256, 0, s>>>(rp, row0, rows, nrows, len);
  return check_launch("csr_perm_len");
}

int launch_csr_perm_ent(const int64_t *rp, const int32_t *ci, const double *v, int64_t row0, const int32_t *rows,
                        int64_t nrows, const int32_t *cmap, int64_t col_off, const int64_t *orp, int32_t *oci,
                        double *ov, hipStream_t s) {
  if (nrows == 0) return 0;
  k_csr_perm_ent<<<(unsigned)((nrows + 255) / 256), 256, 0, s>>>(rp, ci, v, row0, rows, nrows, cmap, col_off, orp,
                                                                  oci, ov);
  return check_launch("csr_perm_ent");
}

// ---- the passes between the block-local solves ----
// y[q] = x[map[q]]
__global__ void k_gather(const double *x, const int32_t *map, int64_t n, double *y) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q < n) y[q] = x[map[q]];
}

int launch_gather(const double *x, const int32_t *map, int64_t n, double *y, hipStream_t s) {
  if (n == 0) return 0;
  k_gather<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, map, n, y);
  return check_launch("gather");
}

// Rows whose dependencies are all solved, one thread each, summed in column
// order from the right-hand side b[bmap[i]]: the rows of W after the
// block-local L_B solve (g' = g - W f', Section 3.2), with W's rows in the
// order of out and its columns in the order of x.
__global__ void k_rows_lower(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *b,
                             const int32_t *bmap, const double *x, double *out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = b[bmap[i]];
  for (int64_t p = rp[i]; p < rp[i + 1]; p++) s = fma(-v[p], x[ci[p]], s);
  out[i] = s;
}

int launch_rows_lower(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *b,
                      const int32_t *bmap, const double *x, double *out, hipStream_t s) {
  if (n == 0) return 0;
  k_rows_lower<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, v, n, b, bmap, x, out);
  return check_launch("rows_lower");
}

// Right-hand side of the block-local U_B solve, in its position order:
// out[q] = f[fmap[q]] - sum_j Z_qj y_j (Z's rows in that order, its columns
// in y's order), sequentially in column order: the f'' = f' - Z y step of the
// two-level solve (Section 3.2).  f == NULL reads as zero: out = -Z y, the
// interior half of the prolongation P y = (-U_B^-1 Z y; y) of Section 3.3.
__global__ void k_upper_rhs(const int32_t *fmap, int64_t n, const double *f, const int64_t *rp, const int32_t *ci,
                            const double *v, const double *y, double *out) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  double s = f ? f[fmap[q]] : 0.0;
  for (int64_t p = rp[q]; p < rp[q + 1]; p++) s = fma(-v[p], y[ci[p]], s);
  out[q] = s;
}

int launch_upper_rhs(const int32_t *fmap, int64_t n, const double *f, const int64_t *rp, const int32_t *ci,
                     const double *v, const double *y, double *out, hipStream_t s) {
  if (n == 0) return 0;
  k_upper_rhs<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(fmap, n, f, rp, ci, v, y, out);
  return check_launch("upper_rhs");
}

// z[mb[q]] = u[q] (q < nb) and z[ms[q]] = y[q] (q < ns): both halves of the
// preconditioned vector back to the caller's numbering.  With `add`, each
// element is added to add[] at the same index (the multiplicative method's
// z = x + P y, Section 3.3).
__global__ void k_finish(const double *u, const int32_t *mb, int64_t nb, const double *y, const int32_t *ms,
                         int64_t ns, const double *add, double *z) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int32_t t;
  double v;
  if (i < nb) {
    t = mb[i];
    v = u[i];
  } else if (i < nb + ns) {
    t = ms[i - nb];
    v = y[i - nb];
  } else {
    return;
  }
  z[t] = add ? add[t] + v : v;
}

int launch_finish(const double *u, const int32_t *mb, int64_t nb, const double *y, const int32_t *ms, int64_t ns,
                  const double *add, double *z, hipStream_t s) {
  if (nb + ns == 0) return 0;
  k_finish<<<(unsigned)((nb + ns + 255) / 256), 256, 0, s>>>(u, mb, nb, y, ms, ns, add, z);
  return check_launch("finish");
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
  a.v_lp = t.v_lp;
  a.diag_lp = t.prec != 0 && t.diag ? t.diag_lp : nullptr;
  a.scale_lp = t.scale_lp;
  a.f64_row = t.f64_row;
  if (t.prec != 0 && (!t.v_lp || (t.diag && !t.diag_lp) || (t.prec == 2 && !t.scale_lp))) return ILU_ERR_INVALID_ARG;
  const int64_t grid = t.nchunks < t.max_waves ? t.nchunks : t.max_waves;
  const unsigned gr = (unsigned)grid;
#define SILU_TRSV_ROLES(P_)                                 \
  switch (t.role) {                                         \
    case 0: k_trsv<0, P_><<<gr, WAVE, 0, s>>>(a); break;    \
    case 1: k_trsv<1, P_><<<gr, WAVE, 0, s>>>(a); break;    \
    case 2: k_trsv<2, P_><<<gr, WAVE, 0, s>>>(a); break;    \
    default: k_trsv<3, P_><<<gr, WAVE, 0, s>>>(a); break;   \
  }
  if (t.prec == 1) {
    SILU_TRSV_ROLES(1)
  } else if (t.prec == 2) {
    SILU_TRSV_ROLES(2)
  } else {
    SILU_TRSV_ROLES(0)
  }
#undef SILU_TRSV_ROLES
  return check_launch("trsv");
}

}  // namespace silu
