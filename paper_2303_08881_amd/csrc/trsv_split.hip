// trsv_split.hip -- the block-local triangular solve with a block split over
// several workgroups ("parts"), and the setup of the values they exchange.
//
// A triangular solve of one subdomain (Section 3.1: rows of one level are
// solved together, one barrier per level) runs on one CU, and for the
// interior factors of a large subdomain the rate at which that CU's vector
// memory path delivers the factor entries bounds it, not the level chain.
// Splitting the block's rows into K ranges that are contiguous in the
// solve order gives each range its own workgroup and CU.  A row depends only
// on rows earlier in the solve order, so part k needs values of parts before
// it and never of parts after it; the parts' levels overlap (the rows of a
// later part start a few levels after those of an earlier one), so the K
// workgroups walk the levels side by side, each with about 1/K of the rows.
//
// Exchange.  Each value a part needs from another part (an "import") has
// its own slot in a device array (a row that several parts need has a slot
// for each).  The part that solves the row writes the value there with a
// device-scope store; until then the slot holds a
// signalling-NaN pattern, which no arithmetic produces.  Every value is its
// own flag: no fence and no counter.  In the importing part one extra wave
// does nothing else: it loads the imports of a level AHEAD levels (several
// microseconds) before the level runs, which is as long as a device-scope
// load takes to come back, and at the level before, waits on a slot that
// still holds the pattern, writes the value into an LDS ring of IWIN imports
// beside the solution window (entries name the ring by their own window
// slots) and puts the pattern back for the next solve.  So the compute
// waves' pipeline holds no device-scope load: an importing part runs as fast
// as the others once it trails the part it reads from by AHEAD levels.  A
// slot has one writer and one reader per solve.  Solves of one factor must
// therefore not overlap in time (they do not: a handle's solves run in
// stream order).
//
// Waiting.  A part takes its index in start order from a ticket (a 64-bit
// counter that grows by the grid size per solve), and parts are numbered so
// that every import comes from a smaller index.  A part waits only on parts
// that started before it and wait only on earlier ones in turn, so every
// wait ends whatever else runs on the device.  A wait is also bounded: past
// SPIN_LIMIT polls it raises ILU_ERR_TIMEOUT and uses NaN.
//
// The arithmetic of every row is that of the unsplit solve (same entries in
// the same lanes and order, the same lane combination), so the two give
// identical results.
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"
#include "trsv_lds.hpp"

namespace silu {

static_assert(XLEVELS == SPLIT_LEVELS, "split solve level capacity");

struct XchgArgs {
  double *xv;                  // [nimp + 128 nblk] exchange slots, then 128 words per part, two per lane of
                               // its loader wave, that its idle lanes load (the first 64, never written
                               // during a solve) and store (the other 64) instead
  const int2 *xe;              // [nimp + 1] exports by (part, level): {position, slot}; entry nimp is idle
  const int32_t *elp;          // [nblk * nlev + 1] exports by (part, level at which the part solves the row)
  const int32_t *ilp;          // [nblk * nlev + 1] imports by (part, level that first needs them)
  const int2 *lrange;          // [nblk] first level of each part and its number of levels (<= XLEVELS)
  uint32_t nimp;
  uint32_t nblk;
  unsigned long long *ticket;  // start order of the parts (grows by nblk per solve)
  Status *st;
};

// Exchange wave: levels ahead at which it loads an import (a multiple of the
// compute waves' LOOK, at least 12 levels, a few microseconds of the solve).
template <int E, int P>
constexpr int ahead_split() {
  return look_of<E, P>() * ((12 + look_of<E, P>() - 1) / look_of<E, P>());
}
constexpr int AHEAD_MAX = 20;
constexpr int XPAD = 2 * AHEAD_MAX + 4;  // level pointers past the last level

__device__ __forceinline__ bool is_unset(double v) {
  return __double_as_longlong(v) == (long long)XCHG_UNSET;
}

// Poll slot ii until its part has written it (bounded).
__device__ __forceinline__ double wait_import(const XchgArgs &x, uint32_t ii) {
  long it = 0;
  double v;
  do {
    if (++it > SPIN_LIMIT) {
      raise_error(x.st, ILU_ERR_TIMEOUT, ii);
      return __builtin_nan("");
    }
    if ((it & 255) == 0 && ld_relaxed(&x.st->abort)) return __builtin_nan("");
    __builtin_amdgcn_s_sleep(1);
    v = ld_dev(&x.xv[ii]);
  } while (is_unset(v));
  // nothing of this path left in flight where it joins the pipelined one (see
  // slow_row)
  __builtin_amdgcn_s_waitcnt(0);
  return v;
}

// One step l of the loader wave, between the barriers that end steps l - 1
// and l: the imports of level l + 1 (loaded AHEAD levels earlier) into the
// LDS ring, waiting on a slot still unset, each slot reset for the next
// solve; this lane's export entry of step l + 1 (loaded AHEAD steps
// earlier) into the LDS staging ring of the export wave; then the loads of
// the imports of level l + 1 + AHEAD and of the export entries of step
// l + 1 + AHEAD.  Lanes with nothing to move load and store their own words
// of the part's pad instead (never a word shared with other lanes or
// parts; words they load are never stored to, so these device-scope loads
// find clean lines), so a step issues the same three operations every time
// (a store, then two loads) and the wave's waits are for the loads of AHEAD
// steps before.  The reset is a plain store: the next solve is another
// launch, which sees it.
template <int AHEAD, class A>
__device__ __forceinline__ void lstep(const XchgArgs &x, A *win, int2 *xent, const int32_t *ip, const int32_t *ep,
                                      int32_t ibase, int32_t l, uint32_t pad, int32_t lane, int2 &ev, double &iv) {
  const int32_t n0 = ip[l + 1], n1 = ip[l + 2];
  const int32_t m0 = ip[l + 1 + AHEAD], m1 = ip[l + 2 + AHEAD];
  const int32_t f0 = ep[l + 1 + AHEAD], f1 = ep[l + 2 + AHEAD];
  const int32_t ii = n0 + lane;
  const bool real = ii < n1;
  double v = iv;
  if (real && is_unset(v)) v = wait_import(x, (uint32_t)ii);
  if (real) win[XWIN + 1 + ((ii - ibase) & (IWIN - 1))] = (A)v;
  xent[((l + 1) & 1) * WAVE + lane] = ev;
  at32(x.xv, real ? (uint32_t)ii : pad + WAVE) = __longlong_as_double((long long)XCHG_UNSET);
  const uint32_t jj = (uint32_t)(m0 + lane), fe = (uint32_t)(f0 + lane);
  iv = ld_dev(&at32(x.xv, jj < (uint32_t)m1 ? jj : pad));
  ev = at32(x.xe, fe < (uint32_t)f1 ? fe : x.nimp);
}

// One step l of the export wave: the rows of level l - 1 that later parts
// read (ep is shifted by one level: [ep[l], ep[l + 1]) are those of level
// l - 1), from the LDS window (the compute waves wrote them before the last
// barrier) to their slots, with device-scope stores.  The wave loads
// nothing from memory, so it never waits for these stores: a device-scope
// store is acknowledged only once it reaches memory, and the in-order
// counter would make any later load of the same wave wait for it.
template <class A>
__device__ __forceinline__ void estep(const XchgArgs &x, const A *win, const int2 *xent, const int32_t *ep, int32_t l,
                                      int32_t lane) {
  if (ep[l] + lane < ep[l + 1]) {
    const int2 ent = xent[(l & 1) * WAVE + lane];
    st_dev(&at32(x.xv, (uint32_t)ent.y), (double)win[ent.x & (XWIN - 1)]);
  }
}

// a.bt compute threads (the unsplit check-free step), a loader wave and an
// export wave.  LDS: the solution window, its zero slot and the import ring;
// the level, import and (shifted) export pointers of this part, and empty
// levels past its end; the export entries of two steps.  Every wave takes
// the same number of steps (the levels rounded up to a multiple of AHEAD),
// one barrier each.
template <int G, int E, bool DIAG, int P>
__global__ void __launch_bounds__(BT_MAX) k_trsv_lds_x(LdsTrsvArgs a, XchgArgs x) {
  using A = typename Acc<P>::T;
  constexpr int LOOK = look_of<E, P>();
  constexpr int AHEAD = ahead_split<E, P>();
  static_assert(AHEAD % LOOK == 0 && AHEAD <= AHEAD_MAX, "exchange lookahead");
  __shared__ A win[XWIN + 1 + IWIN];
  __shared__ int32_t lp[XLEVELS + XPAD];
  __shared__ int32_t ip[XLEVELS + XPAD];
  __shared__ int32_t ep[XLEVELS + XPAD];
  __shared__ int2 xent[2 * WAVE];
  __shared__ int32_t part;
  const int32_t tid = (int32_t)threadIdx.x, nth = a.bt + 2 * WAVE;
  if (tid == 0) part = (int32_t)(atomicAdd(x.ticket, 1ull) % (unsigned long long)x.nblk);
  __syncthreads();
  // this part's own levels only: its rows lie in levels lo .. lo + nlev - 1
  // (the others are empty for it; what it needs from other parts comes
  // through the exchange, not through their levels)
  const int2 lr = x.lrange[part];
  const int64_t base = (int64_t)part * a.nlev + lr.x;
  const int32_t nlev = lr.y;
  for (int32_t l = tid; l <= nlev; l += nth) {
    lp[l] = a.lev_ptr[base + l];
    ip[l] = x.ilp[base + l];
    ep[l + 1] = x.elp[base + l];
  }
  if (tid == 0) ep[0] = x.elp[base];
  for (int32_t k = tid; k <= XWIN + IWIN; k += nth) win[k] = A(0);
  if (tid < 2 * WAVE) xent[tid] = make_int2(0, 0);
  __syncthreads();
  if (tid >= a.bt && tid < a.bt + WAVE) {
    // the imports of the part's first level, before its first step
    const int32_t ii = ip[0] + (tid - a.bt);
    if (ii < ip[1]) {
      double v = ld_dev(&at32(x.xv, (uint32_t)ii));
      if (is_unset(v)) v = wait_import(x, (uint32_t)ii);
      win[XWIN + 1 + ((ii - ip[0]) & (IWIN - 1))] = (A)v;
      at32(x.xv, (uint32_t)ii) = __longlong_as_double((long long)XCHG_UNSET);
    }
  }
  if (tid < XPAD - 2) {
    lp[nlev + 1 + tid] = lp[nlev];
    ip[nlev + 1 + tid] = ip[nlev];
    ep[nlev + 2 + tid] = ep[nlev + 1];
  }
  __syncthreads();
  const int32_t steps = (nlev + AHEAD - 1) / AHEAD * AHEAD;
  const bool idle = ip[nlev] == ip[0] && ep[nlev + 1] == ep[0];  // neither imports nor exports
  if (tid < a.bt) {
    const int32_t j = tid / G, g = tid % G;
    PSet<E, P> S[LOOK];
#pragma unroll
    for (int k = 0; k < LOOK; k++) {
      refill<G, E, P>(a, lp[k], lp[k + 1], j, g, S[k]);
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int32_t l = 0; l < steps; l += LOOK) {
#pragma unroll
      for (int k = 0; k < LOOK; k++) pstep<G, E, DIAG, P, true, LOOK>(a, win, lp, l + k, j, g, S[k]);
    }
  } else if (idle) {
    for (int32_t l = 0; l < steps; l++) __syncthreads();
  } else if (tid < a.bt + WAVE) {
    const int32_t lane = tid - a.bt, ibase = ip[0];
    const uint32_t pad = x.nimp + (uint32_t)(2 * WAVE * part + lane);  // loads; pad + WAVE: stores
    int2 ev[AHEAD];    // ev[m % AHEAD]: this lane's export entry of step m
    double iv[AHEAD];  // iv[m % AHEAD]: this lane's import of level m
    // the first loads, in the steps' own order of memory operations (a store
    // to the pad, then the two loads): the compiler merges the state at loop
    // entry with the state at the back edge, and counts its waits from the
    // one with fewer operations in flight.  Step 0 exports nothing (level -1).
#pragma unroll
    for (int k = 0; k < AHEAD; k++) {
      const int32_t m = k == 0 ? AHEAD : k;
      at32(x.xv, pad + WAVE) = 0.0;
      const uint32_t jj = (uint32_t)(ip[m] + lane), fe = (uint32_t)(ep[m] + lane);
      iv[k] = ld_dev(&at32(x.xv, jj < (uint32_t)ip[m + 1] ? jj : pad));
      ev[k] = at32(x.xe, fe < (uint32_t)ep[m + 1] ? fe : x.nimp);
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int32_t l = 0; l < steps; l += AHEAD) {
#pragma unroll
      for (int k = 0; k < AHEAD; k++) {
        lstep<AHEAD>(x, win, xent, ip, ep, ibase, l + k, pad, lane, ev[(k + 1) % AHEAD], iv[(k + 1) % AHEAD]);
        __syncthreads();
      }
    }
  } else {
    const int32_t lane = tid - a.bt - WAVE;
    for (int32_t l = 0; l < steps; l++) {
      estep(x, win, xent, ep, l, lane);
      __syncthreads();
    }
    // the exports of the last step's level (its rows were written before the
    // last barrier, its entries staged before it)
    estep(x, win, xent, ep, steps, lane);
  }
}

template <bool DIAG, int P>
static void launch_x_p(int G, int E, unsigned grid, unsigned bt, const LdsTrsvArgs &a, const XchgArgs &x,
                       hipStream_t s) {
  if (E == 2)
    k_trsv_lds_x<1, 2, DIAG, P><<<grid, bt, 0, s>>>(a, x);
  else if (E == 4)
    k_trsv_lds_x<1, 4, DIAG, P><<<grid, bt, 0, s>>>(a, x);
  else if (G == 1)
    k_trsv_lds_x<1, 8, DIAG, P><<<grid, bt, 0, s>>>(a, x);
  else if (G == 2)
    k_trsv_lds_x<2, 8, DIAG, P><<<grid, bt, 0, s>>>(a, x);
  else if (G == 4)
    k_trsv_lds_x<4, 8, DIAG, P><<<grid, bt, 0, s>>>(a, x);
  else
    k_trsv_lds_x<8, 8, DIAG, P><<<grid, bt, 0, s>>>(a, x);
}
template <bool DIAG>
static void launch_x(int G, int E, int prec, unsigned grid, unsigned bt, const LdsTrsvArgs &a, const XchgArgs &x,
                     hipStream_t s) {
  if (prec == 1)
    launch_x_p<DIAG, 1>(G, E, grid, bt, a, x, s);
  else if (prec == 2)
    launch_x_p<DIAG, 2>(G, E, grid, bt, a, x, s);
  else
    launch_x_p<DIAG, 0>(G, E, grid, bt, a, x, s);
}

int launch_trsv_lds_split(const TrsvLaunch &t, hipStream_t s) {
  if (t.nblk == 0 || t.nrows == 0) return 0;
  const bool ge_ok = ((t.lds_e == 2 || t.lds_e == 4) && t.lds_g == 1) ||
                     (t.lds_e == 8 && (t.lds_g == 1 || t.lds_g == 2 || t.lds_g == 4 || t.lds_g == 8));
  if (!t.lds_fast || !ge_ok || t.xlevels > XLEVELS || t.lds_bt < 64 || t.lds_bt > BT_MAX - 2 * WAVE ||
      t.lds_bt % 64 != 0 || !t.b || !t.x || !t.out_map || !t.xv || !t.xe || !t.elp || !t.ilp || !t.lrange ||
      !t.xticket || t.nblk > (int64_t)UINT32_MAX)
    return ILU_ERR_INVALID_ARG;
  LdsTrsvArgs a{};
  a.ent_c = t.lds_c;
  a.ent_v = t.lds_v;
  a.nent = (uint32_t)((t.nrows + 1) * t.lds_g);
  a.rec = reinterpret_cast<const int4 *>(t.lds_rec);
  a.lev_ptr = t.blk_lev_ptr;
  a.nlev = (int32_t)t.nlev_blk;
  a.npos = (int32_t)t.nrows;
  a.bt = t.lds_bt;
  a.rp = t.rp;
  a.ci = t.ci;
  a.v = t.v;
  a.split = t.split_col;
  a.b = t.b;
  a.out = t.x;
  a.omap = t.out_map;
  XchgArgs x{t.xv,
             reinterpret_cast<const int2 *>(t.xe),
             t.elp,
             t.ilp,
             reinterpret_cast<const int2 *>(t.lrange),
             (uint32_t)t.nimp,
             (uint32_t)t.nblk,
             t.xticket,
             static_cast<Status *>(t.status)};
  const unsigned g = (unsigned)t.nblk, bt = (unsigned)t.lds_bt + 2 * WAVE;  // compute, loader and export waves
  if (t.diag)
    launch_x<true>(t.lds_g, t.lds_e, t.prec, g, bt, a, x, s);
  else
    launch_x<false>(t.lds_g, t.lds_e, t.prec, g, bt, a, x, s);
  return check_launch("trsv_lds_split");
}

// ---- setup: the parts and the values they exchange ----

// part of each row: the K ranges of equal length of its block, numbered
// b K + k (forward) or b K + K - 1 - k (backward solve: the later rows are
// solved first)
__global__ void k_split_parts(const int64_t *bs, int32_t nblk, int64_t n, int32_t K, bool backward, int32_t *part) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  int32_t lo = 0, hi = nblk - 1;  // last block start <= r
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (bs[mid] <= r)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t b0 = bs[lo], len = bs[lo + 1] - b0;
  const int32_t k = (int32_t)(((r - b0) * K) / len);
  part[r] = lo * K + (backward ? K - 1 - k : k);
}

int launch_split_parts(const int64_t *bs, int32_t nblk, int64_t n, int32_t K, bool backward, int32_t *part,
                       hipStream_t s) {
  if (n == 0) return 0;
  k_split_parts<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(bs, nblk, n, K, backward, part);
  return check_launch("split_parts");
}

// dependencies of each row on rows of other parts (columns < split)
__global__ void k_cross_count(const int64_t *rp, const int32_t *ci, int64_t n, int64_t split, const int32_t *part,
                              int64_t *cnt) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  int64_t k = 0;
  for (int64_t p = rp[r]; p < rp[r + 1]; p++) {
    const int32_t c = ci[p];
    k += c < split && part[c] != part[r];
  }
  cnt[r] = k;
}

// one record per cross dependency: source row, and (importing part, level
// of the importing row) as part * nlev + level
__global__ void k_cross_emit(const int64_t *rp, const int32_t *ci, int64_t n, int64_t split, const int32_t *part,
                             const int32_t *level, int64_t nlev, const int64_t *off, uint32_t *src, int32_t *key) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  int64_t o = off[r];
  const int32_t kk = (int32_t)((int64_t)part[r] * nlev + level[r]);
  for (int64_t p = rp[r]; p < rp[r + 1]; p++) {
    const int32_t c = ci[p];
    if (c < split && part[c] != part[r]) {
      src[o] = (uint32_t)c;
      key[o] = kk;
      o++;
    }
  }
}

// Records sorted by source row, and by key within a source (so by importing
// part, then level): the first record of each (source, importing part) is an
// import, with the earliest level that needs it.  bad[1]: a source in a part
// that does not come before the importing one.
__global__ void k_cross_heads(const uint32_t *src, const int32_t *key, int64_t m, const int32_t *part, int64_t nlev,
                              int64_t *head, int32_t *bad) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t imp = (int32_t)(key[i] / nlev);
  const bool h = i == 0 || src[i] != src[i - 1] || imp != (int32_t)(key[i - 1] / nlev);
  head[i] = h ? 1 : 0;
  if (h && part[src[i]] >= imp) atomicOr(&bad[1], 1);
}

__global__ void k_cross_compact(const uint32_t *src, const int32_t *key, int64_t m, const int64_t *head,
                                 const int64_t *rank, uint32_t *isrc, uint32_t *ikey) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m || !head[i]) return;
  isrc[rank[i]] = src[i];
  ikey[rank[i]] = (uint32_t)key[i];
}

// Import index of each (source row, importing part): xrow[row * K1 + (part
// - part[row] - 1)], the importing part being one of the K1 = K - 1 later
// parts of the row's subdomain (-1 where that part imports nothing of it).
__global__ void k_cross_slots(const int32_t *isrc, const uint32_t *ikey, int64_t nimp, const int32_t *part,
                              int64_t nlev, int32_t K1, int32_t *xrow) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nimp) return;
  const int32_t r = isrc[i], imp = (int32_t)(ikey[i] / nlev);
  xrow[(int64_t)r * K1 + (imp - part[r] - 1)] = (int32_t)i;
}

// Every import must still be in its part's LDS ring when a row reads it:
// the ring holds the last IWIN imports brought in, and while level l runs
// the imports of levels <= l + 1 may be in (those of level l + 1 go in
// during level l).  Also: no import needed at level 0 (level 0 has no
// dependency at all, so this only guards the layout).
__global__ void k_cross_check(const int64_t *rp, const int32_t *ci, int64_t n, int64_t split, const int32_t *part,
                              const int32_t *level, int64_t nlev, const int32_t *xrow, int32_t K1, const int32_t *ilp,
                              int32_t *bad) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t kb = (int64_t)part[r] * nlev + level[r];
  for (int64_t p = rp[r]; p < rp[r + 1]; p++) {
    const int32_t c = ci[p];
    if (c < split && part[c] != part[r]) {
      const int32_t gi = xrow[(int64_t)c * K1 + (part[r] - part[c] - 1)];
      const int64_t in = level[r] + 1 < nlev ? ilp[kb + 2] : ilp[kb + 1];
      if (gi < 0 || level[r] == 0 || (int64_t)gi < in - IWIN) atomicOr(&bad[2], 1);
    }
  }
}

__global__ void k_cross_width(const int32_t *ilp, int64_t nkeys, int32_t *bad) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < nkeys && ilp[k + 1] - ilp[k] > 64) atomicOr(&bad[3], 1);
}

__global__ void k_fill_unset(double *xv, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) xv[i] = __longlong_as_double((long long)XCHG_UNSET);
}

int launch_cross_count(const int64_t *rp, const int32_t *ci, int64_t n, int64_t split, const int32_t *part,
                       int64_t *cnt, hipStream_t s) {
  if (n == 0) return 0;
  k_cross_count<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, n, split, part, cnt);
  return check_launch("cross_count");
}
int launch_cross_emit(const int64_t *rp, const int32_t *ci, int64_t n, int64_t split, const int32_t *part,
                      const int32_t *level, int64_t nlev, const int64_t *off, uint32_t *src, int32_t *key,
                      hipStream_t s) {
  if (n == 0) return 0;
  k_cross_emit<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, n, split, part, level, nlev, off, src, key);
  return check_launch("cross_emit");
}
int launch_cross_heads(const uint32_t *src, const int32_t *key, int64_t m, const int32_t *part, int64_t nlev,
                       int64_t *head, int32_t *bad, hipStream_t s) {
  if (m == 0) return 0;
  k_cross_heads<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(src, key, m, part, nlev, head, bad);
  return check_launch("cross_heads");
}
int launch_cross_compact(const uint32_t *src, const int32_t *key, int64_t m, const int64_t *head, const int64_t *rank,
                         uint32_t *isrc, uint32_t *ikey, hipStream_t s) {
  if (m == 0) return 0;
  k_cross_compact<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(src, key, m, head, rank, isrc, ikey);
  return check_launch("cross_compact");
}
int launch_cross_slots(const int32_t *isrc, const uint32_t *ikey, int64_t nimp, const int32_t *part, int64_t nlev,
                       int32_t K1, int32_t *xrow, hipStream_t s) {
  if (nimp == 0) return 0;
  k_cross_slots<<<(unsigned)((nimp + 255) / 256), 256, 0, s>>>(isrc, ikey, nimp, part, nlev, K1, xrow);
  return check_launch("cross_slots");
}
int launch_cross_check(const int64_t *rp, const int32_t *ci, int64_t n, int64_t split, const int32_t *part,
                       const int32_t *level, int64_t nlev, const int32_t *xrow, int32_t K1, const int32_t *ilp,
                       int32_t *bad, hipStream_t s) {
  if (n == 0) return 0;
  k_cross_check<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, n, split, part, level, nlev, xrow, K1, ilp, bad);
  return check_launch("cross_check");
}
// lowest and highest level of each part's rows (lmin preset to INT_MAX, lmax
// to -1).  Consecutive rows mostly share a part: a wave whose rows all do
// reduces first and updates the part once (a few parts take every row, and
// one atomic per row on so few words serialises).
__global__ void k_part_levels(const int32_t *part, const int32_t *level, int64_t n, int32_t *lmin, int32_t *lmax) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool in = r < n;
  const int32_t p = in ? part[r] : -1, lv = in ? level[r] : 0;
  const int32_t p0 = __shfl(p, 0, WAVE);
  if (__all(p == p0) && p0 >= 0) {
    const int32_t mx = wave_max_int(lv), mn = -wave_max_int(-lv);
    if (lane_id() == 0) {
      atomicMin(&lmin[p0], mn);
      atomicMax(&lmax[p0], mx);
    }
  } else if (in) {
    atomicMin(&lmin[p], lv);
    atomicMax(&lmax[p], lv);
  }
}

int launch_part_levels(const int32_t *part, const int32_t *level, int64_t n, int32_t *lmin, int32_t *lmax,
                       hipStream_t s) {
  if (n == 0) return 0;
  k_part_levels<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(part, level, n, lmin, lmax);
  return check_launch("part_levels");
}

__global__ void k_export_keys(const int32_t *isrc, int64_t nimp, const int32_t *part, const int32_t *level,
                              int64_t nlev, uint32_t *key, int32_t *val) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nimp) return;
  const int32_t r = isrc[i];
  key[i] = (uint32_t)((int64_t)part[r] * nlev + level[r]);
  val[i] = (int32_t)i;
}

__global__ void k_export_fill(const int32_t *egi, const int32_t *isrc, const int32_t *pos, int64_t nimp, int2 *xe) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < nimp) xe[e] = make_int2(pos[isrc[egi[e]]], egi[e]);
  if (e == nimp) xe[e] = make_int2(0, 0);
}

int launch_export_keys(const int32_t *isrc, int64_t nimp, const int32_t *part, const int32_t *level, int64_t nlev,
                       uint32_t *key, int32_t *val, hipStream_t s) {
  if (nimp == 0) return 0;
  k_export_keys<<<(unsigned)((nimp + 255) / 256), 256, 0, s>>>(isrc, nimp, part, level, nlev, key, val);
  return check_launch("export_keys");
}
int launch_export_fill(const int32_t *egi, const int32_t *isrc, const int32_t *pos, int64_t nimp, int32_t *xe,
                       hipStream_t s) {
  k_export_fill<<<(unsigned)((nimp + 1 + 255) / 256), 256, 0, s>>>(egi, isrc, pos, nimp, reinterpret_cast<int2 *>(xe));
  return check_launch("export_fill");
}

int launch_cross_width(const int32_t *ilp, int64_t nkeys, int32_t *bad, hipStream_t s) {
  if (nkeys == 0) return 0;
  k_cross_width<<<(unsigned)((nkeys + 255) / 256), 256, 0, s>>>(ilp, nkeys, bad);
  return check_launch("cross_width");
}
int launch_fill_unset(double *xv, int64_t n, hipStream_t s) {
  if (n == 0) return 0;
  k_fill_unset<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(xv, n);
  return check_launch("fill_unset");
}

}  // namespace silu
