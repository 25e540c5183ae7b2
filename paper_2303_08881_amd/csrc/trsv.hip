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

namespace silu {

// fused multiply-add in the solve's precision (FP64, or FP32 for factors
// stored in FP32 / FP16), and an FP16 value given by its bits
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ float half_bits(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(h & 0xffffu));
}
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

// ---------------------------------------------------------------------------
// Block-local solve.  The subdomains are independent, so each block of rows
// (one subdomain) is solved by one workgroup that walks the block's levels
// with a workgroup barrier between consecutive levels; there is no
// communication between workgroups.  Rows are listed block-major,
// level-minor ("positions"); lev_ptr[b * nlev + l] .. [.. + 1] delimits the
// positions of level l in block b.
//
// Every vector the solve touches is in an order that makes the accesses of a
// level contiguous: the right-hand side is given in position order, and the
// solution of position q goes to out[rec.y], an index fixed at setup (q
// itself, or the position of the row in the solve that consumes it next).
// Storage (built at setup):
//   ent_c/ent_v  the dependency entries of each position, G*E of them (G
//                lanes per row of E = 2, 4 or 8 entries each): column order,
//                each column replaced by the slot of its position in the LDS
//                solution window, padded with the window's zero slot and 0.0.
//                A lane's slots (16 bits each) form one word and its values
//                words of 16 bytes (or of E values), stored in planes, one
//                per load of a lane (lanes consecutive), so that each load
//                of a wave reads one contiguous range: a lane-major layout
//                makes a wave's load touch a cache line per lane, and the
//                bytes every lane loads pass the CU's vector memory path,
//                whose rate bounds the interior solves;
//   rec          {row (or ~row for a slow row), output index, 1 / diagonal}.
// A row is handled by G consecutive lanes, lane g summing entries
// gE..gE+E-1 with fma (lane 0 starting from the right-hand side); the G
// partial sums are combined pairwise across lanes (fixed order, so results
// are reproducible run to run; the sum order differs from the sequential one
// by rounding only) and the sum is multiplied once by the reciprocal of the
// diagonal (within an ulp of the division).
//
// Latency is the whole cost of this solve (a level holds tens to hundreds of
// rows), so every load is issued LOOK levels before its use (LOOK = 10, 8, 6
// for E = 2, 4, 8): each thread keeps LOOK register sets that rotate by
// unrolling the level loop LOOK times.  All pipeline addresses come from the
// level pointers in LDS -- none depends on a load of the same pipeline stage
// -- and every pipeline load is unconditional (idle lanes read a dummy
// position), so the number of memory operations between a load and its use
// is fixed: the compiler's in-order waits before level l then cover only
// level l's own loads.  LOOK times the loads and the store of a level stay
// under the 63 memory operations that the counter tracks.
//
// The solution of the last XWIN positions lives in an LDS ring.  Rows with
// more than G*E entries, with a dependency older than the ring, or beyond
// blockDim/G rows in their level are "slow": they are summed sequentially in
// column order from the natural-order factor, reading each dependency from
// out[omap[column]] (written by this workgroup before an earlier barrier).
// Columns outside the solve (the Z block of the U_B solve) are applied to
// the right-hand side before the solve.
// ---------------------------------------------------------------------------
constexpr int XWIN = 8192;            // solution window (positions), power of two
constexpr int BT_MAX = 512;           // threads per block-local solve
constexpr int BT_WIDE = 1024;         // one-lane rows of at most 4 entries: up to 16 waves (one block whose
                                      // levels are wider than 512 rows, e.g. a single large subdomain)
constexpr int BT_LDS_LEVELS = 16384;  // level pointers kept in LDS
constexpr int LOOK_MAX = 10;

// loads per level: E/4 (columns; one for E = 2) + E/2 (values; one for E = 2)
// + record + right-hand side, and one store: LOOK times that stays within
// the 63 operations the counter tracks
template <int E, int P = 0>
constexpr int look_of() {
  return P == 0 ? (E == 8 ? 6 : E == 4 ? 8 : 10) : (P == 1 && E == 8) ? 8 : 10;
}

struct LdsTrsvArgs {
  const void *ent_c;       // [nent] words of E 16-bit window slots (Cols<E>::W)
  const void *ent_v;       // [E / vpw][nent] words of vpw values (see VWord)
  uint32_t nent;           // lanes of entries: (npos + 1) * G
  const int4 *rec;         // [npos + 1]
  const int32_t *lev_ptr;  // [nblk * nlev + 1]
  int32_t nlev;
  int32_t npos;            // positions; index npos is the dummy read by idle lanes
  int32_t bt;              // blockDim.x, passed as an argument: reading blockDim
                           // is a load from the dispatch packet with a full wait
  const int64_t *rp;       // natural-order factor (slow rows)
  const int32_t *ci;
  const double *v;
  int64_t split;           // dependency columns are < split
  const double *b;         // right-hand side in position order [npos]
  double *out;             // solution of position q at out[rec[q].y]
  const int32_t *omap;     // row -> its index in out (slow rows)
};

// window slots of a lane's entries, 16 bits each (a slot is at most XWIN),
// in one word per lane: uint32 for E = 2, uint2 for E = 4, uint4 for E = 8
template <int E>
struct Cols;
template <>
struct Cols<2> {
  using W = uint32_t;
  W v;
  __device__ __forceinline__ int32_t get(int k) const { return (int32_t)((v >> (16 * k)) & 0xffffu); }
};
template <>
struct Cols<4> {
  using W = uint2;
  W v;
  __device__ __forceinline__ int32_t get(int k) const {
    return (int32_t)(((k >> 1 ? v.y : v.x) >> (16 * (k & 1))) & 0xffffu);
  }
};
template <>
struct Cols<8> {
  using W = uint4;
  W v;
  __device__ __forceinline__ int32_t get(int k) const {
    const uint32_t u = (k >> 1) == 0 ? v.x : (k >> 1) == 1 ? v.y : (k >> 1) == 2 ? v.z : v.w;
    return (int32_t)((u >> (16 * (k & 1))) & 0xffffu);
  }
};

// Storage precision of the factor values (ilu_options_t factor_prec):
// P = 0 FP64; P = 1 FP32; P = 2 FP16 scaled per row (each stored value is the
// entry divided by the largest magnitude of its row, which the record holds).
// P = 1 and 2 solve in FP32: window, products and sums; right-hand side and
// solution vectors stay FP64.
template <int P>
struct Acc {
  using T = float;
};
template <>
struct Acc<0> {
  using T = double;
};


// A lane's E values in NW words of vpw values each (one load per word):
// FP64 double2; FP32 float2 (E = 2) or float4; FP16 one word of E halves.
template <int P, int E>
struct VWord;
template <int E>
struct VWord<0, E> {
  using W = double2;
  static constexpr int NW = E / 2;
  __device__ static __forceinline__ double get(const W *w, int k) { return (k & 1) ? w[k >> 1].y : w[k >> 1].x; }
};
template <>
struct VWord<1, 2> {
  using W = float2;
  static constexpr int NW = 1;
  __device__ static __forceinline__ float get(const W *w, int k) { return k ? w[0].y : w[0].x; }
};
template <int E>
struct VWord<1, E> {
  using W = float4;
  static constexpr int NW = E / 4;
  __device__ static __forceinline__ float get(const W *w, int k) {
    const float4 &q = w[k >> 2];
    return (k & 3) == 0 ? q.x : (k & 3) == 1 ? q.y : (k & 3) == 2 ? q.z : q.w;
  }
};
template <>
struct VWord<2, 2> {
  using W = uint32_t;
  static constexpr int NW = 1;
  __device__ static __forceinline__ float get(const W *w, int k) { return half_bits(w[0] >> (16 * k)); }
};
template <>
struct VWord<2, 4> {
  using W = uint2;
  static constexpr int NW = 1;
  __device__ static __forceinline__ float get(const W *w, int k) {
    return half_bits((k >> 1 ? w[0].y : w[0].x) >> (16 * (k & 1)));
  }
};
template <>
struct VWord<2, 8> {
  using W = uint4;
  static constexpr int NW = 1;
  __device__ static __forceinline__ float get(const W *w, int k) {
    const uint32_t u = (k >> 1) == 0 ? w[0].x : (k >> 1) == 1 ? w[0].y : (k >> 1) == 2 ? w[0].z : w[0].w;
    return half_bits(u >> (16 * (k & 1)));
  }
};

template <int E, int P>
struct PSet {
  Cols<E> c;
  typename VWord<P, E>::W w[VWord<P, E>::NW];
  int4 rec;
  double rhs;
};

// record: {row or ~row, output index, 1 / diagonal (FP64 in z|w; FP32 in z),
// row scale (FP32 in w, FP16 storage)}
template <int P>
__device__ __forceinline__ double rec_diag(const int4 &r) {
  if constexpr (P == 0)
    return __hiloint2double(r.w, r.z);
  else
    return (double)__int_as_float(r.z);
}

// Element idx of an array whose byte size is below 2^32 (checked at setup):
// a 32-bit byte offset from a base held in scalar registers, so a load or
// store needs one 32-bit multiply-add for its address instead of 64-bit
// arithmetic per lane.
template <class T>
__device__ __forceinline__ const T &at32(const T *base, uint32_t idx) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (idx * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ T &at32(T *base, uint32_t idx) {
  return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (idx * (uint32_t)sizeof(T)));
}

// DPP lane exchanges inside groups of 2, 4, 8 lanes (quad permutations, and
// the mirror of 8 lanes, which pairs each lane with one of the other quad)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int G>
__device__ __forceinline__ double group_sum(double s) {
  if (G >= 2) s = s + dpp_f64<0xB1>(s);   // quad_perm [1,0,3,2]
  if (G >= 4) s = s + dpp_f64<0x4E>(s);   // quad_perm [2,3,0,1]
  if (G >= 8) s = s + dpp_f64<0x141>(s);  // row_half_mirror
  return s;
}
template <int G>
__device__ __forceinline__ float group_sum(float s) {
  if (G >= 2) s = s + dpp_f32<0xB1>(s);
  if (G >= 4) s = s + dpp_f32<0x4E>(s);
  if (G >= 8) s = s + dpp_f32<0x141>(s);
  return s;
}

template <bool DIAG>
__device__ __forceinline__ double slow_row(const LdsTrsvArgs &a, int32_t r, int32_t q, double d) {
  double s = a.b[q];
  for (int64_t p = a.rp[r]; p < a.rp[r + 1]; p++) {
    const int32_t c = a.ci[p];
    if (c < a.split) s = fma(-a.v[p], a.out[a.omap[c]], s);
  }
  if (DIAG) s = s * d;  // d: the reciprocal of the diagonal
  // Drain this path's loads here: otherwise the compiler cannot tell, where
  // the slow and fast paths join, that the temporaries of the slow path are
  // no longer in flight, and it would wait for every outstanding load (the
  // fast path's prefetches included) on every level.
  __builtin_amdgcn_s_waitcnt(0);
  return s;
}

// Load the pipeline set of the row handled by this lane in a level whose
// positions are [lo, hi) (idle lanes read the dummy position and the first
// right-hand side).
template <int G, int E, int P>
__device__ __forceinline__ void refill(const LdsTrsvArgs &a, int32_t lo, int32_t hi, int32_t j, int32_t g,
                                       PSet<E, P> &S) {
  const uint32_t q = (uint32_t)(lo + j);
  const bool in = q < (uint32_t)hi;
  const uint32_t qc = in ? q : (uint32_t)a.npos;
  const uint32_t e = qc * G + g;
  S.c.v = at32(reinterpret_cast<const typename Cols<E>::W *>(a.ent_c), e);
  using VW = VWord<P, E>;
#pragma unroll
  for (int i = 0; i < VW::NW; i++) S.w[i] = at32(reinterpret_cast<const typename VW::W *>(a.ent_v), i * a.nent + e);
  S.rec = at32(a.rec, qc);
  S.rhs = at32(a.b, in ? q : 0u);
}

// FAST: the factor has no slow row and every level fits the workgroup (known
// at setup), so the step carries neither check.
template <int G, int E, bool DIAG, int P, bool FAST, int LK = 0>
__device__ __forceinline__ void pstep(const LdsTrsvArgs &a, typename Acc<P>::T *win, const int32_t *lp, int32_t l,
                                      int32_t j, int32_t g, PSet<E, P> &S) {
  using A = typename Acc<P>::T;
  using VW = VWord<P, E>;
  constexpr int LOOK = LK ? LK : look_of<E, P>();
  // every LDS read of the step first, so that a single wait covers them: the
  // bounds of levels l and l + LOOK and the window values
  const int32_t q0 = lp[l], q1 = lp[l + 1];
  const int32_t f0 = lp[l + LOOK], f1 = lp[l + LOOK + 1];
  A xv[E];
#pragma unroll
  for (int k = 0; k < E; k++) xv[k] = win[S.c.get(k)];
  const int32_t q = q0 + j;
  const bool mine = q < q1;
  A s;
  if constexpr (P == 2) {
    // scaled entries: the row sum times the row's scale, subtracted once
    s = A(0);
#pragma unroll
    for (int k = 0; k < E; k++) s = fma_t(VW::get(S.w, k), xv[k], s);
    s = group_sum<G>(s);
    s = fma_t(-__int_as_float(S.rec.w), s, (A)S.rhs);
  } else {
    s = g == 0 ? (A)S.rhs : A(0);
#pragma unroll
    for (int k = 0; k < E; k++) s = fma_t(-(A)VW::get(S.w, k), xv[k], s);
    s = group_sum<G>(s);
  }
  if (DIAG) s = s * (A)rec_diag<P>(S.rec);  // the record holds 1 / d
  // Rows of at most 2 entries: every lane computes its sum (idle lanes on the
  // dummy position's zero entries), so the window reads are issued with the
  // reads of the level bounds instead of after the test of `mine`, which
  // waits for those (for longer rows this placement measured slower).
  if constexpr (E == 2) asm volatile("" : "+v"(s));
  if constexpr (!FAST) {
    const bool slow = S.rec.x < 0;
    const int32_t r = slow ? ~S.rec.x : S.rec.x;
    if (mine && slow) s = (A)slow_row<DIAG>(a, r, q, rec_diag<P>(S.rec));
  }
  if (mine && g == 0) {
    win[q & (XWIN - 1)] = s;
    at32(a.out, (uint32_t)S.rec.y) = (double)s;
  }
  if constexpr (!FAST) {
    // rows beyond bt/G in this level: one thread each, slow path
    const int32_t cap = a.bt / G;
    for (int32_t qq = q0 + cap + (int32_t)threadIdx.x; qq < q1; qq += a.bt) {
      const int4 rc = a.rec[qq];
      const int32_t rr = rc.x < 0 ? ~rc.x : rc.x;
      const A s2 = (A)slow_row<DIAG>(a, rr, qq, rec_diag<P>(rc));
      win[qq & (XWIN - 1)] = s2;
      a.out[(uint32_t)rc.y] = (double)s2;
      __builtin_amdgcn_s_waitcnt(0);
    }
  }
  __syncthreads();  // also for an empty level: the step stays branch-free
  refill<G, E, P>(a, f0, f1, j, g, S);
}

// One subdomain's solve by the calling workgroup (win: XWIN + 1 values of the
// solve's precision, lp: BT_LDS_LEVELS + 2 LOOK_MAX + 2 ints of LDS); returns
// after the last level's barrier.
// LK: pipeline depth (0: look_of)
template <int G, int E, bool DIAG, int P, bool FAST, int LK = 0>
__device__ __forceinline__ void block_solve(const LdsTrsvArgs &a, typename Acc<P>::T *win, int32_t *lp) {
  using A = typename Acc<P>::T;
  constexpr int LOOK = LK ? LK : look_of<E, P>();
  const int64_t base = (int64_t)blockIdx.x * a.nlev;
  const int32_t tid = (int32_t)threadIdx.x;
  const int32_t nlev = a.nlev;
  for (int32_t l = tid; l <= nlev; l += a.bt) lp[l] = a.lev_ptr[base + l];
  for (int32_t k = tid; k <= XWIN; k += a.bt) win[k] = A(0);
  __syncthreads();
  if (tid < 2 * LOOK + 1) lp[nlev + 1 + tid] = lp[nlev];  // empty levels past the end
  __syncthreads();
  const int32_t j = tid / G, g = tid % G;
  PSet<E, P> S[LOOK];
  // prologue in the loop's own load order (pinned by scheduling barriers):
  // the compiler merges the state at loop entry with the state at the back
  // edge, and any load that looked more recent at entry would be waited for
  // on every iteration
#pragma unroll
  for (int k = 0; k < LOOK; k++) {
    refill<G, E, P>(a, lp[k], lp[k + 1], j, g, S[k]);
    __builtin_amdgcn_sched_barrier(0);
  }
  // LOOK levels per iteration, a whole number of iterations (the extra levels
  // are empty): the loop has a single exit, the compiler keeps the steps in
  // order and the register sets keep their names
  for (int32_t l = 0; l < nlev; l += LOOK) {
#pragma unroll
    for (int k = 0; k < LOOK; k++) pstep<G, E, DIAG, P, FAST, LK>(a, win, lp, l + k, j, g, S[k]);
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
// output index of position q is omap[rows[q]].
__global__ void k_lds_fill(const int32_t *rows, const int64_t *rp, const int32_t *ci, const double *v,
                           const double *diag, int64_t n, int64_t split, const int32_t *pos, const int32_t *lev_ptr,
                           int64_t nseg, int G, int E, int prec, const int32_t *omap, uint16_t *oc, void *ov,
                           int4 *rec, int *any_slow) {
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
  for (int64_t p = rp[r]; p < rp[r + 1]; p++)
    if (ci[p] < split) {
      const int32_t pc = pos[ci[p]];
      mind = min(mind, pc);
      if (k < cap) {
        oc[at_c(k)] = (uint16_t)(pc & (XWIN - 1));
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
                    hipStream_t s) {
  k_lds_fill<<<(unsigned)((n + 1 + 255) / 256), 256, 0, s>>>(rows, rp, ci, v, diag, n, split, pos, lev_ptr, nseg, G, E,
                                                              prec, omap, oc, ov, reinterpret_cast<int4 *>(rec),
                                                              any_slow);
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
