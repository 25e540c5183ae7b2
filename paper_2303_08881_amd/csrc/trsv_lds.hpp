// trsv_lds.hpp -- the block-local triangular solve: storage layout, the
// pipelined level step and the walk over one block's levels (Section 3.1:
// rows of one level are solved together), shared by the kernels of
// trsv.hip (one workgroup per block) and trsv_split.hip (a block split
// over several workgroups).
#pragma once
#include <type_traits>

#include "common.hpp"

namespace silu {

// fused multiply-add in the solve's precision (FP64, or FP32 for factors
// stored in FP32 / FP16), and an FP16 value given by its bits
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ float half_bits(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(h & 0xffffu));
}

// ---------------------------------------------------------------------------
// Block-local solve.  The subdomains are independent, so each block of rows
// (one subdomain) is solved by one workgroup that walks the block's levels
// with a workgroup barrier between consecutive levels; there is no
// communication between workgroups (a block split over several workgroups,
// which pass values to each other, is the variant of trsv_split.hip).  Rows are listed block-major,
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
// split solve (trsv_split.hip): imported values kept in an LDS ring after the
// window (slots XWIN + 1 ..), the levels it takes, and the pattern of an
// exchange slot not written yet (a signalling NaN, which no arithmetic yields)
constexpr int IWIN = 2048;
constexpr int XLEVELS = 4096;
constexpr unsigned long long XCHG_UNSET = 0x7ff4000000000000ull;

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

}  // namespace silu
