// batch.hip -- many independent small systems, each factored with ILU(0) and
// solved with right-preconditioned GMRES(m), all in ONE persistent launch.
//
// The paper's block-Jacobi solve (Section 3.1) treats the subdomain blocks as
// independent; here the blocks are independent systems with their own
// right-hand sides and their own convergence, so each is taken whole by one
// workgroup: no work crosses a CU, and every synchronisation is a workgroup
// barrier (or, for narrow levels, a wavefront barrier).
//
// Per system, in one workgroup:
//  1. ILU(0) numeric factorization (Section 2.3, IKJ form) level by level in
//     the order of the L levels (a row depends on the rows of its L pattern
//     only); one thread per row, the row held in registers; the factor values
//     are written on A's pattern.
//  2. Repack: the strict L and U entries of every row, in the order of the
//     level-sorted positions of each solve, with their right-hand-side slots.
//  3. GMRES(m) with right preconditioning (Arnoldi on A M^-1, only V kept,
//     x += M^-1 V c at the end of a cycle), modified Gram-Schmidt, Givens
//     rotations, convergence on |g_{j+1}| <= rtol ||b|| confirmed by the true
//     residual.
//
// Triangular solves walk the levels of one system with the solution of the
// last XW positions in an LDS ring (dependencies of a row are read from the
// ring by precomputed slot), every row in one thread, entries summed in
// column order with fma and the upper solve ending in one true division:
// the sequential definition's rounding.  Every vector a solve reads is in
// its position order and every index it needs is stored per position: the
// lower solve reads a copy of its right-hand side gathered into L position
// order and writes its solution at the rows' U positions, the upper solve
// reads that and writes the natural order.  So every load of a level
// depends on the level pointers alone (LDS) and is issued LOOK levels ahead
// of its use (LOOK register sets rotating through an unrolled loop): a level
// waits for loads issued LOOK - 1 levels earlier, never for one it has just
// issued.  Levels of at most `merge` rows run on the first wavefront alone,
// with a wavefront barrier instead of a workgroup one.
//
// Reductions are deterministic: every thread sums its strided elements in
// order, the 64 lanes of a wavefront combine by a fixed butterfly and the
// wavefronts in a fixed order.  SpMV, residual and vector updates use the
// sequential definition's per-element operations, so they match the
// oracle bit for bit; only dot products differ from it, by summation order.
//
// Work distribution: systems are taken from a ticket counter in a
// largest-first order (longest processing time first), so the big systems
// start at once and the small ones fill the CUs as others finish.
#include "common.hpp"
#include "launch.hpp"

namespace silu {

namespace {

// BT (template parameter of the kernel): threads per workgroup, 256 or 512
constexpr int XW = BATCH_RING;     // solution ring (positions), power of two; slot XW reads 0
constexpr int MMAX = BATCH_MMAX;   // largest restart length
constexpr int LEVMAX = BATCH_LEVMAX;
constexpr int RMAX = BATCH_RMAX;   // entries per row of A (factorization registers)
// elements per thread and vector loaded at once in an MGS pass (about 72 KB
// (256 threads) or 96 KB (512) of a workgroup in flight, within the registers)
template <int BT>
constexpr int mgs_u() {
  return BT == 512 ? 8 : 12;
}

// levels of loads in flight in a triangular solve (register sets per thread;
// 512 threads leave at most 256 registers a lane)
template <int E, int BT = 256>
constexpr int look_of() {
  return E == 2 ? (BT == 512 ? 7 : 8) : 6;
}
// Empty levels kept past the last one.  run() reads the pointers of levels
// up to nlev + 2 LOOK - 2 (a trip's last refill is LOOK levels past a level
// that may itself be LOOK - 1 past the end), so the pad is 2 LOOK entries.
constexpr int LOOK_PAD = 16;
static_assert(LOOK_PAD >= 2 * look_of<2>() && LOOK_PAD >= 2 * look_of<4>(), "level pointer pad too short");

template <int BT>
struct Shared {
  double ring[XW + 1];
  double H[(MMAX + 1) * (MMAX + 1)];
  double cs[MMAX + 1], sn[MMAX + 1], g[MMAX + 2], c[MMAX + 1];
  double red[BT / WAVE];
  double scal[4];
  int32_t levL[LEVMAX + 1 + LOOK_PAD], levU[LEVMAX + 1 + LOOK_PAD];
  int32_t flag[4];
  int32_t sys;
};

// Wavefront barrier that also orders the wavefront's global stores before its
// later global loads (the factorization's narrow levels read factor rows
// that other lanes of the wavefront just stored).
__device__ __forceinline__ void wave_sync_global() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Sum of v over the workgroup, the same value in every thread.
template <int BT>
__device__ __forceinline__ double wg_sum(Shared<BT> &S, double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  if (lane_id() == 0) S.red[threadIdx.x / WAVE] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < BT / WAVE; w++) t += S.red[w];
  __syncthreads();
  return t;
}

// Row products with a system's CSR rows [0, n) (at most ROW entries each,
// columns in [r0, r0 + n)), U rows per thread at a time: every load of a chunk
// is issued before any of its values is used -- row bounds, then all entries
// (a padding slot re-reads the row's first entry), then the x values they pick
// -- so a chunk costs three trips to memory instead of a dependent chain per
// entry.  Row i is summed from init(i) in column order with fma (entries
// negated when NEG), the sequential definition's rounding; use(i, s) gets the
// sum, rows in the plain strided order.
template <int BT, int ROW, int U, bool NEG, typename Init, typename Use>
__device__ __forceinline__ void csr_rows(int n, const int64_t *rp, const int32_t *ci, const double *av, int64_t r0,
                                         const double *x, Init init, Use use) {
  for (int base = (int)threadIdx.x; base < n; base += U * BT) {
    int64_t lo[U], hi[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int i = base + u * BT;
      lo[u] = i < n ? rp[i] : 0;
      hi[u] = i < n ? rp[i + 1] : 0;
    }
    int32_t c[U][ROW];
    double v[U][ROW];
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int k = 0; k < ROW; k++) {
        const int64_t p = lo[u] + k < hi[u] ? lo[u] + k : lo[u];
        c[u][k] = (int32_t)(ci[p] - r0);
        v[u][k] = av[p];
      }
    double xv[U][ROW];
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int k = 0; k < ROW; k++) xv[u][k] = x[c[u][k]];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int i = base + u * BT;
      if (i < n) {
        double s = init(i);
#pragma unroll
        for (int k = 0; k < ROW; k++)
          if (lo[u] + k < hi[u]) s = __builtin_fma(NEG ? -v[u][k] : v[u][k], xv[u][k], s);
        use(i, s);
      }
    }
  }
}

// Row data of one position of a triangular solve (one register set).
template <int E>
struct RowSet {
  uint32_t slot[E / 2];
  double val[E];
  double diag;
  double rhs;
  int32_t out;
};

// One triangular solve of a system: positions [0, n) in level order, level l
// holding positions lev[l] .. lev[l+1] (lev padded with LOOK_PAD copies of
// n).  UP: upper with diagonal, else unit lower.  rhs is in position order;
// the solution of position q goes to out[outi[q]].
template <int E, bool UP, int BT>
struct Solve {
  const uint32_t *slot;  // [n * E/2] ring slots of the entries, two per word
  const double *val;     // [n * E] entry values (padding: 0 with slot XW)
  const double *diag;    // [n] reciprocal of the diagonal (UP)
  const int32_t *outi;   // [n] index of each position's solution in out
  const int32_t *lev;    // LDS level pointers
  int nlev;
  int n;                 // positions
  const double *rhs;     // [n] right-hand side in position order
  double *out;
  int merge;

  // Loads of level l for this thread: its position if the level has one for
  // it, else position 0 (every system has one), so the loads never branch.
  __device__ __forceinline__ void load(RowSet<E> &s, int l) const {
    const int q = lev[l] + (int)threadIdx.x;
    const int qc = (q < lev[l + 1] && q < n) ? q : 0;
#pragma unroll
    for (int k = 0; k < E / 2; k++) s.slot[k] = slot[(size_t)qc * (E / 2) + k];
#pragma unroll
    for (int k = 0; k < E; k++) s.val[k] = val[(size_t)qc * E + k];
    if (UP) s.diag = diag[qc];
    s.rhs = rhs[qc];
    s.out = outi[qc];
  }
  // Every lane forms its sum (idle lanes on position 0's data, whose ring
  // slots and diagonal are valid), and only the store depends on the lane:
  // with the loads' uses outside any divergent branch, the compiler waits
  // for exactly the register set at hand, not for every load in flight.
  __device__ __forceinline__ void compute(Shared<BT> &S, const RowSet<E> &s, int l, bool &prev_small) const {
    const int p0 = lev[l], w = lev[l + 1] - p0;
    const bool small = w <= merge;
    if (!(small && prev_small)) __syncthreads();
    double acc = s.rhs;
#pragma unroll
    for (int k = 0; k < E; k++) {
      const int sl = (int)((s.slot[k >> 1] >> (16 * (k & 1))) & 0xffffu);
      acc = __builtin_fma(-s.val[k], S.ring[sl], acc);
    }
    if (UP) acc = acc * s.diag;
    if ((int)threadIdx.x < w) {
      S.ring[(p0 + (int)threadIdx.x) & (XW - 1)] = acc;
      out[s.out] = acc;
    }
    if (small) wave_sync();
    prev_small = small;
  }

  // levels wider than the workgroup: plain loop, no prefetch
  __device__ void run_wide(Shared<BT> &S) const {
    for (int l = 0; l < nlev; l++) {
      const int p0 = lev[l], p1 = lev[l + 1];
      __syncthreads();
      for (int q = p0 + (int)threadIdx.x; q < p1; q += BT) {
        double acc = rhs[q];
        for (int k = 0; k < E; k++) {
          const int sl = (int)((slot[(size_t)q * (E / 2) + (k >> 1)] >> (16 * (k & 1))) & 0xffffu);
          acc = __builtin_fma(-val[(size_t)q * E + k], S.ring[sl], acc);
        }
        if (UP) acc = acc * diag[q];
        S.ring[q & (XW - 1)] = acc;
        out[outi[q]] = acc;
      }
    }
    __syncthreads();
  }

  // The pipelined solve runs on the first ST threads: a level wider than
  // BATCH_THREADS rows marks the system wide (run_wide), so more threads would
  // only load the dummy position's data, and every level's loads pass
  // through the CU's vector memory path.  The other threads keep the
  // workgroup barriers in step (the same levels, the same merge test).
  static constexpr int ST = BT < BATCH_THREADS ? BT : BATCH_THREADS;
  __device__ void run(Shared<BT> &S, bool wide) const {
    if (wide) {
      run_wide(S);
      return;
    }
    constexpr int LOOK = look_of<E, BT>();  // the register budget is that of BT threads
    if (ST < BT && (int)threadIdx.x >= ST) {
      bool prev_small = false;
      for (int l = 0; l < nlev; l += LOOK) {
#pragma unroll
        for (int k = 0; k < LOOK; k++) {
          const bool small = lev[l + k + 1] - lev[l + k] <= merge;
          if (!(small && prev_small)) __syncthreads();
          prev_small = small;
        }
      }
      __syncthreads();
      return;
    }
    RowSet<E> R[LOOK];
    bool prev_small = false;
    // prologue in the loop's own load order, pinned by scheduling barriers:
    // the compiler merges the wait state at loop entry with the one at the
    // back edge, and a load that looked more recent at entry would be waited
    // for on every trip
#pragma unroll
    for (int k = 0; k < LOOK; k++) {
      load(R[k], k);
      __builtin_amdgcn_sched_barrier(0);
    }
    // LOOK levels per trip (the levels past the end are empty), so the
    // register sets keep their names and each refill is LOOK levels ahead
    for (int l = 0; l < nlev; l += LOOK) {
#pragma unroll
      for (int k = 0; k < LOOK; k++) {
        compute(S, R[k], l + k, prev_small);
        load(R[k], l + k + LOOK);
      }
    }
    __syncthreads();
  }
};

}  // namespace

struct BatchArgs {
  int32_t nsys;
  const int64_t *sys_row;  // [nsys + 1]
  const int32_t *order;    // [nsys] processing order
  const int32_t *nlevL, *nlevU;
  const int32_t *levL, *levU;  // per system (LEVMAX + 1) relative level pointers
  const uint8_t *wide;         // per system: some level wider than the workgroup
  const int64_t *rp;
  const int32_t *ci;
  const double *av;
  const int64_t *dpos;  // [n] CSR index of each row's diagonal
  double *lu;           // [nnz] factor values on A's pattern
  const int32_t *Lrow, *Urow;  // [n] system-local row of each L (U) position
  const int32_t *Lout;         // [n] system-local U position of each L position's row
  const uint32_t *Lslot, *Uslot;
  const int64_t *Lsrc, *Usrc;  // [n * E] CSR index of each entry, -1 for padding
  double *Lval, *Uval, *Udiag;
  const double *b;
  double *x;
  double *V;                 // [(m + 1) * n]
  double *y, *u, *z, *t;     // [n] work vectors
  double rtol;
  int m, maxit, merge;
  unsigned int *ticket;
  int32_t *iters, *status;
  double *relres;
};

template <int E, int BT>
__global__ void __launch_bounds__(BT) k_batch_solve(BatchArgs a) {
  __shared__ Shared<BT> S;
  const int tid = (int)threadIdx.x;
  for (;;) {
    if (tid == 0) {
      const unsigned int k = atomicAdd(a.ticket, 1u);
      S.sys = k < (unsigned int)a.nsys ? a.order[k] : -1;
    }
    __syncthreads();
    const int sys = S.sys;
    __syncthreads();
    if (sys < 0) return;
    const int64_t r0 = a.sys_row[sys];
    const int n = (int)(a.sys_row[sys + 1] - r0);
    const int nlL = a.nlevL[sys], nlU = a.nlevU[sys];
    const bool wide = a.wide[sys] != 0;
    for (int l = tid; l <= nlL + LOOK_PAD; l += BT)
      S.levL[l] = a.levL[(size_t)sys * (LEVMAX + 1) + (l <= nlL ? l : nlL)];
    for (int l = tid; l <= nlU + LOOK_PAD; l += BT)
      S.levU[l] = a.levU[(size_t)sys * (LEVMAX + 1) + (l <= nlU ? l : nlU)];
    if (tid == 0) S.flag[0] = 0;
    if (tid <= 0) S.ring[XW] = 0.0;
    __syncthreads();

    // ---- 1. ILU(0) numeric factorization, in the order of the L levels ----
    {
      bool prev_small = false;
      for (int l = 0; l < nlL; l++) {
        const int p0 = S.levL[l], w = S.levL[l + 1] - p0;
        const bool small = w <= a.merge;
        if (!(small && prev_small)) __syncthreads();
        for (int i = tid; i < w; i += BT) {
          const int64_t r = r0 + a.Lrow[r0 + p0 + i];
          const int64_t rb = a.rp[r];
          const int len = (int)(a.rp[r + 1] - rb);
          int32_t c[RMAX];
          double wv[RMAX];
#pragma unroll
          for (int e = 0; e < RMAX; e++) {
            c[e] = e < len ? a.ci[rb + e] : -1;
            wv[e] = e < len ? a.av[rb + e] : 0.0;
          }
          const int nL = (int)(a.dpos[r] - rb);
#pragma unroll
          for (int e = 0; e < RMAX; e++) {
            if (e < nL) {
              const int64_t k = c[e];
              const int64_t dk = a.dpos[k];
              const double wk = wv[e] / a.lu[dk];
              wv[e] = wk;
              const int64_t ke = a.rp[k + 1];
              for (int64_t pp = dk + 1; pp < ke; pp++) {
                const int32_t j = a.ci[pp];
                const double ukj = a.lu[pp];
#pragma unroll
                for (int f = 0; f < RMAX; f++)
                  if (f < len && c[f] == j) wv[f] = __builtin_fma(-wk, ukj, wv[f]);
              }
            }
          }
          double d = 0.0;
#pragma unroll
          for (int e = 0; e < RMAX; e++)
            if (e == nL) d = wv[e];
          if (d == 0.0 || !__builtin_isfinite(d)) S.flag[0] = 1;
#pragma unroll
          for (int e = 0; e < RMAX; e++)
            if (e < len) a.lu[rb + e] = wv[e];
        }
        if (small) wave_sync_global();
        prev_small = small;
      }
      __syncthreads();
    }
    if (S.flag[0]) {
      if (tid == 0) {
        a.status[sys] = ILU_ERR_ZERO_PIVOT;
        a.iters[sys] = 0;
        a.relres[sys] = -1.0;
      }
      continue;
    }

    // ---- 2. entries of every position in solve order ----
    for (int q = tid; q < n; q += BT) {
      const size_t g = (size_t)(r0 + q);
#pragma unroll
      for (int e = 0; e < E; e++) {
        const int64_t sl = a.Lsrc[g * E + e], su = a.Usrc[g * E + e];
        a.Lval[g * E + e] = sl >= 0 ? a.lu[sl] : 0.0;
        a.Uval[g * E + e] = su >= 0 ? a.lu[su] : 0.0;
      }
      a.Udiag[g] = 1.0 / a.lu[a.dpos[r0 + a.Urow[g]]];
    }
    __syncthreads();

    const double *b = a.b + r0;
    double *x = a.x + r0, *y = a.y + r0, *u = a.u + r0, *z = a.z + r0, *t = a.t + r0;
    double *V = a.V + (size_t)(a.m + 1) * (size_t)r0;
    const int64_t *rp = a.rp + r0;
    const int32_t *ci = a.ci;
    const double *av = a.av;
    const int32_t *Lrow = a.Lrow + r0;
    // L: rhs y (L order), solution to u at the rows' U positions; U: rhs u, solution to z (natural order)
    const Solve<E, false, BT> SL{a.Lslot + (size_t)r0 * (E / 2), a.Lval + (size_t)r0 * E, nullptr, a.Lout + r0,
                             S.levL, nlL, n, y, u, a.merge};
    const Solve<E, true, BT> SU{a.Uslot + (size_t)r0 * (E / 2), a.Uval + (size_t)r0 * E, a.Udiag + r0, a.Urow + r0,
                            S.levU, nlU, n, u, z, a.merge};
    // z = M^-1 v (v natural order): y = v gathered into L order, u = L^-1 y, z = U^-1 u
    auto precond = [&](const double *v) {
#pragma unroll 8
      for (int q = tid; q < n; q += BT) y[q] = v[Lrow[q]];
      __syncthreads();
      SL.run(S, wide);
      SU.run(S, wide);
    };
    // t = b - A x, returns ||t||
    constexpr int ROW = 2 * E + 1;         // entries per row: the diagonal and at most E on each side
    constexpr int SPMV_U = E == 2 ? 4 : 1;  // rows per thread and chunk of a product (registers)
    auto residual = [&]() {
      double p = 0.0;
      csr_rows<BT, ROW, SPMV_U, true>(
          n, rp, ci, av, r0, x, [&](int i) { return b[i]; },
          [&](int i, double s) {
            t[i] = s;
            p = __builtin_fma(s, s, p);
          });
      return sqrt(wg_sum(S, p));
    };

    double pb = 0.0;
    #pragma unroll 4
    for (int i = tid; i < n; i += BT) pb = __builtin_fma(b[i], b[i], pb);
    const double bnorm = sqrt(wg_sum(S, pb));
    int its = 0, st = 0;
    bool conv = false;
    double rel = 0.0;
    if (bnorm == 0.0) {
      #pragma unroll 4
      for (int i = tid; i < n; i += BT) x[i] = 0.0;
      conv = true;
    } else if (!__builtin_isfinite(bnorm)) {
      st = ILU_ERR_BREAKDOWN;
    } else {
      double beta = residual();
      rel = beta / bnorm;
      if (!__builtin_isfinite(beta)) st = ILU_ERR_BREAKDOWN;
      else if (beta <= a.rtol * bnorm) conv = true;
      const int ldh = a.m + 1;
      while (!st && !conv && its < a.maxit) {
        #pragma unroll 4
        for (int i = tid; i < n; i += BT) V[i] = t[i] / beta;
        if (tid == 0) S.g[0] = beta;
        int jm = 0;
        bool stop = false;
        for (int j = 0; j < a.m && !stop; j++) {
          double *vj = V + (size_t)j * n, *w = V + (size_t)(j + 1) * n;
          __syncthreads();
          precond(vj);
          // w = A z, then the first dot <w, v_0>
          double p = 0.0;
          csr_rows<BT, ROW, SPMV_U, false>(
              n, rp, ci, av, r0, z, [](int) { return 0.0; },
              [&](int i, double s) {
                w[i] = s;
                p = __builtin_fma(s, V[i], p);
              });
          double h = wg_sum(S, p);
          // modified Gram-Schmidt: pass i removes h_{i-1} v_{i-1} and forms <w, v_i>
          // (with w itself in the last pass).  mgs_u elements per thread and
          // vector are loaded before any is used, so a workgroup keeps tens of
          // KB in flight (one workgroup streams a whole system's vectors); the
          // sum runs in the same order as the plain strided loop.
          for (int i = 0; i <= j; i++) {
            if (tid == 0) S.H[i + ldh * j] = h;
            const bool self = i == j;
            const double *vi = V + (size_t)i * n, *vn = self ? w : V + (size_t)(i + 1) * n;
            double q = 0.0;
            int e = tid;
            constexpr int MU = mgs_u<BT>();
            for (; e + (MU - 1) * BT < n; e += MU * BT) {
              double wv[MU], av[MU], cv[MU];
#pragma unroll
              for (int u = 0; u < MU; u++) {
                wv[u] = w[e + u * BT];
                av[u] = vi[e + u * BT];
                cv[u] = self ? 0.0 : vn[e + u * BT];
              }
#pragma unroll
              for (int u = 0; u < MU; u++) {
                const double wn = __builtin_fma(-h, av[u], wv[u]);
                w[e + u * BT] = wn;
                q = __builtin_fma(wn, self ? wn : cv[u], q);
              }
            }
            for (; e < n; e += BT) {
              const double wn = __builtin_fma(-h, vi[e], w[e]);
              w[e] = wn;
              q = __builtin_fma(wn, self ? wn : vn[e], q);
            }
            h = wg_sum(S, q);
          }
          const double hn = sqrt(h);
          if (tid == 0) {
            double *H = S.H;
            H[(j + 1) + ldh * j] = hn;
            for (int i = 0; i < j; i++) {
              const double x0 = H[i + ldh * j], x1 = H[(i + 1) + ldh * j];
              H[i + ldh * j] = __builtin_fma(S.cs[i], x0, S.sn[i] * x1);
              H[(i + 1) + ldh * j] = __builtin_fma(-S.sn[i], x0, S.cs[i] * x1);
            }
            const double ha = H[j + ldh * j], hb = H[(j + 1) + ldh * j];
            const double rr = sqrt(__builtin_fma(ha, ha, hb * hb));
            S.cs[j] = ha / rr;
            S.sn[j] = hb / rr;
            H[j + ldh * j] = rr;
            H[(j + 1) + ldh * j] = 0.0;
            S.g[j + 1] = -S.sn[j] * S.g[j];
            S.g[j] = S.cs[j] * S.g[j];
            // bit 0: exact breakdown (w = 0, nothing to normalise), bit 1: the
            // estimate reached the tolerance or the step limit; 4: non-finite
            int f = 0;
            if (!__builtin_isfinite(hn) || !__builtin_isfinite(S.g[j + 1])) {
              f = 4;
            } else {
              if (hn == 0.0) f = 1;
              if (fabs(S.g[j + 1]) <= a.rtol * bnorm || its + 1 >= a.maxit) f |= 2;
            }
            S.flag[1] = f;
          }
          __syncthreads();
          const int f = S.flag[1];
          its++;
          jm = j + 1;
          if (f == 4) {
            st = ILU_ERR_BREAKDOWN;
            break;
          }
          if (!(f & 1))
            #pragma unroll 4
            for (int i = tid; i < n; i += BT) w[i] = w[i] / hn;
          if (f) stop = true;
        }
        if (st) break;
        // c = R^-1 g, u = V c, x += M^-1 u
        if (tid == 0) {
          for (int i = jm - 1; i >= 0; i--) {
            double s = S.g[i];
            for (int l = i + 1; l < jm; l++) s = __builtin_fma(-S.H[i + ldh * l], S.c[l], s);
            S.c[i] = s / S.H[i + ldh * i];
          }
        }
        __syncthreads();
        #pragma unroll 4
        for (int e = tid; e < n; e += BT) {
          double u = 0.0;
          for (int i = 0; i < jm; i++) u = __builtin_fma(S.c[i], V[(size_t)i * n + e], u);
          t[e] = u;
        }
        __syncthreads();
        precond(t);
        #pragma unroll 4
        for (int e = tid; e < n; e += BT) x[e] = x[e] + z[e];
        __syncthreads();
        beta = residual();
        rel = beta / bnorm;
        if (!__builtin_isfinite(beta)) st = ILU_ERR_BREAKDOWN;
        else if (beta <= a.rtol * bnorm) conv = true;
      }
    }
    if (tid == 0) {
      a.iters[sys] = its;
      a.relres[sys] = rel;
      a.status[sys] = st ? st : (conv ? 0 : ILU_NOT_CONVERGED);
    }
    __syncthreads();
  }
}

__global__ void k_batch_reset(unsigned int *ticket) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ticket = 0u;
}

int launch_batch_solve(const BatchLaunch &L, hipStream_t s) {
  BatchArgs a;
  a.nsys = L.nsys;
  a.sys_row = L.sys_row;
  a.order = L.order;
  a.nlevL = L.nlevL;
  a.nlevU = L.nlevU;
  a.levL = L.levL;
  a.levU = L.levU;
  a.wide = L.wide;
  a.rp = L.rp;
  a.ci = L.ci;
  a.av = L.av;
  a.dpos = L.dpos;
  a.lu = L.lu;
  a.Lrow = L.Lrow;
  a.Urow = L.Urow;
  a.Lout = L.Lout;
  a.Lslot = L.Lslot;
  a.Uslot = L.Uslot;
  a.Lsrc = L.Lsrc;
  a.Usrc = L.Usrc;
  a.Lval = L.Lval;
  a.Uval = L.Uval;
  a.Udiag = L.Udiag;
  a.b = L.b;
  a.x = L.x;
  a.V = L.V;
  a.y = L.y;
  a.u = L.u;
  a.z = L.z;
  a.t = L.t;
  a.rtol = L.rtol;
  a.m = L.m;
  a.maxit = L.maxit;
  a.merge = L.merge;
  a.ticket = L.ticket;
  a.iters = L.iters;
  a.status = L.status;
  a.relres = L.relres;
  if (L.m < 1 || L.m > MMAX || L.grid < 1 || (L.bt != 256 && L.bt != 512)) return ILU_ERR_INVALID_ARG;
  k_batch_reset<<<1, 64, 0, s>>>(L.ticket);
  const unsigned g = (unsigned)L.grid;
  if (L.E == 2) {
    if (L.bt == 512)
      k_batch_solve<2, 512><<<g, 512, 0, s>>>(a);
    else
      k_batch_solve<2, 256><<<g, 256, 0, s>>>(a);
  } else {
    if (L.bt == 512)
      k_batch_solve<4, 512><<<g, 512, 0, s>>>(a);
    else
      k_batch_solve<4, 256><<<g, 256, 0, s>>>(a);
  }
  return check_launch("batch_solve");
}

int batch_resident_groups(int num_cu, int E, int bt) {
  int per = 0;
  hipError_t e;
  if (E == 2)
    e = bt == 512 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_solve<2, 512>, 512, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_solve<2, 256>, 256, 0);
  else
    e = bt == 512 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_solve<4, 512>, 512, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch_solve<4, 256>, 256, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return per * num_cu;
}

// ---- setup: per-position data of the two solves ----
// Level of each row of A's strict lower (upper) pattern inside its system is
// known; the positions are the rows sorted by (system, level, row).  For each
// position: its row (system-local), the CSR index of each strict entry in
// column order (-1 padding), and the ring slot of the position of that
// entry's column; plus the diagonal's CSR index of every row.  A dependency
// older than the ring, a row with more entries than E or RMAX, or a column
// outside the row's system is reported in err (bit 0 ring, 1 entries, 2
// system).
__global__ void k_batch_fill(const int32_t *pos_rows, int64_t n, const int64_t *sys_row, const int32_t *row_sys,
                             const int32_t *inv_pos, const int32_t *lev_of, const int32_t *levrel, int levmax1,
                             const int64_t *rp, const int32_t *ci, bool upper, int E, int32_t *prow, uint32_t *pslot,
                             int64_t *psrc, int64_t *dpos, int32_t *err) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int32_t r = pos_rows[q];
  const int32_t k = row_sys[r];
  const int64_t r0 = sys_row[k];
  prow[q] = (int32_t)(r - r0);
  const int64_t qs = q - r0;                                             // position inside the system
  const int64_t lend = levrel[(int64_t)k * levmax1 + lev_of[r] + 1];    // end of q's level (relative)
  int cnt = 0;
  const int64_t rb = rp[r], re = rp[r + 1];
  if (re - rb > BATCH_RMAX) atomicOr(err, 2);
  for (int e = 0; e < E; e++) psrc[q * E + e] = -1;
  for (int e = 0; e < E / 2; e++) pslot[q * (E / 2) + e] = ((uint32_t)XW << 16) | (uint32_t)XW;
  for (int64_t p = rb; p < re; p++) {
    const int32_t c = ci[p];
    if (c < r0 || c >= sys_row[k + 1]) atomicOr(err, 4);
    if (c == r && !upper) dpos[r] = p;
    if (upper ? c <= r : c >= r) continue;
    if (cnt >= E) {
      atomicOr(err, 2);
      break;
    }
    const int64_t cp = inv_pos[c] - r0;  // position of the dependency in this solve
    if (lend - cp > XW) atomicOr(err, 1);
    psrc[q * E + cnt] = p;
    uint32_t &w = pslot[q * (E / 2) + (cnt >> 1)];
    const uint32_t sl = (uint32_t)(cp & (XW - 1));
    w = (cnt & 1) ? ((w & 0xffffu) | (sl << 16)) : ((w & 0xffff0000u) | sl);
    cnt++;
  }
  (void)qs;
}

int launch_batch_fill(const int32_t *pos_rows, int64_t n, const int64_t *sys_row, const int32_t *row_sys,
                      const int32_t *inv_pos, const int32_t *lev_of, const int32_t *levrel, int levmax1,
                      const int64_t *rp, const int32_t *ci, bool upper, int E, int32_t *prow, uint32_t *pslot,
                      int64_t *psrc, int64_t *dpos, int32_t *err, hipStream_t s) {
  if (n == 0) return 0;
  k_batch_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(pos_rows, n, sys_row, row_sys, inv_pos, lev_of, levrel,
                                                           levmax1, rp, ci, upper, E, prow, pslot, psrc, dpos, err);
  return check_launch("batch_fill");
}

// out[q] = the system-local U position of the row at L position q
__global__ void k_batch_lout(const int32_t *lrows, const int32_t *upos, const int64_t *sys_row,
                             const int32_t *row_sys, int64_t n, int32_t *out) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int32_t r = lrows[q];
  out[q] = (int32_t)(upos[r] - sys_row[row_sys[r]]);
}

int launch_batch_lout(const int32_t *lrows, const int32_t *upos, const int64_t *sys_row, const int32_t *row_sys,
                      int64_t n, int32_t *out, hipStream_t s) {
  if (n == 0) return 0;
  k_batch_lout<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(lrows, upos, sys_row, row_sys, n, out);
  return check_launch("batch_lout");
}

// system of every row (rows of system k are [sys_row[k], sys_row[k+1]))
__global__ void k_row_sys(const int64_t *sys_row, int32_t nsys, int32_t *row_sys) {
  const int32_t k = blockIdx.x;
  if (k >= nsys) return;
  for (int64_t r = sys_row[k] + threadIdx.x; r < sys_row[k + 1]; r += blockDim.x) row_sys[r] = k;
}

// relative level pointers of each system (stride levmax1), from the pointers
// of the (system, level)-sorted positions, and each system's level count
// (the wide flag: some level has more rows than a workgroup has threads)
__global__ void k_batch_levels(const int32_t *blk_lev_ptr, int64_t nlev_all, const int64_t *sys_row, int32_t nsys,
                               int levmax1, int32_t *levrel, int32_t *nlev, uint8_t *wide, bool or_wide) {
  const int32_t k = blockIdx.x;
  if (k >= nsys) return;
  const int64_t r0 = sys_row[k];
  __shared__ int cnt;
  __shared__ int wflag;
  if (threadIdx.x == 0) {
    cnt = 0;
    wflag = 0;
  }
  __syncthreads();
  for (int64_t l = threadIdx.x; l < nlev_all; l += blockDim.x) {
    const int64_t a = blk_lev_ptr[(int64_t)k * nlev_all + l], b = blk_lev_ptr[(int64_t)k * nlev_all + l + 1];
    if (b > a) atomicMax(&cnt, (int)l + 1);
    if (b - a > BATCH_THREADS) wflag = 1;
    if (l < levmax1) levrel[(int64_t)k * levmax1 + l] = (int32_t)(a - r0);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    nlev[k] = cnt;
    if (cnt < levmax1) levrel[(int64_t)k * levmax1 + cnt] = (int32_t)(sys_row[k + 1] - r0);
    wide[k] = (uint8_t)((or_wide ? wide[k] : 0) | wflag);
  }
  __syncthreads();
  for (int64_t l = cnt + 1 + threadIdx.x; l < levmax1; l += blockDim.x)
    levrel[(int64_t)k * levmax1 + l] = (int32_t)(sys_row[k + 1] - r0);
}

int launch_row_sys(const int64_t *sys_row, int32_t nsys, int32_t *row_sys, hipStream_t s) {
  if (nsys == 0) return 0;
  k_row_sys<<<(unsigned)nsys, 256, 0, s>>>(sys_row, nsys, row_sys);
  return check_launch("row_sys");
}

int launch_batch_levels(const int32_t *blk_lev_ptr, int64_t nlev_all, const int64_t *sys_row, int32_t nsys,
                        int levmax1, int32_t *levrel, int32_t *nlev, uint8_t *wide, bool or_wide, hipStream_t s) {
  if (nsys == 0) return 0;
  k_batch_levels<<<(unsigned)nsys, 256, 0, s>>>(blk_lev_ptr, nlev_all, sys_row, nsys, levmax1, levrel, nlev, wide,
                                                or_wide);
  return check_launch("batch_levels");
}

}  // namespace silu
