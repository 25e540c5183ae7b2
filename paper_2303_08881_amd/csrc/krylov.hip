// krylov.hip -- CSR SpMV / residual and the vector kernels of the (flexible)
// GMRES iterations of Section 4.1 and of the reduced-system solve of
// Section 3.2 (eq. (18)-(19)).
//
// * SpMV and residual: one row per lane, entries summed in column order with
//   fma (the sequential definition, so results are reproducible bit for bit).
// * Reductions are deterministic: a grid of red_blocks(n) blocks (a function
//   of the vector length only) writes one partial per block, and every
//   consumer re-reduces the partials in the same fixed order, so all blocks
//   agree on the value without atomics.
// * Modified Gram-Schmidt runs as j+1 fused passes: pass i subtracts
//   h_{i-1} v_{i-1} from w and forms the partial dot with v_i.
// * The Hessenberg column update, Givens rotation and residual estimate run
//   in the first thread of the normalisation kernel; a device stop word lets
//   the reduced-system GMRES run its fixed number of steps with no host
//   synchronisation.
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"

namespace silu {

constexpr int RED_THREADS = 256;

// s (+/-)= sum_p v[p] x[ci[p]] over p in [pb, pe), in column order: the
// entries are taken SPMV_B at a time, their columns and values loaded first,
// then the x values, so a row costs about two memory latencies, not one per
// entry.
constexpr int SPMV_B = 8;

template <bool NEG>
__device__ __forceinline__ double row_dot(const int32_t *__restrict__ ci, const double *__restrict__ v,
                                          const double *__restrict__ x, int64_t pb, int64_t pe, double s) {
  for (int64_t p0 = pb; p0 < pe; p0 += SPMV_B) {
    int32_t c[SPMV_B];
    double a[SPMV_B], xv[SPMV_B];
#pragma unroll
    for (int k = 0; k < SPMV_B; k++)
      if (p0 + k < pe) {
        c[k] = ci[p0 + k];
        a[k] = v[p0 + k];
      }
#pragma unroll
    for (int k = 0; k < SPMV_B; k++)
      if (p0 + k < pe) xv[k] = x[c[k]];
#pragma unroll
    for (int k = 0; k < SPMV_B; k++)
      if (p0 + k < pe) s = fma(NEG ? -a[k] : a[k], xv[k], s);
  }
  return s;
}

// TAG only names the instance (SpmvTag): the same code for A and C_off
template <int TAG>
__global__ void k_spmv(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci, const double *__restrict__ v,
                       int64_t n, const double *__restrict__ x, double *__restrict__ y) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = row_dot<false>(ci, v, x, rp[i], rp[i + 1], 0.0);
}

__global__ void k_residual(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ v, int64_t n, const double *__restrict__ b,
                           const double *__restrict__ x, double *__restrict__ r) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  r[i] = row_dot<true>(ci, v, x, rp[i], rp[i + 1], b[i]);
}

int launch_spmv(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *x, double *y,
                hipStream_t s, SpmvTag tag) {
  if (n == 0) return 0;
  const unsigned g = (unsigned)((n + 255) / 256);
  if (tag == SPMV_A)
    k_spmv<SPMV_A><<<g, 256, 0, s>>>(rp, ci, v, n, x, y);
  else if (tag == SPMV_COFF)
    k_spmv<SPMV_COFF><<<g, 256, 0, s>>>(rp, ci, v, n, x, y);
  else
    k_spmv<SPMV_USER><<<g, 256, 0, s>>>(rp, ci, v, n, x, y);
  return check_launch("spmv");
}

int launch_residual(const int64_t *rp, const int32_t *ci, const double *v, int64_t n, const double *b,
                    const double *x, double *r, hipStream_t s) {
  if (n == 0) return 0;
  k_residual<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, v, n, b, x, r);
  return check_launch("residual");
}

// ---- deterministic reductions -------------------------------------------
__device__ double block_sum(double v) {
  __shared__ double ws[RED_THREADS / WAVE];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  if (lane_id() == 0) ws[threadIdx.x / WAVE] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < RED_THREADS / WAVE; w++) t += ws[w];
  __syncthreads();
  return t;  // valid in thread 0
}

// every caller gets the same value: lane l sums partials l, l+64, ... in
// order, then a fixed butterfly
__device__ double reduce_partials(const double *p, int nb) {
  const int lane = lane_id();
  double s = 0.0;
  for (int k = lane; k < nb; k += WAVE) s += p[k];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
  return s;
}

// Vector passes take 16-byte loads (two elements) when every operand allows
// it (VEC: n even, pointers 16-byte aligned); each thread still accumulates
// its elements in a fixed order, so the partials are the same on every run.
constexpr int VB = 8;  // element pairs per thread loaded before use (see the vector passes below)

// Blocks (and partials) of the reductions over vectors of length n: enough
// for VB element pairs per thread, at most RED_BLOCKS.  A function of n only,
// so every pass of one Krylov process agrees on it.
static int red_blocks(int64_t n) {
  const int64_t per = 2LL * VB * RED_THREADS;
  return (int)std::max<int64_t>(1, std::min<int64_t>(RED_BLOCKS, (n + per - 1) / per));
}

static bool vec2_ok(int64_t n, const void *a, const void *b, const void *c) {
  auto al = [](const void *p) { return p == nullptr || ((uintptr_t)p & 15) == 0; };
  return (n & 1) == 0 && al(a) && al(b) && al(c);
}

// The vector passes below load a batch of up to VB elements per thread (pairs
// with VEC) before using any of them: the stores of a pass may alias its
// loads in the compiler's eyes, so a plain loop would wait for one memory
// latency per element.  Each thread still takes its elements in the order
// i0, i0 + stride, ..., so the partials are the same as an element-by-element
// loop's.

template <bool VEC>
struct Lane2 {
  double x, y;
};

template <bool VEC>
__device__ __forceinline__ Lane2<VEC> ld2(const double *__restrict__ p, int64_t i) {
  if constexpr (VEC) {
    const double2 t = reinterpret_cast<const double2 *>(p)[i];
    return {t.x, t.y};
  } else {
    return {p[i], 0.0};
  }
}
template <bool VEC>
__device__ __forceinline__ void st2(double *__restrict__ p, int64_t i, const Lane2<VEC> &v) {
  if constexpr (VEC)
    reinterpret_cast<double2 *>(p)[i] = make_double2(v.x, v.y);
  else
    p[i] = v.x;
}
// s += a . b over one element (pair): x then y
template <bool VEC>
__device__ __forceinline__ double dot2(const Lane2<VEC> &a, const Lane2<VEC> &b, double s) {
  s = fma(a.x, b.x, s);
  if constexpr (VEC) s = fma(a.y, b.y, s);
  return s;
}

template <bool VEC>
__global__ void __launch_bounds__(RED_THREADS) k_dot_partial(const double *__restrict__ x,
                                                            const double *__restrict__ y, int64_t n,
                                                            double *__restrict__ partials) {
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  const int64_t i0 = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x;
  const int64_t m = VEC ? n / 2 : n;
  for (int64_t base = i0; base < m; base += VB * stride) {
    Lane2<VEC> a[VB], b[VB];
#pragma unroll
    for (int k = 0; k < VB; k++)
      if (base + k * stride < m) {
        a[k] = ld2<VEC>(x, base + k * stride);
        b[k] = ld2<VEC>(y, base + k * stride);
      }
#pragma unroll
    for (int k = 0; k < VB; k++)
      if (base + k * stride < m) s = dot2<VEC>(a[k], b[k], s);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

int launch_dot_partial(const double *x, const double *y, int64_t n, double *partials, hipStream_t s) {
  if (vec2_ok(n, x, y, nullptr))
    k_dot_partial<true><<<red_blocks(n), RED_THREADS, 0, s>>>(x, y, n, partials);
  else
    k_dot_partial<false><<<red_blocks(n), RED_THREADS, 0, s>>>(x, y, n, partials);
  return check_launch("dot_partial");
}

// w = a + b and the partials of <w, v> in one pass, each thread summing its
// elements in the order k_dot_partial uses
template <bool VEC>
__global__ void __launch_bounds__(RED_THREADS) k_sum_dot(double *__restrict__ w, const double *__restrict__ a,
                                                        const double *__restrict__ b, const double *__restrict__ v,
                                                        int64_t n, double *__restrict__ partials) {
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  const int64_t i0 = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x;
  const int64_t m = VEC ? n / 2 : n;
  for (int64_t base = i0; base < m; base += VB * stride) {
    Lane2<VEC> x[VB], y[VB], u[VB];
#pragma unroll
    for (int k = 0; k < VB; k++)
      if (base + k * stride < m) {
        x[k] = ld2<VEC>(a, base + k * stride);
        y[k] = ld2<VEC>(b, base + k * stride);
        u[k] = ld2<VEC>(v, base + k * stride);
      }
#pragma unroll
    for (int k = 0; k < VB; k++)
      if (base + k * stride < m) {
        Lane2<VEC> t;
        t.x = x[k].x + y[k].x;
        t.y = x[k].y + y[k].y;
        st2<VEC>(w, base + k * stride, t);
        s = dot2<VEC>(t, u[k], s);
      }
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

int launch_sum_dot(double *w, const double *a, const double *b, const double *v, int64_t n, double *partials,
                   hipStream_t s) {
  const bool vec = vec2_ok(n, w, a, b) && vec2_ok(n, v, nullptr, nullptr);
  if (vec)
    k_sum_dot<true><<<red_blocks(n), RED_THREADS, 0, s>>>(w, a, b, v, n, partials);
  else
    k_sum_dot<false><<<red_blocks(n), RED_THREADS, 0, s>>>(w, a, b, v, n, partials);
  return check_launch("sum_dot");
}

// One MGS pass: w -= h v_prev with h the sum of the previous pass's partials,
// then the partials of <w, v_next> (of <w, w> without v_next).  The first
// batch of w, v_prev and v_next is loaded before h is reduced, so the loads
// overlap the reduction.
template <bool VEC, bool NEXT>
__global__ void __launch_bounds__(RED_THREADS) k_mgs_step(double *__restrict__ w, const double *__restrict__ v_prev,
                                                         const double *__restrict__ pp, double *__restrict__ h_out,
                                                         const double *__restrict__ v_next, int64_t n,
                                                         double *__restrict__ pn) {
  __shared__ double sh;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  const int64_t i0 = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x;
  const int64_t m = VEC ? n / 2 : n;
  double s = 0.0, h = 0.0;
  for (int64_t base = i0, batch = 0;; base += VB * stride, batch++) {
    Lane2<VEC> wv[VB], pv[VB], nv[VB];
#pragma unroll
    for (int k = 0; k < VB; k++)
      if (base + k * stride < m) {
        wv[k] = ld2<VEC>(w, base + k * stride);
        pv[k] = ld2<VEC>(v_prev, base + k * stride);
        if (NEXT) nv[k] = ld2<VEC>(v_next, base + k * stride);
      }
    if (batch == 0) {  // every thread of the block takes this branch once
      if (threadIdx.x < WAVE) {
        const double hh = reduce_partials(pp, (int)gridDim.x);
        if (threadIdx.x == 0) {
          sh = hh;
          if (blockIdx.x == 0) *h_out = hh;
        }
      }
      __syncthreads();
      h = sh;
    }
#pragma unroll
    for (int k = 0; k < VB; k++)
      if (base + k * stride < m) {
        Lane2<VEC> t;
        t.x = fma(-h, pv[k].x, wv[k].x);
        t.y = fma(-h, pv[k].y, wv[k].y);
        st2<VEC>(w, base + k * stride, t);
        s = dot2<VEC>(t, NEXT ? nv[k] : t, s);
      }
    if (base + VB * stride >= m) break;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) pn[blockIdx.x] = s;
}

int launch_mgs_step(double *w, const double *v_prev, const double *partials_prev, double *h_out,
                    const double *v_next, int64_t n, double *partials_next, const int *stop, hipStream_t s) {
  (void)stop;
  const bool vec = vec2_ok(n, w, v_prev, v_next);
  if (vec && v_next)
    k_mgs_step<true, true><<<red_blocks(n), RED_THREADS, 0, s>>>(w, v_prev, partials_prev, h_out, v_next, n,
                                                              partials_next);
  else if (vec)
    k_mgs_step<true, false><<<red_blocks(n), RED_THREADS, 0, s>>>(w, v_prev, partials_prev, h_out, v_next, n,
                                                               partials_next);
  else if (v_next)
    k_mgs_step<false, true><<<red_blocks(n), RED_THREADS, 0, s>>>(w, v_prev, partials_prev, h_out, v_next, n,
                                                               partials_next);
  else
    k_mgs_step<false, false><<<red_blocks(n), RED_THREADS, 0, s>>>(w, v_prev, partials_prev, h_out, v_next, n,
                                                                partials_next);
  return check_launch("mgs_step");
}

__global__ void k_reduce_final(const double *partials, int nb, double *out, bool take_sqrt) {
  double s = reduce_partials(partials, nb);
  if (threadIdx.x == 0) *out = take_sqrt ? sqrt(s) : s;
}

int launch_reduce_final(const double *partials, int64_t n, double *out, hipStream_t s) {
  k_reduce_final<<<1, WAVE, 0, s>>>(partials, red_blocks(n), out, true);
  return check_launch("reduce_final");
}

// y = x / (*den)  (skipped when *den == 0)
__global__ void k_scale_div(const double *x, const double *den, double *y, int64_t n) {
  const double d = *den;
  if (d == 0.0) return;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] / d;
}

int launch_scale_copy(const double *x, const double *alpha_num, const double *alpha_den, double *y, int64_t n,
                      const int *stop, hipStream_t s) {
  (void)alpha_num;
  (void)stop;
  if (n == 0) return 0;
  k_scale_div<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, alpha_den, y, n);
  return check_launch("scale_div");
}

__global__ void k_copy(const double *x, double *y, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}
int launch_copy(const double *x, double *y, int64_t n, hipStream_t s) {
  if (n == 0) return 0;
  k_copy<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, y, n);
  return check_launch("copy");
}

__global__ void k_add(const double *x, double *z, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) z[i] = x[i] + z[i];
}
int launch_add(const double *x, double *z, int64_t n, hipStream_t s) {
  if (n == 0) return 0;
  k_add<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, z, n);
  return check_launch("add");
}

__global__ void k_scatter(const double *x, const int32_t *map, int64_t n, double *z) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) z[map[i]] = x[i];
}
int launch_scatter(const double *x, const int32_t *map, int64_t n, double *z, hipStream_t s) {
  if (n == 0) return 0;
  k_scatter<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, map, n, z);
  return check_launch("scatter");
}

// ---- Arnoldi bookkeeping -------------------------------------------------
// stop codes: 1 = exact breakdown (h_{j+1,j} = 0), 2 = estimate below tolerance,
// 3 = non-finite value.
// The Givens step of column j and the normalisation w = w / h_{j+1,j} in one
// launch: every block
// reduces the norm partials itself (the same value in each), block 0 updates
// the Hessenberg column, and all blocks scale their slice (skipped when the
// norm is zero, as in k_scale_div).  The rotation uses r = sqrt(fma(a, a, b*b)).  Only the Givens part looks at the stop
// word: a stopped process leaves H and g alone, and whatever w then holds is
// never used.
template <bool VEC>
__global__ void __launch_bounds__(RED_THREADS) k_givens_scale(double *H, int ldh, double *cs, double *sn, double *g,
                                                             int j, const double *pnorm, int *stop, int *nsteps,
                                                             double *est, double *hn_out, const double *tol_ref,
                                                             double rtol, double *w, int64_t n, int npart) {
  __shared__ double sh;
  if (threadIdx.x < WAVE) {
    const double hn2 = reduce_partials(pnorm, npart);
    if (threadIdx.x == 0) sh = sqrt(hn2);
  }
  __syncthreads();
  const double hn = sh;
  if (blockIdx.x == 0 && threadIdx.x == 0 && !*stop) {
    *hn_out = hn;
    double *col = H + (int64_t)ldh * j;
    col[j + 1] = hn;
    for (int i = 0; i < j; i++) {
      const double a = col[i], b = col[i + 1];
      col[i] = fma(cs[i], a, sn[i] * b);
      col[i + 1] = fma(-sn[i], a, cs[i] * b);
    }
    const double a = col[j], b = col[j + 1];
    const double r = sqrt(fma(a, a, b * b));
    cs[j] = a / r;
    sn[j] = b / r;
    col[j] = r;
    col[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    *nsteps = j + 1;
    const double e = fabs(g[j + 1]);
    *est = e;
    if (!isfinite(hn) || !isfinite(e))
      *stop = 3;
    else if (hn == 0.0)
      *stop = 1;
    else if (e <= rtol * (*tol_ref))
      *stop = 2;
  }
  if (hn == 0.0) return;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  const int64_t i0 = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x;
  const int64_t m = VEC ? n / 2 : n;
  for (int64_t base = i0; base < m; base += VB * stride) {
    Lane2<VEC> t[VB];
#pragma unroll
    for (int k = 0; k < VB; k++)
      if (base + k * stride < m) t[k] = ld2<VEC>(w, base + k * stride);
#pragma unroll
    for (int k = 0; k < VB; k++)
      if (base + k * stride < m) {
        t[k].x = t[k].x / hn;
        t[k].y = t[k].y / hn;
        st2<VEC>(w, base + k * stride, t[k]);
      }
  }
}

int launch_givens_scale(double *H, int ldh, double *cs, double *sn, double *g, int j, const double *pnorm, int *stop,
                        int *nsteps, double *est, double *hn_out, const double *tol_ref, double rtol, double *w,
                        int64_t n, hipStream_t s, int npart) {
  const int np = npart > 0 ? npart : red_blocks(n);
  if (vec2_ok(n, w, nullptr, nullptr))
    k_givens_scale<true><<<red_blocks(n), RED_THREADS, 0, s>>>(H, ldh, cs, sn, g, j, pnorm, stop, nsteps, est, hn_out,
                                                           tol_ref, rtol, w, n, np);
  else
    k_givens_scale<false><<<red_blocks(n), RED_THREADS, 0, s>>>(H, ldh, cs, sn, g, j, pnorm, stop, nsteps, est, hn_out,
                                                            tol_ref, rtol, w, n, np);
  return check_launch("givens_scale");
}

// k_givens_scale for a w kept apart from the basis (wt), fused with the next
// Arnoldi step's sparse product: every block writes its slice of
// v = wt / ||wt|| and computes y = C v for its rows, reading each needed
// element as wt[c] / ||wt|| -- the same division as the stored value, so y is
// bit for bit the product with the stored v.  wt is only read, so the blocks
// need no ordering.  A zero norm leaves v = wt (as k_givens_scale leaves w).
template <bool VEC>
__global__ void __launch_bounds__(RED_THREADS)
    k_givens_scale_spmv(double *H, int ldh, double *cs, double *sn, double *g, int j, const double *pnorm, int *stop,
                        int *nsteps, double *est, double *hn_out, const double *tol_ref, double rtol,
                        const double *__restrict__ wt, double *__restrict__ v, int64_t n,
                        const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                        const double *__restrict__ cv, double *__restrict__ y, int npart) {
  __shared__ double sh;
  if (threadIdx.x < WAVE) {
    const double hn2 = reduce_partials(pnorm, npart);
    if (threadIdx.x == 0) sh = sqrt(hn2);
  }
  __syncthreads();
  const double hn = sh;
  if (blockIdx.x == 0 && threadIdx.x == 0 && !*stop) {
    *hn_out = hn;
    double *col = H + (int64_t)ldh * j;
    col[j + 1] = hn;
    for (int i = 0; i < j; i++) {
      const double a = col[i], b = col[i + 1];
      col[i] = fma(cs[i], a, sn[i] * b);
      col[i + 1] = fma(-sn[i], a, cs[i] * b);
    }
    const double a = col[j], b = col[j + 1];
    const double r = sqrt(fma(a, a, b * b));
    cs[j] = a / r;
    sn[j] = b / r;
    col[j] = r;
    col[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    *nsteps = j + 1;
    const double e = fabs(g[j + 1]);
    *est = e;
    if (!isfinite(hn) || !isfinite(e))
      *stop = 3;
    else if (hn == 0.0)
      *stop = 1;
    else if (e <= rtol * (*tol_ref))
      *stop = 2;
  }
  const bool scale = hn != 0.0;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  const int64_t i0 = blockIdx.x * (int64_t)RED_THREADS + threadIdx.x;
  const int64_t m = VEC ? n / 2 : n;
  for (int64_t base = i0; base < m; base += VB * stride) {
    Lane2<VEC> t[VB];
#pragma unroll
    for (int k = 0; k < VB; k++)
      if (base + k * stride < m) t[k] = ld2<VEC>(wt, base + k * stride);
#pragma unroll
    for (int k = 0; k < VB; k++)
      if (base + k * stride < m) {
        if (scale) {
          t[k].x = t[k].x / hn;
          t[k].y = t[k].y / hn;
        }
        st2<VEC>(v, base + k * stride, t[k]);
      }
  }
  // one row per thread (the grid covers the rows), entries in column order
  for (int64_t i = i0; i < n; i += stride) {
    double acc = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
      const double x = scale ? wt[ci[p]] / hn : wt[ci[p]];
      acc = fma(cv[p], x, acc);
    }
    y[i] = acc;
  }
}

int launch_givens_scale_spmv(double *H, int ldh, double *cs, double *sn, double *g, int j, const double *pnorm,
                             int *stop, int *nsteps, double *est, double *hn_out, const double *tol_ref, double rtol,
                             const double *wt, double *v, int64_t n, const int64_t *rp, const int32_t *ci,
                             const double *cv, double *y, hipStream_t s, int npart) {
  // a grid of one thread per row for the product; npart norm partials
  // (red_blocks(n) when 0: those of a per-pass reduction)
  const int np = npart > 0 ? npart : red_blocks(n);
  const unsigned grid = (unsigned)std::max<int64_t>(np, (n + RED_THREADS - 1) / RED_THREADS);
  if (vec2_ok(n, wt, v, nullptr))
    k_givens_scale_spmv<true><<<grid, RED_THREADS, 0, s>>>(H, ldh, cs, sn, g, j, pnorm, stop, nsteps, est, hn_out,
                                                           tol_ref, rtol, wt, v, n, rp, ci, cv, y, np);
  else
    k_givens_scale_spmv<false><<<grid, RED_THREADS, 0, s>>>(H, ldh, cs, sn, g, j, pnorm, stop, nsteps, est, hn_out,
                                                            tol_ref, rtol, wt, v, n, rp, ci, cv, y, np);
  return check_launch("givens_scale_spmv");
}

// ---- one Arnoldi orthogonalisation per launch -----------------------------
// The modified Gram-Schmidt of step j as one launch instead of a dot launch
// and j + 1 pass launches.  Each workgroup keeps its slice of w in registers
// for the whole step: w is read and written once, each v_i is streamed once
// (v_{i+1} is loaded while the blocks wait for the sum of pass i).  Pass i:
// h_i = <w, v_i>, w -= h_i v_i, as in the one-launch-per-pass route; the
// partials of <w, w> are left for the Givens kernel.
//
// The grid-wide sums need no counter: block b writes its partial of pass i to
// its own slot, and a slot holding a signalling-NaN pattern (which no
// arithmetic produces) has not been written yet, so the value is its own
// ready flag and one round of device-scope loads both waits for and gathers
// the partials.  A dedicated ninth wave does this (its loads never queue
// behind the data waves' prefetches).  Above 64 blocks the sum has two
// levels: the first block of each group of 16 sums its group's slots into a
// group slot, and every block gathers the group slots.  All sums run in one
// fixed order, so every block gets the same h_i and every run the same bits;
// the result equals the per-pass route's up to the grouping of these sums.
// Slots are never reused within a launch (one row of slots per pass); two
// sets alternate between launches, and each launch resets the other set for
// the next one (the kernel boundary orders the resets before its loads).
// Every wait is bounded (SPIN_LIMIT polls, then ILU_ERR_TIMEOUT in the status
// word and no further waiting).  The launch is an ordinary one (a cooperative
// launch costs about 20 us, this kernel a few us a pass) whose grid fits on
// the device at once (one workgroup per CU at most, checked against the
// occupancy): on an otherwise idle device every block runs from the start,
// and a block held back by other work is waited for.
constexpr int ARN_T = 512;             // data threads per workgroup
constexpr int ARN_TT = ARN_T + WAVE;   // plus the wave that gathers the sums
constexpr int ARN_KMAX = 8;            // element pairs per thread and vector (16 would spill registers)
constexpr int ARN_GROUP = 16;          // blocks per first-level group above ARN_FLAT blocks
constexpr int ARN_FLAT = WAVE;
constexpr unsigned long long ARN_EMPTY = 0x7ff4000000000000ull;  // a signalling NaN: "not written yet"

struct ArnoldiArgs {
  double *w;              // in (unless a): the new direction; out: orthogonalised against v_0..v_j
  const double *a, *b;    // when a is set, w starts as a + b (and is only written)
  const double *V;        // v_i at V + i n
  int64_t n;              // even, every vector 16-byte aligned
  int j;
  double *hcol;           // H[0..j] of column j
  unsigned long long *slots;  // this launch's set: [npass][slot_row] (first level, then groups)
  unsigned long long *next;   // the other set, reset here for the next launch
  int npass;              // rows of slots per set (>= j + 1)
  int slot_row;           // slots per pass: RED_BLOCKS block slots + RED_BLOCKS / ARN_GROUP group slots
  double *pnorm;          // [gridDim.x] partials of <w, w>
  Status *st;
};

__device__ __forceinline__ bool arn_ready(unsigned long long v) { return v != ARN_EMPTY; }

// Wave-wide wait until the slots [0, cnt) at p are all written, then their
// sum (lane-strided in slot order, then a butterfly: the same value in every
// lane).  Returns false after a timed-out wait (the sum is then garbage).
__device__ __forceinline__ bool arn_gather(const unsigned long long *p, int cnt, Status *st, bool live,
                                           double *sum) {
  const int lane = lane_id();
  double t = 0.0;
  bool ok = true;
  for (int k0 = 0; k0 < cnt; k0 += WAVE) {
    const int k = k0 + lane;
    unsigned long long v = 0;
    long it = 0;
    for (;;) {
      v = k < cnt ? ld_dev(p + k) : 0ull;
      const bool ready = k >= cnt || arn_ready(v);
      if (!ballot(!ready) || !live) break;
      if (++it > SPIN_LIMIT) {
        if (lane == 0) raise_error(st, ILU_ERR_TIMEOUT, -1);
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (!ok) break;
    if (k < cnt) t += __longlong_as_double((long long)v);
  }
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, WAVE);
  *sum = t;
  return ok;
}

template <int K, bool SUM>
__global__ void __launch_bounds__(ARN_TT) k_arnoldi(ArnoldiArgs a) {
  __shared__ double red[ARN_T / WAVE];
  __shared__ double hsh;
  const bool gatherer = threadIdx.x >= ARN_T;  // the ninth wave (wave-uniform)
  const uint32_t G = gridDim.x;
  const uint32_t m = (uint32_t)(a.n / 2);  // element pairs (n < 2^31)
  const uint32_t stride = G * (uint32_t)ARN_T;
  const uint32_t t0 = blockIdx.x * (uint32_t)ARN_T + (gatherer ? 0u : threadIdx.x);
  const double2 *V2 = reinterpret_cast<const double2 *>(a.V);
  const bool grouped = G > (uint32_t)ARN_FLAT;
  const int ngroups = (int)((G + ARN_GROUP - 1) / ARN_GROUP);
  // reset this block's slots of the other set for the next launch
  if (gatherer) {
    for (int p = lane_id(); p < a.npass; p += WAVE) {
      unsigned long long *row = a.next + (size_t)p * a.slot_row;
      st_dev(row + blockIdx.x, ARN_EMPTY);
      if (blockIdx.x % ARN_GROUP == 0) st_dev(row + RED_BLOCKS + blockIdx.x / ARN_GROUP, ARN_EMPTY);
    }
  }
  // pair k of this thread: t0 + k stride; past the end the loads read pair 0
  // and the values are replaced by zeros, so no load is conditional
  auto at = [&](int k) -> uint32_t {
    const uint32_t p = t0 + (uint32_t)k * stride;
    return p < m ? p : 0u;
  };
  auto in = [&](int k) -> bool { return !gatherer && t0 + (uint32_t)k * stride < m; };
  double2 w[K], v[K], u[K];
  double s = 0.0;
  if (!gatherer) {
#pragma unroll
    for (int k = 0; k < K; k++) {
      if constexpr (SUM) {
        const double2 x = reinterpret_cast<const double2 *>(a.a)[at(k)];
        const double2 y = reinterpret_cast<const double2 *>(a.b)[at(k)];
        w[k] = make_double2(x.x + y.x, x.y + y.y);
      } else {
        w[k] = reinterpret_cast<const double2 *>(a.w)[at(k)];
      }
      v[k] = V2[at(k)];
    }
#pragma unroll
    for (int k = 0; k < K; k++) {
      if (!in(k)) {
        w[k] = make_double2(0.0, 0.0);
        v[k] = w[k];
      }
      s = fma(w[k].x, v[k].x, s);
      s = fma(w[k].y, v[k].y, s);
    }
  }
  bool live = true;  // the gathering wave's: no wait has timed out
  for (int i = 0;; i++) {
    // data waves: this pass's partial to LDS, then v_{i+1} on its way
    if (!gatherer) {
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
      if (lane_id() == 0) red[threadIdx.x / WAVE] = s;
      if (i < a.j) {
#pragma unroll
        for (int k = 0; k < K; k++) u[k] = V2[(size_t)(i + 1) * m + at(k)];
      }
    }
    __syncthreads();
    if (gatherer) {
      unsigned long long *row = a.slots + (size_t)i * a.slot_row;
      double t = 0.0;
      for (int k = 0; k < ARN_T / WAVE; k++) t += red[k];
      if (lane_id() == 0) st_dev(row + blockIdx.x, (unsigned long long)__double_as_longlong(t));
      double h = 0.0;
      if (!grouped) {
        live = arn_gather(row, (int)G, a.st, live, &h) && live;
      } else {
        if (blockIdx.x % ARN_GROUP == 0) {
          const int cnt = (int)min((uint32_t)ARN_GROUP, G - blockIdx.x);
          double gs = 0.0;
          live = arn_gather(row + blockIdx.x, cnt, a.st, live, &gs) && live;
          if (lane_id() == 0)
            st_dev(row + RED_BLOCKS + blockIdx.x / ARN_GROUP, (unsigned long long)__double_as_longlong(gs));
        }
        live = arn_gather(row + RED_BLOCKS, ngroups, a.st, live, &h) && live;
      }
      if (lane_id() == 0) hsh = h;
    }
    __syncthreads();
    const double h = hsh;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.hcol[i] = h;
    if (!gatherer) {
#pragma unroll
      for (int k = 0; k < K; k++) {
        w[k].x = fma(-h, v[k].x, w[k].x);
        w[k].y = fma(-h, v[k].y, w[k].y);
      }
    }
    if (i == a.j) break;
    if (!gatherer) {
      s = 0.0;
#pragma unroll
      for (int k = 0; k < K; k++) {
        v[k] = in(k) ? u[k] : make_double2(0.0, 0.0);
        s = fma(w[k].x, v[k].x, s);
        s = fma(w[k].y, v[k].y, s);
      }
    }
  }
  // the partials of <w, w> for the Givens kernel, and w
  if (!gatherer) {
    s = 0.0;
#pragma unroll
    for (int k = 0; k < K; k++) {
      s = fma(w[k].x, w[k].x, s);
      s = fma(w[k].y, w[k].y, s);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = s;
    double2 *W2 = reinterpret_cast<double2 *>(a.w);
#pragma unroll
    for (int k = 0; k < K; k++)
      if (in(k)) W2[at(k)] = w[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < ARN_T / WAVE; k++) t += red[k];
    a.pnorm[blockIdx.x] = t;
  }
}

__global__ void k_arnoldi_reset(unsigned long long *p, int64_t cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = ARN_EMPTY;
}

int64_t arnoldi_slots(int passes) { return 2LL * passes * (RED_BLOCKS + RED_BLOCKS / ARN_GROUP); }

int launch_arnoldi_reset(unsigned long long *slots, int passes, hipStream_t s) {
  const int64_t cnt = arnoldi_slots(passes);
  k_arnoldi_reset<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(slots, cnt);
  return check_launch("arnoldi_reset");
}

template <int K, bool SUM>
static int arnoldi_capacity(int num_cu) {
  // resident workgroups per CU of this instance, a property of the code
  // object: asked once (a thread-safe static initialisation)
  static const int per_cu = [] {
    int p = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p, k_arnoldi<K, SUM>, ARN_TT, 0) != hipSuccess) p = 0;
    return p;
  }();
  return std::min(per_cu, 1) * num_cu;
}

template <int K, bool SUM>
static bool arnoldi_launch_k(const ArnoldiArgs &a, unsigned grid, int num_cu, hipStream_t s) {
  if ((int)grid > arnoldi_capacity<K, SUM>(num_cu)) return false;
  k_arnoldi<K, SUM><<<grid, ARN_TT, 0, s>>>(a);
  return true;
}

template <bool SUM>
static bool arnoldi_launch(int K, const ArnoldiArgs &a, unsigned grid, int num_cu, hipStream_t s) {
  switch (K) {
    case 1: return arnoldi_launch_k<1, SUM>(a, grid, num_cu, s);
    case 2: return arnoldi_launch_k<2, SUM>(a, grid, num_cu, s);
    case 4: return arnoldi_launch_k<4, SUM>(a, grid, num_cu, s);
    default: return arnoldi_launch_k<8, SUM>(a, grid, num_cu, s);
  }
}

// Launch shape of the one-launch orthogonalisation for vectors of length n:
// the fewest workgroups that hold the vectors at ARN_KMAX element pairs per
// thread (fewer blocks make shorter sums), at most one per CU and per slot;
// K pairs per thread.  False when the kernel cannot take the vectors.
static bool arnoldi_shape(int64_t n, const void *w, const void *a, const void *b, const void *V, int num_cu,
                          int64_t *grid, int *K) {
  auto al = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
  if (n < 2 || (n & 1) || n >= ((int64_t)1 << 31) || !al(w) || !al(V) || (a && (!al(a) || !al(b))) || num_cu < 1)
    return false;
  const int64_t m = n / 2;
  const int64_t per = (int64_t)ARN_T * ARN_KMAX;
  *grid = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(num_cu, RED_BLOCKS), (m + per - 1) / per));
  *K = 1;
  while ((int64_t)*K * *grid * ARN_T < m) *K *= 2;
  return *K <= ARN_KMAX;
}

bool arnoldi_fits(int64_t n, const void *w, const void *a, const void *b, const void *V, int num_cu) {
  int64_t grid;
  int K;
  return arnoldi_shape(n, w, a, b, V, num_cu, &grid, &K);
}

int launch_arnoldi(double *w, const double *a, const double *b, const double *V, int64_t n, int j, double *hcol,
                   unsigned long long *slots, int passes, unsigned long long *launches, double *pnorm, int num_cu,
                   void *status, ArnoldiOut *out, hipStream_t s) {
  out->done = false;
  int64_t grid;
  int K;
  if (j < 0 || j + 1 > passes || !arnoldi_shape(n, w, a, b, V, num_cu, &grid, &K)) return 0;
  const int64_t set = (int64_t)(*launches & 1ull) * passes * (RED_BLOCKS + RED_BLOCKS / ARN_GROUP);
  const int64_t other = (int64_t)((*launches + 1) & 1ull) * passes * (RED_BLOCKS + RED_BLOCKS / ARN_GROUP);
  ArnoldiArgs args{w,     a,      b,    V,     n, j, hcol, slots + set, slots + other, passes,
                   RED_BLOCKS + RED_BLOCKS / ARN_GROUP, pnorm, static_cast<Status *>(status)};
  const bool ok = a ? arnoldi_launch<true>(K, args, (unsigned)grid, num_cu, s)
                    : arnoldi_launch<false>(K, args, (unsigned)grid, num_cu, s);
  if (!ok) return 0;
  *launches += 1;
  out->done = true;
  out->pnorm = pnorm;
  out->npart = (int)grid;
  return check_launch("arnoldi");
}

// R c = g by back substitution (sizes from *nsteps)
__global__ void k_backsolve(const double *H, int ldh, const double *g, const int *nsteps, double *c) {
  if (threadIdx.x != 0) return;
  const int m = *nsteps;
  for (int i = m - 1; i >= 0; i--) {
    double s = g[i];
    for (int l = i + 1; l < m; l++) s = fma(-H[i + (int64_t)ldh * l], c[l], s);
    c[i] = s / H[i + (int64_t)ldh * i];
  }
}

int launch_backsolve(const double *H, int ldh, const double *g, const int *nsteps, double *c, hipStream_t s) {
  k_backsolve<<<1, WAVE, 0, s>>>(H, ldh, g, nsteps, c);
  return check_launch("backsolve");
}

// y (+)= sum_i c_i V_i, i < *nsteps, accumulated in i order per element
__global__ void k_combine(double *y, const double *V, int64_t ldv, const double *c, const int *nsteps, int64_t n,
                          bool accumulate) {
  int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l >= n) return;
  const int m = *nsteps;
  double s = accumulate ? y[l] : 0.0;
  for (int i = 0; i < m; i++) s = fma(c[i], V[(int64_t)i * ldv + l], s);
  y[l] = s;
}

int launch_combine(double *y, const double *V, int64_t ldv, const double *c, const int *nsteps, int64_t n,
                   bool accumulate, hipStream_t s) {
  if (n == 0) return 0;
  k_combine<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(y, V, ldv, c, nsteps, n, accumulate);
  return check_launch("combine");
}

// g[0] = beta; stop = (beta == 0); nsteps = 0
__global__ void k_init_krylov(double *g, const double *beta, int *stop, int *nsteps) {
  if (threadIdx.x != 0) return;
  const double b = *beta;
  g[0] = b;
  *nsteps = 0;
  *stop = (b == 0.0) ? 1 : (!isfinite(b) ? 3 : 0);
}

int launch_init_krylov(double *g, const double *beta, int *stop, int *nsteps, hipStream_t s) {
  k_init_krylov<<<1, WAVE, 0, s>>>(g, beta, stop, nsteps);
  return check_launch("init_krylov");
}

}  // namespace silu
