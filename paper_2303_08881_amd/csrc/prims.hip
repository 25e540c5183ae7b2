// prims.hip -- integer primitives for the setup phase: exclusive scan, stable
// LSD radix sort, key histogram, fills.  All results are exact integers and
// independent of scheduling (no order-dependent atomics on outputs).
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"

namespace silu {

// ---------------------------------------------------------------- scan
constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ int64_t block_exclusive_scan(int64_t v, int64_t *total) {
  __shared__ int64_t wsum[SCAN_THREADS / WAVE];
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  int64_t incl = v;
  for (int o = 1; o < WAVE; o <<= 1) {
    int64_t t = __shfl_up(incl, o, WAVE);
    if (lane >= o) incl += t;
  }
  if (lane == WAVE - 1) wsum[w] = incl;
  __syncthreads();
  if (w == 0) {
    int64_t s = lane < SCAN_THREADS / WAVE ? wsum[lane] : 0;
    int64_t si = s;
    for (int o = 1; o < WAVE; o <<= 1) {
      int64_t t = __shfl_up(si, o, WAVE);
      if (lane >= o) si += t;
    }
    if (lane < SCAN_THREADS / WAVE) wsum[lane] = si - s;
    if (lane == WAVE - 1) *total = si;
  }
  __syncthreads();
  int64_t r = wsum[w] + incl - v;
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const int64_t *in, int64_t n, int64_t *bsum) {
  __shared__ int64_t total;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; k++)
    if (base + k < n) s += in[base + k];
  block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_apply(const int64_t *in, int64_t n, const int64_t *boff,
                                                            int64_t *out, bool write_total) {
  __shared__ int64_t total;
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int64_t x[SCAN_ITEMS];
  int64_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; k++) {
    x[k] = base + k < n ? in[base + k] : 0;
    s += x[k];
  }
  int64_t run = block_exclusive_scan(s, &total) + (boff ? boff[blockIdx.x] : 0);
  for (int k = 0; k < SCAN_ITEMS; k++) {
    if (base + k < n) out[base + k] = run;
    run += x[k];
  }
  if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
    out[n] = total + (boff ? boff[blockIdx.x] : 0);
}

size_t scan_tmp_bytes(int64_t n) {
  size_t b = 0;
  int64_t m = n;
  while (m > SCAN_TILE) {
    int64_t nb = (m + SCAN_TILE - 1) / SCAN_TILE;
    b += 2 * (size_t)(nb + 1) * sizeof(int64_t);
    m = nb;
  }
  return b + 64;
}

static int scan_rec(const int64_t *in, int64_t *out, int64_t n, bool total, int64_t *tmp, hipStream_t s) {
  if (n <= 0) {
    if (total) return fill_i64(out, 0, 1, s);
    return check_launch("scan0");
  }
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 1) {
    k_scan_apply<<<1, SCAN_THREADS, 0, s>>>(in, n, nullptr, out, total);
    return check_launch("scan_apply");
  }
  int64_t *bsum = tmp, *boff = tmp + (nb + 1);
  k_scan_reduce<<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, n, bsum);
  if (int rc = check_launch("scan_reduce")) return rc;
  if (int rc = scan_rec(bsum, boff, nb, false, tmp + 2 * (nb + 1), s)) return rc;
  k_scan_apply<<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, n, boff, out, total);
  return check_launch("scan_apply");
}

int scan_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp, size_t tmp_bytes, hipStream_t s) {
  if (tmp_bytes < scan_tmp_bytes(n)) return ILU_ERR_INVALID_ARG;
  return scan_rec(in, out, n, true, (int64_t *)tmp, s);
}

// ---------------------------------------------------------------- radix sort
constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;

__global__ void __launch_bounds__(RS_THREADS) k_radix_hist(const uint32_t *key, int64_t n, int shift,
                                                           int64_t nblocks, int64_t *counts) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; r++) {
    int64_t i = base + r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & 255], 1);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(RS_THREADS) k_radix_scatter(const uint32_t *key, const int32_t *val, int64_t n,
                                                              int shift, int64_t nblocks, const int64_t *offsets,
                                                              uint32_t *key_out, int32_t *val_out) {
  __shared__ int run[256];
  __shared__ int wcount[RS_THREADS / WAVE][256];
  const int lane = lane_id(), w = threadIdx.x / WAVE;
  run[threadIdx.x] = 0;
  for (int q = 0; q < RS_THREADS / WAVE; q++) wcount[q][threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < RS_ROUNDS; r++) {
    const int64_t i = base + r * RS_THREADS + threadIdx.x;
    const bool valid = i < n;
    const uint32_t k = valid ? key[i] : 0u;
    const int32_t v = valid ? val[i] : 0;
    const int d = (k >> shift) & 255;
    unsigned long long peers = ballot(valid);
    for (int b = 0; b < 8; b++) {
      const unsigned long long m = ballot(valid && ((d >> b) & 1));
      peers &= ((d >> b) & 1) ? m : ~m;
    }
    const int rank = popc64(peers & lt);
    if (valid && rank == 0) wcount[w][d] = popc64(peers);
    __syncthreads();
    if (valid) {
      int64_t o = offsets[(int64_t)d * nblocks + blockIdx.x] + run[d] + rank;
      for (int q = 0; q < w; q++) o += wcount[q][d];
      key_out[o] = k;
      val_out[o] = v;
    }
    __syncthreads();
    {
      int add = 0;
      for (int q = 0; q < RS_THREADS / WAVE; q++) {
        add += wcount[q][threadIdx.x];
        wcount[q][threadIdx.x] = 0;
      }
      run[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

size_t radix_tmp_bytes(int64_t n) {
  const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
  const int64_t nc = 256 * nb;
  return (size_t)n * 8 * 2 + (size_t)(nc + 1) * 8 * 2 + scan_tmp_bytes(nc) + 256;
}

int radix_sort(const uint32_t *key_in, const int32_t *val_in, uint32_t *key_out, int32_t *val_out, int64_t n,
               int key_bits, void *tmp, size_t tmp_bytes, hipStream_t s) {
  if (tmp_bytes < radix_tmp_bytes(n)) return ILU_ERR_INVALID_ARG;
  if (n == 0) return 0;
  const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
  const int64_t nc = 256 * nb;
  char *p = (char *)tmp;
  uint32_t *ka = (uint32_t *)p;
  p += (size_t)n * 4;
  uint32_t *kb = (uint32_t *)p;
  p += (size_t)n * 4;
  int32_t *va = (int32_t *)p;
  p += (size_t)n * 4;
  int32_t *vb = (int32_t *)p;
  p += (size_t)n * 4;
  int64_t *counts = (int64_t *)p;
  p += (size_t)(nc + 1) * 8;
  int64_t *offs = (int64_t *)p;
  p += (size_t)(nc + 1) * 8;
  void *stmp = p;
  const size_t stb = scan_tmp_bytes(nc);
  int passes = (key_bits + 7) / 8;
  if (passes < 1) passes = 1;
  const uint32_t *ki = key_in;
  const int32_t *vi = val_in;
  for (int ps = 0; ps < passes; ps++) {
    const bool last = ps == passes - 1;
    uint32_t *ko = last ? key_out : ((ps & 1) ? kb : ka);
    int32_t *vo = last ? val_out : ((ps & 1) ? vb : va);
    k_radix_hist<<<(unsigned)nb, RS_THREADS, 0, s>>>(ki, n, 8 * ps, nb, counts);
    if (int rc = check_launch("radix_hist")) return rc;
    if (int rc = scan_i64(counts, offs, nc, stmp, stb, s)) return rc;
    k_radix_scatter<<<(unsigned)nb, RS_THREADS, 0, s>>>(ki, vi, n, 8 * ps, nb, offs, ko, vo);
    if (int rc = check_launch("radix_scatter")) return rc;
    ki = ko;
    vi = vo;
  }
  return 0;
}

// ---------------------------------------------------------------- misc
// exact integer counts; bins below HIST_LDS are counted in LDS per block
// first (few bins receive most keys, e.g. subdomain ids), the rest directly
constexpr int HIST_LDS = 4096;

__global__ void __launch_bounds__(256) k_histogram(const uint32_t *key, int64_t n, int64_t nbins, int64_t *counts) {
  __shared__ int h[HIST_LDS];
  const int nl = nbins < HIST_LDS ? (int)nbins : HIST_LDS;
  for (int b = threadIdx.x; b < nl; b += 256) h[b] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += stride) {
    const uint32_t k = key[i];
    if (k < (uint32_t)nl)
      atomicAdd(&h[k], 1);
    else if (k < (uint64_t)nbins)
      atomicAdd((unsigned long long *)&counts[k], 1ull);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nl; b += 256)
    if (h[b]) atomicAdd((unsigned long long *)&counts[b], (unsigned long long)h[b]);
}

int histogram_keys(const uint32_t *key, int64_t n, int64_t nbins, int64_t *counts, hipStream_t s) {
  if (int rc = fill_i64(counts, 0, nbins, s)) return rc;
  if (n == 0) return 0;
  int64_t blocks = (n + 256 * 16 - 1) / (256 * 16);
  if (blocks > 2048) blocks = 2048;
  k_histogram<<<(unsigned)blocks, 256, 0, s>>>(key, n, nbins, counts);
  return check_launch("histogram");
}

template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

int fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return 0;
  k_fill<int32_t><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
  return check_launch("fill_i32");
}
int fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return 0;
  k_fill<int64_t><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
  return check_launch("fill_i64");
}
int fill_f64(double *p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return 0;
  k_fill<double><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
  return check_launch("fill_f64");
}

__global__ void k_iota(int32_t *p, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}
int iota_i32(int32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return 0;
  k_iota<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
  return check_launch("iota");
}

// max over the grid: each block folds its grid-stride share, then one atomic
// per block (a single counter hit by every wave would serialise)
constexpr int MAX_BLOCKS = 1024;
__device__ inline void block_max_atomic(int v, int32_t *out) {
  __shared__ int wm[256 / WAVE];
  v = wave_max_int(v);
  if (lane_id() == 0) wm[threadIdx.x / WAVE] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = wm[0];
    for (int k = 1; k < (int)(blockDim.x / WAVE); k++) m = max(m, wm[k]);
    if (m >= 0) atomicMax(out, m);
  }
}
__global__ void __launch_bounds__(256) k_max_i32(const int32_t *p, int64_t n, int32_t *out) {
  int v = -1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v = max(v, p[i]);
  block_max_atomic(v, out);
}
int max_i32(const int32_t *p, int64_t n, int32_t *d_out, hipStream_t s) {
  if (int rc = fill_i32(d_out, -1, 1, s)) return rc;
  if (n <= 0) return 0;
  const int64_t g = std::min<int64_t>((n + 255) / 256, MAX_BLOCKS);
  k_max_i32<<<(unsigned)g, 256, 0, s>>>(p, n, d_out);
  return check_launch("max_i32");
}

}  // namespace silu
