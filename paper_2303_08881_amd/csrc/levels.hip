// levels.hip -- level sets of sparse triangular factors (Section 3.1: the
// analysis phase that lets the rows of one level be processed together).
//
// level(r) = 0 when row r has no dependency, else 1 + max level(dependency);
// for a lower factor the dependencies of r are its columns in [lo, r), for an
// upper factor its columns in (r, hi).
//
// Also here: the keys that sort rows by level (and by block, then level) and
// the chunk table of the cross-workgroup triangular solve.
#include "common.hpp"
#include "launch.hpp"

namespace silu {

// Level of every row of a triangular factor by a dependency-ordered sweep:
// level(r) = 1 + max level of the rows r depends on (0 without any).  The
// rows come in chunks of consecutive rows (a line, from the top down for an
// upper factor) grouped in streams, exactly like the factorization's schedule.
// A workgroup of LEVEL_WAVES waves takes a chunk, its waves taking the rows in
// turn, one row at a time: dependencies inside the chunk come from the
// workgroup's LDS (polled until the other wave has written them), the others
// from the completion flag of their row, which holds level + 1 (0 = not yet
// known) -- the value is its own payload, so no fence is needed on either
// side.  While one wave waits on a flag, the other works on its row.  Waits
// are bounded.
__device__ inline int wait_nonzero(const int *flag, Status *st, int64_t row) {
  long it = 0;
  int v;
  while ((v = ld_relaxed(flag)) == 0) {
    if (++it > SPIN_LIMIT) {
      raise_error(st, ILU_ERR_TIMEOUT, row);
      return -1;
    }
    if ((it & 255) == 0 && ld_relaxed(&st->abort)) return -1;
    __builtin_amdgcn_s_sleep(1);
  }
  return v;
}

// level of an earlier row of this chunk, once its wave has stored it
__device__ inline int32_t wait_lds_level(const volatile int32_t *slot, Status *st, int64_t row) {
  long it = 0;
  int32_t v;
  while ((v = *slot) < 0) {
    if (++it > SPIN_LIMIT) {
      raise_error(st, ILU_ERR_TIMEOUT, row);
      return -1;
    }
    if ((it & 255) == 0 && ld_relaxed(&st->abort)) return -1;
    __builtin_amdgcn_s_sleep(1);
  }
  return v;
}

__global__ void __launch_bounds__(WAVE *LEVEL_WAVES) k_levels_stream(const int64_t *rp, const int32_t *ci, bool lower,
                                                                    int64_t lo, int64_t hi, const int2 *chunks,
                                                                    int64_t nstreams, int64_t ninit,
                                                                    const int64_t *stream_chunk, unsigned int *ticket,
                                                                    int32_t *level, int *done, Status *st) {
  __shared__ int32_t clev[LEVEL_CHUNK_MAX];
  __shared__ long long sh_t;
  const int lane = lane_id();
  const int w = (int)(threadIdx.x / WAVE);
  int64_t sid = (int64_t)blockIdx.x % ninit;
  for (;;) {
    __syncthreads();  // every wave is done with the previous chunk
    if (w == 0) {
      int64_t t = -1;
      for (int64_t tries = 0; tries < nstreams && t < 0; tries++) {
        const int64_t c0 = stream_chunk[sid], nc = stream_chunk[sid + 1] - c0;
        if ((int64_t)uniform_i32(ld_relaxed(reinterpret_cast<const int *>(ticket + sid))) < nc) {
          const unsigned int tl = wave_ticket(ticket + sid);
          if ((int64_t)tl < nc) t = c0 + (int64_t)tl;
        }
        if (t < 0) sid = sid + 1 < nstreams ? sid + 1 : 0;
      }
      if (ld_relaxed(&st->abort)) t = -1;
      if (threadIdx.x == 0) sh_t = t;
    }
    for (int i = (int)threadIdx.x; i < LEVEL_CHUNK_MAX; i += WAVE * LEVEL_WAVES) clev[i] = -1;
    __syncthreads();
    const int64_t t = sh_t;
    if (t < 0) return;
    const int2 ch = chunks[t];
    const int64_t first = ch.x;
    for (int32_t i = w; i < ch.y; i += LEVEL_WAVES) {
      const int64_t r = lower ? first + i : first - i;
      int32_t m = 0;
      bool ok = true;
      for (int64_t base = rp[r]; base < rp[r + 1]; base += WAVE) {
        const int64_t p = base + lane;
        if (p < rp[r + 1]) {
          const int64_t c = ci[p];
          if (lower ? (c >= lo && c < r) : (c > r && c < hi)) {
            const int64_t off = lower ? c - first : first - c;  // position in this chunk
            int32_t lv;
            if (off >= 0 && off < i) {
              lv = wait_lds_level(&clev[off], st, r);
              ok = ok && lv >= 0;
            } else {
              const int v = wait_nonzero(&done[c], st, r);
              ok = ok && v > 0;
              lv = v - 1;
            }
            m = max(m, lv + 1);
          }
        }
      }
      if (ballot(!ok)) break;
      m = uniform_i32(wave_max_int(m));
      if (lane == 0) {
        level[r] = m;
        st_dev(&done[r], m + 1);
        __hip_atomic_store(&clev[i], m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
}

int levels_resident_groups(int num_cu) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_levels_stream, WAVE * LEVEL_WAVES, 0) != hipSuccess)
    return 0;
  return per_cu * num_cu;
}

int launch_levels_stream(const int64_t *rp, const int32_t *ci, bool lower, int64_t lo, int64_t hi,
                         const int32_t *chunks, int64_t nstreams, int64_t ninit, const int64_t *stream_chunk,
                         unsigned int *ticket, int32_t *level, int *done, void *status, int64_t grid, hipStream_t s) {
  if (nstreams == 0) return 0;
  if (grid < ninit || ninit < 1 || ninit > nstreams) return ILU_ERR_INVALID_ARG;
  const int2 *ch = reinterpret_cast<const int2 *>(chunks);
  Status *st = (Status *)status;
  void *args[] = {(void *)&rp, (void *)&ci, (void *)&lower, (void *)&lo, (void *)&hi, (void *)&ch,
                  (void *)&nstreams, (void *)&ninit, (void *)&stream_chunk, (void *)&ticket, (void *)&level,
                  (void *)&done, (void *)&st};
  // all workgroups resident at once, as in the factorization
  const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_levels_stream),
                                                  dim3((unsigned)grid), dim3(WAVE * LEVEL_WAVES), args, 0, s);
  if (e != hipSuccess) return ILU_ERR_HIP;
  return check_launch("levels_stream");
}

// Levels of rows [row0, n) whose dependencies (columns in [lo, hi), below the
// row) all have their levels already: one thread per row.
__global__ void k_rows_level(const int64_t *rp, const int32_t *ci, int64_t row0, int64_t n, int64_t lo, int64_t hi,
                             int32_t *level) {
  const int64_t r = row0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  int32_t m = 0;
  for (int64_t p = rp[r]; p < rp[r + 1]; p++) {
    const int64_t c = ci[p];
    if (c >= lo && c < hi && c < r) m = max(m, level[c] + 1);
  }
  level[r] = m;
}

int launch_rows_level(const int64_t *rp, const int32_t *ci, int64_t row0, int64_t n, int64_t lo, int64_t hi,
                      int32_t *level, hipStream_t s) {
  if (n <= row0) return 0;
  k_rows_level<<<(unsigned)((n - row0 + 255) / 256), 256, 0, s>>>(rp, ci, row0, n, lo, hi, level);
  return check_launch("rows_level");
}

__global__ void k_levels_to_keys(const int32_t *level, int64_t n, uint32_t *key, int32_t *val) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = (uint32_t)level[i];
  val[i] = (int32_t)i;
}

int launch_levels_to_keys(const int32_t *level, int64_t n, uint32_t *key, int32_t *val, hipStream_t s) {
  if (n == 0) return 0;
  k_levels_to_keys<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(level, n, key, val);
  return check_launch("levels_to_keys");
}

// block (subdomain) of each row: rows below `split` use the ascending block
// starts s1[0..nblk], the others s2[0..nblk] (NULL: s1 for every row); the
// block is the last one whose start is <= r (empty blocks are skipped).
__device__ inline int32_t last_start_le(const int64_t *s, int32_t nblk, int64_t r) {
  int32_t lo = 0, hi = nblk + 1;  // first index with s[idx] > r, in [0, nblk+1]
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (s[mid] <= r)
      lo = mid + 1;
    else
      hi = mid;
  }
  const int32_t b = lo - 1;
  return b < 0 ? 0 : (b >= nblk ? nblk - 1 : b);
}

__global__ void k_row_blocks(int64_t nrows, int32_t nblk, const int64_t *s1, const int64_t *s2, int64_t split,
                             int32_t *blk) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  blk[r] = last_start_le((s2 && r >= split) ? s2 : s1, nblk, r);
}

int launch_row_blocks(int64_t nrows, int32_t nblk, const int64_t *s1, const int64_t *s2, int64_t split, int32_t *blk,
                      hipStream_t s) {
  if (nrows == 0) return 0;
  k_row_blocks<<<(unsigned)((nrows + 255) / 256), 256, 0, s>>>(nrows, nblk, s1, s2, split, blk);
  return check_launch("row_blocks");
}

// ---- connected components of a symmetric pattern (union-find) ----------
// Every label points to a smaller or equal index, so a find follows a
// strictly decreasing chain and ends; a union hooks the larger root under
// the smaller with a compare-and-swap and retries from what it finds when
// another thread got there first, so one pass over the edges joins every
// component (no iteration to a fixed point).  A find halves its path: a
// label that is not a root is pointed at its grandparent, still an ancestor
// in the same tree (only roots are ever hooked), which keeps the chains
// short on path-like patterns.  Labels are read with device-scope loads: a
// stale copy only sends a find along an older, longer chain, and the swap
// sees the current value.
__device__ __forceinline__ int32_t cc_find(int32_t *lab, int32_t x) {
  for (;;) {
    const int32_t p = ld_dev(lab + x);
    if (p == x) return x;
    const int32_t gp = ld_dev(lab + p);
    if (gp != p) st_dev(lab + x, gp);
    x = p;
  }
}

__global__ void k_cc_init(int32_t *lab, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) lab[i] = (int32_t)i;
}

// edges (r, c) of rows [0, n) with columns in [0, n), c != r
__global__ void k_cc_hook(const int64_t *rp, const int32_t *ci, int64_t n, int32_t *lab) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int64_t p = rp[r]; p < rp[r + 1]; p++) {
    const int64_t c = ci[p];
    if (c < 0 || c >= n || c == r) continue;
    int32_t a = cc_find(lab, (int32_t)r), b = cc_find(lab, (int32_t)c);
    while (a != b) {
      if (a < b) {
        const int32_t t = a;
        a = b;
        b = t;
      }
      // a > b: hook root a under b, unless a is no longer a root
      const int32_t old = atomicCAS(lab + a, a, b);
      if (old == a) break;
      a = cc_find(lab, old);
      b = cc_find(lab, b);
    }
  }
}

// root[i] = the smallest index of i's component; isroot[i] = (root[i] == i)
__global__ void k_cc_flatten(int32_t *lab, int64_t n, int32_t *root, int64_t *isroot) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t r = cc_find(lab, (int32_t)i);
  root[i] = r;
  isroot[i] = r == (int32_t)i ? 1 : 0;
}

// comp[i] = number of the component of i (roots numbered in index order)
__global__ void k_cc_number(const int32_t *root, const int64_t *rank, int64_t n, int32_t *comp) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) comp[i] = (int32_t)rank[root[i]];
}

int launch_cc_label(const int64_t *rp1, const int32_t *ci1, const int64_t *rp2, const int32_t *ci2, int64_t n,
                    int32_t *lab, int32_t *root, int64_t *isroot, hipStream_t s) {
  if (n == 0) return 0;
  const unsigned g = (unsigned)((n + 255) / 256);
  k_cc_init<<<g, 256, 0, s>>>(lab, n);
  k_cc_hook<<<g, 256, 0, s>>>(rp1, ci1, n, lab);
  if (rp2) k_cc_hook<<<g, 256, 0, s>>>(rp2, ci2, n, lab);
  k_cc_flatten<<<g, 256, 0, s>>>(lab, n, root, isroot);
  return check_launch("cc_label");
}

int launch_cc_number(const int32_t *root, const int64_t *rank, int64_t n, int32_t *comp, hipStream_t s) {
  if (n == 0) return 0;
  k_cc_number<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(root, rank, n, comp);
  return check_launch("cc_number");
}

__global__ void k_block_level_keys(const int32_t *level, const int32_t *blk, int64_t n, int64_t nlev, uint32_t *key,
                                   int32_t *val) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = (uint32_t)((int64_t)blk[i] * nlev + level[i]);
  val[i] = (int32_t)i;
}

int launch_block_level_keys(const int32_t *level, const int32_t *blk, int64_t n, int64_t nlev, uint32_t *key,
                            int32_t *val, hipStream_t s) {
  if (n == 0) return 0;
  k_block_level_keys<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(level, blk, n, nlev, key, val);
  return check_launch("block_level_keys");
}

__global__ void k_i64_to_i32(const int64_t *in, int32_t *out, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int32_t)in[i];
}

int launch_i64_to_i32(const int64_t *in, int32_t *out, int64_t n, hipStream_t s) {
  if (n == 0) return 0;
  k_i64_to_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(in, out, n);
  return check_launch("i64_to_i32");
}

// number of <=64-row chunks in each level
__global__ void k_level_chunk_counts(const int64_t *level_ptr, int64_t nlev, int64_t *cnt) {
  int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l >= nlev) return;
  cnt[l] = (level_ptr[l + 1] - level_ptr[l] + WAVE - 1) / WAVE;
}

int launch_level_chunk_counts(const int64_t *level_ptr, int64_t nlev, int64_t *cnt, hipStream_t s) {
  if (nlev == 0) return 0;
  k_level_chunk_counts<<<(unsigned)((nlev + 255) / 256), 256, 0, s>>>(level_ptr, nlev, cnt);
  return check_launch("level_chunk_counts");
}

__global__ void k_level_chunks(const int64_t *level_ptr, int64_t nlev, const int64_t *chunk_base,
                               int32_t *chunk_start, int32_t *chunk_level) {
  int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l >= nlev) return;
  const int64_t b = level_ptr[l], e = level_ptr[l + 1];
  int64_t c = chunk_base[l];
  for (int64_t x = b; x < e; x += WAVE, c++) {
    chunk_start[c] = (int32_t)x;
    chunk_level[c] = (int32_t)l;
  }
  if (l == nlev - 1) chunk_start[chunk_base[nlev]] = (int32_t)e;
}

int launch_level_chunks(const int64_t *level_ptr, int64_t nlev, const int64_t *chunk_base, int32_t *chunk_start,
                        int32_t *chunk_level, hipStream_t s) {
  if (nlev == 0) return 0;
  k_level_chunks<<<(unsigned)((nlev + 255) / 256), 256, 0, s>>>(level_ptr, nlev, chunk_base, chunk_start,
                                                                 chunk_level);
  return check_launch("level_chunks");
}

}  // namespace silu
