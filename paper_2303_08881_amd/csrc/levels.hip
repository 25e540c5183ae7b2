// levels.hip -- level sets of sparse triangular factors (Section 3.1: the
// analysis phase that lets the rows of one level be processed together).
//
// level(r) = 0 when row r has no dependency, else 1 + max level(dependency);
// for a lower factor the dependencies of r are its columns in [lo, r), for an
// upper factor its columns in (r, hi).
//
// Sync-free evaluation: a wave takes 64 consecutive rows (in dependency
// order: ascending for lower, descending for upper) by atomic ticket.  A row
// first waits, with bounded polls, for the completion flags of dependencies
// outside its chunk, then the chunk resolves its internal chain in rounds
// (each round finishes every row whose in-chunk dependencies are done).
#include "common.hpp"
#include "launch.hpp"

namespace silu {

__global__ void __launch_bounds__(WAVE) k_levels(const int64_t *rp, const int32_t *ci, int64_t n, bool lower,
                                                  int64_t lo, int64_t hi, int32_t *level, int *done, int epoch,
                                                  unsigned int *ticket, Status *st) {
  __shared__ int32_t lev_s[WAVE];
  __shared__ int32_t ok_s[WAVE];
  const int lane = lane_id();
  const int64_t nchunks = (n + WAVE - 1) / WAVE;
  for (;;) {
    const int64_t t = wave_ticket(ticket);
    if (t >= nchunks) return;
    const int64_t q = t * WAVE + lane;  // position in dependency order
    const bool valid = q < n;
    const int64_t r = lower ? q : n - 1 - q;
    const int64_t cb = t * WAVE;        // chunk covers positions [cb, cb+64)
    int32_t m = 0;                       // max over resolved dependencies of level+1
    bool ok = true;
    if (valid) {
      for (int64_t p = rp[r]; p < rp[r + 1]; p++) {
        const int64_t c = ci[p];
        const bool dep = lower ? (c >= lo && c < r) : (c > r && c < hi);
        if (!dep) continue;
        const int64_t qc = lower ? c : n - 1 - c;
        if (qc >= cb) continue;  // inside this chunk: resolved below
        if (!wait_flag_eq(&done[c], epoch, st, r)) {
          ok = false;
          break;
        }
      }
    }
    if (ballot(!ok)) return;
    fence_acquire();
    if (valid) {
      for (int64_t p = rp[r]; p < rp[r + 1]; p++) {
        const int64_t c = ci[p];
        const bool dep = lower ? (c >= lo && c < r) : (c > r && c < hi);
        if (!dep) continue;
        const int64_t qc = lower ? c : n - 1 - c;
        if (qc >= cb) continue;
        m = max(m, level[c] + 1);
      }
    }
    ok_s[lane] = valid ? 0 : 1;
    lev_s[lane] = m;
    __syncthreads();
    // in-chunk chain: dependencies sit at smaller positions, i.e. lower lanes
    for (int round = 0; round < WAVE; round++) {
      bool ready = true;
      int32_t mm = m;
      if (valid && !ok_s[lane]) {
        for (int64_t p = rp[r]; p < rp[r + 1]; p++) {
          const int64_t c = ci[p];
          const bool dep = lower ? (c >= lo && c < r) : (c > r && c < hi);
          if (!dep) continue;
          const int64_t qc = lower ? c : n - 1 - c;
          if (qc < cb) continue;
          const int l2 = (int)(qc - cb);
          if (!ok_s[l2]) {
            ready = false;
            break;
          }
          mm = max(mm, lev_s[l2] + 1);
        }
      }
      __syncthreads();
      if (valid && !ok_s[lane] && ready) {
        lev_s[lane] = mm;
        ok_s[lane] = 1;
      }
      __syncthreads();
      if (!ballot(ok_s[lane] == 0)) break;
    }
    if (valid) {
      level[r] = lev_s[lane];
      st_release(&done[r], epoch);
    }
    __syncthreads();
  }
}

// Chunked variant: tickets hand out short runs of consecutive rows of one
// subdomain in dependency order (ascending for lower factors, descending for
// upper ones; subdomains interleaved).  A wave processes its rows one after
// the other; for each row all lanes gather the levels of its dependencies --
// from LDS when the dependency is an earlier row of the same chunk, else
// after a bounded wait on its completion flag -- and a wave max gives the
// level.  Any topological order is deadlock-free: every dependency outside
// the chunk belongs to an earlier ticket.
__global__ void __launch_bounds__(WAVE) k_levels_seq(const int64_t *rp, const int32_t *ci, bool lower, int64_t lo,
                                                     int64_t hi, int64_t nchunks, const int64_t *chunk_ptr,
                                                     const int32_t *order, int32_t *level, int *done, int epoch,
                                                     unsigned int *ticket, Status *st) {
  __shared__ int32_t crow[LEVEL_CHUNK_ROWS];
  __shared__ int32_t clev[LEVEL_CHUNK_ROWS];
  const int lane = lane_id();
  for (;;) {
    const unsigned int t = wave_ticket(ticket);
    if (t >= (unsigned long long)nchunks) return;
    const int64_t cb = chunk_ptr[t], ce = chunk_ptr[t + 1];
    for (int64_t oi = cb; oi < ce; oi++) {
      const int32_t j = (int32_t)(oi - cb);
      const int64_t r = order[oi];
      int32_t m = 0;
      bool ok = true;
      for (int64_t base = rp[r]; base < rp[r + 1]; base += WAVE) {
        const int64_t p = base + lane;
        if (p < rp[r + 1]) {
          const int64_t c = ci[p];
          const bool dep = lower ? (c >= lo && c < r) : (c > r && c < hi);
          if (dep) {
            int32_t lv = -1;
            for (int32_t k = 0; k < j; k++)
              if (crow[k] == (int32_t)c) lv = clev[k];
            if (lv < 0) {
              if (!wait_flag_eq(&done[c], epoch, st, r)) {
                ok = false;
              } else {
                fence_acquire();
                lv = level[c];
              }
            }
            m = max(m, lv + 1);
          }
        }
      }
      if (ballot(!ok)) return;
      m = uniform_i32(wave_max_int(m));
      if (lane == 0) {
        level[r] = m;
        crow[j] = (int32_t)r;
        clev[j] = m;
      }
      __syncthreads();
      if (lane == 0) st_release(&done[r], epoch);
    }
    __syncthreads();
  }
}

int launch_levels_seq(const int64_t *rp, const int32_t *ci, bool lower, int64_t lo, int64_t hi, int64_t nchunks,
                      const int64_t *chunk_ptr, const int32_t *order, int32_t *level, int *done, int epoch,
                      unsigned int *ticket, void *status, int64_t max_waves, hipStream_t s) {
  if (nchunks == 0) return 0;
  const int64_t grid = nchunks < max_waves ? nchunks : max_waves;
  k_levels_seq<<<(unsigned)grid, WAVE, 0, s>>>(rp, ci, lower, lo, hi, nchunks, chunk_ptr, order, level, done, epoch,
                                               ticket, (Status *)status);
  return check_launch("levels_seq");
}

int launch_levels(const int64_t *rp, const int32_t *ci, int64_t n, bool lower, int64_t lo, int64_t hi,
                  int32_t *level, int *done, int epoch, unsigned int *ticket, void *status, int64_t max_waves,
                  hipStream_t s) {
  if (n == 0) return 0;
  const int64_t nchunks = (n + WAVE - 1) / WAVE;
  const int64_t grid = nchunks < max_waves ? nchunks : max_waves;
  k_levels<<<(unsigned)grid, WAVE, 0, s>>>(rp, ci, n, lower, lo, hi, level, done, epoch, ticket, (Status *)status);
  return check_launch("levels");
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
