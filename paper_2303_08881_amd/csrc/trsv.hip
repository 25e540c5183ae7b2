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
  k_trsv<<<(unsigned)grid, WAVE, 0, s>>>(a);
  return check_launch("trsv");
}

}  // namespace silu
