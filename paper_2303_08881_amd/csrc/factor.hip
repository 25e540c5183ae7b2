// factor.hip -- row-wise incomplete LU on the device: ILU(0), MILU(0), ILUT,
// full rows and partial (Schur-complement) rows.
//
// What is computed (per row r, columns ascending):
//   * w = row r of M;  tau_r = droptol * ||row r of M||_2 (ILUT only);
//   * for each pivot column k < lim (lim = r for full rows, nfull for the
//     partial rows of eq. (17)) in ascending order:
//       w_k = w_k / u_kk; ILUT: if |w_k| < tau_r drop it and skip;
//       w_j = fma(-w_k, u_kj, w_j) for u_kj in the U part of row k;
//       a u_kj outside the current row is new fill (ILUT), dropped and summed
//       into the diagonal (MILU, Section 2.3 eq. (16)), or dropped (ILU(0));
//   * ILUT: off-diagonal entries of the U / Schur part below tau_r are
//     dropped; each part keeps its lfil largest magnitudes (ties: smaller
//     column first); the diagonal is always kept.
//
// GPU organisation (no level analysis is needed, so fill may appear anywhere):
//   * one wavefront per row, rows handed out by an atomic ticket in a
//     topological order: subdomains are independent, and inside a subdomain
//     every dependency of a row precedes it in the local (interior-first)
//     order.  A ticket covers CHUNK consecutive local rows of one subdomain,
//     processed one after the other by the same wave, and tickets interleave
//     the subdomains round-robin;
//   * a row waits on the per-row completion flag of each pivot k (agent-scope
//     release, then device-scope loads of the pivot row); every wait is
//     bounded;
//   * the working row is kept sorted by column in LDS; the pivot walk is a
//     scan of its prefix; fill is merged in place (one wave: read all, then
//     write all);
//   * results go to fixed-capacity per-row slots (ELL-like, capacities from a
//     scan) and are compacted into CSR afterwards.
#include "common.hpp"
#include "launch.hpp"

namespace silu {

constexpr int FACT_CAP = 512;  // working-row capacity (entries) per wave
constexpr int FACT_UCACHE = 768;  // LDS entries caching the U rows of a round's pivots (>= FACT_CAP, so a
                                  // round's first pivot always fits)
constexpr int FACT_UROW = 20;     // entries of a cached U row fetched with the diagonal (the fill limit
                                  // of the usual ILUT settings, so one trip to memory reads the row)
constexpr int FACT_UTAIL = 8;     // entries per lane in each further batch of a longer row

struct FactArgs {
  const int64_t *rp;
  const int32_t *ci;
  const double *v;
  int64_t n, nfull;
  int32_t method;
  double droptol;
  int32_t lfil;
  int32_t pivot_mode;
  double pivot_tol;
  // schedule: chunks of consecutive rows {first row, count}, grouped in
  // streams (contiguous runs of chunks in row order, each with a ticket
  // counter); workgroup w starts on stream w mod ninit and, once that stream
  // has handed out all its chunks, joins the next stream that has chunks left
  int64_t nchunks;
  const int2 *chunks;
  int64_t nstreams, ninit;
  const int64_t *stream_chunk;  // [nstreams+1] first chunk of each stream
  unsigned int *ticket;         // [nstreams]
  // outputs
  const int64_t *Lrp;
  int32_t *Lc;
  double *Lv;
  int32_t *Llen;
  const int64_t *Urp;
  int32_t *Uc;
  double *Uv;
  int32_t *Ulen;
  const int64_t *Rrp;
  int32_t *Rc;
  double *Rv;
  int32_t *Rlen;
  double *D;
  int *done;
  int epoch;
  Status *st;
};

__device__ inline int lower_bound_lds(const int32_t *a, int lo, int hi, int32_t key) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Keep-set of a part [b, e) of the working row: predicate p(e) and, for ILUT,
// the lfil largest magnitudes.  Writes kept entries in column order to
// (oc, ov) and returns their count.  extra_diag >= 0 marks an index that is
// always kept and does not count toward lfil.
__device__ int emit_part(const int32_t *wc, const double *wv, const uint8_t *wd, int b, int e, bool ilut,
                         double tau, int lfil, int always, int32_t *oc, double *ov, bool tau_drop) {
  const int lane = lane_id();
  // candidates: not dropped, and (tau_drop -> |w| >= tau); `always` is separate
  int ncand = 0;
  for (int base = b; base < e; base += WAVE) {
    int x = base + lane;
    bool c = x < e && x != always && !wd[x] && !(ilut && tau_drop && fabs(wv[x]) < tau);
    ncand += popc64(ballot(c));
  }
  const bool limit = ilut && lfil >= 0 && ncand > lfil;
  int out = 0;
  for (int base = b; base < e; base += WAVE) {
    int x = base + lane;
    bool keep = false;
    if (x < e) {
      if (x == always) {
        keep = true;
      } else {
        keep = !wd[x] && !(ilut && tau_drop && fabs(wv[x]) < tau);
        if (keep && limit) {
          const double m = fabs(wv[x]);
          const int32_t cx = wc[x];
          int rank = 0;
          for (int y = b; y < e; y++) {
            if (y == always || wd[y]) continue;
            const double my = fabs(wv[y]);
            if (tau_drop && my < tau) continue;
            if (my > m || (my == m && wc[y] < cx)) rank++;
          }
          keep = rank < lfil;
        }
      }
    }
    unsigned long long mk = ballot(keep);
    if (keep) {
      int at = out + mbcnt(mk);
      st_dev(oc + at, wc[x]);
      st_dev(ov + at, wv[x]);
    }
    out += popc64(mk);
  }
  return out;
}

// LDS working state of one wave
struct FactLds {
  int32_t *wc;
  double *wv;
  uint8_t *wd;
  int32_t *fins, *fcol;
  double *fval;
  uint8_t *ws;  // slot of each working entry's cached pivot row
  int32_t *cc;
  double *cv;
};

// Factor row r with one wave.  Returns false after recording an error (or
// when a wait gave up), true once the row is stored and its flag released.
__device__ __forceinline__ bool factor_row(const FactArgs &a, int64_t r, const FactLds &L) {
  int32_t *const wc = L.wc;
  double *const wv = L.wv;
  uint8_t *const wd = L.wd;
  int32_t *const fins = L.fins, *const fcol = L.fcol;
  double *const fval = L.fval;
  uint8_t *const ws = L.ws;
  int32_t *const cc = L.cc;
  double *const cv = L.cv;
  const int lane = lane_id();
  const bool ilut = a.method == ILU_FACT_ILUT;
  const bool milu = a.method == ILU_FACT_MILU0;
  const int64_t lim = r < a.nfull ? r : a.nfull;
  const int64_t rb = a.rp[r];
  int len = (int)(a.rp[r + 1] - rb);
  if (len > FACT_CAP) {
    if (lane == 0) raise_error(a.st, ILU_ERR_CAPACITY, r);
    return false;
  }
  for (int x = lane; x < len; x += WAVE) {
    wc[x] = a.ci[rb + x];
    wv[x] = a.v[rb + x];
    wd[x] = 0;
  }
  wave_sync();
  double tau = 0.0, rowinf = 0.0;
  if (ilut) {
    double s = 0.0;
    if (lane == 0)
      for (int x = 0; x < len; x++) s = fma(wv[x], wv[x], s);
    tau = uniform_f64(a.droptol * sqrt(__shfl(s, 0, WAVE)));
  }
  if (a.pivot_mode == ILU_PIVOT_PERTURB) {
    double m = 0.0;
    for (int x = lane; x < len; x += WAVE) m = fmax(m, fabs(wv[x]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, WAVE));
    rowinf = uniform_f64(m);
  }
  double drop = 0.0;  // MILU: dropped fill of this row, summed in (k, j) order (lane 0)
  bool failed = false;

  // the round's slot table in registers: lane s holds the diagonal, the
  // cache offset and the length of the U row cached in slot s
  double t_dk = 0.0;
  int t_off = 0, t_len = 0;
  bool first = true;
  for (int pos = 0;; pos++) {
    // every value that decides the control flow below is made wave-uniform
    const int32_t k = uniform_i32(pos < len ? wc[pos] : 0x7fffffff);
    if (k >= lim) break;
    // Dependencies are waited for in rounds: the lanes wait together for
    // every pivot still ahead in the working row.  A fill that becomes a
    // pivot later (marked by bit 1 of wd) starts the next round when it
    // is reached.  A pivot row's D, length and U row are then read with
    // device-scope loads: its wave wrote them with write-through stores
    // before releasing its flag, so no acquire fence (which would drop
    // this XCD's cached lines for every wave on it) is needed.
    //
    // The round also fetches, all in parallel, the diagonal and the U row
    // of the first WAVE pivots from pos on into an LDS cache (as many as
    // fit), and tags their working entries with the slot; a pivot left
    // out is marked like a new fill and starts the next round.  Every
    // round re-caches all pivots from its position on, so no slot of an
    // earlier round is read after being overwritten.
    if (first || uniform_i32((int)(wd[pos] & 2))) {
      first = false;
      // the pivot at pos is waited for; the pivots after it are taken as far
      // as they are already complete (one poll each), so a row eliminates its
      // early pivots while a later one is still being factored.  The poll and
      // the slot of each candidate's U row (start and capacity, fixed before
      // the launch) are read in one trip; the diagonal, the length and the
      // first FACT_UROW entries of the slot (those past the length are read
      // and ignored) in a second one.
      const int x = pos + lane;
      const int32_t kx0 = x < len ? wc[x] : 0x7fffffff;
      const bool cand = kx0 < lim;  // true on lane 0: kx0 == k
      int flag = 0, ucap = 0;
      int64_t ub = 0;
      if (cand) {
        flag = ld_relaxed(&a.done[kx0]);
        ub = a.Urp[kx0];
        ucap = (int)(a.Urp[kx0 + 1] - ub);
      }
      bool ok = true;
      if (lane == 0 && flag != a.epoch) ok = wait_flag_eq(&a.done[k], a.epoch, a.st, r);
      if (!uniform_i32((int)ok)) {
        failed = true;
        break;
      }
      const bool ready = cand && (x == pos || flag == a.epoch);
      const unsigned long long waiting = ballot(cand && !ready);
      const int nready = waiting ? __ffsll((long long)waiting) - 1 : WAVE;  // covered pivots: lanes [0, nready)
      const bool piv = cand && lane < nready;  // the covered pivots are a prefix of [pos, len)
      const int32_t kx = piv ? kx0 : 0;
      double dk = 0.0;
      int ul = 0;
      int32_t uc_[FACT_UROW];
      double uv_[FACT_UROW];
      if (piv) {
        dk = ld_dev(a.D + kx);
        ul = ld_dev(a.Ulen + kx);
#pragma unroll
        for (int q = 0; q < FACT_UROW; q++) {
          if (q < ucap) {
            uc_[q] = ld_dev(a.Uc + ub + q);
            uv_[q] = ld_dev(a.Uv + ub + q);
          }
        }
      }
      // exclusive prefix sum of the row lengths over the lanes
      int off = ul;
      for (int o = 1; o < WAVE; o <<= 1) {
        const int v = __shfl_up(off, o, WAVE);
        if (lane >= o) off += v;
      }
      off -= ul;
      const bool cached = piv && off + ul <= FACT_UCACHE;
#pragma unroll
      for (int q = 0; q < FACT_UROW; q++) {
        if (cached && q < ul) {
          cc[off + q] = uc_[q];
          cv[off + q] = uv_[q];
        }
      }
      // longer rows: the rest in batches of FACT_UTAIL loads per lane
      for (int q0 = FACT_UROW; ballot(cached && q0 < ul); q0 += FACT_UTAIL) {
        int32_t tc_[FACT_UTAIL];
        double tv_[FACT_UTAIL];
#pragma unroll
        for (int q = 0; q < FACT_UTAIL; q++) {
          if (cached && q0 + q < ul) {
            tc_[q] = ld_dev(a.Uc + ub + q0 + q);
            tv_[q] = ld_dev(a.Uv + ub + q0 + q);
          }
        }
#pragma unroll
        for (int q = 0; q < FACT_UTAIL; q++) {
          if (cached && q0 + q < ul) {
            cc[off + q0 + q] = tc_[q];
            cv[off + q0 + q] = tv_[q];
          }
        }
      }
      if (cached) {
        t_dk = dk;
        t_off = off;
        t_len = ul;
      }
      wave_sync();
      if (x < len) {
        if (cached) {
          ws[x] = (uint8_t)lane;
          wd[x] &= (uint8_t)~2u;
        } else if (kx0 < lim) {
          wd[x] |= 2;
        }
      }
      for (int y = pos + WAVE + lane; y < len; y += WAVE)
        if (wc[y] < lim) wd[y] |= 2;
      wave_sync();
    }
    // Only lane 0 writes wv[pos] and wd[pos] below, and nothing before the
    // row is stored reads them again (lookups and shifts start at pos + 1);
    // the wave's LDS operations execute in order, so no wait is needed.
    const int slot = uniform_i32((int)ws[pos]);
    const double wk = uniform_f64(wv[pos] / readlane_f64(t_dk, slot));
    if (ilut && fabs(wk) < tau) {
      if (lane == 0) {
        wv[pos] = 0.0;
        wd[pos] = 1;
      }
      continue;
    }
    if (lane == 0) wv[pos] = wk;
    const int ub = __builtin_amdgcn_readlane(t_off, slot);
    const int ul = __builtin_amdgcn_readlane(t_len, slot);
    for (int base = 0; base < ul; base += WAVE) {
      const int j = base + lane;
      const bool have = j < ul;
      const int32_t c = have ? cc[ub + j] : 0x7fffffff;
      const double u = have ? cv[ub + j] : 0.0;
      const int idx = have ? lower_bound_lds(wc, pos + 1, len, c) : len;
      const bool found = have && idx < len && wc[idx] == c;
      if (found) wv[idx] = fma(-wk, u, wv[idx]);
      const bool fill = have && !found;
      const unsigned long long fm = ballot(fill);
      if (fm == 0ull) {
        wave_sync();
        continue;
      }
      if (ilut) {
        const int nf = popc64(fm);
        if (len + nf > FACT_CAP) {
          if (lane == 0) raise_error(a.st, ILU_ERR_CAPACITY, r);
          return false;
        }
        if (fill) {
          const int rk = mbcnt(fm);
          fins[rk] = idx;
          fcol[rk] = c;
          fval[rk] = fma(-wk, u, 0.0);
        }
        wave_sync();
        // Shift every working entry after the pivot to make room: the
        // upper half of the slots first, each half read completely before
        // it is written (destinations only move up and never cross).
        constexpr int NS = FACT_CAP / WAVE, HS = NS / 2;
#pragma unroll 1
        for (int h = 1; h >= 0; h--) {
          int32_t rc_[HS];
          double rv_[HS];
          uint8_t rd_[HS], rs_[HS];
          int np_[HS];
#pragma unroll
          for (int qq = 0; qq < HS; qq++) {
            const int x = pos + 1 + (h * HS + qq) * WAVE + lane;
            np_[qq] = -1;
            if (x < len) {
              rc_[qq] = wc[x];
              rv_[qq] = wv[x];
              rd_[qq] = wd[x];
              rs_[qq] = ws[x];
              // number of fills inserted at or before x
              int lo = 0, hi = nf;
              while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (fins[mid] <= x)
                  lo = mid + 1;
                else
                  hi = mid;
              }
              np_[qq] = x + lo;
            }
          }
          wave_sync();
#pragma unroll
          for (int qq = 0; qq < HS; qq++) {
            if (np_[qq] >= 0) {
              wc[np_[qq]] = rc_[qq];
              wv[np_[qq]] = rv_[qq];
              wd[np_[qq]] = rd_[qq];
              ws[np_[qq]] = rs_[qq];
            }
          }
          wave_sync();
        }
        if (lane < nf) {
          const int at = fins[lane] + lane;
          wc[at] = fcol[lane];
          wv[at] = fval[lane];
          wd[at] = fcol[lane] < lim ? 2 : 0;  // a new pivot: not covered by the last round
        }
        len += nf;
        wave_sync();
      } else if (milu) {
        // sum the dropped products in column order, exactly as written
        unsigned long long m = fm;
        while (m) {
          const int b = __ffsll((long long)m) - 1;
          m &= m - 1;
          const double ubv = __shfl(u, b, WAVE);
          if (lane == 0) drop = fma(-wk, ubv, drop);
        }
        wave_sync();
      } else {
        wave_sync();
      }
    }
  }
  if (failed) return false;
  wave_sync();

  if (r < a.nfull) {  // full row: L | d | U
    const int pd = uniform_i32(lower_bound_lds(wc, 0, len, (int32_t)r));
    double d = wv[pd];
    if (milu) d = d + __shfl(drop, 0, WAVE);
    d = uniform_f64(d);
    if (a.pivot_mode == ILU_PIVOT_PERTURB) {
      const double thr = a.pivot_tol * rowinf;
      if (fabs(d) < thr) d = (d < 0.0) ? -thr : thr;
    }
    if (d == 0.0 || !isfinite(d)) {
      if (lane == 0) raise_error(a.st, ILU_ERR_ZERO_PIVOT, r);
      return false;
    }
    if (lane == 0) st_dev(a.D + r, d);
    const int nl = emit_part(wc, wv, wd, 0, pd, ilut, tau, a.lfil, -1, a.Lc + a.Lrp[r], a.Lv + a.Lrp[r], false);
    const int nu =
        emit_part(wc, wv, wd, pd + 1, len, ilut, tau, a.lfil, -1, a.Uc + a.Urp[r], a.Uv + a.Urp[r], true);
    if (lane == 0) {
      st_dev(a.Llen + r, nl);
      st_dev(a.Ulen + r, nu);
    }
  } else {  // partial row: L (interior columns) | Schur remainder R
    const int pl = uniform_i32(lower_bound_lds(wc, 0, len, (int32_t)a.nfull));
    const int pd = uniform_i32(lower_bound_lds(wc, pl, len, (int32_t)r));
    if (milu) {
      wave_sync();
      if (lane == 0) wv[pd] = wv[pd] + drop;
      wave_sync();
    }
    const int nl = emit_part(wc, wv, wd, 0, pl, ilut, tau, a.lfil, -1, a.Lc + a.Lrp[r], a.Lv + a.Lrp[r], false);
    const int64_t ro = a.Rrp[r - a.nfull];
    const int nr = emit_part(wc, wv, wd, pl, len, ilut, tau, a.lfil, pd, a.Rc + ro, a.Rv + ro, true);
    if (lane == 0) {
      st_dev(a.Llen + r, nl);
      st_dev(a.Rlen + (r - a.nfull), nr);
    }
  }
  wave_sync();
  if (lane == 0) st_release(&a.done[r], a.epoch);
  wave_sync();
  return true;
}

// A workgroup of FACT_WAVES waves takes a chunk of rows at a time; wave w
// factors rows first + w, first + w + FACT_WAVES, ...: a row's early pivots
// (rows finished long before) are eliminated while the row before it is still
// in progress on another wave.  The waves of a chunk are resident together,
// so the waits between them always end.
__global__ void __launch_bounds__(WAVE *FACT_WAVES, 2) k_factor_rows(FactArgs a) {
  __shared__ int32_t wc[FACT_WAVES][FACT_CAP];
  __shared__ double wv[FACT_WAVES][FACT_CAP];
  __shared__ uint8_t wd[FACT_WAVES][FACT_CAP];
  __shared__ int32_t fins[FACT_WAVES][WAVE];
  __shared__ int32_t fcol[FACT_WAVES][WAVE];
  __shared__ double fval[FACT_WAVES][WAVE];
  __shared__ uint8_t ws[FACT_WAVES][FACT_CAP];
  __shared__ int32_t cc[FACT_WAVES][FACT_UCACHE];
  __shared__ double cv[FACT_WAVES][FACT_UCACHE];
  __shared__ long long sh_t;
  const int w = (int)(threadIdx.x / WAVE);
  const FactLds L{wc[w], wv[w], wd[w], fins[w], fcol[w], fval[w], ws[w], cc[w], cv[w]};

  int64_t sid = (int64_t)blockIdx.x % a.ninit;
  for (;;) {
    __syncthreads();  // every wave is done with the previous chunk
    if (w == 0) {
      // A stream is left only once it has handed out all its chunks, so every
      // stream keeps a workgroup until then; a stream that no row depends on
      // (interface rows of a partial factorization) may start without one.
      int64_t t = -1;
      for (int64_t tries = 0; tries < a.nstreams && t < 0; tries++) {
        const int64_t c0 = a.stream_chunk[sid], nc = a.stream_chunk[sid + 1] - c0;
        if ((int64_t)uniform_i32(ld_relaxed(reinterpret_cast<const int *>(a.ticket + sid))) < nc) {
          const unsigned int tl = wave_ticket(a.ticket + sid);
          if ((int64_t)tl < nc) t = c0 + (int64_t)tl;
        }
        if (t < 0) sid = sid + 1 < a.nstreams ? sid + 1 : 0;
      }
      if (ld_relaxed(&a.st->abort)) t = -1;
      if (threadIdx.x == 0) sh_t = t;
    }
    __syncthreads();
    const int64_t t = sh_t;
    if (t < 0) return;
    const int2 ch = a.chunks[t];
    for (int64_t r = ch.x + w; r < (int64_t)ch.x + ch.y; r += FACT_WAVES)
      if (!factor_row(a, r, L)) break;
  }
}

// ---------------------------------------------------------------------------
// capacities of the per-row output slots
// ---------------------------------------------------------------------------
__global__ void k_fact_caps(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nfull, int32_t method,
                            int32_t lfil, int64_t *Lcap, int64_t *Ucap, int64_t *Rcap) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t lim = r < nfull ? r : nfull;
  int64_t cl = 0, cu = 0, cr = 0;
  if (method == ILU_FACT_ILUT) {
    cl = lfil >= 0 ? (lfil < lim ? lfil : lim) : lim;
    if (r < nfull) {
      const int64_t hi = n - r - 1;
      cu = lfil >= 0 ? (lfil < hi ? lfil : hi) : hi;
    } else {
      const int64_t hi = n - nfull - 1;
      cr = (lfil >= 0 ? (lfil < hi ? lfil : hi) : hi) + 1;
    }
  } else {
    for (int64_t p = rp[r]; p < rp[r + 1]; p++) {
      const int64_t c = ci[p];
      if (c < lim)
        cl++;
      else if (r < nfull && c > r)
        cu++;
      else if (r >= nfull)
        cr++;
    }
  }
  Lcap[r] = cl;
  if (r < nfull)
    Ucap[r] = cu;
  else
    Rcap[r - nfull] = cr;
}

// compaction of per-row slots into CSR (one thread per row)
__global__ void k_compact_rows(int64_t nrows, const int64_t *cap_rp, const int32_t *len, const int32_t *sc,
                               const double *sv, const int64_t *out_rp, int32_t *oc, double *ov, int64_t col_lo,
                               int64_t col_hi, int64_t shift) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int64_t b = cap_rp[r];
  int64_t o = out_rp[r];
  for (int64_t p = b; p < b + len[r]; p++) {
    const int64_t c = sc[p];
    if (c >= col_lo && c < col_hi) {
      oc[o] = (int32_t)(c - shift);
      ov[o] = sv[p];
      o++;
    }
  }
}

__global__ void k_count_rows(int64_t nrows, const int64_t *cap_rp, const int32_t *len, const int32_t *sc,
                             int64_t col_lo, int64_t col_hi, int64_t *cnt) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const int64_t b = cap_rp[r];
  int64_t k = 0;
  for (int64_t p = b; p < b + len[r]; p++) {
    const int64_t c = sc[p];
    k += (c >= col_lo && c < col_hi);
  }
  cnt[r] = k;
}

}  // namespace silu

// ---------------------------------------------------------------------------
// host launchers (called from the runtime)
// ---------------------------------------------------------------------------

namespace silu {

int launch_fact_caps(const int64_t *rp, const int32_t *ci, int64_t n, int64_t nfull, int32_t method, int32_t lfil,
                     int64_t *Lcap, int64_t *Ucap, int64_t *Rcap, hipStream_t s) {
  if (n == 0) return 0;
  k_fact_caps<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, n, nfull, method, lfil, Lcap, Ucap, Rcap);
  return check_launch("fact_caps");
}

// ILU(0) / MILU(0), one level of the lower pattern (over the interior
// columns) per launch: every pivot row of a level lies in an earlier level, so it is complete
// when the launch starts, and no row waits.  One thread per row.  The
// operations are factor_row's, in its order: pivots in column order,
// w_k / d_k, one fma per updated entry, the dropped products of MILU(0)
// summed in (pivot, column) order, the same pivot test.  So the factors are
// identical to the dependency-flag kernel's, without its per-row round
// trips.  A row of at most FL_ROW entries is held in registers, the
// diagonals and U-row extents of all its pivots are fetched in one round,
// and each pivot's U row (at most FL_U entries) in one more; longer rows
// work in their output slots in memory instead.
constexpr int FL_ROW = 12;
constexpr int FL_U = 12;

// the general row: working in the output slots (L entries in column order,
// then U), any length
__device__ void factor_level_row_mem(const FactLaunch &f, int64_t r) {
  const bool milu = f.method == ILU_FACT_MILU0;
  const int64_t rb = f.rp[r], re = f.rp[r + 1], lb = f.Lrp[r], ub = f.Urp[r];
  int nl = 0, nu = 0;
  double d = 0.0, rowinf = 0.0;
  for (int64_t e = rb; e < re; e++) {
    const int32_t c = f.ci[e];
    const double x = f.v[e];
    rowinf = fmax(rowinf, fabs(x));
    if (c < r) {
      f.Lc[lb + nl] = c;
      f.Lv[lb + nl] = x;
      nl++;
    } else if (c == r) {
      d = x;
    } else {
      f.Uc[ub + nu] = c;
      f.Uv[ub + nu] = x;
      nu++;
    }
  }
  double drop = 0.0;
  for (int p = 0; p < nl; p++) {
    const int32_t k = f.Lc[lb + p];
    const double wk = f.Lv[lb + p] / f.D[k];
    f.Lv[lb + p] = wk;
    // row k's U entries (ascending) against this row's entries after column
    // k (ascending): the L entries after p, the diagonal, the U entries
    const int64_t kb = f.Urp[k];
    const int kl = f.Ulen[k];
    int q = p + 1;  // L entry q (< nl), the diagonal (q == nl), U entry q - nl - 1
    for (int t = 0; t < kl; t++) {
      const int32_t uc = f.Uc[kb + t];
      const double u = f.Uv[kb + t];
      int32_t cq;
      for (;;) {
        cq = q < nl ? f.Lc[lb + q] : q == nl ? (int32_t)r : q - nl - 1 < nu ? f.Uc[ub + q - nl - 1] : INT32_MAX;
        if (cq >= uc) break;
        q++;
      }
      if (cq == uc) {
        if (q < nl)
          f.Lv[lb + q] = fma(-wk, u, f.Lv[lb + q]);
        else if (q == nl)
          d = fma(-wk, u, d);
        else
          f.Uv[ub + q - nl - 1] = fma(-wk, u, f.Uv[ub + q - nl - 1]);
      } else if (milu) {
        drop = fma(-wk, u, drop);
      }
    }
  }
  if (milu) d = d + drop;
  if (f.pivot_mode == ILU_PIVOT_PERTURB) {
    const double thr = f.pivot_tol * rowinf;
    if (fabs(d) < thr) d = (d < 0.0) ? -thr : thr;
  }
  if (d == 0.0 || !isfinite(d)) {
    raise_error(static_cast<Status *>(f.status), ILU_ERR_ZERO_PIVOT, r);
    return;
  }
  f.D[r] = d;
  f.Llen[r] = nl;
  f.Ulen[r] = nu;
}

// A partial row (r >= nfull, a row of the local Schur complement), in
// memory: eliminated by its interior pivots (columns < nfull) only, as
// factor_row does, into its L entries (interior columns) and its remainder
// R (columns >= nfull, the diagonal among them; with MILU(0) the dropped
// products are added to the diagonal).  No pivot test: R is not a pivot.
__device__ void factor_level_partial_mem(const FactLaunch &f, int64_t r) {
  const bool milu = f.method == ILU_FACT_MILU0;
  const int64_t rb = f.rp[r], re = f.rp[r + 1], lb = f.Lrp[r], ro = f.Rrp[r - f.nfull];
  int nl = 0, nr = 0;
  for (int64_t e = rb; e < re; e++) {
    const int32_t c = f.ci[e];
    const double x = f.v[e];
    if (c < f.nfull) {
      f.Lc[lb + nl] = c;
      f.Lv[lb + nl] = x;
      nl++;
    } else {
      f.Rc[ro + nr] = c;
      f.Rv[ro + nr] = x;
      nr++;
    }
  }
  double drop = 0.0;
  for (int p = 0; p < nl; p++) {
    const int32_t k = f.Lc[lb + p];
    const double wk = f.Lv[lb + p] / f.D[k];
    f.Lv[lb + p] = wk;
    const int64_t kb = f.Urp[k];
    const int kl = f.Ulen[k];
    int q = p + 1;  // L entry q (< nl), else R entry q - nl
    for (int t = 0; t < kl; t++) {
      const int32_t uc = f.Uc[kb + t];
      const double u = f.Uv[kb + t];
      int32_t cq;
      for (;;) {
        cq = q < nl ? f.Lc[lb + q] : q - nl < nr ? f.Rc[ro + q - nl] : INT32_MAX;
        if (cq >= uc) break;
        q++;
      }
      if (cq == uc) {
        if (q < nl)
          f.Lv[lb + q] = fma(-wk, u, f.Lv[lb + q]);
        else
          f.Rv[ro + q - nl] = fma(-wk, u, f.Rv[ro + q - nl]);
      } else if (milu) {
        drop = fma(-wk, u, drop);
      }
    }
  }
  if (milu)
    for (int q = 0; q < nr; q++)
      if (f.Rc[ro + q] == r) f.Rv[ro + q] = f.Rv[ro + q] + drop;
  f.Llen[r] = nl;
  f.Rlen[r - f.nfull] = nr;
}

__global__ void __launch_bounds__(128) k_factor_level(FactLaunch f, const int32_t *rows, int64_t cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int64_t r = rows[i];
  const int64_t rb = f.rp[r];
  const int len = (int)(f.rp[r + 1] - rb);
  // a partial row's pivots are its interior columns, a full row's those below it
  const bool part = r >= f.nfull;
  const int64_t lim = part ? f.nfull : r;
  if (len > FL_ROW) {
    if (part)
      factor_level_partial_mem(f, r);
    else
      factor_level_row_mem(f, r);
    return;
  }
  const bool milu = f.method == ILU_FACT_MILU0;
  // the row, in column order, in registers
  int32_t c[FL_ROW];
  double w[FL_ROW];
#pragma unroll
  for (int e = 0; e < FL_ROW; e++) {
    c[e] = e < len ? f.ci[rb + e] : INT32_MAX;
    w[e] = e < len ? f.v[rb + e] : 0.0;
  }
  double rowinf = 0.0;
  int nl = 0;
#pragma unroll
  for (int e = 0; e < FL_ROW; e++) {
    rowinf = fmax(rowinf, fabs(w[e]));
    nl += c[e] < lim;
  }
  // every pivot's diagonal and U-row extent in one round
  double dk[FL_ROW];
  int64_t kb[FL_ROW];
  int kl[FL_ROW];
#pragma unroll
  for (int e = 0; e < FL_ROW; e++) {
    const bool piv = e < nl;
    const int32_t k = piv ? c[e] : 0;
    dk[e] = piv ? f.D[k] : 1.0;
    kb[e] = piv ? f.Urp[k] : 0;
    kl[e] = piv ? f.Ulen[k] : 0;
  }
  bool fits = true;
#pragma unroll
  for (int e = 0; e < FL_ROW; e++) fits = fits && kl[e] <= FL_U;
  if (!fits) {
    if (part)
      factor_level_partial_mem(f, r);
    else
      factor_level_row_mem(f, r);
    return;
  }
  double drop = 0.0;
#pragma unroll
  for (int p = 0; p < FL_ROW; p++) {
    if (p < nl) {
      int32_t uc[FL_U];
      double uv[FL_U];
#pragma unroll
      for (int t = 0; t < FL_U; t++) {
        uc[t] = t < kl[p] ? f.Uc[kb[p] + t] : INT32_MAX;
        uv[t] = t < kl[p] ? f.Uv[kb[p] + t] : 0.0;
      }
      const double wk = w[p] / dk[p];
      w[p] = wk;
      // each U entry (in column order) updates the row entry of its column,
      // or is a dropped fill
#pragma unroll
      for (int t = 0; t < FL_U; t++) {
        if (t < kl[p]) {
          bool hit = false;
#pragma unroll
          for (int e = 0; e < FL_ROW; e++) {
            if (e > p && c[e] == uc[t]) {
              w[e] = fma(-wk, uv[t], w[e]);
              hit = true;
            }
          }
          if (!hit && milu) drop = fma(-wk, uv[t], drop);
        }
      }
    }
  }
  if (part) {
    const int64_t lb = f.Lrp[r], ro = f.Rrp[r - f.nfull];
#pragma unroll
    for (int e = 0; e < FL_ROW; e++) {
      if (milu && c[e] == r) w[e] = w[e] + drop;
      if (e < nl) {
        f.Lc[lb + e] = c[e];
        f.Lv[lb + e] = w[e];
      } else if (e < len) {
        f.Rc[ro + e - nl] = c[e];
        f.Rv[ro + e - nl] = w[e];
      }
    }
    f.Llen[r] = nl;
    f.Rlen[r - f.nfull] = len - nl;
    return;
  }
  double d = 0.0;
#pragma unroll
  for (int e = 0; e < FL_ROW; e++)
    if (c[e] == r) d = w[e];
  if (milu) d = d + drop;
  if (f.pivot_mode == ILU_PIVOT_PERTURB) {
    const double thr = f.pivot_tol * rowinf;
    if (fabs(d) < thr) d = (d < 0.0) ? -thr : thr;
  }
  if (d == 0.0 || !isfinite(d)) {
    raise_error(static_cast<Status *>(f.status), ILU_ERR_ZERO_PIVOT, r);
    return;
  }
  const int64_t lb = f.Lrp[r], ub = f.Urp[r];
  int nu = 0;
#pragma unroll
  for (int e = 0; e < FL_ROW; e++) {
    if (e < nl) {
      f.Lc[lb + e] = c[e];
      f.Lv[lb + e] = w[e];
    } else if (e < len && c[e] > r) {
      f.Uc[ub + nu] = c[e];
      f.Uv[ub + nu] = w[e];
      nu++;
    }
  }
  f.D[r] = d;
  f.Llen[r] = nl;
  f.Ulen[r] = nu;
}

int launch_factor_level(const FactLaunch &f, const int32_t *rows, int64_t cnt, hipStream_t s) {
  if (cnt == 0) return 0;
  k_factor_level<<<(unsigned)((cnt + 127) / 128), 128, 0, s>>>(f, rows, cnt);
  return check_launch("factor_level");
}

// longest row of rows [0, n)
__global__ void k_row_len_max(const int64_t *rp, int64_t n, int *out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int len = r < n ? (int)(rp[r + 1] - rp[r]) : 0;
  len = wave_max_int(len);
  if (lane_id() == 0) atomicMax(out, len);
}

int launch_row_len_max(const int64_t *rp, int64_t n, int *out, hipStream_t s) {
  if (n == 0) return 0;
  k_row_len_max<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, n, out);
  return check_launch("row_len_max");
}

int launch_factor_rows(const FactLaunch &f, hipStream_t s) {
  FactArgs a;
  a.rp = f.rp;
  a.ci = f.ci;
  a.v = f.v;
  a.n = f.n;
  a.nfull = f.nfull;
  a.method = f.method;
  a.droptol = f.droptol;
  a.lfil = f.lfil;
  a.pivot_mode = f.pivot_mode;
  a.pivot_tol = f.pivot_tol;
  a.nchunks = f.nchunks;
  a.chunks = reinterpret_cast<const int2 *>(f.chunks);
  a.nstreams = f.nstreams;
  a.ninit = f.ninit;
  a.stream_chunk = f.stream_chunk;
  a.ticket = f.ticket;
  a.Lrp = f.Lrp;
  a.Lc = f.Lc;
  a.Lv = f.Lv;
  a.Llen = f.Llen;
  a.Urp = f.Urp;
  a.Uc = f.Uc;
  a.Uv = f.Uv;
  a.Ulen = f.Ulen;
  a.Rrp = f.Rrp;
  a.Rc = f.Rc;
  a.Rv = f.Rv;
  a.Rlen = f.Rlen;
  a.D = f.D;
  a.done = f.done;
  a.epoch = f.epoch;
  a.st = (Status *)f.status;
  if (f.nchunks == 0) return 0;
  // Every stream needs a workgroup that runs (a stream's rows may wait on an
  // earlier stream of the same segment, never on a later one): the grid is
  // launched cooperatively, which guarantees that all its workgroups are
  // resident at once, and has at least one workgroup per stream.
  if (f.grid < f.ninit || f.ninit < 1 || f.ninit > f.nstreams) return ILU_ERR_INVALID_ARG;
  void *args[] = {&a};
  const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_factor_rows),
                                                  dim3((unsigned)f.grid), dim3(WAVE * FACT_WAVES), args, 0, s);
  if (e != hipSuccess) return ILU_ERR_HIP;
  return check_launch("factor_rows");
}

// Workgroups of k_factor_rows that fit on the device at once.
int factor_resident_groups(int num_cu) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_factor_rows, WAVE * FACT_WAVES, 0) != hipSuccess)
    return 0;
  return per_cu * num_cu;
}

// Histograms of log2 of each row's distance to its second-nearest lower
// neighbour (i - max{j < i - 1 : a_ij != 0}) and to its farthest one
// (i - min{j < i - 1}); with `upper`, of the mirrored distances to upper
// neighbours (min{j > i + 1} - i and max{j > i + 1} - i).  In a natural
// ordering of a grid the dominant values are the length of a line and of a
// plane: consecutive rows along a line depend on one another, and a plane
// depends on the plane before it.
__global__ void k_gap_hist(const int64_t *rp, const int32_t *ci, int64_t n, bool upper, unsigned long long *hist) {
  __shared__ unsigned long long h[64];
  if (threadIdx.x < 64) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    int64_t near = -1, far = -1;
    for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
      const int64_t d = upper ? (int64_t)ci[p] - i : i - (int64_t)ci[p];
      if (d > 1) {
        if (near < 0 || d < near) near = d;
        if (d > far) far = d;
      }
    }
    if (near > 0) {
      atomicAdd(&h[63 - __clzll((long long)near)], 1ull);
      atomicAdd(&h[32 + 63 - __clzll((long long)far)], 1ull);
    }
  }
  __syncthreads();
  if (threadIdx.x < 64 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

int launch_gap_hist(const int64_t *rp, const int32_t *ci, int64_t n, bool upper, unsigned long long *hist,
                    hipStream_t s) {
  if (n == 0) return 0;
  k_gap_hist<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rp, ci, n, upper, hist);
  return check_launch("gap_hist");
}

int launch_compact_rows(int64_t nrows, const int64_t *cap_rp, const int32_t *len, const int32_t *sc,
                        const double *sv, const int64_t *out_rp, int32_t *oc, double *ov, int64_t col_lo,
                        int64_t col_hi, int64_t shift, hipStream_t s) {
  if (nrows == 0) return 0;
  k_compact_rows<<<(unsigned)((nrows + 255) / 256), 256, 0, s>>>(nrows, cap_rp, len, sc, sv, out_rp, oc, ov, col_lo,
                                                                  col_hi, shift);
  return check_launch("compact_rows");
}

int launch_count_rows(int64_t nrows, const int64_t *cap_rp, const int32_t *len, const int32_t *sc, int64_t col_lo,
                      int64_t col_hi, int64_t *cnt, hipStream_t s) {
  if (nrows == 0) return 0;
  k_count_rows<<<(unsigned)((nrows + 255) / 256), 256, 0, s>>>(nrows, cap_rp, len, sc, col_lo, col_hi, cnt);
  return check_launch("count_rows");
}

}  // namespace silu
