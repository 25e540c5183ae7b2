// capi.cpp -- runtime and C ABI of libschurilu (see include/schurilu.h).
//
// The host side only sequences kernels, owns device memory and reads back a
// handful of scalars (sizes during setup, the residual estimate once per
// outer Krylov step).  Every arithmetic step of setup and solve runs in the
// gfx950 kernels of factor.hip, levels.hip, trsv.hip, krylov.hip, setup.hip
// and prims.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "launch.hpp"

using namespace silu;

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

namespace silu {
int api_fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
}  // namespace silu

int silu_hip_fail(hipError_t e, int line) {
  return fail(ILU_ERR_HIP, "HIP error '%s' (capi.cpp:%d)", hipGetErrorString(e), line);
}

namespace silu {
int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ILU_ERR_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
  return 0;
}
}  // namespace silu

#define HIPCK(x)                                        \
  do {                                                  \
    hipError_t _e = (x);                                \
    if (_e != hipSuccess) return silu_hip_fail(_e, __LINE__); \
  } while (0)
#define RC(x)                   \
  do {                          \
    int _r = (x);               \
    if (_r) return _r;          \
  } while (0)

// ---------------------------------------------------------------------------
// device memory owner
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Device memory cache.  hipFree synchronises the device and both it and
// hipMalloc cost tens of microseconds per call, so freed blocks are kept per
// device and handed out again to requests of at most their size and at
// least half of it (repeated setups of one problem reuse them all).  Blocks
// are returned only after the device has finished with them (Mem::release
// synchronises first).  A failed hipMalloc empties the cache and retries;
// ilu_memory_trim empties it on request.
// ---------------------------------------------------------------------------
namespace {
struct MemCache {
  std::mutex mu;
  std::multimap<std::pair<int, size_t>, void *> free_;     // (device, size) -> block
  std::unordered_map<void *, std::pair<int, size_t>> own;  // every block handed out or cached
};
MemCache &mem_cache() {
  static MemCache *c = new MemCache();  // never destroyed: blocks may outlive static destructors
  return *c;
}
size_t cache_round(size_t b) {
  const size_t g = b <= ((size_t)1 << 20) ? 256 : ((size_t)2 << 20);
  return (b + g - 1) / g * g;
}
void cache_trim() {
  MemCache &c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto &kv : c.free_) {
    (void)hipSetDevice(kv.first.first);
    (void)hipFree(kv.second);
    c.own.erase(kv.second);
  }
  c.free_.clear();
  (void)hipSetDevice(cur);
}
hipError_t cache_alloc(void **p, size_t bytes) {
  MemCache &c = mem_cache();
  int dev = 0;
  (void)hipGetDevice(&dev);
  const size_t want = cache_round(bytes);
  {
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.free_.lower_bound({dev, want});
    if (it != c.free_.end() && it->first.first == dev && it->first.second <= 2 * want) {
      *p = it->second;
      c.free_.erase(it);
      return hipSuccess;
    }
  }
  hipError_t e = hipMalloc(p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    cache_trim();
    e = hipMalloc(p, want);
  }
  if (e == hipSuccess) {
    std::lock_guard<std::mutex> lk(c.mu);
    c.own[*p] = {dev, want};
  }
  return e;
}
void cache_free(void *p) {
  MemCache &c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.own.find(p);
  if (it == c.own.end()) return;
  c.free_.emplace(it->second, p);
}
}  // namespace

struct Mem {
  std::vector<void *> ptrs;
  size_t bytes = 0;  // requested bytes of the blocks held
  ~Mem() { release(); }
  // sync = false: the owner has already waited for every stream that used
  // these blocks, so the device-wide wait (which would also wait for other
  // streams' unrelated work) is skipped
  void release(bool sync = true) {
    if (ptrs.empty()) return;
    if (sync) (void)hipDeviceSynchronize();  // kernels queued on these blocks have finished
    for (void *p : ptrs) cache_free(p);
    ptrs.clear();
    bytes = 0;
  }
  template <typename T>
  int alloc(T **out, int64_t count) {
    *out = nullptr;
    size_t nb = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    void *p = nullptr;
    hipError_t e = cache_alloc(&p, nb);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(ILU_ERR_OOM, "device allocation of %zu bytes failed: %s", nb, hipGetErrorString(e));
    }
    ptrs.push_back(p);
    bytes += nb;
    *out = (T *)p;
    return 0;
  }
  // take over every block of `from` (which is left empty)
  void adopt(Mem &from) {
    ptrs.insert(ptrs.end(), from.ptrs.begin(), from.ptrs.end());
    bytes += from.bytes;
    from.ptrs.clear();
    from.bytes = 0;
  }
};

// ---------------------------------------------------------------------------
// kernel timing: HIP events around each launch of the solve-phase kernels,
// resolved at host synchronisation points (profiling aid; process-global)
// ---------------------------------------------------------------------------
struct KStat {
  double ms = 0.0, bytes = 0.0;
  int64_t launches = 0;
};
struct PendingTiming {
  hipEvent_t a, b;
  int kind;
  double bytes;
};
static uint32_t g_timing = 0;  // bit k: kernel class k is timed
static KStat g_kstat[ILU_K_COUNT];
static std::vector<PendingTiming> g_pending;
static std::vector<hipEvent_t> g_event_pool;

static hipEvent_t pool_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static void timing_collect() {
  for (auto &p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_kstat[p.kind].ms += ms;
      g_kstat[p.kind].bytes += p.bytes;
      g_kstat[p.kind].launches++;
    }
    g_event_pool.push_back(p.a);
    g_event_pool.push_back(p.b);
  }
  g_pending.clear();
}

template <typename F>
static int timed(int kind, double bytes, hipStream_t s, F &&launch) {
  if (!((g_timing >> kind) & 1u)) return launch();
  hipEvent_t a = pool_event(), b = pool_event();
  if (!a || !b) return launch();
  (void)hipEventRecord(a, s);
  int rc = launch();
  (void)hipEventRecord(b, s);
  g_pending.push_back({a, b, kind, bytes});
  if (g_pending.size() > 4096) timing_collect();
  return rc;
}

struct Csr {
  int64_t n = 0, nnz = 0;
  int64_t *rp = nullptr;
  int32_t *ci = nullptr;
  double *v = nullptr;
};

struct Schedule {
  int64_t nrows = 0, nlev = 0, nchunks = 0;
  int32_t *rows = nullptr, *chunk_start = nullptr, *chunk_level = nullptr, *level_of = nullptr;
  int64_t *level_ptr = nullptr;
  unsigned long long *level_done = nullptr, *ticket = nullptr;
  unsigned long long epoch = 0, ticket_base = 0;
  int64_t grid = 0;
  // block-local variant: one workgroup per subdomain
  bool block_ok = false;  // levels and blocks fit the block-local solve
  bool use_block = false;
  int64_t nblk = 0;
  int32_t *blk_rows = nullptr, *blk_lev_ptr = nullptr;
  int32_t *pos = nullptr;            // row -> position (inverse of blk_rows)
  const int32_t *out_map = nullptr;  // row -> index of its solution in the output vector
  // storage of the factor for the block-local solve (values in the storage
  // precision)
  uint16_t *lds_c = nullptr;
  int32_t *lds_rec = nullptr;
  void *lds_v = nullptr;
  // level-scheduled solve with factors stored in FP32 / FP16: the values, the
  // FP32 diagonal and (FP16) the row scales
  void *v_lp = nullptr;
  float *diag_lp = nullptr, *scale_lp = nullptr;
  int32_t lds_g = 1, lds_e = 4, lds_bt = 64;
  bool lds_fast = false;  // no slow row and no level wider than the workgroup
  int64_t ext_col = 0;  // dependency columns of the block-local solve are < ext_col
  int64_t nloc = 0;     // rows in the block-local solve (the rows of W follow in their own pass)
  // each block split over split_k workgroups (nblk counts the parts): the
  // exchange slots, the exports ({position, slot}) and imports by (part,
  // level), their number and the start-order ticket
  int32_t split_k = 1;
  double *xv = nullptr;
  int32_t *xe = nullptr, *elp = nullptr, *ilp = nullptr, *lrange = nullptr;
  int64_t xlevels = 0;  // the most levels of any part
  int64_t nimp = 0;
  unsigned long long *xticket = nullptr;
};

// Buffers of one FGMRES(m) process on vectors of length n.  With the two
// events the host reads each step's residual estimate one step late (the
// read-back overlaps the next step); without them it reads it synchronously.
struct KrylovBufs {
  int64_t n = 0;
  int m = 0;
  double *V = nullptr, *Zb = nullptr, *r = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr,
         *c = nullptr, *pa = nullptr, *pb = nullptr, *scal = nullptr;  // scal: [0] bnorm [1] beta [2] hn [3] est
  int *flags = nullptr;                                                // [0] stop [1] nsteps
  // one-launch orthogonalisation: its sum slots (arnoldi_slots(m) words) and
  // the launches since they were reset
  unsigned long long *aslots = nullptr;
  unsigned long long alaunch = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};  // read-backs of two consecutive steps
};

struct GmresWork : KrylovBufs {
  Mem mem;
  ~GmresWork() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

struct ilu_precond {
  int device = 0;
  int64_t n = 0, nB = 0, nS = 0;
  int32_t nparts = 1;
  ilu_options_t opt;
  int num_cu = 256;
  Mem mem;
  int32_t *perm = nullptr, *iperm = nullptr;
  uint8_t *iface = nullptr;
  std::vector<int64_t> offsets;  // 2*nparts+2
  Csr L1, U1, LS, US, Coff, Zb;
  double *DB = nullptr, *DS = nullptr;
  Schedule sL1, sU1, sLS, sUS;
  double *xp = nullptr;
  // Block-local solves (all four or none).  Each solve reads its right-hand
  // side in its own position order and writes its solution contiguously:
  // L_B into bL -> fL (L_B order), the W rows into gS (L_S order), L_S into
  // the U_S order, U_S in place; the reduced-system vectors live in U_S order;
  // U_B takes bU (U_B order, f' - Z y) into uU; k_finish scatters uU and yS.
  bool block_mode = false;
  Csr Wr, Zr, Coffr;  // W (columns in L_B order), Z and C_off (columns in U_S order)
  int32_t *gmapL = nullptr, *gmapW = nullptr, *fmapU = nullptr, *finB = nullptr, *finS = nullptr;
  double *bL = nullptr, *fL = nullptr, *gS = nullptr, *yS = nullptr, *bU = nullptr, *uU = nullptr;
  // reduced-system GMRES
  double *iV = nullptr, *iW = nullptr, *it1 = nullptr, *it2 = nullptr, *iH = nullptr, *ics = nullptr, *isn = nullptr,
         *ig = nullptr, *ic = nullptr, *ipa = nullptr, *ipb = nullptr, *iscal = nullptr;
  int *iflags = nullptr;
  unsigned long long *islots = nullptr, ilaunch = 0;  // sum slots of the one-launch orthogonalisation
  bool arnoldi_coop = true;  // Arnoldi orthogonalisation as one launch per step (arnoldi_mode)
  Status *status = nullptr;
  double *host_pinned = nullptr;  // 8 doubles for read-backs
  int64_t *blk_starts = nullptr;  // device: interior starts, interface starts, interface starts (local)
  double setup_ms = 0.0;
  GmresWork *gw = nullptr;
  // multiplicative (RAP) method: a copy of A, the smoother (a block-Jacobi
  // preconditioner of its own), and work vectors of length n (rx: the
  // smoothed iterate, rw, ru: products with A) and n_S (ry: the coarse
  // correction in the level-scheduled mode)
  Csr Acp;
  ilu_precond *smoother = nullptr;
  double *rx = nullptr, *rw = nullptr, *ru = nullptr, *ry = nullptr;
  ~ilu_precond();
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
static int read_i64(const int64_t *d, int64_t *h, hipStream_t s) {
  HIPCK(hipMemcpyAsync(h, d, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  return 0;
}

static int check_status(ilu_precond *P, hipStream_t s, const char *phase, const int32_t *row_map, int64_t row_off) {
  Status h;
  HIPCK(hipMemcpyAsync(&h, P->status, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  if (h.code == 0) return 0;
  int64_t row = h.row;
  if (row_map && row >= 0) {
    int32_t orig = -1;
    if (hipMemcpy(&orig, row_map + row_off + row, sizeof(int32_t), hipMemcpyDeviceToHost) == hipSuccess) row = orig;
  }
  switch (h.code) {
    case ILU_ERR_ZERO_PIVOT:
      return fail(ILU_ERR_ZERO_PIVOT, "%s: zero or non-finite pivot at row %lld (original numbering)", phase,
                  (long long)row);
    case ILU_ERR_CAPACITY:
      return fail(ILU_ERR_CAPACITY, "%s: working row %lld exceeds the on-chip capacity", phase, (long long)row);
    case ILU_ERR_TIMEOUT:
      return fail(ILU_ERR_TIMEOUT, "%s: dependency wait expired at row %lld", phase, (long long)row);
    default:
      return fail(h.code, "%s: device error %d at row %lld", phase, h.code, (long long)row);
  }
}

static int bits_for(uint64_t maxkey) {
  int b = 1;
  while (b < 32 && (maxkey >> b)) b++;
  return b;
}

// scan of a device count array into a freshly allocated row pointer; returns total
static int make_rp(Mem &mem, const int64_t *cnt, int64_t n, int64_t **rp, int64_t *total, void *tmp, size_t tmpb,
                   hipStream_t s) {
  RC(mem.alloc(rp, n + 1));
  RC(scan_i64(cnt, *rp, n, tmp, tmpb, s));
  return read_i64(*rp + n, total, s);
}

// compact per-row slots to CSR keeping columns in [lo, hi), shifted by -shift
static int slots_to_csr(Mem &mem, int64_t nrows, const int64_t *cap_rp, const int32_t *len, const int32_t *sc,
                        const double *sv, int64_t lo, int64_t hi, int64_t shift, Csr *out, int64_t *cnt_tmp,
                        void *tmp, size_t tmpb, hipStream_t s) {
  out->n = nrows;
  RC(launch_count_rows(nrows, cap_rp, len, sc, lo, hi, cnt_tmp, s));
  RC(make_rp(mem, cnt_tmp, nrows, &out->rp, &out->nnz, tmp, tmpb, s));
  RC(mem.alloc(&out->ci, out->nnz));
  RC(mem.alloc(&out->v, out->nnz));
  return launch_compact_rows(nrows, cap_rp, len, sc, sv, out->rp, out->ci, out->v, lo, hi, shift, s);
}

struct Slots {
  int64_t *Lcap = nullptr, *Ucap = nullptr, *Rcap = nullptr, *Lrp = nullptr, *Urp = nullptr, *Rrp = nullptr;
  int32_t *Lc = nullptr, *Uc = nullptr, *Rc = nullptr, *Llen = nullptr, *Ulen = nullptr, *Rlen = nullptr;
  double *Lv = nullptr, *Uv = nullptr, *Rv = nullptr, *D = nullptr;
};

// Schedule of the factorization, built on the host as a table of chunks
// (runs of consecutive rows) grouped in streams.  Part A of each segment (its
// rows factored in full) is cut into chunks of `ca` rows -- a line: rows along
// a line depend on one another, so a workgroup that owns one serialises
// nothing that could overlap -- and its chunk sequence into streams of `pa`
// rows -- a plane.  Every plane then advances at once, each a few lines behind
// the one it depends on; streams of one segment only wait on earlier streams.
// Part B (interface rows of a partial factorization, which depend on part A
// only and not on one another) becomes one stream per segment of `cb`-row
// chunks that starts without workgroups: workgroups join it, and any other
// stream with chunks left, once their own stream has handed out all its
// chunks.  The part-A streams come first (ninit of them) and get the grid.
static int build_streams(Mem &tmp, const std::vector<int64_t> &a_start, const std::vector<int64_t> &a_len,
                         const std::vector<int64_t> &b_start, const std::vector<int64_t> &b_len, int64_t ca,
                         int64_t pa, int64_t cb, bool reverse, int64_t grid, int64_t *nchunks_out,
                         int32_t **chunks_out, int64_t *nstreams_out, int64_t *ninit_out, int64_t **stream_chunk_out,
                         hipStream_t s) {
  const int32_t nseg = (int32_t)a_start.size();
  *nchunks_out = 0;
  *chunks_out = nullptr;
  *nstreams_out = 0;
  *ninit_out = 0;
  *stream_chunk_out = nullptr;
  // plane length in whole chunks; planes merge until every part-A stream can
  // have a workgroup of its own.  Without a plane longer than a line (a 2D
  // grid, or no grid) a segment is one stream, and every workgroup that joins
  // it takes the next line: the lines of the segment pipeline behind one
  // another instead of running in consecutive groups on one workgroup each.
  int64_t per = pa > ca ? std::max<int64_t>(1, pa / ca) : ((int64_t)1 << 40);
  for (;;) {
    int64_t na = 0;
    for (int k = 0; k < nseg; k++) na += (a_len[k] + ca * per - 1) / (ca * per);
    if (na <= grid) break;
    per *= 2;
  }
  std::vector<int32_t> ch;  // {first row, rows} pairs
  std::vector<int64_t> sc;
  // a chunk is {first row, rows}; in reverse its rows run downwards from the
  // first, and the chunks and streams of a segment start at its last row
  auto add_stream = [&](int64_t r0, int64_t len, int64_t csize) {
    sc.push_back((int64_t)ch.size() / 2);
    for (int64_t o = 0; o < len; o += csize) {
      ch.push_back((int32_t)(reverse ? r0 - o : r0 + o));
      ch.push_back((int32_t)std::min<int64_t>(csize, len - o));
    }
  };
  for (int k = 0; k < nseg; k++)
    for (int64_t o = 0; o < a_len[k]; o += ca * per)
      add_stream(reverse ? a_start[k] + a_len[k] - 1 - o : a_start[k] + o, std::min(ca * per, a_len[k] - o), ca);
  int64_t ninit = (int64_t)sc.size();
  for (int k = 0; k < nseg; k++)
    if (b_len[k] > 0) add_stream(reverse ? b_start[k] + b_len[k] - 1 : b_start[k], b_len[k], cb);
  const int64_t ns = (int64_t)sc.size();
  if (ns == 0) return 0;
  if (ninit == 0) ninit = std::min<int64_t>(ns, grid);  // no part A: part-B streams start the work
  if (ninit > grid) return fail(ILU_ERR_INVALID_ARG, "factorization: %lld streams for %lld workgroups",
                                (long long)ninit, (long long)grid);
  sc.push_back((int64_t)ch.size() / 2);
  const int64_t nch = (int64_t)ch.size() / 2;
  int32_t *dch;
  int64_t *dsc;
  RC(tmp.alloc(&dch, 2 * nch));
  RC(tmp.alloc(&dsc, ns + 1));
  HIPCK(hipMemcpyAsync(dch, ch.data(), sizeof(int32_t) * ch.size(), hipMemcpyHostToDevice, s));
  HIPCK(hipMemcpyAsync(dsc, sc.data(), sizeof(int64_t) * sc.size(), hipMemcpyHostToDevice, s));
  HIPCK(hipStreamSynchronize(s));  // the host vectors go out of scope
  *nchunks_out = nch;
  *chunks_out = dch;
  *nstreams_out = ns;
  *ninit_out = ninit;
  *stream_chunk_out = dsc;
  return 0;
}

// Line and plane lengths of the rows [0, nrows) of M: the dominant distances
// to a row's second-nearest and farthest lower (upper) neighbours, lines
// clamped to [16, 256].
static int row_geometry(Mem &tmp, const Csr &M, int64_t nrows, bool upper, hipStream_t s, int64_t *line,
                        int64_t *plane) {
  unsigned long long *dh;
  RC(tmp.alloc(&dh, 64));
  HIPCK(hipMemsetAsync(dh, 0, 64 * sizeof(unsigned long long), s));
  RC(launch_gap_hist(M.rp, M.ci, nrows, upper, dh, s));
  unsigned long long h[64];
  HIPCK(hipMemcpyAsync(h, dh, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  auto mode = [&](const unsigned long long *v) {
    int best = -1;
    for (int b = 0; b < 32; b++)
      if (v[b] && (best < 0 || v[b] > v[best])) best = b;
    return best;
  };
  const int bl = mode(h), bp = mode(h + 32);
  *line = std::min<int64_t>(256, std::max<int64_t>(16, bl < 0 ? 16 : ((int64_t)1 << bl)));
  *plane = std::max<int64_t>(*line, bp < 0 ? *line : ((int64_t)1 << bp));
  return 0;
}

// Factor M (rows < nfull full, the rest partial) with the schedule of the
// given segments.  Scratch goes to `tmp`.
// ILU(0) / MILU(0) by levels of the lower pattern over the interior columns
// (partial rows, those of the local Schur complement, take interior pivots
// only and are needed by no row), one launch per level
// (launch_factor_level: the same factors as the dependency-flag kernel,
// without a memory round trip per row on the chain).
// The levels come from the level analysis's sweep over the factorization's
// own row schedule.  *done = false (nothing factored) when the pattern has
// too many levels for one launch each to pay: more than 65,536, or fewer
// than 16 rows per level on average; with partial rows, also when a row has
// more than FACT_LEVEL_PARTIAL_ROW entries.
constexpr int FACT_LEVEL_PARTIAL_ROW = 32;
static int factor_by_levels(ilu_precond *P, Mem &tmp, const Csr &M, const FactLaunch &f,
                            const std::vector<int64_t> &a_start, const std::vector<int64_t> &a_len,
                            const std::vector<int64_t> &b_start, const std::vector<int64_t> &b_len, hipStream_t s,
                            bool *done) {
  *done = false;
  const int64_t n = M.n;
  if (n == 0) return 0;
  if (f.nfull < n) {
    // with the rows of local Schur complements, only matrices of short rows:
    // one thread per row pays for a long row (a power-law hub) on the chain
    int *dlen, hlen = 0;
    RC(tmp.alloc(&dlen, 1));
    HIPCK(hipMemsetAsync(dlen, 0, sizeof(int), s));
    RC(launch_row_len_max(M.rp, n, dlen, s));
    HIPCK(hipMemcpyAsync(&hlen, dlen, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    if (hlen > FACT_LEVEL_PARTIAL_ROW) return 0;
  }
  int64_t line = 16, plane = 16, nch = 0, ns = 0, ninit = 0, *sc = nullptr;
  int32_t *chunks = nullptr, *level;
  const int64_t grid = std::min<int64_t>(levels_resident_groups(P->num_cu), (int64_t)P->num_cu * 32 / LEVEL_WAVES);
  if (grid < 1) return 0;
  RC(tmp.alloc(&level, n));
  RC(row_geometry(tmp, M, n, false, s, &line, &plane));
  RC(build_streams(tmp, a_start, a_len, b_start, b_len, line, plane, FACT_PART_B_CHUNK, false, grid, &nch, &chunks,
                   &ns, &ninit, &sc, s));
  int *flag;
  unsigned int *ticket;
  RC(tmp.alloc(&flag, n));
  RC(tmp.alloc(&ticket, std::max<int64_t>(ns, 1)));
  HIPCK(hipMemsetAsync(flag, 0, sizeof(int) * n, s));
  HIPCK(hipMemsetAsync(ticket, 0, sizeof(unsigned int) * std::max<int64_t>(ns, 1), s));
  // a row's pivots are its interior columns below it (partial rows: every
  // interior column), so only those count
  RC(launch_levels_stream(M.rp, M.ci, true, 0, f.nfull, chunks, ns, ninit, sc, ticket, level, flag, P->status, grid,
                          s));
  RC(check_status(P, s, "factorization levels", nullptr, 0));
  int32_t *dmax, hmax = 0;
  RC(tmp.alloc(&dmax, 1));
  RC(max_i32(level, n, dmax, s));
  HIPCK(hipMemcpyAsync(&hmax, dmax, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  const int64_t nlev = (int64_t)hmax + 1;
  if (nlev > 65536 || n < 16 * nlev) return 0;
  // rows sorted by level
  uint32_t *key, *key2;
  int32_t *val, *rows;
  RC(tmp.alloc(&key, n));
  RC(tmp.alloc(&key2, n));
  RC(tmp.alloc(&val, n));
  RC(tmp.alloc(&rows, n));
  RC(launch_levels_to_keys(level, n, key, val, s));
  const size_t rtb = radix_tmp_bytes(n);
  void *rtmp;
  RC(tmp.alloc((char **)&rtmp, (int64_t)rtb));
  RC(radix_sort(key, val, key2, rows, n, bits_for((uint64_t)hmax), rtmp, rtb, s));
  int64_t *cnt, *lp, tot = 0;
  RC(tmp.alloc(&cnt, nlev));
  RC(histogram_keys(key2, n, nlev, cnt, s));
  const size_t stb = scan_tmp_bytes(nlev) + 64;
  void *stmp;
  RC(tmp.alloc((char **)&stmp, (int64_t)stb));
  RC(make_rp(tmp, cnt, nlev, &lp, &tot, stmp, stb, s));
  std::vector<int64_t> hlp(nlev + 1);
  HIPCK(hipMemcpyAsync(hlp.data(), lp, sizeof(int64_t) * (nlev + 1), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  for (int64_t l = 0; l < nlev; l++) RC(launch_factor_level(f, rows + hlp[l], hlp[l + 1] - hlp[l], s));
  *done = true;
  return 0;
}

static int run_factor(ilu_precond *P, Mem &tmp, const Csr &M, int64_t nfull, int32_t method,
                      const std::vector<int64_t> &a_start, const std::vector<int64_t> &a_len,
                      const std::vector<int64_t> &b_start, const std::vector<int64_t> &b_len, Slots &S,
                      const int32_t *row_map, int64_t row_off, void *stmp, size_t stmpb, hipStream_t s,
                      const char *phase) {
  const int64_t n = M.n;
  if (method == ILU_FACT_ILUT && P->opt.lfil < 0 && n > 4096)
    return fail(ILU_ERR_INVALID_ARG, "ILUT with unlimited fill (lfil < 0) is limited to n <= 4096");
  // capacities
  RC(tmp.alloc(&S.Lcap, n));
  RC(tmp.alloc(&S.Ucap, nfull));
  RC(tmp.alloc(&S.Rcap, n - nfull));
  RC(launch_fact_caps(M.rp, M.ci, n, nfull, method, P->opt.lfil, S.Lcap, S.Ucap, S.Rcap, s));
  int64_t tl, tu, tr;
  RC(make_rp(tmp, S.Lcap, n, &S.Lrp, &tl, stmp, stmpb, s));
  RC(make_rp(tmp, S.Ucap, nfull, &S.Urp, &tu, stmp, stmpb, s));
  RC(make_rp(tmp, S.Rcap, n - nfull, &S.Rrp, &tr, stmp, stmpb, s));
  RC(tmp.alloc(&S.Lc, tl));
  RC(tmp.alloc(&S.Lv, tl));
  RC(tmp.alloc(&S.Uc, tu));
  RC(tmp.alloc(&S.Uv, tu));
  RC(tmp.alloc(&S.Rc, tr));
  RC(tmp.alloc(&S.Rv, tr));
  RC(tmp.alloc(&S.Llen, n));
  RC(tmp.alloc(&S.Ulen, nfull));
  RC(tmp.alloc(&S.Rlen, n - nfull));
  RC(tmp.alloc(&S.D, nfull));
  RC(fill_i32(S.Ulen, 0, nfull, s));
  if (method != ILU_FACT_ILUT && n > 0) {
    FactLaunch f{};
    f.rp = M.rp;
    f.ci = M.ci;
    f.v = M.v;
    f.n = n;
    f.nfull = nfull;
    f.method = method;
    f.droptol = P->opt.droptol;
    f.lfil = P->opt.lfil;
    f.pivot_mode = P->opt.pivot_mode;
    f.pivot_tol = P->opt.pivot_tol;
    f.Lrp = S.Lrp;
    f.Lc = S.Lc;
    f.Lv = S.Lv;
    f.Llen = S.Llen;
    f.Urp = S.Urp;
    f.Uc = S.Uc;
    f.Uv = S.Uv;
    f.Ulen = S.Ulen;
    f.Rrp = S.Rrp;
    f.Rc = S.Rc;
    f.Rv = S.Rv;
    f.Rlen = S.Rlen;
    f.D = S.D;
    f.status = P->status;
    bool done = false;
    RC(factor_by_levels(P, tmp, M, f, a_start, a_len, b_start, b_len, s, &done));
    if (done) return check_status(P, s, phase, row_map, row_off);
  }
  int64_t nchunks = 0, nstreams = 0, ninit = 0, *stream_chunk = nullptr, line = 16, plane = 16;
  int32_t *chunks = nullptr;
  const int64_t grid = std::min<int64_t>(factor_resident_groups(P->num_cu), (int64_t)P->num_cu * 16 / FACT_WAVES);
  if (grid < 1) return fail(ILU_ERR_HIP, "%s: no resident workgroups for the factorization", phase);
  RC(row_geometry(tmp, M, nfull, false, s, &line, &plane));
  RC(build_streams(tmp, a_start, a_len, b_start, b_len, line, plane, FACT_PART_B_CHUNK, false, grid, &nchunks,
                   &chunks, &nstreams, &ninit, &stream_chunk, s));
  if (nchunks > 0) {
    int *done;
    unsigned int *ticket;
    RC(tmp.alloc(&done, n));
    RC(tmp.alloc(&ticket, nstreams));
    HIPCK(hipMemsetAsync(done, 0, sizeof(int) * std::max<int64_t>(n, 1), s));
    HIPCK(hipMemsetAsync(ticket, 0, sizeof(unsigned int) * nstreams, s));
    FactLaunch f;
    f.rp = M.rp;
    f.ci = M.ci;
    f.v = M.v;
    f.n = n;
    f.nfull = nfull;
    f.method = method;
    f.droptol = P->opt.droptol;
    f.lfil = P->opt.lfil;
    f.pivot_mode = P->opt.pivot_mode;
    f.pivot_tol = P->opt.pivot_tol;
    f.nchunks = nchunks;
    f.chunks = chunks;
    f.nstreams = nstreams;
    f.ninit = ninit;
    f.stream_chunk = stream_chunk;
    f.ticket = ticket;
    f.Lrp = S.Lrp;
    f.Lc = S.Lc;
    f.Lv = S.Lv;
    f.Llen = S.Llen;
    f.Urp = S.Urp;
    f.Uc = S.Uc;
    f.Uv = S.Uv;
    f.Ulen = S.Ulen;
    f.Rrp = S.Rrp;
    f.Rc = S.Rc;
    f.Rv = S.Rv;
    f.Rlen = S.Rlen;
    f.D = S.D;
    f.done = done;
    f.epoch = 1;
    f.status = P->status;
    f.grid = grid;
    RC(launch_factor_rows(f, s));
    RC(check_status(P, s, phase, row_map, row_off));
  }
  return 0;
}

// level schedule of a triangular factor
struct Segs {
  std::vector<int64_t> a_start, a_len, b_start, b_len;
};

// Level analysis and the cross-workgroup (global) schedule of one factor;
// S.block_ok tells whether the block-local solve can take it.
// Rows [0, nsweep) are swept in dependency order (the segments cover them);
// rows from nsweep on depend only on rows below nsweep (the rows of W in
// [L_B; W]) and take their levels in one parallel pass after the sweep.
static int build_schedule(ilu_precond *P, Mem &tmp, const Csr &T, bool lower, int64_t lo, int64_t hi,
                          int64_t nsweep, Schedule &S, const Segs &seg, hipStream_t s, const char *phase) {
  const int64_t n = T.n;
  S.nrows = n;
  if (n == 0) return 0;
  Mem &mem = P->mem;
  RC(mem.alloc(&S.level_of, n));
  if (nsweep > 0) {
    // level sweep on the factorization's kind of schedule (lines and planes
    // of this factor's own pattern, from the bottom for L, the top for U)
    int64_t line = 16, plane = 16, nch = 0, ns = 0, ninit = 0, *sc = nullptr;
    int32_t *chunks = nullptr;
    const int64_t grid = std::min<int64_t>(levels_resident_groups(P->num_cu), (int64_t)P->num_cu * 32 / LEVEL_WAVES);
    if (grid < 1) return fail(ILU_ERR_HIP, "%s: no resident workgroups for the level sweep", phase);
    RC(row_geometry(tmp, T, nsweep, !lower, s, &line, &plane));
    RC(build_streams(tmp, seg.a_start, seg.a_len, seg.b_start, seg.b_len, line, plane, 4, !lower, grid, &nch, &chunks,
                     &ns, &ninit, &sc, s));
    int *done;
    unsigned int *ticket;
    RC(tmp.alloc(&done, n));
    RC(tmp.alloc(&ticket, std::max<int64_t>(ns, 1)));
    HIPCK(hipMemsetAsync(done, 0, sizeof(int) * n, s));
    HIPCK(hipMemsetAsync(ticket, 0, sizeof(unsigned int) * std::max<int64_t>(ns, 1), s));
    RC(launch_levels_stream(T.rp, T.ci, lower, lo, hi, chunks, ns, ninit, sc, ticket, S.level_of, done, P->status,
                            grid, s));
    RC(check_status(P, s, phase, nullptr, 0));
  }
  RC(launch_rows_level(T.rp, T.ci, nsweep, n, lo, nsweep, S.level_of, s));
  int32_t *dmax;
  RC(tmp.alloc(&dmax, 1));
  RC(max_i32(S.level_of, n, dmax, s));
  int32_t hmax = 0;
  HIPCK(hipMemcpyAsync(&hmax, dmax, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  S.nlev = (int64_t)hmax + 1;
  S.nblk = P->nparts;
  const uint64_t nkeys = (uint64_t)S.nblk * (uint64_t)S.nlev;
  S.block_ok = S.nlev <= 16384 && nkeys < (1ull << 31);
  return 0;
}

// The cross-workgroup schedule of one factor: rows sorted by level, the
// level pointers and the chunk table of k_trsv.
static int build_global(ilu_precond *P, Mem &tmp, Schedule &S, void *stmp, size_t stmpb, hipStream_t s) {
  const int64_t n = S.nrows;
  if (n == 0) return 0;
  Mem &mem = P->mem;
  const int32_t hmax = (int32_t)(S.nlev - 1);
  uint32_t *key, *key2;
  int32_t *val;
  RC(tmp.alloc(&key, n));
  RC(tmp.alloc(&key2, n));
  RC(tmp.alloc(&val, n));
  RC(mem.alloc(&S.rows, n));
  RC(launch_levels_to_keys(S.level_of, n, key, val, s));
  void *rtmp;
  const size_t rtb = radix_tmp_bytes(n);
  RC(tmp.alloc((char **)&rtmp, (int64_t)rtb));
  RC(radix_sort(key, val, key2, S.rows, n, bits_for((uint64_t)hmax), rtmp, rtb, s));
  int64_t *cnt;
  RC(tmp.alloc(&cnt, S.nlev));
  RC(histogram_keys(key2, n, S.nlev, cnt, s));
  int64_t tot;
  RC(make_rp(mem, cnt, S.nlev, &S.level_ptr, &tot, stmp, stmpb, s));
  int64_t *ccnt, *cbase;
  RC(tmp.alloc(&ccnt, S.nlev));
  RC(launch_level_chunk_counts(S.level_ptr, S.nlev, ccnt, s));
  RC(make_rp(tmp, ccnt, S.nlev, &cbase, &S.nchunks, stmp, stmpb, s));
  RC(mem.alloc(&S.chunk_start, S.nchunks + 1));
  RC(mem.alloc(&S.chunk_level, S.nchunks));
  RC(launch_level_chunks(S.level_ptr, S.nlev, cbase, S.chunk_start, S.chunk_level, s));
  RC(mem.alloc(&S.level_done, S.nlev));
  RC(mem.alloc(&S.ticket, 1));
  HIPCK(hipMemsetAsync(S.level_done, 0, sizeof(unsigned long long) * S.nlev, s));
  HIPCK(hipMemsetAsync(S.ticket, 0, sizeof(unsigned long long), s));
  S.epoch = 0;
  S.ticket_base = 0;
  S.grid = std::min<int64_t>(S.nchunks, (int64_t)P->num_cu * 16);
  return 0;
}

// FP32 / FP16 copy of a factor (and FP32 diagonal) for the level-scheduled
// solve.
static int build_lowp(ilu_precond *P, Schedule &S, const Csr &T, const double *diag, int64_t col_lim, hipStream_t s) {
  if (T.n == 0) return 0;
  Mem &mem = P->mem;
  const int prec = P->opt.factor_prec;
  double *vbuf;
  RC(mem.alloc(&vbuf, (T.nnz * (prec == ILU_PREC_F32 ? 4 : 2) + 7) / 8 + 1));
  S.v_lp = vbuf;
  if (diag) RC(mem.alloc(&S.diag_lp, T.n));
  if (prec == ILU_PREC_F16) RC(mem.alloc(&S.scale_lp, T.n));
  return launch_lowp_factor(T.rp, T.ci, T.v, T.n, col_lim, prec, S.v_lp, S.scale_lp, diag, S.diag_lp, s);
}

// Block-local storage of one factor: rows sorted by (subdomain, level), the
// fixed-stride entries and the records.  omap (row -> output index) places
// each solution; NULL puts it at its own position.  row_blk, when given,
// replaces the subdomains by S.nblk sets of rows of its own (independent of
// each other), one workgroup each.
static int build_block(ilu_precond *P, Mem &tmp, const Csr &T, Schedule &S, const int64_t *bs1, const int64_t *bs2,
                       int64_t split, const double *diag, int64_t ext_col, const int32_t *omap, hipStream_t s,
                       const char *phase, const int32_t *row_blk = nullptr, const int32_t *xrow = nullptr,
                       int32_t K1 = 0, Mem *into = nullptr) {
  const int64_t n = T.n;
  S.use_block = true;
  S.ext_col = ext_col;
  // Rows from split on in a factor with two block-start tables (the rows of
  // W in [L_B; W]) depend only on rows below split: they are left out of the
  // block-local solve and computed by one parallel pass after it.
  const int64_t nloc = bs2 ? split : n;
  S.nloc = nloc;
  if (nloc == 0) return 0;
  Mem &mem = into ? *into : P->mem;  // the split's attempt keeps its blocks apart until it succeeds
  const uint64_t nkeys = (uint64_t)S.nblk * (uint64_t)S.nlev;
  uint32_t *key, *key2;
  int32_t *val;
  RC(tmp.alloc(&key, nloc));
  RC(tmp.alloc(&key2, nloc));
  RC(tmp.alloc(&val, nloc));
  void *rtmp;
  const size_t rtb = radix_tmp_bytes(nloc);
  RC(tmp.alloc((char **)&rtmp, (int64_t)rtb));
  const int32_t *blk = row_blk;
  if (!blk) {
    int32_t *b;
    RC(tmp.alloc(&b, nloc));
    RC(launch_row_blocks(nloc, (int32_t)S.nblk, bs1, nullptr, split, b, s));
    blk = b;
  }
  RC(launch_block_level_keys(S.level_of, blk, nloc, S.nlev, key, val, s));
  RC(mem.alloc(&S.blk_rows, nloc));
  RC(radix_sort(key, val, key2, S.blk_rows, nloc, bits_for(nkeys - 1), rtmp, rtb, s));
  int64_t *bcnt, *bptr, btot;
  RC(tmp.alloc(&bcnt, (int64_t)nkeys));
  RC(histogram_keys(key2, nloc, (int64_t)nkeys, bcnt, s));
  const size_t stb2 = scan_tmp_bytes((int64_t)nkeys) + 64;
  void *stmp2;
  RC(tmp.alloc((char **)&stmp2, (int64_t)stb2));
  RC(make_rp(tmp, bcnt, (int64_t)nkeys, &bptr, &btot, stmp2, stb2, s));
  RC(mem.alloc(&S.blk_lev_ptr, (int64_t)nkeys + 1));
  RC(launch_i64_to_i32(bptr, S.blk_lev_ptr, (int64_t)nkeys + 1, s));
  // fixed-stride storage: G lanes of E entries per row; threads per
  // workgroup cover the widest level (rows beyond take the slow path)
  int32_t *dm;
  RC(mem.alloc(&S.pos, nloc));
  RC(tmp.alloc(&dm, 2));
  RC(fill_i32(dm, 0, 2, s));
  RC(launch_lds_prepare(S.blk_rows, T.rp, T.ci, nloc, ext_col, S.blk_lev_ptr, (int64_t)nkeys, S.pos, dm, dm + 1, s));
  int32_t hm[2] = {0, 0};
  HIPCK(hipMemcpyAsync(hm, dm, sizeof(hm), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  // entries per lane E and lanes per row G: one lane of 2 or 4 for short
  // rows, else lanes of 8, as few as cover the longest row (at most 8)
  int G = 1, E = hm[0] <= 2 ? 2 : hm[0] <= 4 ? 4 : 8;
  while (E == 8 && G < 8 && 8 * G < hm[0]) G *= 2;
  if ((nloc + 1) * (int64_t)G * E >= ((int64_t)1 << 29))  // byte offsets of the values below 2^32
    return fail(ILU_ERR_INVALID_ARG, "%s: factor too large for the block solve", phase);
  // threads cover the widest level: up to 512, or 1024 for one-lane rows of
  // at most 4 entries (the wide instance, 16 waves)
  const int64_t bt = ((int64_t)std::max(hm[1], 1) * G + 63) / 64 * 64;
  const int64_t bt_cap = (G == 1 && E <= 4) ? 1024 : 512;
  S.lds_g = G;
  S.lds_e = E;
  S.lds_bt = (int32_t)std::min<int64_t>(bt, bt_cap);
  const bool fits = bt <= bt_cap;
  const int64_t ne = (nloc + 1) * G * E;
  const int prec = P->opt.factor_prec;
  const int64_t vbytes = prec == ILU_PREC_F64 ? 8 : prec == ILU_PREC_F32 ? 4 : 2;
  RC(mem.alloc(&S.lds_c, ne));  // 16-bit window slots
  double *vstore;
  RC(mem.alloc(&vstore, (ne * vbytes + 7) / 8));
  S.lds_v = vstore;
  RC(mem.alloc(&S.lds_rec, 4 * (nloc + 1)));
  S.out_map = omap ? omap : S.pos;
  RC(fill_i32(dm, 0, 1, s));  // reused as the slow-row flag
  // with xrow (a split block), dependencies across parts name import slots
  RC(launch_lds_fill(S.blk_rows, T.rp, T.ci, T.v, diag, nloc, ext_col, S.pos, S.blk_lev_ptr, (int64_t)nkeys, G, E, prec,
                     S.out_map, S.lds_c, S.lds_v, S.lds_rec, dm, xrow ? row_blk : nullptr, xrow, K1, S.ilp, S.nlev,
                     s));
  int32_t any_slow = 1;
  HIPCK(hipMemcpyAsync(&any_slow, dm, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  S.lds_fast = fits && any_slow == 0;
  return 0;
}

// Workgroups per subdomain of the block-local solve of an interior factor
// (nloc rows in the block-local solve): block_split, or under 0 (auto) one
// per 24,576 rows of a subdomain, at least two for subdomains of 32,768
// rows and more, at most 16 (more parts shorten each part's levels but
// lengthen the chain of parts that each trail the one before), while the
// parts fit the CUs.
static int32_t split_parts(const ilu_precond *P, int64_t nloc) {
  const int32_t k = P->opt.block_split;
  if (k == 1 || nloc == 0 || P->nparts < 1) return 1;
  if (k >= 2) return k;
  const int64_t rows = nloc / P->nparts;
  if (rows < 32768) return 1;
  int64_t n = std::max<int64_t>(2, std::min<int64_t>(16, rows / 24576));
  while (n > 1 && P->nparts * n > P->num_cu) n--;
  return (int32_t)n;
}

// The split of each subdomain's block-local solve over K workgroups
// (trsv_split.hip): the part of each row (K ranges of the block, numbered
// from its end for a backward solve) and the values parts pass to each
// other, one import per (source row, importing part), sorted by (importing
// part, level that first needs them).  Leaves the schedule unsplit (*ok =
// false) for a part spanning more than SPLIT_LEVELS levels, an import by a
// part that does not come later, an import that would leave its part's LDS
// ring before it is read, or more than 64 imports for one level of one
// part.  *part, *xrow ((row, later part of its subdomain) -> import index,
// or -1) and *isrc (import -> source row) live in tmp and feed build_block
// and build_exports.
static int build_split(ilu_precond *P, Mem &tmp, Mem &keep, const Csr &T, Schedule &S, const int64_t *bs,
                       int64_t nloc, int64_t ext_col, int32_t K, bool backward, hipStream_t s, int32_t **part_out,
                       int32_t **xrow_out, int32_t **isrc_out, bool *ok) {
  *ok = false;
  const int64_t nblk = (int64_t)P->nparts * K, nlev = S.nlev;
  const uint64_t nkeys = (uint64_t)nblk * (uint64_t)nlev;
  if (nloc == 0 || nkeys >= (1ull << 31)) return 0;
  int32_t *part, *xrow, *bad;
  int64_t *cnt, *off, m = 0;
  RC(tmp.alloc(&part, nloc));
  RC(tmp.alloc(&cnt, nloc));
  RC(tmp.alloc(&bad, 4));
  RC(fill_i32(bad, 0, 4, s));
  RC(launch_split_parts(bs, P->nparts, nloc, K, backward, part, s));
  // each part walks its own levels only: at most SPLIT_LEVELS of them
  int32_t *lmin, *lmax;
  RC(tmp.alloc(&lmin, nblk));
  RC(tmp.alloc(&lmax, nblk));
  RC(fill_i32(lmin, INT32_MAX, nblk, s));
  RC(fill_i32(lmax, -1, nblk, s));
  RC(launch_part_levels(part, S.level_of, nloc, lmin, lmax, s));
  std::vector<int32_t> hmin(nblk), hmax(nblk), hr(2 * nblk);
  HIPCK(hipMemcpyAsync(hmin.data(), lmin, sizeof(int32_t) * nblk, hipMemcpyDeviceToHost, s));
  HIPCK(hipMemcpyAsync(hmax.data(), lmax, sizeof(int32_t) * nblk, hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  int64_t most = 0;
  for (int64_t p = 0; p < nblk; p++) {
    const bool empty = hmax[p] < 0;
    hr[2 * p] = empty ? 0 : hmin[p];
    hr[2 * p + 1] = empty ? 0 : hmax[p] - hmin[p] + 1;
    most = std::max<int64_t>(most, hr[2 * p + 1]);
  }
  if (most > SPLIT_LEVELS) return 0;
  RC(launch_cross_count(T.rp, T.ci, nloc, ext_col, part, cnt, s));
  size_t stb = scan_tmp_bytes(std::max<int64_t>(nloc, (int64_t)nkeys)) + 64;
  void *stmp;
  RC(tmp.alloc((char **)&stmp, (int64_t)stb));
  RC(make_rp(tmp, cnt, nloc, &off, &m, stmp, stb, s));
  if (m >= ((int64_t)1 << 31)) return 0;
  const int64_t mm = std::max<int64_t>(m, 1);
  uint32_t *src, *k1, *k2;
  int32_t *key, *v1, *v2;
  RC(tmp.alloc(&src, mm));
  RC(tmp.alloc(&key, mm));
  RC(tmp.alloc(&k1, mm));
  RC(tmp.alloc(&v1, mm));
  RC(tmp.alloc(&k2, mm));
  RC(tmp.alloc(&v2, mm));
  RC(launch_cross_emit(T.rp, T.ci, nloc, ext_col, part, S.level_of, nlev, off, src, key, s));
  const size_t rtb = radix_tmp_bytes(mm);
  void *rtmp;
  RC(tmp.alloc((char **)&rtmp, (int64_t)rtb));
  // by key, then (stable) by source row: each source's records in key order
  RC(radix_sort(reinterpret_cast<const uint32_t *>(key), reinterpret_cast<const int32_t *>(src), k1, v1, m,
                bits_for(nkeys - 1), rtmp, rtb, s));
  RC(radix_sort(reinterpret_cast<const uint32_t *>(v1), reinterpret_cast<const int32_t *>(k1), k2, v2, m,
                bits_for((uint64_t)std::max<int64_t>(nloc - 1, 1)), rtmp, rtb, s));
  int64_t *head, *rank, nimp = 0;
  RC(tmp.alloc(&head, mm));
  RC(launch_cross_heads(k2, v2, m, part, nlev, head, bad, s));
  const size_t stb2 = scan_tmp_bytes(mm) + 64;
  void *stmp2;
  RC(tmp.alloc((char **)&stmp2, (int64_t)stb2));
  RC(make_rp(tmp, head, m, &rank, &nimp, stmp2, stb2, s));
  const int64_t ni = std::max<int64_t>(nimp, 1);
  uint32_t *isrc, *ikey, *ikey2;
  int32_t *isrc2;
  RC(tmp.alloc(&isrc, ni));
  RC(tmp.alloc(&ikey, ni));
  RC(tmp.alloc(&ikey2, ni));
  RC(tmp.alloc(&isrc2, ni));
  RC(launch_cross_compact(k2, v2, m, head, rank, isrc, ikey, s));
  const size_t rtb2 = radix_tmp_bytes(ni);
  void *rtmp2;
  RC(tmp.alloc((char **)&rtmp2, (int64_t)rtb2));
  // imports by (part, level), source rows ascending within each
  RC(radix_sort(ikey, reinterpret_cast<const int32_t *>(isrc), ikey2, isrc2, nimp, bits_for(nkeys - 1), rtmp2, rtb2,
                s));
  int64_t *icnt, *iptr, itot = 0;
  RC(tmp.alloc(&icnt, (int64_t)nkeys));
  RC(histogram_keys(ikey2, nimp, (int64_t)nkeys, icnt, s));
  RC(make_rp(tmp, icnt, (int64_t)nkeys, &iptr, &itot, stmp, stb, s));
  int32_t *ilp;
  RC(keep.alloc(&ilp, (int64_t)nkeys + 1));
  RC(launch_i64_to_i32(iptr, ilp, (int64_t)nkeys + 1, s));
  RC(tmp.alloc(&xrow, nloc * (K - 1)));
  RC(fill_i32(xrow, -1, nloc * (K - 1), s));
  RC(launch_cross_slots(isrc2, ikey2, nimp, part, nlev, K - 1, xrow, s));
  RC(launch_cross_check(T.rp, T.ci, nloc, ext_col, part, S.level_of, nlev, xrow, K - 1, ilp, bad, s));
  RC(launch_cross_width(ilp, (int64_t)nkeys, bad, s));
  int32_t hb[4] = {0, 0, 0, 0};
  HIPCK(hipMemcpyAsync(hb, bad, sizeof(hb), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  if (hb[1] || hb[2] || hb[3] || nimp + 128 * nblk >= ((int64_t)1 << 29)) return 0;
  // the slots, then a pad of 128 words per part for the idle lanes of its loader wave
  RC(keep.alloc(&S.xv, nimp + 128 * nblk));
  RC(launch_fill_unset(S.xv, nimp + 128 * nblk, s));
  RC(keep.alloc(&S.xticket, 1));
  HIPCK(hipMemsetAsync(S.xticket, 0, sizeof(unsigned long long), s));
  RC(keep.alloc(&S.lrange, 2 * nblk));
  HIPCK(hipMemcpyAsync(S.lrange, hr.data(), sizeof(int32_t) * 2 * nblk, hipMemcpyHostToDevice, s));
  HIPCK(hipStreamSynchronize(s));  // hr is host memory on this stack
  S.xlevels = most;
  S.ilp = ilp;
  S.nimp = nimp;
  S.split_k = K;
  S.nblk = nblk;
  *part_out = part;
  *xrow_out = xrow;
  *isrc_out = isrc2;
  *ok = true;
  return 0;
}

// The exports of a split solve, once the positions are known: one per
// import, sorted by (exporting part, level of the source row) and stored as
// {position, slot}.  *ok = false when a level of a part exports more than 64
// rows (one lane each in the exchange wave).
static int build_exports(Mem &tmp, Mem &keep, Schedule &S, const int32_t *part, const int32_t *isrc,
                         hipStream_t s, bool *ok) {
  *ok = false;
  const int64_t nimp = S.nimp, nkeys = S.nblk * S.nlev, ni = std::max<int64_t>(nimp, 1);
  uint32_t *key, *key2;
  int32_t *val, *egi, *bad;
  RC(tmp.alloc(&key, ni));
  RC(tmp.alloc(&val, ni));
  RC(tmp.alloc(&key2, ni));
  RC(tmp.alloc(&egi, ni));
  RC(tmp.alloc(&bad, 4));
  RC(fill_i32(bad, 0, 4, s));
  RC(launch_export_keys(isrc, nimp, part, S.level_of, S.nlev, key, val, s));
  const size_t rtb = radix_tmp_bytes(ni);
  void *rtmp;
  RC(tmp.alloc((char **)&rtmp, (int64_t)rtb));
  RC(radix_sort(key, val, key2, egi, nimp, bits_for((uint64_t)nkeys - 1), rtmp, rtb, s));
  int64_t *cnt, *ptr, tot = 0;
  RC(tmp.alloc(&cnt, nkeys));
  RC(histogram_keys(key2, nimp, nkeys, cnt, s));
  const size_t stb = scan_tmp_bytes(nkeys) + 64;
  void *stmp;
  RC(tmp.alloc((char **)&stmp, (int64_t)stb));
  RC(make_rp(tmp, cnt, nkeys, &ptr, &tot, stmp, stb, s));
  int32_t *elp, *xe;
  RC(keep.alloc(&elp, nkeys + 1));
  RC(launch_i64_to_i32(ptr, elp, nkeys + 1, s));
  RC(launch_cross_width(elp, nkeys, bad, s));
  int32_t hb[4] = {0, 0, 0, 0};
  HIPCK(hipMemcpyAsync(hb, bad, sizeof(hb), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  if (hb[3]) return 0;
  RC(keep.alloc(&xe, 2 * (nimp + 1)));
  RC(launch_export_fill(egi, isrc, S.pos, nimp, xe, s));
  S.elp = elp;
  S.xe = xe;
  *ok = true;
  return 0;
}

// Block-local storage of an interior factor (L_B with the W rows after it,
// or U_B), split over several workgroups per subdomain when split_parts
// asks for it and the split applies; unsplit otherwise.
static int build_block_interior(ilu_precond *P, Mem &tmp, const Csr &T, Schedule &S, const int64_t *bs1,
                                const int64_t *bs2, int64_t split, const double *diag, int64_t ext_col,
                                bool backward, hipStream_t s, const char *phase) {
  const int64_t nloc = bs2 ? split : T.n;
  const int32_t K = split_parts(P, nloc);
  if (K > 1) {
    int32_t *part = nullptr, *xrow = nullptr, *isrc = nullptr;
    bool ok = false;
    Mem trial;  // the attempt's device blocks: kept only if the split applies
    RC(build_split(P, tmp, trial, T, S, bs1, nloc, ext_col, K, backward, s, &part, &xrow, &isrc, &ok));
    if (ok) {
      RC(build_block(P, tmp, T, S, bs1, bs2, split, diag, ext_col, nullptr, s, phase, part, xrow, K - 1, &trial));
      // check-free factors only, the compute threads and the two exchange waves within 512
      ok = S.lds_fast && S.lds_bt <= 384;
      if (ok) RC(build_exports(tmp, trial, S, part, isrc, s, &ok));
    }
    if (ok) {
      P->mem.adopt(trial);
      return 0;
    }
    HIPCK(hipStreamSynchronize(s));  // the attempt's kernels are done with its blocks
    trial.release(false);
    // build the unsplit solve
    S.split_k = 1;
    S.xv = nullptr;
    S.xe = S.elp = S.ilp = S.lrange = nullptr;
    S.xlevels = 0;
    S.nimp = 0;
    S.xticket = nullptr;
    S.nblk = P->nparts;
  }
  return build_block(P, tmp, T, S, bs1, bs2, split, diag, ext_col, nullptr, s, phase);
}

// The reduced system's rows split into the connected components of the
// pattern of L_S + U_S: rows in different components never meet in a
// triangular solve (the two interface planes of a slab, for instance), so
// each component can be solved by its own workgroup, with half as many rows
// per level or fewer.  Used when it gives a few more workgroups (more than
// one component in some subdomain, at most 4 per subdomain on average and
// one per CU); *ncomp = 0 keeps one workgroup per subdomain.  Components
// never span subdomains (the local Schur factors are block diagonal) and
// are numbered by their first row.
static int schur_components(ilu_precond *P, Mem &tmp, int32_t **comp, int64_t *ncomp, void *stmp, size_t stmpb,
                            hipStream_t s) {
  const int64_t nS = P->nS;
  *comp = nullptr;
  *ncomp = 0;
  if (nS == 0) return 0;
  int32_t *lab, *root;
  int64_t *isroot, *rank, total = 0;
  RC(tmp.alloc(&lab, nS));
  RC(tmp.alloc(&root, nS));
  RC(tmp.alloc(&isroot, nS));
  RC(launch_cc_label(P->LS.rp, P->LS.ci, P->US.rp, P->US.ci, nS, lab, root, isroot, s));
  RC(make_rp(tmp, isroot, nS, &rank, &total, stmp, stmpb, s));
  if (total <= P->nparts || total > std::min<int64_t>(4LL * P->nparts, P->num_cu)) return 0;
  RC(tmp.alloc(comp, nS));
  RC(launch_cc_number(root, rank, nS, *comp, s));
  *ncomp = total;
  return 0;
}

// A CSR whose row q is row row0 + rows[q] of A, columns c -> cmap[c - col_off]
static int csr_permute(Mem &mem, Mem &tmp, const Csr &A, int64_t row0, const int32_t *rows, int64_t nrows,
                       const int32_t *cmap, int64_t col_off, Csr *out, void *stmp, size_t stmpb, hipStream_t s) {
  out->n = nrows;
  int64_t *len;
  RC(tmp.alloc(&len, nrows));
  RC(launch_csr_perm_len(A.rp, row0, rows, nrows, len, s));
  RC(make_rp(mem, len, nrows, &out->rp, &out->nnz, stmp, stmpb, s));
  RC(mem.alloc(&out->ci, out->nnz));
  RC(mem.alloc(&out->v, out->nnz));
  return launch_csr_perm_ent(A.rp, A.ci, A.v, row0, rows, nrows, cmap, col_off, out->rp, out->ci, out->v, s);
}

// The orders that connect the four block-local solves (see ilu_precond):
// index maps, the renumbered copies of W, Z and C_off, and the vectors.
static int build_block_flow(ilu_precond *P, Mem &tmp, void *stmp, size_t stmpb, hipStream_t s) {
  Mem &mem = P->mem;
  const int64_t nB = P->nB, nS = P->nS;
  RC(mem.alloc(&P->bL, nB));
  RC(mem.alloc(&P->fL, nB));
  RC(mem.alloc(&P->bU, nB));
  RC(mem.alloc(&P->uU, nB));
  RC(mem.alloc(&P->gS, nS));
  RC(mem.alloc(&P->yS, nS));
  RC(mem.alloc(&P->gmapL, nB));
  RC(mem.alloc(&P->fmapU, nB));
  RC(mem.alloc(&P->finB, nB));
  RC(mem.alloc(&P->finS, nS));
  RC(mem.alloc(&P->gmapW, nS));
  RC(launch_gather_i32(P->perm, P->sL1.blk_rows, nB, P->gmapL, s));      // r index of each L_B position
  RC(launch_gather_i32(P->sL1.pos, P->sU1.blk_rows, nB, P->fmapU, s));   // L_B position of each U_B position
  RC(launch_gather_i32(P->perm, P->sU1.blk_rows, nB, P->finB, s));       // z index of each U_B position
  RC(launch_gather_i32(P->perm + nB, P->sUS.blk_rows, nS, P->finS, s));  // z index of each U_S position
  RC(launch_gather_i32(P->perm + nB, P->sLS.blk_rows, nS, P->gmapW, s));  // r index of each L_S position
  // W rows in L_S order (columns in L_B order); Z rows in U_B order and C_off
  // rows in L_S order (columns in U_S order)
  RC(csr_permute(mem, tmp, P->L1, nB, P->sLS.blk_rows, nS, P->sL1.pos, 0, &P->Wr, stmp, stmpb, s));
  RC(csr_permute(mem, tmp, P->Zb, 0, P->sU1.blk_rows, nB, P->sUS.pos, nB, &P->Zr, stmp, stmpb, s));
  RC(csr_permute(mem, tmp, P->Coff, 0, P->sLS.blk_rows, nS, P->sUS.pos, 0, &P->Coffr, stmp, stmpb, s));
  HIPCK(hipStreamSynchronize(s));
  return 0;
}

// Algorithmic bytes of one triangular solve, counted as the survey's
// measurement table does: each strict-triangle entry once (int32 column and
// the value in the storage precision), int32 row pointers, the right-hand
// side read and the solution written once (FP64 vectors), and the diagonal
// of an upper solve in the storage precision (FP64 8, FP32 4, FP16 2 bytes
// per row).  Gather and scatter maps, the FP16 row scales and the layout's
// padding are the kernel's own overheads, not algorithmic bytes.
static double trsv_bytes(int64_t n, int64_t nnz, bool diag, int prec) {
  const double vb = prec == ILU_PREC_F64 ? 8.0 : prec == ILU_PREC_F32 ? 4.0 : 2.0;
  double b = (4.0 + vb) * (double)nnz + 4.0 * (double)(n + 1) + 16.0 * (double)n;
  if (diag) b += vb * (double)n;
  return b;
}

// Launch description of one solve.  Block-local schedules take b in position
// order and write x through the schedule's output map.
static TrsvLaunch make_launch(ilu_precond *P, Schedule &S, const Csr &T, const double *diag, int64_t split,
                              const double *b, const int32_t *bmap, double *x, double *scat, const int32_t *smap,
                              int role) {
  TrsvLaunch t;
  t.nrows = S.nrows;
  t.rows = S.rows;
  t.chunk_start = S.chunk_start;
  t.chunk_level = S.chunk_level;
  t.nchunks = S.nchunks;
  t.level_ptr = S.level_ptr;
  t.level_done = S.level_done;
  t.ticket = S.ticket;
  t.rp = T.rp;
  t.ci = T.ci;
  t.v = T.v;
  t.diag = diag;
  t.split_col = split;
  t.b = b;
  t.b_map = bmap;
  t.x = x;
  t.scatter_out = scat;
  t.scatter_map = smap;
  t.status = P->status;
  t.max_waves = S.grid;
  t.role = role;
  if (S.use_block) {
    t.nblk = S.nblk;
    t.nlev_blk = S.nlev;
    t.blk_rows = S.blk_rows;
    t.blk_lev_ptr = S.blk_lev_ptr;
    t.lds_c = S.lds_c;
    t.lds_v = S.lds_v;
    t.lds_rec = S.lds_rec;
    t.out_map = S.out_map;
    t.lds_g = S.lds_g;
    t.lds_e = S.lds_e;
    t.lds_bt = S.lds_bt;
    t.lds_fast = S.lds_fast ? 1 : 0;
    t.split_col = S.ext_col;
    t.nrows = S.nloc;
    if (S.split_k > 1) {
      t.xv = S.xv;
      t.xe = S.xe;
      t.elp = S.elp;
      t.lrange = S.lrange;
      t.xlevels = S.xlevels;
      t.ilp = S.ilp;
      t.nimp = S.nimp;
      t.xticket = S.xticket;
    }
  }
  t.prec = P->opt.factor_prec;
  t.f64_row = role == 0 ? P->nB : INT64_MAX;
  t.v_lp = S.v_lp;
  t.diag_lp = S.diag_lp;
  t.scale_lp = S.scale_lp;
  return t;
}

// `after` runs inside the timed region (the W rows of the L_B solve).
static int trsv(ilu_precond *P, Schedule &S, const Csr &T, const double *diag, int64_t split, const double *b,
                const int32_t *bmap, double *x, double *scat, const int32_t *smap, hipStream_t s, int role,
                const std::function<int()> &after = nullptr) {
  if (S.nrows == 0) return 0;
  TrsvLaunch t = make_launch(P, S, T, diag, split, b, bmap, x, scat, smap, role);
  // the block-local U_B solve reads no Z entry (Z y is applied before it)
  const int64_t nnz = T.nnz - (S.use_block && role == 1 ? P->Zb.nnz : 0);
  const double bytes = trsv_bytes(S.nrows, nnz, diag != nullptr, P->opt.factor_prec);
  if (S.use_block) {
    if (bmap || scat) return fail(ILU_ERR_INVALID_ARG, "internal: block-local solves take no gather or scatter map");
    return timed(ILU_K_TRSV_LB + role, bytes, s, [&] {
      RC(t.xv ? launch_trsv_lds_split(t, s) : launch_trsv_lds(t, s));
      if (after) RC(after());
      return 0;
    });
  }
  S.epoch++;
  t.epoch = S.epoch;
  t.ticket_base = S.ticket_base;
  S.ticket_base += (unsigned long long)(S.nchunks + S.grid);
  return timed(ILU_K_TRSV_LB + role, bytes, s, [&] { return launch_trsv(t, s); });
}

// x = U_S^-1 L_S^-1 b (x may be b in the global mode; in block mode b is in
// L_S order and x in U_S order): one launch when both solves are block-local
// with the same lane shape, timed as the L_S class with the bytes of both.
static int trsv_schur(ilu_precond *P, const double *b, double *x, hipStream_t s) {
  if (P->nS == 0) return 0;
  if (P->block_mode) {
    TrsvLaunch lo = make_launch(P, P->sLS, P->LS, nullptr, 0, b, nullptr, x, nullptr, nullptr, 2);
    TrsvLaunch up = make_launch(P, P->sUS, P->US, P->DS, INT64_MAX, x, nullptr, x, nullptr, nullptr, 3);
    if (trsv_lds_pair_ok(lo, up)) {
      const int fp = P->opt.factor_prec;
      const double bytes = trsv_bytes(P->sLS.nrows, P->LS.nnz, false, fp) + trsv_bytes(P->sUS.nrows, P->US.nnz, true, fp);
      return timed(ILU_K_TRSV_LS, bytes, s, [&] { return launch_trsv_lds_pair(lo, up, s); });
    }
  }
  RC(trsv(P, P->sLS, P->LS, nullptr, 0, b, nullptr, x, nullptr, nullptr, s, 2));
  return trsv(P, P->sUS, P->US, P->DS, INT64_MAX, x, nullptr, x, nullptr, nullptr, s, 3);
}

// Algorithmic bytes of one SpMV: 12 per entry, int32 row pointers, x and y
// once each (and b for the residual form).
static double spmv_bytes(int64_t n, int64_t nnz, bool resid) {
  return 12.0 * (double)nnz + 4.0 * (double)(n + 1) + 16.0 * (double)n + (resid ? 8.0 * (double)n : 0.0);
}

ilu_precond::~ilu_precond() {
  if (host_pinned) (void)hipHostFree(host_pinned);
  host_pinned = nullptr;
  delete gw;
  delete smoother;
}

namespace silu {
int64_t precond_bytes(const ilu_precond *P) {
  if (!P) return 0;
  int64_t b = (int64_t)P->mem.bytes;
  if (P->gw) b += (int64_t)P->gw->mem.bytes;
  return b + precond_bytes(P->smoother);
}

static void release_nosync(ilu_precond *P) {
  if (!P) return;
  P->mem.release(false);
  if (P->gw) P->gw->mem.release(false);
  release_nosync(P->smoother);
}

void precond_destroy_idle(ilu_precond *P) {
  if (!P) return;
  (void)hipSetDevice(P->device);
  release_nosync(P);
  delete P;
}

int dev_alloc(void **p, size_t bytes) {
  const hipError_t e = cache_alloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(ILU_ERR_OOM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  }
  return 0;
}

void dev_free(void *p) {
  if (p) cache_free(p);
}
}  // namespace silu

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void ilu_default_options(ilu_options_t *o) {
  if (!o) return;
  o->method = ILU_METHOD_BJ;
  o->interior_fact = ILU_FACT_ILU0;
  o->interface_fact = ILU_FACT_ILU0;
  o->droptol = 0.0;
  o->lfil = -1;
  o->inner_iters = 3;
  o->inner_rtol = 0.0;
  o->pivot_mode = ILU_PIVOT_ERROR;
  o->pivot_tol = 0.0;
  o->trsv_mode = ILU_TRSV_AUTO;
  o->factor_prec = ILU_PREC_F64;
  o->smooth_fact = ILU_FACT_ILU0;
  o->arnoldi_mode = ILU_ARNOLDI_AUTO;
  o->block_split = 0;
}

const char *ilu_last_error(void) { return g_err.c_str(); }

static int setup_impl(const ilu_csr_t *A, const int32_t *d_part, int32_t nparts, const ilu_options_t *opt,
                      hipStream_t s, ilu_precond *P) {
  const int64_t n = A->n;
  HIPCK(hipGetDevice(&P->device));
  {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, P->device) == hipSuccess && cu > 0)
      P->num_cu = cu;
  }
  Mem &mem = P->mem;
  Mem tmp;
  RC(mem.alloc(&P->status, 1));
  HIPCK(hipMemsetAsync(P->status, 0, sizeof(Status), s));
  HIPCK(hipHostMalloc((void **)&P->host_pinned, 8 * sizeof(double), hipHostMallocDefault));

  const size_t stmpb = scan_tmp_bytes(std::max<int64_t>(n + 1, 256 * ((n + 2047) / 2048) + 1) + 64);
  void *stmp;
  RC(tmp.alloc((char **)&stmp, (int64_t)stmpb));

  // 1. validation
  int32_t *err;
  RC(tmp.alloc(&err, 2));
  RC(fill_i32(err, 0x7fffffff, 2, s));
  RC(launch_validate(A->d_row_ptr, A->d_col, n, A->nnz, d_part, nparts, err, s));
  int32_t herr[2];
  HIPCK(hipMemcpyAsync(herr, err, sizeof(herr), hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  if (herr[0] != 0x7fffffff)
    return fail(ILU_ERR_CSR, "invalid CSR at row %d (row pointers, unsorted/duplicate/out-of-range columns, or "
                "missing diagonal)", herr[0]);
  if (herr[1] != 0x7fffffff) return fail(ILU_ERR_INVALID_ARG, "partition value out of range at row %d", herr[1]);

  // 2. interface classification, 3. permutation
  RC(mem.alloc(&P->iface, n));
  HIPCK(hipMemsetAsync(P->iface, 0, std::max<int64_t>(n, 1), s));
  RC(launch_classify(A->d_row_ptr, A->d_col, n, d_part, P->iface, s));
  RC(mem.alloc(&P->perm, n));
  RC(mem.alloc(&P->iperm, n));
  {
    uint32_t *key, *key2;
    int32_t *val;
    RC(tmp.alloc(&key, n));
    RC(tmp.alloc(&key2, n));
    RC(tmp.alloc(&val, n));
    RC(launch_perm_keys(n, d_part, nparts, P->iface, key, val, s));
    void *rtmp;
    const size_t rtb = radix_tmp_bytes(n);
    RC(tmp.alloc((char **)&rtmp, (int64_t)rtb));
    RC(radix_sort(key, val, key2, P->perm, n, bits_for((uint64_t)(2 * nparts)), rtmp, rtb, s));
    RC(launch_inverse_perm(n, P->perm, P->iperm, s));
    int64_t *cnt, *starts, tot;
    RC(tmp.alloc(&cnt, 2 * nparts));
    RC(histogram_keys(key2, n, 2 * nparts, cnt, s));
    RC(make_rp(tmp, cnt, 2 * nparts, &starts, &tot, stmp, stmpb, s));
    std::vector<int64_t> h(2 * nparts + 1);
    HIPCK(hipMemcpyAsync(h.data(), starts, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    P->offsets.assign(2 * nparts + 2, 0);
    for (int k = 0; k <= nparts; k++) P->offsets[k] = h[k];
    for (int k = 0; k <= nparts; k++) P->offsets[nparts + 1 + k] = h[nparts + k];
  }
  P->nB = P->offsets[nparts];
  P->nS = n - P->nB;
  const int64_t nB = P->nB, nS = P->nS;

  // 4. permuted subdomain blocks and the cross-subdomain coupling
  Csr Ah;
  Ah.n = n;
  P->Coff.n = nS;
  {
    int64_t *ca, *cc;
    RC(tmp.alloc(&ca, n));
    RC(tmp.alloc(&cc, nS));
    RC(launch_extract_counts(A->d_row_ptr, A->d_col, n, nB, d_part, P->perm, ca, cc, s));
    RC(make_rp(tmp, ca, n, &Ah.rp, &Ah.nnz, stmp, stmpb, s));
    RC(make_rp(mem, cc, nS, &P->Coff.rp, &P->Coff.nnz, stmp, stmpb, s));
    RC(tmp.alloc(&Ah.ci, Ah.nnz));
    RC(tmp.alloc(&Ah.v, Ah.nnz));
    RC(mem.alloc(&P->Coff.ci, P->Coff.nnz));
    RC(mem.alloc(&P->Coff.v, P->Coff.nnz));
    RC(launch_extract_fill(A->d_row_ptr, A->d_col, A->d_val, n, nB, d_part, P->perm, P->iperm, Ah.rp, Ah.ci, Ah.v,
                           P->Coff.rp, P->Coff.ci, P->Coff.v, s));
  }

  // 5. factorization of the subdomain blocks
  const bool schur = opt->method == ILU_METHOD_SCHUR;
  std::vector<int64_t> as(nparts), al(nparts), bs(nparts), bl(nparts);
  for (int k = 0; k < nparts; k++) {
    as[k] = P->offsets[k];
    al[k] = P->offsets[k + 1] - P->offsets[k];
    bs[k] = P->offsets[nparts + 1 + k];
    bl[k] = P->offsets[nparts + 2 + k] - P->offsets[nparts + 1 + k];
  }
  Slots F;
  RC(run_factor(P, tmp, Ah, schur ? nB : n, opt->interior_fact, as, al, bs, bl, F, P->perm, 0, stmp, stmpb, s,
                "factorization"));
  int64_t *cnt_tmp;
  RC(tmp.alloc(&cnt_tmp, n + 1));
  // L1 = [L_B; W]: all rows, interior columns
  RC(slots_to_csr(mem, n, F.Lrp, F.Llen, F.Lc, F.Lv, 0, nB, 0, &P->L1, cnt_tmp, stmp, stmpb, s));
  // U1 = [U_B | Z]: interior rows, every column; Zb = the Z block alone
  RC(slots_to_csr(mem, nB, F.Urp, F.Ulen, F.Uc, F.Uv, 0, n, 0, &P->U1, cnt_tmp, stmp, stmpb, s));
  RC(slots_to_csr(mem, nB, F.Urp, F.Ulen, F.Uc, F.Uv, nB, n, 0, &P->Zb, cnt_tmp, stmp, stmpb, s));
  RC(mem.alloc(&P->DB, nB));
  if (nB) HIPCK(hipMemcpyAsync(P->DB, F.D, sizeof(double) * nB, hipMemcpyDeviceToDevice, s));
  RC(mem.alloc(&P->DS, nS));
  if (!schur) {
    RC(slots_to_csr(mem, nS, F.Lrp + nB, F.Llen + nB, F.Lc, F.Lv, nB, n, nB, &P->LS, cnt_tmp, stmp, stmpb, s));
    RC(slots_to_csr(mem, nS, F.Urp + nB, F.Ulen + nB, F.Uc, F.Uv, nB, n, nB, &P->US, cnt_tmp, stmp, stmpb, s));
    if (nS) HIPCK(hipMemcpyAsync(P->DS, F.D + nB, sizeof(double) * nS, hipMemcpyDeviceToDevice, s));
  } else if (nS > 0) {
    Csr St;
    RC(slots_to_csr(tmp, nS, F.Rrp, F.Rlen, F.Rc, F.Rv, nB, n, nB, &St, cnt_tmp, stmp, stmpb, s));
    std::vector<int64_t> sa(nparts), sl(nparts), sb(nparts, 0), sbl(nparts, 0);
    for (int k = 0; k < nparts; k++) {
      sa[k] = bs[k] - nB;
      sl[k] = bl[k];
    }
    Slots G;
    RC(run_factor(P, tmp, St, nS, opt->interface_fact, sa, sl, sb, sbl, G, P->perm, nB, stmp, stmpb, s,
                  "interface factorization"));
    RC(slots_to_csr(mem, nS, G.Lrp, G.Llen, G.Lc, G.Lv, 0, nS, 0, &P->LS, cnt_tmp, stmp, stmpb, s));
    RC(slots_to_csr(mem, nS, G.Urp, G.Ulen, G.Uc, G.Uv, 0, nS, 0, &P->US, cnt_tmp, stmp, stmpb, s));
    HIPCK(hipMemcpyAsync(P->DS, G.D, sizeof(double) * nS, hipMemcpyDeviceToDevice, s));
  } else {
    P->LS.n = P->US.n = 0;
  }

  // 6. level schedules of the four triangular solves
  {
    std::vector<int64_t> hb(3 * (nparts + 1));
    for (int k = 0; k <= nparts; k++) {
      hb[k] = P->offsets[k];
      hb[nparts + 1 + k] = P->offsets[nparts + 1 + k];
      hb[2 * (nparts + 1) + k] = P->offsets[nparts + 1 + k] - nB;
    }
    RC(mem.alloc(&P->blk_starts, (int64_t)hb.size()));
    HIPCK(hipMemcpyAsync(P->blk_starts, hb.data(), sizeof(int64_t) * hb.size(), hipMemcpyHostToDevice, s));
  }
  const int64_t *bs_int = P->blk_starts, *bs_ifc = P->blk_starts + (nparts + 1),
                *bs_loc = P->blk_starts + 2 * (nparts + 1);
  // the interior rows of L1 are swept; its W rows follow in one parallel pass
  Segs seg_l1{as, al, as, std::vector<int64_t>(nparts, 0)}, seg_u1{as, al, as, std::vector<int64_t>(nparts, 0)}, seg_s;
  for (int k = 0; k < nparts; k++) {
    seg_s.a_start.push_back(bs[k] - nB);
    seg_s.a_len.push_back(bl[k]);
    seg_s.b_start.push_back(0);
    seg_s.b_len.push_back(0);
  }
  RC(build_schedule(P, tmp, P->L1, true, 0, n, nB, P->sL1, seg_l1, s, "levels L"));
  RC(build_schedule(P, tmp, P->U1, false, 0, nB, nB, P->sU1, seg_u1, s, "levels U"));
  RC(build_schedule(P, tmp, P->LS, true, 0, nS, nS, P->sLS, seg_s, s, "levels L_S"));
  RC(build_schedule(P, tmp, P->US, false, 0, nS, nS, P->sUS, seg_s, s, "levels U_S"));
  // block-local solves for all four factors, or for none
  {
    const Schedule *all[4] = {&P->sL1, &P->sU1, &P->sLS, &P->sUS};
    bool ok = true;
    int64_t worst = 0;
    for (const Schedule *x : all)
      if (x->nrows > 0 && !x->block_ok) {
        ok = false;
        worst = std::max(worst, x->nlev);
      }
    const int mode = opt->trsv_mode;
    if (mode == ILU_TRSV_BLOCK && !ok)
      return fail(ILU_ERR_INVALID_ARG, "block-local solve needs <= 16384 levels per factor (has %lld)",
                  (long long)worst);
    // AUTO: block-local unless a subdomain is large AND its levels are wide
    // on average (beyond the 1024 threads of the widest workgroup); a level-
    // scheduled solve pays a cross-CU wait per level, one workgroup does not
    const int64_t nlev = std::max<int64_t>(std::max(P->sL1.nlev, P->sU1.nlev), 1);
    const bool narrow = n / nparts / nlev <= 1024;
    const bool want = mode == ILU_TRSV_BLOCK ||
                      (mode == ILU_TRSV_AUTO && (n / nparts <= ((int64_t)1 << 20) || narrow));
    P->block_mode = ok && want;
  }
  if (!P->block_mode) {
    RC(build_global(P, tmp, P->sL1, stmp, stmpb, s));
    RC(build_global(P, tmp, P->sU1, stmp, stmpb, s));
    RC(build_global(P, tmp, P->sLS, stmp, stmpb, s));
    RC(build_global(P, tmp, P->sUS, stmp, stmpb, s));
    if (P->opt.factor_prec != ILU_PREC_F64) {
      RC(build_lowp(P, P->sL1, P->L1, nullptr, INT64_MAX, s));
      RC(build_lowp(P, P->sU1, P->U1, P->DB, nB, s));
      RC(build_lowp(P, P->sLS, P->LS, nullptr, INT64_MAX, s));
      RC(build_lowp(P, P->sUS, P->US, P->DS, INT64_MAX, s));
    }
  } else {
    RC(build_block_interior(P, tmp, P->L1, P->sL1, bs_int, bs_ifc, nB, nullptr, INT64_MAX, false, s, "levels L"));
    RC(build_block_interior(P, tmp, P->U1, P->sU1, bs_int, nullptr, 0, P->DB, nB, true, s, "levels U"));
    int32_t *scomp = nullptr;
    int64_t ncomp = 0;
    RC(schur_components(P, tmp, &scomp, &ncomp, stmp, stmpb, s));
    if (ncomp > 0 && (uint64_t)ncomp * (uint64_t)std::max(P->sLS.nlev, P->sUS.nlev) < (1ull << 31)) {
      P->sLS.nblk = P->sUS.nblk = ncomp;
    } else {
      scomp = nullptr;
    }
    RC(build_block(P, tmp, P->US, P->sUS, bs_loc, nullptr, 0, P->DS, INT64_MAX, nullptr, s, "levels U_S", scomp));
    RC(build_block(P, tmp, P->LS, P->sLS, bs_loc, nullptr, 0, nullptr, INT64_MAX, P->sUS.pos, s, "levels L_S",
                   scomp));
    RC(build_block_flow(P, tmp, stmp, stmpb, s));
  }

  // 7. workspaces
  RC(mem.alloc(&P->xp, n));
  const bool rap = opt->method == ILU_METHOD_RAP;
  if (rap) {
    // the coarse operator R A P multiplies by A itself: keep a copy
    P->Acp.n = n;
    P->Acp.nnz = A->nnz;
    RC(mem.alloc(&P->Acp.rp, n + 1));
    RC(mem.alloc(&P->Acp.ci, A->nnz));
    RC(mem.alloc(&P->Acp.v, A->nnz));
    HIPCK(hipMemcpyAsync(P->Acp.rp, A->d_row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, s));
    if (A->nnz) {
      HIPCK(hipMemcpyAsync(P->Acp.ci, A->d_col, sizeof(int32_t) * A->nnz, hipMemcpyDeviceToDevice, s));
      HIPCK(hipMemcpyAsync(P->Acp.v, A->d_val, sizeof(double) * A->nnz, hipMemcpyDeviceToDevice, s));
    }
    RC(mem.alloc(&P->rx, n));
    RC(mem.alloc(&P->rw, n));
    RC(mem.alloc(&P->ru, n));
    RC(mem.alloc(&P->ry, nS));
  }
  if ((schur || rap) && nS > 0) {
    const int k = std::max(opt->inner_iters, 0);
    RC(mem.alloc(&P->iV, (int64_t)(k + 1) * nS));
    RC(mem.alloc(&P->iW, nS));
    RC(mem.alloc(&P->it1, nS));
    RC(mem.alloc(&P->it2, nS));
    RC(mem.alloc(&P->iH, (int64_t)(k + 1) * (k + 1)));
    RC(mem.alloc(&P->ics, k + 1));
    RC(mem.alloc(&P->isn, k + 1));
    RC(mem.alloc(&P->ig, k + 2));
    RC(mem.alloc(&P->ic, k + 1));
    RC(mem.alloc(&P->ipa, RED_BLOCKS));
    RC(mem.alloc(&P->ipb, RED_BLOCKS));
    RC(mem.alloc(&P->iscal, 8));
    RC(mem.alloc(&P->iflags, 4));
    RC(mem.alloc(&P->islots, arnoldi_slots(std::max(k, 1))));
    RC(launch_arnoldi_reset(P->islots, std::max(k, 1), s));
    P->ilaunch = 0;
  }
  HIPCK(hipStreamSynchronize(s));
  tmp.release(false);  // the stream has finished with the temporaries
  return 0;
}

int ilu_setup(const ilu_csr_t *A, const int32_t *d_part, int32_t nparts, const ilu_options_t *opt_in, void *stream,
              ilu_precond_t **out) {
  if (!out) return fail(ILU_ERR_INVALID_ARG, "P must not be NULL");
  *out = nullptr;
  if (!A || A->n < 0 || A->nnz < 0) return fail(ILU_ERR_INVALID_ARG, "invalid matrix descriptor");
  if (A->n > 0 && (!A->d_row_ptr || !A->d_col || !A->d_val)) return fail(ILU_ERR_INVALID_ARG, "NULL matrix array");
  if (A->n >= 0x7fffffff || A->nnz >= ((int64_t)1 << 40)) return fail(ILU_ERR_INVALID_ARG, "matrix too large");
  if (nparts < 1 || (!d_part && nparts != 1)) return fail(ILU_ERR_INVALID_ARG, "nparts must be >= 1 (1 without part)");
  ilu_options_t opt;
  ilu_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (opt.method != ILU_METHOD_BJ && opt.method != ILU_METHOD_SCHUR && opt.method != ILU_METHOD_RAP)
    return fail(ILU_ERR_INVALID_ARG, "unknown method %d", opt.method);
  for (int f : {opt.interior_fact, opt.interface_fact, opt.smooth_fact})
    if (f != ILU_FACT_ILU0 && f != ILU_FACT_MILU0 && f != ILU_FACT_ILUT)
      return fail(ILU_ERR_INVALID_ARG, "unknown factorization %d", f);
  if (opt.inner_iters < 0 || opt.inner_iters > 1000) return fail(ILU_ERR_INVALID_ARG, "inner_iters out of range");
  if (!(opt.droptol >= 0.0) || !(opt.inner_rtol >= 0.0) || !(opt.pivot_tol >= 0.0))
    return fail(ILU_ERR_INVALID_ARG, "negative tolerance");
  if (opt.factor_prec < ILU_PREC_F64 || opt.factor_prec > ILU_PREC_F16)
    return fail(ILU_ERR_INVALID_ARG, "factor_prec must be ILU_PREC_F64, ILU_PREC_F32 or ILU_PREC_F16");
  if (opt.trsv_mode < ILU_TRSV_AUTO || opt.trsv_mode > ILU_TRSV_BLOCK)
    return fail(ILU_ERR_INVALID_ARG, "unknown trsv_mode %d", opt.trsv_mode);
  if (opt.arnoldi_mode != ILU_ARNOLDI_AUTO && opt.arnoldi_mode != ILU_ARNOLDI_PER_PASS)
    return fail(ILU_ERR_INVALID_ARG, "unknown arnoldi_mode %d", opt.arnoldi_mode);
  if (opt.block_split < 0 || opt.block_split > 64)
    return fail(ILU_ERR_INVALID_ARG, "block_split must be in [0, 64] (is %d)", opt.block_split);
  hipStream_t s = (hipStream_t)stream;
  ilu_precond *P = new ilu_precond();
  P->n = A->n;
  P->nparts = nparts;
  P->opt = opt;
  P->arnoldi_coop = opt.arnoldi_mode == ILU_ARNOLDI_AUTO;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    delete P;
    return fail(ILU_ERR_HIP, "hipEventCreate failed");
  }
  (void)hipEventRecord(e0, s);
  int rc = setup_impl(A, d_part, nparts, &opt, s, P);
  if (rc == 0 && opt.method == ILU_METHOD_RAP) {
    // the smoother: block Jacobi on the same subdomains with smooth_fact
    ilu_options_t so = opt;
    so.method = ILU_METHOD_BJ;
    so.interior_fact = opt.smooth_fact;
    P->smoother = new ilu_precond();
    P->smoother->n = A->n;
    P->smoother->nparts = nparts;
    P->smoother->opt = so;
    rc = setup_impl(A, d_part, nparts, &so, s, P->smoother);
  }
  (void)hipEventRecord(e1, s);
  if (rc == 0) {
    float ms = 0.f;
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(&ms, e0, e1);
    P->setup_ms = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    (void)hipStreamSynchronize(s);
    ilu_destroy(P);
    return rc;
  }
  *out = P;
  return 0;
}



void ilu_destroy(ilu_precond_t *P) {
  if (!P) return;
  (void)hipSetDevice(P->device);
  delete P;
}

// The sum slots of the one-launch orthogonalisation start empty with every
// solve and apply (a launch that gave up on a wait leaves some behind).
static int reset_arnoldi(ilu_precond *P, KrylovBufs *w, hipStream_t s) {
  if (w && w->aslots && P->arnoldi_coop) {
    RC(launch_arnoldi_reset(w->aslots, w->m, s));
    w->alaunch = 0;
  }
  if (P->islots && P->arnoldi_coop) {
    RC(launch_arnoldi_reset(P->islots, std::max(P->opt.inner_iters, 1), s));
    P->ilaunch = 0;
  }
  return 0;
}

// Orthogonalisation of Arnoldi step j: w (or a + b, stored to w, when a is
// given) minus its modified Gram-Schmidt projections on v_0..v_j (v_i at
// V + i n), H column j to hcol, and the partials of <w, w> for the Givens
// step (*pnorm; *npart of them, 0 meaning a per-pass reduction's count).
// One launch per step when the handle allows it and the vectors fit,
// else a dot pass (fused with the sum) and one launch per MGS pass.
// kind >= 0: the launches are timed as that kernel class.
static int orthogonalize(ilu_precond *P, double *w, const double *a, const double *b, const double *V, int64_t n,
                         int j, double *hcol, double *pa, double *pb, unsigned long long *slots, int passes,
                         unsigned long long *launches, int *stop, int kind, hipStream_t s, double **pnorm,
                         int *npart) {
  auto run = [&](double bytes, auto &&f) -> int { return kind >= 0 ? timed(kind, bytes, s, f) : f(); };
  if (P->arnoldi_coop && slots && arnoldi_fits(n, w, a, b, V, P->num_cu)) {
    ArnoldiOut o;
    // v_0..v_j, w (or a and b) read, w written
    const double bytes = 8.0 * (double)n * (double)(j + 3 + (a ? 1 : 0));
    RC(run(bytes, [&] {
      return launch_arnoldi(w, a, b, V, n, j, hcol, slots, passes, launches, pa, P->num_cu, P->status, &o, s);
    }));
    if (o.done) {
      *pnorm = o.pnorm;
      *npart = o.npart;
      return 0;
    }
  }
  double *pc = pa, *pn = pb;
  if (a)
    RC(launch_sum_dot(w, a, b, V, n, pc, s));
  else
    RC(launch_dot_partial(w, V, n, pc, s));
  for (int i = 0; i <= j; i++) {
    const double *vnext = i < j ? V + (int64_t)(i + 1) * n : nullptr;
    RC(run(32.0 * (double)n, [&] { return launch_mgs_step(w, V + (int64_t)i * n, pc, hcol + i, vnext, n, pn, stop, s); }));
    std::swap(pc, pn);
  }
  *pnorm = pc;
  *npart = 0;
  return 0;
}

// y = the reduced-system GMRES approximation for rhs g' (both in interface numbering)
static int inner_gmres(ilu_precond *P, const double *gp, double *y, hipStream_t s) {
  const int64_t nS = P->nS;
  const int k = P->opt.inner_iters;
  double *V = P->iV;
  RC(trsv_schur(P, gp, V, s));
  if (k == 0) return launch_copy(V, y, nS, s);
  double *beta = P->iscal, *hn = P->iscal + 1, *est = P->iscal + 2;
  int *stop = P->iflags, *nsteps = P->iflags + 1;
  const int ldh = k + 1;
  RC(launch_dot_partial(V, V, nS, P->ipa, s));
  RC(launch_reduce_final(P->ipa, nS, beta, s));
  RC(launch_init_krylov(P->ig, beta, stop, nsteps, s));
  RC(launch_scale_copy(V, nullptr, beta, V, nS, nullptr, s));
  // C_off (in block mode its rows are in L_S order, its columns in U_S order)
  const Csr &C = P->block_mode ? P->Coffr : P->Coff;
  // C_off v_0; later products come with the normalisation of the step before
  RC(timed(ILU_K_SPMV_COFF, spmv_bytes(nS, C.nnz, false), s,
           [&] { return launch_spmv(C.rp, C.ci, C.v, nS, V, P->it1, s, SPMV_COFF); }));
  double *w = P->iW;  // the new direction, orthogonalised apart from the basis
  for (int j = 0; j < k; j++) {
    double *vj = V + (int64_t)j * nS, *vn = V + (int64_t)(j + 1) * nS;
    RC(trsv_schur(P, P->it1, P->it2, s));
    // w = v_j + D^-1 C_off v_j, orthogonalised against v_0..v_j
    double *pc = nullptr;
    int np = 0;
    RC(orthogonalize(P, w, vj, P->it2, V, nS, j, P->iH + (int64_t)ldh * j, P->ipa, P->ipb, P->islots, k,
                     &P->ilaunch, stop, -1, s, &pc, &np));
    if (j + 1 < k) {
      // v_{j+1} = w / ||w|| and C_off v_{j+1} in one launch
      RC(timed(ILU_K_SPMV_COFF, spmv_bytes(nS, C.nnz, false) + 16.0 * (double)nS, s, [&] {
        return launch_givens_scale_spmv(P->iH, ldh, P->ics, P->isn, P->ig, j, pc, stop, nsteps, est, hn, beta,
                                        P->opt.inner_rtol, w, vn, nS, C.rp, C.ci, C.v, P->it1, s, np);
      }));
    } else {
      RC(launch_givens_scale(P->iH, ldh, P->ics, P->isn, P->ig, j, pc, stop, nsteps, est, hn, beta,
                             P->opt.inner_rtol, w, nS, s, np));
    }
  }
  RC(launch_backsolve(P->iH, ldh, P->ig, nsteps, P->ic, s));
  return launch_combine(y, V, nS, P->ic, nsteps, nS, false, s);
}

// z = M^-1 r with the block-local solves (orders as in ilu_precond)
static int apply_block(ilu_precond *P, const double *r, double *z, hipStream_t s) {
  const int64_t nB = P->nB, nS = P->nS;
  // f' = L_B^-1 r_B, then g' = r_S - W f' in L_S position order
  RC(launch_gather(r, P->gmapL, nB, P->bL, s));
  RC(trsv(P, P->sL1, P->L1, nullptr, 0, P->bL, nullptr, P->fL, nullptr, nullptr, s, 0, [&] {
    return launch_rows_lower(P->Wr.rp, P->Wr.ci, P->Wr.v, nS, r, P->gmapW, P->fL, P->gS, s);
  }));
  if (nS > 0) {
    if (P->opt.method == ILU_METHOD_SCHUR) {
      RC(inner_gmres(P, P->gS, P->yS, s));
    } else {
      RC(trsv_schur(P, P->gS, P->yS, s));
    }
  }
  // f'' = f' - Z y in U_B position order, u = U_B^-1 f'', then both halves to z
  RC(launch_upper_rhs(P->fmapU, nB, P->fL, P->Zr.rp, P->Zr.ci, P->Zr.v, P->yS, P->bU, s));
  RC(trsv(P, P->sU1, P->U1, P->DB, nB, P->bU, nullptr, P->uU, nullptr, nullptr, s, 1));
  return launch_finish(P->uU, P->finB, nB, P->yS, P->finS, nS, nullptr, z, s);
}

// ---- multiplicative two-level method (Section 3.3) ----
// out = R A P v with R = (-W L_B^-1, I) and P = (-U_B^-1 Z; I) unformed
// (eq. (28)): a U_B solve with the Z columns, the product with A, an L_B
// solve with the W rows.  Block mode: v in U_S position order, out in L_S
// position order (the orders of the reduced-system vectors); level-scheduled
// mode: both in the interface numbering.  Uses xp, bL, fL, bU, uU, ru, rw.
static int rap_product(ilu_precond *P, const double *v, double *out, hipStream_t s) {
  const int64_t n = P->n, nB = P->nB, nS = P->nS;
  const Csr &A = P->Acp;
  auto product = [&] {
    return timed(ILU_K_SPMV, spmv_bytes(n, A.nnz, false), s,
                 [&] { return launch_spmv(A.rp, A.ci, A.v, n, P->ru, P->rw, s, SPMV_A); });
  };
  if (P->block_mode) {
    // P v: u = -U_B^-1 Z v in U_B order, then (u; v) in A's numbering
    RC(launch_upper_rhs(P->fmapU, nB, nullptr, P->Zr.rp, P->Zr.ci, P->Zr.v, v, P->bU, s));
    RC(trsv(P, P->sU1, P->U1, P->DB, nB, P->bU, nullptr, P->uU, nullptr, nullptr, s, 1));
    RC(launch_finish(P->uU, P->finB, nB, v, P->finS, nS, nullptr, P->ru, s));
    RC(product());
    // R w = w_S - W L_B^-1 w_B, in L_S order
    RC(launch_gather(P->rw, P->gmapL, nB, P->bL, s));
    return trsv(P, P->sL1, P->L1, nullptr, 0, P->bL, nullptr, P->fL, nullptr, nullptr, s, 0, [&] {
      return launch_rows_lower(P->Wr.rp, P->Wr.ci, P->Wr.v, nS, P->rw, P->gmapW, P->fL, out, s);
    });
  }
  // the U solve of [U_B | Z] with a zero interior right-hand side and v in
  // the interface slots gives -U_B^-1 Z v; both halves land in ru
  double *xp = P->xp;
  RC(fill_f64(xp, 0.0, nB, s));
  RC(launch_copy(v, xp + nB, nS, s));
  RC(launch_scatter(v, P->perm + nB, nS, P->ru, s));
  RC(trsv(P, P->sU1, P->U1, P->DB, nB, xp, nullptr, xp, P->ru, P->perm, s, 1));
  RC(product());
  // [L_B; W] in one pass: xp_B = L_B^-1 w_B, xp_S = w_S - W xp_B
  RC(trsv(P, P->sL1, P->L1, nullptr, 0, P->rw, P->perm, xp, nullptr, nullptr, s, 0));
  return launch_copy(xp + nB, out, nS, s);
}

// k GMRES steps on (L_S U_S)^-1 R A P v = (L_S U_S)^-1 g (zero initial guess,
// modified Gram-Schmidt, Givens; the early exits of inner_gmres), y = v
static int inner_gmres_rap(ilu_precond *P, const double *gp, double *y, hipStream_t s) {
  const int64_t nS = P->nS;
  const int k = P->opt.inner_iters;
  double *V = P->iV;
  RC(trsv_schur(P, gp, V, s));
  if (k == 0) return launch_copy(V, y, nS, s);
  double *beta = P->iscal, *hn = P->iscal + 1, *est = P->iscal + 2;
  int *stop = P->iflags, *nsteps = P->iflags + 1;
  const int ldh = k + 1;
  RC(launch_dot_partial(V, V, nS, P->ipa, s));
  RC(launch_reduce_final(P->ipa, nS, beta, s));
  RC(launch_init_krylov(P->ig, beta, stop, nsteps, s));
  RC(launch_scale_copy(V, nullptr, beta, V, nS, nullptr, s));
  for (int j = 0; j < k; j++) {
    double *vj = V + (int64_t)j * nS, *w = V + (int64_t)(j + 1) * nS;
    RC(rap_product(P, vj, P->it1, s));
    RC(trsv_schur(P, P->it1, w, s));
    double *pc = nullptr;
    int np = 0;
    RC(orthogonalize(P, w, nullptr, nullptr, V, nS, j, P->iH + (int64_t)ldh * j, P->ipa, P->ipb, P->islots, k,
                     &P->ilaunch, stop, -1, s, &pc, &np));
    RC(launch_givens_scale(P->iH, ldh, P->ics, P->isn, P->ig, j, pc, stop, nsteps, est, hn, beta,
                           P->opt.inner_rtol, w, nS, s, np));
  }
  RC(launch_backsolve(P->iH, ldh, P->ig, nsteps, P->ic, s));
  return launch_combine(y, V, nS, P->ic, nsteps, nS, false, s);
}

static int apply_impl(ilu_precond *P, const double *r, double *z, hipStream_t s);

// x = the smoother's solve of r; g = R (r - A x); v from inner_gmres_rap;
// z = x + P v
static int apply_rap(ilu_precond *P, const double *r, double *z, hipStream_t s) {
  const int64_t n = P->n, nB = P->nB, nS = P->nS;
  const Csr &A = P->Acp;
  RC(apply_impl(P->smoother, r, P->rx, s));
  if (nS == 0) return launch_copy(P->rx, z, n, s);
  RC(launch_residual(A.rp, A.ci, A.v, n, r, P->rx, P->rw, s));
  if (P->block_mode) {
    RC(launch_gather(P->rw, P->gmapL, nB, P->bL, s));
    RC(trsv(P, P->sL1, P->L1, nullptr, 0, P->bL, nullptr, P->fL, nullptr, nullptr, s, 0, [&] {
      return launch_rows_lower(P->Wr.rp, P->Wr.ci, P->Wr.v, nS, P->rw, P->gmapW, P->fL, P->gS, s);
    }));
    RC(inner_gmres_rap(P, P->gS, P->yS, s));
    RC(launch_upper_rhs(P->fmapU, nB, nullptr, P->Zr.rp, P->Zr.ci, P->Zr.v, P->yS, P->bU, s));
    RC(trsv(P, P->sU1, P->U1, P->DB, nB, P->bU, nullptr, P->uU, nullptr, nullptr, s, 1));
    return launch_finish(P->uU, P->finB, nB, P->yS, P->finS, nS, P->rx, z, s);
  }
  double *xp = P->xp;
  RC(trsv(P, P->sL1, P->L1, nullptr, 0, P->rw, P->perm, xp, nullptr, nullptr, s, 0));
  RC(inner_gmres_rap(P, xp + nB, P->ry, s));
  RC(fill_f64(xp, 0.0, nB, s));
  RC(launch_copy(P->ry, xp + nB, nS, s));
  RC(launch_scatter(P->ry, P->perm + nB, nS, z, s));
  RC(trsv(P, P->sU1, P->U1, P->DB, nB, xp, nullptr, xp, z, P->perm, s, 1));
  return launch_add(P->rx, z, n, s);
}

static int apply_impl(ilu_precond *P, const double *r, double *z, hipStream_t s) {
  const int64_t n = P->n, nB = P->nB, nS = P->nS;
  if (n == 0) return 0;
  if (P->opt.method == ILU_METHOD_RAP) return apply_rap(P, r, z, s);
  if (P->block_mode) return apply_block(P, r, z, s);
  double *xp = P->xp;
  // f' = L_B^-1 r[perm_B] and g' = r[perm_S] - W f' in one level-scheduled pass
  RC(trsv(P, P->sL1, P->L1, nullptr, 0, r, P->perm, xp, nullptr, nullptr, s, 0));
  if (nS > 0) {
    double *gp = xp + nB;
    if (P->opt.method == ILU_METHOD_SCHUR) {
      RC(inner_gmres(P, gp, gp, s));
    } else {
      RC(trsv_schur(P, gp, gp, s));
    }
    RC(launch_scatter(gp, P->perm + nB, nS, z, s));
  }
  // u = U_B^-1 (f' - Z y), scattered to z
  RC(trsv(P, P->sU1, P->U1, P->DB, nB, xp, nullptr, xp, z, P->perm, s, 1));
  return 0;
}

int ilu_apply(ilu_precond_t *P, const double *d_r, double *d_z, void *stream) {
  if (!P || (P->n > 0 && (!d_r || !d_z))) return fail(ILU_ERR_INVALID_ARG, "NULL argument");
  if (d_r == d_z && P->n > 0) return fail(ILU_ERR_INVALID_ARG, "r and z must not alias");
  HIPCK(hipSetDevice(P->device));
  RC(reset_arnoldi(P, nullptr, (hipStream_t)stream));
  return apply_impl(P, d_r, d_z, (hipStream_t)stream);
}

int ilu_rap_matvec(ilu_precond_t *P, const double *d_v, double *d_out, void *stream) {
  if (!P || P->opt.method != ILU_METHOD_RAP) return fail(ILU_ERR_INVALID_ARG, "ilu_rap_matvec needs a RAP handle");
  if (P->nS == 0) return 0;
  if (!d_v || !d_out) return fail(ILU_ERR_INVALID_ARG, "NULL argument");
  if (d_v == d_out) return fail(ILU_ERR_INVALID_ARG, "v and out must not alias");
  HIPCK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  const int64_t nS = P->nS;
  if (!P->block_mode) return rap_product(P, d_v, d_out, s);
  // interface numbering to the U_S position order and back from L_S order
  RC(launch_gather(d_v, P->sUS.blk_rows, nS, P->yS, s));
  RC(rap_product(P, P->yS, P->gS, s));
  return launch_scatter(P->gS, P->sLS.blk_rows, nS, d_out, s);
}

int csr_spmv(const ilu_csr_t *A, const double *d_x, double *d_y, void *stream) {
  if (!A || A->n < 0 || (A->n > 0 && (!d_x || !d_y || !A->d_row_ptr || !A->d_col || !A->d_val)))
    return fail(ILU_ERR_INVALID_ARG, "invalid arguments");
  return launch_spmv(A->d_row_ptr, A->d_col, A->d_val, A->n, d_x, d_y, (hipStream_t)stream);
}

static int read_scalars(ilu_precond *P, const double *d, int cnt, hipStream_t s) {
  HIPCK(hipMemcpyAsync(P->host_pinned, d, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  return 0;
}

// Krylov workspace of FGMRES(m) on vectors of length n; n and m are set
// last, so a partly built workspace never passes for a complete one.
static int gmres_work_alloc(GmresWork &w, int64_t n, int m) {
  RC(w.mem.alloc(&w.V, (int64_t)(m + 1) * n));
  RC(w.mem.alloc(&w.Zb, (int64_t)m * n));
  RC(w.mem.alloc(&w.r, n));
  RC(w.mem.alloc(&w.H, (int64_t)(m + 1) * (m + 1)));
  RC(w.mem.alloc(&w.cs, m + 1));
  RC(w.mem.alloc(&w.sn, m + 1));
  RC(w.mem.alloc(&w.g, m + 2));
  RC(w.mem.alloc(&w.c, m + 1));
  RC(w.mem.alloc(&w.pa, RED_BLOCKS));
  RC(w.mem.alloc(&w.pb, RED_BLOCKS));
  RC(w.mem.alloc(&w.scal, 8));
  RC(w.mem.alloc(&w.flags, 4));
  RC(w.mem.alloc(&w.aslots, arnoldi_slots(m)));
  for (hipEvent_t &e : w.ev) HIPCK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  w.n = n;
  w.m = m;
  return 0;
}

static int fgmres_core(const ilu_csr_t *A, ilu_precond *P, KrylovBufs &w, const double *b, double *x, double rtol,
                       int m, int maxit, hipStream_t s, ilu_result_t *res, double *hist);

static int fgmres_impl(const ilu_csr_t *A, ilu_precond *P, const double *b, double *x, double rtol, int m, int maxit,
                       hipStream_t s, ilu_result_t *res, double *hist) {
  const int64_t n = A->n;
  if (!P->gw || P->gw->n != n || P->gw->m != m) {
    // The sizes are recorded only once every buffer and event exists: a
    // workspace left behind by a failed allocation is dropped, never reused.
    delete P->gw;
    P->gw = nullptr;
    GmresWork *nw = new GmresWork();
    const int rc = gmres_work_alloc(*nw, n, m);
    if (rc) {
      delete nw;
      return rc;
    }
    P->gw = nw;
  }
  return fgmres_core(A, P, *P->gw, b, x, rtol, m, maxit, s, res, hist);
}

static int fgmres_core(const ilu_csr_t *A, ilu_precond *P, KrylovBufs &w, const double *b, double *x, double rtol,
                       int m, int maxit, hipStream_t s, ilu_result_t *res, double *hist) {
  const int64_t n = A->n;
  double *bnorm = w.scal, *beta = w.scal + 1, *hn = w.scal + 2, *est = w.scal + 3;
  int *stop = w.flags, *nsteps = w.flags + 1;
  const int ldh = m + 1;
  const int64_t *rp = A->d_row_ptr;
  const int32_t *ci = A->d_col;
  const double *av = A->d_val;
  int its = 0, converged = 0;
  double relres = 0.0;

  RC(reset_arnoldi(P, &w, s));
  RC(launch_dot_partial(b, b, n, w.pa, s));
  RC(launch_reduce_final(w.pa, n, bnorm, s));
  RC(read_scalars(P, bnorm, 1, s));
  const double hb = P->host_pinned[0];
  if (!std::isfinite(hb)) return fail(ILU_ERR_BREAKDOWN, "non-finite ||b||");
  if (hb == 0.0) {
    RC(fill_f64(x, 0.0, n, s));
    HIPCK(hipStreamSynchronize(s));
    if (hist) hist[0] = 0.0;
    converged = 1;
  } else {
    RC(launch_residual(rp, ci, av, n, b, x, w.r, s));
    RC(launch_dot_partial(w.r, w.r, n, w.pa, s));
    RC(launch_reduce_final(w.pa, n, beta, s));
    RC(read_scalars(P, beta, 1, s));
    double hbeta = P->host_pinned[0];
    relres = hbeta / hb;
    if (hist) hist[0] = relres;
    if (!std::isfinite(hbeta)) return fail(ILU_ERR_BREAKDOWN, "non-finite initial residual");
    if (hbeta <= rtol * hb) converged = 1;
    while (!converged && its < maxit) {
      RC(launch_scale_copy(w.r, nullptr, beta, w.V, n, nullptr, s));
      RC(launch_init_krylov(w.g, beta, stop, nsteps, s));
      // Step j is enqueued before the estimate and stop word of step j - 1
      // are read back (two pinned slots, one event each), so the host round
      // trip overlaps step j.  A step enqueued after one that stopped leaves
      // H, g and nsteps alone (the Givens kernel sees the stop word); no step
      // is enqueued beyond maxit.
      double *hest = P->host_pinned + 2;                          // [2] estimates
      int *hflag = reinterpret_cast<int *>(P->host_pinned + 4);  // [2] stop words
      int pending = -1;  // slot of the step whose results are not read yet
      bool cycle_done = false;
      auto consume = [&](int slot) -> int {
        if (w.ev[slot]) {
          HIPCK(hipEventSynchronize(w.ev[slot]));
        } else {
          HIPCK(hipStreamSynchronize(s));
        }
        its++;
        if (g_timing) timing_collect();
        if (hist) hist[its] = hest[slot] / hb;
        if (hflag[slot] == 3) return fail(ILU_ERR_BREAKDOWN, "non-finite value in the Arnoldi process at step %d", its);
        if (hflag[slot] || its >= maxit) cycle_done = true;
        return 0;
      };
      for (int j = 0; j < m && !cycle_done; j++) {
        if (its + (pending >= 0 ? 1 : 0) >= maxit) break;
        double *vj = w.V + (int64_t)j * n, *wv = w.V + (int64_t)(j + 1) * n, *zj = w.Zb + (int64_t)j * n;
        RC(apply_impl(P, vj, zj, s));
        RC(timed(ILU_K_SPMV, spmv_bytes(n, A->nnz, false), s, [&] { return launch_spmv(rp, ci, av, n, zj, wv, s, SPMV_A); }));
        double *pc = nullptr;
        int np = 0;
        RC(orthogonalize(P, wv, nullptr, nullptr, w.V, n, j, w.H + (int64_t)ldh * j, w.pa, w.pb, w.aslots, m,
                         &w.alaunch, stop, ILU_K_MGS, s, &pc, &np));
        RC(launch_givens_scale(w.H, ldh, w.cs, w.sn, w.g, j, pc, stop, nsteps, est, hn, bnorm, rtol, wv, n, s, np));
        const int slot = j & 1;
        HIPCK(hipMemcpyAsync(hest + slot, est, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCK(hipMemcpyAsync(hflag + slot, stop, sizeof(int), hipMemcpyDeviceToHost, s));
        if (!w.ev[slot]) {  // no events: read this step's results now
          RC(consume(slot));
          continue;
        }
        HIPCK(hipEventRecord(w.ev[slot], s));
        if (pending >= 0) RC(consume(pending));
        pending = slot;
      }
      if (pending >= 0 && !cycle_done) RC(consume(pending));
      RC(launch_backsolve(w.H, ldh, w.g, nsteps, w.c, s));
      RC(launch_combine(x, w.Zb, n, w.c, nsteps, n, true, s));
      RC(launch_residual(rp, ci, av, n, b, x, w.r, s));
      RC(launch_dot_partial(w.r, w.r, n, w.pa, s));
      RC(launch_reduce_final(w.pa, n, beta, s));
      RC(read_scalars(P, beta, 1, s));
      hbeta = P->host_pinned[0];
      relres = hbeta / hb;
      if (!std::isfinite(hbeta)) return fail(ILU_ERR_BREAKDOWN, "non-finite residual");
      if (hbeta <= rtol * hb) converged = 1;
    }
  }
  RC(check_status(P, s, "solve", nullptr, 0));
  if (res) {
    res->iterations = its;
    res->converged = converged;
    res->final_relres = relres;
  }
  return converged ? ILU_OK : ILU_NOT_CONVERGED;
}

int fgmres_solve(const ilu_csr_t *A, ilu_precond_t *P, const double *d_b, double *d_x, double rtol, int32_t restart,
                 int32_t maxit, void *stream, ilu_result_t *res, double *h_hist) {
  if (!A || !P || A->n != P->n) return fail(ILU_ERR_INVALID_ARG, "matrix and preconditioner sizes differ");
  if (A->n > 0 && (!d_b || !d_x)) return fail(ILU_ERR_INVALID_ARG, "NULL vector");
  if (restart < 1 || restart > 1000 || maxit < 0 || !(rtol >= 0.0))
    return fail(ILU_ERR_INVALID_ARG, "restart/maxit/rtol out of range");
  HIPCK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIPCK(hipEventCreate(&e0));
  HIPCK(hipEventCreate(&e1));
  (void)hipEventRecord(e0, s);
  int rc = fgmres_impl(A, P, d_b, d_x, rtol, restart, maxit, s, res, h_hist);
  (void)hipEventRecord(e1, s);
  float ms = 0.f;
  (void)hipEventSynchronize(e1);
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (res) {
    res->setup_ms = P->setup_ms;
    res->solve_ms = ms;
  }
  return rc;
}

// ---------------------------------------------------------------------------
// FGMRES with no allocation: the Krylov workspace lives in one fixed device
// array per GPU instead of blocks allocated on the first call.
// ---------------------------------------------------------------------------
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
// Host code must not use this name as a device address: the address of each
// device's copy comes from hipGetSymbolAddress (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Address of the current device's copy of `scratch` (looked up once per device).
static int noalloc_scratch(int dev, char **out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(ILU_ERR_INVALID_ARG, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ILU_ERR_HIP, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = (char *)g_scratch_ptr[dev];
  return 0;
}

// Carve the buffers of fgmres_core from `base` (256-byte aligned pieces);
// with base == nullptr only the size is computed.  No events: each step's
// results are read back synchronously.
static size_t noalloc_layout(char *base, int64_t n, int m, KrylovBufs &w) {
  size_t off = 0;
  auto take = [&](size_t count, size_t es) -> char * {
    off = (off + 255) & ~(size_t)255;
    char *p = base ? base + off : nullptr;
    off += std::max<size_t>(count, 1) * es;
    return p;
  };
  w.V = (double *)take((size_t)(m + 1) * (size_t)n, 8);
  w.Zb = (double *)take((size_t)m * (size_t)n, 8);
  w.r = (double *)take((size_t)n, 8);
  w.H = (double *)take((size_t)(m + 1) * (size_t)(m + 1), 8);
  w.cs = (double *)take((size_t)m + 1, 8);
  w.sn = (double *)take((size_t)m + 1, 8);
  w.g = (double *)take((size_t)m + 2, 8);
  w.c = (double *)take((size_t)m + 1, 8);
  w.pa = (double *)take(RED_BLOCKS, 8);
  w.pb = (double *)take(RED_BLOCKS, 8);
  w.scal = (double *)take(8, 8);
  w.flags = (int *)take(4, sizeof(int));
  w.aslots = (unsigned long long *)take((size_t)arnoldi_slots(m), sizeof(unsigned long long));
  w.n = n;
  w.m = m;
  w.ev[0] = w.ev[1] = nullptr;
  return off;
}

int fgmres_solve_noalloc(const ilu_csr_t *A, ilu_precond_t *P, const double *d_b, double *d_x, double rtol,
                         int32_t restart, int32_t maxit, void *stream, ilu_result_t *res, double *h_hist) {
  if (!A || !P || A->n != P->n) return fail(ILU_ERR_INVALID_ARG, "matrix and preconditioner sizes differ");
  if (A->n > 0 && (!d_b || !d_x)) return fail(ILU_ERR_INVALID_ARG, "NULL vector");
  if (restart < 1 || restart > 1000 || maxit < 0 || !(rtol >= 0.0))
    return fail(ILU_ERR_INVALID_ARG, "restart/maxit/rtol out of range");
  if (g_timing)
    return fail(ILU_ERR_INVALID_ARG, "kernel timing creates HIP events: switch it off for the allocation-free solve");
  KrylovBufs w;
  const size_t need = noalloc_layout(nullptr, A->n, restart, w);
  if (need > NOALLOC_BYTES)
    return fail(ILU_ERR_CAPACITY,
                "allocation-free FGMRES(%d) on n = %lld needs %zu bytes of workspace; the fixed array holds %zu "
                "((2 restart + 2) n doubles must stay below it)",
                restart, (long long)A->n, need, NOALLOC_BYTES);
  HIPCK(hipSetDevice(P->device));
  char *base = nullptr;
  RC(noalloc_scratch(P->device, &base));
  noalloc_layout(base, A->n, restart, w);
  hipStream_t s = (hipStream_t)stream;
  const auto t0 = std::chrono::steady_clock::now();
  const int rc = fgmres_core(A, P, w, d_b, d_x, rtol, restart, maxit, s, res, h_hist);
  HIPCK(hipStreamSynchronize(s));
  if (res) {
    res->setup_ms = P->setup_ms;
    res->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return rc;
}

void ilu_memory_trim(void) {
  timing_collect();
  for (hipEvent_t e : g_event_pool) (void)hipEventDestroy(e);
  g_event_pool.clear();
  cache_trim();
}

void ilu_kernel_timing(int32_t classes) {
  if (!classes) timing_collect();
  g_timing = (uint32_t)classes & (uint32_t)ILU_K_ALL;
}

int ilu_kernel_stats(int32_t kind, double *total_ms, int64_t *launches, double *bytes, int32_t reset) {
  if (kind < 0 || kind >= ILU_K_COUNT) return fail(ILU_ERR_INVALID_ARG, "unknown kernel class %d", kind);
  timing_collect();
  if (total_ms) *total_ms = g_kstat[kind].ms;
  if (launches) *launches = g_kstat[kind].launches;
  if (bytes) *bytes = g_kstat[kind].bytes;
  if (reset) g_kstat[kind] = KStat();
  return 0;
}

int ilu_info(ilu_precond_t *P, int64_t *n, int64_t *nB, int64_t *nS, int32_t *nparts) {
  if (!P) return fail(ILU_ERR_INVALID_ARG, "NULL handle");
  if (n) *n = P->n;
  if (nB) *nB = P->nB;
  if (nS) *nS = P->nS;
  if (nparts) *nparts = P->nparts;
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched systems: ILU(0) + GMRES(m) of many independent systems in one
// persistent launch (batch.hip).  Setup analyses the pattern once: levels of
// A's strict lower and upper parts per system (the level sweep of the
// single-system setup, with one segment per system), the (system, level)
// sorted positions of both solves and their ring slots, and a largest-first
// order of the systems.  A solve is one reset kernel and the persistent
// kernel, with no host synchronisation: it can be captured in a HIP graph.
// ---------------------------------------------------------------------------
static int export_raw(const void *d, int64_t cnt, size_t es, void *h, int64_t *len);

struct ilu_batch {
  ilu_precond core;  // device memory, status word, CU count, level sweeps
  int32_t nsys = 0;
  int64_t n = 0, nnz = 0;
  int E = 2, m_alloc = 0, merge = 32, wpc = 1, bt = BATCH_THREADS;
  int64_t grid = 1;
  std::vector<int64_t> h_sys_row;
  int64_t *sys_row = nullptr, *rp = nullptr, *dpos = nullptr, *Lsrc = nullptr, *Usrc = nullptr;
  int32_t *ci = nullptr, *order = nullptr, *nlevL = nullptr, *nlevU = nullptr, *levL = nullptr, *levU = nullptr,
          *Lrow = nullptr, *Urow = nullptr, *Lout = nullptr, *iters = nullptr, *bstatus = nullptr;
  uint8_t *wide = nullptr;
  uint32_t *Lslot = nullptr, *Uslot = nullptr;
  unsigned int *ticket = nullptr;
  double *lu = nullptr, *Lval = nullptr, *Uval = nullptr, *Udiag = nullptr, *V = nullptr, *y = nullptr, *u = nullptr,
         *z = nullptr, *t = nullptr, *relres = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  ~ilu_batch() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

// Positions of one triangular solve of every system: rows sorted by (system,
// level), the per-system level tables, and the per-position entries.
static int batch_solve_order(ilu_batch *B, Mem &tmp, const Csr &A, const int32_t *row_sys, bool upper, int E,
                             void *stmp, size_t stmpb, hipStream_t s, int32_t **prow, uint32_t **pslot,
                             int64_t **psrc, int32_t **nlev, int32_t **lev, int32_t *err, bool refill_only,
                             Schedule &S, int32_t **rows_out, int32_t **inv_out) {
  ilu_precond *P = &B->core;
  Mem &mem = P->mem;
  const int64_t n = A.n;
  const int levmax1 = BATCH_LEVMAX + 1;
  if (!refill_only) {
    Segs seg;
    for (int k = 0; k < B->nsys; k++) {
      seg.a_start.push_back(B->h_sys_row[k]);
      seg.a_len.push_back(B->h_sys_row[k + 1] - B->h_sys_row[k]);
      seg.b_start.push_back(0);
      seg.b_len.push_back(0);
    }
    RC(build_schedule(P, tmp, A, !upper, 0, n, n, S, seg, s, upper ? "batch levels U" : "batch levels L"));
    if (S.nlev > BATCH_LEVMAX)
      return fail(ILU_ERR_CAPACITY, "batched solve: %lld levels in one triangular factor (at most %d)",
                  (long long)S.nlev, BATCH_LEVMAX);
  }
  const uint64_t nkeys = (uint64_t)B->nsys * (uint64_t)S.nlev;
  if (nkeys >= (1ull << 31)) return fail(ILU_ERR_CAPACITY, "batched solve: too many (system, level) pairs");
  uint32_t *key, *key2;
  int32_t *val, *rows, *inv;
  RC(tmp.alloc(&key, n));
  RC(tmp.alloc(&key2, n));
  RC(tmp.alloc(&val, n));
  RC(tmp.alloc(&rows, n));
  RC(tmp.alloc(&inv, n));
  void *rtmp;
  const size_t rtb = radix_tmp_bytes(n);
  RC(tmp.alloc((char **)&rtmp, (int64_t)rtb));
  RC(launch_block_level_keys(S.level_of, row_sys, n, S.nlev, key, val, s));
  RC(radix_sort(key, val, key2, rows, n, bits_for(nkeys - 1), rtmp, rtb, s));
  RC(launch_inverse_perm(n, rows, inv, s));
  int64_t *cnt, *bptr, btot;
  RC(tmp.alloc(&cnt, (int64_t)nkeys));
  RC(histogram_keys(key2, n, (int64_t)nkeys, cnt, s));
  const size_t stb2 = scan_tmp_bytes((int64_t)nkeys) + 64;
  void *stmp2;
  RC(tmp.alloc((char **)&stmp2, (int64_t)stb2));
  RC(make_rp(tmp, cnt, (int64_t)nkeys, &bptr, &btot, stmp2, stb2, s));
  int32_t *bptr32;
  RC(tmp.alloc(&bptr32, (int64_t)nkeys + 1));
  RC(launch_i64_to_i32(bptr, bptr32, (int64_t)nkeys + 1, s));
  if (!*nlev) {
    RC(mem.alloc(nlev, B->nsys));
    RC(mem.alloc(lev, (int64_t)B->nsys * levmax1));
  }
  RC(launch_batch_levels(bptr32, S.nlev, B->sys_row, B->nsys, levmax1, *lev, *nlev, B->wide, upper, s));
  if (!*prow) RC(mem.alloc(prow, n));
  RC(mem.alloc(pslot, n * (E / 2)));
  RC(mem.alloc(psrc, n * E));
  RC(launch_batch_fill(rows, n, B->sys_row, row_sys, inv, S.level_of, *lev, levmax1, A.rp, A.ci, upper, E, *prow,
                       *pslot, *psrc, B->dpos, err, s));
  *rows_out = rows;  // global row at each position, and the position of each row (setup temporaries)
  *inv_out = inv;
  (void)stmp;
  (void)stmpb;
  return 0;
}

static int batch_setup_impl(ilu_batch *B, const ilu_csr_t *A, int32_t restart, hipStream_t s) {
  ilu_precond *P = &B->core;
  Mem &mem = P->mem;
  Mem tmp;
  const int64_t n = A->n, nnz = A->nnz;
  HIPCK(hipGetDevice(&P->device));
  {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, P->device) == hipSuccess && cu > 0)
      P->num_cu = cu;
  }
  RC(mem.alloc(&P->status, 1));
  HIPCK(hipMemsetAsync(P->status, 0, sizeof(Status), s));
  RC(mem.alloc(&B->sys_row, B->nsys + 1));
  HIPCK(hipMemcpyAsync(B->sys_row, B->h_sys_row.data(), sizeof(int64_t) * (B->nsys + 1), hipMemcpyHostToDevice, s));
  int32_t *row_sys;
  RC(mem.alloc(&row_sys, n));
  RC(launch_row_sys(B->sys_row, B->nsys, row_sys, s));
  // 1. validation (the system of a row plays the partition; columns outside
  //    the row's system are rejected below)
  int32_t *err;
  RC(tmp.alloc(&err, 3));
  RC(fill_i32(err, 0x7fffffff, 2, s));
  RC(fill_i32(err + 2, 0, 1, s));
  RC(launch_validate(A->d_row_ptr, A->d_col, n, nnz, row_sys, B->nsys, err, s));
  int32_t herr[3];
  HIPCK(hipMemcpyAsync(herr, err, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  if (herr[0] != 0x7fffffff)
    return fail(ILU_ERR_CSR, "invalid CSR at row %d (row pointers, unsorted/duplicate/out-of-range columns, or "
                "missing diagonal)", herr[0]);
  // 2. the pattern, owned by the handle
  RC(mem.alloc(&B->rp, n + 1));
  RC(mem.alloc(&B->ci, nnz));
  HIPCK(hipMemcpyAsync(B->rp, A->d_row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, s));
  HIPCK(hipMemcpyAsync(B->ci, A->d_col, sizeof(int32_t) * std::max<int64_t>(nnz, 1), hipMemcpyDeviceToDevice, s));
  Csr Ap;
  Ap.n = n;
  Ap.nnz = nnz;
  Ap.rp = B->rp;
  Ap.ci = B->ci;
  RC(mem.alloc(&B->dpos, n));
  RC(mem.alloc(&B->wide, B->nsys));
  // 3. levels, positions and entries of both solves; E = 2 entries per row
  //    and triangle when that suffices, else 4
  const size_t stmpb = scan_tmp_bytes(n + 1) + 64;
  void *stmp;
  RC(tmp.alloc((char **)&stmp, (int64_t)stmpb));
  Schedule SL, SU;
  int32_t *rowsL = nullptr, *invL = nullptr, *rowsU = nullptr, *invU = nullptr;
  for (int E = 2;; E = 4) {
    RC(fill_i32(err + 2, 0, 1, s));
    const bool again = E == 4;
    RC(batch_solve_order(B, tmp, Ap, row_sys, false, E, stmp, stmpb, s, &B->Lrow, &B->Lslot, &B->Lsrc, &B->nlevL,
                         &B->levL, err + 2, again, SL, &rowsL, &invL));
    RC(batch_solve_order(B, tmp, Ap, row_sys, true, E, stmp, stmpb, s, &B->Urow, &B->Uslot, &B->Usrc, &B->nlevU,
                         &B->levU, err + 2, again, SU, &rowsU, &invU));
    HIPCK(hipMemcpyAsync(herr + 2, err + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    B->E = E;
    if (!(herr[2] & 2) || E == 4) break;
  }
  if (herr[2] & 4) return fail(ILU_ERR_INVALID_ARG, "batched systems: a column lies outside its row's system");
  if (herr[2] & 2)
    return fail(ILU_ERR_CAPACITY, "batched solve: a row has more than 4 entries in a triangle or more than %d in all",
                BATCH_RMAX);
  if (herr[2] & 1) return fail(ILU_ERR_CAPACITY, "batched solve: a dependency lies beyond the %d-position ring",
                               BATCH_RING);
  // the lower solve writes each solution at its row's U position
  RC(mem.alloc(&B->Lout, n));
  RC(launch_batch_lout(rowsL, invU, B->sys_row, row_sys, n, B->Lout, s));
  (void)invL;
  (void)rowsU;
  // level arrays of the rows, kept for export
  B->core.sL1 = SL;
  B->core.sU1 = SU;
  // 4. largest-first order of the systems
  {
    std::vector<int32_t> ord(B->nsys);
    for (int k = 0; k < B->nsys; k++) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
      return B->h_sys_row[a + 1] - B->h_sys_row[a] > B->h_sys_row[b + 1] - B->h_sys_row[b];
    });
    RC(mem.alloc(&B->order, B->nsys));
    HIPCK(hipMemcpyAsync(B->order, ord.data(), sizeof(int32_t) * B->nsys, hipMemcpyHostToDevice, s));
  }
  // 5. factor values, repacked entries, Krylov workspace, results
  RC(mem.alloc(&B->lu, nnz));
  RC(mem.alloc(&B->Lval, n * B->E));
  RC(mem.alloc(&B->Uval, n * B->E));
  RC(mem.alloc(&B->Udiag, n));
  RC(mem.alloc(&B->V, (int64_t)(restart + 1) * n));
  RC(mem.alloc(&B->y, n));
  RC(mem.alloc(&B->u, n));
  RC(mem.alloc(&B->z, n));
  RC(mem.alloc(&B->t, n));
  RC(mem.alloc(&B->iters, B->nsys));
  RC(mem.alloc(&B->bstatus, B->nsys));
  RC(mem.alloc(&B->relres, B->nsys));
  RC(mem.alloc(&B->ticket, 1));
  RC(fill_i32(B->iters, 0, B->nsys, s));
  RC(fill_i32(B->bstatus, 0, B->nsys, s));
  B->m_alloc = restart;
  const int per = batch_resident_groups(P->num_cu, B->E, B->bt) / std::max(P->num_cu, 1);
  if (per < 1) return fail(ILU_ERR_HIP, "batched solve: no resident workgroups");
  B->wpc = std::min(per, 2);
  B->grid = std::min<int64_t>(B->nsys, (int64_t)B->wpc * P->num_cu);
  HIPCK(hipStreamSynchronize(s));
  return 0;
}

static int batch_launch(ilu_batch *B, const double *val, const double *b, double *x, double rtol, int m, int maxit,
                        hipStream_t s) {
  BatchLaunch L;
  L.nsys = B->nsys;
  L.sys_row = B->sys_row;
  L.order = B->order;
  L.nlevL = B->nlevL;
  L.nlevU = B->nlevU;
  L.levL = B->levL;
  L.levU = B->levU;
  L.wide = B->wide;
  L.rp = B->rp;
  L.ci = B->ci;
  L.av = val;
  L.dpos = B->dpos;
  L.lu = B->lu;
  L.Lrow = B->Lrow;
  L.Urow = B->Urow;
  L.Lout = B->Lout;
  L.Lslot = B->Lslot;
  L.Uslot = B->Uslot;
  L.Lsrc = B->Lsrc;
  L.Usrc = B->Usrc;
  L.Lval = B->Lval;
  L.Uval = B->Uval;
  L.Udiag = B->Udiag;
  L.b = b;
  L.x = x;
  L.V = B->V;
  L.y = B->y;
  L.u = B->u;
  L.z = B->z;
  L.t = B->t;
  L.rtol = rtol;
  L.m = m;
  L.maxit = maxit;
  L.merge = B->merge;
  L.E = B->E;
  L.bt = B->bt;
  L.grid = B->grid;
  L.ticket = B->ticket;
  L.iters = B->iters;
  L.status = B->bstatus;
  L.relres = B->relres;
  const int rc = launch_batch_solve(L, s);
  if (rc == ILU_ERR_INVALID_ARG) return fail(rc, "batched solve: bad restart or grid");
  return rc;
}

static int batch_check_args(ilu_batch *B, const double *val, const double *b, double *x, double rtol, int m,
                            int maxit) {
  if (!B) return fail(ILU_ERR_INVALID_ARG, "NULL batch handle");
  if (B->n > 0 && (!val || !b || !x)) return fail(ILU_ERR_INVALID_ARG, "NULL vector");
  if (m < 1 || m > B->m_alloc || m > BATCH_MMAX || maxit < 0 || !(rtol >= 0.0))
    return fail(ILU_ERR_INVALID_ARG, "restart must be in [1, %d] (the setup's restart) and maxit, rtol >= 0",
                std::min(B->m_alloc, BATCH_MMAX));
  return 0;
}

extern "C" {

int ilu_batch_setup(const ilu_csr_t *A, const int64_t *h_sys_row, int32_t nsys, int32_t restart, void *stream,
                    ilu_batch_t **out) {
  if (!out) return fail(ILU_ERR_INVALID_ARG, "B must not be NULL");
  *out = nullptr;
  if (!A || A->n < 1 || A->nnz < 1 || !A->d_row_ptr || !A->d_col || !h_sys_row || nsys < 1)
    return fail(ILU_ERR_INVALID_ARG, "invalid batch description");
  if (A->n >= 0x7fffffff || A->nnz >= ((int64_t)1 << 40)) return fail(ILU_ERR_INVALID_ARG, "batch too large");
  if (restart < 1 || restart > BATCH_MMAX)
    return fail(ILU_ERR_INVALID_ARG, "restart must be in [1, %d] for the batched solve", BATCH_MMAX);
  if (h_sys_row[0] != 0 || h_sys_row[nsys] != A->n)
    return fail(ILU_ERR_INVALID_ARG, "system offsets must start at 0 and end at n");
  for (int32_t k = 0; k < nsys; k++)
    if (h_sys_row[k + 1] <= h_sys_row[k]) return fail(ILU_ERR_INVALID_ARG, "system %d is empty", k);
  ilu_batch *B = new ilu_batch();
  ilu_default_options(&B->core.opt);
  B->nsys = nsys;
  B->n = A->n;
  B->nnz = A->nnz;
  B->core.n = A->n;
  B->h_sys_row.assign(h_sys_row, h_sys_row + nsys + 1);
  hipStream_t s = (hipStream_t)stream;
  const int rc = batch_setup_impl(B, A, restart, s);
  if (rc) {
    (void)hipStreamSynchronize(s);
    delete B;
    return rc;
  }
  *out = B;
  return 0;
}

int ilu_batch_solve(ilu_batch_t *B, const double *d_val, const double *d_b, double *d_x, double rtol,
                    int32_t restart, int32_t maxit, void *stream) {
  RC(batch_check_args(B, d_val, d_b, d_x, rtol, restart, maxit));
  HIPCK(hipSetDevice(B->core.device));
  return batch_launch(B, d_val, d_b, d_x, rtol, restart, maxit, (hipStream_t)stream);
}

int ilu_batch_schedule(ilu_batch_t *B, int32_t merge, int32_t wpc, int32_t threads) {
  if (!B) return fail(ILU_ERR_INVALID_ARG, "NULL batch handle");
  if (threads != 256 && threads != 512) return fail(ILU_ERR_INVALID_ARG, "threads must be 256 or 512");
  const int per = batch_resident_groups(B->core.num_cu, B->E, threads) / std::max(B->core.num_cu, 1);
  if (merge < 0 || merge > WAVE || wpc < 1 || wpc > per)
    return fail(ILU_ERR_INVALID_ARG, "merge must be in [0, %d] and workgroups per CU in [1, %d]", WAVE, per);
  B->merge = merge;
  B->wpc = wpc;
  B->bt = threads;
  B->grid = std::min<int64_t>(B->nsys, (int64_t)wpc * B->core.num_cu);
  return 0;
}

int ilu_batch_tune(ilu_batch_t *B, const double *d_val, const double *d_b, double *d_x, double rtol,
                   int32_t restart, int32_t maxit, void *stream, int32_t *h_merge, int32_t *h_wpc,
                   int32_t *h_threads, double *h_ms) {
  RC(batch_check_args(B, d_val, d_b, d_x, rtol, restart, maxit));
  HIPCK(hipSetDevice(B->core.device));
  hipStream_t s = (hipStream_t)stream;
  // every candidate starts from the caller's initial guess (a solve
  // overwrites x, and a converged x would make the next candidate's solve
  // end at once)
  Mem tmp;
  double *x0 = nullptr;
  RC(tmp.alloc(&x0, B->n));
  HIPCK(hipMemcpyAsync(x0, d_x, sizeof(double) * B->n, hipMemcpyDeviceToDevice, s));
  hipEvent_t e0, e1;
  HIPCK(hipEventCreate(&e0));
  HIPCK(hipEventCreate(&e1));
  double best = 1e300;
  int bm = B->merge, bw = B->wpc, bb = B->bt;
  const int merges[] = {0, 16, 32, 64};
  int rc = 0;
  for (int th : {256, 512}) {
    const int per = batch_resident_groups(B->core.num_cu, B->E, th) / std::max(B->core.num_cu, 1);
    for (int w = 1; w <= per && !rc; w++)
      for (int mg : merges) {
        if ((rc = ilu_batch_schedule(B, mg, w, th))) break;
        if (hipMemcpyAsync(d_x, x0, sizeof(double) * B->n, hipMemcpyDeviceToDevice, s) != hipSuccess) {
          rc = fail(ILU_ERR_HIP, "batched tuning: restoring the initial guess failed");
          break;
        }
        (void)hipEventRecord(e0, s);
        if ((rc = batch_launch(B, d_val, d_b, d_x, rtol, restart, maxit, s))) break;
        (void)hipEventRecord(e1, s);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = fail(ILU_ERR_HIP, "batched tuning: event timing failed");
          break;
        }
        if (ms < best) {
          best = ms;
          bm = mg;
          bw = w;
          bb = th;
        }
      }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!rc && hipMemcpyAsync(d_x, x0, sizeof(double) * B->n, hipMemcpyDeviceToDevice, s) != hipSuccess)
    rc = fail(ILU_ERR_HIP, "batched tuning: restoring the initial guess failed");
  (void)hipStreamSynchronize(s);
  RC(rc);
  RC(ilu_batch_schedule(B, bm, bw, bb));
  if (h_merge) *h_merge = bm;
  if (h_wpc) *h_wpc = bw;
  if (h_threads) *h_threads = bb;
  if (h_ms) *h_ms = best;
  return 0;
}

int ilu_batch_capture(ilu_batch_t *B, const double *d_val, const double *d_b, double *d_x, double rtol,
                      int32_t restart, int32_t maxit, void *stream) {
  RC(batch_check_args(B, d_val, d_b, d_x, rtol, restart, maxit));
  if (!stream) return fail(ILU_ERR_INVALID_ARG, "graph capture needs a stream other than the default one");
  HIPCK(hipSetDevice(B->core.device));
  hipStream_t s = (hipStream_t)stream;
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->gexec = nullptr;
  B->graph = nullptr;
  HIPCK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const int rc = batch_launch(B, d_val, d_b, d_x, rtol, restart, maxit, s);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return silu_hip_fail(e, __LINE__);
  B->graph = g;
  HIPCK(hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0));
  return 0;
}

int ilu_batch_replay(ilu_batch_t *B, void *stream) {
  if (!B || !B->gexec) return fail(ILU_ERR_INVALID_ARG, "no captured batch solve");
  HIPCK(hipSetDevice(B->core.device));
  HIPCK(hipGraphLaunch(B->gexec, (hipStream_t)stream));
  return 0;
}

int ilu_batch_results(ilu_batch_t *B, int32_t *h_iters, double *h_relres, int32_t *h_status, void *stream) {
  if (!B) return fail(ILU_ERR_INVALID_ARG, "NULL batch handle");
  HIPCK(hipSetDevice(B->core.device));
  hipStream_t s = (hipStream_t)stream;
  if (h_iters) HIPCK(hipMemcpyAsync(h_iters, B->iters, sizeof(int32_t) * B->nsys, hipMemcpyDeviceToHost, s));
  if (h_relres) HIPCK(hipMemcpyAsync(h_relres, B->relres, sizeof(double) * B->nsys, hipMemcpyDeviceToHost, s));
  if (h_status) HIPCK(hipMemcpyAsync(h_status, B->bstatus, sizeof(int32_t) * B->nsys, hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  return 0;
}

int ilu_batch_export(ilu_batch_t *B, int32_t what, void *h_buf, int64_t *len) {
  if (!B || !len) return fail(ILU_ERR_INVALID_ARG, "NULL argument");
  switch (what) {
    case 0: return export_raw(B->lu, B->nnz, 8, h_buf, len);
    case 1: return export_raw(B->core.sL1.level_of, B->n, 4, h_buf, len);
    case 2: return export_raw(B->core.sU1.level_of, B->n, 4, h_buf, len);
    case 3: {
      const int32_t v[5] = {B->E, B->merge, B->wpc, (int32_t)B->grid, B->bt};
      if (!h_buf) {
        *len = 5;
        return 0;
      }
      if (*len < 5) return fail(ILU_ERR_INVALID_ARG, "export buffer too small");
      *len = 5;
      memcpy(h_buf, v, sizeof(v));
      return 0;
    }
    default: return fail(ILU_ERR_INVALID_ARG, "unknown batch export code %d", what);
  }
}

void ilu_batch_destroy(ilu_batch_t *B) {
  if (!B) return;
  (void)hipSetDevice(B->core.device);
  delete B;
}

static int export_csr(const Csr &c, int field, void *h, int64_t *len) {
  const int64_t cnt = field == 0 ? (c.rp ? c.n + 1 : 0) : c.nnz;
  if (!h) {
    *len = cnt;
    return 0;
  }
  if (*len < cnt) return fail(ILU_ERR_INVALID_ARG, "export buffer too small");
  *len = cnt;
  if (cnt == 0) return 0;
  const void *src = field == 0 ? (const void *)c.rp : field == 1 ? (const void *)c.ci : (const void *)c.v;
  const size_t es = field == 0 ? 8 : field == 1 ? 4 : 8;
  HIPCK(hipMemcpy(h, src, es * cnt, hipMemcpyDeviceToHost));
  return 0;
}

static int export_raw(const void *d, int64_t cnt, size_t es, void *h, int64_t *len) {
  if (!h) {
    *len = cnt;
    return 0;
  }
  if (*len < cnt) return fail(ILU_ERR_INVALID_ARG, "export buffer too small");
  *len = cnt;
  if (cnt > 0) HIPCK(hipMemcpy(h, d, es * cnt, hipMemcpyDeviceToHost));
  return 0;
}

// L_B / W / U_B / Z are views of L1 / U1 restricted by rows / columns: exported
// through a host-side split of the copied arrays.
static int export_split(const Csr &c, int64_t r0, int64_t r1, int64_t c0, int64_t c1, int64_t shift, int field,
                        void *h, int64_t *len) {
  std::vector<int64_t> rp(c.n + 1, 0);
  std::vector<int32_t> ci(c.nnz);
  std::vector<double> v(c.nnz);
  if (c.n > 0) HIPCK(hipMemcpy(rp.data(), c.rp, 8 * (c.n + 1), hipMemcpyDeviceToHost));
  if (c.nnz > 0) {
    HIPCK(hipMemcpy(ci.data(), c.ci, 4 * c.nnz, hipMemcpyDeviceToHost));
    HIPCK(hipMemcpy(v.data(), c.v, 8 * c.nnz, hipMemcpyDeviceToHost));
  }
  std::vector<int64_t> orp(1, 0);
  std::vector<int32_t> oci;
  std::vector<double> ov;
  for (int64_t r = r0; r < r1; r++) {
    for (int64_t p = rp[r]; p < rp[r + 1]; p++)
      if (ci[p] >= c0 && ci[p] < c1) {
        oci.push_back((int32_t)(ci[p] - shift));
        ov.push_back(v[p]);
      }
    orp.push_back((int64_t)oci.size());
  }
  const int64_t cnt = field == 0 ? (int64_t)orp.size() : (int64_t)oci.size();
  if (!h) {
    *len = cnt;
    return 0;
  }
  if (*len < cnt) return fail(ILU_ERR_INVALID_ARG, "export buffer too small");
  *len = cnt;
  if (field == 0) memcpy(h, orp.data(), 8 * cnt);
  if (field == 1) memcpy(h, oci.data(), 4 * cnt);
  if (field == 2) memcpy(h, ov.data(), 8 * cnt);
  return 0;
}

int ilu_export(ilu_precond_t *P, int32_t what, void *h, int64_t *len) {
  if (!P || !len) return fail(ILU_ERR_INVALID_ARG, "NULL argument");
  const int64_t n = P->n, nB = P->nB, nS = P->nS;
  switch (what) {
    case 0: return export_raw(P->perm, n, 4, h, len);
    case 1: return export_raw(P->iperm, n, 4, h, len);
    case 2: return export_raw(P->iface, n, 1, h, len);
    case 3: {
      const int64_t cnt = (int64_t)P->offsets.size();
      if (!h) {
        *len = cnt;
        return 0;
      }
      if (*len < cnt) return fail(ILU_ERR_INVALID_ARG, "export buffer too small");
      *len = cnt;
      memcpy(h, P->offsets.data(), 8 * cnt);
      return 0;
    }
    case 16: return export_raw(P->DB, nB, 8, h, len);
    case 29: return export_raw(P->DS, nS, 8, h, len);
    case 40: return export_raw(P->sL1.level_of, nB, 4, h, len);
    case 41: return export_raw(P->sU1.level_of, nB, 4, h, len);
    case 42: return export_raw(P->sLS.level_of, nS, 4, h, len);
    case 43: return export_raw(P->sUS.level_of, nS, 4, h, len);
    case 44: {  // schedule of the four solves, then whether L_S and U_S run as one launch
      const Schedule *sch[4] = {&P->sL1, &P->sU1, &P->sLS, &P->sUS};
      int32_t v[22] = {0};
      for (int k = 0; k < 4; k++) {
        v[4 * k] = sch[k]->use_block ? 1 : 0;
        v[4 * k + 1] = sch[k]->lds_g;
        v[4 * k + 2] = sch[k]->lds_e;
        v[4 * k + 3] = sch[k]->lds_bt;
      }
      if (P->block_mode && nS > 0) {
        const TrsvLaunch lo = make_launch(P, P->sLS, P->LS, nullptr, 0, P->gS, nullptr, P->yS, nullptr, nullptr, 2);
        const TrsvLaunch up = make_launch(P, P->sUS, P->US, P->DS, INT64_MAX, P->yS, nullptr, P->yS, nullptr, nullptr, 3);
        v[16] = trsv_lds_pair_ok(lo, up) ? 1 : 0;
      }
      for (int k = 0; k < 4; k++) v[17] |= (sch[k]->use_block && sch[k]->lds_fast ? 1 : 0) << k;
      v[18] = P->opt.factor_prec;
      v[19] = P->sLS.use_block ? (int32_t)P->sLS.nblk : 0;
      v[20] = P->sL1.use_block ? P->sL1.split_k : 0;
      v[21] = P->sU1.use_block ? P->sU1.split_k : 0;
      if (!h) {
        *len = 22;
        return 0;
      }
      if (*len < 22) return fail(ILU_ERR_INVALID_ARG, "export buffer too small");
      *len = 22;
      memcpy(h, v, sizeof(v));
      return 0;
    }
    default: break;
  }
  if (what >= 10 && what <= 12) return export_split(P->L1, 0, nB, 0, nB, 0, what - 10, h, len);
  if (what >= 13 && what <= 15) return export_split(P->U1, 0, nB, 0, nB, 0, what - 13, h, len);
  if (what >= 17 && what <= 19) return export_split(P->U1, 0, nB, nB, n, 0, what - 17, h, len);
  if (what >= 20 && what <= 22) return export_split(P->L1, nB, n, 0, nB, 0, what - 20, h, len);
  if (what >= 23 && what <= 25) return export_csr(P->LS, what - 23, h, len);
  if (what >= 26 && what <= 28) return export_csr(P->US, what - 26, h, len);
  if (what >= 30 && what <= 32) return export_csr(P->Coff, what - 30, h, len);
  return fail(ILU_ERR_INVALID_ARG, "unknown export code %d", what);
}

}  // extern "C"
