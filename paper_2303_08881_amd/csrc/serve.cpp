// serve.cpp -- request server: continuous batching of sparse solves on one GPU.
//
// A request is one solve A x = b with the preconditioner of the server's
// options (for instance the two-level ILU with FP32 factors), keyed by a
// matrix id.  The factors of every id stay resident in device memory, so a
// repeated right-hand side for a known id skips the setup: the split between
// setup and solve phases that the paper times separately (Section 4).
//
// Execution: `slots` worker threads, each with its own HIP stream (default
// priority), take requests from one queue; the setups and solves of
// different requests therefore overlap on the device, and a request that
// arrives while others run is started as soon as a slot and enough memory
// are free (continuous batching, not a queue drained one request at a time).
// A worker takes the OLDEST queued request that can start now:
//   * its matrix is not being set up or used by another running request (a
//     preconditioner handle holds its own workspace and is not re-entrant);
//   * the device bytes it needs fit into the budget beside the resident
//     factors and the reservations of the running requests.  Idle factors
//     are evicted least-recently-used first to make room.  A request that
//     cannot fit even into an empty server fails with ILU_ERR_OOM.
// Each request runs the same library calls (ilu_setup, fgmres_solve) on its
// slot's stream as a caller would alone, and every kernel on the path is
// deterministic, so its result does not depend on what else is running.
//
// Setups run one at a time: the factorization and the level analysis are
// launched cooperatively with a grid of every workgroup the device can hold
// and rely on a workgroup per row stream being resident, which two such
// launches side by side could not both be sure of.  For the same reason the
// server's handles orthogonalise their Arnoldi steps with one launch per
// pass instead of one launch per step whose workgroups wait for each
// other.  Solves then never wait
// on a workgroup that has not started (their waits follow ticket order), so
// they overlap with each other and with the one running setup.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "common.hpp"
#include "launch.hpp"

using namespace silu;

namespace {
using Clock = std::chrono::steady_clock;

struct Entry {
  int64_t id = 0;
  bool ready = false;  // factors built
  bool busy = false;   // a running request uses it (or is building it)
  ilu_csr_t A{};       // device copy of the matrix, owned by the entry
  void *rp = nullptr, *ci = nullptr, *v = nullptr;
  ilu_precond_t *P = nullptr;
  int64_t bytes = 0;  // counted against the budget while resident
  uint64_t last = 0;  // least-recently-used stamp
};

struct Req {
  ilu_request_t out{};
  ilu_csr_t A{};
  bool has_A = false;
  const int32_t *part = nullptr;
  int32_t nparts = 1;
  const double *b = nullptr;
  double *x = nullptr;
  double rtol = 0.0;
  int32_t restart = 30, maxit = 1000;
  int64_t reserve = 0;  // bytes reserved while it runs
  Entry *e = nullptr;
  std::string err;
};

// Device bytes of one FGMRES(m) workspace on n unknowns: the basis V, the
// preconditioned directions Z and the residual.
int64_t work_bytes(int64_t n, int m) { return 8 * n * (2 * (int64_t)m + 2); }

int64_t matrix_bytes(const ilu_csr_t &A) { return 12 * A.nnz + 8 * (A.n + 1); }

// Bound on the device bytes of a setup before it has run: the factors on A's
// pattern with their solve layouts, the level schedules, permutations and
// work vectors stay within about six times the matrix's own bytes plus 160
// bytes per row for ILU(0)/MILU(0); ILUT may add its fill (lfil entries per
// row and part); the multiplicative method holds two factor sets and A.  The
// measured figure replaces the bound once the setup has finished.
int64_t setup_bound(const ilu_csr_t &A, const ilu_options_t &o) {
  int64_t f = 6 * matrix_bytes(A) + 160 * A.n;
  if (o.interior_fact == ILU_FACT_ILUT) f += 2 * 12 * (int64_t)(o.lfil > 0 ? o.lfil : 64) * A.n;
  if (o.method == ILU_METHOD_RAP) f = 2 * f + matrix_bytes(A);
  return f;
}

double us_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
}
}  // namespace

struct ilu_server {
  int device = 0;
  int slots = 1;
  int64_t budget = 0;
  ilu_options_t opt{};
  Clock::time_point t0;
  std::mutex mu;
  std::mutex setup_mu;  // one setup on the device at a time
  std::condition_variable cv_work, cv_done;
  std::deque<Req *> queue;
  std::unordered_map<int64_t, Entry *> cache;
  std::unordered_map<int64_t, Req *> done;  // finished, not collected
  std::deque<int64_t> done_order;           // completion order of `done`
  std::unordered_set<int64_t> outstanding;  // submitted, not collected
  int64_t used = 0, peak = 0, next_ticket = 0;
  uint64_t clock = 0;
  int64_t hits = 0, misses = 0, evictions = 0;
  int running = 0;
  bool stop = false;
  std::vector<std::thread> workers;
};

namespace {

void destroy_entry(Entry *e) {
  if (!e) return;
  // the entry is idle: the stream of the request that last used it was synchronised
  precond_destroy_idle(e->P);
  dev_free(e->rp);
  dev_free(e->ci);
  dev_free(e->v);
  delete e;
}

// a request that cannot run: straight to the completed set (lock held)
void reject(ilu_server *S, Req *r, int code, const char *msg) {
  r->out.status = code;
  r->err = msg;
  r->out.start_us = r->out.done_us = us_since(S->t0);
  r->out.slot = -1;
  S->done[r->out.ticket] = r;
  S->done_order.push_back(r->out.ticket);
  S->cv_done.notify_all();
}

// The oldest queued request that can start now, with its memory reserved and
// its entry marked busy; idle entries evicted on the way go to `victims` (to
// be destroyed outside the lock).  Lock held.
Req *pick(ilu_server *S, std::vector<Entry *> &victims) {
  for (size_t i = 0; i < S->queue.size();) {
    Req *r = S->queue[i];
    auto ce = S->cache.find(r->out.matrix_id);
    Entry *e = ce == S->cache.end() ? nullptr : ce->second;
    if (e && (!e->ready || e->busy)) {  // being set up or in use: later
      i++;
      continue;
    }
    if (!e && !r->has_A) {
      // an older queued request may bring this id's matrix: wait for it
      bool coming = false;
      for (size_t j = 0; j < i && !coming; j++)
        coming = S->queue[j]->has_A && S->queue[j]->out.matrix_id == r->out.matrix_id;
      if (coming) {
        i++;
        continue;
      }
      S->queue.erase(S->queue.begin() + (ptrdiff_t)i);
      reject(S, r, ILU_ERR_INVALID_ARG, "matrix id is not resident and the request carries no matrix");
      continue;
    }
    const int64_t need = e ? work_bytes(e->A.n, r->restart)
                           : matrix_bytes(r->A) + setup_bound(r->A, S->opt) + work_bytes(r->A.n, r->restart);
    if (need > S->budget) {
      S->queue.erase(S->queue.begin() + (ptrdiff_t)i);
      reject(S, r, ILU_ERR_OOM, "request needs more device memory than the server's budget");
      continue;
    }
    while (S->used + need > S->budget) {
      Entry *lru = nullptr;
      for (auto &kv : S->cache) {
        Entry *c = kv.second;
        if (c != e && c->ready && !c->busy && (!lru || c->last < lru->last)) lru = c;
      }
      if (!lru) break;
      S->cache.erase(lru->id);
      S->used -= lru->bytes;
      S->evictions++;
      victims.push_back(lru);
    }
    if (S->used + need > S->budget) {  // waits for running requests to release memory
      i++;
      continue;
    }
    S->queue.erase(S->queue.begin() + (ptrdiff_t)i);
    r->reserve = need;
    S->used += need;
    S->peak = std::max(S->peak, S->used);
    if (e) {
      r->out.cache_hit = 1;
      S->hits++;
    } else {
      e = new Entry();
      e->id = r->out.matrix_id;
      S->cache[e->id] = e;
      S->misses++;
    }
    e->busy = true;
    r->e = e;
    return r;
  }
  return nullptr;
}

// Run one request on the slot's stream (no lock held).
void run(ilu_server *S, Req *r, hipStream_t st) {
  Entry *e = r->e;
  int rc = 0;
  r->out.start_us = us_since(S->t0);
  if (!r->out.cache_hit) {
    const ilu_csr_t &A = r->A;
    rc = dev_alloc(&e->rp, sizeof(int64_t) * (size_t)(A.n + 1));
    if (!rc) rc = dev_alloc(&e->ci, sizeof(int32_t) * (size_t)std::max<int64_t>(A.nnz, 1));
    if (!rc) rc = dev_alloc(&e->v, sizeof(double) * (size_t)std::max<int64_t>(A.nnz, 1));
    if (!rc) {
      hipError_t he = hipMemcpyAsync(e->rp, A.d_row_ptr, sizeof(int64_t) * (A.n + 1), hipMemcpyDeviceToDevice, st);
      if (he == hipSuccess && A.nnz)
        he = hipMemcpyAsync(e->ci, A.d_col, sizeof(int32_t) * A.nnz, hipMemcpyDeviceToDevice, st);
      if (he == hipSuccess && A.nnz)
        he = hipMemcpyAsync(e->v, A.d_val, sizeof(double) * A.nnz, hipMemcpyDeviceToDevice, st);
      if (he != hipSuccess) rc = api_fail(ILU_ERR_HIP, "copy of the matrix failed: %s", hipGetErrorString(he));
    }
    if (!rc) {
      e->A = ilu_csr_t{A.n, A.nnz, (const int64_t *)e->rp, (const int32_t *)e->ci, (const double *)e->v};
      std::lock_guard<std::mutex> lk(S->setup_mu);
      rc = ilu_setup(&e->A, r->part, r->nparts, &S->opt, st, &e->P);
    }
  }
  if (!rc) {
    ilu_result_t res{};
    rc = fgmres_solve(&e->A, e->P, r->b, r->x, r->rtol, r->restart, r->maxit, st, &res, nullptr);
    r->out.iterations = res.iterations;
    r->out.final_relres = res.final_relres;
    r->out.solve_ms = res.solve_ms;
    if (!r->out.cache_hit) r->out.setup_ms = res.setup_ms;
  }
  if (rc < 0) r->err = ilu_last_error();
  (void)hipStreamSynchronize(st);
  r->out.status = rc;
  r->out.done_us = us_since(S->t0);
}

// Bookkeeping after a request ran (lock held).
void finish(ilu_server *S, Req *r, std::vector<Entry *> &victims) {
  Entry *e = r->e;
  S->used -= r->reserve;
  r->reserve = 0;
  if (!e->P) {  // the setup failed: drop the entry
    S->cache.erase(e->id);
    S->used -= e->bytes;
    e->bytes = 0;
    victims.push_back(e);
  } else {
    S->used -= e->bytes;
    e->bytes = matrix_bytes(e->A) + precond_bytes(e->P);
    S->used += e->bytes;
    S->peak = std::max(S->peak, S->used);
    e->ready = true;
    e->busy = false;
    e->last = ++S->clock;
  }
  r->e = nullptr;
  S->done[r->out.ticket] = r;
  S->done_order.push_back(r->out.ticket);
}

void worker_main(ilu_server *S, int slot) {
  (void)hipSetDevice(S->device);
  hipStream_t st = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  std::vector<Entry *> victims;
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    Req *r = nullptr;
    for (;;) {
      r = pick(S, victims);
      if (r || !victims.empty() || (S->stop && S->queue.empty())) break;
      S->cv_work.wait(lk);
    }
    if (!victims.empty()) {
      std::vector<Entry *> v;
      v.swap(victims);
      lk.unlock();
      for (Entry *e : v) destroy_entry(e);
      lk.lock();
    }
    if (!r) {
      if (S->stop && S->queue.empty()) break;
      continue;
    }
    r->out.slot = slot;
    S->running++;
    lk.unlock();
    if (have_stream) {
      run(S, r, st);
    } else {
      r->out.status = api_fail(ILU_ERR_HIP, "the slot's stream could not be created");
      r->err = ilu_last_error();
    }
    lk.lock();
    S->running--;
    finish(S, r, victims);
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  lk.unlock();
  for (Entry *e : victims) destroy_entry(e);
  if (have_stream) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

int ilu_server_create(int32_t slots, int64_t budget_bytes, const ilu_options_t *opt, ilu_server_t **out) {
  if (!out) return api_fail(ILU_ERR_INVALID_ARG, "S must not be NULL");
  *out = nullptr;
  if (slots < 1 || slots > 64) return api_fail(ILU_ERR_INVALID_ARG, "slots must be in [1, 64]");
  if (budget_bytes <= 0) return api_fail(ILU_ERR_INVALID_ARG, "budget must be positive");
  ilu_server *S = new ilu_server();
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return api_fail(ILU_ERR_HIP, "no HIP device");
  }
  S->slots = slots;
  S->budget = budget_bytes;
  ilu_default_options(&S->opt);
  if (opt) S->opt = *opt;
  // the slots' solves run side by side: their Arnoldi steps take one launch
  // per pass, never a launch per step that waits for its whole grid
  S->opt.arnoldi_mode = ILU_ARNOLDI_PER_PASS;
  S->t0 = Clock::now();
  for (int i = 0; i < slots; i++) S->workers.emplace_back(worker_main, S, i);
  *out = S;
  return 0;
}

int ilu_server_submit(ilu_server_t *S, int64_t matrix_id, const ilu_csr_t *A, const int32_t *d_part, int32_t nparts,
                      const double *d_b, double *d_x, double rtol, int32_t restart, int32_t maxit, int64_t *ticket) {
  if (!S || !d_b || !d_x || !ticket) return api_fail(ILU_ERR_INVALID_ARG, "NULL argument");
  if (restart < 1 || restart > 1000 || maxit < 0 || !(rtol >= 0.0))
    return api_fail(ILU_ERR_INVALID_ARG, "restart/maxit/rtol out of range");
  if (A && (A->n < 1 || A->nnz < 1 || !A->d_row_ptr || !A->d_col || !A->d_val))
    return api_fail(ILU_ERR_INVALID_ARG, "invalid matrix descriptor");
  if (A && (nparts < 1 || (!d_part && nparts != 1)))
    return api_fail(ILU_ERR_INVALID_ARG, "nparts must be >= 1 (1 without part)");
  Req *r = new Req();
  if (A) {
    r->A = *A;
    r->has_A = true;
  }
  r->part = d_part;
  r->nparts = nparts;
  r->b = d_b;
  r->x = d_x;
  r->rtol = rtol;
  r->restart = restart;
  r->maxit = maxit;
  r->out.matrix_id = matrix_id;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
      delete r;
      return api_fail(ILU_ERR_INVALID_ARG, "server is shutting down");
    }
    r->out.ticket = S->next_ticket++;
    r->out.submit_us = us_since(S->t0);
    S->outstanding.insert(r->out.ticket);
    S->queue.push_back(r);
    *ticket = r->out.ticket;
  }
  S->cv_work.notify_one();
  return 0;
}

int ilu_server_wait(ilu_server_t *S, int64_t ticket, ilu_request_t *out) {
  if (!S || !out) return api_fail(ILU_ERR_INVALID_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  Req *r = nullptr;
  if (ticket >= 0) {
    if (!S->outstanding.count(ticket)) return api_fail(ILU_ERR_INVALID_ARG, "unknown or collected ticket");
    S->cv_done.wait(lk, [&] { return S->done.count(ticket) > 0; });
    r = S->done[ticket];
    S->done_order.erase(std::find(S->done_order.begin(), S->done_order.end(), ticket));
  } else {
    if (S->outstanding.empty()) return api_fail(ILU_ERR_INVALID_ARG, "no request outstanding");
    S->cv_done.wait(lk, [&] { return !S->done_order.empty(); });
    const int64_t t = S->done_order.front();
    S->done_order.pop_front();
    r = S->done[t];
  }
  S->done.erase(r->out.ticket);
  S->outstanding.erase(r->out.ticket);
  lk.unlock();
  *out = r->out;
  if (r->out.status < 0) api_fail(r->out.status, "%s", r->err.c_str());
  delete r;
  return 0;
}

int ilu_server_stats(ilu_server_t *S, int64_t *h_stats, int32_t count) {
  if (!S || !h_stats || count < 0) return api_fail(ILU_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  const int64_t v[9] = {S->used, S->peak, (int64_t)S->cache.size(), S->hits, S->misses,
                        S->evictions, (int64_t)S->queue.size(), (int64_t)S->running, S->budget};
  for (int i = 0; i < count && i < 9; i++) h_stats[i] = v[i];
  return 0;
}

void ilu_server_destroy(ilu_server_t *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (std::thread &t : S->workers) t.join();
  (void)hipSetDevice(S->device);
  for (auto &kv : S->cache) destroy_entry(kv.second);
  for (auto &kv : S->done) delete kv.second;
  delete S;
}

}  // extern "C"
