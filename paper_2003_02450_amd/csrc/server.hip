// Continuous-batching server: walks arrive one at a time, each on its own
// graph; they share one batch engine (qsw_engine_*), so a walk that arrives
// while others run joins the next cycle as soon as its vectors fit.
//
//  * Operator cache: superoperators are kept on the device under a byte
//    budget, keyed by a 64-bit FNV-1a hash of (N, graph CSR, omega, gamma,
//    flags) and checked against the stored key, so a repeated graph is not
//    rebuilt.  Operators no walk uses are evicted least recently used first.
//  * Admission: pending walks are admitted in arrival order, each when the
//    engine arena has room for its work vectors (the engine refuses it
//    otherwise); an admitted walk never waits for memory again.
//  * Operators are built off the serving loop: a cache miss queues the build
//    for a builder thread, which runs it on its own (non-blocking) stream,
//    so walks already on the device keep advancing meanwhile; the walk waits
//    in the queue until its operator is ready, without holding back walks
//    behind it whose operators are.
//  * Operator memory counts against the cache budget before it is built (an
//    upper bound from the graph, replaced by the handle's size once built):
//    a build that would exceed the budget while every cached operator is in
//    use waits until walks finish and release some.
//  * Two lanes.  A walk whose operator is large enough to fill the device on
//    its own (graph order at least QSW_SERVER_DIRECT_N, default 384; 0
//    turns the lane off) gains nothing from sharing launches, and would
//    slow every cycle of the engine down to its own pace: it runs through
//    qsw_propagate (launch pacing 2) on a runner thread and stream of its
//    own, one such walk at a time in arrival order, while the smaller walks
//    keep cycling in the engine.  The runner's workspace, and the output
//    series of a walk that asked for populations only, are device buffers
//    the server keeps and grows as needed.
//  * Every walk's result is bitwise what it would be alone, in either lane:
//    the engine keeps walks independent and equal to qsw_propagate.
#include "handle.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace qsw;

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void *p, size_t bytes) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < bytes; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  }
};

// What identifies an operator: the arguments of qsw_superop_build.
struct OpKey {
  int32_t N = 0;
  double omega = 0.0, gamma = 1.0;
  uint32_t flags = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> col;
  std::vector<double> w;
  bool operator==(const OpKey &o) const {
    return N == o.N && omega == o.omega && gamma == o.gamma && flags == o.flags && rp == o.rp &&
           col == o.col && w == o.w;
  }
};

struct CachedOp {
  OpKey key;
  uint64_t hash = 0;
  qsw_superop_t op = nullptr;  // null until built
  size_t bytes = 0;            // device bytes (an upper bound until built)
  int users = 0;               // walks pending or running on it
  int state = 0;               // 0 built, 1 waiting for cache room, 2 building, 3 failed
  qsw_status_t error = QSW_OK;
};

struct Request {
  int64_t id = 0;
  uint64_t hash = 0;
  CachedOp *cop = nullptr;
  bool direct = false;  // runs in the direct lane
  qsw_walk_t walk{};
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
  int64_t ticket = -1;
  int state = 0;  // 0 pending, 1 running, 2 done
};

// Device bytes a handle holds: CSR, wave-jagged copy (padded; complex or
// phase-split values), single-precision copy if any, row blocks of the
// stream layout.
size_t op_bytes(const qsw_superop_s *h) {
  const size_t n = (size_t)h->n, nnz = (size_t)h->nnz, pnz = (size_t)h->wentries + kWavePad;
  const size_t nwb = (n + 63) / 64;
  size_t b = 8 * (n + 1) + 4 * nnz + 16 * nnz;  // CSR
  b += 4 * pnz + 4 * n + n + 24 * nwb + 16 * (size_t)nwb * (size_t)h->wsh_stride;  // columns, rows, blocks, shared
  b += h->split ? 8 * pnz + 16 * n : 16 * pnz;    // values
  if (h->wval32) b += 8 * pnz;
  if (h->wcoef32) b += 4 * pnz + 8 * n;
  b += 4 * ((size_t)h->nblk + 1);
  return b;
}

// Upper bound of op_bytes before the build, from the graph alone: the
// undirected companion has at most 2E off-diagonal entries for E arcs, so L
// has at most 2N(2E) + N^2 + E + N entries (dephasing included).
size_t op_bytes_bound(int32_t N, int64_t E) {
  const double n = (double)N * N;
  const double nnz = 2.0 * N * 2.0 * (double)E + n + (double)E + N;
  return (size_t)(64.0 * nnz + 160.0 * n + 4096.0);
}

}  // namespace

struct qsw_server_s {
  int device = -1;
  hipStream_t stream = nullptr;
  // builder thread: jobs in, finished builds out (under mu)
  hipStream_t build_stream = nullptr;
  std::thread builder;
  std::mutex mu;
  std::condition_variable cv_job, cv_done;
  std::deque<CachedOp *> jobs;
  std::vector<std::pair<CachedOp *, qsw_superop_t>> built;
  std::vector<std::pair<CachedOp *, qsw_status_t>> failed;
  std::vector<double> build_ms;
  int in_flight = 0;
  bool stop = false;
  // direct lane: runner thread, its stream and buffers (runner only), its
  // queue and results (under mu)
  int32_t direct_min_N = 384;
  hipStream_t direct_stream = nullptr;
  std::thread runner;
  std::deque<Request *> djobs;
  std::vector<std::pair<Request *, qsw_status_t>> ddone;
  int d_in_flight = 0;
  void *dws = nullptr, *dout = nullptr;
  size_t dws_bytes = 0, dout_bytes = 0;
  void *arena = nullptr;
  qsw_engine_t engine = nullptr;
  size_t cache_budget = 0, cache_used = 0;
  std::unordered_multimap<uint64_t, CachedOp *> cache;  // hash -> entries
  std::list<CachedOp *> lru;                            // entries, newest first
  std::deque<CachedOp *> waiting;   // operators waiting for cache room, first come first
  std::deque<Request *> pending;
  std::unordered_map<int64_t, Request *> by_id;
  std::unordered_map<int64_t, Request *> by_ticket;
  std::vector<int64_t> done_ids;
  int64_t next_id = 0;
  qsw_server_stats_t stats{};
};

namespace {

void touch(qsw_server_s *s, CachedOp *c) {
  s->lru.remove(c);
  s->lru.push_front(c);
}

void evict_unused(qsw_server_s *s, size_t need) {
  while (s->cache_used + need > s->cache_budget) {
    CachedOp *victim = nullptr;
    for (auto it = s->lru.rbegin(); it != s->lru.rend(); ++it)
      if ((*it)->users == 0 && (*it)->state == 0) {
        victim = *it;
        break;
      }
    if (!victim) return;  // everything cached is in use
    s->lru.remove(victim);
    auto range = s->cache.equal_range(victim->hash);
    for (auto it = range.first; it != range.second; ++it)
      if (it->second == victim) {
        s->cache.erase(it);
        break;
      }
    s->cache_used -= victim->bytes;
    qsw_superop_destroy(victim->op);
    delete victim;
    ++s->stats.evictions;
  }
}

CachedOp *find_op(qsw_server_s *s, uint64_t hash, const OpKey &key) {
  auto range = s->cache.equal_range(hash);
  for (auto it = range.first; it != range.second; ++it)
    if (it->second->key == key) return it->second;
  return nullptr;
}

// Admit pending walks in arrival order while the engine takes them; a walk
// whose operator is still being built is passed over (it does not hold the
// walks behind it back), a walk that does not fit stops the admission.
qsw_status_t admit(qsw_server_s *s) {
  for (auto it = s->pending.begin(); it != s->pending.end();) {
    Request *r = *it;
    if (r->cop->state != 0) {
      ++it;
      continue;
    }
    r->walk.op = r->cop->op;
    if (s->direct_min_N > 0 && r->cop->op->N >= s->direct_min_N) {
      // the direct lane, in arrival order
      r->direct = true;
      r->state = 1;
      r->t_admit = now_ms();
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->djobs.push_back(r);
        ++s->d_in_flight;
        s->cv_job.notify_all();
      }
      it = s->pending.erase(it);
      continue;
    }
    int64_t ticket = -1;
    const qsw_status_t st = qsw_engine_submit(s->engine, &r->walk, &ticket);
    if (st == QSW_ERR_OOM) break;  // waits until running walks free space
    if (st != QSW_OK) return st;
    r->ticket = ticket;
    r->state = 1;
    r->t_admit = now_ms();
    s->by_ticket[ticket] = r;
    it = s->pending.erase(it);
  }
  return QSW_OK;
}

// The builder thread: builds queued operators on its own stream.
void builder_main(qsw_server_s *s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_job.wait(lk, [s] { return s->stop || !s->jobs.empty(); });
    if (s->jobs.empty()) return;  // stop requested and nothing queued
    CachedOp *c = s->jobs.front();
    s->jobs.pop_front();
    lk.unlock();
    const OpKey &k = c->key;  // not modified while the build is in flight
    const double t0 = now_ms();
    qsw_superop_t op = nullptr;
    const qsw_status_t st =
        qsw_superop_build(k.N, k.rp.data(), k.col.empty() ? nullptr : k.col.data(),
                          k.w.empty() ? nullptr : k.w.data(), k.omega, k.gamma, k.flags,
                          s->build_stream, &op);
    const double ms = now_ms() - t0;
    lk.lock();
    if (st == QSW_OK)
      s->built.emplace_back(c, op);
    else
      s->failed.emplace_back(c, st);
    s->build_ms.push_back(ms);
    --s->in_flight;
    s->cv_done.notify_all();
  }
}

// Grow a device buffer of the direct lane to at least `bytes` (the runner
// thread alone uses it; the lane's earlier work has finished).  It grows by
// at least half its size each time: a reallocation waits for the device.
hipError_t grow(void **buf, size_t *have, size_t bytes) {
  if (*have >= bytes) return hipSuccess;
  const size_t want = std::max(bytes, *have + *have / 2);
  if (*buf) (void)hipFree(*buf);
  *buf = nullptr;
  *have = 0;
  hipError_t e = hipMalloc(buf, want);
  if (e != hipSuccess && want > bytes) {
    (void)hipGetLastError();
    e = hipMalloc(buf, bytes);
    if (e == hipSuccess) *have = bytes;
    return e;
  }
  if (e == hipSuccess) *have = want;
  return e;
}

// One walk of the direct lane: qsw_propagate of its whole grid, then its
// populations when asked for, on the lane's stream.
qsw_status_t run_direct(qsw_server_s *s, Request *r) {
  const qsw_walk_t &w = r->walk;
  const size_t ws = qsw_propagate_workspace_bytes(w.op, w.t0, w.dt, w.n_steps);
  if (ws == 0) return QSW_ERR_ARG;
  HIP_TRY(grow(&s->dws, &s->dws_bytes, ws));
  void *out = w.out;
  if (!out) {
    HIP_TRY(grow(&s->dout, &s->dout_bytes,
                 (size_t)(w.n_steps + 1) * (size_t)w.op->n * sizeof(double2)));
    out = s->dout;
  }
  qsw_status_t st = qsw_propagate(w.op, w.rho0, w.t0, w.dt, w.n_steps, out, s->dws, ws,
                                  s->direct_stream);
  if (st != QSW_OK) return st;
  if (w.pops) {
    st = qsw_populations(w.op, out, w.n_steps + 1, w.pops, s->direct_stream);
    if (st != QSW_OK) return st;
  }
  HIP_TRY(hipStreamSynchronize(s->direct_stream));
  qsw_stats_t ps{};
  st = qsw_last_stats(w.op, &ps);
  return st == QSW_ERR_NONFINITE ? QSW_OK : st;
}

void runner_main(qsw_server_s *s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_job.wait(lk, [s] { return s->stop || !s->djobs.empty(); });
    if (s->djobs.empty()) return;
    Request *r = s->djobs.front();
    s->djobs.pop_front();
    lk.unlock();
    const qsw_status_t st = run_direct(s, r);
    lk.lock();
    s->ddone.emplace_back(r, st);
    s->cv_done.notify_all();
  }
}

// Queue the builds of waiting operators, first come first, while the cache
// budget allows them (evicting unused operators first); an operator larger
// than the whole budget is built once nothing else is cached.
void start_builds(qsw_server_s *s) {
  while (!s->waiting.empty()) {
    CachedOp *c = s->waiting.front();
    evict_unused(s, c->bytes);
    if (s->cache_used + c->bytes > s->cache_budget && s->cache_used > 0) break;
    s->waiting.pop_front();
    c->state = 2;
    s->cache_used += c->bytes;
    std::lock_guard<std::mutex> lk(s->mu);
    s->jobs.push_back(c);
    ++s->in_flight;
    s->cv_job.notify_all();  // the runner waits on it too
  }
}

// Finish a request without running it (its operator failed to build, or its
// vectors can never fit the arena).
void drop_request(qsw_server_s *s, Request *r) {
  r->state = 2;
  r->t_done = now_ms();
  --r->cop->users;
  s->done_ids.push_back(r->id);
  ++s->stats.completed;
  for (auto it = s->pending.begin(); it != s->pending.end(); ++it)
    if (*it == r) {
      s->pending.erase(it);
      break;
    }
}

// Take the builder's results: built operators become usable (their size
// replaces the bound), failed ones finish their requests.  Returns the first
// build error, if any.
qsw_status_t drain_builds(qsw_server_s *s) {
  std::vector<std::pair<CachedOp *, qsw_superop_t>> built;
  std::vector<std::pair<CachedOp *, qsw_status_t>> failed;
  std::vector<double> ms;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    built.swap(s->built);
    failed.swap(s->failed);
    ms.swap(s->build_ms);
  }
  for (double m : ms) s->stats.build_ms += m;
  qsw_status_t err = QSW_OK;
  for (auto &bc : built) {
    CachedOp *c = bc.first;
    c->op = bc.second;
    const size_t actual = op_bytes(c->op);
    s->cache_used = s->cache_used - c->bytes + actual;
    c->bytes = actual;
    c->state = 0;
  }
  for (auto &fc : failed) {
    CachedOp *c = fc.first;
    c->state = 3;
    c->error = fc.second;
    if (err == QSW_OK) err = fc.second;
  }
  // requests on failed operators, or too large for the arena, finish now
  std::vector<Request *> drop;
  for (Request *r : s->pending) {
    if (r->cop->state == 3) {
      drop.push_back(r);
    } else if (r->cop->state == 0) {
      r->walk.op = r->cop->op;
      const size_t need = qsw_walk_bytes(&r->walk, 1);
      if (need == 0 || need > engine_pool_bytes(s->engine)) {
        if (err == QSW_OK) err = need == 0 ? QSW_ERR_ARG : QSW_ERR_OOM;
        drop.push_back(r);
      }
    }
  }
  for (Request *r : drop) drop_request(s, r);
  // failed operators nobody waits for leave the cache
  for (auto &fc : failed) {
    CachedOp *c = fc.first;
    if (c->users > 0) continue;
    s->lru.remove(c);
    auto range = s->cache.equal_range(c->hash);
    for (auto it = range.first; it != range.second; ++it)
      if (it->second == c) {
        s->cache.erase(it);
        break;
      }
    s->cache_used -= c->bytes;
    delete c;
  }
  // operators of the direct lane run with launch pacing
  for (auto &bc : built)
    if (s->direct_min_N > 0 && bc.first->op->N >= s->direct_min_N)
      (void)qsw_superop_set_pacing(bc.first->op, 2);
  return err;
}

// Walks the direct lane finished.  Returns the first error of one.
qsw_status_t drain_direct(qsw_server_s *s) {
  std::vector<std::pair<Request *, qsw_status_t>> done;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    done.swap(s->ddone);
    s->d_in_flight -= (int)done.size();
  }
  qsw_status_t err = QSW_OK;
  const double t = now_ms();
  for (auto &rd : done) {
    Request *r = rd.first;
    r->state = 2;
    r->t_done = t;
    s->done_ids.push_back(r->id);
    ++s->stats.completed;
    --r->cop->users;
    if (rd.second != QSW_OK && err == QSW_OK) err = rd.second;
  }
  return err;
}

}  // namespace

extern "C" {

qsw_status_t qsw_server_create(size_t arena_bytes, size_t cache_bytes, int32_t max_walks,
                               void *hip_stream, qsw_server_t *out) {
  if (!out) return QSW_ERR_ARG;
  *out = nullptr;
  if (max_walks < 1 || arena_bytes == 0) return QSW_ERR_ARG;
  qsw_server_s *s = new (std::nothrow) qsw_server_s();
  if (!s) return QSW_ERR_OOM;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return QSW_ERR_DEVICE;
  }
  s->stream = (hipStream_t)hip_stream;
  s->cache_budget = cache_bytes;
  if (hipMalloc(&s->arena, arena_bytes) != hipSuccess) {
    delete s;
    return QSW_ERR_OOM;
  }
  const qsw_status_t st = qsw_engine_create(max_walks, 1, s->arena, arena_bytes, hip_stream,
                                            &s->engine);
  if (st != QSW_OK) {
    (void)hipFree(s->arena);
    delete s;
    return st;
  }
  // builds overlap the engine's work: a stream that does not wait for the
  // legacy default stream (default priority)
  if (hipStreamCreateWithFlags(&s->build_stream, hipStreamNonBlocking) != hipSuccess) {
    qsw_engine_destroy(s->engine);
    (void)hipFree(s->arena);
    delete s;
    return QSW_ERR_DEVICE;
  }
  s->direct_min_N = env_int("QSW_SERVER_DIRECT_N", 384);
  if (hipStreamCreateWithFlags(&s->direct_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipStreamDestroy(s->build_stream);
    qsw_engine_destroy(s->engine);
    (void)hipFree(s->arena);
    delete s;
    return QSW_ERR_DEVICE;
  }
  try {
    s->builder = std::thread(builder_main, s);
    s->runner = std::thread(runner_main, s);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
      s->cv_job.notify_all();
    }
    if (s->builder.joinable()) s->builder.join();
    (void)hipStreamDestroy(s->build_stream);
    (void)hipStreamDestroy(s->direct_stream);
    qsw_engine_destroy(s->engine);
    (void)hipFree(s->arena);
    delete s;
    return QSW_ERR_OOM;
  }
  *out = s;
  return QSW_OK;
}

void qsw_server_destroy(qsw_server_t s) {
  if (!s) return;
  DeviceGuard g(s->device);
  {
    // queued builds are dropped; the one in flight finishes
    std::lock_guard<std::mutex> lk(s->mu);
    s->in_flight -= (int)s->jobs.size();
    s->jobs.clear();
    s->d_in_flight -= (int)s->djobs.size();
    s->djobs.clear();
    s->stop = true;
    s->cv_job.notify_all();
  }
  if (s->builder.joinable()) s->builder.join();
  if (s->runner.joinable()) s->runner.join();
  (void)drain_builds(s);
  (void)drain_direct(s);
  if (s->dws) (void)hipFree(s->dws);
  if (s->dout) (void)hipFree(s->dout);
  if (s->direct_stream) (void)hipStreamDestroy(s->direct_stream);
  qsw_engine_destroy(s->engine);
  for (CachedOp *c : s->lru) {
    if (c->op) qsw_superop_destroy(c->op);
    delete c;
  }
  if (s->build_stream) (void)hipStreamDestroy(s->build_stream);
  for (auto &kv : s->by_id) delete kv.second;
  if (s->arena) (void)hipFree(s->arena);
  delete s;
}

qsw_status_t qsw_server_submit(qsw_server_t s, int32_t N, const int64_t *row_ptr,
                               const int32_t *col_idx, const double *w, double omega,
                               double gamma, uint32_t flags, const void *rho0, double t0,
                               double dt, int32_t n_steps, void *out, void *pops,
                               int64_t *request) {
  if (!s || !row_ptr || !rho0 || !request || N < 1 || n_steps < 0) return QSW_ERR_ARG;
  DeviceGuard g(s->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  const double t_submit = now_ms();
  OpKey key;
  key.N = N;
  key.omega = omega;
  key.gamma = gamma;
  key.flags = flags;
  const int64_t E = row_ptr[N];
  if (E < 0 || (E > 0 && (!col_idx || !w))) return QSW_ERR_ARG;
  key.rp.assign(row_ptr, row_ptr + N + 1);
  key.col.assign(col_idx, col_idx + E);
  key.w.assign(w, w + E);
  Fnv f;
  f.add(&N, sizeof N);
  f.add(&omega, sizeof omega);
  f.add(&gamma, sizeof gamma);
  f.add(&flags, sizeof flags);
  f.add(key.rp.data(), key.rp.size() * sizeof(int64_t));
  f.add(key.col.data(), key.col.size() * sizeof(int32_t));
  f.add(key.w.data(), key.w.size() * sizeof(double));
  CachedOp *c = find_op(s, f.h, key);
  if (c) {
    ++s->stats.cache_hits;
  } else {
    // built by the builder thread once the cache has room for it
    ++s->stats.cache_misses;
    c = new (std::nothrow) CachedOp();
    if (!c) return QSW_ERR_OOM;
    c->key = std::move(key);
    c->hash = f.h;
    c->bytes = op_bytes_bound(N, E);
    c->state = 1;
    s->cache.emplace(f.h, c);
    s->lru.push_front(c);
    s->waiting.push_back(c);
  }
  touch(s, c);
  ++c->users;
  Request *r = new (std::nothrow) Request();
  if (!r) {
    --c->users;
    return QSW_ERR_OOM;
  }
  r->id = s->next_id++;
  r->hash = f.h;
  r->cop = c;
  r->walk.op = c->op;
  r->walk.n0 = 1;
  r->walk.rho0 = rho0;
  r->walk.t0 = t0;
  r->walk.dt = dt;
  r->walk.n_steps = n_steps;
  r->walk.out = out;
  r->walk.pops = pops;
  r->t_submit = t_submit;
  if (c->state == 0) {
    const size_t need = qsw_walk_bytes(&r->walk, 1);
    if (need == 0 || need > engine_pool_bytes(s->engine)) {  // bad, or can never fit
      --c->users;
      delete r;
      return need == 0 ? QSW_ERR_ARG : QSW_ERR_OOM;
    }
  }
  s->by_id[r->id] = r;
  s->pending.push_back(r);
  ++s->stats.submitted;
  *request = r->id;
  start_builds(s);
  return admit(s);
}

qsw_status_t qsw_server_step(qsw_server_t s, int32_t max_cycles, int32_t *running,
                             int32_t *pending) {
  if (!s || max_cycles < 0) return QSW_ERR_ARG;
  DeviceGuard g(s->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  qsw_status_t build_err = drain_builds(s);
  {
    const qsw_status_t e2 = drain_direct(s);
    if (build_err == QSW_OK) build_err = e2;
  }
  start_builds(s);
  qsw_status_t st = admit(s);
  if (st != QSW_OK) return st;
  qsw_engine_stats_t es0{};
  (void)qsw_engine_stats(s->engine, &es0);
  if (es0.live == 0) {
    // the engine is idle and the other threads are busy (builds, the direct
    // lane): wait a little for one of them instead of returning at once
    bool busy;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      busy = (s->in_flight > 0 && !s->pending.empty()) || s->d_in_flight > 0;
      if (busy && s->built.empty() && s->failed.empty() && s->ddone.empty())
        s->cv_done.wait_for(lk, std::chrono::milliseconds(5));
    }
    if (busy) {
      qsw_status_t e2 = drain_builds(s);
      if (build_err == QSW_OK) build_err = e2;
      e2 = drain_direct(s);
      if (build_err == QSW_OK) build_err = e2;
      start_builds(s);
      st = admit(s);
      if (st != QSW_OK) return st;
    }
  }
  int32_t live = 0;
  st = qsw_engine_run(s->engine, max_cycles, &live);
  if (st != QSW_OK && st != QSW_ERR_NONFINITE) return st;
  int64_t tickets[256];
  int32_t cnt = 0;
  do {
    const qsw_status_t ps = qsw_engine_poll(s->engine, tickets, 256, &cnt);
    if (ps != QSW_OK) return ps;
    const double t = now_ms();
    for (int32_t i = 0; i < cnt; ++i) {
      auto it = s->by_ticket.find(tickets[i]);
      if (it == s->by_ticket.end()) continue;
      Request *r = it->second;
      s->by_ticket.erase(it);
      r->state = 2;
      r->t_done = t;
      s->done_ids.push_back(r->id);
      ++s->stats.completed;
      --r->cop->users;
    }
  } while (cnt == 256);
  {
    const qsw_status_t e2 = drain_direct(s);
    if (build_err == QSW_OK) build_err = e2;
  }
  evict_unused(s, 0);  // operators the finished walks released, if over budget
  start_builds(s);     // builds that waited for cache room
  st = admit(s);  // iteration-level admission into the space just freed
  if (st != QSW_OK) return st;
  int d_live = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    d_live = s->d_in_flight;
  }
  if (running) *running = live + d_live;
  if (pending) *pending = (int32_t)s->pending.size();
  qsw_engine_stats_t es{};
  (void)qsw_engine_stats(s->engine, &es);
  s->stats.cycles = es.cycles;
  s->stats.products = es.products;
  s->stats.cache_bytes = (int64_t)s->cache_used;
  return build_err;
}

qsw_status_t qsw_server_poll(qsw_server_t s, int64_t *requests, double *latency_ms,
                             int32_t capacity, int32_t *count) {
  if (!s || !count || capacity < 0 || (capacity > 0 && !requests)) return QSW_ERR_ARG;
  const int32_t n = (int32_t)std::min<size_t>((size_t)capacity, s->done_ids.size());
  for (int32_t i = 0; i < n; ++i) {
    const int64_t id = s->done_ids[i];
    requests[i] = id;
    auto it = s->by_id.find(id);
    if (it != s->by_id.end()) {
      if (latency_ms) latency_ms[i] = it->second->t_done - it->second->t_submit;
      delete it->second;
      s->by_id.erase(it);
    }
  }
  s->done_ids.erase(s->done_ids.begin(), s->done_ids.begin() + n);
  *count = n;
  return QSW_OK;
}

qsw_status_t qsw_server_stats(qsw_server_t s, qsw_server_stats_t *st) {
  if (!s || !st) return QSW_ERR_ARG;
  *st = s->stats;
  st->cache_bytes = (int64_t)s->cache_used;
  return QSW_OK;
}

}  // extern "C"
