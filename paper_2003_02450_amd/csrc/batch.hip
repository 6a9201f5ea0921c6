// Batched walks: the engine behind qsw_engine_* and qsw_batch_propagate.
//
// Many walks (each a handle, up to four density matrices as right-hand
// sides, and its own time grid) advance together.  A cycle is one launch of
// the control kernel (one thread per walk decides the walk's next operation
// from the norms of the one it just finished) and one launch of the work
// kernel (every 64-row block of every running walk carries out its walk's
// operation).  Small walks therefore share launches instead of each filling
// the GPU alone, each walk's matrix is read once for all its right-hand
// sides, and the host only waits between chunks of cycles.
//
// A chunk of cycles (kChunk control + work launch pairs) is captured once in
// a HIP graph and replayed while the running walks and the launch shape stay
// the same (a walk finishing or joining changes the arguments and the graph
// is captured again), so the host enqueues one graph launch per chunk.  The
// launch shape (workgroups per work launch and rho-row staging) is tuned on
// the first chunks of a run for the batch's key (right-hand sides, value
// precision, largest graph order, entries per row) and remembered for the
// process; no choice changes any sum, so results are bitwise the same.
//
// Device memory is the caller's arena: the tables at its start, then the
// walks' vectors, handed out first-fit and returned when a walk finishes.
// A walk is admitted only when its vectors fit (qsw_engine_submit returns
// QSW_ERR_OOM otherwise), so the footprint never exceeds the arena.
#include "handle.h"
#include "params.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>
#include <new>
#include <vector>

using namespace qsw;

namespace {

constexpr int kChunk = 16;  // cycles between host checks

// First-fit allocator over [0, size) in 256-byte units, coalescing on free.
class Pool {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool take(size_t bytes, size_t *off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    bytes = align256(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
};

// Bytes of one walk's vectors for R right-hand sides, and the most cycles
// its program can take (every Taylor term and power computed).
struct WalkPlan {
  Plan P;
  size_t vec = 0;    // one work vector (aligned)
  size_t total = 0;  // V[2], F[2], B[2], K[m] (series), kn
  int64_t max_cycles = 0;
};

qsw_status_t plan_walk(const qsw_walk_t *w, int32_t rhs, WalkPlan &W) {
  if (!w || !w->op || !w->rho0 || w->n0 < 1 || w->n0 > rhs || w->n_steps < 0) return QSW_ERR_ARG;
  qsw_status_t st = make_plan(w->op, w->t0, w->dt, w->n_steps, W.P);
  if (st != QSW_OK) return st;
  // single-precision products (one single-time application per interval):
  // two hi + lo state pairs and two terms of complex64
  const bool p32 = w->op->prec == QSW_PREC_FP32;
  W.vec = align256((size_t)w->op->n * rhs * (p32 ? sizeof(float2) : sizeof(double2)));
  W.total = 6 * W.vec;
  if (W.P.branch == 1)
    W.total += (size_t)W.P.m * W.vec + align256((size_t)(W.P.m + 1) * kBatchMaxRhs * sizeof(double));
  const int64_t q = w->n_steps;
  int64_t c = 3 + (int64_t)W.P.m0 * W.P.s0;  // load, start, first emit
  if (W.P.branch == 0)
    c += q * ((int64_t)W.P.m * W.P.s + 1);
  else
    c += ((int64_t)W.P.j + 1) * (1 + (int64_t)W.P.d * (W.P.m + 1));
  if (p32) c += q + 2;  // the reference trace and one trace check per point
  W.max_cycles = c + 2;
  return QSW_OK;
}

// Tables at the start of the arena for `cap` walks.
struct Tables {
  size_t inst = 0, ctl = 0, op = 0, slots = 0, act = 0, blk = 0, live = 0, nonfinite = 0,
         total = 0;
  explicit Tables(int32_t cap) {
    size_t o = 0;
    inst = o;  o += align256(sizeof(BatchInst) * (size_t)cap);
    ctl = o;   o += align256(sizeof(BatchCtl) * (size_t)cap);
    op = o;    o += align256(sizeof(BatchOp) * (size_t)cap);
    slots = o; o += align256(sizeof(BatchSlots) * (size_t)cap);
    act = o;   o += align256(sizeof(int32_t) * (size_t)cap);
    blk = o;   o += align256(sizeof(int64_t) * ((size_t)cap + 1));
    live = o;  o += 256;
    nonfinite = o; o += 256;
    total = o;
  }
};

// Entries of the block map for a pool of `pool` bytes: a walk's six work
// vectors take at least 6 * 64 * rhs * 8 bytes per full 64-row block
// (complex64 vectors), plus one ragged block per walk.
int64_t map_entries(size_t pool, int32_t rhs, int32_t cap) {
  return (int64_t)(pool / (6 * 64 * 8 * (size_t)rhs)) + cap + 1;
}

// Host copy of the control state read back after each chunk.
struct Readback {
  unsigned int live;
  int nonfinite;
};

}  // namespace

struct qsw_engine_s {
  int device = -1;
  int32_t cap = 0, rhs = 1;
  hipStream_t stream = nullptr;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  Tables tab{1};
  Pool pool;
  size_t pool_base = 0;
  BatchArgs args{};
  int resident = 0;
  // per slot
  std::vector<int64_t> ticket;   // -1: free
  std::vector<size_t> off, bytes;
  std::vector<int64_t> nwb;
  std::vector<int32_t> N;         // graph order of the walk in the slot
  std::vector<int64_t> deadline;  // cycle count by which the walk must have finished
  std::vector<char> running;
  std::vector<int32_t> act;      // running slots in block order
  std::vector<int64_t> finished; // tickets not yet polled
  int64_t next_ticket = 0;
  // pinned host staging
  BatchCtl *h_ctl = nullptr;     // cap entries
  Readback *h_rb = nullptr;
  int32_t *h_act = nullptr;
  int64_t *h_blk = nullptr;
  BatchInst *h_inst = nullptr;   // one entry (staging for a submit)
  int64_t blkmap_cap = 0;        // entries of the block map in the arena
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  qsw_engine_stats_t stats{};
  std::vector<double> wbytes;    // per slot: algorithmic bytes of one product
  std::vector<int> f32;          // per slot: single-precision values
  std::vector<int> p32;          // per slot: single-precision products
  std::vector<double> went;      // per slot: stored entries of the walk's layout
  // chunk graph: captured on a private stream, launched on `stream`
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  BatchArgs gargs{};
  int ggrid = 0, gchunk = 0, gkinds = 0;
  bool use_graph = true;
  // launch shape: work-launch grid = rounds x resident workgroups (at most
  // one wave per block), rho-row staging on or off
  int rounds = 1, stage = 1;
  bool tuned = false;
};

namespace {

void destroy_engine(qsw_engine_s *e) {
  if (!e) return;
  DeviceGuard g(e->device);
  if (e->h_ctl) (void)hipHostFree(e->h_ctl);
  if (e->h_rb) (void)hipHostFree(e->h_rb);
  if (e->h_act) (void)hipHostFree(e->h_act);
  if (e->h_blk) (void)hipHostFree(e->h_blk);
  if (e->h_inst) (void)hipHostFree(e->h_inst);
  if (e->ev0) (void)hipEventDestroy(e->ev0);
  if (e->ev1) (void)hipEventDestroy(e->ev1);
  if (e->ev_t0) (void)hipEventDestroy(e->ev_t0);
  if (e->ev_t1) (void)hipEventDestroy(e->ev_t1);
  if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
  if (e->cap_stream) (void)hipStreamDestroy(e->cap_stream);
  delete e;
}

// Upload the running list and its block prefix (stream-ordered).
qsw_status_t upload_active(qsw_engine_s *e) {
  e->act.clear();
  for (int32_t b = 0; b < e->cap; ++b)
    if (e->running[b]) e->act.push_back(b);
  int64_t acc = 0;
  for (size_t i = 0; i < e->act.size(); ++i) {
    e->h_act[i] = e->act[i];
    e->h_blk[i] = acc;
    acc += e->nwb[e->act[i]];
  }
  e->h_blk[e->act.size()] = acc;
  e->args.nact = (int32_t)e->act.size();
  e->args.nblocks = acc;
  // LDS for the largest rho-row (all rhs columns) that fits the staging budget
  int64_t sb = 0;
  for (int32_t b : e->act) {
    const int64_t need = (int64_t)e->rhs * e->N[b] * (int64_t)sizeof(double2);
    if (need <= (int64_t)kStageMaxBytes && need > sb) sb = need;
  }
  e->args.stage_bytes = (e->stage && env_int("QSW_STAGE", 1)) ? (int32_t)sb : 0;
  if (acc > e->blkmap_cap) return QSW_ERR_STATE;  // admission reserves the map entries
  if (!e->act.empty())
    HIP_TRY(hipMemcpyAsync(e->arena + e->tab.act, e->h_act, sizeof(int32_t) * e->act.size(),
                           hipMemcpyHostToDevice, e->stream));
  HIP_TRY(hipMemcpyAsync(e->arena + e->tab.blk, e->h_blk, sizeof(int64_t) * (e->act.size() + 1),
                         hipMemcpyHostToDevice, e->stream));
  HIP_TRY(launch_batch_blocks(e->args, e->stream));
  HIP_TRY(hipStreamSynchronize(e->stream));  // the staging buffers are reused
  return QSW_OK;
}

int64_t total_blocks(const qsw_engine_s *e) {
  int64_t t = 0;
  for (int32_t b : e->act) t += e->nwb[b];
  return t;
}

// Work kernels a cycle needs: bit 0 double products, bit 1 single-precision
// products (a walk's load, checks and emissions run in its own kind).
int work_kinds(const qsw_engine_s *e) {
  int k = 0;
  for (int32_t b : e->act) k |= e->p32[b] ? 2 : 1;
  return k;
}

hipError_t launch_cycle(const qsw_engine_s *e, int grid, int kinds, hipStream_t s) {
  hipError_t err = launch_batch_control(e->args, s);
  if (err == hipSuccess && (kinds & 1)) err = launch_batch_work(e->args, e->rhs, false, grid, s);
  if (err == hipSuccess && (kinds & 2)) err = launch_batch_work(e->args, e->rhs, true, grid, s);
  return err;
}

// Read back the control state; release finished walks.
qsw_status_t collect(qsw_engine_s *e) {
  HIP_TRY(hipMemcpyAsync(e->h_ctl, e->arena + e->tab.ctl, sizeof(BatchCtl) * (size_t)e->cap,
                         hipMemcpyDeviceToHost, e->stream));
  HIP_TRY(hipMemcpyAsync(&e->h_rb->live, e->arena + e->tab.live, sizeof(unsigned int),
                         hipMemcpyDeviceToHost, e->stream));
  HIP_TRY(hipMemcpyAsync(&e->h_rb->nonfinite, e->arena + e->tab.nonfinite, sizeof(int),
                         hipMemcpyDeviceToHost, e->stream));
  HIP_TRY(hipStreamSynchronize(e->stream));
  bool changed = false;
  for (int32_t b = 0; b < e->cap; ++b) {
    if (!e->running[b] || !e->h_ctl[b].done) continue;
    e->running[b] = 0;
    e->stats.products += e->h_ctl[b].products;
    e->stats.bytes += (double)e->h_ctl[b].products * e->wbytes[b];
    double tdev = 0.0;  // non-negative: its bits order as the values
    std::memcpy(&tdev, &e->h_ctl[b].trace_dev, sizeof(double));
    e->stats.trace_dev = std::max(e->stats.trace_dev, tdev);
    e->finished.push_back(e->ticket[b]);
    e->ticket[b] = -1;
    e->pool.give(e->off[b] - e->pool_base, e->bytes[b]);
    changed = true;
  }
  if (e->h_rb->nonfinite) e->stats.nonfinite = 1;
  int32_t live = 0;
  for (int32_t b = 0; b < e->cap; ++b) live += e->running[b] ? 1 : 0;
  e->stats.live = live;
  if (changed) return upload_active(e);
  return QSW_OK;
}

// Candidate launch shapes {rounds of resident workgroups, staging}.
constexpr int kTuneCount = 4;
constexpr int kTuneShapes[kTuneCount][2] = {{1, 1}, {2, 1}, {1, 0}, {2, 0}};

struct TuneKey {
  int rhs = 0, f32 = 0, p32 = 0, nlog = 0, epr = 0;
  bool operator<(const TuneKey &o) const {
    return std::tie(rhs, f32, p32, nlog, epr) < std::tie(o.rhs, o.f32, o.p32, o.nlog, o.epr);
  }
};

std::map<TuneKey, std::pair<int, int>> &tune_cache() {
  static std::map<TuneKey, std::pair<int, int>> c;
  return c;
}

// The batch's key: right-hand sides, single-precision values and
// single-precision products on any walk, log2 of the largest graph order,
// entries per row of all running walks.
TuneKey tune_key(const qsw_engine_s *e) {
  TuneKey k;
  k.rhs = e->rhs;
  int32_t nmax = 1;
  double ent = 0.0, rows = 0.0;
  for (int32_t b : e->act) {
    nmax = std::max(nmax, e->N[b]);
    k.f32 |= e->f32[b];
    k.p32 |= e->p32[b];
    ent += e->went[b];
    rows += (double)e->N[b] * e->N[b];
  }
  k.nlog = (int)std::ceil(std::log2((double)nmax));
  k.epr = rows > 0 ? (int)std::lround(ent / rows) : 0;
  return k;
}

void set_shape(qsw_engine_s *e, int rounds, int stage) {
  e->rounds = rounds;
  e->stage = stage;
}

// kChunk cycles (or fewer): control + work launch pairs, through the chunk
// graph when possible.  The graph is captured again when the arguments or
// the shape changed; any capture failure falls back to direct launches.
hipError_t run_chunk(qsw_engine_s *e, int grid, int chunk) {
  const int kinds = work_kinds(e);
  if (e->use_graph) {
    const bool same = e->gexec && e->ggrid == grid && e->gchunk == chunk && e->gkinds == kinds &&
                      std::memcmp(&e->gargs, &e->args, sizeof(BatchArgs)) == 0;
    if (!same) {
      if (e->gexec) {
        (void)hipGraphExecDestroy(e->gexec);
        e->gexec = nullptr;
      }
      hipError_t err = hipStreamBeginCapture(e->cap_stream, hipStreamCaptureModeThreadLocal);
      if (err == hipSuccess) {
        for (int c = 0; c < chunk && err == hipSuccess; ++c)
          err = launch_cycle(e, grid, kinds, e->cap_stream);
        hipGraph_t graph = nullptr;
        const hipError_t end = hipStreamEndCapture(e->cap_stream, &graph);
        if (err == hipSuccess) err = end;
        if (err == hipSuccess) err = hipGraphInstantiate(&e->gexec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
      }
      if (err != hipSuccess || !e->gexec) {
        (void)hipGetLastError();
        if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
        e->gexec = nullptr;
        e->use_graph = false;  // direct launches from now on
      } else {
        e->gargs = e->args;
        e->ggrid = grid;
        e->gchunk = chunk;
        e->gkinds = kinds;
        e->stats.graphs += 1;
      }
    }
    if (e->use_graph) {
      e->stats.graph_launches += 1;
      return hipGraphLaunch(e->gexec, e->stream);
    }
  }
  for (int c = 0; c < chunk; ++c) {
    hipError_t err = launch_cycle(e, grid, kinds, e->stream);
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

}  // namespace

size_t qsw::engine_pool_bytes(const qsw_engine_s *e) {
  return e ? e->arena_bytes - e->pool_base : 0;
}

extern "C" {

size_t qsw_walk_bytes(const qsw_walk_t *walk, int32_t rhs) {
  if (rhs != 1 && rhs != 2 && rhs != 4) return 0;
  WalkPlan W;
  if (plan_walk(walk, rhs, W) != QSW_OK) return 0;
  return W.total;
}

size_t qsw_engine_table_bytes(int32_t max_walks) {
  if (max_walks < 1) return 0;
  return Tables(max_walks).total;
}

qsw_status_t qsw_engine_create(int32_t max_walks, int32_t rhs, void *arena, size_t arena_bytes,
                               void *hip_stream, qsw_engine_t *out) {
  if (!out) return QSW_ERR_ARG;
  *out = nullptr;
  if (max_walks < 1 || (rhs != 1 && rhs != 2 && rhs != 4) || !arena) return QSW_ERR_ARG;
  if ((uintptr_t)arena & 255) return QSW_ERR_STATE;
  Tables tab(max_walks);
  if (arena_bytes < tab.total) return QSW_ERR_STATE;
  qsw_engine_s *e = new (std::nothrow) qsw_engine_s();
  if (!e) return QSW_ERR_OOM;
  auto fail = [&](qsw_status_t st) {
    destroy_engine(e);
    return st;
  };
  if (hipGetDevice(&e->device) != hipSuccess) return fail(QSW_ERR_DEVICE);
  e->cap = max_walks;
  e->rhs = rhs;
  e->stream = (hipStream_t)hip_stream;
  e->arena = (char *)arena;
  e->arena_bytes = arena_bytes;
  e->tab = tab;
  e->blkmap_cap = map_entries(arena_bytes - tab.total, rhs, max_walks);
  const size_t map_bytes = align256(sizeof(int2) * (size_t)e->blkmap_cap);
  if (arena_bytes < tab.total + map_bytes) return fail(QSW_ERR_STATE);
  e->pool_base = tab.total + map_bytes;
  e->pool.reset(arena_bytes - e->pool_base);
  e->ticket.assign(max_walks, -1);
  e->off.assign(max_walks, 0);
  e->bytes.assign(max_walks, 0);
  e->nwb.assign(max_walks, 0);
  e->N.assign(max_walks, 0);
  e->deadline.assign(max_walks, 0);
  e->running.assign(max_walks, 0);
  e->wbytes.assign(max_walks, 0.0);
  e->f32.assign(max_walks, 0);
  e->p32.assign(max_walks, 0);
  e->went.assign(max_walks, 0.0);
  e->use_graph = env_int("QSW_BATCH_GRAPH", 1) != 0;
  if (hipStreamCreate(&e->cap_stream) != hipSuccess) return fail(QSW_ERR_DEVICE);
  if (hipHostMalloc((void **)&e->h_ctl, sizeof(BatchCtl) * (size_t)max_walks) != hipSuccess ||
      hipHostMalloc((void **)&e->h_rb, sizeof(Readback)) != hipSuccess ||
      hipHostMalloc((void **)&e->h_act, sizeof(int32_t) * ((size_t)max_walks + 1)) != hipSuccess ||
      hipHostMalloc((void **)&e->h_blk, sizeof(int64_t) * ((size_t)max_walks + 1)) != hipSuccess ||
      hipHostMalloc((void **)&e->h_inst, sizeof(BatchInst)) != hipSuccess)
    return fail(QSW_ERR_OOM);
  if (hipEventCreate(&e->ev0) != hipSuccess || hipEventCreate(&e->ev1) != hipSuccess ||
      hipEventCreate(&e->ev_t0) != hipSuccess || hipEventCreate(&e->ev_t1) != hipSuccess)
    return fail(QSW_ERR_DEVICE);
  BatchArgs &A = e->args;
  A.inst = (const BatchInst *)(e->arena + tab.inst);
  A.ctl = (BatchCtl *)(e->arena + tab.ctl);
  A.op = (BatchOp *)(e->arena + tab.op);
  A.slots = (BatchSlots *)(e->arena + tab.slots);
  A.act = (const int32_t *)(e->arena + tab.act);
  A.blk_start = (const int64_t *)(e->arena + tab.blk);
  A.count = max_walks;
  A.nact = 0;
  A.live = (unsigned int *)(e->arena + tab.live);
  A.nonfinite = (int *)(e->arena + tab.nonfinite);
  A.blkmap = (int2 *)(e->arena + tab.total);
  // every slot starts finished (control skips it), no op, zero slots
  if (launch_zero(e->arena, tab.total, e->stream) != hipSuccess) return fail(QSW_ERR_DEVICE);
  for (int32_t b = 0; b < max_walks; ++b) {
    std::memset(&e->h_ctl[b], 0, sizeof(BatchCtl));
    e->h_ctl[b].done = 1;
  }
  if (hipMemcpyAsync(e->arena + tab.ctl, e->h_ctl, sizeof(BatchCtl) * (size_t)max_walks,
                     hipMemcpyHostToDevice, e->stream) != hipSuccess)
    return fail(QSW_ERR_DEVICE);
  if (upload_active(e) != QSW_OK) return fail(QSW_ERR_DEVICE);
  e->resident = batch_resident_workgroups(rhs);
  *out = e;
  return QSW_OK;
}

void qsw_engine_destroy(qsw_engine_t e) {
  if (!e) return;
  {
    DeviceGuard g(e->device);
    (void)hipStreamSynchronize(e->stream);
  }
  destroy_engine(e);
}

qsw_status_t qsw_engine_submit(qsw_engine_t e, const qsw_walk_t *w, int64_t *ticket) {
  if (!e || !w || !ticket) return QSW_ERR_ARG;
  WalkPlan W;
  qsw_status_t st = plan_walk(w, e->rhs, W);  // checks w->op
  if (st != QSW_OK) return st;
  if (w->op->device != e->device) return QSW_ERR_STATE;
  int32_t b = -1;
  for (int32_t i = 0; i < e->cap; ++i)
    if (e->ticket[i] < 0) {
      b = i;
      break;
    }
  size_t off = 0;
  if (b < 0 || total_blocks(e) + w->op->nwb > e->blkmap_cap || !e->pool.take(W.total, &off))
    return QSW_ERR_OOM;  // not admitted now
  DeviceGuard g(e->device);
  if (!g.ok) {
    e->pool.give(off, W.total);
    return QSW_ERR_DEVICE;
  }
  const qsw_superop_s *h = w->op;
  char *base = e->arena + e->pool_base + off;
  BatchInst &I = *e->h_inst;
  std::memset(&I, 0, sizeof(I));
  I.rp = h->row_ptr;
  I.wcol = h->wcol;
  I.wval = h->wval;
  I.wval32 = h->wval32;
  I.wcoef = h->wcoef;
  I.wcoef32 = h->wcoef32;
  I.wdiag = h->wdiag;
  I.wdiag32 = h->wdiag32;
  I.wstart = h->wstart;
  I.wshn = h->wshared > 0 ? h->wshn : nullptr;
  I.wshs = h->wshs;
  I.wsh_stride = h->wsh_stride;
  I.wsh = h->wsh;
  I.split = h->split ? 1 : 0;
  I.wlen = h->wlen;
  I.wperm = h->wperm;
  I.n = h->n;
  I.nwb = h->nwb;
  I.vlen = h->n * e->rhs;
  I.N = h->N;
  I.f32 = h->prec == QSW_PREC_SINGLE ? 1 : 0;
  I.branch = W.P.branch;
  I.m = W.P.m;
  I.s = W.P.s;
  I.m0 = W.P.m0;
  I.s0 = W.P.s0;
  I.d = W.P.d;
  I.jb = W.P.j;
  I.r = W.P.r;
  I.q = w->n_steps;
  I.n0 = w->n0;
  I.t0 = w->t0;
  I.dt = w->dt;
  I.tol = tol_of(h->prec);
  for (int v = 0; v < 2; ++v) {
    I.V[v] = (double2 *)(base + (size_t)v * W.vec);
    I.F[v] = (double2 *)(base + (size_t)(2 + v) * W.vec);
    I.B[v] = (double2 *)(base + (size_t)(4 + v) * W.vec);
  }
  size_t o = 6 * W.vec;
  if (W.P.branch == 1) {
    I.K = (double2 *)(base + o);
    o += (size_t)W.P.m * W.vec;
    I.kn = (double *)(base + o);
  }
  I.rho0 = (const double2 *)w->rho0;
  I.out = (double2 *)w->out;
  I.pops = (double *)w->pops;
  I.prec32 = h->prec == QSW_PREC_FP32 ? 1 : 0;
  if (I.prec32) {
    // the same six vectors as hi + lo state pairs and terms of complex64
    for (int v = 0; v < 2; ++v) {
      I.Ph[v] = (float2 *)(base + (size_t)(2 * v) * W.vec);
      I.Pl[v] = (float2 *)(base + (size_t)(2 * v + 1) * W.vec);
      I.B32[v] = (float2 *)(base + (size_t)(4 + v) * W.vec);
      I.V[v] = I.F[v] = I.B[v] = nullptr;
    }
  }
  BatchCtl &C = e->h_ctl[b];
  std::memset(&C, 0, sizeof(C));
  C.pc = 0;  // load
  HIP_TRY(hipMemcpyAsync(e->arena + e->tab.inst + sizeof(BatchInst) * (size_t)b, &I,
                         sizeof(BatchInst), hipMemcpyHostToDevice, e->stream));
  HIP_TRY(hipMemcpyAsync(e->arena + e->tab.ctl + sizeof(BatchCtl) * (size_t)b, &C,
                         sizeof(BatchCtl), hipMemcpyHostToDevice, e->stream));
  HIP_TRY(launch_zero(e->arena + e->tab.slots + sizeof(BatchSlots) * (size_t)b,
                      sizeof(BatchSlots), e->stream));
  e->ticket[b] = e->next_ticket++;
  e->off[b] = e->pool_base + off;
  e->bytes[b] = W.total;
  e->nwb[b] = h->nwb;
  {
    // one product: each stored entry's column and value, the block-shared
    // entries, row data and the diagonal per row, and for every column x
    // read, the term written and the accumulator read and written (64
    // bytes per element; 48 with single-precision products: complex64 x and
    // term, the accumulator a pair of complex64)
    const bool p32 = I.prec32 != 0;
    const bool f32 = I.f32 != 0 || p32, split = I.split != 0;
    const double entry = split ? (f32 ? 8.0 : 12.0) : (f32 ? 12.0 : 20.0);
    const double diag = split ? (f32 ? 8.0 : 16.0) : 0.0;
    e->wbytes[b] = entry * (double)h->wentries + 16.0 * (double)h->wshared +
                   8.0 * (double)(h->n + 1) + diag * (double)h->n +
                   (p32 ? 48.0 : 64.0) * (double)e->rhs * (double)h->n;
    e->f32[b] = I.f32 != 0 ? 1 : 0;
    e->p32[b] = p32 ? 1 : 0;
    e->went[b] = (double)h->wentries;
  }
  e->N[b] = h->N;
  e->deadline[b] = e->stats.cycles + W.max_cycles + kChunk;
  e->running[b] = 1;
  *ticket = e->ticket[b];
  return upload_active(e);  // synchronises: the staging entries are free again
}

qsw_status_t qsw_engine_run(qsw_engine_t e, int32_t max_cycles, int32_t *live) {
  if (!e || max_cycles < 0) return QSW_ERR_ARG;
  DeviceGuard g(e->device);
  if (!g.ok) return QSW_ERR_DEVICE;
  HIP_TRY(hipEventRecord(e->ev0, e->stream));
  int32_t done_cycles = 0;
  // tuning: one chunk per candidate shape, timed on the stream, while the
  // batch's key has no remembered shape
  TuneKey key{};
  int cand = -1;
  std::vector<double> cand_us;
  if (!e->tuned && env_int("QSW_BATCH_TUNE", 1) != 0 && !e->act.empty()) {
    key = tune_key(e);
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
      set_shape(e, it->second.first, it->second.second);
      e->tuned = true;
    } else {
      cand = 0;
      set_shape(e, kTuneShapes[0][0], kTuneShapes[0][1]);
    }
  }
  while (done_cycles < max_cycles && !e->act.empty()) {
    const int64_t tb = total_blocks(e);
    const int64_t want = (tb + kBlockThreads / 64 - 1) / (kBlockThreads / 64);
    const int64_t res = (int64_t)std::max(e->resident, 1) * e->rounds;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, res));
    const int chunk = std::min(kChunk, max_cycles - done_cycles);
    if (cand >= 0) HIP_TRY(hipEventRecord(e->ev_t0, e->stream));
    HIP_TRY(run_chunk(e, grid, chunk));
    if (cand >= 0) HIP_TRY(hipEventRecord(e->ev_t1, e->stream));
    done_cycles += chunk;
    e->stats.cycles += chunk;
    qsw_status_t st = collect(e);
    if (st != QSW_OK) return st;
    if (cand >= 0) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e->ev_t0, e->ev_t1));
      // per block of work, so that shrinking batches compare fairly
      cand_us.push_back(1e3 * ms / (double)std::max<int64_t>(1, tb));
      ++cand;
      if (cand < kTuneCount && !e->act.empty()) {
        set_shape(e, kTuneShapes[cand][0], kTuneShapes[cand][1]);
      } else {
        const int best = (int)(std::min_element(cand_us.begin(), cand_us.end()) - cand_us.begin());
        set_shape(e, kTuneShapes[best][0], kTuneShapes[best][1]);
        tune_cache()[key] = {e->rounds, e->stage};
        e->tuned = true;
        cand = -1;
      }
      if (e->stage != (e->args.stage_bytes > 0 ? 1 : 0)) {
        st = upload_active(e);  // staging changed: new LDS size
        if (st != QSW_OK) return st;
      }
    }
    for (int32_t b : e->act)
      if (e->stats.cycles > e->deadline[b]) return QSW_ERR_STATE;  // cannot happen
  }
  HIP_TRY(hipEventRecord(e->ev1, e->stream));
  HIP_TRY(hipEventSynchronize(e->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e->ev0, e->ev1));
  e->stats.ms = ms;
  e->stats.rounds = e->rounds;
  e->stats.staged = e->stage;
  if (live) *live = e->stats.live;
  return e->stats.nonfinite ? QSW_ERR_NONFINITE : QSW_OK;
}

qsw_status_t qsw_engine_poll(qsw_engine_t e, int64_t *tickets, int32_t capacity, int32_t *count) {
  if (!e || !count || capacity < 0 || (capacity > 0 && !tickets)) return QSW_ERR_ARG;
  const int32_t n = (int32_t)std::min<size_t>((size_t)capacity, e->finished.size());
  for (int32_t i = 0; i < n; ++i) tickets[i] = e->finished[i];
  e->finished.erase(e->finished.begin(), e->finished.begin() + n);
  *count = n;
  return QSW_OK;
}

qsw_status_t qsw_engine_stats(qsw_engine_t e, qsw_engine_stats_t *st) {
  if (!e || !st) return QSW_ERR_ARG;
  *st = e->stats;
  return QSW_OK;
}

size_t qsw_batch_workspace_bytes(const qsw_walk_t *walks, int32_t count, int32_t rhs) {
  if (!walks || count < 1 || (rhs != 1 && rhs != 2 && rhs != 4)) return 0;
  const size_t tab = Tables(count).total;
  size_t walks_bytes = 0;
  for (int32_t i = 0; i < count; ++i) {
    WalkPlan W;
    if (plan_walk(&walks[i], rhs, W) != QSW_OK) return 0;
    walks_bytes += W.total;
  }
  // X = walks + map(X): the engine reserves the map from what follows the
  // tables, so X leaves exactly walks_bytes for the walks (+256 for the
  // map's rounding)
  size_t X = walks_bytes + 256;
  for (int it = 0; it < 8; ++it) {
    const size_t nx = walks_bytes + 256 + align256(sizeof(int2) * (size_t)map_entries(X, rhs, count));
    if (nx == X) break;
    X = nx;
  }
  return tab + X;
}

qsw_status_t qsw_batch_propagate(const qsw_walk_t *walks, int32_t count, int32_t rhs,
                                 void *workspace, size_t ws_bytes, void *hip_stream,
                                 qsw_engine_stats_t *stats) {
  if (!walks || count < 1) return QSW_ERR_ARG;
  const size_t need = qsw_batch_workspace_bytes(walks, count, rhs);
  if (need == 0) return QSW_ERR_ARG;
  if (ws_bytes < need) return QSW_ERR_STATE;
  qsw_engine_t e = nullptr;
  qsw_status_t st = qsw_engine_create(count, rhs, workspace, ws_bytes, hip_stream, &e);
  if (st != QSW_OK) return st;
  for (int32_t i = 0; i < count && st == QSW_OK; ++i) {
    int64_t t = 0;
    st = qsw_engine_submit(e, &walks[i], &t);
  }
  if (st == QSW_OK) {
    int32_t live = 0;
    // every walk's op count is finite; the bound guards against a runaway
    st = qsw_engine_run(e, INT32_MAX, &live);
    if (st == QSW_OK && live != 0) st = QSW_ERR_STATE;
  }
  if (stats) (void)qsw_engine_stats(e, stats);
  qsw_engine_destroy(e);
  return st;
}

}  // extern "C"
