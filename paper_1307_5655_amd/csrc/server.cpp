// Serving loop: continuous batching of evaluate and compose requests on one
// GPU.
//
// A host thread owns the device side.  Requests are queued by
// fpe_server_submit and admitted in arrival order while an in-flight slot is
// free and the bytes they use (points, outputs, condition output, fallback
// list, composition workspace, tree image) fit the HBM budget.  Admitted
// FP64 / compensated-FP32 evaluate requests are packed into a work table (two
// tables: walks of depth <= 8 and deeper ones) and run as one fused launch
// per table, replayed from a HIP graph whose nodes are
//   copy host table -> device, zero the fallback counters, fused walk,
//   fused FP64 fallback, copy counters device -> host;
// mod-p evaluate requests, FP64 requests on the term-parallel path and
// compose requests of the same batch run as their own launches after the
// graphs.  A graph is built once per slot and table and
// replayed unchanged: a batch is described entirely by the work table it
// copies in.  The two batch slots have a stream each (default priority), so
// the next batch is admitted, staged and launched while the previous one
// still runs, and its walk fills the previous one's fallback tail.  Each
// point's result depends only on its own walk, so a request's output is the
// same alone and in any mix.
//
// Device memory is the caller's: one buffer holds the slots' work tables and
// the pool that fallback lists and composition workspaces come from.
// Completed requests keep no state: a ticket below the next one that is not
// pending has completed.  Latencies go into a log-spaced histogram (bins
// 0.5 % wide), so statistics take constant memory however long the loop runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fpe_internal.h"

using namespace fpe;

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  fpe_request r;
  uint64_t ticket = 0;
  Clock::time_point t_submit;
  size_t ws_off = 0, ws_bytes = 0;   // pool scratch: fallback list or composition workspace
  size_t acct = 0;                   // bytes counted against the budget
  double term_evals = 0;
};

// First-fit allocator over [0, size), 256-byte granules.
struct Pool {
  size_t size = 0;
  std::map<size_t, size_t> free_;   // offset -> size
  void init(size_t b) {
    size = b;
    free_.clear();
    if (b) free_[0] = b;
  }
  bool alloc(size_t n, size_t& off) {
    n = (n + 255) & ~size_t(255);
    if (n == 0) {
      off = 0;
      return true;
    }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        off = it->first;
        size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~size_t(255);
    if (n == 0) return;
    auto it = free_.emplace(off, n).first;
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
};

// Latency histogram: bin k holds latencies in [kLo g^k, kLo g^(k+1)) ms,
// g = 1.005; bin 0 also takes everything below kLo.
constexpr double kLatLo = 1e-3;
constexpr double kLatG = 1.005;
constexpr int kLatBins = 4200;   // up to about 1.3e6 ms
struct LatHist {
  std::vector<int64_t> bins = std::vector<int64_t>(kLatBins, 0);
  int64_t n = 0;
  double sum = 0;
  void add(double ms) {
    int k = ms <= kLatLo ? 0 : (int)(std::log(ms / kLatLo) / std::log(kLatG));
    bins[std::min(std::max(k, 0), kLatBins - 1)]++;
    n++;
    sum += ms;
  }
  // the upper edge of the bin holding the q-quantile
  double quantile(double q) const {
    if (n == 0) return 0;
    const int64_t want = std::max<int64_t>(1, (int64_t)std::ceil(q * (double)n));
    int64_t c = 0;
    for (int k = 0; k < kLatBins; ++k) {
      c += bins[k];
      if (c >= want) return kLatLo * std::pow(kLatG, k + 1);
    }
    return kLatLo * std::pow(kLatG, kLatBins);
  }
};

struct Slot {
  // two work tables: [0] walks of depth <= 8, [1] deeper walks
  WorkTable* host[2] = {nullptr, nullptr};     // pinned staging
  WorkTable* dev[2] = {nullptr, nullptr};      // in the caller's workspace
  int64_t* host_counters[2] = {nullptr, nullptr};   // pinned copy-back
  hipGraph_t graph[2] = {nullptr, nullptr};   // one graph per table, launched only if it has work
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  void* args[2][1];
  WorkTable* argv[2];
  hipStream_t stream = nullptr;
  hipEvent_t ready_ev = nullptr;   // recorded on the caller's stream before the batch
  hipEvent_t done_ev = nullptr;
  bool busy = false;
  std::vector<Req> reqs[2];        // the fused requests of each table, in table order
  std::vector<Req> others;         // mod-p evaluate, FP64 term-path and compose requests
  double busy_start = 0;
};

}  // namespace

struct fpe_server {
  int device = 0;
  hipStream_t caller = nullptr;
  int32_t max_inflight = 64;
  size_t budget = 0, acct_used = 0;
  char* pool_dev = nullptr;
  Pool pool;
  Slot slots[2];
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req> queue;
  std::unordered_map<uint64_t, int> pending;   // queued or in flight
  uint64_t next_ticket = 1;
  int32_t inflight = 0;
  std::thread loop;
  std::atomic<bool> stop{false};
  std::string dev_err;
  // stats
  LatHist lat;
  int64_t submitted = 0, completed = 0, rejected = 0, batches = 0, compose_instances = 0;
  double term_evals = 0, busy_s = 0, fb_points = 0, f32c_points = 0;
  int busy_slots = 0;
  double busy_since = 0;
  Clock::time_point t0;
};

namespace {

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
inline size_t tables_bytes() { return 2 * 2 * align256(work_table_bytes()); }

// Scratch a request takes from the pool, and the bytes it counts against the
// budget.
size_t req_scratch(const fpe_request& r) {
  if (r.kind == FPE_REQ_COMPOSE) return compose_workspace_bytes(r.tree, r.dq);
  return r.domain == FPE_F32C ? (size_t)r.npts * sizeof(int32_t) : 0;
}
size_t req_bytes(const fpe_request& r) {
  const fpe_tree* t = r.tree;
  size_t b = t->dev_bytes + align256(req_scratch(r));
  if (r.kind == FPE_REQ_COMPOSE) {
    int32_t dp = 0;
    for (size_t i = 0; i < t->nodes.size(); ++i) dp = std::max(dp, t->exps[i * t->nvars]);
    b += (size_t)t->batch * ((size_t)(r.dq + 1) + (size_t)dp * r.dq + 1) * sizeof(uint32_t);
  } else {
    b += (size_t)r.npts * (8 * (size_t)t->nvars + 8 + (r.cond_out ? 4 : 0));
  }
  return b;
}
// Requests of the fused walk: compensated FP32, and FP64 on the tree walk
// (path 0, or 1 where the cost model keeps the walk).
bool fused(const fpe_request& r) {
  if (r.kind != FPE_REQ_EVALUATE) return false;
  if (r.domain == FPE_F32C) return true;
  return r.domain == FPE_F64 && (r.path == 0 || (r.path == 1 && !terms_preferred(r.tree, r.npts)));
}

fpe_status build_slot(fpe_server* s, Slot& sl, char* tables) {
  const size_t tb = work_table_bytes();
  for (int c = 0; c < 2; ++c) {
    if (hipHostMalloc((void**)&sl.host[c], tb, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.host_counters[c], sizeof(int64_t) * kMaxServe, hipHostMallocDefault) !=
            hipSuccess)
      return fail(FPE_ENOMEM, "server: pinned staging allocation failed");
    sl.dev[c] = (WorkTable*)(tables + c * align256(tb));
    std::memset(sl.host[c], 0, tb);
    std::memset(sl.host_counters[c], 0, sizeof(int64_t) * kMaxServe);
  }
  if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
    return fail(FPE_EDEVICE, "server: stream creation failed");
  if (hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&sl.ready_ev, hipEventDisableTiming) != hipSuccess)
    return fail(FPE_EDEVICE, "server: event creation failed");
  // one graph per table: copy -> zero -> walk -> fallback -> copy back (a
  // batch launches the graph of a table only when the table has requests)
  ServeKernels K = serve_kernels();
  for (int c = 0; c < 2; ++c) {
    if (hipGraphCreate(&sl.graph[c], 0) != hipSuccess) return fail(FPE_EDEVICE, "server: hipGraphCreate failed");
    sl.argv[c] = sl.dev[c];
    sl.args[c][0] = &sl.argv[c];
    hipGraphNode_t cp, z, w, f, back;
    if (hipGraphAddMemcpyNode1D(&cp, sl.graph[c], nullptr, 0, sl.dev[c], sl.host[c], tb, hipMemcpyHostToDevice) !=
        hipSuccess)
      return fail(FPE_EDEVICE, "server: graph memcpy node failed");
    hipKernelNodeParams zp{};
    zp.func = (void*)K.zero;
    zp.gridDim = dim3(1);
    zp.blockDim = dim3(256);
    zp.sharedMemBytes = 0;
    zp.kernelParams = sl.args[c];
    if (hipGraphAddKernelNode(&z, sl.graph[c], &cp, 1, &zp) != hipSuccess)
      return fail(FPE_EDEVICE, "server: graph kernel node failed");
    hipKernelNodeParams wp{};
    wp.func = (void*)(c == 0 ? K.walk8 : K.walk16);
    wp.gridDim = dim3(kServeGrid);
    wp.blockDim = dim3(64);
    wp.sharedMemBytes = (unsigned)K.walk_lds;
    wp.kernelParams = sl.args[c];
    if (hipGraphAddKernelNode(&w, sl.graph[c], &z, 1, &wp) != hipSuccess)
      return fail(FPE_EDEVICE, "server: graph kernel node failed");
    hipKernelNodeParams fp = wp;
    fp.func = (void*)(c == 0 ? K.fallback8 : K.fallback16);
    fp.sharedMemBytes = (unsigned)K.fallback_lds;
    fp.gridDim = dim3(kServeGrid);
    if (hipGraphAddKernelNode(&f, sl.graph[c], &w, 1, &fp) != hipSuccess)
      return fail(FPE_EDEVICE, "server: graph kernel node failed");
    if (hipGraphAddMemcpyNode1D(&back, sl.graph[c], &f, 1, sl.host_counters[c], table_counters(sl.dev[c]),
                                sizeof(int64_t) * kMaxServe, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(FPE_EDEVICE, "server: graph memcpy node failed");
    if (hipGraphInstantiate(&sl.exec[c], sl.graph[c], nullptr, nullptr, 0) != hipSuccess)
      return fail(FPE_EDEVICE, "server: hipGraphInstantiate failed");
  }
  (void)s;
  return FPE_OK;
}

double now_s(const fpe_server* s) { return std::chrono::duration<double>(Clock::now() - s->t0).count(); }

// Admit queued requests into a free slot and launch it.  Called with mu held.
bool try_launch(fpe_server* s, Slot& sl) {
  for (int c = 0; c < 2; ++c) sl.reqs[c].clear();
  sl.others.clear();
  // admit in arrival order (first come, first admitted) while a slot is free
  // and the request's bytes fit the budget
  int admitted = 0;
  while (!s->queue.empty() && s->inflight < s->max_inflight) {
    Req& q = s->queue.front();
    const int c = q.r.tree->depth <= 8 ? 0 : 1;
    if (fused(q.r) && (int)sl.reqs[c].size() == kMaxServe) break;
    if (s->acct_used + q.acct > s->budget) break;   // wait for memory to free up (FIFO)
    size_t off = 0;
    const size_t need = req_scratch(q.r);
    if (!s->pool.alloc(need, off)) break;
    q.ws_off = off;
    q.ws_bytes = need;
    s->acct_used += q.acct;
    s->inflight++;
    if (fused(q.r)) sl.reqs[c].push_back(q);
    else sl.others.push_back(q);
    s->queue.pop_front();
    ++admitted;
  }
  if (admitted == 0) return false;
  // lay the fused batch out with the longest walks first: the fused grid
  // takes blocks in table order, so the blocks that run longest start first
  // and the batch does not end on a tail of them
  int64_t blocks[2] = {0, 0};
  for (int c = 0; c < 2; ++c) {
    std::stable_sort(sl.reqs[c].begin(), sl.reqs[c].end(),
                     [](const Req& x, const Req& y) { return x.r.tree->ops64.size() > y.r.tree->ops64.size(); });
    int n = 0;
    for (const Req& q : sl.reqs[c]) {
      WorkItem& it = table_items(sl.host[c])[n];
      std::memset(&it, 0, sizeof it);
      it.tree = dev_view(q.r.tree);
      // requests walk the same programs as fpe_evaluate (runs for
      // chain-like trees), the double-double fallback of a compensated
      // request its FP64 program with runs
      if (q.r.domain == FPE_F64) it.tree.ops64 = it.tree.ops64r;
      if (q.r.domain == FPE_F32C) {
        it.tree.ops32 = it.tree.ops32r;
        it.tree.ops64 = it.tree.ops64r;
      }
      for (int j = 0; j < q.r.tree->nvars; ++j) it.pts[j] = (const double*)q.r.pts[j];
      it.out = (double*)q.r.out;
      it.cond = q.r.cond_out;
      it.list = (int32_t*)(s->pool_dev + q.ws_off);
      it.npts = q.r.npts;
      it.tol = q.r.tol > 0 ? q.r.tol : 1e-12;
      it.domain = q.r.domain;
      table_prefix(sl.host[c])[n] = blocks[c];
      blocks[c] += (q.r.npts + 63) / 64;
      n++;
    }
    sl.host[c]->n_items = n;
    sl.host[c]->total_blocks = blocks[c];
    table_prefix(sl.host[c])[n] = blocks[c];
  }
  // the batch waits for what the caller enqueued on its stream so far
  bool ok = hipEventRecord(sl.ready_ev, s->caller) == hipSuccess &&
            hipStreamWaitEvent(sl.stream, sl.ready_ev, 0) == hipSuccess;
  for (int c = 0; c < 2 && ok; ++c)
    if (!sl.reqs[c].empty()) ok = hipGraphLaunch(sl.exec[c], sl.stream) == hipSuccess;
  for (const Req& q : sl.others) {
    if (!ok) break;
    fpe_status st;
    if (q.r.kind == FPE_REQ_COMPOSE)
      st = launch_compose(q.r.tree, q.r.q, q.r.dq, (uint32_t*)q.r.out, s->pool_dev + q.ws_off, q.ws_bytes,
                          sl.stream);
    else {
      fpe_eval_opts eo{};
      eo.path = q.r.path;
      st = launch_eval(q.r.tree, q.r.pts, q.r.npts, q.r.out, &eo, sl.stream);
    }
    ok = st == FPE_OK;
  }
  if (!ok || hipEventRecord(sl.done_ev, sl.stream) != hipSuccess) s->dev_err = "server: batch launch failed";
  sl.busy = true;
  s->batches++;
  const double t = now_s(s);
  if (s->busy_slots++ == 0) s->busy_since = t;
  sl.busy_start = t;
  return true;
}

void complete(fpe_server* s, const Req& q, Clock::time_point now) {
  s->pool.release(q.ws_off, q.ws_bytes);
  s->acct_used -= q.acct;
  s->inflight--;
  s->completed++;
  s->term_evals += q.term_evals;
  if (q.r.kind == FPE_REQ_COMPOSE) s->compose_instances += q.r.tree->batch;
  s->lat.add(std::chrono::duration<double, std::milli>(now - q.t_submit).count());
  s->pending.erase(q.ticket);
}

void finish_slot(fpe_server* s, Slot& sl) {
  const auto now = Clock::now();
  for (int c = 0; c < 2; ++c) {
    for (size_t k = 0; k < sl.reqs[c].size(); ++k) {
      const Req& q = sl.reqs[c][k];
      if (q.r.domain == FPE_F32C) {
        s->f32c_points += (double)q.r.npts;
        s->fb_points += (double)sl.host_counters[c][k];
      }
      complete(s, q, now);
    }
    sl.reqs[c].clear();
  }
  for (const Req& q : sl.others) complete(s, q, now);
  sl.others.clear();
  sl.busy = false;
  if (--s->busy_slots == 0) s->busy_s += now_s(s) - s->busy_since;
}

void run_loop(fpe_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    bool progressed = false;
    for (auto& sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done_ev);
      if (q == hipSuccess) {
        finish_slot(s, sl);
        progressed = true;
        s->cv_done.notify_all();
      } else if (q != hipErrorNotReady) {
        // a failed batch: report it to every waiter instead of waiting forever
        s->dev_err = std::string("server: batch failed: ") + hipGetErrorString(q);
        s->cv_done.notify_all();
      }
    }
    if (!s->dev_err.empty()) {
      s->cv_done.notify_all();
      s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
      continue;
    }
    for (auto& sl : s->slots) {
      if (!sl.busy && !s->queue.empty()) {
        if (try_launch(s, sl)) progressed = true;
        break;   // one new batch per pass keeps the two slots alternating
      }
    }
    if (!progressed) {
      const bool any_busy = s->slots[0].busy || s->slots[1].busy;
      if (any_busy) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      } else {
        s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
      }
    }
  }
}

void release(fpe_server* s) {
  for (auto& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    for (int c = 0; c < 2; ++c) {
      if (sl.exec[c]) (void)hipGraphExecDestroy(sl.exec[c]);
      if (sl.graph[c]) (void)hipGraphDestroy(sl.graph[c]);
    }
    if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
    if (sl.ready_ev) (void)hipEventDestroy(sl.ready_ev);
    for (int c = 0; c < 2; ++c) {
      if (sl.host[c]) (void)hipHostFree(sl.host[c]);
      if (sl.host_counters[c]) (void)hipHostFree(sl.host_counters[c]);
    }
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete s;
}

}  // namespace

extern "C" {

size_t fpe_server_workspace_bytes(size_t hbm_budget) {
  // the pool holds the scratch of admitted requests, which the budget also
  // counts; granules of 256 bytes per request on top
  return tables_bytes() + align256(hbm_budget) + (size_t)256 * kMaxServe;
}

fpe_status fpe_server_create(void* workspace, size_t workspace_bytes, size_t hbm_budget, int32_t max_inflight,
                             void* stream, fpe_server** out) {
  if (!out) return fail(FPE_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_inflight < 1) return fail(FPE_EINVAL, "max_inflight must be >= 1");
  if (!workspace) return fail(FPE_EINVAL, "workspace is NULL");
  if (((uintptr_t)workspace) & 255) return fail(FPE_EINVAL, "workspace must be 256-byte aligned");
  if (workspace_bytes < fpe_server_workspace_bytes(hbm_budget))
    return fail(FPE_ENOMEM, "workspace smaller than fpe_server_workspace_bytes()");
  auto* s = new fpe_server();
  s->max_inflight = std::min<int32_t>(max_inflight, kMaxServe);
  s->t0 = Clock::now();
  s->caller = (hipStream_t)stream;
  s->budget = hbm_budget;
  (void)hipGetDevice(&s->device);
  char* base = (char*)workspace;
  s->pool_dev = base + tables_bytes();
  s->pool.init(workspace_bytes - tables_bytes());
  for (int k = 0; k < 2; ++k) {
    fpe_status st = build_slot(s, s->slots[k], base + k * 2 * align256(work_table_bytes()));
    if (st != FPE_OK) {
      release(s);
      return st;
    }
  }
  s->loop = std::thread(run_loop, s);
  *out = s;
  return FPE_OK;
}

fpe_status fpe_server_submit(fpe_server* s, const fpe_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return fail(FPE_EINVAL, "NULL argument");
  const fpe_tree* t = r->tree;
  if (!t || !t->dev) return fail(FPE_EINVAL, "request tree is not uploaded");
  if (t->domain != r->domain) return fail(FPE_EINVAL, "request domain differs from the tree's");
  if (r->kind == FPE_REQ_COMPOSE) {
    if (t->domain != FPE_MODP || t->modulus != kP31 || t->nvars != 1)
      return fail(FPE_EINVAL, "a compose request needs a univariate tree compiled mod 2^31-1");
    if (r->dq < 1 || !r->q || !r->out) return fail(FPE_EINVAL, "a compose request needs q, dq >= 1 and out");
    if (t->n_offtable > 0) return fail(FPE_EUNSUPPORTED, "composition needs every power in the table");
  } else if (r->kind == FPE_REQ_EVALUATE) {
    if (r->domain != FPE_F64 && r->domain != FPE_F32C && r->domain != FPE_MODP)
      return fail(FPE_EINVAL, "an evaluate request's domain must be F64, F32C or MODP");
    if (r->domain == FPE_MODP && t->modulus != kP61) return fail(FPE_EINVAL, "evaluation modulus must be 2^61-1");
    if (t->batch != 1) return fail(FPE_EINVAL, "a batch tree is for composition");
    if (r->npts < 0 || r->npts > 0x7fffffff) return fail(FPE_EINVAL, "npts out of range");
    if (!r->out && r->npts > 0) return fail(FPE_EINVAL, "NULL output array");
    for (int j = 0; j < t->nvars; ++j)
      if (r->npts > 0 && !r->pts[j]) return fail(FPE_EINVAL, "NULL point array");
    if (r->path < 0 || r->path > 2 || (r->domain == FPE_F32C && r->path != 0))
      return fail(FPE_EINVAL, "request path must be 0, 1 or 2 (0 for FPE_F32C)");
    if (r->path == 2 && !terms_eligible(t))
      return fail(FPE_EUNSUPPORTED, "the term-parallel path takes FPE_F64 and FPE_MODP (2^61-1) trees");
  } else {
    return fail(FPE_EINVAL, "unknown request kind");
  }
  if (t->depth > kMaxDepth) return fail(FPE_EUNSUPPORTED, "walk deeper than the kernels hold");
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->dev_err.empty()) return fail(FPE_EDEVICE, s->dev_err);
  Req q;
  q.r = *r;
  q.acct = req_bytes(*r);
  if (q.acct > s->budget || align256(req_scratch(*r)) > s->pool.size) {
    s->rejected++;
    return fail(FPE_EBUDGET, "request needs more bytes than the server's HBM budget");
  }
  q.ticket = s->next_ticket++;
  q.t_submit = Clock::now();
  q.term_evals = r->kind == FPE_REQ_EVALUATE ? (double)t->n_terms * (double)r->npts : 0.0;
  s->submitted++;
  *ticket = q.ticket;
  if (r->kind == FPE_REQ_EVALUATE && r->npts == 0) {
    s->completed++;
    s->lat.add(0.0);
    return FPE_OK;
  }
  s->pending.emplace(q.ticket, 0);
  s->queue.push_back(q);
  s->cv_work.notify_one();
  return FPE_OK;
}

fpe_status fpe_server_poll(fpe_server* s, uint64_t ticket, int32_t* done) {
  if (!s || !done) return fail(FPE_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->dev_err.empty()) return fail(FPE_EDEVICE, s->dev_err);
  if (ticket == 0 || ticket >= s->next_ticket) return fail(FPE_EINVAL, "unknown ticket");
  *done = s->pending.count(ticket) ? 0 : 1;
  return FPE_OK;
}

fpe_status fpe_server_wait(fpe_server* s, uint64_t ticket) {
  if (!s) return fail(FPE_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  if (ticket == 0 || ticket >= s->next_ticket) return fail(FPE_EINVAL, "unknown ticket");
  s->cv_done.wait(lk, [&] { return !s->pending.count(ticket) || !s->dev_err.empty(); });
  if (!s->dev_err.empty()) return fail(FPE_EDEVICE, s->dev_err);
  return FPE_OK;
}

fpe_status fpe_server_drain(fpe_server* s) {
  if (!s) return fail(FPE_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending.empty() || !s->dev_err.empty(); });
  if (!s->dev_err.empty()) return fail(FPE_EDEVICE, s->dev_err);
  return FPE_OK;
}

fpe_status fpe_server_stats(fpe_server* s, fpe_stats* st) {
  if (!s || !st) return fail(FPE_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(st, 0, sizeof *st);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->rejected = s->rejected;
  st->batches = s->batches;
  st->p50_ms = s->lat.quantile(0.50);
  st->p99_ms = s->lat.quantile(0.99);
  st->mean_ms = s->lat.n ? s->lat.sum / (double)s->lat.n : 0.0;
  st->term_evals = s->term_evals;
  st->busy_s = s->busy_s + (s->busy_slots > 0 ? now_s(s) - s->busy_since : 0.0);
  st->fallback_frac = s->f32c_points > 0 ? s->fb_points / s->f32c_points : 0.0;
  st->hbm_in_use = (int64_t)s->acct_used;
  st->compose_instances = s->compose_instances;
  return FPE_OK;
}

void fpe_server_destroy(fpe_server* s) {
  if (!s) return;
  if (s->loop.joinable()) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_done.wait(lk, [&] { return s->pending.empty() || !s->dev_err.empty(); });
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->loop.join();
  }
  release(s);
}

}  // extern "C"
