// Serving loop: continuous batching of evaluate requests on one GPU.
//
// A host thread owns the device side.  Requests are queued by
// fpe_server_submit and admitted in arrival order while a slot is free and
// their workspace fits the HBM budget (the fallback index list of a
// compensated-FP32 request: 4 bytes per point).  Admitted requests are packed
// into a work table (two tables: walks of depth <= 8 and deeper ones) and run
// as one fused launch per table, replayed from a HIP graph whose nodes are
//   copy host table -> device, zero the fallback counters, fused walk (x2),
//   fused FP64 fallback (x2), copy counters device -> host.
// The graph is built once per slot and replayed unchanged: a batch is
// described entirely by the work table it copies in.  Two batch slots alternate, so the next
// batch is admitted and staged while the previous one runs; requests that
// arrive meanwhile join the next batch.  Each point's result depends only on
// its own walk, so a request's output is the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
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
  uint64_t ticket;
  Clock::time_point t_submit;
  size_t ws_off = 0, ws_bytes = 0;
  bool done = false;
  fpe_status status = FPE_OK;
  double term_evals = 0;
};

// First-fit allocator over [0, budget), 256-byte granules.
struct Pool {
  size_t budget = 0;
  std::map<size_t, size_t> free_;   // offset -> size
  size_t used = 0;
  void init(size_t b) {
    budget = b;
    free_.clear();
    if (b) free_[0] = b;
    used = 0;
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
        used += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~size_t(255);
    if (n == 0) return;
    used -= n;
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

struct Slot {
  // two work tables: [0] walks of depth <= 8, [1] deeper walks
  WorkTable* host[2] = {nullptr, nullptr};     // pinned staging
  WorkTable* dev[2] = {nullptr, nullptr};
  int64_t* host_counters[2] = {nullptr, nullptr};   // pinned copy-back
  hipGraph_t graph[2] = {nullptr, nullptr};   // one graph per table, launched only if it has work
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  void* args[2][1];
  WorkTable* argv[2];
  hipEvent_t done_ev = nullptr;
  bool busy = false;
  std::vector<uint64_t> tickets[2];
  double busy_start = 0;
};

}  // namespace

struct fpe_server {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int32_t max_inflight = 64;
  char* pool_dev = nullptr;
  Pool pool;
  Slot slots[2];
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Req> reqs;
  uint64_t next_ticket = 1;
  int32_t inflight = 0;
  std::thread loop;
  std::atomic<bool> stop{false};
  std::string dev_err;
  // stats
  std::vector<double> lat_ms;
  int64_t submitted = 0, completed = 0, rejected = 0, batches = 0;
  double term_evals = 0, busy_s = 0, fb_points = 0, f32c_points = 0;
  Clock::time_point t0;
};

namespace {

size_t req_ws_bytes(const fpe_request& r) {
  return r.domain == FPE_F32C ? (size_t)r.npts * sizeof(int32_t) : 0;
}

fpe_status build_slot(fpe_server* s, Slot& sl) {
  const size_t tb = work_table_bytes();
  for (int c = 0; c < 2; ++c) {
    if (hipHostMalloc((void**)&sl.host[c], tb, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&sl.dev[c], tb) != hipSuccess ||
        hipHostMalloc((void**)&sl.host_counters[c], sizeof(int64_t) * kMaxServe, hipHostMallocDefault) !=
            hipSuccess)
      return fail(FPE_ENOMEM, "server: table allocation failed");
    std::memset(sl.host[c], 0, tb);
    std::memset(sl.host_counters[c], 0, sizeof(int64_t) * kMaxServe);
  }
  if (hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming) != hipSuccess)
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

// Admit queued requests into a free slot and launch it.  Called with mu held.
bool try_launch(fpe_server* s, Slot& sl) {
  sl.tickets[0].clear();
  sl.tickets[1].clear();
  int n[2] = {0, 0};
  int64_t blocks[2] = {0, 0};
  // admit in arrival order (first come, first admitted) ...
  std::vector<Req*> adm[2];
  while (!s->queue.empty() && s->inflight < s->max_inflight) {
    Req& q = s->reqs[s->queue.front()];
    const int c = q.r.tree->depth <= 8 ? 0 : 1;
    if ((int)adm[c].size() == kMaxServe) break;
    size_t need = req_ws_bytes(q.r);
    size_t off = 0;
    if (!s->pool.alloc(need, off)) break;     // wait for memory to free up (FIFO)
    q.ws_off = off;
    q.ws_bytes = need;
    s->queue.pop_front();
    s->inflight++;
    adm[c].push_back(&q);
  }
  // ... and lay the batch out with the longest walks first: the fused grid
  // takes blocks in table order, so the blocks that run longest start first
  // and the batch does not end on a tail of them
  for (int c = 0; c < 2; ++c)
    std::stable_sort(adm[c].begin(), adm[c].end(),
                     [](const Req* x, const Req* y) { return x->r.tree->ops64.size() > y->r.tree->ops64.size(); });
  for (int c = 0; c < 2; ++c) {
    for (Req* qp : adm[c]) {
      Req& q = *qp;
      WorkItem& it = table_items(sl.host[c])[n[c]];
      std::memset(&it, 0, sizeof it);
      it.tree = dev_view(q.r.tree);
      for (int j = 0; j < q.r.tree->nvars; ++j) it.pts[j] = q.r.pts[j];
      it.out = q.r.out;
      it.cond = q.r.cond_out;
      it.list = (int32_t*)(s->pool_dev + q.ws_off);
      it.npts = q.r.npts;
      it.tol = q.r.tol > 0 ? q.r.tol : 1e-12;
      it.domain = q.r.domain;
      table_prefix(sl.host[c])[n[c]] = blocks[c];
      blocks[c] += (q.r.npts + 63) / 64;
      sl.tickets[c].push_back(q.ticket);
      n[c]++;
    }
  }
  if (n[0] + n[1] == 0) return false;
  for (int c = 0; c < 2; ++c) {
    sl.host[c]->n_items = n[c];
    sl.host[c]->total_blocks = blocks[c];
    table_prefix(sl.host[c])[n[c]] = blocks[c];
  }
  bool ok = true;
  for (int c = 0; c < 2; ++c)
    if (n[c] > 0) ok = ok && hipGraphLaunch(sl.exec[c], s->stream) == hipSuccess;
  if (!ok || hipEventRecord(sl.done_ev, s->stream) != hipSuccess) s->dev_err = "server: graph launch failed";
  sl.busy = true;
  s->batches++;
  sl.busy_start = std::chrono::duration<double>(Clock::now() - s->t0).count();
  return true;
}

void finish_slot(fpe_server* s, Slot& sl) {
  const auto now = Clock::now();
  for (int c = 0; c < 2; ++c) {
    for (size_t k = 0; k < sl.tickets[c].size(); ++k) {
      auto it = s->reqs.find(sl.tickets[c][k]);
      if (it == s->reqs.end()) continue;
      Req& q = it->second;
      q.done = true;
      s->pool.release(q.ws_off, q.ws_bytes);
      s->inflight--;
      s->completed++;
      s->term_evals += q.term_evals;
      if (q.r.domain == FPE_F32C) {
        s->f32c_points += (double)q.r.npts;
        s->fb_points += (double)sl.host_counters[c][k];
      }
      s->lat_ms.push_back(std::chrono::duration<double, std::milli>(now - q.t_submit).count());
    }
  }
  s->busy_s += std::chrono::duration<double>(now - s->t0).count() - sl.busy_start;
  sl.busy = false;
}

void run_loop(fpe_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    bool progressed = false;
    for (auto& sl : s->slots) {
      if (sl.busy && hipEventQuery(sl.done_ev) == hipSuccess) {
        finish_slot(s, sl);
        progressed = true;
        s->cv_done.notify_all();
      }
    }
    for (auto& sl : s->slots) {
      if (!sl.busy && !s->queue.empty()) {
        if (try_launch(s, sl)) progressed = true;
        break;   // one new batch per pass keeps the two slots alternating
      }
    }
    if (!progressed) {
      bool any_busy = s->slots[0].busy || s->slots[1].busy;
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

}  // namespace

extern "C" {

fpe_status fpe_server_create(size_t hbm_budget, int32_t max_inflight, void* stream, fpe_server** out) {
  if (!out) return fail(FPE_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_inflight < 1) return fail(FPE_EINVAL, "max_inflight must be >= 1");
  auto* s = new fpe_server();
  s->max_inflight = std::min<int32_t>(max_inflight, kMaxServe);
  s->t0 = Clock::now();
  (void)hipGetDevice(&s->device);
  if (stream) {
    s->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      delete s;
      return fail(FPE_EDEVICE, "server: stream creation failed");
    }
    s->own_stream = true;
  }
  s->pool.init(hbm_budget);
  if (hbm_budget && hipMalloc((void**)&s->pool_dev, hbm_budget) != hipSuccess) {
    delete s;
    return fail(FPE_ENOMEM, "server: HBM budget allocation failed");
  }
  for (auto& sl : s->slots) {
    fpe_status st = build_slot(s, sl);
    if (st != FPE_OK) {
      fpe_server_destroy(s);
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
  if (r->domain != FPE_F64 && r->domain != FPE_F32C) return fail(FPE_EINVAL, "request domain must be F64 or F32C");
  if (t->domain != r->domain) return fail(FPE_EINVAL, "request domain differs from the tree's");
  if (t->batch != 1) return fail(FPE_EINVAL, "a batch tree is for fpe_compose");
  if (r->npts < 0 || r->npts > 0x7fffffff) return fail(FPE_EINVAL, "npts out of range");
  if (t->depth > kMaxDepth) return fail(FPE_EUNSUPPORTED, "walk deeper than the kernels hold");
  if (!r->out || (r->npts > 0 && !r->pts[0])) return fail(FPE_EINVAL, "NULL point or output array");
  for (int j = 0; j < t->nvars; ++j)
    if (r->npts > 0 && !r->pts[j]) return fail(FPE_EINVAL, "NULL point array");
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->dev_err.empty()) return fail(FPE_EDEVICE, s->dev_err);
  const size_t need = (req_ws_bytes(*r) + 255) & ~size_t(255);
  if (need > s->pool.budget) {
    s->rejected++;
    return fail(FPE_EBUDGET, "request workspace exceeds the server's HBM budget");
  }
  Req q;
  q.r = *r;
  q.ticket = s->next_ticket++;
  q.t_submit = Clock::now();
  q.term_evals = (double)t->n_terms * (double)r->npts;
  if (r->npts == 0) {
    q.done = true;
    s->completed++;
    s->lat_ms.push_back(0.0);
  } else {
    s->queue.push_back(q.ticket);
  }
  s->reqs.emplace(q.ticket, q);
  s->submitted++;
  *ticket = q.ticket;
  s->cv_work.notify_one();
  return FPE_OK;
}

fpe_status fpe_server_poll(fpe_server* s, uint64_t ticket, int32_t* done) {
  if (!s || !done) return fail(FPE_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->dev_err.empty()) return fail(FPE_EDEVICE, s->dev_err);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(FPE_EINVAL, "unknown ticket");
  *done = it->second.done ? 1 : 0;
  return FPE_OK;
}

fpe_status fpe_server_wait(fpe_server* s, uint64_t ticket) {
  if (!s) return fail(FPE_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(FPE_EINVAL, "unknown ticket");
  s->cv_done.wait(lk, [&] { return s->reqs[ticket].done || !s->dev_err.empty(); });
  if (!s->dev_err.empty()) return fail(FPE_EDEVICE, s->dev_err);
  return FPE_OK;
}

fpe_status fpe_server_drain(fpe_server* s) {
  if (!s) return fail(FPE_EINVAL, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] {
    return (s->queue.empty() && s->inflight == 0) || !s->dev_err.empty();
  });
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
  std::vector<double> v = s->lat_ms;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      size_t k = (size_t)std::min<double>((double)v.size() - 1, p * (double)(v.size() - 1) + 0.5);
      return v[k];
    };
    st->p50_ms = pct(0.50);
    st->p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    st->mean_ms = sum / (double)v.size();
  }
  st->term_evals = s->term_evals;
  st->busy_s = s->busy_s;
  st->fallback_frac = s->f32c_points > 0 ? s->fb_points / s->f32c_points : 0.0;
  st->hbm_in_use = (int64_t)s->pool.used;
  return FPE_OK;
}

void fpe_server_destroy(fpe_server* s) {
  if (!s) return;
  if (s->loop.joinable()) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_done.wait(lk, [&] { return (s->queue.empty() && s->inflight == 0) || !s->dev_err.empty(); });
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->loop.join();
  }
  (void)hipStreamSynchronize(s->stream);
  for (auto& sl : s->slots) {
    for (int c = 0; c < 2; ++c) {
      if (sl.exec[c]) (void)hipGraphExecDestroy(sl.exec[c]);
      if (sl.graph[c]) (void)hipGraphDestroy(sl.graph[c]);
    }
    if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
    for (int c = 0; c < 2; ++c) {
      if (sl.host[c]) (void)hipHostFree(sl.host[c]);
      if (sl.dev[c]) (void)hipFree(sl.dev[c]);
      if (sl.host_counters[c]) (void)hipHostFree(sl.host_counters[c]);
    }
  }
  if (s->pool_dev) (void)hipFree(s->pool_dev);
  if (s->own_stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
