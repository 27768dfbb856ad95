// gc_serve.hip -- a request server with continuous batching.
//
// Clients register graphs (raw pairs kept in host memory) and submit queries:
// a triangle count (Sec. III-A) or the size of a k-truss (Sec. III-B) of a
// registered graph.  A scheduler thread owns the device:
//   * a device CSR cache: a graph is built on first use (gc_build_csr) and
//     kept until memory is needed; eviction is least-recently-used among
//     graphs no request is using;
//   * admission by HBM footprint: a build is started only if the budget holds
//     its peak (raw pairs, sort buffers and the CSR it produces); otherwise
//     idle graphs are evicted, and if that is not enough the request waits;
//   * continuous batching: every triangle-count request whose graph is
//     resident is taken into the next batch, and a batch is one launch per
//     degree bin over all its graphs (device descriptors, per-graph counters).
//     While a batch runs, newly arrived requests are admitted and built, and
//     form the next batch as soon as the running one completes;
//   * k-truss requests run on a worker thread with its own stream (their
//     rounds synchronise with the host), overlapping the count batches.
// Mode 1 ("per call") serves one request at a time in arrival order with the
// same cache, for comparison.
//
// Timestamps are CLOCK_MONOTONIC seconds (std::chrono::steady_clock).
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gc_graph.h"

struct gc_server_graph {
  std::vector<int32_t> src, dst;
  int32_t n = 0;
  gc_graph *g = nullptr;   // resident device CSR, or null
  int64_t charged = 0;     // bytes charged against the budget while resident
  int pins = 0;            // admitted requests that need it resident
  uint64_t last_use = 0;
  bool building = false;
};

struct gc_server_req {
  int64_t ticket = 0;
  int32_t graph_id = 0, kind = 0, k = 0;
  int32_t status = GC_PENDING;
  int64_t value = 0;
  int64_t edges = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  bool admitted = false;
};

struct gc_server {
  int device = 0;
  int64_t budget = 0;
  int64_t used = 0, peak = 0;
  int32_t mode = 0;  // 0 continuous batching, 1 one request at a time
  std::deque<gc_server_graph> graphs;  // deque: references stay valid as graphs are added
  std::unordered_map<int64_t, gc_server_req> reqs;
  std::deque<int64_t> pending;   // not yet admitted, arrival order
  std::deque<int64_t> ready_tc;  // admitted triangle counts waiting for a batch
  std::deque<int64_t> truss_q;   // admitted k-truss queries for the worker
  int64_t next_ticket = 1;
  uint64_t clock = 0;
  bool stop = false;
  std::mutex mu;
  std::condition_variable cv, done_cv, truss_cv;
  std::thread sched, worker;
  hipStream_t s_count = nullptr, s_build = nullptr, s_truss = nullptr;
  // running count batch
  std::vector<int64_t> batch;     // tickets
  std::vector<int32_t> batch_g;   // graph ids
  hipEvent_t batch_done = nullptr;
  bool batch_running = false;
  // batch buffers
  gc::DeviceBuffer d_desc, d_pre, d_out;
  // pinned host staging (reused only after the batch that read it completed)
  gc::GraphDesc *h_desc = nullptr;
  int64_t *h_pre = nullptr;
  unsigned long long *h_out = nullptr;
  size_t h_cap = 0;
  // statistics
  int64_t n_done = 0, n_batches = 0, max_batch = 0, n_builds = 0, n_evict = 0, n_deferred = 0;
  int truss_running = 0;
  std::string error;
};

namespace gc {

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Bytes reserved for building a graph of P pairs and n vertices: the raw
// pairs and the build's sort / scan buffers (about 80 bytes per pair), and
// never less than what the graph is charged once resident (below), since
// m <= P: the handle holds about 57 m + 32 n bytes, the k-truss rounds need
// up to 64 m + 16 n more.
static int64_t build_peak_bytes(int64_t P, int64_t n) {
  return 128 * P + 64 * n + (64 << 20);
}

// Bytes a resident graph is charged: its handle plus room for k-truss rounds,
// capped by its build reservation.
static int64_t resident_bytes(const gc_graph *g, int64_t P) {
  const int64_t want = (int64_t)g->device_bytes() + 64 * g->m + 16 * (int64_t)g->n + (16 << 20);
  return std::min(want, build_peak_bytes(P, g->n));
}

// Evict idle resident graphs (least recently used first) until `need` fits.
static bool make_room(gc_server *sv, int64_t need) {
  while (sv->used + need > sv->budget) {
    int best = -1;
    for (size_t i = 0; i < sv->graphs.size(); ++i) {
      const gc_server_graph &G = sv->graphs[i];
      if (G.g && G.pins == 0 && !G.building &&
          (best < 0 || G.last_use < sv->graphs[best].last_use))
        best = (int)i;
    }
    if (best < 0) return false;
    gc_server_graph &G = sv->graphs[best];
    gc_graph_free(G.g);
    G.g = nullptr;
    sv->used -= G.charged;
    G.charged = 0;
    ++sv->n_evict;
  }
  return true;
}

// Build graph `id` (called with the lock released; `building` set by caller).
static gc_status build_graph(gc_server *sv, gc_server_graph &G) {
  const int64_t P = (int64_t)G.src.size();
  DeviceBuffer ds, dd;  // freed below on every path
  gc_status st = dalloc(ds, sizeof(int32_t) * (size_t)(P + 1));
  if (st == GC_OK) st = dalloc(dd, sizeof(int32_t) * (size_t)(P + 1));
  if (st == GC_OK && P > 0) {
    if (hipMemcpyAsync(ds.ptr, G.src.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice,
                       sv->s_build) != hipSuccess ||
        hipMemcpyAsync(dd.ptr, G.dst.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice,
                       sv->s_build) != hipSuccess)
      st = GC_EDEVICE;
  }
  gc_graph *g = nullptr;
  if (st == GC_OK)
    st = gc_build_csr(static_cast<int32_t *>(ds.ptr), static_cast<int32_t *>(dd.ptr), P, G.n, 0,
                      sv->s_build, &g);
  if (st == GC_OK && g->m > 0) {
    st = build_units(g->csr.view(g->n, (int32_t)g->m), g->units, g->ws, sv->s_build);
    if (st == GC_OK) g->units_ready = true;
  }
  dfree(ds);
  dfree(dd);
  if (st != GC_OK) {
    gc_graph_free(g);
    return st;
  }
  G.g = g;
  return GC_OK;
}

static void finish(gc_server *sv, gc_server_req &r, int32_t status, int64_t value) {
  r.status = status;
  r.value = value;
  r.t_done = now_s();
  gc_server_graph &G = sv->graphs[r.graph_id];
  if (r.admitted) G.pins--;
  r.edges = G.g ? G.g->m : 0;
  G.last_use = ++sv->clock;
  ++sv->n_done;
}

// Launch one count batch over the tickets in sv->batch (lock held).
static gc_status launch_batch(gc_server *sv) {
  const int32_t nh = (int32_t)sv->batch.size();
  if ((size_t)nh > sv->h_cap) {
    if (sv->h_desc) (void)hipHostFree(sv->h_desc);
    if (sv->h_pre) (void)hipHostFree(sv->h_pre);
    if (sv->h_out) (void)hipHostFree(sv->h_out);
    sv->h_desc = nullptr;
    sv->h_pre = nullptr;
    sv->h_out = nullptr;
    sv->h_cap = 0;
    const size_t cap = (size_t)nh * 2;
    GC_HIP(hipHostMalloc((void **)&sv->h_desc, sizeof(GraphDesc) * cap));
    GC_HIP(hipHostMalloc((void **)&sv->h_pre, sizeof(int64_t) * kCountBins * (cap + 1)));
    GC_HIP(hipHostMalloc((void **)&sv->h_out, sizeof(unsigned long long) * cap));
    sv->h_cap = cap;
  }
  const size_t npre = (size_t)kCountBins * (nh + 1);
  memset(sv->h_pre, 0, sizeof(int64_t) * npre);
  for (int32_t i = 0; i < nh; ++i) {
    const gc_graph *g = sv->graphs[sv->batch_g[i]].g;
    GraphDesc &d = sv->h_desc[i];
    d.c = g->csr.view(g->n, (int32_t)g->m);
    d.units = static_cast<const int4 *>(g->units.units.ptr);
    for (int b = 0; b < kCountBins; ++b) {
      d.bin_begin[b] = g->units.bin_begin[b];
      sv->h_pre[(size_t)b * (nh + 1) + i + 1] =
          sv->h_pre[(size_t)b * (nh + 1) + i] + (g->m > 0 ? g->units.bin_count[b] : 0);
    }
  }
  GC_TRY(dalloc(sv->d_desc, sizeof(GraphDesc) * (size_t)nh));
  GC_TRY(dalloc(sv->d_pre, sizeof(int64_t) * npre));
  GC_TRY(dalloc(sv->d_out, sizeof(unsigned long long) * (size_t)nh));
  GC_HIP(hipMemcpyAsync(sv->d_desc.ptr, sv->h_desc, sizeof(GraphDesc) * nh, hipMemcpyHostToDevice,
                        sv->s_count));
  GC_HIP(hipMemcpyAsync(sv->d_pre.ptr, sv->h_pre, sizeof(int64_t) * npre, hipMemcpyHostToDevice,
                        sv->s_count));
  GC_TRY(count_multi_launch(static_cast<const GraphDesc *>(sv->d_desc.ptr),
                            static_cast<const int64_t *>(sv->d_pre.ptr), sv->h_pre, nh,
                            static_cast<unsigned long long *>(sv->d_out.ptr), sv->s_count));
  GC_HIP(hipMemcpyAsync(sv->h_out, sv->d_out.ptr, sizeof(unsigned long long) * nh,
                        hipMemcpyDeviceToHost, sv->s_count));
  GC_HIP(hipEventRecord(sv->batch_done, sv->s_count));
  const double t = now_s();
  for (int64_t tk : sv->batch) sv->reqs[tk].t_start = t;
  sv->batch_running = true;
  ++sv->n_batches;
  sv->max_batch = std::max<int64_t>(sv->max_batch, nh);
  return GC_OK;
}

// Admit pending requests in arrival order (lock held; may release it to build).
// Returns how many were admitted or failed.
static int admit(gc_server *sv, std::unique_lock<std::mutex> &lk) {
  int moved = 0;
  size_t scanned = 0;
  while (scanned < sv->pending.size()) {
    const int64_t tk = sv->pending[scanned];
    gc_server_req &r = sv->reqs[tk];
    gc_server_graph &G = sv->graphs[r.graph_id];
    if (G.building) { ++scanned; continue; }
    if (!G.g) {
      const int64_t peak = build_peak_bytes((int64_t)G.src.size(), G.n);
      if (!make_room(sv, peak)) {
        // not enough memory now: running work will release graphs; requests
        // behind this one whose graphs are resident may still go ahead
        ++sv->n_deferred;
        ++scanned;
        if (sv->mode == 1) break;
        continue;
      }
      G.building = true;
      sv->used += peak;
      sv->peak = std::max(sv->peak, sv->used);
      lk.unlock();
      gc_status st = build_graph(sv, G);
      lk.lock();
      G.building = false;
      sv->used -= peak;
      if (st != GC_OK) {
        // the request fails; the server keeps running
        sv->pending.erase(sv->pending.begin() + scanned);
        r.t_start = now_s();
        finish(sv, r, st, 0);
        sv->done_cv.notify_all();
        ++moved;
        continue;
      }
      G.charged = resident_bytes(G.g, (int64_t)G.src.size());
      sv->used += G.charged;
      sv->peak = std::max(sv->peak, sv->used);
      ++sv->n_builds;
      if (sv->used > sv->budget) make_room(sv, 0);
    }
    G.last_use = ++sv->clock;
    r.admitted = true;
    G.pins++;
    sv->pending.erase(sv->pending.begin() + scanned);
    if (r.kind == 0) sv->ready_tc.push_back(tk);
    else { sv->truss_q.push_back(tk); sv->truss_cv.notify_one(); }
    ++moved;
    if (sv->mode == 1) break;  // one at a time
  }
  return moved;
}

static void scheduler_loop(gc_server *sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (!sv->stop) {
    bool progressed = false;
    // complete the running batch (a failed batch fails its requests rather
    // than leaving them pending for ever)
    const hipError_t q = sv->batch_running ? hipEventQuery(sv->batch_done) : hipErrorNotReady;
    if (sv->batch_running && q != hipErrorNotReady) {
      progressed = true;
      if (q != hipSuccess) {
        (void)hipGetLastError();
        sv->error = std::string("count batch: ") + hipGetErrorString(q);
      }
      for (size_t i = 0; i < sv->batch.size(); ++i)
        finish(sv, sv->reqs[sv->batch[i]], q == hipSuccess ? GC_OK : GC_EDEVICE,
               q == hipSuccess ? (int64_t)sv->h_out[i] : 0);
      sv->batch.clear();
      sv->batch_g.clear();
      sv->batch_running = false;
      sv->done_cv.notify_all();
    }
    const bool idle_one = sv->mode == 1 && (sv->batch_running || sv->truss_running ||
                                            !sv->truss_q.empty() || !sv->ready_tc.empty());
    if (!idle_one && admit(sv, lk) > 0) progressed = true;
    if (!sv->batch_running && !sv->ready_tc.empty()) {
      progressed = true;
      const size_t take = sv->mode == 1 ? 1 : sv->ready_tc.size();
      for (size_t i = 0; i < take; ++i) {
        sv->batch.push_back(sv->ready_tc.front());
        sv->batch_g.push_back(sv->reqs[sv->ready_tc.front()].graph_id);
        sv->ready_tc.pop_front();
      }
      if (launch_batch(sv) != GC_OK) {
        for (int64_t tk : sv->batch) finish(sv, sv->reqs[tk], GC_EDEVICE, 0);
        sv->batch.clear();
        sv->batch_g.clear();
        sv->done_cv.notify_all();
      }
    }
    // Always release the lock here: the k-truss worker needs it to complete
    // requests (and so unpin graphs that a deferred build may be waiting for).
    if (sv->batch_running) {
      // poll the running batch while staying responsive to arrivals
      sv->cv.wait_for(lk, std::chrono::microseconds(20));
    } else if (!progressed) {
      sv->cv.wait_for(lk, std::chrono::milliseconds(2));
    }
  }
}

static void truss_loop(gc_server *sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (!sv->stop) {
    if (sv->truss_q.empty()) {
      sv->truss_cv.wait_for(lk, std::chrono::milliseconds(5));
      continue;
    }
    const int64_t tk = sv->truss_q.front();
    sv->truss_q.pop_front();
    gc_server_req &r = sv->reqs[tk];
    gc_graph *g = sv->graphs[r.graph_id].g;
    const int32_t k = r.k;
    r.t_start = now_s();
    ++sv->truss_running;
    lk.unlock();
    DeviceBuffer mask;
    int64_t mk = 0;
    gc_status st = dalloc(mask, (size_t)g->m + 1);
    if (st == GC_OK) st = gc_ktruss(g, k, static_cast<uint8_t *>(mask.ptr), g->m, sv->s_truss, &mk);
    dfree(mask);
    lk.lock();
    --sv->truss_running;
    finish(sv, sv->reqs[tk], st, mk);
    sv->done_cv.notify_all();
    sv->cv.notify_one();
  }
}

}  // namespace gc

using namespace gc;

extern "C" gc_status gc_server_create(int64_t budget_bytes, gc_server **out) {
  clear_error();
  if (!out || budget_bytes <= 0) {
    set_error("gc_server_create: invalid argument");
    return GC_EINVAL;
  }
  *out = nullptr;
  gc_server *sv = new (std::nothrow) gc_server();
  if (!sv) {
    set_error("gc_server_create: host allocation of the handle failed");
    return GC_ENOMEM;
  }
  sv->budget = budget_bytes;
  if (hipGetDevice(&sv->device) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->s_count, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->s_build, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->s_truss, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&sv->batch_done, hipEventDisableTiming) != hipSuccess) {
    set_error("gc_server_create: stream or event creation failed");
    gc_server_destroy(sv);
    return GC_EDEVICE;
  }
  // a thread that cannot start: stop and join the one that did, then free
  const gc_status st = guard_host("gc_server_create", [&]() -> gc_status {
    sv->sched = std::thread(scheduler_loop, sv);
    sv->worker = std::thread(truss_loop, sv);
    return GC_OK;
  });
  if (st != GC_OK) {
    gc_server_destroy(sv);
    return st;
  }
  *out = sv;
  return GC_OK;
}

extern "C" gc_status gc_server_set_mode(gc_server *sv, int32_t mode) {
  clear_error();
  if (!sv || (mode != 0 && mode != 1)) {
    set_error("gc_server_set_mode: invalid argument");
    return GC_EINVAL;
  }
  std::lock_guard<std::mutex> g(sv->mu);
  sv->mode = mode;
  return GC_OK;
}

extern "C" gc_status gc_server_add_graph(gc_server *sv, const int32_t *h_src, const int32_t *h_dst,
                                         int64_t n_pairs, int32_t n_vertices, int32_t *graph_id) {
  clear_error();
  if (!sv || !graph_id || n_pairs < 0 || n_vertices < 0 || (n_pairs > 0 && (!h_src || !h_dst))) {
    set_error("gc_server_add_graph: invalid argument");
    return GC_EINVAL;
  }
  for (int64_t i = 0; i < n_pairs; ++i)
    if (h_src[i] < 0 || h_src[i] >= n_vertices || h_dst[i] < 0 || h_dst[i] >= n_vertices) {
      set_error("gc_server_add_graph: vertex id outside [0, n_vertices)");
      return GC_ERANGE;
    }
  return guard_host("gc_server_add_graph", [&]() -> gc_status {
    gc_server_graph G;
    G.src.assign(h_src, h_src + n_pairs);
    G.dst.assign(h_dst, h_dst + n_pairs);
    G.n = n_vertices;
    std::lock_guard<std::mutex> g(sv->mu);
    if (build_peak_bytes(n_pairs, n_vertices) > sv->budget) {
      set_error("gc_server_add_graph: graph cannot fit in the server's memory budget");
      return GC_ENOMEM;
    }
    *graph_id = (int32_t)sv->graphs.size();
    sv->graphs.push_back(std::move(G));
    return GC_OK;
  });
}

extern "C" gc_status gc_server_submit(gc_server *sv, const gc_request *req, int64_t *ticket) {
  clear_error();
  if (!sv || !req || !ticket || (req->kind != 0 && req->kind != 1) ||
      (req->kind == 1 && req->k < 2)) {
    set_error("gc_server_submit: invalid argument");
    return GC_EINVAL;
  }
  return guard_host("gc_server_submit", [&]() -> gc_status {
    std::lock_guard<std::mutex> g(sv->mu);
    if (req->graph_id < 0 || req->graph_id >= (int32_t)sv->graphs.size()) {
      set_error("gc_server_submit: unknown graph id");
      return GC_EINVAL;
    }
    gc_server_req r;
    r.ticket = sv->next_ticket++;
    r.graph_id = req->graph_id;
    r.kind = req->kind;
    r.k = req->k;
    r.t_submit = now_s();
    auto it = sv->reqs.emplace(r.ticket, r).first;
    try {
      sv->pending.push_back(r.ticket);
    } catch (...) {
      sv->reqs.erase(it);  // not queued: forget it, so no wait() can block on it
      throw;
    }
    *ticket = r.ticket;
    sv->cv.notify_one();
    return GC_OK;
  });
}

static gc_status take_result(gc_server *sv, int64_t ticket, gc_result *out) {
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) {
    set_error("gc_server: unknown or already collected ticket");
    return GC_EINVAL;
  }
  if (it->second.status == GC_PENDING) return GC_PENDING;
  const gc_server_req &r = it->second;
  out->status = r.status;
  out->kind = r.kind;
  out->value = r.value;
  out->edges = r.edges;
  out->t_submit = r.t_submit;
  out->t_start = r.t_start;
  out->t_done = r.t_done;
  sv->reqs.erase(it);
  return GC_OK;
}

extern "C" gc_status gc_server_poll(gc_server *sv, int64_t ticket, gc_result *out) {
  clear_error();
  if (!sv || !out) {
    set_error("gc_server_poll: invalid argument");
    return GC_EINVAL;
  }
  std::lock_guard<std::mutex> g(sv->mu);
  return take_result(sv, ticket, out);
}

extern "C" gc_status gc_server_wait(gc_server *sv, int64_t ticket, gc_result *out) {
  clear_error();
  if (!sv || !out) {
    set_error("gc_server_wait: invalid argument");
    return GC_EINVAL;
  }
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    gc_status st = take_result(sv, ticket, out);
    if (st != GC_PENDING) return st;
    sv->done_cv.wait_for(lk, std::chrono::milliseconds(50));
  }
}

extern "C" gc_status gc_server_stats(gc_server *sv, int64_t *h_stats) {
  clear_error();
  if (!sv || !h_stats) {
    set_error("gc_server_stats: invalid argument");
    return GC_EINVAL;
  }
  std::lock_guard<std::mutex> g(sv->mu);
  int64_t resident = 0;
  for (const auto &G : sv->graphs) resident += G.g ? 1 : 0;
  const int64_t v[10] = {sv->n_done, sv->n_batches, sv->max_batch, sv->n_builds, sv->n_evict,
                         sv->used, sv->peak, sv->n_deferred, resident, sv->budget};
  memcpy(h_stats, v, sizeof(v));
  return GC_OK;
}

extern "C" void gc_server_destroy(gc_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  sv->truss_cv.notify_all();
  if (sv->sched.joinable()) sv->sched.join();
  if (sv->worker.joinable()) sv->worker.join();
  if (sv->s_count) (void)hipStreamSynchronize(sv->s_count);
  for (auto &G : sv->graphs)
    if (G.g) gc_graph_free(G.g);
  dfree(sv->d_desc);
  dfree(sv->d_pre);
  dfree(sv->d_out);
  if (sv->h_out) (void)hipHostFree(sv->h_out);
  if (sv->h_desc) (void)hipHostFree(sv->h_desc);
  if (sv->h_pre) (void)hipHostFree(sv->h_pre);
  if (sv->batch_done) (void)hipEventDestroy(sv->batch_done);
  if (sv->s_count) (void)hipStreamDestroy(sv->s_count);
  if (sv->s_build) (void)hipStreamDestroy(sv->s_build);
  if (sv->s_truss) (void)hipStreamDestroy(sv->s_truss);
  delete sv;
}
