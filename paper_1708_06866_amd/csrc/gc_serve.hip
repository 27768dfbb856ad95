// gc_serve.hip -- a request server with continuous batching.
//
// Clients register graphs (raw pairs kept in host memory) and submit queries:
// a triangle count (Sec. III-A) or the size of a k-truss (Sec. III-B) of a
// registered graph.
//
// Device CSR cache and admission by HBM footprint: a graph is built on first
// use and kept until memory is needed; eviction is least-recently-used among
// graphs no request is using.  A build starts only once the budget holds its
// peak (raw pairs, sort buffers and the CSR it produces); idle graphs are
// evicted for it, and if that is not enough it waits for running work.
//
// Work runs in two lanes, one for small graphs and one for large ones
// (above kLargePairs raw pairs), so that short requests never wait behind
// long ones.  Each lane has
//   * count batches: every triangle-count request of the lane whose graph is
//     resident goes into the lane's next batch, one launch per degree bin over
//     all its graphs (device descriptors, per-graph counters); requests that
//     arrive while a batch runs form the next one as soon as it completes;
//   * a builder thread, which builds the lane's graphs in turn and admits
//     the requests waiting for a graph as soon as it is resident (so it
//     cannot be evicted before its first use);
//   * a k-truss worker: the lane's queued k-truss requests with the oldest
//     one's k become one batch.  Several graphs are peeled as one disjoint
//     union, assembled on the device by concatenating their oriented CSRs
//     (vertex and edge ids shifted per graph), once up to level k; each
//     graph's k-truss size is the count of surviving edges in its slice.  A
//     triangle never spans two graphs, so every graph's k-truss is the one it
//     has alone.  A batch of one graph peels the graph's own handle.  The
//     batch's memory is charged to the budget while it runs.
// A scheduler thread admits requests and runs both lanes' count batches.
// Mode 1 ("per call") serves one request at a time in arrival order with the
// same cache, each k-truss on its graph's own handle, for comparison.
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
  int lane = 0;              // 0 small, 1 large
  gc_graph *g = nullptr;     // resident device CSR, or null
  int64_t charged = 0;       // bytes charged against the budget while resident
  int64_t reserved = 0;      // bytes reserved for a build in progress
  int pins = 0;              // admitted requests that need it resident
  uint64_t last_use = 0;
  bool building = false;     // queued for, or in, a build
};

struct gc_server_req {
  int64_t ticket = 0;
  int32_t graph_id = 0, kind = 0, k = 0;
  int32_t status = GC_PENDING;
  int64_t value = 0;
  int64_t edges = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  bool admitted = false;
  bool deferred = false;  // counted once among the admissions deferred for memory
};

// One lane's queues, streams, threads and batch state.
struct gc_serve_lane {
  std::deque<int64_t> ready_tc;  // admitted triangle counts waiting for a batch
  std::deque<int64_t> truss_q;   // admitted k-truss queries for the worker
  std::deque<int32_t> build_q;   // graphs to build, in order of first request
  std::condition_variable truss_cv, build_cv;
  std::thread worker, builder;
  hipStream_t s_count = nullptr;  // count batches
  hipStream_t s_work = nullptr;   // builds and k-truss batches
  // running count batch
  std::vector<int64_t> batch;    // tickets
  std::vector<int32_t> batch_g;  // graph ids
  hipEvent_t batch_done = nullptr;
  bool batch_running = false;
  gc::DeviceBuffer d_desc, d_pre, d_out;
  // pinned host staging (reused only after the batch that read it completed)
  gc::GraphDesc *h_desc = nullptr;
  int64_t *h_pre = nullptr;
  unsigned long long *h_out = nullptr;
  size_t h_cap = 0;
  gc::DeviceBuffer t_desc, t_cnt;  // k-truss batch descriptors and counters
  int truss_running = 0, n_building = 0;
};

struct gc_server {
  int device = 0;
  int64_t budget = 0;
  int64_t used = 0, peak = 0;
  int32_t mode = 0;  // 0 continuous batching, 1 one request at a time
  std::deque<gc_server_graph> graphs;  // deque: references stay valid as graphs are added
  std::unordered_map<int64_t, gc_server_req> reqs;
  std::deque<int64_t> pending;  // not yet admitted, arrival order
  gc_serve_lane lanes[2];
  int64_t next_ticket = 1;
  uint64_t clock = 0;
  bool stop = false;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::thread sched;
  hipStream_t s_free = nullptr;  // releases evicted graphs (no work runs on it)
  // statistics
  int64_t n_done = 0, n_batches = 0, max_batch = 0, n_builds = 0, n_evict = 0, n_deferred = 0;
  int64_t n_truss_batches = 0, max_truss_batch = 0;
  int64_t truss_waiting = 0;  // bytes a k-truss batch waits for: builds hold back
  std::string error;
};

namespace gc {

// Graphs above this many raw pairs use the large lane (R-MAT scale 18 and
// up at edge factor 16).
constexpr int64_t kLargePairs = int64_t(1) << 22;

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Bytes reserved for building a graph of P pairs and n vertices: the raw
// pairs and the build's sort / scan buffers (about 80 bytes per pair), and
// never less than what the graph is charged once resident (below), since
// m <= P: the handle holds about 57 m + 48 n bytes.
static int64_t build_peak_bytes(int64_t P, int64_t n) {
  return 128 * P + 64 * n + (64 << 20);
}

// Bytes a resident graph is charged: what the allocator holds for its
// handle's arrays, and 1 MiB for the allocator's own rounding beyond that
// (measured on MI355X at 0.8 MiB per resident graph).
static int64_t resident_bytes(const gc_graph *g) {
  return (int64_t)g->device_bytes_held() + (1 << 20);
}

// Bytes a k-truss batch holds while it runs, for a union of m edges and n
// vertices: the concatenated CSR (28 m + 8 n), the support work units
// (16 n + m / 8), the peeling state (26 m, and the compacted CSR copies,
// 40 m at most), the frontier sort buffers (24 m) and the mask (m).
static int64_t union_peak_bytes(int64_t m, int64_t n) {
  return 128 * m + 32 * n + (32 << 20);
}

// Bytes one k-truss on a graph's own handle holds: the peeling state,
// compacted copies, sort buffers and mask, without a CSR copy.
static int64_t handle_truss_bytes(int64_t m, int64_t n) {
  return 96 * m + 16 * n + (32 << 20);
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
    {
      // no work in flight uses an idle graph: release it on the idle stream
      FreeScope fs(sv->s_free);
      gc_graph_free(G.g);
    }
    G.g = nullptr;
    sv->used -= G.charged;
    G.charged = 0;
    ++sv->n_evict;
  }
  return true;
}

// Build graph `G` on stream `s` (called with the lock released).
static gc_status build_graph(gc_server_graph &G, hipStream_t s) {
  const int64_t P = (int64_t)G.src.size();
  DeviceBuffer ds, dd;  // freed below on every path
  gc_status st = dalloc(ds, sizeof(int32_t) * (size_t)(P + 1));
  if (st == GC_OK) st = dalloc(dd, sizeof(int32_t) * (size_t)(P + 1));
  if (st == GC_OK && P > 0) {
    if (hipMemcpyAsync(ds.ptr, G.src.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(dd.ptr, G.dst.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice, s) !=
            hipSuccess)
      st = GC_EDEVICE;
  }
  gc_graph *g = nullptr;
  if (st == GC_OK)
    st = gc_build_csr(static_cast<int32_t *>(ds.ptr), static_cast<int32_t *>(dd.ptr), P, G.n, 0,
                      s, &g);
  if (st == GC_OK && g->m > 0) {
    st = build_units(g->csr.view(g->n, (int32_t)g->m), g->units, g->ws, s);
    if (st == GC_OK) g->units_ready = true;
  }
  if (st == GC_OK && hipStreamSynchronize(s) != hipSuccess) st = GC_EDEVICE;
  dfree(ds);
  dfree(dd);
  if (st != GC_OK) {
    gc_graph_free(g);
    return st;
  }
  G.g = g;
  return GC_OK;
}

// Release what a k-truss on a graph's own handle left on it (compacted CSR
// copies, round state, workspace), so its resident charge stays exact.
static void drop_truss_state(gc_graph *g) {
  g->work[0].release();
  g->work[1].release();
  dfree(g->work_units.units);
  dfree(g->t_sup);
  dfree(g->t_flag);
  dfree(g->t_pos);
  dfree(g->t_misc);
  dfree(g->ws.buf);
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

// Launch the lane's count batch over the tickets in L.batch (lock held).
static gc_status launch_batch(gc_server *sv, gc_serve_lane &L) {
  const int32_t nh = (int32_t)L.batch.size();
  AllocScope as(L.s_count);
  if ((size_t)nh > L.h_cap) {
    if (L.h_desc) (void)hipHostFree(L.h_desc);
    if (L.h_pre) (void)hipHostFree(L.h_pre);
    if (L.h_out) (void)hipHostFree(L.h_out);
    L.h_desc = nullptr;
    L.h_pre = nullptr;
    L.h_out = nullptr;
    L.h_cap = 0;
    const size_t cap = (size_t)nh * 2;
    GC_HIP(hipHostMalloc((void **)&L.h_desc, sizeof(GraphDesc) * cap));
    GC_HIP(hipHostMalloc((void **)&L.h_pre, sizeof(int64_t) * kCountBins * (cap + 1)));
    GC_HIP(hipHostMalloc((void **)&L.h_out, sizeof(unsigned long long) * cap));
    L.h_cap = cap;
  }
  const size_t npre = (size_t)kCountBins * (nh + 1);
  memset(L.h_pre, 0, sizeof(int64_t) * npre);
  for (int32_t i = 0; i < nh; ++i) {
    const gc_graph *g = sv->graphs[L.batch_g[i]].g;
    GraphDesc &d = L.h_desc[i];
    d.c = g->csr.view(g->n, (int32_t)g->m);
    d.units = static_cast<const int4 *>(g->units.units.ptr);
    for (int b = 0; b < kCountBins; ++b) {
      d.bin_begin[b] = g->units.bin_begin[b];
      L.h_pre[(size_t)b * (nh + 1) + i + 1] =
          L.h_pre[(size_t)b * (nh + 1) + i] + (g->m > 0 ? g->units.bin_count[b] : 0);
    }
  }
  GC_TRY(dalloc(L.d_desc, sizeof(GraphDesc) * (size_t)nh));
  GC_TRY(dalloc(L.d_pre, sizeof(int64_t) * npre));
  GC_TRY(dalloc(L.d_out, sizeof(unsigned long long) * (size_t)nh));
  GC_HIP(hipMemcpyAsync(L.d_desc.ptr, L.h_desc, sizeof(GraphDesc) * nh, hipMemcpyHostToDevice,
                        L.s_count));
  GC_HIP(hipMemcpyAsync(L.d_pre.ptr, L.h_pre, sizeof(int64_t) * npre, hipMemcpyHostToDevice,
                        L.s_count));
  GC_TRY(count_multi_launch(static_cast<const GraphDesc *>(L.d_desc.ptr),
                            static_cast<const int64_t *>(L.d_pre.ptr), L.h_pre, nh,
                            static_cast<unsigned long long *>(L.d_out.ptr), L.s_count));
  GC_HIP(hipMemcpyAsync(L.h_out, L.d_out.ptr, sizeof(unsigned long long) * nh,
                        hipMemcpyDeviceToHost, L.s_count));
  GC_HIP(hipEventRecord(L.batch_done, L.s_count));
  const double t = now_s();
  for (int64_t tk : L.batch) sv->reqs[tk].t_start = t;
  L.batch_running = true;
  ++sv->n_batches;
  sv->max_batch = std::max<int64_t>(sv->max_batch, nh);
  return GC_OK;
}

// Admit one pending request whose graph is resident: pin the graph and queue
// the request for its lane's next count batch or k-truss worker (lock held).
static void admit_request(gc_server *sv, int64_t tk) {
  gc_server_req &r = sv->reqs[tk];
  gc_server_graph &G = sv->graphs[r.graph_id];
  gc_serve_lane &L = sv->lanes[G.lane];
  G.last_use = ++sv->clock;
  r.admitted = true;
  G.pins++;
  if (r.kind == 0) L.ready_tc.push_back(tk);
  else { L.truss_q.push_back(tk); L.truss_cv.notify_one(); }
}

// Admit pending requests in arrival order (lock held).  A request whose graph
// is not resident queues the graph for its lane's builder (once) and waits;
// the builder admits it when the graph is built.  Returns how many requests
// moved.
static int admit(gc_server *sv) {
  int moved = 0;
  size_t scanned = 0;
  while (scanned < sv->pending.size()) {
    const int64_t tk = sv->pending[scanned];
    gc_server_req &r = sv->reqs[tk];
    gc_server_graph &G = sv->graphs[r.graph_id];
    if (!G.g) {
      if (!G.building) {
        gc_serve_lane &L = sv->lanes[G.lane];
        G.building = true;
        L.build_q.push_back(r.graph_id);
        ++L.n_building;
        L.build_cv.notify_one();
        ++moved;
      }
      ++scanned;
      if (sv->mode == 1) break;
      continue;
    }
    sv->pending.erase(sv->pending.begin() + scanned);
    admit_request(sv, tk);
    ++moved;
    if (sv->mode == 1) break;  // one at a time
  }
  return moved;
}

// Mode 1: is any request in progress anywhere?
static bool busy(const gc_server *sv) {
  for (const gc_serve_lane &L : sv->lanes)
    if (L.batch_running || L.truss_running || L.n_building > 0 || !L.truss_q.empty() ||
        !L.ready_tc.empty())
      return true;
  return false;
}

static void scheduler_loop(gc_server *sv) {
  (void)hipSetDevice(sv->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  while (!sv->stop) {
    bool progressed = false, running = false;
    for (gc_serve_lane &L : sv->lanes) {
      // complete the lane's running batch (a failed batch fails its requests
      // rather than leaving them pending for ever)
      const hipError_t q = L.batch_running ? hipEventQuery(L.batch_done) : hipErrorNotReady;
      if (L.batch_running && q != hipErrorNotReady) {
        progressed = true;
        if (q != hipSuccess) {
          (void)hipGetLastError();
          sv->error = std::string("count batch: ") + hipGetErrorString(q);
        }
        for (size_t i = 0; i < L.batch.size(); ++i)
          finish(sv, sv->reqs[L.batch[i]], q == hipSuccess ? GC_OK : GC_EDEVICE,
                 q == hipSuccess ? (int64_t)L.h_out[i] : 0);
        L.batch.clear();
        L.batch_g.clear();
        L.batch_running = false;
        sv->done_cv.notify_all();
      }
    }
    if (!(sv->mode == 1 && busy(sv)) && admit(sv) > 0) progressed = true;
    for (gc_serve_lane &L : sv->lanes) {
      if (!L.batch_running && !L.ready_tc.empty()) {
        progressed = true;
        const size_t take = sv->mode == 1 ? 1 : L.ready_tc.size();
        for (size_t i = 0; i < take; ++i) {
          L.batch.push_back(L.ready_tc.front());
          L.batch_g.push_back(sv->reqs[L.ready_tc.front()].graph_id);
          L.ready_tc.pop_front();
        }
        if (launch_batch(sv, L) != GC_OK) {
          for (int64_t tk : L.batch) finish(sv, sv->reqs[tk], GC_EDEVICE, 0);
          L.batch.clear();
          L.batch_g.clear();
          sv->done_cv.notify_all();
        }
      }
      running = running || L.batch_running;
    }
    // Always release the lock here: the builders and the k-truss workers need
    // it to complete their work.
    if (running) {
      // poll the running batches while staying responsive to arrivals
      sv->cv.wait_for(lk, std::chrono::microseconds(20));
    } else if (!progressed) {
      sv->cv.wait_for(lk, std::chrono::milliseconds(2));
    }
  }
}

// A lane's builder: builds the lane's queued graphs one at a time.  A build
// starts once the budget holds its peak (idle graphs are evicted for it; a
// waiting k-truss batch goes first); when it is done, the requests waiting
// for the graph are admitted at once, so the graph cannot be evicted before
// its first use.
static void build_loop(gc_server *sv, int lane) {
  (void)hipSetDevice(sv->device);
  gc_serve_lane &L = sv->lanes[lane];
  std::unique_lock<std::mutex> lk(sv->mu);
  while (!sv->stop) {
    if (L.build_q.empty()) {
      L.build_cv.wait_for(lk, std::chrono::milliseconds(5));
      continue;
    }
    const int32_t id = L.build_q.front();
    gc_server_graph &G = sv->graphs[id];
    const int64_t peak = build_peak_bytes((int64_t)G.src.size(), G.n);
    if (!make_room(sv, peak + sv->truss_waiting)) {
      // running work will release graphs: count the waiting requests once
      for (int64_t tk : sv->pending) {
        gc_server_req &r = sv->reqs[tk];
        if (r.graph_id == id && !r.deferred) {
          r.deferred = true;
          ++sv->n_deferred;
        }
      }
      L.build_cv.wait_for(lk, std::chrono::milliseconds(1));
      continue;
    }
    L.build_q.pop_front();
    G.reserved = peak;
    sv->used += peak;
    sv->peak = std::max(sv->peak, sv->used);
    lk.unlock();
    gc_status st;
    {
      AllocScope as(L.s_work);
      st = build_graph(G, L.s_work);
    }
    lk.lock();
    G.building = false;
    sv->used -= G.reserved;
    G.reserved = 0;
    --L.n_building;
    if (st == GC_OK) {
      G.charged = resident_bytes(G.g);
      sv->used += G.charged;
      sv->peak = std::max(sv->peak, sv->used);
      ++sv->n_builds;
    }
    // the requests waiting for this graph: admitted, or failed with the build
    for (size_t i = 0; i < sv->pending.size();) {
      const int64_t tk = sv->pending[i];
      gc_server_req &r = sv->reqs[tk];
      if (r.graph_id != id) { ++i; continue; }
      sv->pending.erase(sv->pending.begin() + i);
      if (st == GC_OK) {
        admit_request(sv, tk);
        if (sv->mode == 1) break;  // one at a time: the rest wait their turn
      } else {
        r.t_start = now_s();
        finish(sv, r, st, 0);
      }
    }
    if (st != GC_OK) sv->done_cv.notify_all();
    sv->cv.notify_one();
  }
}

// ---- k-truss batches over a device-side union of resident graphs ---------

// Graph i of a union: its oriented CSR and where its vertices (ranks) and
// slots start in the union.
struct CatDesc {
  CsrView c;
  int32_t vbase, ebase;
};

__device__ __forceinline__ int32_t slice_of(const int64_t *__restrict__ off, int32_t n, int64_t x) {
  int32_t lo = 0, hi = n;  // upper bound of x in off[0, n), minus one
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo - 1;
}

// Union row offsets and in-list offsets: vertex x of graph i is x - vbase_i
// there, and its offsets move by ebase_i.
static __global__ void k_cat_rows(const CatDesc *__restrict__ d, const int64_t *__restrict__ voff,
                           int32_t nh, int32_t N, int32_t M, int32_t *__restrict__ row_ptr,
                           int32_t *__restrict__ in_ptr) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= N;
       x += (int64_t)gridDim.x * blockDim.x) {
    if (x == N) {
      row_ptr[N] = M;
      in_ptr[N] = M;
      continue;
    }
    const int32_t i = slice_of(voff, nh + 1, x);
    const int32_t r = (int32_t)(x - d[i].vbase);
    row_ptr[x] = d[i].c.row_ptr[r] + d[i].ebase;
    in_ptr[x] = d[i].c.in_ptr[r] + d[i].ebase;
  }
}

// Union slots: heads and sources move by vbase_i, canonical ids, slot
// positions in the in-list entries and tail ranges by ebase_i.
static __global__ void k_cat_slots(const CatDesc *__restrict__ d, const int64_t *__restrict__ eoff,
                            int32_t nh, int32_t M, int32_t *__restrict__ col,
                            int32_t *__restrict__ src, int32_t *__restrict__ eid,
                            int2 *__restrict__ in_tail, int2 *__restrict__ in_edge) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < M;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = slice_of(eoff, nh + 1, p);
    const CsrView &c = d[i].c;
    const int32_t vb = d[i].vbase, eb = d[i].ebase;
    const int32_t q = (int32_t)(p - eb);
    col[p] = c.col[q] + vb;
    src[p] = c.src[q] + vb;
    eid[p] = c.eid[q] + eb;
    const int2 t = c.in_tail[q];
    in_tail[p] = make_int2(t.x + eb, t.y + eb);
    const int2 e = c.in_edge[q];
    in_edge[p] = make_int2(e.x + vb, e.y + eb);
  }
}

// cnt[i] = edges of graph i's slice [eoff[i], eoff[i+1]) whose mask byte is
// set.  Each wave takes 64 consecutive edges per step: a step inside one
// slice adds its wave sum with one atomic, a step across slices one atomic
// per set edge.
static __global__ void k_slice_counts(const uint8_t *__restrict__ mask, int64_t M,
                               const int64_t *__restrict__ eoff, int32_t nh,
                               unsigned long long *__restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t base = wave * 64; base < M; base += nwaves * 64) {
    const int64_t e = base + lane;
    const int32_t on = (e < M && mask[e]) ? 1 : 0;
    const int64_t last = base + 63 < M ? base + 63 : M - 1;
    const int32_t i0 = slice_of(eoff, nh + 1, base);
    if (last < eoff[i0 + 1]) {
      const int32_t sum = wave_sum_i32(on);
      if (lane == 0 && sum) atomicAdd(&cnt[i0], (unsigned long long)sum);
    } else if (on) {
      atomicAdd(&cnt[slice_of(eoff, nh + 1, e)], 1ull);
    }
  }
}

static __global__ void k_zero_counts(unsigned long long *__restrict__ x, int32_t n) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    x[i] = 0;
}

static unsigned grid256(int64_t work) { return grid_for(work, 256, 65536); }

// k-truss sizes of the graphs `gs` (resident, pinned) by one peeling of their
// union, into mk[i].  Runs with the lock released, on the lane's work stream.
static gc_status union_ktruss(gc_server *sv, gc_serve_lane &L, const std::vector<gc_graph *> &gs,
                              int32_t k, std::vector<int64_t> &mk) {
  const int32_t nh = (int32_t)gs.size();
  hipStream_t s = L.s_work;
  std::vector<CatDesc> desc((size_t)nh);
  std::vector<int64_t> off(2 * ((size_t)nh + 1), 0);  // vertex offsets, then edge offsets
  int64_t *voff = off.data(), *eoff = off.data() + nh + 1;
  for (int32_t i = 0; i < nh; ++i) {
    voff[i + 1] = voff[i] + gs[i]->n;
    eoff[i + 1] = eoff[i] + gs[i]->m;
  }
  const int64_t N = voff[nh], M = eoff[nh];
  mk.assign((size_t)nh, 0);
  if (k <= 2) {  // the 2-truss is the whole graph
    for (int32_t i = 0; i < nh; ++i) mk[i] = gs[i]->m;
    return GC_OK;
  }
  if (M == 0) return GC_OK;
  if (N >= INT32_MAX || M >= INT32_MAX) {
    set_error("k-truss batch: union beyond 2^31 vertices or edges");
    return GC_EOVERFLOW;
  }
  for (int32_t i = 0; i < nh; ++i) {
    desc[i].c = gs[i]->csr.view(gs[i]->n, (int32_t)gs[i]->m);
    desc[i].vbase = (int32_t)voff[i];
    desc[i].ebase = (int32_t)eoff[i];
  }
  gc_graph *ug = new (std::nothrow) gc_graph();
  if (!ug) {
    set_error("k-truss batch: host allocation of the union handle failed");
    return GC_ENOMEM;
  }
  struct Free {
    gc_graph *g;
    ~Free() { gc_graph_free(g); }
  } free_ug{ug};
  ug->device = sv->device;
  ug->n = (int32_t)N;
  ug->m = M;
  ug->bits = ceil_log2_u64((uint64_t)(N > 1 ? N : 2));
  CsrStore &u = ug->csr;
  GC_TRY(dalloc(u.row_ptr, sizeof(int32_t) * (size_t)(N + 1)));
  GC_TRY(dalloc(u.in_ptr, sizeof(int32_t) * (size_t)(N + 1)));
  GC_TRY(dalloc(u.col, sizeof(int32_t) * (size_t)M));
  GC_TRY(dalloc(u.src, sizeof(int32_t) * (size_t)M));
  GC_TRY(dalloc(u.eid, sizeof(int32_t) * (size_t)M));
  GC_TRY(dalloc(u.in_tail, sizeof(int2) * (size_t)M));
  GC_TRY(dalloc(u.in_edge, sizeof(int2) * (size_t)M));
  const size_t dbytes = abytes<CatDesc>((size_t)nh) + abytes<int64_t>(off.size());
  GC_TRY(dalloc(L.t_desc, dbytes));
  CatDesc *d_desc = static_cast<CatDesc *>(L.t_desc.ptr);
  int64_t *d_off = reinterpret_cast<int64_t *>(static_cast<char *>(L.t_desc.ptr) +
                                               abytes<CatDesc>((size_t)nh));
  GC_HIP(hipMemcpyAsync(d_desc, desc.data(), sizeof(CatDesc) * nh, hipMemcpyHostToDevice, s));
  GC_HIP(hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice, s));
  k_cat_rows<<<grid256(N + 1), 256, 0, s>>>(d_desc, d_off, nh, (int32_t)N, (int32_t)M,
                                           static_cast<int32_t *>(u.row_ptr.ptr),
                                           static_cast<int32_t *>(u.in_ptr.ptr));
  GC_LAUNCH_CHECK();
  k_cat_slots<<<grid256(M), 256, 0, s>>>(d_desc, d_off + nh + 1, nh, (int32_t)M,
                                         static_cast<int32_t *>(u.col.ptr),
                                         static_cast<int32_t *>(u.src.ptr),
                                         static_cast<int32_t *>(u.eid.ptr),
                                         static_cast<int2 *>(u.in_tail.ptr),
                                         static_cast<int2 *>(u.in_edge.ptr));
  GC_LAUNCH_CHECK();
  // (synchronises s: the host descriptor arrays are no longer read after it)
  GC_TRY(build_units_support(u.view(ug->n, (int32_t)M), ug->units_sup, ug->ws, s));
  ug->units_sup_ready = true;
  GC_TRY(dalloc(ug->t_misc, (size_t)M + 1));  // the mask, freed with the union
  uint8_t *mask = static_cast<uint8_t *>(ug->t_misc.ptr);
  GC_TRY(decomposition_peel(ug, nullptr, nullptr, s, k, mask, nullptr));
  GC_TRY(dalloc(L.t_cnt, sizeof(unsigned long long) * (size_t)nh));
  unsigned long long *cnt = static_cast<unsigned long long *>(L.t_cnt.ptr);
  k_zero_counts<<<grid256(nh), 256, 0, s>>>(cnt, nh);
  GC_LAUNCH_CHECK();
  k_slice_counts<<<grid256(M), 256, 0, s>>>(mask, M, d_off + nh + 1, nh, cnt);
  GC_LAUNCH_CHECK();
  std::vector<unsigned long long> h((size_t)nh);
  GC_HIP(hipMemcpyAsync(h.data(), cnt, sizeof(unsigned long long) * nh, hipMemcpyDeviceToHost, s));
  GC_HIP(hipStreamSynchronize(s));
  for (int32_t i = 0; i < nh; ++i) mk[i] = (int64_t)h[i];
  return GC_OK;
}

// One k-truss on the graph's own handle, its working state dropped
// afterwards.  Runs with the lock released.
static gc_status handle_ktruss(gc_graph *g, int32_t k, hipStream_t s, int64_t *mk) {
  DeviceBuffer mask;
  gc_status st = dalloc(mask, (size_t)g->m + 1);
  if (st == GC_OK) st = gc_ktruss(g, k, static_cast<uint8_t *>(mask.ptr), g->m, s, mk);
  dfree(mask);
  drop_truss_state(g);
  return st;
}

// Largest union of a k-truss batch, in edges: more requests wait for the
// next batch, which bounds both the union's memory and how long the requests
// behind a batch wait.  A single graph above it forms a batch of its own.
constexpr int64_t kTrussBatchEdges = int64_t(1) << 25;

// A lane's k-truss worker: the lane's queued k-truss requests with the
// oldest one's k, in arrival order up to kTrussBatchEdges of distinct
// graphs, become one batch (mode 0), or one request at a time (mode 1).  A
// batch of one graph peels the graph's own handle; a batch of several peels
// their union.  A batch runs once the budget holds it; if it cannot, it is
// halved, and a single graph that does not fit waits (new builds hold back
// meanwhile).
static void truss_loop(gc_server *sv, int lane) {
  (void)hipSetDevice(sv->device);
  gc_serve_lane &L = sv->lanes[lane];
  std::unique_lock<std::mutex> lk(sv->mu);
  while (!sv->stop) {
    if (L.truss_q.empty()) {
      L.truss_cv.wait_for(lk, std::chrono::milliseconds(5));
      continue;
    }
    std::vector<int64_t> tks;
    std::vector<int32_t> gids, slot;  // distinct graphs; slot of each ticket's graph
    int64_t need = 0;
    size_t take = 0;
    const int32_t k = sv->reqs[L.truss_q.front()].k;
    const gc_status hs = guard_host("k-truss batch", [&]() -> gc_status {
      int64_t m = 0;
      for (int64_t tk : L.truss_q) {
        const gc_server_req &r = sv->reqs[tk];
        if (r.k != k) continue;
        const bool known = std::find(gids.begin(), gids.end(), r.graph_id) != gids.end();
        if (!known) {
          const int64_t mg = sv->graphs[r.graph_id].g->m;
          if (!gids.empty() && m + mg > kTrussBatchEdges) break;
          gids.push_back(r.graph_id);
          m += mg;
        }
        tks.push_back(tk);
        if (sv->mode == 1) break;
      }
      take = tks.size();
      for (;;) {
        gids.clear();
        slot.clear();
        int64_t mm = 0, n = 0;
        for (size_t j = 0; j < take; ++j) {
          const int32_t id = sv->reqs[tks[j]].graph_id;
          const auto it = std::find(gids.begin(), gids.end(), id);
          slot.push_back((int32_t)(it - gids.begin()));
          if (it == gids.end()) {
            gids.push_back(id);
            mm += sv->graphs[id].g->m;
            n += sv->graphs[id].g->n;
          }
        }
        need = gids.size() == 1 ? handle_truss_bytes(mm, n) : union_peak_bytes(mm, n);
        if (make_room(sv, need) || gids.size() == 1) return GC_OK;
        take = (take + 1) / 2;
      }
    });
    if (hs != GC_OK) {  // host memory exhausted: retry later
      L.truss_cv.wait_for(lk, std::chrono::milliseconds(2));
      continue;
    }
    if (sv->used + need > sv->budget) {  // even one graph does not fit yet
      sv->truss_waiting = std::max(sv->truss_waiting, need);
      L.truss_cv.wait_for(lk, std::chrono::milliseconds(2));
      continue;
    }
    sv->truss_waiting = 0;
    tks.resize(take);
    for (int64_t tk : tks) L.truss_q.erase(std::find(L.truss_q.begin(), L.truss_q.end(), tk));
    sv->used += need;
    sv->peak = std::max(sv->peak, sv->used);
    const double t = now_s();
    for (int64_t tk : tks) sv->reqs[tk].t_start = t;
    ++L.truss_running;
    ++sv->n_truss_batches;
    sv->max_truss_batch = std::max<int64_t>(sv->max_truss_batch, (int64_t)tks.size());
    std::vector<gc_graph *> gs;
    std::vector<int64_t> mk;
    gc_status st = guard_host("k-truss batch", [&]() -> gc_status {
      for (int32_t id : gids) gs.push_back(sv->graphs[id].g);
      return GC_OK;
    });
    lk.unlock();
    if (st == GC_OK) {
      AllocScope as(L.s_work);
      if (gs.size() == 1) {
        mk.assign(1, 0);
        st = handle_ktruss(gs[0], k, L.s_work, &mk[0]);
      } else {
        st = guard_host("k-truss batch",
                        [&]() -> gc_status { return union_ktruss(sv, L, gs, k, mk); });
      }
    }
    lk.lock();
    sv->used -= need;
    --L.truss_running;
    for (size_t j = 0; j < tks.size(); ++j)
      finish(sv, sv->reqs[tks[j]], st, st == GC_OK ? mk[slot[j]] : 0);
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
  bool ok = hipGetDevice(&sv->device) == hipSuccess &&
            hipStreamCreateWithFlags(&sv->s_free, hipStreamNonBlocking) == hipSuccess;
  for (gc_serve_lane &L : sv->lanes)
    ok = ok && hipStreamCreateWithFlags(&L.s_count, hipStreamNonBlocking) == hipSuccess &&
         hipStreamCreateWithFlags(&L.s_work, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&L.batch_done, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    set_error("gc_server_create: stream or event creation failed");
    gc_server_destroy(sv);
    return GC_EDEVICE;
  }
  // a thread that cannot start: stop and join the ones that did, then free
  const gc_status st = guard_host("gc_server_create", [&]() -> gc_status {
    sv->sched = std::thread(scheduler_loop, sv);
    for (int i = 0; i < 2; ++i) {
      sv->lanes[i].worker = std::thread(truss_loop, sv, i);
      sv->lanes[i].builder = std::thread(build_loop, sv, i);
    }
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
    G.lane = n_pairs > kLargePairs ? 1 : 0;
    std::lock_guard<std::mutex> g(sv->mu);
    // its build, and a k-truss batch of it alone beside it once resident
    if (build_peak_bytes(n_pairs, n_vertices) + union_peak_bytes(n_pairs, n_vertices) >
        sv->budget) {
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
  const int64_t v[12] = {sv->n_done,    sv->n_batches, sv->max_batch, sv->n_builds,
                         sv->n_evict,   sv->used,      sv->peak,      sv->n_deferred,
                         resident,      sv->budget,    sv->n_truss_batches,
                         sv->max_truss_batch};
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
  for (gc_serve_lane &L : sv->lanes) {
    L.truss_cv.notify_all();
    L.build_cv.notify_all();
  }
  if (sv->sched.joinable()) sv->sched.join();
  for (gc_serve_lane &L : sv->lanes) {
    if (L.worker.joinable()) L.worker.join();
    if (L.builder.joinable()) L.builder.join();
    if (L.s_count) (void)hipStreamSynchronize(L.s_count);
  }
  for (auto &G : sv->graphs)
    if (G.g) gc_graph_free(G.g);  // stream-ordered: released on the lanes' streams
  for (gc_serve_lane &L : sv->lanes) {
    dfree(L.d_desc);
    dfree(L.d_pre);
    dfree(L.d_out);
    dfree(L.t_desc);
    dfree(L.t_cnt);
    if (L.h_out) (void)hipHostFree(L.h_out);
    if (L.h_desc) (void)hipHostFree(L.h_desc);
    if (L.h_pre) (void)hipHostFree(L.h_pre);
    if (L.batch_done) (void)hipEventDestroy(L.batch_done);
  }
  // the frees above are queued on these streams: let them run, then destroy
  for (gc_serve_lane &L : sv->lanes)
    for (hipStream_t st : {L.s_count, L.s_work})
      if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
      }
  if (sv->s_free) {
    (void)hipStreamSynchronize(sv->s_free);
    (void)hipStreamDestroy(sv->s_free);
  }
  delete sv;
}
