// gc_batch.hip -- many independent graphs in one device CSR and one launch
// per degree bin.
//
// The G graphs are shifted into disjoint vertex ranges [base_g, base_g + n_g)
// and built as one graph (their disjoint union).  A triangle never spans two
// graphs, so the union's triangles, supports and k-trusses are exactly the
// per-graph ones; canonical edges of graph g form the contiguous slice
// [edge_off[g], edge_off[g+1]) of the union's canonical order, each slice in
// that graph's own canonical order (shifted by base_g).  Work units of all
// graphs share the per-bin queues, so the counting kernels run once per bin
// for the whole batch and add each unit's hits to the counter of its graph.
//
// Autotuning: for every bin that has work, every admissible strategy (LDS
// hash at two load factors, binary search in HBM) is timed on the batch with
// HIP events and the fastest is kept; choices can be saved to and loaded from
// a text cache keyed by (device architecture, bin).  The count sequence is
// captured once into a HIP graph and replayed.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "gc_graph.h"

struct gc_batch {
  int device = 0;
  int32_t G = 0;
  int64_t pairs = 0;
  gc_graph *g = nullptr;
  gc::DeviceBuffer vbase;          // int32 [G+1] vertex base per graph
  gc::DeviceBuffer graph_of_rank;  // int32 [n]
  gc::DeviceBuffer tbuf;           // u64 [G] per-graph triangle counters
  std::vector<int64_t> edge_off;   // host [G+1]
  int strategy[gc::kCountBins] = {0, 0, 0, 0, 2};
  float tuned_ms[gc::kCountBins][gc::kCountStrategies] = {};
  bool captured = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t own_stream = nullptr;  // capture stream when the caller passes the null stream
  // the k-truss of every graph as a second recorded launch sequence
  gc::PeelReplay kt;
  gc::DeviceBuffer kt_mask, kt_cnt;  // its mask (uint8 [m]) and per-graph sizes (u64 [G])
  int32_t kt_k = 0;                  // k it was recorded for
  int32_t kt_rounds = 32;            // rounds recorded per level
  hipGraph_t kt_graph = nullptr;
  hipGraphExec_t kt_exec = nullptr;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    captured = false;
  }
  void drop_kt_graph() {
    if (kt_exec) (void)hipGraphExecDestroy(kt_exec);
    if (kt_graph) (void)hipGraphDestroy(kt_graph);
    kt_exec = nullptr;
    kt_graph = nullptr;
    kt_k = 0;
  }
};

namespace gc {

__device__ __forceinline__ int32_t upper_bound_i64(const int64_t *a, int32_t n, int64_t x) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int32_t upper_bound_i32(const int32_t *a, int32_t n, int32_t x) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Shift graph-local ids into the union's id space; out-of-range ids raise err.
__global__ void k_shift_pairs(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                              int64_t P, const int64_t *__restrict__ pair_off, int32_t G,
                              const int32_t *__restrict__ vbase, int32_t one,
                              int32_t *__restrict__ os, int32_t *__restrict__ od,
                              int32_t *__restrict__ err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = upper_bound_i64(pair_off, G + 1, i) - 1;
    const int32_t nv = vbase[g + 1] - vbase[g];
    const int32_t a = src[i] - one, b = dst[i] - one;
    if (a < 0 || a >= nv || b < 0 || b >= nv) {
      atomicOr(err, 1);
      os[i] = vbase[g];
      od[i] = vbase[g];  // a self-loop: dropped
    } else {
      os[i] = vbase[g] + a;
      od[i] = vbase[g] + b;
    }
  }
}

__global__ void k_graph_of_rank(const int32_t *__restrict__ vid, int32_t n,
                                const int32_t *__restrict__ vbase, int32_t G,
                                int32_t *__restrict__ out) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x)
    out[r] = upper_bound_i32(vbase, G + 1, vid[r]) - 1;
}

// edge_off[g] = first canonical edge whose u >= vbase[g].
__global__ void k_edge_offsets(const int32_t *__restrict__ u, int64_t m,
                               const int32_t *__restrict__ vbase, int32_t G,
                               int64_t *__restrict__ off) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= G;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = vbase[g];
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (u[mid] < x) lo = mid + 1; else hi = mid;
    }
    off[g] = lo;
  }
}

__global__ void k_zero_u64(unsigned long long *__restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0;
}

__global__ void k_copy_u64(const unsigned long long *__restrict__ a, int64_t n,
                           int64_t *__restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (int64_t)a[i];
}

// cnt[g] += the marked edges of graph g.  Batch edges are in graph order, so
// the marked edges of a wave mostly belong to one graph: each run of equal
// graphs along the wave takes one atomic (one per marked edge serialised on
// the few counters of a batch's graphs: 160 ms for the 6e8 edges of the
// 4,096-graph batch).  Every lane of a wave runs the same iterations.
__global__ void k_mask_counts(const uint8_t *__restrict__ mask, const int32_t *__restrict__ u,
                              int64_t m, const int32_t *__restrict__ vbase, int32_t G,
                              unsigned long long *__restrict__ cnt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t span = (m + stride - 1) / stride * stride;
  const int lane = (int)__lane_id();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < span; e += stride) {
    const bool marked = e < m && mask[e] != 0;
    const int32_t gi = marked ? upper_bound_i32(vbase, G + 1, u[e]) - 1 : -1;
    const int32_t prev = __shfl_up(gi, 1, 64);
    const bool head = lane == 0 || gi != prev;
    const uint64_t bounds = __ballot(head);
    if (marked && head) {
      const uint64_t after = lane == 63 ? 0ull : (bounds >> (lane + 1));
      const int len = after ? __ffsll((long long)after) : 64 - lane;
      atomicAdd(&cnt[gi], (unsigned long long)len);
    }
  }
}

static unsigned gsz(int64_t work) { return grid_for(work, 256, 65536); }

static gc_status batch_units(gc_batch *b, hipStream_t s) {
  gc_graph *g = b->g;
  if (!g->units_ready && g->m > 0) {
    GC_TRY(build_units(g->csr.view(g->n, (int32_t)g->m), g->units, g->ws, s));
    g->units_ready = true;
  }
  return GC_OK;
}

static gc_status batch_count_launches(gc_batch *b, hipStream_t s) {
  gc_graph *g = b->g;
  k_zero_u64<<<gsz(b->G), 256, 0, s>>>(static_cast<unsigned long long *>(b->tbuf.ptr), b->G);
  GC_LAUNCH_CHECK();
  if (g->m == 0) return GC_OK;
  return count_triangles_ex(g->csr.view(g->n, (int32_t)g->m), g->units, nullptr,
                            static_cast<unsigned long long *>(b->tbuf.ptr),
                            static_cast<const int32_t *>(b->graph_of_rank.ptr), b->strategy, s);
}

}  // namespace gc

using namespace gc;

extern "C" gc_status gc_batch_build(const int32_t *d_src, const int32_t *d_dst,
                                    const int64_t *h_pair_off, const int32_t *h_nv, int32_t G,
                                    uint32_t flags, gc_stream stream, gc_batch **out) {
  clear_error();
  if (!out) {
    set_error("gc_batch_build: out is NULL");
    return GC_EINVAL;
  }
  *out = nullptr;
  if (G < 0 || (G > 0 && (!h_pair_off || !h_nv)) || (flags & ~GC_INPUT_ONE_BASED) != 0) {
    set_error("gc_batch_build: invalid argument");
    return GC_EINVAL;
  }
  std::vector<int32_t> vbase;
  GC_TRY(guard_host("gc_batch_build", [&]() -> gc_status {
    vbase.assign((size_t)G + 1, 0);
    return GC_OK;
  }));
  int64_t nsum = 0;
  for (int32_t i = 0; i < G; ++i) {
    if (h_nv[i] < 0 || h_pair_off[i + 1] < h_pair_off[i] || (i == 0 && h_pair_off[0] != 0)) {
      set_error("gc_batch_build: bad pair offsets or vertex counts");
      return GC_EINVAL;
    }
    nsum += h_nv[i];
    if (nsum >= INT32_MAX) {
      set_error("gc_batch_build: total vertex count must be < 2^31");
      return GC_EOVERFLOW;
    }
    vbase[i + 1] = (int32_t)nsum;
  }
  const int64_t P = G > 0 ? h_pair_off[G] : 0;
  if (P > 0 && (!d_src || !d_dst)) {
    set_error("gc_batch_build: NULL pair arrays");
    return GC_EINVAL;
  }
  if (P >= (int64_t)INT32_MAX - 8) {
    set_error("gc_batch_build: total pairs must be < 2^31");
    return GC_EOVERFLOW;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  gc_batch *b = new (std::nothrow) gc_batch();
  if (!b) {
    set_error("gc_batch_build: host allocation of the handle failed");
    return GC_ENOMEM;
  }
  b->G = G;
  b->pairs = P;
  auto fail = [&](gc_status st) {
    gc_batch_free(b);
    return st;
  };
  if (hipGetDevice(&b->device) != hipSuccess) {
    set_error("gc_batch_build: hipGetDevice failed");
    return fail(GC_EDEVICE);
  }
  const gc_status hs = guard_host("gc_batch_build", [&]() -> gc_status {
    b->edge_off.assign((size_t)G + 1, 0);
    return GC_OK;
  });
  if (hs != GC_OK) return fail(hs);
  DeviceBuffer d_off, d_shift, d_err;
  struct Cleanup {
    DeviceBuffer *a, *b, *c;
    ~Cleanup() { dfree(*a); dfree(*b); dfree(*c); }
  } cleanup{&d_off, &d_shift, &d_err};
  gc_status st;
  if ((st = dalloc(b->vbase, sizeof(int32_t) * ((size_t)G + 1))) != GC_OK) return fail(st);
  if ((st = dalloc(b->tbuf, sizeof(unsigned long long) * ((size_t)G + 1))) != GC_OK) return fail(st);
  if ((st = dalloc(d_off, sizeof(int64_t) * ((size_t)G + 1))) != GC_OK) return fail(st);
  if ((st = dalloc(d_shift, sizeof(int32_t) * 2 * ((size_t)P + 1))) != GC_OK) return fail(st);
  if ((st = dalloc(d_err, 256)) != GC_OK) return fail(st);
  if (hipMemcpyAsync(b->vbase.ptr, vbase.data(), sizeof(int32_t) * (G + 1), hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      (G > 0 && hipMemcpyAsync(d_off.ptr, h_pair_off, sizeof(int64_t) * (G + 1),
                               hipMemcpyHostToDevice, s) != hipSuccess) ||
      hipMemsetAsync(d_err.ptr, 0, sizeof(int32_t), s) != hipSuccess) {
    set_error("gc_batch_build: copy of batch descriptors failed");
    return fail(GC_EDEVICE);
  }
  int32_t *s2 = static_cast<int32_t *>(d_shift.ptr);
  int32_t *d2 = s2 + P + 1;
  if (P > 0) {
    k_shift_pairs<<<gsz(P), 256, 0, s>>>(d_src, d_dst, P, static_cast<const int64_t *>(d_off.ptr),
                                         G, static_cast<const int32_t *>(b->vbase.ptr),
                                         (flags & GC_INPUT_ONE_BASED) ? 1 : 0, s2, d2,
                                         static_cast<int32_t *>(d_err.ptr));
    if (hipGetLastError() != hipSuccess) return fail(GC_EDEVICE);
  }
  int32_t herr = 0;
  if (hipMemcpyAsync(&herr, d_err.ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(GC_EDEVICE);
  if (herr) {
    set_error("gc_batch_build: a vertex id is outside its graph's range");
    return fail(GC_ERANGE);
  }
  if ((st = gc_build_csr(s2, d2, P, (int32_t)nsum, 0, stream, &b->g)) != GC_OK) return fail(st);
  gc_graph *g = b->g;
  if ((st = dalloc(b->graph_of_rank, sizeof(int32_t) * ((size_t)g->n + 1))) != GC_OK) return fail(st);
  if (g->n > 0) {
    k_graph_of_rank<<<gsz(g->n), 256, 0, s>>>(static_cast<const int32_t *>(g->vid.ptr), g->n,
                                              static_cast<const int32_t *>(b->vbase.ptr), G,
                                              static_cast<int32_t *>(b->graph_of_rank.ptr));
  }
  k_edge_offsets<<<gsz((int64_t)G + 1), 256, 0, s>>>(static_cast<const int32_t *>(g->u.ptr), g->m,
                                                     static_cast<const int32_t *>(b->vbase.ptr), G,
                                                     static_cast<int64_t *>(d_off.ptr));
  if (hipMemcpyAsync(b->edge_off.data(), d_off.ptr, sizeof(int64_t) * (G + 1),
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(GC_EDEVICE);
  load_strategy_cache(b->device, b->strategy, nullptr);
  // rounds recorded per level of the replayed k-truss (GC_BATCH_KTRUSS_ROUNDS)
  if (const char *ev = getenv("GC_BATCH_KTRUSS_ROUNDS")) {
    const long r = strtol(ev, nullptr, 10);
    if (r >= 1 && r <= 4096) b->kt_rounds = (int32_t)r;
  }
  *out = b;
  return GC_OK;
}

extern "C" gc_status gc_batch_info(const gc_batch *b, int32_t *n_graphs, int64_t *n_edges,
                                   int64_t *device_bytes) {
  clear_error();
  if (!b) {
    set_error("gc_batch_info: NULL batch");
    return GC_EINVAL;
  }
  if (n_graphs) *n_graphs = b->G;
  if (n_edges) *n_edges = b->g ? b->g->m : 0;
  if (device_bytes)
    *device_bytes = (int64_t)((b->g ? b->g->device_bytes() : 0) + b->vbase.bytes +
                              b->graph_of_rank.bytes + b->tbuf.bytes);
  return GC_OK;
}

extern "C" gc_status gc_batch_edge_offsets(const gc_batch *b, int64_t *h_off) {
  clear_error();
  if (!b || !h_off) {
    set_error("gc_batch_edge_offsets: invalid argument");
    return GC_EINVAL;
  }
  memcpy(h_off, b->edge_off.data(), sizeof(int64_t) * ((size_t)b->G + 1));
  return GC_OK;
}

extern "C" gc_graph *gc_batch_graph(gc_batch *b) { return b ? b->g : nullptr; }

extern "C" gc_status gc_batch_autotune(gc_batch *b, gc_stream stream, int32_t *h_strategy,
                                       float *h_ms) {
  clear_error();
  if (!b) {
    set_error("gc_batch_autotune: NULL batch");
    return GC_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  GC_TRY(batch_units(b, s));
  gc_graph *g = b->g;
  b->drop_graph();
  if (g->m > 0) {
    GC_TRY(autotune_bins(g->csr.view(g->n, (int32_t)g->m), g->units, b->strategy, &b->tuned_ms[0][0],
                         nullptr, static_cast<unsigned long long *>(b->tbuf.ptr),
                         static_cast<const int32_t *>(b->graph_of_rank.ptr), s));
  }
  save_strategy_cache(b->device, b->strategy, nullptr);
  if (h_strategy)
    for (int bin = 0; bin < kCountBins; ++bin) h_strategy[bin] = b->strategy[bin];
  if (h_ms)
    for (int bin = 0; bin < kCountBins; ++bin)
      for (int st = 0; st < kCountStrategies; ++st)
        h_ms[bin * kCountStrategies + st] = b->tuned_ms[bin][st];
  return GC_OK;
}

extern "C" gc_status gc_batch_set_strategy(gc_batch *b, const int32_t *h_strategy) {
  clear_error();
  if (!b || !h_strategy) {
    set_error("gc_batch_set_strategy: invalid argument");
    return GC_EINVAL;
  }
  for (int bin = 0; bin < kCountBins; ++bin)
    if (!count_strategy_valid(bin, h_strategy[bin])) {
      set_error("gc_batch_set_strategy: strategy not admissible for its bin");
      return GC_EINVAL;
    }
  for (int bin = 0; bin < kCountBins; ++bin) b->strategy[bin] = h_strategy[bin];
  b->drop_graph();
  return GC_OK;
}

extern "C" gc_status gc_batch_triangle_count(gc_batch *b, int64_t *d_T, gc_stream stream) {
  clear_error();
  if (!b || (b->G > 0 && !d_T)) {
    set_error("gc_batch_triangle_count: invalid argument");
    return GC_EINVAL;
  }
  if (b->G == 0) return GC_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  GC_TRY(batch_units(b, s));
  // The null stream cannot be captured: use a blocking stream of our own,
  // which the null stream orders against implicitly.
  hipStream_t cs = s;
  if (!cs) {
    if (!b->own_stream) GC_HIP(hipStreamCreate(&b->own_stream));
    cs = b->own_stream;
  }
  if (!b->captured) {
    // capture the zeroing + per-bin count launches once, replay afterwards
    GC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    gc_status st = batch_count_launches(b, cs);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (st != GC_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    GC_HIP(e);
    b->graph = graph;
    GC_HIP(hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0));
    b->captured = true;
  }
  GC_HIP(hipGraphLaunch(b->exec, cs));
  k_copy_u64<<<gsz(b->G), 256, 0, s>>>(static_cast<const unsigned long long *>(b->tbuf.ptr), b->G,
                                       d_T);
  GC_LAUNCH_CHECK();
  return GC_OK;
}

extern "C" gc_status gc_batch_edge_support(gc_batch *b, int32_t *d_support, int64_t cap,
                                           gc_stream stream) {
  clear_error();
  if (!b) {
    set_error("gc_batch_edge_support: NULL batch");
    return GC_EINVAL;
  }
  return gc_edge_support(b->g, d_support, cap, stream);
}

namespace gc {

// The k-truss of every graph of the batch from the recorded launch sequence
// (recorded on the first call for this k): levels 3 .. k of the peeling, a
// fixed number of rounds each, then the union's mask and each graph's count.
// Returns GC_OK with *converged false when a level needed more rounds than
// were recorded (the caller then peels eagerly, and the next call records
// twice the rounds).
static gc_status batch_ktruss_replay(gc_batch *b, int32_t k, hipStream_t s, hipStream_t cs,
                                     bool *converged) {
  gc_graph *g = b->g;
  *converged = false;
  if (!b->kt_exec || b->kt_k != k) {
    b->drop_kt_graph();
    GC_TRY(b->kt.prepare((int32_t)g->m));
    GC_TRY(dalloc(b->kt_mask, (size_t)g->m + 1));
    GC_TRY(dalloc(b->kt_cnt, sizeof(unsigned long long) * ((size_t)b->G + 1)));
    GC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    unsigned long long *cnt = static_cast<unsigned long long *>(b->kt_cnt.ptr);
    uint8_t *mask = static_cast<uint8_t *>(b->kt_mask.ptr);
    gc_status st = ktruss_launches(g, k, b->kt_rounds, b->kt, mask, cs);
    if (st == GC_OK) {
      k_zero_u64<<<gsz(b->G), 256, 0, cs>>>(cnt, b->G);
      k_mask_counts<<<gsz(g->m), 256, 0, cs>>>(mask, static_cast<const int32_t *>(g->u.ptr), g->m,
                                              static_cast<const int32_t *>(b->vbase.ptr), b->G,
                                              cnt);
      if (hipGetLastError() != hipSuccess) st = GC_EDEVICE;
    }
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (st != GC_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    GC_HIP(e);
    b->kt_graph = graph;
    GC_HIP(hipGraphInstantiate(&b->kt_exec, graph, nullptr, nullptr, 0));
    b->kt_k = k;
  }
  GC_HIP(hipGraphLaunch(b->kt_exec, cs));
  int32_t left[64];
  GC_HIP(hipMemcpyAsync(left, b->kt.leftover(), sizeof(int32_t) * (k - 2), hipMemcpyDeviceToHost,
                        cs));
  GC_HIP(hipStreamSynchronize(cs));
  (void)s;
  bool all = true;
  for (int32_t i = 0; i < k - 2; ++i) all = all && left[i] == 0;
  *converged = all;
  return GC_OK;
}

}  // namespace gc

extern "C" gc_status gc_batch_ktruss(gc_batch *b, int32_t k, uint8_t *d_mask, int64_t cap,
                                     int64_t *d_mk, gc_stream stream) {
  clear_error();
  if (!b || (b->G > 0 && !d_mk) || k < 2 || (b->g && b->g->m > 0 && !d_mask)) {
    set_error("gc_batch_ktruss: invalid argument");
    return GC_EINVAL;
  }
  if (b->g && cap < b->g->m) {
    set_error("gc_batch_ktruss: cap < m");
    return GC_ECAPACITY;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (b->G > 0 && b->g->m > 0 && k > 2 && k - 2 <= 64 && b->kt_rounds > 0) {
    // the recorded sequence, on the caller's stream (or an own blocking one
    // for the null stream, which cannot be captured)
    hipStream_t cs = s;
    if (!cs) {
      if (!b->own_stream) GC_HIP(hipStreamCreate(&b->own_stream));
      cs = b->own_stream;
    }
    bool converged = false;
    GC_TRY(batch_ktruss_replay(b, k, s, cs, &converged));
    if (converged) {
      GC_HIP(hipMemcpyAsync(d_mask, b->kt_mask.ptr, (size_t)b->g->m, hipMemcpyDeviceToDevice, s));
      k_copy_u64<<<gsz(b->G), 256, 0, s>>>(static_cast<const unsigned long long *>(b->kt_cnt.ptr),
                                           b->G, d_mk);
      GC_LAUNCH_CHECK();
      GC_HIP(hipStreamSynchronize(s));
      return GC_OK;
    }
    // a level needed more rounds than were recorded: peel eagerly now, and
    // record twice the rounds on the next call (up to 1024 rounds per level;
    // beyond that the sequence would hold too many launches, and this batch
    // keeps peeling eagerly)
    b->kt_rounds = b->kt_rounds < 1024 ? b->kt_rounds * 2 : 0;
    b->drop_kt_graph();
  }
  GC_TRY(gc_ktruss(b->g, k, d_mask, cap, stream, nullptr));
  if (b->G == 0) return GC_OK;
  unsigned long long *cnt = static_cast<unsigned long long *>(b->tbuf.ptr);
  k_zero_u64<<<gsz(b->G), 256, 0, s>>>(cnt, b->G);
  GC_LAUNCH_CHECK();
  if (b->g->m > 0) {
    k_mask_counts<<<gsz(b->g->m), 256, 0, s>>>(d_mask, static_cast<const int32_t *>(b->g->u.ptr),
                                               b->g->m, static_cast<const int32_t *>(b->vbase.ptr),
                                               b->G, cnt);
    GC_LAUNCH_CHECK();
  }
  k_copy_u64<<<gsz(b->G), 256, 0, s>>>(cnt, b->G, d_mk);
  GC_LAUNCH_CHECK();
  return GC_OK;
}

extern "C" void gc_batch_free(gc_batch *b) {
  if (!b) return;
  b->drop_graph();
  b->drop_kt_graph();
  b->kt.release();
  dfree(b->kt_mask);
  dfree(b->kt_cnt);
  if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
  if (b->g) gc_graph_free(b->g);
  dfree(b->vbase);
  dfree(b->graph_of_rank);
  dfree(b->tbuf);
  delete b;
}
