// gc_api.hip -- handle accessors, status text, device memory helpers and the
// counting entry points gc_triangle_count / gc_edge_support /
// gc_edge_support_noalloc.
#include <mutex>
#include <new>

#include "gc_graph.h"

namespace gc {

static thread_local std::string t_last_error;

void set_error(const std::string &msg) { t_last_error = msg; }
void clear_error() { t_last_error.clear(); }

void note_host_failure(const char *where, const char *what) noexcept {
  try {
    t_last_error = std::string(where) + ": host allocation or thread start failed: " + what;
  } catch (...) {
    t_last_error.clear();
  }
}

static thread_local hipStream_t t_alloc_stream = nullptr;  // AllocScope
static thread_local hipStream_t t_free_stream = nullptr;   // FreeScope

AllocScope::AllocScope(hipStream_t s) : prev(t_alloc_stream) { t_alloc_stream = s; }
AllocScope::~AllocScope() { t_alloc_stream = prev; }
FreeScope::FreeScope(hipStream_t s) : prev(t_free_stream) { t_free_stream = s; }
FreeScope::~FreeScope() { t_free_stream = prev; }

gc_status dalloc(DeviceBuffer &b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.ptr && b.bytes >= bytes) return GC_OK;
  dfree(b);
  const bool ordered = t_alloc_stream != nullptr;
  hipError_t e = ordered ? hipMallocAsync(&b.ptr, bytes, t_alloc_stream) : hipMalloc(&b.ptr, bytes);
  if (e != hipSuccess) {
    b.ptr = nullptr;
    b.bytes = 0;
    (void)hipGetLastError();
    set_error(std::string(ordered ? "hipMallocAsync(" : "hipMalloc(") + std::to_string(bytes) +
              "): " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? GC_ENOMEM : GC_EDEVICE;
  }
  b.bytes = bytes;
  b.ordered = ordered;
  b.ord = t_alloc_stream;
  return GC_OK;
}

void dfree(DeviceBuffer &b) {
  if (b.ptr) {
    if (b.ordered) (void)hipFreeAsync(b.ptr, t_free_stream ? t_free_stream : b.ord);
    else (void)hipFree(b.ptr);
  }
  b.ptr = nullptr;
  b.bytes = 0;
  b.ord = nullptr;
  b.ordered = false;
}

// Run `fn` with the handle's device current, restoring the caller's device.
template <class F>
static gc_status on_device(const gc_graph *g, F &&fn) {
  int prev = 0;
  GC_HIP(hipGetDevice(&prev));
  if (prev != g->device) GC_HIP(hipSetDevice(g->device));
  gc_status st = fn();
  if (prev != g->device) (void)hipSetDevice(prev);
  return st;
}

__global__ void k_slot_to_canonical(const int32_t *__restrict__ sup,
                                    const int32_t *__restrict__ eid, int32_t m,
                                    int32_t *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    out[eid[i]] = sup[i];
}

static __global__ void k_zero_i32(int32_t *__restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Slot-order support of gc_edge_support_noalloc: one int32 per oriented edge
// of the graph being counted.  Every GPU the library runs on holds its own
// copy until the process ends, and every call on that GPU shares it (calls
// that overlap on one GPU race).  In host code `scratch` names a host-side
// stand-in, never the device array: kernels get the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) int32_t scratch[GC_NOALLOC_MAX_EDGES];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static int32_t *g_scratch_ptr[kScratchDevices] = {nullptr};

// Device address of `scratch` on device `dev`, which must be current.  The
// symbol is looked up once per device, on the first call there.
static gc_status scratch_on_device(int dev, int32_t **out) {
  if (dev < 0 || dev >= kScratchDevices) {
    set_error("gc_edge_support_noalloc: device ordinal beyond the library's table");
    return GC_EDEVICE;
  }
  try {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void *p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        return GC_EDEVICE;
      }
      g_scratch_ptr[dev] = static_cast<int32_t *>(p);
    }
    *out = g_scratch_ptr[dev];
  } catch (const std::exception &e) {
    note_host_failure("gc_edge_support_noalloc", e.what());
    return GC_ENOMEM;
  }
  return GC_OK;
}

}  // namespace gc

using namespace gc;

extern "C" gc_status gc_graph_info(const gc_graph *g, int64_t *n_vertices, int64_t *n_edges,
                                   int64_t *device_bytes) {
  clear_error();
  if (!g) {
    set_error("gc_graph_info: NULL handle");
    return GC_EINVAL;
  }
  if (n_vertices) *n_vertices = g->n;
  if (n_edges) *n_edges = g->m;
  if (device_bytes) *device_bytes = (int64_t)g->device_bytes();
  return GC_OK;
}

extern "C" gc_status gc_graph_edges(gc_graph *g, int32_t *d_u, int32_t *d_v, int64_t cap,
                                    gc_stream stream) {
  clear_error();
  if (!g || (g->m > 0 && (!d_u || !d_v))) {
    set_error("gc_graph_edges: invalid argument");
    return GC_EINVAL;
  }
  if (cap < g->m) {
    set_error("gc_graph_edges: cap < m");
    return GC_ECAPACITY;
  }
  return on_device(g, [&]() -> gc_status {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->m > 0) {
      GC_HIP(hipMemcpyAsync(d_u, g->u.ptr, sizeof(int32_t) * g->m, hipMemcpyDeviceToDevice, s));
      GC_HIP(hipMemcpyAsync(d_v, g->v.ptr, sizeof(int32_t) * g->m, hipMemcpyDeviceToDevice, s));
    }
    return GC_OK;
  });
}

extern "C" gc_status gc_graph_oriented(gc_graph *g, int32_t *d_rank, int32_t *d_row_ptr,
                                       int32_t *d_col, int32_t *d_eid, int64_t cap_n,
                                       int64_t cap_m, gc_stream stream) {
  clear_error();
  if (!g) {
    set_error("gc_graph_oriented: NULL handle");
    return GC_EINVAL;
  }
  if (((d_rank || d_row_ptr) && cap_n < (int64_t)g->n + 1) || ((d_col || d_eid) && cap_m < g->m)) {
    set_error("gc_graph_oriented: capacity too small");
    return GC_ECAPACITY;
  }
  return on_device(g, [&]() -> gc_status {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nb = sizeof(int32_t) * (size_t)g->n, mb = sizeof(int32_t) * (size_t)g->m;
    if (d_rank && nb) GC_HIP(hipMemcpyAsync(d_rank, g->rank.ptr, nb, hipMemcpyDeviceToDevice, s));
    if (d_row_ptr)
      GC_HIP(hipMemcpyAsync(d_row_ptr, g->csr.row_ptr.ptr, nb + sizeof(int32_t),
                            hipMemcpyDeviceToDevice, s));
    if (d_col && mb) GC_HIP(hipMemcpyAsync(d_col, g->csr.col.ptr, mb, hipMemcpyDeviceToDevice, s));
    if (d_eid && mb) GC_HIP(hipMemcpyAsync(d_eid, g->csr.eid.ptr, mb, hipMemcpyDeviceToDevice, s));
    return GC_OK;
  });
}

extern "C" gc_status gc_triangle_count(gc_graph *g, gc_stream stream, int64_t *h_count) {
  clear_error();
  if (!g || !h_count) {
    set_error("gc_triangle_count: invalid argument");
    return GC_EINVAL;
  }
  return on_device(g, [&]() -> gc_status {
    hipStream_t s = static_cast<hipStream_t>(stream);
    *h_count = 0;
    if (g->m == 0) return GC_OK;
    const CsrView c = g->csr.view(g->n, (int32_t)g->m);
    if (!g->units_ready) {
      GC_TRY(build_units(c, g->units, g->ws, s, g->tile));
      g->units_ready = true;
    }
    GC_TRY(g->ws.reserve(256));
    unsigned long long *d = g->ws.take<unsigned long long>(1);
    GC_HIP(hipMemsetAsync(d, 0, sizeof(unsigned long long), s));
    // one launch per degree bin, each bracketed by events for gc_graph_count_times
    for (hipEvent_t &e : g->count_ev)
      if (!e) GC_HIP(hipEventCreate(&e));
    GC_HIP(hipEventRecord(g->count_ev[0], s));
    for (int b = 0; b < kCountBins; ++b) {
      GC_TRY(count_bin(c, g->units, b, g->strategy[b], d, nullptr, nullptr, s));
      GC_HIP(hipEventRecord(g->count_ev[b + 1], s));
    }
    unsigned long long h = 0;
    GC_HIP(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s));
    GC_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < kCountBins; ++b)
      GC_HIP(hipEventElapsedTime(&g->count_ms[b], g->count_ev[b], g->count_ev[b + 1]));
    *h_count = (int64_t)h;
    return GC_OK;
  });
}

extern "C" gc_status gc_graph_autotune(gc_graph *g, gc_stream stream, int32_t *h_strategy,
                                       float *h_ms) {
  clear_error();
  if (!g) {
    set_error("gc_graph_autotune: NULL handle");
    return GC_EINVAL;
  }
  return on_device(g, [&]() -> gc_status {
    hipStream_t s = static_cast<hipStream_t>(stream);
    float ms[kCountBins * kCountStrategies];
    for (float &x : ms) x = -1.f;
    if (g->m > 0) {
      // every unit size in turn (the units of all bins rebuilt with it), every
      // admissible strategy per bin at each; per bin the fastest pair wins
      // (a later one by 3%, so near-ties keep the larger units)
      const CsrView c = g->csr.view(g->n, (int32_t)g->m);
      constexpr int nt = (int)(sizeof(kTiles) / sizeof(kTiles[0]));
      float ms_t[nt][kCountBins * kCountStrategies];
      int st_t[nt][kCountBins];
      float best[kCountBins];
      int pick[kCountBins];
      for (int b = 0; b < kCountBins; ++b) best[b] = -1.f, pick[b] = 0;
      for (int t = 0; t < nt; ++t) {
        int ch[kCountBins];
        for (int b = 0; b < kCountBins; ++b) ch[b] = kTiles[t], st_t[t][b] = g->strategy[b];
        g->units_ready = false;
        GC_TRY(build_units(c, g->units, g->ws, s, ch));
        GC_TRY(g->ws.reserve(256));
        unsigned long long *d = g->ws.take<unsigned long long>(1);
        GC_TRY(autotune_bins(c, g->units, st_t[t], ms_t[t], d, nullptr, nullptr, s));
        for (int b = 0; b < kCountBins; ++b) {
          const float x = ms_t[t][b * kCountStrategies + st_t[t][b]];
          if (x >= 0 && (best[b] < 0 || x < 0.97f * best[b])) best[b] = x, pick[b] = t;
        }
      }
      for (int b = 0; b < kCountBins; ++b) {
        g->strategy[b] = st_t[pick[b]][b];
        g->tile[b] = kTiles[pick[b]];
        for (int k = 0; k < kCountStrategies; ++k)
          ms[b * kCountStrategies + k] = ms_t[pick[b]][b * kCountStrategies + k];
      }
      GC_TRY(build_units(c, g->units, g->ws, s, g->tile));
      g->units_ready = true;
      save_strategy_cache(g->device, g->strategy, g->tile);
    }
    if (h_strategy)
      for (int b = 0; b < kCountBins; ++b) h_strategy[b] = g->strategy[b];
    if (h_ms)
      for (int i = 0; i < kCountBins * kCountStrategies; ++i) h_ms[i] = ms[i];
    return GC_OK;
  });
}

extern "C" gc_status gc_graph_truss_stats(const gc_graph *g, int64_t *h_stats, int32_t cap) {
  clear_error();
  if (!g || !h_stats || cap < 0) {
    set_error("gc_graph_truss_stats: invalid argument");
    return GC_EINVAL;
  }
  constexpr int32_t kStats = (int32_t)(sizeof(g->peel_stats) / sizeof(g->peel_stats[0]));
  for (int32_t i = 0; i < cap && i < kStats; ++i) h_stats[i] = g->peel_stats[i];
  return GC_OK;
}

extern "C" gc_status gc_graph_count_times(const gc_graph *g, float *h_ms, int32_t cap) {
  clear_error();
  if (!g || !h_ms || cap < 0) {
    set_error("gc_graph_count_times: invalid argument");
    return GC_EINVAL;
  }
  for (int32_t b = 0; b < cap && b < kCountBins; ++b) h_ms[b] = g->count_ms[b];
  return GC_OK;
}

extern "C" gc_status gc_graph_set_strategy(gc_graph *g, const int32_t *h_strategy) {
  clear_error();
  if (!g || !h_strategy) {
    set_error("gc_graph_set_strategy: invalid argument");
    return GC_EINVAL;
  }
  for (int b = 0; b < kCountBins; ++b)
    if (!count_strategy_valid(b, h_strategy[b])) {
      set_error("gc_graph_set_strategy: strategy not admissible for its bin");
      return GC_EINVAL;
    }
  for (int b = 0; b < kCountBins; ++b) g->strategy[b] = h_strategy[b];
  return GC_OK;
}

extern "C" gc_status gc_graph_set_tile(gc_graph *g, const int32_t *h_tile) {
  clear_error();
  if (!g || !h_tile) {
    set_error("gc_graph_set_tile: invalid argument");
    return GC_EINVAL;
  }
  for (int b = 0; b < kCountBins; ++b)
    if (!unit_chunk_valid(h_tile[b])) {
      set_error("gc_graph_set_tile: a unit size is not 32, 64 or 128");
      return GC_EINVAL;
    }
  bool same = true;
  for (int b = 0; b < kCountBins; ++b) same = same && g->tile[b] == h_tile[b];
  if (same) return GC_OK;
  for (int b = 0; b < kCountBins; ++b) g->tile[b] = h_tile[b];
  g->units_ready = false;  // the next count rebuilds its units
  return GC_OK;
}

extern "C" gc_status gc_graph_count_config(const gc_graph *g, int32_t *h_strategy,
                                           int32_t *h_tile) {
  clear_error();
  if (!g) {
    set_error("gc_graph_count_config: NULL handle");
    return GC_EINVAL;
  }
  for (int b = 0; b < kCountBins; ++b) {
    if (h_strategy) h_strategy[b] = g->strategy[b];
    if (h_tile) h_tile[b] = g->tile[b];
  }
  return GC_OK;
}

extern "C" gc_status gc_edge_support(gc_graph *g, int32_t *d_support, int64_t cap,
                                     gc_stream stream) {
  clear_error();
  if (!g || (g->m > 0 && !d_support)) {
    set_error("gc_edge_support: invalid argument");
    return GC_EINVAL;
  }
  if (cap < g->m) {
    set_error("gc_edge_support: cap < m");
    return GC_ECAPACITY;
  }
  return on_device(g, [&]() -> gc_status {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->m == 0) return GC_OK;
    const int32_t m = (int32_t)g->m;
    const CsrView c = g->csr.view(g->n, m);
    if (!g->units_sup_ready) {
      GC_TRY(build_units_support(c, g->units_sup, g->ws, s));
      g->units_sup_ready = true;
    }
    GC_TRY(dalloc(g->t_sup, sizeof(int32_t) * (size_t)m));
    int32_t *sup = static_cast<int32_t *>(g->t_sup.ptr);
    GC_HIP(hipMemsetAsync(sup, 0, sizeof(int32_t) * (size_t)m, s));
    GC_TRY(slot_support(c, g->units_sup, sup, s));
    k_slot_to_canonical<<<grid_for(m, 256, 65536), 256, 0, s>>>(sup, c.eid, m, d_support);
    GC_LAUNCH_CHECK();
    return GC_OK;
  });
}

extern "C" gc_status gc_edge_support_noalloc(gc_graph *g, int32_t *d_support, int64_t cap,
                                             gc_stream stream) {
  clear_error();
  if (!g || (g->m > 0 && !d_support)) {
    set_error("gc_edge_support_noalloc: invalid argument");
    return GC_EINVAL;
  }
  if (cap < g->m) {
    set_error("gc_edge_support_noalloc: cap < m");
    return GC_ECAPACITY;
  }
  if (g->m > (int64_t)GC_NOALLOC_MAX_EDGES) {
    set_error("gc_edge_support_noalloc: m = " + std::to_string(g->m) +
              " edges exceeds GC_NOALLOC_MAX_EDGES = " + std::to_string(GC_NOALLOC_MAX_EDGES) +
              "; use gc_edge_support");
    return GC_ECAPACITY;
  }
  if (g->m > 0 && !g->units_sup_ready) {
    set_error("gc_edge_support_noalloc: the handle has no support work units");
    return GC_EINVAL;
  }
  return on_device(g, [&]() -> gc_status {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->m == 0) return GC_OK;
    const int32_t m = (int32_t)g->m;
    const CsrView c = g->csr.view(g->n, m);
    int32_t *sup = nullptr;
    GC_TRY(scratch_on_device(g->device, &sup));
    // the previous call's counts are still there: clear the part used
    k_zero_i32<<<grid_for(m, 256, 65536), 256, 0, s>>>(sup, m);
    GC_LAUNCH_CHECK();
    GC_TRY(slot_support(c, g->units_sup, sup, s));
    k_slot_to_canonical<<<grid_for(m, 256, 65536), 256, 0, s>>>(sup, c.eid, m, d_support);
    GC_LAUNCH_CHECK();
    return GC_OK;
  });
}

extern "C" void gc_graph_free(gc_graph *g) {
  if (!g) return;
  int prev = 0;
  bool have_prev = hipGetDevice(&prev) == hipSuccess;
  if (have_prev && prev != g->device) (void)hipSetDevice(g->device);
  g->release();
  if (have_prev && prev != g->device) (void)hipSetDevice(prev);
  delete g;
}

extern "C" const char *gc_status_str(gc_status status) {
  switch (status) {
    case GC_OK: return "GC_OK";
    case GC_EINVAL: return "GC_EINVAL: invalid argument";
    case GC_ERANGE: return "GC_ERANGE: vertex id out of range";
    case GC_ECAPACITY: return "GC_ECAPACITY: output buffer too small";
    case GC_ENOMEM: return "GC_ENOMEM: device or host allocation failed";
    case GC_EDEVICE: return "GC_EDEVICE: HIP runtime error";
    case GC_EOVERFLOW: return "GC_EOVERFLOW: size beyond the library's limits";
    default: return "unknown gc_status";
  }
}

extern "C" const char *gc_last_error(void) { return t_last_error.c_str(); }
