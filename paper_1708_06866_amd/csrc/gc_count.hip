// gc_count.hip -- per-edge intersection kernels: the triangle count
// T = sum(A .* (L L)) (Alg. 3's masked product with L in degree order, each
// triangle once) and the per-edge support s(e) = |N(u) cap N(v)| (Sec. III-B).
//
// Schedule ("stage the middle vertex").  Every triangle has ranks a < b < c
// and is seen exactly once, at its middle vertex b: the oriented slot p holds
// edge a -> b, the tail of row a after p holds every c > b with a -> c, and
// the triangle exists iff c is also in N+(b).  A work unit is (b, a chunk of
// b's in-list): the block stages N+(b) once in an LDS hash table, then its
// waves stream the tails of the chunk's in-edges, one tail per wave, 64
// consecutive elements per step (coalesced), probing each element.
//
// Degree bins pick the table: d+(b) <= 32, 256, 2048 and 8192 (count) /
// 4096 (support) use LDS tables of 64, 512, 4096 and 16384 / 8192 slots
// (load factor <= 1/2, linear probing); larger out-lists are binary-searched
// in place in global memory.
//
// Support: a hit (a, b, c) adds one to each of its three edges.  a -> b (the
// in-edge) is summed over the wave and added once per in-edge; b -> c (the
// staged edge) is counted in an LDS counter beside the table entry and
// flushed once per unit; a -> c (the streamed element) takes one global
// atomic.
#include "gc_graph.h"

namespace gc {

constexpr int CBLK = 256;
constexpr int CWAVES = CBLK / 64;
constexpr int UNIT_CHUNK = 128;  // in-edges per work unit
constexpr int NBINS = 5;
constexpr int TC_UNROLL = 4;     // tail loads in flight per lane

// Out-degree bounds of the bins (inclusive); the last bin is unbounded.
__host__ __device__ constexpr int bin_limit_count(int b) {
  return b == 0 ? 32 : b == 1 ? 256 : b == 2 ? 2048 : b == 3 ? 8192 : 0x7fffffff;
}
__host__ __device__ constexpr int bin_limit_support(int b) {
  return b == 0 ? 32 : b == 1 ? 256 : b == 2 ? 2048 : b == 3 ? 4096 : 0x7fffffff;
}

__device__ __forceinline__ uint32_t hslot(int32_t w, int logh) {
  return ((uint32_t)w * 0x9E3779B1u) >> (32 - logh);
}

// ----------------------------------------------------------------------------
// Work units
// ----------------------------------------------------------------------------
__global__ void k_unit_counts(const int32_t *__restrict__ row_ptr,
                              const int32_t *__restrict__ in_ptr, int32_t n, int lo, int hi,
                              int32_t *__restrict__ cnt) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int32_t dout = row_ptr[x + 1] - row_ptr[x];
    const int32_t din = in_ptr[x + 1] - in_ptr[x];
    cnt[x] = (dout > lo && dout <= hi && din > 0) ? (din + UNIT_CHUNK - 1) / UNIT_CHUNK : 0;
  }
}

__global__ void k_unit_fill(const int32_t *__restrict__ in_ptr, const int32_t *__restrict__ off,
                            int32_t n, const int32_t *__restrict__ totals, int bin,
                            int4 *__restrict__ units) {
  int64_t base = 0;
  for (int b = 0; b < bin; ++b) base += totals[b];
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k0 = off[x], k1 = off[x + 1];
    const int32_t ib = in_ptr[x], ie = in_ptr[x + 1];
    for (int32_t k = k0; k < k1; ++k) {
      const int32_t b = ib + (k - k0) * UNIT_CHUNK;
      const int32_t e = b + UNIT_CHUNK < ie ? b + UNIT_CHUNK : ie;
      units[base + k] = make_int4((int32_t)x, b, e, bin);
    }
  }
}

__global__ void k_copy_total(const int32_t *__restrict__ off, int32_t n, int32_t *__restrict__ totals,
                             int bin) {
  if (threadIdx.x == 0 && blockIdx.x == 0) totals[bin] = off[n];
}

// Units for both the count and the support kernels use the support bin
// limits for the split between bins 3 and 4 only when asked; the store keeps
// one list per limit set.
static gc_status build_units_with(const CsrView &c, UnitStore &u, Workspace &ws, hipStream_t s,
                                  bool support_bins) {
  const int32_t n = c.n;
  GC_TRY(ws.reserve(abytes<int32_t>((size_t)n + 2) * 2 + scan_scratch_bytes(n) +
                    abytes<int32_t>(16)));
  int32_t *cnt = ws.take<int32_t>((size_t)n + 2);
  int32_t *off = ws.take<int32_t>((size_t)n + 2);
  void *scr = ws.take<char>(scan_scratch_bytes(n));
  int32_t *totals = ws.take<int32_t>(16);
  // upper bound on units: every vertex with in-edges, plus m / chunk
  const int64_t maxu = (int64_t)n + (int64_t)c.m / UNIT_CHUNK + 1;
  GC_TRY(dalloc(u.units, sizeof(int4) * (size_t)maxu));
  const unsigned g = grid_for(n, 256, 65536);
  for (int b = 0; b < NBINS; ++b) {
    const int lo = b == 0 ? 0 : (support_bins ? bin_limit_support(b - 1) : bin_limit_count(b - 1));
    const int hi = support_bins ? bin_limit_support(b) : bin_limit_count(b);
    k_unit_counts<<<g, 256, 0, s>>>(c.row_ptr, c.in_ptr, n, lo, hi, cnt);
    GC_LAUNCH_CHECK();
    GC_TRY(exclusive_scan(cnt, off, n, scr, s));
    k_copy_total<<<1, 64, 0, s>>>(off, n, totals, b);
    GC_LAUNCH_CHECK();
    k_unit_fill<<<g, 256, 0, s>>>(c.in_ptr, off, n, totals, b, static_cast<int4 *>(u.units.ptr));
    GC_LAUNCH_CHECK();
  }
  int32_t h[NBINS];
  GC_HIP(hipMemcpyAsync(h, totals, sizeof(h), hipMemcpyDeviceToHost, s));
  GC_HIP(hipStreamSynchronize(s));
  int64_t acc = 0;
  for (int b = 0; b < NBINS; ++b) {
    u.bin_begin[b] = acc;
    u.bin_count[b] = h[b];
    acc += h[b];
  }
  return GC_OK;
}

gc_status build_units(const CsrView &c, UnitStore &u, Workspace &ws, hipStream_t s) {
  return build_units_with(c, u, ws, s, false);
}

gc_status build_units_support(const CsrView &c, UnitStore &u, Workspace &ws, hipStream_t s) {
  return build_units_with(c, u, ws, s, true);
}

// ----------------------------------------------------------------------------
// Triangle count
// ----------------------------------------------------------------------------
// Where counts go: one total, or one counter per graph of a batch (the graph
// of a unit is the graph of its middle vertex).
struct CountOut {
  unsigned long long *total = nullptr;
  unsigned long long *per_graph = nullptr;
  const int32_t *graph_of_rank = nullptr;
};

__device__ __forceinline__ void flush_unit(const CountOut &o, int32_t v, int32_t hits,
                                           unsigned long long &total, int lane) {
  const int32_t s = wave_sum_i32(hits);
  if (o.per_graph) {
    if (lane == 0 && s) atomicAdd(&o.per_graph[o.graph_of_rank[v]], (unsigned long long)s);
  } else {
    total += (unsigned)s;
  }
}

template <int LOGH>
__global__ __launch_bounds__(CBLK) void k_tc_hash(CsrView c, const int4 *__restrict__ units,
                                                  int64_t nunits, CountOut out) {
  constexpr int H = 1 << LOGH;
  __shared__ int32_t tab[H];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long total = 0;  // wave-uniform
  for (int64_t ui = blockIdx.x; ui < nunits; ui += gridDim.x) {
    const int4 U = units[ui];
    const int32_t rb = c.row_ptr[U.x], re = c.row_ptr[U.x + 1];
    for (int i = threadIdx.x; i < H; i += CBLK) tab[i] = -1;
    __syncthreads();
    for (int32_t i = rb + threadIdx.x; i < re; i += CBLK) {
      const int32_t w = c.col[i];
      uint32_t h = hslot(w, LOGH);
      while (atomicCAS(&tab[h], -1, w) != -1) h = (h + 1) & (H - 1);
    }
    __syncthreads();
    int32_t hits = 0;
    int32_t j = U.y + wave;
    int2 t = j < U.z ? c.in_tail[j] : make_int2(0, 0);
    for (; j < U.z; j += CWAVES) {
      // prefetch the next in-edge's tail range while this one streams
      const int2 tn = j + CWAVES < U.z ? c.in_tail[j + CWAVES] : make_int2(0, 0);
      for (int32_t p = t.x + lane; p < t.y; p += 64 * TC_UNROLL) {
        int32_t w[TC_UNROLL];
#pragma unroll
        for (int k = 0; k < TC_UNROLL; ++k) w[k] = p + 64 * k < t.y ? c.col[p + 64 * k] : -1;
#pragma unroll
        for (int k = 0; k < TC_UNROLL; ++k) {
          if (w[k] < 0) continue;
          uint32_t h = hslot(w[k], LOGH);
          for (;;) {
            const int32_t x = tab[h];
            if (x == w[k]) { ++hits; break; }
            if (x < 0) break;
            h = (h + 1) & (H - 1);
          }
        }
      }
      t = tn;
    }
    flush_unit(out, U.x, hits, total, lane);
    __syncthreads();
  }
  if (!out.per_graph && lane == 0 && total) atomicAdd(out.total, total);
}

// Out-lists too long for LDS: binary search in the sorted row in global memory.
__global__ __launch_bounds__(CBLK) void k_tc_search(CsrView c, const int4 *__restrict__ units,
                                                    int64_t nunits, CountOut out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long total = 0;
  for (int64_t ui = blockIdx.x; ui < nunits; ui += gridDim.x) {
    const int4 U = units[ui];
    const int32_t rb = c.row_ptr[U.x], re = c.row_ptr[U.x + 1];
    int32_t hits = 0;
    for (int32_t j = U.y + wave; j < U.z; j += CWAVES) {
      const int2 t = c.in_tail[j];
      for (int32_t p = t.x + lane; p < t.y; p += 64) {
        const int32_t w = c.col[p];
        int32_t lo = rb, hi = re;
        while (lo < hi) {
          const int32_t mid = lo + ((hi - lo) >> 1);
          if (c.col[mid] < w) lo = mid + 1; else hi = mid;
        }
        hits += (lo < re && c.col[lo] == w) ? 1 : 0;
      }
    }
    flush_unit(out, U.x, hits, total, lane);
  }
  if (!out.per_graph && lane == 0 && total) atomicAdd(out.total, total);
}

static unsigned unit_grid(int64_t nunits, int per_cu) {
  int64_t g = 256LL * per_cu;
  if (nunits < g) g = nunits;
  return (unsigned)(g < 1 ? 1 : g);
}

// Strategies per bin: 0 = LDS hash at the bin's table size (load <= 1/2),
// 1 = LDS hash with a table twice as large (load <= 1/4), 2 = binary search
// in HBM.  The last bin only admits 2.
bool count_strategy_valid(int bin, int strategy) {
  if (strategy == 2) return true;
  return bin < NBINS - 1 && (strategy == 0 || strategy == 1);
}

static gc_status launch_count_bin(const CsrView &c, const int4 *ub, int64_t nu, int b,
                                  int strategy, const CountOut &o, hipStream_t s) {
  if (strategy == 2 || b == NBINS - 1) {
    k_tc_search<<<unit_grid(nu, 8), CBLK, 0, s>>>(c, ub, nu, o);
  } else {
    const int logh = (b == 0 ? 6 : b == 1 ? 9 : b == 2 ? 12 : 14) + (strategy == 1 ? 1 : 0);
    switch (logh) {
      case 6: k_tc_hash<6><<<unit_grid(nu, 16), CBLK, 0, s>>>(c, ub, nu, o); break;
      case 7: k_tc_hash<7><<<unit_grid(nu, 16), CBLK, 0, s>>>(c, ub, nu, o); break;
      case 9: k_tc_hash<9><<<unit_grid(nu, 16), CBLK, 0, s>>>(c, ub, nu, o); break;
      case 10: k_tc_hash<10><<<unit_grid(nu, 16), CBLK, 0, s>>>(c, ub, nu, o); break;
      case 12: k_tc_hash<12><<<unit_grid(nu, 8), CBLK, 0, s>>>(c, ub, nu, o); break;
      case 13: k_tc_hash<13><<<unit_grid(nu, 4), CBLK, 0, s>>>(c, ub, nu, o); break;
      case 14: k_tc_hash<14><<<unit_grid(nu, 4), CBLK, 0, s>>>(c, ub, nu, o); break;
      default: k_tc_hash<15><<<unit_grid(nu, 2), CBLK, 0, s>>>(c, ub, nu, o); break;
    }
  }
  GC_LAUNCH_CHECK();
  return GC_OK;
}

gc_status count_triangles_ex(const CsrView &c, const UnitStore &u, unsigned long long *d_total,
                             unsigned long long *d_per_graph, const int32_t *graph_of_rank,
                             const int *strategy, hipStream_t s) {
  const int4 *units = static_cast<const int4 *>(u.units.ptr);
  CountOut o;
  o.total = d_total;
  o.per_graph = d_per_graph;
  o.graph_of_rank = graph_of_rank;
  for (int b = 0; b < NBINS; ++b) {
    const int64_t nu = u.bin_count[b];
    if (nu == 0) continue;
    const int st = strategy ? strategy[b] : (b == NBINS - 1 ? 2 : 0);
    GC_TRY(launch_count_bin(c, units + u.bin_begin[b], nu, b, st, o, s));
  }
  return GC_OK;
}

gc_status count_bin(const CsrView &c, const UnitStore &u, int bin, int strategy,
                    unsigned long long *d_total, unsigned long long *d_per_graph,
                    const int32_t *graph_of_rank, hipStream_t s) {
  const int64_t nu = u.bin_count[bin];
  if (nu == 0) return GC_OK;
  CountOut o;
  o.total = d_total;
  o.per_graph = d_per_graph;
  o.graph_of_rank = graph_of_rank;
  return launch_count_bin(c, static_cast<const int4 *>(u.units.ptr) + u.bin_begin[bin], nu, bin,
                          strategy, o, s);
}

gc_status count_triangles(const CsrView &c, const UnitStore &u, unsigned long long *d_count,
                          hipStream_t s) {
  return count_triangles_ex(c, u, d_count, nullptr, nullptr, nullptr, s);
}

// ----------------------------------------------------------------------------
// Per-slot support
// ----------------------------------------------------------------------------
template <int LOGH>
__global__ __launch_bounds__(CBLK) void k_sup_hash(CsrView c, const int4 *__restrict__ units,
                                                   int64_t nunits, int32_t *__restrict__ sup) {
  constexpr int H = 1 << LOGH;
  __shared__ int32_t tab[H];
  __shared__ int32_t tslot[H];
  __shared__ int32_t tcnt[H];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t ui = blockIdx.x; ui < nunits; ui += gridDim.x) {
    const int4 U = units[ui];
    const int32_t rb = c.row_ptr[U.x], re = c.row_ptr[U.x + 1];
    for (int i = threadIdx.x; i < H; i += CBLK) { tab[i] = -1; tcnt[i] = 0; }
    __syncthreads();
    for (int32_t i = rb + threadIdx.x; i < re; i += CBLK) {
      const int32_t w = c.col[i];
      uint32_t h = hslot(w, LOGH);
      while (atomicCAS(&tab[h], -1, w) != -1) h = (h + 1) & (H - 1);
      tslot[h] = i;
    }
    __syncthreads();
    for (int32_t j = U.y + wave; j < U.z; j += CWAVES) {
      const int2 t = c.in_tail[j];
      int32_t mine = 0;
      for (int32_t p = t.x + lane; p < t.y; p += 64 * TC_UNROLL) {
        int32_t w[TC_UNROLL];
#pragma unroll
        for (int k = 0; k < TC_UNROLL; ++k) w[k] = p + 64 * k < t.y ? c.col[p + 64 * k] : -1;
#pragma unroll
        for (int k = 0; k < TC_UNROLL; ++k) {
          if (w[k] < 0) continue;
          uint32_t h = hslot(w[k], LOGH);
          for (;;) {
            const int32_t x = tab[h];
            if (x == w[k]) {
              ++mine;
              atomicAdd(&tcnt[h], 1);             // edge b -> c
              atomicAdd(&sup[p + 64 * k], 1);     // edge a -> c
              break;
            }
            if (x < 0) break;
            h = (h + 1) & (H - 1);
          }
        }
      }
      const int32_t tot = wave_sum_i32(mine);
      if (lane == 0 && tot) atomicAdd(&sup[c.in_slot[j]], tot);  // edge a -> b
    }
    __syncthreads();
    for (int i = threadIdx.x; i < H; i += CBLK)
      if (tcnt[i]) atomicAdd(&sup[tslot[i]], tcnt[i]);
    __syncthreads();
  }
}

__global__ __launch_bounds__(CBLK) void k_sup_search(CsrView c, const int4 *__restrict__ units,
                                                     int64_t nunits, int32_t *__restrict__ sup) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t ui = blockIdx.x; ui < nunits; ui += gridDim.x) {
    const int4 U = units[ui];
    const int32_t rb = c.row_ptr[U.x], re = c.row_ptr[U.x + 1];
    for (int32_t j = U.y + wave; j < U.z; j += CWAVES) {
      const int2 t = c.in_tail[j];
      int32_t mine = 0;
      for (int32_t p = t.x + lane; p < t.y; p += 64) {
        const int32_t w = c.col[p];
        int32_t lo = rb, hi = re;
        while (lo < hi) {
          const int32_t mid = lo + ((hi - lo) >> 1);
          if (c.col[mid] < w) lo = mid + 1; else hi = mid;
        }
        if (lo < re && c.col[lo] == w) {
          ++mine;
          atomicAdd(&sup[lo], 1);
          atomicAdd(&sup[p], 1);
        }
      }
      const int32_t tot = wave_sum_i32(mine);
      if (lane == 0 && tot) atomicAdd(&sup[c.in_slot[j]], tot);
    }
  }
}

gc_status slot_support(const CsrView &c, const UnitStore &u, int32_t *d_sup, hipStream_t s) {
  const int4 *units = static_cast<const int4 *>(u.units.ptr);
  for (int b = 0; b < NBINS; ++b) {
    const int64_t nu = u.bin_count[b];
    if (nu == 0) continue;
    const int4 *ub = units + u.bin_begin[b];
    switch (b) {
      case 0: k_sup_hash<6><<<unit_grid(nu, 16), CBLK, 0, s>>>(c, ub, nu, d_sup); break;
      case 1: k_sup_hash<9><<<unit_grid(nu, 16), CBLK, 0, s>>>(c, ub, nu, d_sup); break;
      case 2: k_sup_hash<12><<<unit_grid(nu, 4), CBLK, 0, s>>>(c, ub, nu, d_sup); break;
      case 3: k_sup_hash<13><<<unit_grid(nu, 1), CBLK, 0, s>>>(c, ub, nu, d_sup); break;
      default: k_sup_search<<<unit_grid(nu, 8), CBLK, 0, s>>>(c, ub, nu, d_sup); break;
    }
    GC_LAUNCH_CHECK();
  }
  return GC_OK;
}

}  // namespace gc
