// gc_count.hip -- per-edge intersection kernels: the triangle count
// T = sum(A .* (L L)) (Alg. 3's masked product with L in degree order, each
// triangle once) and the per-edge support s(e) = |N(u) cap N(v)| (Sec. III-B).
//
// Schedule ("stage the middle vertex").  Every triangle has ranks a < b < c
// and is seen exactly once, at its middle vertex b: the oriented slot p holds
// edge a -> b, the tail of row a after p holds every c > b with a -> c, and
// the triangle exists iff c is also in N+(b).  A work unit is (b, a chunk of
// b's in-list): the block stages N+(b) once in an LDS hash table, then each
// of its waves lays the tails of its in-edges of the chunk end to end and
// streams that concatenation, 64 consecutive elements per load (coalesced
// within a tail), 4 loads in flight per lane, so short tails do not leave
// lanes idle; a lane finds the tail of its next element by stepping on from
// the tail of its last one.
//
// Two LDS table layouts: linear probing over single slots (LinTable), and
// buckets of 4 slots in 16 bytes, filled in slot order, with linear probing
// over buckets (BucketTable): a probe reads one bucket (ds_read_b128) and
// compares 4 keys, and the key is absent as soon as a bucket with a free slot
// is seen.  The reads of the 4 in-flight elements are issued together.
//
// Degree bins pick the table size: d+(b) <= 32, 256, 2048 and 8192 (count) /
// 4096 (support).  Per bin the count chooses one of six strategies (see
// count_strategy_valid): either layout with at most half or a quarter of the
// slots used, binary search of N+(b) in HBM (the only one for the last,
// unbounded bin), or for bins 0 and 1 a lane group per unit with its own
// table, or a merge of each tail with N+(b).  The autotuner times them per
// bin on the graph at hand.
//
// Support: a hit (a, b, c) adds one to each of its three edges.  a -> b (the
// in-edge) is counted in an LDS counter per packed in-edge and added once per
// unit; b -> c (the staged edge) in an 8-bit LDS counter per table slot,
// added once per unit after each staged edge finds its slot again; a -> c
// (the streamed element) takes one global atomic.
#include <stdio.h>
#include <stdlib.h>

#include <string>

#include "gc_graph.h"

namespace gc {

constexpr int CBLK = 256;
constexpr int CWAVES = CBLK / 64;
constexpr int UNIT_CHUNK = 128;  // in-edges per work unit
constexpr int NBINS = 5;
constexpr int TC_UNROLL = 4;     // tail elements in flight per lane

// Out-degree bounds of the bins (inclusive); the last bin is unbounded.
__host__ __device__ constexpr int bin_limit_count(int b) {
  return b == 0 ? 32 : b == 1 ? 256 : b == 2 ? 2048 : b == 3 ? 8192 : 0x7fffffff;
}
__host__ __device__ constexpr int bin_limit_support(int b) {
  return b == 0 ? 32 : b == 1 ? 256 : b == 2 ? 2048 : b == 3 ? 4096 : 0x7fffffff;
}
// log2 of the bucket count holding a bin's out-lists at load <= 1/2
__host__ __device__ constexpr int bin_logb_count(int b) {
  return b == 0 ? 4 : b == 1 ? 7 : b == 2 ? 10 : 12;
}
__host__ __device__ constexpr int bin_logb_support(int b) {
  return b == 0 ? 4 : b == 1 ? 7 : b == 2 ? 10 : 11;
}

__device__ __forceinline__ uint32_t hash_to(int32_t w, int logn) {
  return ((uint32_t)w * 0x9E3779B1u) >> (32 - logn);
}

// ---- LDS hash tables -------------------------------------------------------
// Both keep non-negative keys; -1 marks a free slot.  They are filled by the
// whole block (after clear + barrier) and only read afterwards.

// Linear probing, one key per 4-byte slot, 1 << LOGS slots.
template <int LOGS>
struct LinTable {
  static constexpr int SLOTS = 1 << LOGS;
  using Probe = int32_t;
  __device__ static void clear(int32_t *t) {
    for (int i = threadIdx.x; i < SLOTS; i += CBLK) t[i] = -1;
  }
  __device__ static int32_t insert(int32_t *t, int32_t w) {
    uint32_t h = hash_to(w, LOGS);
    while (atomicCAS(&t[h], -1, w) != -1) h = (h + 1) & (SLOTS - 1);
    return (int32_t)h;
  }
  __device__ static Probe first(const int32_t *t, int32_t w) { return t[hash_to(w, LOGS)]; }
  // slot holding w, or -1; `x` is the value read at w's home slot
  __device__ static int32_t find(const int32_t *t, int32_t w, Probe x) {
    uint32_t h = hash_to(w, LOGS);
    for (;;) {
      if (x == w) return (int32_t)h;
      if (x < 0) return -1;
      h = (h + 1) & (SLOTS - 1);
      x = t[h];
    }
  }
};

// Buckets of 4 slots (16 bytes, one ds_read_b128 per bucket), 1 << LOGB
// buckets, slots of a bucket filled in order, linear probing over buckets: a
// key is absent as soon as a bucket with a free slot is seen.
template <int LOGB>
struct BucketTable {
  static constexpr int SLOTS = 4 << LOGB;
  using Probe = int4;
  __device__ static void clear(int32_t *t) {
    int4 *b = reinterpret_cast<int4 *>(t);
    for (int i = threadIdx.x; i < (1 << LOGB); i += CBLK) b[i] = make_int4(-1, -1, -1, -1);
  }
  __device__ static int32_t insert(int32_t *t, int32_t w) {
    uint32_t b = hash_to(w, LOGB);
    for (;;) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (atomicCAS(&t[b * 4 + k], -1, w) == -1) return (int32_t)(b * 4 + k);
      b = (b + 1) & ((1u << LOGB) - 1);
    }
  }
  __device__ static Probe first(const int32_t *t, int32_t w) {
    return reinterpret_cast<const int4 *>(t)[hash_to(w, LOGB)];
  }
  __device__ static int32_t find(const int32_t *t, int32_t w, Probe k) {
    uint32_t b = hash_to(w, LOGB);
    for (;;) {
      if (k.x == w) return (int32_t)(b * 4);
      if (k.y == w) return (int32_t)(b * 4 + 1);
      if (k.z == w) return (int32_t)(b * 4 + 2);
      if (k.w == w) return (int32_t)(b * 4 + 3);
      if (k.w < 0) return -1;
      b = (b + 1) & ((1u << LOGB) - 1);
      k = reinterpret_cast<const int4 *>(t)[b];
    }
  }
};

// Make this wave's LDS stores visible to its other lanes (and its loads done
// before later stores): within one wave a fence and a wave barrier suffice.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- streaming the tails ---------------------------------------------------
// A unit's staged table is probed with the tails of its in-edges.  Each wave
// takes its in-edges of the unit (at most UNIT_CHUNK / CWAVES of them: j0,
// j0 + CWAVES, ...), lays their tails end to end, and its lanes take
// consecutive elements of that concatenation, 64 * TC_UNROLL per step, so
// short tails do not leave lanes idle; the next step's loads are issued
// before the current step is probed.  offs / xs: this wave's LDS arrays
// (first element of each tail in the concatenation, and its position in
// col).
constexpr int TC_PACK = UNIT_CHUNK / CWAVES;
static_assert(TC_PACK <= 64, "one in-edge per lane");

__device__ __forceinline__ void pack_tails(const CsrView &c, int32_t j0, int32_t j1, int lane,
                                           int32_t *offs, int32_t *xs, int32_t &total) {
  int32_t x = 0, len = 0;
  if (lane < TC_PACK) {
    const int32_t j = j0 + lane * CWAVES;
    if (j < j1) {
      const int2 t = c.in_tail[j];
      x = t.x;
      len = t.y > t.x ? t.y - t.x : 0;
    }
  }
  const int32_t incl = wave_inclusive_scan(len);
  if (lane < TC_PACK) {
    offs[lane] = incl - len;
    xs[lane] = x;
  }
  total = __shfl(incl, 63, 64);
}

// Position in col of tail element number t of the packing, for t that only
// grows from one call to the next (a lane's elements are base + 64 u + lane,
// in order): the in-edge whose tail holds t is found by stepping on from the
// previous one (k, its first element off_k and position x_k, and the next
// tail's first element), so a lane reads LDS only when it crosses into
// another tail, at most TC_PACK times per packing.  Empty tails (equal
// offsets) are stepped over.
struct PackCursor {
  int32_t k, off_k, x_k, off_next;
  __device__ __forceinline__ void init(const int32_t *offs, const int32_t *xs) {
    k = 0;
    off_k = offs[0];
    x_k = xs[0];
    off_next = TC_PACK > 1 ? offs[1] : 0x7fffffff;
  }
  __device__ __forceinline__ int32_t pos(const int32_t *offs, const int32_t *xs, int32_t t) {
    while (t >= off_next) {
      ++k;
      off_k = off_next;
      x_k = xs[k];
      off_next = k + 1 < TC_PACK ? offs[k + 1] : 0x7fffffff;
    }
    return x_k + (t - off_k);
  }
};

template <class TB>
__device__ __forceinline__ int32_t probe_packed(const int32_t *tab, const CsrView &c, int32_t j0,
                                                int32_t j1, int lane, int32_t *offs,
                                                int32_t *xs) {
  int32_t total;
  pack_tails(c, j0, j1, lane, offs, xs, total);
  wave_lds_sync();
  int32_t hits = 0;
  PackCursor cur;
  cur.init(offs, xs);
  // (the tails are in distinct rows, so total <= m < 2^31; positions past it
  // are formed in 64 bits)
  int32_t w[TC_UNROLL];
#pragma unroll
  for (int u = 0; u < TC_UNROLL; ++u) {
    const int32_t t = 64 * u + lane;
    w[u] = t < total ? c.col[cur.pos(offs, xs, t)] : -1;
  }
  for (int64_t base = 0; base < total; base += 64 * TC_UNROLL) {
    int32_t wn[TC_UNROLL];
#pragma unroll
    for (int u = 0; u < TC_UNROLL; ++u) {  // the next step, in flight while we probe
      const int64_t t = base + 64 * TC_UNROLL + 64 * u + lane;
      wn[u] = t < total ? c.col[cur.pos(offs, xs, (int32_t)t)] : -1;
    }
    typename TB::Probe q[TC_UNROLL];
#pragma unroll
    for (int u = 0; u < TC_UNROLL; ++u)
      if (w[u] >= 0) q[u] = TB::first(tab, w[u]);
#pragma unroll
    for (int u = 0; u < TC_UNROLL; ++u)
      if (w[u] >= 0 && TB::find(tab, w[u], q[u]) >= 0) ++hits;
#pragma unroll
    for (int u = 0; u < TC_UNROLL; ++u) w[u] = wn[u];
  }
  wave_lds_sync();  // offs / xs are rewritten for the next unit
  return hits;
}

// ----------------------------------------------------------------------------
// Work units
// ----------------------------------------------------------------------------
__global__ void k_unit_counts(const int32_t *__restrict__ row_ptr,
                              const int32_t *__restrict__ in_ptr, int32_t n, int lo, int hi,
                              int32_t chunk, int32_t *__restrict__ cnt) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int32_t dout = row_ptr[x + 1] - row_ptr[x];
    const int32_t din = in_ptr[x + 1] - in_ptr[x];
    cnt[x] = (dout > lo && dout <= hi && din > 0) ? (din + chunk - 1) / chunk : 0;
  }
}

__global__ void k_unit_fill(const int32_t *__restrict__ in_ptr, const int32_t *__restrict__ off,
                            int32_t n, const int32_t *__restrict__ totals, int bin,
                            int32_t chunk, int4 *__restrict__ units) {
  int64_t base = 0;
  for (int b = 0; b < bin; ++b) base += totals[b];
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k0 = off[x], k1 = off[x + 1];
    const int32_t ib = in_ptr[x], ie = in_ptr[x + 1];
    for (int32_t k = k0; k < k1; ++k) {
      const int32_t b = ib + (k - k0) * chunk;
      const int32_t e = b + chunk < ie ? b + chunk : ie;
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
                                  bool support_bins, const int *chunk) {
  int ch[NBINS];
  int ch_min = UNIT_CHUNK;
  for (int b = 0; b < NBINS; ++b) {
    ch[b] = chunk && unit_chunk_valid(chunk[b]) ? chunk[b] : UNIT_CHUNK;
    ch_min = ch[b] < ch_min ? ch[b] : ch_min;
  }
  const int32_t n = c.n;
  GC_TRY(ws.reserve(abytes<int32_t>((size_t)n + 2) * 2 + scan_scratch_bytes(n) +
                    abytes<int32_t>(16)));
  int32_t *cnt = ws.take<int32_t>((size_t)n + 2);
  int32_t *off = ws.take<int32_t>((size_t)n + 2);
  void *scr = ws.take<char>(scan_scratch_bytes(n));
  int32_t *totals = ws.take<int32_t>(16);
  // upper bound on units: every vertex with in-edges, plus m / chunk
  const int64_t maxu = (int64_t)n + (int64_t)c.m / ch_min + 1;
  GC_TRY(dalloc(u.units, sizeof(int4) * (size_t)maxu));
  const unsigned g = grid_for(n, 256, 65536);
  for (int b = 0; b < NBINS; ++b) {
    const int lo = b == 0 ? 0 : (support_bins ? bin_limit_support(b - 1) : bin_limit_count(b - 1));
    const int hi = support_bins ? bin_limit_support(b) : bin_limit_count(b);
    k_unit_counts<<<g, 256, 0, s>>>(c.row_ptr, c.in_ptr, n, lo, hi, ch[b], cnt);
    GC_LAUNCH_CHECK();
    GC_TRY(exclusive_scan(cnt, off, n, scr, s));
    k_copy_total<<<1, 64, 0, s>>>(off, n, totals, b);
    GC_LAUNCH_CHECK();
    k_unit_fill<<<g, 256, 0, s>>>(c.in_ptr, off, n, totals, b, ch[b],
                                  static_cast<int4 *>(u.units.ptr));
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

gc_status build_units(const CsrView &c, UnitStore &u, Workspace &ws, hipStream_t s,
                      const int *chunk) {
  GC_TRY(build_units_with(c, u, ws, s, false, chunk));
  for (int b = 0; b < NBINS; ++b)
    u.chunk[b] = chunk && unit_chunk_valid(chunk[b]) ? chunk[b] : UNIT_CHUNK;
  return GC_OK;
}

gc_status build_units_support(const CsrView &c, UnitStore &u, Workspace &ws, hipStream_t s) {
  GC_TRY(build_units_with(c, u, ws, s, true, nullptr));
  for (int b = 0; b < NBINS; ++b) u.chunk[b] = UNIT_CHUNK;
  return GC_OK;
}

bool unit_chunk_valid(int chunk) { return chunk == 32 || chunk == 64 || chunk == 128; }

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

// Stage N+(v) (slots [rb, re) of col) into the table; returns after a barrier.
template <class TB>
__device__ __forceinline__ void stage_row(int32_t *tab, const int32_t *__restrict__ col, int32_t rb,
                                          int32_t re) {
  TB::clear(tab);
  __syncthreads();
  for (int32_t i = rb + threadIdx.x; i < re; i += CBLK) TB::insert(tab, col[i]);
  __syncthreads();
}

// contig = 0: block b takes units b, b + grid, ... (interleaved: neighbouring
// units, which have similar costs, spread over the blocks); contig = 1: block
// b takes a contiguous stretch of units, and since the units of one middle
// vertex are consecutive, the block stages N+(b) once for all of its units
// in the stretch instead of once per unit.
template <class TB>
__global__ __launch_bounds__(CBLK) void k_tc_lds(CsrView c, const int4 *__restrict__ units,
                                                 int64_t nunits, CountOut out, int contig) {
  __shared__ int4 mem[TB::SLOTS / 4];
  __shared__ int32_t poffs[CWAVES][TC_PACK], pxs[CWAVES][TC_PACK];
  int32_t *tab = reinterpret_cast<int32_t *>(mem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long total = 0;  // wave-uniform
  const int64_t per = contig ? (nunits + gridDim.x - 1) / gridDim.x : 1;
  const int64_t u0 = contig ? (int64_t)blockIdx.x * per : (int64_t)blockIdx.x;
  const int64_t u1 = contig ? (u0 + per < nunits ? u0 + per : nunits) : nunits;
  const int64_t ustep = contig ? 1 : (int64_t)gridDim.x;
  int32_t staged = -1;  // middle vertex whose N+ the table holds
  for (int64_t ui = u0; ui < u1; ui += ustep) {
    const int4 U = units[ui];
    if (U.x != staged) {  // block-uniform: every thread reads the same unit
      stage_row<TB>(tab, c.col, c.row_ptr[U.x], c.row_ptr[U.x + 1]);
      staged = U.x;
    }
    const int32_t sum =
        wave_sum_i32(probe_packed<TB>(tab, c, U.y + wave, U.z, lane, poffs[wave], pxs[wave]));
    if (out.per_graph) {
      if (lane == 0 && sum) atomicAdd(&out.per_graph[out.graph_of_rank[U.x]], (unsigned long long)sum);
    } else {
      total += (unsigned)sum;
    }
    __syncthreads();
  }
  if (!out.per_graph && lane == 0 && total) atomicAdd(out.total, total);
}

// Short out-lists (strategy 5): a group of GL lanes per unit with a table of
// its own in LDS, so there are no block barriers; the group lays the tails
// of GL in-edges at a time end to end and its lanes take consecutive
// elements.  Suits graphs whose units are many and small (tails of a few
// elements, as in sparse uniform graphs), where a block per unit would mostly
// wait at barriers.  The lanes of a group always hold the same unit, so they
// stay converged; groups of one wave may be at different units (each only
// touches its own table).
template <int LOGS, int GL>
__global__ __launch_bounds__(CBLK) void k_tc_group(CsrView c, const int4 *__restrict__ units,
                                                   int64_t nunits, CountOut out) {
  using TB = LinTable<LOGS>;
  constexpr int GPB = CBLK / GL;  // groups per block
  __shared__ int32_t tabs[GPB][TB::SLOTS];
  const int gl = threadIdx.x % GL;
  int32_t *tab = tabs[threadIdx.x / GL];
  const int64_t gid = ((int64_t)blockIdx.x * CBLK + threadIdx.x) / GL;
  const int64_t ng = (int64_t)gridDim.x * GPB;
  int32_t hits = 0;  // over every unit of this lane (total count)
  for (int64_t ui = gid; ui < nunits; ui += ng) {
    const int4 U = units[ui];
    const int32_t rb = c.row_ptr[U.x], re = c.row_ptr[U.x + 1];
    for (int i = gl; i < TB::SLOTS; i += GL) tab[i] = -1;
    wave_lds_sync();
    for (int32_t i = rb + gl; i < re; i += GL) TB::insert(tab, c.col[i]);
    wave_lds_sync();
    int32_t mine = 0;
    // GL in-edges at a time: their tails laid end to end (offsets by a scan
    // over the group), the group's lanes take consecutive elements, 4 in
    // flight per lane; the tail of an element is found by a search over the
    // GL offsets held in the lanes
    for (int32_t j0 = U.y; j0 < U.z; j0 += GL) {
      const int32_t j = j0 + gl;
      int32_t x = 0, len = 0;
      if (j < U.z) {
        const int2 t = c.in_tail[j];
        x = t.x;
        len = t.y > t.x ? t.y - t.x : 0;
      }
      int32_t incl = len;
#pragma unroll
      for (int o = 1; o < GL; o <<= 1) {
        const int32_t v = __shfl_up(incl, o, GL);
        if (gl >= o) incl += v;
      }
      const int32_t total = __shfl(incl, GL - 1, GL), excl = incl - len;
      for (int32_t t0 = 0; t0 < total; t0 += 4 * GL) {
        int32_t w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t t = t0 + u * GL + gl;
          int k = 0;
#pragma unroll
          for (int s2 = GL / 2; s2 > 0; s2 >>= 1)
            if (__shfl(excl, k + s2, GL) <= t) k += s2;
          const int32_t xk = __shfl(x, k, GL), ek = __shfl(excl, k, GL);
          w[u] = t < total ? c.col[xk + (t - ek)] : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (w[u] >= 0) mine += TB::find(tab, w[u], TB::first(tab, w[u])) >= 0;
      }
    }
    if (out.per_graph) {
      // sum over the group (its lanes are converged) and one atomic per unit
      for (int o = GL / 2; o > 0; o >>= 1) mine += __shfl_xor(mine, o, GL);
      if (gl == 0 && mine)
        atomicAdd(&out.per_graph[out.graph_of_rank[U.x]], (unsigned long long)mine);
    } else {
      hits += mine;
    }
    wave_lds_sync();  // the group is done with the table before it is cleared
  }
  if (!out.per_graph) {
    const int32_t sum = wave_sum_i32(hits);  // all lanes are back together here
    if ((threadIdx.x & 63) == 0 && sum) atomicAdd(out.total, (unsigned long long)sum);
  }
}

// Merge (strategy 6, bins 0 and 1): a group of GL lanes per unit copies the
// sorted N+(b) (at most MAXD entries) to LDS, and each lane takes whole
// in-edges a -> b, merging the sorted tail of a's row with it by two
// pointers: |tail(a) cap N+(b)| in at most |tail| + d+(b) steps.  No hashing
// and no search; suits short lists on both sides.
template <int MAXD, int GL>
__global__ __launch_bounds__(CBLK) void k_tc_merge(CsrView c, const int4 *__restrict__ units,
                                                   int64_t nunits, CountOut out) {
  constexpr int GPB = CBLK / GL;  // groups per block
  __shared__ int32_t rows[GPB][MAXD];
  const int gl = threadIdx.x % GL;
  int32_t *row = rows[threadIdx.x / GL];
  const int64_t gid = ((int64_t)blockIdx.x * CBLK + threadIdx.x) / GL;
  const int64_t ng = (int64_t)gridDim.x * GPB;
  int32_t hits = 0;  // over every unit of this lane (total count)
  for (int64_t ui = gid; ui < nunits; ui += ng) {
    const int4 U = units[ui];
    const int32_t rb = c.row_ptr[U.x], d = c.row_ptr[U.x + 1] - rb;
    for (int32_t i = gl; i < d; i += GL) row[i] = c.col[rb + i];
    wave_lds_sync();
    int32_t mine = 0;
    for (int32_t j = U.y + gl; j < U.z; j += GL) {
      const int2 t = c.in_tail[j];
      int32_t i = t.x, k = 0;
      while (i < t.y && k < d) {
        const int32_t x = c.col[i], y = row[k];
        i += x <= y ? 1 : 0;
        k += y <= x ? 1 : 0;
        mine += x == y ? 1 : 0;
      }
    }
    if (out.per_graph) {
      for (int o = GL / 2; o > 0; o >>= 1) mine += __shfl_xor(mine, o, GL);
      if (gl == 0 && mine)
        atomicAdd(&out.per_graph[out.graph_of_rank[U.x]], (unsigned long long)mine);
    } else {
      hits += mine;
    }
    wave_lds_sync();  // the group is done with the row before it is overwritten
  }
  if (!out.per_graph) {
    const int32_t sum = wave_sum_i32(hits);
    if ((threadIdx.x & 63) == 0 && sum) atomicAdd(out.total, (unsigned long long)sum);
  }
}

// Out-lists too long for LDS: binary search in the sorted row in HBM.
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
    const int32_t sum = wave_sum_i32(hits);
    if (out.per_graph) {
      if (lane == 0 && sum) atomicAdd(&out.per_graph[out.graph_of_rank[U.x]], (unsigned long long)sum);
    } else {
      total += (unsigned)sum;
    }
  }
  if (!out.per_graph && lane == 0 && total) atomicAdd(out.total, total);
}

static unsigned unit_grid(int64_t nunits, int per_cu) {
  int64_t g = 256LL * per_cu;
  if (nunits < g) g = nunits;
  return (unsigned)(g < 1 ? 1 : g);
}

// Strategies per bin (the autotuner's search space):
//   0 linear-probing table, load <= 1/2     1 linear-probing table, load <= 1/4
//   2 binary search in HBM                  3 bucketed table, load <= 1/2
//   4 bucketed table, load <= 1/4           5 one wave per unit, own table
//                                             (bins 0 and 1 only)
//   6 merge of each tail with N+(b) (bins 0 and 1 only)
// The last (unbounded) bin only admits 2.
bool count_strategy_valid(int bin, int strategy) {
  if (strategy == 2) return true;
  if (strategy == 5 || strategy == 6) return bin <= 1;
  return bin < NBINS - 1 && strategy >= 0 && strategy < kCountStrategies;
}

// Blocks of the LDS-table count kernel per CU (the grid is at most 256 times
// this), and whether each block takes a contiguous stretch of units, for a
// table of `bytes` bytes.  Tables of 16 KB and more (bins 2 and up: long
// out-lists, and vertices with many units each) stage N+(b) once per stretch;
// smaller tables interleave their units, whose costs vary more between
// neighbours (R-MAT scale 24: bin 2 45.0 -> 41.3 ms contiguous, bin 1 4.09 ->
// 4.53 ms contiguous, so it keeps interleaving).
constexpr int tc_lds_per_cu(int bytes) {
  // well above the blocks that fit at once: each block takes a short stretch
  // of units, and the dispatcher evens out the end (2x: 79.5 ms, 4x: 76.9 ms,
  // 8x: 73.4 ms, 16x: 72.2 ms for the scale-24 pass; one block per unit:
  // 123 ms)
  return bytes <= 8192 ? 256 : bytes <= 16384 ? 512 : bytes <= 32768 ? 64 : bytes <= 65536 ? 32 : 16;
}
constexpr bool tc_lds_contig(int bytes) { return bytes >= 16384; }

template <class TB>
static void launch_tc_lds(const CsrView &c, const int4 *ub, int64_t nu, const CountOut &o,
                          hipStream_t s) {
  constexpr int bytes = TB::SLOTS * 4;
  k_tc_lds<TB><<<unit_grid(nu, tc_lds_per_cu(bytes)), CBLK, 0, s>>>(c, ub, nu, o,
                                                                    tc_lds_contig(bytes) ? 1 : 0);
}

// log2 of linear-probing slots at load <= 1/2 per bin
__host__ __device__ constexpr int bin_logs_count(int b) {
  return b == 0 ? 6 : b == 1 ? 9 : b == 2 ? 12 : 14;
}

static gc_status launch_count_bin(const CsrView &c, const int4 *ub, int64_t nu, int b,
                                  int strategy, const CountOut &o, hipStream_t s) {
  if (strategy == 2 || b == NBINS - 1) {
    k_tc_search<<<unit_grid(nu, 8), CBLK, 0, s>>>(c, ub, nu, o);
  } else if (strategy == 5) {
    if (b == 0)  // d+ <= 32: groups of 16 lanes, 16 units per block
      k_tc_group<6, 16><<<unit_grid((nu + 15) / 16, 16), CBLK, 0, s>>>(c, ub, nu, o);
    else         // d+ <= 256: a wave per unit
      k_tc_group<9, 64><<<unit_grid((nu + 3) / 4, 16), CBLK, 0, s>>>(c, ub, nu, o);
  } else if (strategy == 6) {
    if (b == 0)  // d+ <= 32: groups of 16 lanes
      k_tc_merge<32, 16><<<unit_grid((nu + 15) / 16, 16), CBLK, 0, s>>>(c, ub, nu, o);
    else         // d+ <= 256: a wave per unit
      k_tc_merge<256, 64><<<unit_grid((nu + 3) / 4, 16), CBLK, 0, s>>>(c, ub, nu, o);
  } else if (strategy == 0 || strategy == 1) {
    switch (bin_logs_count(b) + (strategy == 1 ? 1 : 0)) {
      case 6: launch_tc_lds<LinTable<6>>(c, ub, nu, o, s); break;
      case 7: launch_tc_lds<LinTable<7>>(c, ub, nu, o, s); break;
      case 9: launch_tc_lds<LinTable<9>>(c, ub, nu, o, s); break;
      case 10: launch_tc_lds<LinTable<10>>(c, ub, nu, o, s); break;
      case 12: launch_tc_lds<LinTable<12>>(c, ub, nu, o, s); break;
      case 13: launch_tc_lds<LinTable<13>>(c, ub, nu, o, s); break;
      case 14: launch_tc_lds<LinTable<14>>(c, ub, nu, o, s); break;
      default: launch_tc_lds<LinTable<15>>(c, ub, nu, o, s); break;
    }
  } else {
    switch (bin_logb_count(b) + (strategy == 4 ? 1 : 0)) {
      case 4: launch_tc_lds<BucketTable<4>>(c, ub, nu, o, s); break;
      case 5: launch_tc_lds<BucketTable<5>>(c, ub, nu, o, s); break;
      case 7: launch_tc_lds<BucketTable<7>>(c, ub, nu, o, s); break;
      case 8: launch_tc_lds<BucketTable<8>>(c, ub, nu, o, s); break;
      case 10: launch_tc_lds<BucketTable<10>>(c, ub, nu, o, s); break;
      case 11: launch_tc_lds<BucketTable<11>>(c, ub, nu, o, s); break;
      case 12: launch_tc_lds<BucketTable<12>>(c, ub, nu, o, s); break;
      default: launch_tc_lds<BucketTable<13>>(c, ub, nu, o, s); break;
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

gc_status autotune_bins(const CsrView &c, const UnitStore &u, int *strategy, float *ms,
                        unsigned long long *d_total, unsigned long long *d_per_graph,
                        const int32_t *graph_of_rank, hipStream_t s) {
  for (int i = 0; i < kCountBins * kCountStrategies; ++i) ms[i] = -1.f;
  if (c.m == 0) return GC_OK;
  hipEvent_t e0, e1;
  GC_HIP(hipEventCreate(&e0));
  {
    const hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      set_error(std::string("hipEventCreate: ") + hipGetErrorString(e));
      return GC_EDEVICE;
    }
  }
  gc_status st = GC_OK;
  for (int bin = 0; bin < kCountBins && st == GC_OK; ++bin) {
    if (u.bin_count[bin] == 0) continue;
    float best = -1.f;
    for (int k = 0; k < kCountStrategies && st == GC_OK; ++k) {
      if (!count_strategy_valid(bin, k)) continue;
      float acc = 0;
      for (int rep = 0; rep < 3 && st == GC_OK; ++rep) {  // the first run warms caches
        if (hipEventRecord(e0, s) != hipSuccess) { st = GC_EDEVICE; break; }
        st = count_bin(c, u, bin, k, d_total, d_per_graph, graph_of_rank, s);
        if (st != GC_OK) break;
        float t = 0;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
          st = GC_EDEVICE;
          break;
        }
        if (rep > 0) acc += t;
      }
      if (st != GC_OK) break;
      ms[bin * kCountStrategies + k] = acc / 2;
      // a later strategy must win by 3% to replace an earlier one (stable
      // choices when two are within timing noise)
      if (best < 0 || acc / 2 < 0.97f * best) {
        best = acc / 2;
        strategy[bin] = k;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

static std::string arch_of(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// Lines "<arch> <bin> <strategy> [<tile>]" (a line without a tile keeps the
// tile as it is).
void load_strategy_cache(int device, int *strategy, int *tile) {
  const char *path = getenv("GC_AUTOTUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  const std::string arch = arch_of(device);
  char line[256], a[128];
  int bin, st, t;
  while (fgets(line, sizeof line, f)) {
    const int got = sscanf(line, "%127s %d %d %d", a, &bin, &st, &t);
    if (got < 3 || arch != a || bin < 0 || bin >= kCountBins || !count_strategy_valid(bin, st))
      continue;
    strategy[bin] = st;
    if (got == 4 && tile && unit_chunk_valid(t)) tile[bin] = t;
  }
  fclose(f);
}

void save_strategy_cache(int device, const int *strategy, const int *tile) {
  const char *path = getenv("GC_AUTOTUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "w");
  if (!f) return;
  const std::string arch = arch_of(device);
  for (int bin = 0; bin < kCountBins; ++bin)
    fprintf(f, "%s %d %d %d\n", arch.c_str(), bin, strategy[bin], tile ? tile[bin] : UNIT_CHUNK);
  fclose(f);
}

// ----------------------------------------------------------------------------
// Many graphs (separately built handles) in one launch per bin
// ----------------------------------------------------------------------------
__device__ __forceinline__ int32_t find_graph(const int64_t *__restrict__ pre, int32_t nh,
                                              int64_t ui) {
  int32_t lo = 0, hi = nh + 1;  // upper bound of ui in pre[0..nh]
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= ui) lo = mid + 1; else hi = mid;
  }
  return lo - 1;
}

template <class TB>
__global__ __launch_bounds__(CBLK) void k_tc_lds_multi(const GraphDesc *__restrict__ d,
                                                       const int64_t *__restrict__ pre,
                                                       int32_t nh, int bin,
                                                       unsigned long long *__restrict__ out) {
  __shared__ int4 mem[TB::SLOTS / 4];
  __shared__ int32_t poffs[CWAVES][TC_PACK], pxs[CWAVES][TC_PACK];
  int32_t *tab = reinterpret_cast<int32_t *>(mem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t total = pre[nh];
  for (int64_t ui = blockIdx.x; ui < total; ui += gridDim.x) {
    const int32_t g = find_graph(pre, nh, ui);
    const CsrView c = d[g].c;
    const int4 U = d[g].units[d[g].bin_begin[bin] + (ui - pre[g])];
    stage_row<TB>(tab, c.col, c.row_ptr[U.x], c.row_ptr[U.x + 1]);
    const int32_t sum =
        wave_sum_i32(probe_packed<TB>(tab, c, U.y + wave, U.z, lane, poffs[wave], pxs[wave]));
    if (lane == 0 && sum) atomicAdd(&out[g], (unsigned long long)sum);
    __syncthreads();
  }
}

__global__ __launch_bounds__(CBLK) void k_tc_search_multi(const GraphDesc *__restrict__ d,
                                                          const int64_t *__restrict__ pre,
                                                          int32_t nh, int bin,
                                                          unsigned long long *__restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t total = pre[nh];
  for (int64_t ui = blockIdx.x; ui < total; ui += gridDim.x) {
    const int32_t g = find_graph(pre, nh, ui);
    const CsrView c = d[g].c;
    const int4 U = d[g].units[d[g].bin_begin[bin] + (ui - pre[g])];
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
    const int32_t sum = wave_sum_i32(hits);
    if (lane == 0 && sum) atomicAdd(&out[g], (unsigned long long)sum);
  }
}

__global__ void k_zero_counts(unsigned long long *__restrict__ x, int32_t n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) x[i] = 0;
}

gc_status count_multi_launch(const GraphDesc *d_desc, const int64_t *d_pre, const int64_t *h_pre,
                             int32_t nh, unsigned long long *d_out, hipStream_t s) {
  k_zero_counts<<<grid_for(nh, 256, 1024), 256, 0, s>>>(d_out, nh);
  GC_LAUNCH_CHECK();
  for (int b = 0; b < NBINS; ++b) {
    const int64_t nu = h_pre[(int64_t)b * (nh + 1) + nh];
    if (nu == 0) continue;
    const int64_t *pre = d_pre + (int64_t)b * (nh + 1);
    if (b == NBINS - 1) {
      k_tc_search_multi<<<unit_grid(nu, 8), CBLK, 0, s>>>(d_desc, pre, nh, b, d_out);
    } else {
      switch (b) {
        case 0: k_tc_lds_multi<LinTable<6>><<<unit_grid(nu, 16), CBLK, 0, s>>>(d_desc, pre, nh, b, d_out); break;
        case 1: k_tc_lds_multi<LinTable<9>><<<unit_grid(nu, 16), CBLK, 0, s>>>(d_desc, pre, nh, b, d_out); break;
        case 2: k_tc_lds_multi<LinTable<12>><<<unit_grid(nu, 8), CBLK, 0, s>>>(d_desc, pre, nh, b, d_out); break;
        default: k_tc_lds_multi<LinTable<14>><<<unit_grid(nu, 2), CBLK, 0, s>>>(d_desc, pre, nh, b, d_out); break;
      }
    }
    GC_LAUNCH_CHECK();
  }
  return GC_OK;
}

// ----------------------------------------------------------------------------
// Per-slot support
// ----------------------------------------------------------------------------
template <int LOGS>
__global__ __launch_bounds__(CBLK) void k_sup_lds(CsrView c, const int4 *__restrict__ units,
                                                  int64_t nunits, int32_t *__restrict__ sup) {
  using TB = LinTable<LOGS>;
  constexpr int NS = TB::SLOTS;
  // hits on the staged edge b -> c of table slot t within this unit: byte
  // t % 4 of tcnt[t / 4] (at most one per in-edge of the unit, so < 2^8)
  static_assert(UNIT_CHUNK < (1 << 8), "8-bit hit counters");
  __shared__ int4 mem[NS / 4];
  __shared__ uint32_t tcnt[NS / 4];
  __shared__ int32_t poffs[CWAVES][TC_PACK], pxs[CWAVES][TC_PACK], picnt[CWAVES][TC_PACK];
  int32_t *tab = reinterpret_cast<int32_t *>(mem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t ui = blockIdx.x; ui < nunits; ui += gridDim.x) {
    const int4 U = units[ui];
    const int32_t rb = c.row_ptr[U.x], re = c.row_ptr[U.x + 1];
    TB::clear(tab);
    for (int i = threadIdx.x; i < NS / 4; i += CBLK) tcnt[i] = 0;
    __syncthreads();
    for (int32_t i = rb + threadIdx.x; i < re; i += CBLK) TB::insert(tab, c.col[i]);
    __syncthreads();
    // this wave's in-edges of the unit (U.y + wave, + CWAVES, ...), tails
    // packed end to end as in the count; hits of in-edge k go to icnt[k]
    int32_t *offs = poffs[wave], *xs = pxs[wave], *icnt = picnt[wave];
    if (lane < TC_PACK) icnt[lane] = 0;
    int32_t total;
    pack_tails(c, U.y + wave, U.z, lane, offs, xs, total);
    wave_lds_sync();
    PackCursor cur;
    cur.init(offs, xs);
    for (int64_t base = 0; base < total; base += 64 * TC_UNROLL) {
      int32_t w[TC_UNROLL], pp[TC_UNROLL], kk[TC_UNROLL];
#pragma unroll
      for (int u = 0; u < TC_UNROLL; ++u) {
        const int64_t t = base + 64 * u + lane;
        w[u] = -1;
        if (t < total) {
          pp[u] = cur.pos(offs, xs, (int32_t)t);
          kk[u] = cur.k;
          w[u] = c.col[pp[u]];
        }
      }
      typename TB::Probe q[TC_UNROLL];
#pragma unroll
      for (int u = 0; u < TC_UNROLL; ++u)
        if (w[u] >= 0) q[u] = TB::first(tab, w[u]);
#pragma unroll
      for (int u = 0; u < TC_UNROLL; ++u) {
        if (w[u] < 0) continue;
        const int32_t at = TB::find(tab, w[u], q[u]);
        if (at >= 0) {
          atomicAdd(&icnt[kk[u]], 1);                        // edge a -> b
          atomicAdd(&tcnt[at >> 2], 1u << ((at & 3) << 3));  // edge b -> c
          atomicAdd(&sup[pp[u]], 1);                         // edge a -> c
        }
      }
    }
    wave_lds_sync();
    if (lane < TC_PACK) {
      const int32_t j = U.y + wave + lane * CWAVES;
      if (j < U.z && icnt[lane]) atomicAdd(&sup[c.in_edge[j].y], icnt[lane]);
    }
    __syncthreads();
    // each staged edge finds its table slot again and adds its hits
    for (int32_t i = rb + threadIdx.x; i < re; i += CBLK) {
      const int32_t w = c.col[i];
      const int32_t at = TB::find(tab, w, TB::first(tab, w));
      const uint32_t h = at >= 0 ? (tcnt[at >> 2] >> ((at & 3) << 3)) & 0xffu : 0u;
      if (h) atomicAdd(&sup[i], (int32_t)h);
    }
    __syncthreads();
  }
}

// Short out-lists: a group of GL lanes per unit, as k_tc_group, each with its
// own table, staged-edge slots and counters in LDS; lane l of the group takes
// in-edges first + l, first + l + GL, ... and adds its hits to that in-edge
// once.
template <int LOGS, int GL>
__global__ __launch_bounds__(CBLK) void k_sup_group(CsrView c, const int4 *__restrict__ units,
                                                    int64_t nunits, int32_t *__restrict__ sup) {
  using TB = LinTable<LOGS>;
  constexpr int NS = TB::SLOTS;
  constexpr int GPB = CBLK / GL;  // groups per block
  __shared__ int32_t tabs[GPB][NS];
  __shared__ int32_t slots[GPB][NS];  // oriented slot of the staged edge b -> c
  __shared__ int32_t cnts[GPB][NS];   // hits on that edge within this unit
  __shared__ int32_t icnts[GPB][GL];  // hits of the group's current in-edges
  const int gl = threadIdx.x % GL, grp = threadIdx.x / GL;
  int32_t *tab = tabs[grp], *tslot = slots[grp], *tcnt = cnts[grp], *icnt = icnts[grp];
  const int64_t gid = ((int64_t)blockIdx.x * CBLK + threadIdx.x) / GL;
  const int64_t ng = (int64_t)gridDim.x * GPB;
  for (int64_t ui = gid; ui < nunits; ui += ng) {
    const int4 U = units[ui];
    const int32_t rb = c.row_ptr[U.x], re = c.row_ptr[U.x + 1];
    for (int i = gl; i < NS; i += GL) {
      tab[i] = -1;
      tcnt[i] = 0;
    }
    wave_lds_sync();
    for (int32_t i = rb + gl; i < re; i += GL) tslot[TB::insert(tab, c.col[i])] = i;
    wave_lds_sync();
    // GL in-edges at a time, tails packed as in k_tc_group; hits of in-edge
    // k of the chunk go to icnt[k]
    for (int32_t j0 = U.y; j0 < U.z; j0 += GL) {
      const int32_t j = j0 + gl;
      int32_t x = 0, len = 0;
      if (j < U.z) {
        const int2 t = c.in_tail[j];
        x = t.x;
        len = t.y > t.x ? t.y - t.x : 0;
      }
      icnt[gl] = 0;
      int32_t incl = len;
#pragma unroll
      for (int o = 1; o < GL; o <<= 1) {
        const int32_t v = __shfl_up(incl, o, GL);
        if (gl >= o) incl += v;
      }
      const int32_t total = __shfl(incl, GL - 1, GL), excl = incl - len;
      wave_lds_sync();
      for (int32_t t0 = 0; t0 < total; t0 += 4 * GL) {
        int32_t w[4], pp[4], kk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t t = t0 + u * GL + gl;
          int k = 0;
#pragma unroll
          for (int s2 = GL / 2; s2 > 0; s2 >>= 1)
            if (__shfl(excl, k + s2, GL) <= t) k += s2;
          const int32_t xk = __shfl(x, k, GL), ek = __shfl(excl, k, GL);
          kk[u] = k;
          pp[u] = xk + (t - ek);
          w[u] = t < total ? c.col[pp[u]] : -1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (w[u] < 0) continue;
          const int32_t at = TB::find(tab, w[u], TB::first(tab, w[u]));
          if (at >= 0) {
            atomicAdd(&icnt[kk[u]], 1);  // edge a -> b
            atomicAdd(&tcnt[at], 1);     // edge b -> c
            atomicAdd(&sup[pp[u]], 1);   // edge a -> c
          }
        }
      }
      wave_lds_sync();
      if (j < U.z && icnt[gl]) atomicAdd(&sup[c.in_edge[j].y], icnt[gl]);
      wave_lds_sync();  // icnt is cleared for the next chunk
    }
    wave_lds_sync();
    for (int i = gl; i < NS; i += GL)
      if (tcnt[i]) atomicAdd(&sup[tslot[i]], tcnt[i]);
    wave_lds_sync();  // the group is done with its arrays before they are cleared
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
      if (lane == 0 && tot) atomicAdd(&sup[c.in_edge[j].y], tot);
    }
  }
}

gc_status slot_support(const CsrView &c, const UnitStore &u, int32_t *d_sup, hipStream_t s) {
  const int4 *units = static_cast<const int4 *>(u.units.ptr);
  for (int b = 0; b < NBINS; ++b) {
    const int64_t nu = u.bin_count[b];
    if (nu == 0) continue;
    const int4 *ub = units + u.bin_begin[b];
    // bin 2: many more blocks than fit at once (each takes a few interleaved
    // units; R-MAT scale 24 support pass 115 -> 110 ms from 64 to 1024 per
    // CU; one block per unit: 119 ms)
    switch (b) {
      case 0: k_sup_group<6, 16><<<unit_grid((nu + 15) / 16, 16), CBLK, 0, s>>>(c, ub, nu, d_sup); break;
      case 1: k_sup_lds<9><<<unit_grid(nu, 128), CBLK, 0, s>>>(c, ub, nu, d_sup); break;
      case 2: k_sup_lds<12><<<unit_grid(nu, 1024), CBLK, 0, s>>>(c, ub, nu, d_sup); break;
      case 3: k_sup_lds<13><<<unit_grid(nu, 4), CBLK, 0, s>>>(c, ub, nu, d_sup); break;
      default: k_sup_search<<<unit_grid(nu, 8), CBLK, 0, s>>>(c, ub, nu, d_sup); break;
    }
    GC_LAUNCH_CHECK();
  }
  return GC_OK;
}

}  // namespace gc
