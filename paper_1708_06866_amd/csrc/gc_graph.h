// gc_graph.h -- the handle behind gc_graph* and the device views the counting
// and truss kernels take (internal; not part of the public ABI).
#pragma once

#include "gc_common.h"

namespace gc {

// Degree-oriented CSR over ranks, plus the in-edge index the "stage the middle
// vertex" schedule walks.  For oriented slot p (edge r -> col[p], r = src[p]):
//   tail(p) = [p + 1, row_ptr[r + 1])   the part of N+(r) above col[p]
// and the in-list of vertex x lists, for every slot p with col[p] = x, the
// range tail(p) packed as int2 {p + 1, row_end}, and in_edge[j] = {source
// of p, p} (in-lists are sorted by source; key and slot share one load).
struct CsrView {
  int32_t n = 0;
  int32_t m = 0;
  const int32_t *row_ptr = nullptr;  // [n+1]
  const int32_t *col = nullptr;      // [m]
  const int32_t *src = nullptr;      // [m]
  const int32_t *eid = nullptr;      // [m]
  const int32_t *in_ptr = nullptr;   // [n+1]
  const int2 *in_tail = nullptr;     // [m]
  const int2 *in_edge = nullptr;     // [m] {source, slot} of each in-edge
};

// Owned device arrays of one oriented CSR (base graph or a k-truss working
// copy).
struct CsrStore {
  DeviceBuffer row_ptr, col, src, eid, in_ptr, in_tail, in_edge;
  CsrView view(int32_t n, int32_t m) const {
    CsrView v;
    v.n = n;
    v.m = m;
    v.row_ptr = static_cast<const int32_t *>(row_ptr.ptr);
    v.col = static_cast<const int32_t *>(col.ptr);
    v.src = static_cast<const int32_t *>(src.ptr);
    v.eid = static_cast<const int32_t *>(eid.ptr);
    v.in_ptr = static_cast<const int32_t *>(in_ptr.ptr);
    v.in_tail = static_cast<const int2 *>(in_tail.ptr);
    v.in_edge = static_cast<const int2 *>(in_edge.ptr);
    return v;
  }
  void release() {
    dfree(row_ptr); dfree(col); dfree(src); dfree(eid);
    dfree(in_ptr); dfree(in_tail); dfree(in_edge);
  }
  size_t bytes() const {
    return row_ptr.bytes + col.bytes + src.bytes + eid.bytes + in_ptr.bytes +
           in_tail.bytes + in_edge.bytes;
  }
};

// Per-bin work-unit lists for the counting kernels (built from a CsrView).
struct UnitStore {
  DeviceBuffer units;  // int4 {v, in_begin, in_end, bin}
  int64_t bin_begin[8] = {0};
  int64_t bin_count[8] = {0};
  int chunk[8] = {128, 128, 128, 128, 128, 128, 128, 128};  // in-edges per unit, per bin
};

}  // namespace gc

struct gc_graph {
  int device = 0;
  int32_t n = 0;
  int64_t m = 0;
  int bits = 1;  // bits per vertex id: 2^bits >= n
  gc::DeviceBuffer u, v, rank;
  gc::DeviceBuffer vid;         // vid[r] = original id of the vertex of rank r
  gc::CsrStore csr;
  gc::UnitStore units;      // count-kernel work units of the base CSR
  bool units_ready = false;
  gc::UnitStore units_sup;  // support-kernel work units of the base CSR
  bool units_sup_ready = false;
  gc::Workspace ws;         // scratch for counting / truss calls
  gc::CsrStore work[2];     // k-truss ping-pong working CSRs
  gc::UnitStore work_units;
  gc::DeviceBuffer t_sup, t_flag, t_pos, t_misc;  // k-truss round state
  int strategy[5] = {0, 0, 0, 0, 2};             // count strategy per degree bin
  int tile[5] = {128, 128, 128, 128, 128};       // in-edges per count work unit, per bin
  // last decomposition: [0] levels with removals, [1] rounds, [2] frontier
  // edges, [3] largest frontier, [4] compactions, [5..36] rounds by
  // floor(log2(frontier size)), [37] candidates examined, [38] searched,
  // [39] triangles found, [40] triangles destroyed (subtracted)
  int64_t peel_stats[41] = {0};
  // duration of each degree bin's count launch in the last gc_triangle_count
  // (HIP events around the launches on the call's stream; -1 before one)
  hipEvent_t count_ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  float count_ms[5] = {-1.f, -1.f, -1.f, -1.f, -1.f};
  template <class F>
  void each_buffer(F &&f) const {
    for (const gc::DeviceBuffer *b : {&u, &v, &rank, &vid, &units.units, &units_sup.units, &ws.buf,
                                      &work_units.units, &t_sup, &t_flag, &t_pos, &t_misc})
      f(*b);
    for (const gc::CsrStore *c : {&csr, &work[0], &work[1]})
      for (const gc::DeviceBuffer *b : {&c->row_ptr, &c->col, &c->src, &c->eid, &c->in_ptr,
                                        &c->in_tail, &c->in_edge})
        f(*b);
  }
  // bytes requested from the allocator
  size_t device_bytes() const {
    size_t t = 0;
    each_buffer([&](const gc::DeviceBuffer &b) { t += b.bytes; });
    return t;
  }
  // bytes the allocator holds for them (its rounding included)
  size_t device_bytes_held() const {
    size_t t = 0;
    each_buffer([&](const gc::DeviceBuffer &b) { t += gc::held_bytes(b); });
    return t;
  }
  void release() {
    gc::dfree(u); gc::dfree(v); gc::dfree(rank); gc::dfree(vid);
    csr.release(); work[0].release(); work[1].release();
    gc::dfree(units.units); gc::dfree(units_sup.units); gc::dfree(work_units.units);
    gc::dfree(t_sup); gc::dfree(t_flag); gc::dfree(t_pos); gc::dfree(t_misc);
    gc::dfree(ws.buf);
    for (hipEvent_t &e : count_ev)
      if (e) {
        (void)hipEventDestroy(e);
        e = nullptr;
      }
  }
};

namespace gc {

// Internal entry points shared between translation units.
// (gc_build.hip)
gc_status build_in_lists(int32_t n, int32_t m, int bits, CsrStore &c, Workspace &ws,
                         hipStream_t s);
// (gc_count.hip)
// Count units with `chunk[b]` in-edges per unit in bin b (32, 64 or 128;
// null: 128 in every bin).
gc_status build_units(const CsrView &c, UnitStore &u, Workspace &ws, hipStream_t s,
                      const int *chunk = nullptr);
bool unit_chunk_valid(int chunk);
gc_status build_units_support(const CsrView &c, UnitStore &u, Workspace &ws, hipStream_t s);
gc_status count_triangles(const CsrView &c, const UnitStore &u, unsigned long long *d_count,
                          hipStream_t s);
constexpr int kCountBins = 5;
// 0/1 linear-probing LDS table (load <= 1/2, 1/4), 2 binary search in HBM,
// 3/4 bucketed LDS table (load <= 1/2, 1/4), 5 one wave per unit (bins 0, 1),
// 6 merge of sorted lists (bins 0, 1)
constexpr int kCountStrategies = 7;
bool count_strategy_valid(int bin, int strategy);
// Count with a chosen strategy per bin (strategy may be null = defaults); per
// graph counts if d_per_graph != null (graph_of_rank maps a rank to its graph).
gc_status count_triangles_ex(const CsrView &c, const UnitStore &u, unsigned long long *d_total,
                             unsigned long long *d_per_graph, const int32_t *graph_of_rank,
                             const int *strategy, hipStream_t s);
gc_status count_bin(const CsrView &c, const UnitStore &u, int bin, int strategy,
                    unsigned long long *d_total, unsigned long long *d_per_graph,
                    const int32_t *graph_of_rank, hipStream_t s);
gc_status slot_support(const CsrView &c, const UnitStore &u, int32_t *d_sup, hipStream_t s);
// Time every admissible strategy of every bin that has work (HIP events, the
// first run of each discarded) and return the fastest per bin in strategy[];
// ms[bin * kCountStrategies + st] = mean time (-1 if not run).  Counts go to
// d_total or, per graph, to d_per_graph (graph_of_rank != null).
gc_status autotune_bins(const CsrView &c, const UnitStore &u, int *strategy, float *ms,
                        unsigned long long *d_total, unsigned long long *d_per_graph,
                        const int32_t *graph_of_rank, hipStream_t s);
// Strategy cache file (environment GC_AUTOTUNE_CACHE): load into / save from
// strategy[kCountBins] and tile[kCountBins] (either may be null: not loaded,
// or saved as 128) for the given device.
void load_strategy_cache(int device, int *strategy, int *tile);
void save_strategy_cache(int device, const int *strategy, const int *tile);
// Count-unit sizes the autotuner tries, in order (ties keep the earlier one).
constexpr int kTiles[3] = {128, 64, 32};

// One graph of a multi-graph count launch (device-side descriptor).
struct GraphDesc {
  CsrView c;
  const int4 *units;
  int64_t bin_begin[kCountBins];
};
// Count triangles of nh graphs in one launch per bin: d_desc[nh] descriptors,
// d_pre / h_pre [kCountBins][nh+1] per-bin prefix sums of the graphs' unit
// counts (device and host copies); per-graph counts into d_out[nh].
gc_status count_multi_launch(const GraphDesc *d_desc, const int64_t *d_pre, const int64_t *h_pre,
                             int32_t nh, unsigned long long *d_out, hipStream_t s);
// (gc_peel.hip) truss numbers by peeling with incremental support updates;
// tau holds m entries, or is null (truss numbers not written).  With k_stop,
// peeling ends before the first level above k_stop: mask (m bytes, may be
// null) then marks the edges of the k_stop-truss and *h_mk counts them.
gc_status decomposition_peel(gc_graph *g, int32_t *tau, int32_t *h_kmax, hipStream_t s,
                             int32_t k_stop = 0x7fffffff, uint8_t *mask = nullptr,
                             int64_t *h_mk = nullptr);

// Device buffers of a k-truss whose launches are recorded once into a HIP
// graph and replayed (PeelReplay::prepare allocates them before recording).
struct PeelReplay {
  DeviceBuffer sup, state, front[2], flag, pos, scan, ctl;
  int32_t m = 0;
  gc_status prepare(int32_t m_edges);
  void release() {
    dfree(sup); dfree(state); dfree(front[0]); dfree(front[1]);
    dfree(flag); dfree(pos); dfree(scan); dfree(ctl);
  }
  // frontier still pending after the last recorded round of level l + 3
  // (device, 64 levels at most), 0 where the level ended within its rounds
  int32_t *leftover() const;
};
// The k-truss of g (levels 3 .. k, `rounds` rounds each, no compaction, no
// frontier sort, no min-support jump) as launches only: no allocation, no
// host wait, no memset, so the sequence can be recorded into a HIP graph.
// mask[e] = 1 for the edges of the k-truss when every level ended within
// its rounds (r.leftover() all 0); otherwise the result is incomplete.
gc_status ktruss_launches(const gc_graph *g, int32_t k, int32_t rounds, PeelReplay &r,
                          uint8_t *mask, hipStream_t s);

}  // namespace gc
