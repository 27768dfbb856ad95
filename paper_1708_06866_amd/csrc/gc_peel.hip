// gc_peel.hip -- truss decomposition by level-synchronous peeling with
// incremental support updates.
//
// Alg. 4 of the paper keeps R = EA and, after dropping the rows x, updates it
// by subtracting the contribution of the dropped edges instead of redoing the
// product.  The same idea on the degree-oriented CSR: support is counted once
// for the whole graph; afterwards every round only touches the triangles of
// the edges dropped in that round (the frontier) and subtracts them from the
// surviving edges.
//
// Round at level k (threshold t = k - 2; the frontier holds every live edge
// whose support fell below t):
//   * one wavefront per frontier edge p = (a -> b) enumerates the triangles
//     {a, b, c} still present: c from the out-row of a (c > b: is c in the row
//     of b? c < b: is b in the row of c?) and from the in-list of a (is b in
//     the row of c?), each by binary search in a sorted row;
//   * a triangle is skipped if one of its edges died in an earlier round, or
//     if another frontier edge of it has a smaller slot id (so each destroyed
//     triangle is subtracted exactly once, whichever edges die together);
//     otherwise each surviving edge loses one, and an edge whose support
//     drops from t to t - 1 joins the next frontier (once);
//   * the frontier edges die with truss number k - 1.
// A level ends when the frontier is empty.  The next level is min-support + 3
// (every level in between removes nothing).  When more than half of the
// oriented CSR is dead it is compacted by a scan, carrying support and state.
//
// Results equal the rounds of Alg. 4 (bulk removal per round, same frontier
// sets); only the work per round differs.
#include "gc_graph.h"

namespace gc {

enum : uint8_t { EDGE_ALIVE = 0, EDGE_FRONT = 1, EDGE_DEAD = 2 };

constexpr int PBLK = 256;

__device__ __forceinline__ int32_t find_col(const int32_t *__restrict__ col, int32_t lo,
                                            int32_t hi, int32_t key) {
  const int32_t end = hi;
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (col[mid] < key) lo = mid + 1; else hi = mid;
  }
  return (lo < end && col[lo] == key) ? lo : -1;
}

// Triangle {p, q1, q2} seen from frontier edge p (q2 < 0: no triangle).  Every
// active lane of the wave calls this together, so the next-frontier appends
// are aggregated per wave.
__device__ __forceinline__ void destroy(bool found, int32_t p, int32_t q1, int32_t q2,
                                        int32_t thr, const uint8_t *__restrict__ state,
                                        int32_t *__restrict__ sup, int32_t *__restrict__ next,
                                        int32_t *__restrict__ next_count) {
  bool t1 = false, t2 = false;
  if (found) {
    const uint8_t s1 = state[q1], s2 = state[q2];
    // skip if destroyed in an earlier round, or owned by a smaller frontier edge
    const bool ours = s1 != EDGE_DEAD && s2 != EDGE_DEAD &&
                      !(s1 == EDGE_FRONT && q1 < p) && !(s2 == EDGE_FRONT && q2 < p);
    if (ours) {
      if (s1 == EDGE_ALIVE) t1 = atomicSub(&sup[q1], 1) == thr;
      if (s2 == EDGE_ALIVE) t2 = atomicSub(&sup[q2], 1) == thr;
    }
  }
  int32_t at = wave_append(t1, next_count);
  if (t1) next[at] = q1;
  at = wave_append(t2, next_count);
  if (t2) next[at] = q2;
}

__global__ __launch_bounds__(PBLK) void k_peel(CsrView c, const int32_t *__restrict__ front,
                                               int32_t nfront, int32_t thr,
                                               int32_t *__restrict__ sup,
                                               const uint8_t *__restrict__ state,
                                               int32_t *__restrict__ next,
                                               int32_t *__restrict__ next_count) {
  const int lane = threadIdx.x & 63;
  const int64_t wid = ((int64_t)blockIdx.x * PBLK + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * PBLK) >> 6;
  for (int64_t f = wid; f < nfront; f += nw) {
    const int32_t p = front[f];
    const int32_t a = c.src[p], b = c.col[p];
    const int32_t rb0 = c.row_ptr[b], rb1 = c.row_ptr[b + 1];
    // third vertex from the out-row of a
    const int32_t ra1 = c.row_ptr[a + 1];
    for (int32_t i = c.row_ptr[a] + lane; i < ra1; i += 64) {
      int32_t q2 = -1;
      if (i != p && state[i] != EDGE_DEAD) {
        const int32_t x = c.col[i];
        q2 = x > b ? find_col(c.col, rb0, rb1, x)
                   : find_col(c.col, c.row_ptr[x], c.row_ptr[x + 1], b);
      }
      destroy(q2 >= 0, p, i, q2, thr, state, sup, next, next_count);
    }
    // third vertex below a: from the in-list of a
    const int32_t ia1 = c.in_ptr[a + 1];
    for (int32_t j = c.in_ptr[a] + lane; j < ia1; j += 64) {
      const int32_t q1 = c.in_slot[j];
      int32_t q2 = -1;
      if (state[q1] != EDGE_DEAD) {
        const int32_t x = c.src[q1];
        q2 = find_col(c.col, c.row_ptr[x], c.row_ptr[x + 1], b);
      }
      destroy(q2 >= 0, p, q1, q2, thr, state, sup, next, next_count);
    }
  }
}

// Retire the frontier (truss number k - 1) and mark the next one.
__global__ void k_advance(const int32_t *__restrict__ front, int32_t nfront,
                          const int32_t *__restrict__ next, const int32_t *__restrict__ next_count,
                          uint8_t *__restrict__ state, const int32_t *__restrict__ eid,
                          int32_t *__restrict__ tau, int32_t tau_val) {
  const int32_t nn = *next_count;
  const int64_t lim = nfront > nn ? nfront : nn;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < lim;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nfront) {
      const int32_t p = front[i];
      state[p] = EDGE_DEAD;
      tau[eid[p]] = tau_val;
    }
  }
  __threadfence();
  // the next frontier is disjoint from the current one
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
       i += (int64_t)gridDim.x * blockDim.x)
    state[next[i]] = EDGE_FRONT;
}

__global__ void k_alive_flags(const int32_t *__restrict__ list, int32_t L,
                              const uint8_t *__restrict__ state, int32_t *__restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L;
       i += (int64_t)gridDim.x * blockDim.x)
    flag[i] = state[list[i]] == EDGE_ALIVE ? 1 : 0;
}

__global__ void k_compact_list(const int32_t *__restrict__ list, int32_t L,
                               const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                               const int32_t *__restrict__ sup, int32_t *__restrict__ out,
                               int32_t *__restrict__ dmin) {
  int32_t v = 0x7fffffff;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (flag[i]) {
      const int32_t p = list[i];
      out[pos[i]] = p;
      v = min(v, sup[p]);
    }
  }
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  __shared__ int32_t wmin[4];
  if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    v = min(min(wmin[0], wmin[1]), min(wmin[2], wmin[3]));
    if (v != 0x7fffffff) atomicMin(dmin, v);
  }
}

__global__ void k_collect(const int32_t *__restrict__ list, int32_t L, int32_t thr,
                          const int32_t *__restrict__ sup, uint8_t *__restrict__ state,
                          int32_t *__restrict__ front, int32_t *__restrict__ count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = list[i];
    const bool take = sup[p] < thr;
    const int32_t at = wave_append(take, count);
    if (take) {
      state[p] = EDGE_FRONT;
      front[at] = p;
    }
  }
}

__global__ void k_iota(int32_t *__restrict__ x, int32_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = (int32_t)i;
}

__global__ void k_set_i32(int32_t *__restrict__ x, int32_t a, int32_t b) {
  if (blockIdx.x == 0 && threadIdx.x == 0) { x[0] = a; x[1] = b; }
}

__global__ void k_not_dead(const uint8_t *__restrict__ state, int32_t m, int32_t *__restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    flag[i] = state[i] != EDGE_DEAD ? 1 : 0;
}

__global__ void k_compact_edges(const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                                int32_t m, const int32_t *__restrict__ col,
                                const int32_t *__restrict__ src, const int32_t *__restrict__ eid,
                                const int32_t *__restrict__ sup, const uint8_t *__restrict__ state,
                                int32_t *__restrict__ ncol, int32_t *__restrict__ nsrc,
                                int32_t *__restrict__ neid, int32_t *__restrict__ nsup,
                                uint8_t *__restrict__ nstate) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (flag[i]) {
      const int32_t q = pos[i];
      ncol[q] = col[i];
      nsrc[q] = src[i];
      neid[q] = eid[i];
      nsup[q] = sup[i];
      nstate[q] = state[i];
    }
  }
}

__global__ void k_remap(int32_t *__restrict__ x, int32_t n, const int32_t *__restrict__ pos) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = pos[x[i]];
}

__global__ void k_rows2(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ pos,
                        int32_t n, int32_t *__restrict__ nrow) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n;
       r += (int64_t)gridDim.x * blockDim.x)
    nrow[r] = pos[row_ptr[r]];
}

static unsigned gsz(int64_t work) { return grid_for(work, 256, 65536); }

struct PeelState {
  DeviceBuffer sup[2], state[2], list[2], front[2], flag, pos, misc;
  int cur = 0;  // which sup/state buffer is live
  ~PeelState() {
    for (int i = 0; i < 2; ++i) {
      dfree(sup[i]); dfree(state[i]); dfree(list[i]); dfree(front[i]);
    }
    dfree(flag); dfree(pos); dfree(misc);
  }
};

// Drop dead slots of `c`: new CSR in g->work[next], support/state carried into
// the other PeelState buffers, the frontier remapped.
static gc_status compact_peel(gc_graph *g, PeelState &ps, CsrView &c, int &next, int32_t *front,
                              int32_t nfront, hipStream_t s) {
  const int32_t m = c.m, n = c.n;
  int32_t *flag = static_cast<int32_t *>(ps.flag.ptr);
  int32_t *pos = static_cast<int32_t *>(ps.pos.ptr);
  const uint8_t *state = static_cast<const uint8_t *>(ps.state[ps.cur].ptr);
  const int32_t *sup = static_cast<const int32_t *>(ps.sup[ps.cur].ptr);
  k_not_dead<<<gsz(m), 256, 0, s>>>(state, m, flag);
  GC_LAUNCH_CHECK();
  GC_TRY(g->ws.reserve(scan_scratch_bytes((int64_t)m + 1)));
  GC_TRY(exclusive_scan(flag, pos, m, g->ws.take<char>(scan_scratch_bytes((int64_t)m + 1)), s));
  int32_t kept = 0;
  GC_HIP(hipMemcpyAsync(&kept, pos + m, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  GC_HIP(hipStreamSynchronize(s));
  CsrStore &w = g->work[next];
  GC_TRY(dalloc(w.row_ptr, sizeof(int32_t) * ((size_t)n + 1)));
  GC_TRY(dalloc(w.col, sizeof(int32_t) * ((size_t)kept + 1)));
  GC_TRY(dalloc(w.src, sizeof(int32_t) * ((size_t)kept + 1)));
  GC_TRY(dalloc(w.eid, sizeof(int32_t) * ((size_t)kept + 1)));
  const int o = ps.cur ^ 1;
  k_compact_edges<<<gsz(m), 256, 0, s>>>(
      flag, pos, m, c.col, c.src, c.eid, sup, state, static_cast<int32_t *>(w.col.ptr),
      static_cast<int32_t *>(w.src.ptr), static_cast<int32_t *>(w.eid.ptr),
      static_cast<int32_t *>(ps.sup[o].ptr), static_cast<uint8_t *>(ps.state[o].ptr));
  GC_LAUNCH_CHECK();
  k_rows2<<<gsz((int64_t)n + 1), 256, 0, s>>>(c.row_ptr, pos, n,
                                              static_cast<int32_t *>(w.row_ptr.ptr));
  GC_LAUNCH_CHECK();
  if (nfront > 0) {
    k_remap<<<gsz(nfront), 256, 0, s>>>(front, nfront, pos);
    GC_LAUNCH_CHECK();
  }
  GC_TRY(build_in_lists(n, kept, g->bits, w, g->ws, s));
  c = w.view(n, kept);
  next ^= 1;
  ps.cur = o;
  ++g->peel_stats[4];
  return GC_OK;
}

gc_status decomposition_peel(gc_graph *g, int32_t *tau, int32_t *h_kmax, hipStream_t s) {
  const int32_t m = (int32_t)g->m;
  if (m == 0) {
    if (h_kmax) *h_kmax = 0;
    return GC_OK;
  }
  PeelState ps;
  for (int i = 0; i < 2; ++i) {
    GC_TRY(dalloc(ps.sup[i], sizeof(int32_t) * ((size_t)m + 1)));
    GC_TRY(dalloc(ps.state[i], (size_t)m + 1));
    GC_TRY(dalloc(ps.list[i], sizeof(int32_t) * ((size_t)m + 1)));
    GC_TRY(dalloc(ps.front[i], sizeof(int32_t) * ((size_t)m + 1)));
  }
  GC_TRY(dalloc(ps.flag, sizeof(int32_t) * ((size_t)m + 1)));
  GC_TRY(dalloc(ps.pos, sizeof(int32_t) * ((size_t)m + 2)));
  GC_TRY(dalloc(ps.misc, 256));
  int32_t *misc = static_cast<int32_t *>(ps.misc.ptr);  // [0] count, [1] min
  int32_t *flag = static_cast<int32_t *>(ps.flag.ptr);
  int32_t *pos = static_cast<int32_t *>(ps.pos.ptr);

  CsrView c = g->csr.view(g->n, m);
  // support of the whole graph, all edges alive
  {
    int32_t *sup = static_cast<int32_t *>(ps.sup[0].ptr);
    GC_HIP(hipMemsetAsync(sup, 0, sizeof(int32_t) * (size_t)m, s));
    if (!g->units_sup_ready) {
      GC_TRY(build_units_support(c, g->units_sup, g->ws, s));
      g->units_sup_ready = true;
    }
    GC_TRY(slot_support(c, g->units_sup, sup, s));
    GC_HIP(hipMemsetAsync(ps.state[0].ptr, EDGE_ALIVE, (size_t)m, s));
  }
  int32_t *list = static_cast<int32_t *>(ps.list[0].ptr);
  int32_t *list2 = static_cast<int32_t *>(ps.list[1].ptr);
  int32_t *front = static_cast<int32_t *>(ps.front[0].ptr);
  int32_t *next = static_cast<int32_t *>(ps.front[1].ptr);
  k_iota<<<gsz(m), 256, 0, s>>>(list, m);
  GC_LAUNCH_CHECK();
  int32_t L = m;
  int next_store = 0;
  int32_t kmax = 2;
  int64_t *stats = g->peel_stats;
  for (int i = 0; i < 37; ++i) stats[i] = 0;
  const int peel_grid = 256 * 8;

  for (;;) {
    int32_t *sup = static_cast<int32_t *>(ps.sup[ps.cur].ptr);
    uint8_t *state = static_cast<uint8_t *>(ps.state[ps.cur].ptr);
    // ---- level start: live edges, their minimum support ----
    k_alive_flags<<<gsz(L), 256, 0, s>>>(list, L, state, flag);
    GC_LAUNCH_CHECK();
    GC_TRY(g->ws.reserve(scan_scratch_bytes((int64_t)L + 1)));
    GC_TRY(exclusive_scan(flag, pos, L, g->ws.take<char>(scan_scratch_bytes((int64_t)L + 1)), s));
    k_set_i32<<<1, 64, 0, s>>>(misc, 0, 0x7fffffff);
    k_compact_list<<<grid_for(L, 256, 2048), 256, 0, s>>>(list, L, flag, pos, sup, list2,
                                                          misc + 1);
    GC_LAUNCH_CHECK();
    int32_t h[2];
    GC_HIP(hipMemcpyAsync(&h[0], pos + L, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GC_HIP(hipMemcpyAsync(&h[1], misc + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GC_HIP(hipStreamSynchronize(s));
    L = h[0];
    if (L == 0) break;
    { int32_t *t = list; list = list2; list2 = t; }
    const int32_t k = h[1] + 3;   // first level that removes something
    const int32_t thr = k - 2;
    // compact the CSR when at least half of it is dead
    if ((int64_t)L * 2 < (int64_t)c.m) {
      GC_TRY(compact_peel(g, ps, c, next_store, front, 0, s));
      sup = static_cast<int32_t *>(ps.sup[ps.cur].ptr);
      state = static_cast<uint8_t *>(ps.state[ps.cur].ptr);
      k_iota<<<gsz(c.m), 256, 0, s>>>(list, c.m);
      GC_LAUNCH_CHECK();
      L = c.m;
    }
    k_collect<<<gsz(L), 256, 0, s>>>(list, L, thr, sup, state, front, misc);
    GC_LAUNCH_CHECK();
    int32_t nfront = 0;
    GC_HIP(hipMemcpyAsync(&nfront, misc, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GC_HIP(hipStreamSynchronize(s));
    int64_t dead_since = 0;
    if (nfront > 0) ++stats[0];
    // ---- rounds of level k ----
    while (nfront > 0) {
      kmax = k - 1 > kmax ? k - 1 : kmax;
      ++stats[1];
      stats[2] += nfront;
      if (nfront > stats[3]) stats[3] = nfront;
      ++stats[5 + (31 - __builtin_clz((unsigned)nfront))];
      k_set_i32<<<1, 64, 0, s>>>(misc, 0, 0);
      unsigned pg = (unsigned)((nfront + 3) / 4);
      if (pg > (unsigned)peel_grid) pg = peel_grid;
      k_peel<<<pg, PBLK, 0, s>>>(c, front, nfront, thr, sup, state, next, misc);
      GC_LAUNCH_CHECK();
      k_advance<<<gsz(nfront), 256, 0, s>>>(front, nfront, next, misc, state, c.eid, tau, k - 1);
      GC_LAUNCH_CHECK();
      int32_t nn = 0;
      GC_HIP(hipMemcpyAsync(&nn, misc, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      GC_HIP(hipStreamSynchronize(s));
      dead_since += nfront;
      { int32_t *t = front; front = next; next = t; }
      nfront = nn;
      if (nfront > 0 && (L - dead_since) * 2 < (int64_t)c.m) {
        GC_TRY(compact_peel(g, ps, c, next_store, front, nfront, s));
        sup = static_cast<int32_t *>(ps.sup[ps.cur].ptr);
        state = static_cast<uint8_t *>(ps.state[ps.cur].ptr);
        k_iota<<<gsz(c.m), 256, 0, s>>>(list, c.m);
        GC_LAUNCH_CHECK();
        L = c.m;
        dead_since = 0;
      }
    }
  }
  GC_HIP(hipStreamSynchronize(s));
  if (h_kmax) *h_kmax = kmax;
  return GC_OK;
}

}  // namespace gc
