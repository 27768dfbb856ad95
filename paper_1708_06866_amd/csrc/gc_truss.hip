// gc_truss.hip -- k-truss and truss decomposition by rounds (Sec. III-B,
// Alg. 4): recompute the support of every remaining edge, drop every edge whose
// support is below k-2, compact the edge list by a prefix scan, repeat until
// no edge is dropped.
//
// The oriented CSR keeps its orientation while it shrinks (any strict order
// counts each triangle once), so compaction only filters each row in place:
// new slot = exclusive scan of the keep flags, new row_ptr[r] = scan value at
// the old row start, and the in-edge index is rebuilt for the new slots.
//
// Decomposition runs the rounds with k = 3, 4, ... on the surviving edges
// (the paper passes the k-truss on to k+1).  When a level ends with no
// removal, the support of the remaining edges is already known, so instead of
// a recount the next level starts from min-support + 3: every level in between
// removes nothing.  An edge dropped while working on level k has truss number
// k - 1.
#include <stdlib.h>
#include <string.h>

#include "gc_graph.h"

namespace gc {

__global__ void k_keep_flags(const int32_t *__restrict__ sup, int32_t m, int32_t thr,
                             int32_t *__restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    flag[i] = sup[i] >= thr ? 1 : 0;
}

__global__ void k_compact(const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                          int32_t m, const int32_t *__restrict__ col,
                          const int32_t *__restrict__ src, const int32_t *__restrict__ eid,
                          int32_t *__restrict__ ncol, int32_t *__restrict__ nsrc,
                          int32_t *__restrict__ neid, int32_t *__restrict__ tau, int32_t tau_dropped) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (flag[i]) {
      const int32_t p = pos[i];
      ncol[p] = col[i];
      nsrc[p] = src[i];
      neid[p] = eid[i];
    } else if (tau) {
      tau[eid[i]] = tau_dropped;
    }
  }
}

__global__ void k_rows(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ pos,
                       int32_t n, int32_t *__restrict__ nrow) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n;
       r += (int64_t)gridDim.x * blockDim.x)
    nrow[r] = pos[row_ptr[r]];
}

__global__ void k_min_i32(const int32_t *__restrict__ x, int32_t m, int32_t *__restrict__ out) {
  int32_t v = 0x7fffffff;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    v = min(v, x[i]);
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMin(out, v);
}

__global__ void k_mask_alive(const int32_t *__restrict__ eid, int32_t m, uint8_t *__restrict__ mask) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    mask[eid[i]] = 1;
}

__global__ void k_fill_i32(int32_t *__restrict__ x, int64_t m, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

static unsigned gsz(int64_t work) { return grid_for(work, 256, 65536); }

// Support of every slot of `c` into sup (zeroed here).
static gc_status round_support(gc_graph *g, const CsrView &c, int32_t *sup, hipStream_t s) {
  GC_HIP(hipMemsetAsync(sup, 0, sizeof(int32_t) * (size_t)c.m, s));
  if (c.m == 0) return GC_OK;
  const bool base = c.col == static_cast<const int32_t *>(g->csr.col.ptr);
  if (base) {
    if (!g->units_sup_ready) {
      GC_TRY(build_units_support(c, g->units_sup, g->ws, s));
      g->units_sup_ready = true;
    }
    return slot_support(c, g->units_sup, sup, s);
  }
  GC_TRY(build_units_support(c, g->work_units, g->ws, s));
  return slot_support(c, g->work_units, sup, s);
}

// Drop every slot with sup < thr.  Returns the new view (in work[next]) and
// writes `tau_dropped` into tau[eid] of dropped edges if tau != null.
static gc_status drop_and_compact(gc_graph *g, const CsrView &c, const int32_t *sup, int32_t thr,
                                  int32_t *tau, int32_t tau_dropped, int &next, CsrView &out,
                                  int32_t &kept, hipStream_t s) {
  const int32_t m = c.m, n = c.n;
  int32_t *flag = static_cast<int32_t *>(g->t_flag.ptr);
  int32_t *pos = static_cast<int32_t *>(g->t_pos.ptr);
  k_keep_flags<<<gsz(m), 256, 0, s>>>(sup, m, thr, flag);
  GC_LAUNCH_CHECK();
  GC_TRY(g->ws.reserve(scan_scratch_bytes((int64_t)m + 1)));
  GC_TRY(exclusive_scan(flag, pos, m, g->ws.take<char>(scan_scratch_bytes((int64_t)m + 1)), s));
  int32_t h = 0;
  GC_HIP(hipMemcpyAsync(&h, pos + m, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  GC_HIP(hipStreamSynchronize(s));
  kept = h;
  if (kept == m) {
    out = c;
    return GC_OK;
  }
  CsrStore &w = g->work[next];
  GC_TRY(dalloc(w.row_ptr, sizeof(int32_t) * ((size_t)n + 1)));
  GC_TRY(dalloc(w.col, sizeof(int32_t) * ((size_t)kept + 1)));
  GC_TRY(dalloc(w.src, sizeof(int32_t) * ((size_t)kept + 1)));
  GC_TRY(dalloc(w.eid, sizeof(int32_t) * ((size_t)kept + 1)));
  k_compact<<<gsz(m), 256, 0, s>>>(flag, pos, m, c.col, c.src, c.eid,
                                   static_cast<int32_t *>(w.col.ptr),
                                   static_cast<int32_t *>(w.src.ptr),
                                   static_cast<int32_t *>(w.eid.ptr), tau, tau_dropped);
  GC_LAUNCH_CHECK();
  k_rows<<<gsz((int64_t)n + 1), 256, 0, s>>>(c.row_ptr, pos, n,
                                             static_cast<int32_t *>(w.row_ptr.ptr));
  GC_LAUNCH_CHECK();
  GC_TRY(build_in_lists(n, kept, g->bits, w, g->ws, s));
  out = w.view(n, kept);
  next ^= 1;
  return GC_OK;
}

static gc_status truss_state_alloc(gc_graph *g) {
  const size_t m = (size_t)g->m;
  GC_TRY(dalloc(g->t_sup, sizeof(int32_t) * (m + 1)));
  GC_TRY(dalloc(g->t_flag, sizeof(int32_t) * (m + 1)));
  GC_TRY(dalloc(g->t_pos, sizeof(int32_t) * (m + 2)));
  GC_TRY(dalloc(g->t_misc, 256));
  return GC_OK;
}

static gc_status ktruss_impl(gc_graph *g, int32_t k, uint8_t *mask, int64_t *h_mk,
                             hipStream_t s) {
  const int32_t m = (int32_t)g->m;
  if (m > 0) GC_HIP(hipMemsetAsync(mask, 0, (size_t)m, s));
  CsrView c = g->csr.view(g->n, m);
  if (m > 0 && k > 2) {
    GC_TRY(truss_state_alloc(g));
    int32_t *sup = static_cast<int32_t *>(g->t_sup.ptr);
    int next = 0;
    for (;;) {
      GC_TRY(round_support(g, c, sup, s));
      CsrView nc;
      int32_t kept = 0;
      GC_TRY(drop_and_compact(g, c, sup, k - 2, nullptr, 0, next, nc, kept, s));
      if (kept == c.m) break;
      c = nc;
      if (kept == 0) break;
    }
  }
  if (c.m > 0) {
    k_mask_alive<<<gsz(c.m), 256, 0, s>>>(c.eid, c.m, mask);
    GC_LAUNCH_CHECK();
  }
  GC_HIP(hipStreamSynchronize(s));
  if (h_mk) *h_mk = c.m;
  return GC_OK;
}

static gc_status decomposition_impl(gc_graph *g, int32_t *truss, int32_t *h_kmax, hipStream_t s) {
  const int32_t m = (int32_t)g->m;
  if (m == 0) {
    if (h_kmax) *h_kmax = 0;
    return GC_OK;
  }
  GC_TRY(truss_state_alloc(g));
  int32_t *tau = truss;
  struct Owned {  // truss numbers when the caller passes none, freed on every return
    DeviceBuffer b;
    ~Owned() { dfree(b); }
  } own;
  if (!tau) {
    GC_TRY(dalloc(own.b, sizeof(int32_t) * (size_t)m));
    tau = static_cast<int32_t *>(own.b.ptr);
  }
  k_fill_i32<<<gsz(m), 256, 0, s>>>(tau, m, 2);
  GC_LAUNCH_CHECK();
  int32_t *sup = static_cast<int32_t *>(g->t_sup.ptr);
  int32_t *dmin = static_cast<int32_t *>(g->t_misc.ptr);
  CsrView c = g->csr.view(g->n, m);
  int next = 0;
  int32_t k = 3;
  GC_TRY(round_support(g, c, sup, s));
  gc_status st = GC_OK;
  for (;;) {
    CsrView nc;
    int32_t kept = 0;
    st = drop_and_compact(g, c, sup, k - 2, tau, k - 1, next, nc, kept, s);
    if (st != GC_OK) break;
    if (kept == 0) break;            // level k emptied the graph: kmax = k - 1
    if (kept == c.m) {
      // no removal at level k: every remaining edge has support >= min, so
      // levels k .. min+2 keep them all; continue at min + 3
      k_fill_i32<<<1, 64, 0, s>>>(dmin, 1, 0x7fffffff);
      k_min_i32<<<grid_for(c.m, 256, 2048), 256, 0, s>>>(sup, c.m, dmin);
      int32_t hmin = 0;
      if (hipMemcpyAsync(&hmin, dmin, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        set_error("decomposition: min support readback failed");
        st = GC_EDEVICE;
        break;
      }
      k = (hmin + 3 > k + 1) ? hmin + 3 : k + 1;
      continue;
    }
    c = nc;
    st = round_support(g, c, sup, s);
    if (st != GC_OK) break;
  }
  if (st == GC_OK) {
    if (hipStreamSynchronize(s) != hipSuccess) st = GC_EDEVICE;
    if (h_kmax) *h_kmax = k - 1;
  }
  return st;
}

}  // namespace gc

using namespace gc;

extern "C" gc_status gc_ktruss(gc_graph *g, int32_t k, uint8_t *d_in_truss, int64_t cap,
                               gc_stream stream, int64_t *h_m_k) {
  clear_error();
  if (!g || k < 2 || (g->m > 0 && !d_in_truss)) {
    set_error("gc_ktruss: invalid argument");
    return GC_EINVAL;
  }
  if (cap < g->m) {
    set_error("gc_ktruss: cap < m");
    return GC_ECAPACITY;
  }
  int prev = 0;
  GC_HIP(hipGetDevice(&prev));
  if (prev != g->device) GC_HIP(hipSetDevice(g->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  gc_status st;
  const char *method = getenv("GC_TRUSS_METHOD");
  if (k <= 2 || (method && strcmp(method, "rounds") == 0)) {
    st = ktruss_impl(g, k, d_in_truss, h_m_k, s);
  } else {
    // the k-truss is what survives the peeling levels 3 .. k
    st = decomposition_peel(g, nullptr, nullptr, s, k, d_in_truss, h_m_k);
    if (st == GC_OK && hipStreamSynchronize(s) != hipSuccess) {
      set_error("gc_ktruss: stream synchronize failed");
      st = GC_EDEVICE;
    }
  }
  if (prev != g->device) (void)hipSetDevice(prev);
  return st;
}

extern "C" gc_status gc_truss_decomposition(gc_graph *g, int32_t *d_truss, int64_t cap,
                                            gc_stream stream, int32_t *h_kmax) {
  clear_error();
  if (!g) {
    set_error("gc_truss_decomposition: NULL handle");
    return GC_EINVAL;
  }
  if (d_truss && cap < g->m) {
    set_error("gc_truss_decomposition: cap < m");
    return GC_ECAPACITY;
  }
  int prev = 0;
  GC_HIP(hipGetDevice(&prev));
  if (prev != g->device) GC_HIP(hipSetDevice(g->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  gc_status st;
  const char *method = getenv("GC_TRUSS_METHOD");
  if (method && strcmp(method, "rounds") == 0) {
    st = decomposition_impl(g, d_truss, h_kmax, s);
  } else {
    DeviceBuffer own;
    int32_t *tau = d_truss;
    st = GC_OK;
    if (!tau && g->m > 0) {
      st = dalloc(own, sizeof(int32_t) * (size_t)g->m);
      tau = static_cast<int32_t *>(own.ptr);
    }
    if (st == GC_OK) st = decomposition_peel(g, tau, h_kmax, s);
    dfree(own);
  }
  if (prev != g->device) (void)hipSetDevice(prev);
  return st;
}
