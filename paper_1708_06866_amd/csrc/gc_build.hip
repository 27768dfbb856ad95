// gc_build.hip -- gc_build_csr: raw pairs -> canonical edge list -> degree
// ranks -> degree-oriented CSR -> in-edge index, all on the device.
//
// Steps (Sec. II normalisation, then the (L, U) split of Alg. 3 taken in
// degree order):
//   1. key each pair as (min << bits) | max, self-loops get a sentinel key that
//      sorts last; ids outside [0, n) raise a device error flag;
//   2. radix sort the keys (2*bits significant bits);
//   3. keep the first copy of every distinct key (flag + scan + scatter):
//      the canonical edge list u < v in lexicographic order, m edges;
//   4. degrees by atomic increments; rank of each vertex in the strict order
//      (degree, id) by a radix sort of (degree << bits) | id;
//   5. orient every edge from the lower to the higher rank, key it
//      (rank_lo << bits) | rank_hi with its canonical id as payload, and radix
//      sort: the rows of the oriented CSR come out sorted;
//   6. row pointers = exclusive scan of out-degrees;
//   7. in-edge index: a stable sort of the slots by head vertex.
#include <vector>

#include "gc_graph.h"

namespace gc {

constexpr int BLK = 256;

__global__ void k_norm_keys(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                            int64_t P, int32_t n, int32_t shift, int bits, uint64_t invalid,
                            uint64_t *__restrict__ keys, int32_t *__restrict__ err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = (int64_t)src[i] - shift, b = (int64_t)dst[i] - shift;
    uint64_t k;
    if (a < 0 || a >= n || b < 0 || b >= n) {
      atomicOr(err, 1);
      k = invalid;
    } else if (a == b) {
      k = invalid;
    } else {
      const uint64_t lo = (uint64_t)(a < b ? a : b), hi = (uint64_t)(a < b ? b : a);
      k = (lo << bits) | hi;
    }
    keys[i] = k;
  }
}

__global__ void k_unique_flags(const uint64_t *__restrict__ keys, int64_t P, uint64_t invalid,
                               int32_t *__restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    flag[i] = (k != invalid && (i == 0 || keys[i - 1] != k)) ? 1 : 0;
  }
}

__global__ void k_emit_edges(const uint64_t *__restrict__ keys, int64_t P,
                             const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                             int bits, int32_t *__restrict__ u, int32_t *__restrict__ v) {
  const uint64_t mask = (uint64_t(1) << bits) - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (flag[i]) {
      const uint64_t k = keys[i];
      u[pos[i]] = (int32_t)(k >> bits);
      v[pos[i]] = (int32_t)(k & mask);
    }
  }
}

// u is sorted (canonical order): its counts go per run; v takes atomics.
__global__ void k_degrees(const int32_t *__restrict__ u, const int32_t *__restrict__ v, int64_t m,
                          int32_t *__restrict__ deg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t span = (m + stride - 1) / stride * stride;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < span; e += stride) {
    const bool valid = e < m;
    wave_run_count(valid, valid ? u[e] : 0, deg);
    if (valid) atomicAdd(&deg[v[e]], 1);
  }
}

__global__ void k_vertex_keys(const int32_t *__restrict__ deg, int32_t n, int bits,
                              uint64_t *__restrict__ keys) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x)
    keys[x] = ((uint64_t)deg[x] << bits) | (uint64_t)x;
}

__global__ void k_ranks(const uint64_t *__restrict__ sorted, int32_t n, int bits,
                        int32_t *__restrict__ rank, int32_t *__restrict__ vid) {
  const uint64_t mask = (uint64_t(1) << bits) - 1;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = (int32_t)(sorted[r] & mask);
    rank[x] = (int32_t)r;
    vid[r] = x;
  }
}

__global__ void k_orient(const int32_t *__restrict__ u, const int32_t *__restrict__ v, int64_t m,
                         const int32_t *__restrict__ rank, int bits, uint64_t *__restrict__ keys,
                         uint32_t *__restrict__ vals) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t ru = (uint32_t)rank[u[e]], rv = (uint32_t)rank[v[e]];
    const uint64_t lo = ru < rv ? ru : rv, hi = ru < rv ? rv : ru;
    keys[e] = (lo << bits) | hi;
    vals[e] = (uint32_t)e;
  }
}

// Keys are sorted by (src, dst): out-degrees are counted per run of src.
__global__ void k_csr_fill(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                           int64_t m, int bits, int32_t *__restrict__ col,
                           int32_t *__restrict__ src, int32_t *__restrict__ eid,
                           int32_t *__restrict__ outdeg) {
  const uint64_t mask = (uint64_t(1) << bits) - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t span = (m + stride - 1) / stride * stride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < span; i += stride) {
    const bool valid = i < m;
    int32_t s = 0;
    if (valid) {
      const uint64_t k = keys[i];
      s = (int32_t)(k >> bits);
      col[i] = (int32_t)(k & mask);
      src[i] = s;
      eid[i] = (int32_t)vals[i];
    }
    wave_run_count(valid, s, outdeg);
  }
}

__global__ void k_in_keys(const int32_t *__restrict__ col, int64_t m, uint64_t *__restrict__ keys,
                          uint32_t *__restrict__ vals) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m;
       p += (int64_t)gridDim.x * blockDim.x) {
    keys[p] = (uint64_t)(uint32_t)col[p];
    vals[p] = (uint32_t)p;
  }
}

// Sorted by head vertex: in-degrees per run; the tail range of every in-edge.
__global__ void k_in_fill(const uint64_t *__restrict__ heads, const uint32_t *__restrict__ slots,
                          int64_t m, const int32_t *__restrict__ src,
                          const int32_t *__restrict__ row_ptr, int2 *__restrict__ in_tail,
                          int2 *__restrict__ in_edge, int32_t *__restrict__ indeg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t span = (m + stride - 1) / stride * stride;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < span; j += stride) {
    const bool valid = j < m;
    int32_t x = 0;
    if (valid) {
      const int32_t p = (int32_t)slots[j];
      x = (int32_t)heads[j];
      const int32_t a = src[p];
      in_edge[j] = make_int2(a, p);
      in_tail[j] = make_int2(p + 1, row_ptr[a + 1]);
    }
    wave_run_count(valid, x, indeg);
  }
}

static unsigned gsz(int64_t work) { return grid_for(work, BLK, 65536); }

// In-edge index of an oriented CSR whose row_ptr/col/src are set.
gc_status build_in_lists(int32_t n, int32_t m, int bits, CsrStore &c, Workspace &ws,
                         hipStream_t s) {
  GC_TRY(dalloc(c.in_ptr, sizeof(int32_t) * ((size_t)n + 1)));
  GC_TRY(dalloc(c.in_tail, sizeof(int2) * ((size_t)m + 1)));
  GC_TRY(dalloc(c.in_edge, sizeof(int2) * ((size_t)m + 1)));
  int32_t *in_ptr = static_cast<int32_t *>(c.in_ptr.ptr);
  GC_HIP(hipMemsetAsync(in_ptr, 0, sizeof(int32_t) * ((size_t)n + 1), s));
  if (m == 0) return GC_OK;
  const size_t need = 2 * abytes<uint64_t>(m) + 2 * abytes<uint32_t>(m) +
                      sort_scratch_bytes(m) + scan_scratch_bytes(n) + 1024;
  GC_TRY(ws.reserve(need));
  uint64_t *ka = ws.take<uint64_t>(m), *kb = ws.take<uint64_t>(m);
  uint32_t *va = ws.take<uint32_t>(m), *vb = ws.take<uint32_t>(m);
  void *sscr = ws.take<char>(sort_scratch_bytes(m));
  void *cscr = ws.take<char>(scan_scratch_bytes(n));
  const int32_t *col = static_cast<const int32_t *>(c.col.ptr);
  k_in_keys<<<gsz(m), BLK, 0, s>>>(col, m, ka, va);
  GC_LAUNCH_CHECK();
  uint64_t *ks;
  uint32_t *vs;
  GC_TRY(radix_sort(ka, kb, va, vb, m, bits, sscr, s, &ks, &vs));
  k_in_fill<<<gsz(m), BLK, 0, s>>>(ks, vs, m, static_cast<const int32_t *>(c.src.ptr),
                                   static_cast<const int32_t *>(c.row_ptr.ptr),
                                   static_cast<int2 *>(c.in_tail.ptr),
                                   static_cast<int2 *>(c.in_edge.ptr), in_ptr);
  GC_LAUNCH_CHECK();
  GC_TRY(exclusive_scan(in_ptr, in_ptr, n, cscr, s));
  return GC_OK;
}

static gc_status build_impl(const int32_t *d_src, const int32_t *d_dst, int64_t P, int32_t n,
                            uint32_t flags, hipStream_t s, gc_graph *g) {
  const int bits = ceil_log2_u64((uint64_t)(n > 1 ? n : 2));
  g->bits = bits;
  const int keybits = 2 * bits;
  const uint64_t invalid = (keybits >= 64) ? ~0ull : ((uint64_t(1) << keybits) - 1);
  const int shift = (flags & GC_INPUT_ONE_BASED) ? 1 : 0;

  GC_TRY(dalloc(g->rank, sizeof(int32_t) * ((size_t)n + 1)));
  GC_TRY(dalloc(g->vid, sizeof(int32_t) * ((size_t)n + 1)));
  GC_TRY(dalloc(g->csr.row_ptr, sizeof(int32_t) * ((size_t)n + 1)));

  // ---- workspace for the build (released at the end) ----
  const int64_t big = P > n ? P : n;
  Workspace tmp;
  const size_t need = 2 * abytes<uint64_t>(big + 1) + 2 * abytes<uint32_t>(big + 1) +
                      abytes<int32_t>(big + 1) * 2 + sort_scratch_bytes(big) +
                      scan_scratch_bytes(big + 1) + abytes<int32_t>(n + 1) + 4096;
  GC_TRY(tmp.reserve(need));
  uint64_t *ka = tmp.take<uint64_t>(big + 1), *kb = tmp.take<uint64_t>(big + 1);
  uint32_t *va = tmp.take<uint32_t>(big + 1), *vb = tmp.take<uint32_t>(big + 1);
  int32_t *flag = tmp.take<int32_t>(big + 1), *pos = tmp.take<int32_t>(big + 1);
  void *sscr = tmp.take<char>(sort_scratch_bytes(big));
  void *cscr = tmp.take<char>(scan_scratch_bytes(big + 1));
  int32_t *deg = tmp.take<int32_t>(n + 1);
  int32_t *err = tmp.take<int32_t>(64);
  int32_t *dm = err + 1;  // device copy of m

  GC_HIP(hipMemsetAsync(err, 0, 2 * sizeof(int32_t), s));
  int64_t m = 0;
  if (P > 0) {
    k_norm_keys<<<gsz(P), BLK, 0, s>>>(d_src, d_dst, P, n, shift, bits, invalid, ka, err);
    GC_LAUNCH_CHECK();
    uint64_t *ks;
    GC_TRY(radix_sort(ka, kb, nullptr, nullptr, P, keybits, sscr, s, &ks, nullptr));
    k_unique_flags<<<gsz(P), BLK, 0, s>>>(ks, P, invalid, flag);
    GC_LAUNCH_CHECK();
    GC_TRY(exclusive_scan(flag, pos, P, cscr, s));
    GC_HIP(hipMemcpyAsync(dm, pos + P, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    int32_t h[2] = {0, 0};
    GC_HIP(hipMemcpyAsync(h, err, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GC_HIP(hipStreamSynchronize(s));
    if (h[0]) {
      set_error("gc_build_csr: vertex id outside [0, n_vertices)");
      return GC_ERANGE;
    }
    m = h[1];
    GC_TRY(dalloc(g->u, sizeof(int32_t) * ((size_t)m + 1)));
    GC_TRY(dalloc(g->v, sizeof(int32_t) * ((size_t)m + 1)));
    k_emit_edges<<<gsz(P), BLK, 0, s>>>(ks, P, flag, pos, bits,
                                        static_cast<int32_t *>(g->u.ptr),
                                        static_cast<int32_t *>(g->v.ptr));
    GC_LAUNCH_CHECK();
  } else {
    GC_TRY(dalloc(g->u, sizeof(int32_t)));
    GC_TRY(dalloc(g->v, sizeof(int32_t)));
  }
  g->m = m;
  const int32_t *u = static_cast<const int32_t *>(g->u.ptr);
  const int32_t *v = static_cast<const int32_t *>(g->v.ptr);

  // ---- degrees and ranks ----
  int32_t *rank = static_cast<int32_t *>(g->rank.ptr);
  if (n > 0) {
    GC_HIP(hipMemsetAsync(deg, 0, sizeof(int32_t) * (size_t)n, s));
    if (m > 0) {
      k_degrees<<<gsz(m), BLK, 0, s>>>(u, v, m, deg);
      GC_LAUNCH_CHECK();
    }
    k_vertex_keys<<<gsz(n), BLK, 0, s>>>(deg, n, bits, ka);
    GC_LAUNCH_CHECK();
    uint64_t *ks;
    GC_TRY(radix_sort(ka, kb, nullptr, nullptr, n, keybits, sscr, s, &ks, nullptr));
    k_ranks<<<gsz(n), BLK, 0, s>>>(ks, n, bits, rank, static_cast<int32_t *>(g->vid.ptr));
    GC_LAUNCH_CHECK();
  }

  // ---- oriented CSR ----
  CsrStore &c = g->csr;
  GC_TRY(dalloc(c.col, sizeof(int32_t) * ((size_t)m + 1)));
  GC_TRY(dalloc(c.src, sizeof(int32_t) * ((size_t)m + 1)));
  GC_TRY(dalloc(c.eid, sizeof(int32_t) * ((size_t)m + 1)));
  int32_t *row_ptr = static_cast<int32_t *>(c.row_ptr.ptr);
  GC_HIP(hipMemsetAsync(row_ptr, 0, sizeof(int32_t) * ((size_t)n + 1), s));
  if (m > 0) {
    k_orient<<<gsz(m), BLK, 0, s>>>(u, v, m, rank, bits, ka, va);
    GC_LAUNCH_CHECK();
    uint64_t *ks;
    uint32_t *vs;
    GC_TRY(radix_sort(ka, kb, va, vb, m, keybits, sscr, s, &ks, &vs));
    k_csr_fill<<<gsz(m), BLK, 0, s>>>(ks, vs, m, bits, static_cast<int32_t *>(c.col.ptr),
                                      static_cast<int32_t *>(c.src.ptr),
                                      static_cast<int32_t *>(c.eid.ptr), row_ptr);
    GC_LAUNCH_CHECK();
  }
  GC_TRY(exclusive_scan(row_ptr, row_ptr, n, cscr, s));
  GC_HIP(hipStreamSynchronize(s));
  GC_TRY(build_in_lists(n, (int32_t)m, bits, c, g->ws, s));
  GC_HIP(hipStreamSynchronize(s));
  return GC_OK;
}

}  // namespace gc

extern "C" gc_status gc_build_csr(const int32_t *d_src, const int32_t *d_dst, int64_t n_pairs,
                                  int32_t n_vertices, uint32_t flags, gc_stream stream,
                                  gc_graph **out) {
  gc::clear_error();
  if (!out) {
    gc::set_error("gc_build_csr: out is NULL");
    return GC_EINVAL;
  }
  *out = nullptr;
  if (n_pairs < 0 || n_vertices < 0 || (flags & ~GC_INPUT_ONE_BASED) != 0 ||
      (n_pairs > 0 && (!d_src || !d_dst))) {
    gc::set_error("gc_build_csr: invalid argument");
    return GC_EINVAL;
  }
  if (n_pairs >= (int64_t)INT32_MAX - 8) {
    gc::set_error("gc_build_csr: n_pairs must be < 2^31");
    return GC_EOVERFLOW;
  }
  if (n_pairs > 0 && n_vertices == 0) {
    gc::set_error("gc_build_csr: vertex id outside [0, n_vertices)");
    return GC_ERANGE;
  }
  gc_graph *g = new (std::nothrow) gc_graph();
  if (!g) {
    gc::set_error("gc_build_csr: host allocation of the handle failed");
    return GC_ENOMEM;
  }
  g->n = n_vertices;
  hipError_t e = hipGetDevice(&g->device);
  if (e != hipSuccess) {
    gc::set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    delete g;
    return GC_EDEVICE;
  }
  gc::load_strategy_cache(g->device, g->strategy, g->tile);
  gc_status st = gc::build_impl(d_src, d_dst, n_pairs, n_vertices, flags,
                                static_cast<hipStream_t>(stream), g);
  // The support kernels' work units belong to the handle from the start, so
  // support (and the allocation-free gc_edge_support_noalloc) needs no
  // device allocation later.
  if (st == GC_OK && g->m > 0) {
    st = gc::build_units_support(g->csr.view(g->n, (int32_t)g->m), g->units_sup, g->ws,
                                 static_cast<hipStream_t>(stream));
    if (st == GC_OK) g->units_sup_ready = true;
  }
  if (st != GC_OK) {
    gc_graph_free(g);
    return st;
  }
  *out = g;
  return GC_OK;
}
