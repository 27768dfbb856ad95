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
//   * the triangles {a, b, x} of each frontier edge p = (a -> b) still present
//     are enumerated in three cases by the rank of x, each intersecting a
//     sorted list of a with one of b (the shorter iterated, each entry
//     binary-searched in the other); large frontiers go in lane-balanced
//     batches of up to 64 edges per wave, small ones give each edge whole
//     waves (see k_peel);
//   * a triangle is skipped if one of its edges died in an earlier round, or
//     if another frontier edge of it has a smaller slot id (so each destroyed
//     triangle is subtracted exactly once, whichever edges die together);
//     otherwise each surviving edge loses one, and an edge whose support
//     drops from t to t - 1 joins the next frontier (once);
//   * the frontier edges die with truss number k - 1.
// A level ends when the frontier is empty.  The next level is min-support + 3
// (every level in between removes nothing); one tiled pass over the slots
// finds the minimum and collects the level's first frontier.  When a quarter
// of the oriented CSR is dead it is compacted by a scan, carrying support and
// state, and its in-lists are filtered in place.
//
// Results equal the rounds of Alg. 4 (bulk removal per round, same frontier
// sets); only the work per round differs.
#include "gc_graph.h"

namespace gc {

enum : uint8_t { EDGE_ALIVE = 0, EDGE_FRONT = 1, EDGE_DEAD = 2 };

constexpr int PBLK = 256;

constexpr int PEEL_U = 4;  // candidates per lane in flight
// waves of a peel launch: 56 per CU on the 256 CUs of an MI355X
constexpr int64_t kPeelWaves = 256 * 56;

// Triangles {p[u], q1[u], q2[u]} seen from frontier edges p[u] (found[u]
// false: no triangle), the PEEL_U of a lane at once: their state loads, then
// their support decrements, are issued together, and the next-frontier
// appends of the whole wave take one atomic.  Every lane of the wave calls
// this.  r[u] bit 0: the triangle is still present (no edge of it died in an
// earlier round); bit 1: this call destroyed it (p[u] is its smallest frontier
// edge), and each surviving edge of it lost one; an edge whose support drops
// from thr to thr - 1 joins the next frontier (once).
__device__ __forceinline__ void destroy_many(const bool (&found)[PEEL_U],
                                             const int32_t (&p)[PEEL_U],
                                             const int32_t (&q1)[PEEL_U],
                                             const int32_t (&q2)[PEEL_U], int32_t thr,
                                             const uint8_t *__restrict__ state,
                                             int32_t *__restrict__ sup,
                                             int32_t *__restrict__ next,
                                             int32_t *__restrict__ next_count,
                                             int (&r)[PEEL_U]) {
  uint8_t s1[PEEL_U], s2[PEEL_U];
#pragma unroll
  for (int u = 0; u < PEEL_U; ++u) {
    s1[u] = s2[u] = EDGE_DEAD;
    if (found[u]) {
      s1[u] = state[q1[u]];
      s2[u] = state[q2[u]];
    }
  }
  int32_t o1[PEEL_U], o2[PEEL_U];
#pragma unroll
  for (int u = 0; u < PEEL_U; ++u) {
    const bool present = s1[u] != EDGE_DEAD && s2[u] != EDGE_DEAD;
    const bool ours = present && !(s1[u] == EDGE_FRONT && q1[u] < p[u]) &&
                      !(s2[u] == EDGE_FRONT && q2[u] < p[u]);
    r[u] = (present ? 1 : 0) | (ours ? 2 : 0);
    o1[u] = o2[u] = 0;
    if (ours && s1[u] == EDGE_ALIVE) o1[u] = atomicSub(&sup[q1[u]], 1);
    if (ours && s2[u] == EDGE_ALIVE) o2[u] = atomicSub(&sup[q2[u]], 1);
  }
  // an edge whose support drops from thr to thr - 1 joins the next frontier
  int32_t cnt = 0;
  bool t1[PEEL_U], t2[PEEL_U];
#pragma unroll
  for (int u = 0; u < PEEL_U; ++u) {
    t1[u] = (r[u] & 2) && s1[u] == EDGE_ALIVE && o1[u] == thr;
    t2[u] = (r[u] & 2) && s2[u] == EDGE_ALIVE && o2[u] == thr;
    cnt += (t1[u] ? 1 : 0) + (t2[u] ? 1 : 0);
  }
  if (__ballot(cnt > 0) == 0) return;
  const int32_t incl = wave_inclusive_scan(cnt);
  int32_t at = 0;
  if (__lane_id() == 63) at = atomicAdd(next_count, incl);
  at = __shfl(at, 63, 64) + incl - cnt;
#pragma unroll
  for (int u = 0; u < PEEL_U; ++u) {
    if (t1[u]) next[at++] = q1[u];
    if (t2[u]) next[at++] = q2[u];
  }
}

// Keys of the two list layouts: a row holds the neighbour (its slot is the
// position), an in-list entry holds {neighbour, slot}.
__device__ __forceinline__ int32_t key_of(int32_t e) { return e; }
__device__ __forceinline__ int32_t key_of(int2 e) { return e.x; }
__device__ __forceinline__ int32_t slot_of(int32_t, int32_t pos) { return pos; }
__device__ __forceinline__ int32_t slot_of(int2 e, int32_t) { return e.y; }

// Searches of PEEL_U keys in one sorted list arr[lo, hi), run in lockstep so
// their loads overlap; out[u] = slot of the edge holding key[u], or -1 (also
// -1 where act[u] is false, which loads nothing).
template <class T>
__device__ __forceinline__ void find_many(const T *__restrict__ arr, int32_t lo, int32_t hi,
                                          const int32_t (&key)[PEEL_U], const bool (&act)[PEEL_U],
                                          int32_t (&out)[PEEL_U]) {
  int32_t l[PEEL_U], n[PEEL_U];
#pragma unroll
  for (int u = 0; u < PEEL_U; ++u) { l[u] = lo; n[u] = act[u] ? hi - lo : 0; }
  for (;;) {
    bool any = false;
    int32_t v[PEEL_U];
#pragma unroll
    for (int u = 0; u < PEEL_U; ++u) v[u] = n[u] > 0 ? key_of(arr[l[u] + (n[u] >> 1)]) : 0;
#pragma unroll
    for (int u = 0; u < PEEL_U; ++u) {
      if (n[u] > 0) {
        const int32_t half = n[u] >> 1;
        if (v[u] < key[u]) { l[u] += half + 1; n[u] -= half + 1; } else { n[u] = half; }
        any |= n[u] > 0;
      }
    }
    if (!any) break;
  }
#pragma unroll
  for (int u = 0; u < PEEL_U; ++u) {
    out[u] = -1;
    if (act[u] && l[u] < hi) {
      const T e = arr[l[u]];
      if (key_of(e) == key[u]) out[u] = slot_of(e, l[u]);
    }
  }
}

template <class T>
__device__ __forceinline__ int32_t lower_bound_key(const T *__restrict__ a, int32_t lo, int32_t hi,
                                                   int32_t key) {
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (key_of(a[mid]) < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// The lists around frontier edge p = (a -> b): rows and in-lists of a and b,
// and the position of a in b's in-list.
struct PeelEdge {
  int32_t ra0, ra1, rb0, rb1, ia0, ia1, ib0, ib1, ibA;
};

__device__ __forceinline__ PeelEdge peel_edge(const CsrView &c, int32_t a, int32_t b) {
  PeelEdge e;
  e.ra0 = c.row_ptr[a]; e.ra1 = c.row_ptr[a + 1];
  e.rb0 = c.row_ptr[b]; e.rb1 = c.row_ptr[b + 1];
  e.ia0 = c.in_ptr[a]; e.ia1 = c.in_ptr[a + 1];
  e.ib0 = c.in_ptr[b]; e.ib1 = c.in_ptr[b + 1];
  e.ibA = lower_bound_key(c.in_edge, e.ib0, e.ib1, a);  // in_edge[ibA] = {a, p}
  return e;
}

// One of the three intersections (see k_peel): iterate A[A0, A0 + nA), search
// B[B0, B0 + nB); nA = 0 when either side is empty.  flags: bit 0 A is an
// in-list, bit 1 B is an in-list (entries {neighbour, slot} of in_edge; else a
// stretch of col, slot = position).
struct PeelCase {
  int32_t A0, nA, B0, nB;
  uint32_t flags;
};

__device__ __forceinline__ PeelCase peel_case(const PeelEdge &e, int32_t p, int cs) {
  int32_t A0, A1, B0, B1;
  bool A_in, B_in;
  if (cs == 0) { A0 = p + 1; A1 = e.ra1; A_in = false; B0 = e.rb0; B1 = e.rb1; B_in = false; }
  else if (cs == 1) { A0 = e.ra0; A1 = p; A_in = false; B0 = e.ibA + 1; B1 = e.ib1; B_in = true; }
  else { A0 = e.ia0; A1 = e.ia1; A_in = true; B0 = e.ib0; B1 = e.ibA; B_in = true; }
  if (A1 - A0 > B1 - B0) {  // iterate the shorter side
    int32_t t;
    t = A0; A0 = B0; B0 = t;
    t = A1; A1 = B1; B1 = t;
    const bool tb = A_in; A_in = B_in; B_in = tb;
  }
  PeelCase pc;
  pc.A0 = A0;
  pc.B0 = B0;
  pc.nB = B1 - B0;
  pc.nA = (A1 - A0 > 0 && B1 - B0 > 0) ? A1 - A0 : 0;
  pc.flags = (A_in ? 1u : 0u) | (B_in ? 2u : 0u);
  return pc;
}

// Lane-balanced batches (large frontiers): a wave takes up to 64 frontier
// edges at once, lays their candidates end to end (edge by edge, case by case)
// and gives each lane the next candidate of that concatenation, so a batch of
// short lists keeps every lane busy.  The batch lives in LDS, one per wave.
struct PeelBatch {
  long long off[64];  // first candidate of edge e in the concatenation
  int32_t p[64], need[64], seen[64];
  int32_t A0[3][64], B0[3][64], B1[3][64];
  int32_t cum[2][64];  // candidates of case 0, of cases 0 and 1
  uint32_t flags[64];  // bit 2cs: A of case cs is an in-list; bit 2cs + 1: B is
};

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Edge of the batch holding candidate t for t that only grows from one call
// to the next: stepped on from the last one.
struct BatchCursor {
  int e;
  long long next;
  __device__ __forceinline__ void init(const PeelBatch &B) { e = 0; next = B.off[1]; }
  __device__ __forceinline__ int edge(const PeelBatch &B, long long t) {
    while (t >= next) {
      ++e;
      next = e < 63 ? B.off[e + 1] : 0x7fffffffffffffffLL;
    }
    return e;
  }
};

// Edge of the batch holding candidate t (the last e with off[e] <= t).
__device__ __forceinline__ int batch_edge(const PeelBatch &B, long long t) {
  int e = 0;
#pragma unroll
  for (int s = 32; s > 0; s >>= 1)
    if (B.off[e + s] <= t) e += s;
  return e;
}

// Key of entry i of a sorted list: a stretch of col (stride 4 bytes) or of
// in_edge (stride 8 bytes, key first).
__device__ __forceinline__ int32_t list_key(const char *base, uint32_t sh, int32_t i) {
  return *reinterpret_cast<const int32_t *>(base + ((uint64_t)(uint32_t)i << sh));
}

// find_many with a list per search: key[u] in col (bin[u] false) or in_edge
// (bin[u] true) over [lo[u], hi[u]); out[u] = slot of the matching edge, or
// -1.
__device__ __forceinline__ void find_many_lists(const CsrView &c, const bool (&bin)[PEEL_U],
                                                const int32_t (&lo)[PEEL_U],
                                                const int32_t (&hi)[PEEL_U],
                                                const int32_t (&key)[PEEL_U],
                                                const bool (&act)[PEEL_U],
                                                int32_t (&out)[PEEL_U]) {
  const char *colp = reinterpret_cast<const char *>(c.col);
  const char *inp = reinterpret_cast<const char *>(c.in_edge);
  int32_t l[PEEL_U], n[PEEL_U];
#pragma unroll
  for (int u = 0; u < PEEL_U; ++u) { l[u] = lo[u]; n[u] = act[u] ? hi[u] - lo[u] : 0; }
  for (;;) {
    bool any = false;
    int32_t v[PEEL_U];
#pragma unroll
    for (int u = 0; u < PEEL_U; ++u)
      v[u] = n[u] > 0 ? list_key(bin[u] ? inp : colp, bin[u] ? 3 : 2, l[u] + (n[u] >> 1)) : 0;
#pragma unroll
    for (int u = 0; u < PEEL_U; ++u) {
      if (n[u] > 0) {
        const int32_t half = n[u] >> 1;
        if (v[u] < key[u]) { l[u] += half + 1; n[u] -= half + 1; } else { n[u] = half; }
        any |= n[u] > 0;
      }
    }
    if (!any) break;
  }
#pragma unroll
  for (int u = 0; u < PEEL_U; ++u) {
    out[u] = -1;
    if (act[u] && l[u] < hi[u]) {
      if (bin[u]) {
        const int2 ie = c.in_edge[l[u]];
        if (ie.x == key[u]) out[u] = ie.y;
      } else if (c.col[l[u]] == key[u]) {
        out[u] = l[u];
      }
    }
  }
}

// One round of level k over the frontier front[0, *front_count); the size is
// read here, so rounds can be queued without the host knowing it.  `wpe`
// waves share each frontier edge p = (a -> b).
// Its triangles {a, b, x} split by the rank of x, and each case intersects two
// sorted lists, iterating the shorter (A) and searching the longer (B):
//   x > b      tail of a's row after p (a -> x)   vs  b's row (b -> x)
//   a < x < b  head of a's row before p (a -> x)  vs  b's in-list, sources in (a, b)
//   x < a      a's in-list (x -> a)               vs  b's in-list, sources < a
// Each lane takes PEEL_U candidates of A per step (stride 64 * wpe), searched
// in lockstep.  When a round starts, the support of a frontier edge equals the
// number of its triangles still present (every earlier destruction of one of
// them decremented it while the edge was alive), so an edge with support 0 is
// skipped and a wave that scans an edge alone stops after that many.  The
// cases go by falling rank of x and each A is walked from its end (highest
// rank first): in a degree order the high ranks are the hubs, which close
// most triangles, so the edge's triangles are met early and the scan stops
// sooner (R-MAT scale 24: 54.4 G candidates instead of 57.8 G).
// `work` (optional) holds 4 counters per wave: candidates, searches,
// triangles found still present, triangles destroyed.
// At most 72 VGPRs, so 7 waves fit per SIMD instead of 6 (a few registers
// spill to scratch; the extra waves in flight win: R-MAT scale 24
// decomposition 1300 -> 1289 ms; at 8 waves the spills cost more).
__global__ __launch_bounds__(PBLK) __attribute__((amdgpu_waves_per_eu(7)))
void k_peel(CsrView c, const int32_t *__restrict__ front, const int32_t *__restrict__ front_count,
            int32_t thr, int32_t *__restrict__ sup, const uint8_t *__restrict__ state,
            int32_t *__restrict__ next, int32_t *__restrict__ next_count,
            unsigned long long *__restrict__ work, int32_t lb_min) {
  const int lane = threadIdx.x & 63;
  int32_t n_cand = 0, n_search = 0, n_found = 0, n_ours = 0;  // this wave's work (uniform)
  const int64_t gw = ((int64_t)blockIdx.x * PBLK + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * PBLK) >> 6;
  const int32_t nfront = *front_count;
  __shared__ PeelBatch batches[PBLK / 64];
  if (nfront >= lb_min) {
    PeelBatch &B = batches[threadIdx.x >> 6];
    // edges per batch: 64, fewer when the frontier does not fill every wave
    int32_t E = 64;
    while (E > 1 && (int64_t)nfront < nw * E) E >>= 1;
    const int64_t nbatch = ((int64_t)nfront + E - 1) / E;
    for (int64_t bi = gw; bi < nbatch; bi += nw) {
      // ---- the batch's edges, one per lane ----
      const int64_t f = bi * E + lane;
      int32_t p = -1, need = 0, tot = 0;
      if (lane < E && f < nfront) {
        p = front[f];
        need = sup[p];
      }
      uint32_t fl = 0;
      int32_t cum0 = 0, cum1 = 0;
      if (need > 0) {
        const PeelEdge pe = peel_edge(c, c.src[p], c.col[p]);
#pragma unroll
        for (int cs = 0; cs < 3; ++cs) {
          const PeelCase pc = peel_case(pe, p, cs);
          B.A0[cs][lane] = pc.A0 + pc.nA - 1;  // the last entry: walked downwards
          B.B0[cs][lane] = pc.B0;
          B.B1[cs][lane] = pc.B0 + pc.nB;
          fl |= pc.flags << (2 * cs);
          tot += pc.nA;
          if (cs == 0) cum0 = tot;
          if (cs == 1) cum1 = tot;
        }
      }
      B.p[lane] = p;
      B.need[lane] = need;
      B.seen[lane] = 0;
      B.cum[0][lane] = cum0;
      B.cum[1][lane] = cum1;
      B.flags[lane] = fl;
      long long incl = tot;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const long long t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
      }
      B.off[lane] = incl - tot;
      const long long T = __shfl(incl, 63, 64);
      wave_lds_fence();
      // ---- the concatenated candidates, 64 * PEEL_U per step ----
      long long base = 0;
      BatchCursor cur;
      cur.init(B);
      for (;;) {
        // skip edges that have seen all their triangles
        while (base < T) {
          const int e0 = batch_edge(B, base);
          if (B.seen[e0] < B.need[e0]) break;
          base = e0 < 63 ? B.off[e0 + 1] : T;
        }
        if (base >= T) break;
        int32_t eu[PEEL_U], qk[PEEL_U], key[PEEL_U], lo[PEEL_U], hi[PEEL_U], hit[PEEL_U];
        bool bin[PEEL_U], act[PEEL_U], cd[PEEL_U];
#pragma unroll
        for (int u = 0; u < PEEL_U; ++u) {
          const long long t = base + u * 64 + lane;
          cd[u] = false;
          eu[u] = 0;
          qk[u] = -1;
          key[u] = 0;
          lo[u] = 0;
          hi[u] = 0;
          bin[u] = false;
          act[u] = false;
          if (t < T) {
            const int e = cur.edge(B, t);
            eu[u] = e;
            if (B.seen[e] < B.need[e]) {
              const int32_t local = (int32_t)(t - B.off[e]);
              const int32_t c0 = B.cum[0][e], c1 = B.cum[1][e];
              const int cs = local < c0 ? 0 : (local < c1 ? 1 : 2);
              const int32_t li = local - (cs == 0 ? 0 : (cs == 1 ? c0 : c1));
              const uint32_t f2 = B.flags[e] >> (2 * cs);
              const int32_t i = B.A0[cs][e] - li;
              cd[u] = true;
              int32_t q, x;
              if (f2 & 1u) {
                const int2 ie = c.in_edge[i];
                x = ie.x;
                q = ie.y;
              } else {
                x = c.col[i];
                q = i;
              }
              if (state[q] != EDGE_DEAD) {
                qk[u] = q;
                key[u] = x;
                lo[u] = B.B0[cs][e];
                hi[u] = B.B1[cs][e];
                bin[u] = (f2 & 2u) != 0;
                act[u] = true;
              }
            }
          }
        }
#pragma unroll
        for (int u = 0; u < PEEL_U; ++u) {
          n_cand += __popcll(__ballot(cd[u]));
          n_search += __popcll(__ballot(act[u]));
        }
        find_many_lists(c, bin, lo, hi, key, act, hit);
        bool fnd[PEEL_U];
        int32_t pe[PEEL_U];
        int r[PEEL_U];
#pragma unroll
        for (int u = 0; u < PEEL_U; ++u) {
          fnd[u] = hit[u] >= 0;
          pe[u] = act[u] ? B.p[eu[u]] : 0;
        }
        destroy_many(fnd, pe, qk, hit, thr, state, sup, next, next_count, r);
#pragma unroll
        for (int u = 0; u < PEEL_U; ++u) {
          n_found += __popcll(__ballot(r[u] & 1));
          n_ours += __popcll(__ballot(r[u] >> 1));
          if (r[u] & 1) atomicAdd(&B.seen[eu[u]], 1);
        }
        wave_lds_fence();
        base += 64 * PEEL_U;
      }
      wave_lds_fence();
    }
  } else {
  // keep every wave busy: a small frontier shares each edge among wpe waves
  int32_t wpe = 1;
  while (wpe < 16 && (int64_t)nfront * wpe * 2 <= nw) wpe *= 2;
  const int64_t groups = nw / wpe;
  const int32_t sub = (int32_t)(gw % wpe);
  const int32_t stride = 64 * wpe;
  for (int64_t f = gw / wpe; f < nfront && gw < groups * wpe; f += groups) {
    const int32_t p = front[f];
    // p's support is the number of its triangles still present: none -> no
    // work; and a wave that scans p alone may stop once it has seen them all
    const int32_t need = sup[p];
    if (need == 0) continue;
    int32_t seen = 0;
    const int32_t a = c.src[p], b = c.col[p];
    const PeelEdge e = peel_edge(c, a, b);
#pragma unroll 1
    for (int cs = 0; cs < 3 && !(wpe == 1 && seen >= need); ++cs) {
      const PeelCase pc = peel_case(e, p, cs);
      const int32_t nA = pc.nA, A0 = pc.A0, B0 = pc.B0, B1 = pc.B0 + pc.nB;
      if (nA == 0) continue;
      const bool A_in = pc.flags & 1u, B_in = pc.flags & 2u;
      for (int32_t t0 = sub * 64 + lane; t0 - lane < nA && !(wpe == 1 && seen >= need);
           t0 += stride * PEEL_U) {
        int32_t qk[PEEL_U], key[PEEL_U], hit[PEEL_U];
        bool act[PEEL_U], cd[PEEL_U];
#pragma unroll
        for (int u = 0; u < PEEL_U; ++u) {
          const int32_t t = t0 + u * stride;
          cd[u] = t < nA;
          qk[u] = -1;
          key[u] = 0;
          act[u] = false;
          if (t < nA) {
            const int32_t i = A0 + nA - 1 - t;  // highest rank first
            int32_t q, x;
            if (A_in) {
              const int2 ie = c.in_edge[i];
              x = ie.x;
              q = ie.y;
            } else {
              x = c.col[i];
              q = i;
            }
            if (state[q] != EDGE_DEAD) {
              qk[u] = q;
              key[u] = x;
              act[u] = true;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < PEEL_U; ++u) {
          n_cand += __popcll(__ballot(cd[u]));
          n_search += __popcll(__ballot(act[u]));
        }
        if (B_in) find_many(c.in_edge, B0, B1, key, act, hit);
        else find_many(c.col, B0, B1, key, act, hit);
        // q1, q2: the edges between x and the two ends of p (either order)
        bool fnd[PEEL_U];
        int32_t pe[PEEL_U];
        int r[PEEL_U];
#pragma unroll
        for (int u = 0; u < PEEL_U; ++u) {
          fnd[u] = hit[u] >= 0;
          pe[u] = p;
        }
        destroy_many(fnd, pe, qk, hit, thr, state, sup, next, next_count, r);
#pragma unroll
        for (int u = 0; u < PEEL_U; ++u) {
          const int32_t fu = __popcll(__ballot(r[u] & 1));
          n_found += fu;
          n_ours += __popcll(__ballot(r[u] >> 1));
          seen += fu;
        }
      }
    }
  }
  }
  if (work && lane == 0) {  // this wave's own slots: no other wave writes them
    work[gw * 4 + 0] += (unsigned long long)n_cand;
    work[gw * 4 + 1] += (unsigned long long)n_search;
    work[gw * 4 + 2] += (unsigned long long)n_found;
    work[gw * 4 + 3] += (unsigned long long)n_ours;
  }
}

__global__ void k_sum_work(const unsigned long long *__restrict__ w, int64_t nw,
                           unsigned long long *__restrict__ out) {
  unsigned long long acc[4] = {0, 0, 0, 0};
  for (int64_t i = threadIdx.x; i < nw; i += blockDim.x)
    for (int k = 0; k < 4; ++k) acc[k] += w[i * 4 + k];
  for (int k = 0; k < 4; ++k) {
    unsigned long long v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&out[k], v);
  }
}

// Retire the frontier (truss number k - 1) and mark the next one.  Also
// clears the counter the round after next appends to (the one this round's
// predecessor read), and keeps the round statistics: st[0] rounds, st[1]
// edges removed, st[2] largest round, st[3 + i] rounds with floor(log2 r) = i.
// With box != null (host-mapped memory) it also leaves the next frontier's
// size in box[0] and edges removed so far in box[1..2] (low, high 32 bits),
// so the host reads them after a stream wait, with no copy.
__global__ void k_advance(const int32_t *__restrict__ front, const int32_t *__restrict__ front_count,
                          const int32_t *__restrict__ next, const int32_t *__restrict__ next_count,
                          int32_t *__restrict__ spare_count, uint8_t *__restrict__ state,
                          const int32_t *__restrict__ eid, int32_t *__restrict__ tau,
                          int32_t tau_val, long long *__restrict__ st,
                          volatile int32_t *__restrict__ box) {
  const int32_t nfront = *front_count, nn = *next_count;
  const int64_t lim = nfront > nn ? nfront : nn;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < lim;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nfront) {
      const int32_t p = front[i];
      state[p] = EDGE_DEAD;
      if (tau) tau[eid[p]] = tau_val;
    }
  }
  // the next frontier is disjoint from the current one (its edges were alive
  // during the round), so the two loops never store to the same state byte
  // and need no ordering between them
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
       i += (int64_t)gridDim.x * blockDim.x)
    state[next[i]] = EDGE_FRONT;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *spare_count = 0;
    if (nfront > 0) {
      st[0] += 1;
      st[1] += nfront;
      if (nfront > st[2]) st[2] = nfront;
      st[3 + (31 - __clz(nfront))] += 1;
    }
    if (box) {
      const long long removed = st[1];
      box[0] = nn;
      box[1] = (int32_t)(removed & 0xffffffffLL);
      box[2] = (int32_t)(removed >> 32);
    }
  }
}

// Start of the rounds of a level: the first frontier's size becomes counter
// 0, counters 1 and 2 start at zero.
__global__ void k_level_start(int32_t *__restrict__ cnt, int32_t nfront) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cnt[0] = nfront;
    cnt[1] = 0;
    cnt[2] = 0;
  }
}

// The level's first frontier, tile by tile over the slots of the current
// CSR: block b takes slots [b * CT_TILE, (b + 1) * CT_TILE), CT_PER
// consecutive ones per thread (one 16-byte load of states, four of
// supports), marks the live edges with support < thr as frontier, and writes
// them in slot order to tmp from the tile's own start; tile_cnt[b] = their
// number.  With dmin != null it also takes the minimum support (atomicMin
// into *dmin) and the number (atomicAdd into *dalive) of the live edges.
constexpr int CT_PER = 16;
constexpr int CT_TILE = 256 * CT_PER;

__global__ __launch_bounds__(256) void k_collect_tiles(int32_t m, int32_t thr,
                                                       uint8_t *__restrict__ state,
                                                       const int32_t *__restrict__ sup,
                                                       int32_t *__restrict__ tmp,
                                                       int32_t *__restrict__ tile_cnt,
                                                       int32_t *__restrict__ tile_min,
                                                       int32_t *__restrict__ tile_live) {
  __shared__ int32_t wtot[4], wmin[4], wlive[4];
  const int64_t tile0 = (int64_t)blockIdx.x * CT_TILE;
  const int64_t i0 = tile0 + (int64_t)threadIdx.x * CT_PER;
  uint8_t st[CT_PER];
  int32_t sv[CT_PER];
  if (i0 + CT_PER <= m) {
    const uint4 b = *reinterpret_cast<const uint4 *>(state + i0);
    const uint32_t w[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int k = 0; k < CT_PER; ++k) st[k] = (uint8_t)(w[k >> 2] >> ((k & 3) * 8));
    const int4 *s4 = reinterpret_cast<const int4 *>(sup + i0);
#pragma unroll
    for (int q = 0; q < CT_PER / 4; ++q) {
      const int4 v = s4[q];
      sv[4 * q] = v.x;
      sv[4 * q + 1] = v.y;
      sv[4 * q + 2] = v.z;
      sv[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < CT_PER; ++k) {
      st[k] = i0 + k < m ? state[i0 + k] : (uint8_t)EDGE_DEAD;
      sv[k] = i0 + k < m ? sup[i0 + k] : 0;
    }
  }
  uint32_t take = 0;  // bit k: slot i0 + k joins the frontier
  int32_t vmin = 0x7fffffff, live = 0;
#pragma unroll
  for (int k = 0; k < CT_PER; ++k)
    if (st[k] == EDGE_ALIVE) {
      vmin = min(vmin, sv[k]);
      ++live;
      if (sv[k] < thr) take |= 1u << k;
    }
  const int32_t cnt = __popc(take);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int32_t incl = wave_inclusive_scan(cnt);
  if (lane == 63) wtot[w] = incl;
  if (tile_min) {
    for (int o = 32; o > 0; o >>= 1) {
      vmin = min(vmin, __shfl_xor(vmin, o, 64));
      live += __shfl_xor(live, o, 64);
    }
    if (lane == 0) {
      wmin[w] = vmin;
      wlive[w] = live;
    }
  }
  __syncthreads();
  if (tile_min && threadIdx.x == 0) {
    // per tile: one atomic per tile on a single address serialises the
    // tiles (62 ms of a scale-24 decomposition), so the minimum and count
    // are reduced by k_min_live instead
    tile_min[blockIdx.x] = min(min(wmin[0], wmin[1]), min(wmin[2], wmin[3]));
    tile_live[blockIdx.x] = wlive[0] + wlive[1] + wlive[2] + wlive[3];
  }
  int32_t off = incl - cnt;
  for (int i = 0; i < w; ++i) off += wtot[i];
  if (threadIdx.x == 255) tile_cnt[blockIdx.x] = off + cnt;
  int32_t *out = tmp + tile0 + off;
#pragma unroll
  for (int k = 0; k < CT_PER; ++k)
    if ((take >> k) & 1u) {
      state[i0 + k] = EDGE_FRONT;
      *out++ = (int32_t)(i0 + k);
    }
}

// dmin = the smallest of tile_min[0, n), dalive = the sum of tile_live[0, n)
// (one block).
__global__ __launch_bounds__(1024) void k_min_live(const int32_t *__restrict__ tile_min,
                                                   const int32_t *__restrict__ tile_live,
                                                   int32_t n, int32_t *__restrict__ dmin,
                                                   int32_t *__restrict__ dalive,
                                                   volatile int32_t *__restrict__ box) {
  __shared__ int32_t smin[16], slive[16];
  int32_t vmin = 0x7fffffff, live = 0;
  for (int32_t i = threadIdx.x; i < n; i += 1024) {
    vmin = min(vmin, tile_min[i]);
    live += tile_live[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    vmin = min(vmin, __shfl_xor(vmin, o, 64));
    live += __shfl_xor(live, o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    smin[w] = vmin;
    slive[w] = live;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    vmin = smin[0];
    live = slive[0];
    for (int i = 1; i < 16; ++i) {
      vmin = min(vmin, smin[i]);
      live += slive[i];
    }
    *dmin = vmin;
    *dalive = live;
    if (box) {  // host-mapped: read after a stream wait
      box[0] = vmin;
      box[1] = live;
    }
  }
}

// Copy tile b's tile_cnt[b] entries of tmp to front[tile_pos[b] ...).
__global__ void k_gather_tiles(const int32_t *__restrict__ tmp, const int32_t *__restrict__ tile_cnt,
                               const int32_t *__restrict__ tile_pos, int32_t ntiles,
                               int32_t *__restrict__ front, volatile int32_t *__restrict__ box) {
  // the frontier's size, for the host (host-mapped, may be null)
  if (box && blockIdx.x == 0 && threadIdx.x == 0) *box = tile_pos[ntiles];
  for (int64_t b = blockIdx.x; b < ntiles; b += gridDim.x) {
    const int32_t cnt = tile_cnt[b], at = tile_pos[b];
    const int32_t *src = tmp + b * CT_TILE;
    for (int32_t i = threadIdx.x; i < cnt; i += blockDim.x) front[at + i] = src[i];
  }
}

// mask[eid[p]] = 1 for every slot p whose edge is not dead
__global__ void k_mask_live(const uint8_t *__restrict__ state, const int32_t *__restrict__ eid,
                            int32_t m, uint8_t *__restrict__ mask) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    if (state[i] != EDGE_DEAD) mask[eid[i]] = 1;
}

// Sort keys of a frontier: the higher endpoint of each edge.
__global__ void k_front_keys(const int32_t *__restrict__ front, int32_t n,
                             const int32_t *__restrict__ col, uint64_t *__restrict__ keys,
                             uint32_t *__restrict__ vals) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = front[i];
    keys[i] = (uint64_t)(uint32_t)col[p];
    vals[i] = (uint32_t)p;
  }
}

__global__ void k_front_store(const uint32_t *__restrict__ vals, int32_t n,
                              int32_t *__restrict__ front) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    front[i] = (int32_t)vals[i];
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

// In-list entries whose edge survives a compaction keep their order (each
// list stays sorted by source).  pos is the exclusive scan of the slots'
// survival flags, so slot s survives iff pos[s + 1] > pos[s], and pos[s] is
// its new number: one random read of two neighbouring words per entry gives
// iflag[j] (entry j survives) and nslot[j] (its slot's new number).
__global__ void k_in_alive(const int2 *__restrict__ in_edge, int32_t m,
                           const int32_t *__restrict__ pos, int32_t *__restrict__ iflag,
                           int32_t *__restrict__ nslot) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t sl = in_edge[j].y;
    const int32_t p0 = pos[sl], p1 = pos[sl + 1];
    iflag[j] = p1 > p0 ? 1 : 0;
    nslot[j] = p0;
  }
}

// Surviving in-list entries to their new places, with their slots renumbered
// (every read coalesced).
__global__ void k_in_compact(const int2 *__restrict__ in_edge, int32_t m,
                             const int32_t *__restrict__ iflag, const int32_t *__restrict__ ipos,
                             const int32_t *__restrict__ nslot, int2 *__restrict__ nin) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m;
       j += (int64_t)gridDim.x * blockDim.x)
    if (iflag[j]) nin[ipos[j]] = make_int2(in_edge[j].x, nslot[j]);
}

// one element per thread up to 2^28 elements: the compaction kernels do a
// random load per element, and more threads keep more of them in flight
// (R-MAT scale 24 decomposition 1269 -> 1265 ms against 65,536 blocks)
static unsigned gsz(int64_t work) { return grid_for(work, 256, 1 << 20); }

struct PeelState {
  DeviceBuffer sup[2], state[2], front[2], flag, pos, misc, work, ctl;
  int cur = 0;  // which sup/state buffer is live
  ~PeelState() {
    for (int i = 0; i < 2; ++i) {
      dfree(sup[i]); dfree(state[i]); dfree(front[i]);
    }
    dfree(flag); dfree(pos); dfree(misc); dfree(work); dfree(ctl);
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
  // in-lists: drop the dead entries in place order and renumber their slots
  // (no sort; the peel reads in_ptr and in_edge only, so the working copy
  // carries no in_tail)
  GC_TRY(dalloc(w.in_ptr, sizeof(int32_t) * ((size_t)n + 1)));
  GC_TRY(dalloc(w.in_edge, sizeof(int2) * ((size_t)kept + 1)));
  const size_t need = 3 * abytes<int32_t>((size_t)m + 1) + scan_scratch_bytes((int64_t)m + 1);
  GC_TRY(g->ws.reserve(need));
  int32_t *iflag = g->ws.take<int32_t>((size_t)m + 1), *ipos = g->ws.take<int32_t>((size_t)m + 1);
  int32_t *nslot = g->ws.take<int32_t>((size_t)m + 1);
  void *iscr = g->ws.take<char>(scan_scratch_bytes((int64_t)m + 1));
  k_in_alive<<<gsz(m), 256, 0, s>>>(c.in_edge, m, pos, iflag, nslot);
  GC_LAUNCH_CHECK();
  GC_TRY(exclusive_scan(iflag, ipos, m, iscr, s));
  k_in_compact<<<gsz(m), 256, 0, s>>>(c.in_edge, m, iflag, ipos, nslot,
                                      static_cast<int2 *>(w.in_edge.ptr));
  GC_LAUNCH_CHECK();
  k_rows2<<<gsz((int64_t)n + 1), 256, 0, s>>>(c.in_ptr, ipos, n,
                                              static_cast<int32_t *>(w.in_ptr.ptr));
  GC_LAUNCH_CHECK();
  c = w.view(n, kept);
  c.in_tail = nullptr;
  next ^= 1;
  ps.cur = o;
  ++g->peel_stats[4];
  return GC_OK;
}

// ---- the k-truss as a replayable launch sequence -------------------------

static __global__ void k_fill_u8(uint8_t *__restrict__ x, int64_t n, uint8_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

static __global__ void k_fill_i32n(int32_t *__restrict__ x, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

// A level's first frontier size, read on the device: counter 0 takes it,
// counters 1 and 2 start at zero.
static __global__ void k_level_start_dev(int32_t *__restrict__ cnt,
                                         const int32_t *__restrict__ nfront) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cnt[0] = *nfront;
    cnt[1] = 0;
    cnt[2] = 0;
  }
}

static __global__ void k_copy_i32(const int32_t *__restrict__ from, int32_t *__restrict__ to) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *to = *from;
}

// ctl layout: cnt[16], st[40] (long long), leftover[64]
struct ReplayCtl {
  int32_t cnt[16];
  long long st[40];
  int32_t leftover[64];
};

gc_status PeelReplay::prepare(int32_t m_edges) {
  m = m_edges;
  const size_t mm = (size_t)m_edges + 1;
  GC_TRY(dalloc(sup, sizeof(int32_t) * mm));
  GC_TRY(dalloc(state, mm));
  GC_TRY(dalloc(front[0], sizeof(int32_t) * mm));
  GC_TRY(dalloc(front[1], sizeof(int32_t) * mm));
  GC_TRY(dalloc(flag, sizeof(int32_t) * mm));
  GC_TRY(dalloc(pos, sizeof(int32_t) * (mm + 64)));
  const int32_t ntiles = (int32_t)(((int64_t)m_edges + CT_TILE - 1) / CT_TILE);
  GC_TRY(dalloc(scan, scan_scratch_bytes((int64_t)ntiles + 1)));
  GC_TRY(dalloc(ctl, sizeof(ReplayCtl)));
  return GC_OK;
}

int32_t *PeelReplay::leftover() const { return static_cast<ReplayCtl *>(ctl.ptr)->leftover; }

gc_status ktruss_launches(const gc_graph *g, int32_t k, int32_t rounds, PeelReplay &r,
                          uint8_t *mask, hipStream_t s) {
  const int32_t m = (int32_t)g->m;
  if (m == 0) return GC_OK;
  if (m != r.m || k - 2 > 64) {
    set_error("k-truss launches: buffers prepared for another size, or k above 66");
    return GC_EINVAL;
  }
  const CsrView c = g->csr.view(g->n, m);
  int32_t *sup = static_cast<int32_t *>(r.sup.ptr);
  uint8_t *state = static_cast<uint8_t *>(r.state.ptr);
  int32_t *buf[2] = {static_cast<int32_t *>(r.front[0].ptr), static_cast<int32_t *>(r.front[1].ptr)};
  int32_t *flag = static_cast<int32_t *>(r.flag.ptr), *pos = static_cast<int32_t *>(r.pos.ptr);
  ReplayCtl *ctl = static_cast<ReplayCtl *>(r.ctl.ptr);
  k_fill_i32n<<<gsz(sizeof(ReplayCtl) / 4), 256, 0, s>>>(reinterpret_cast<int32_t *>(ctl),
                                                         (int64_t)(sizeof(ReplayCtl) / 4), 0);
  k_fill_i32n<<<gsz(m), 256, 0, s>>>(sup, m, 0);
  k_fill_u8<<<gsz(m), 256, 0, s>>>(state, m, EDGE_ALIVE);
  GC_LAUNCH_CHECK();
  GC_TRY(slot_support(c, g->units_sup, sup, s));
  const int64_t peel_waves = kPeelWaves;
  const unsigned peel_blocks = (unsigned)(peel_waves / (PBLK / 64));
  const int32_t lb_min = (int32_t)peel_waves;
  const int32_t ntiles = (int32_t)(((int64_t)m + CT_TILE - 1) / CT_TILE);
  int32_t *tile_cnt = pos, *tile_pos = pos + ntiles + 1, *tile_live = pos + 3 * (ntiles + 1);
  for (int32_t kk = 3; kk <= k; ++kk) {
    const int32_t thr = kk - 2;
    // first frontier: the live edges with support < thr, in slot order
    k_collect_tiles<<<ntiles, 256, 0, s>>>(m, thr, state, sup, flag, tile_cnt, nullptr, tile_live);
    GC_LAUNCH_CHECK();
    GC_TRY(exclusive_scan(tile_cnt, tile_pos, ntiles, r.scan.ptr, s));
    k_gather_tiles<<<grid_for(ntiles, 1, 4096), 256, 0, s>>>(flag, tile_cnt, tile_pos, ntiles,
                                                             buf[0], nullptr);
    k_level_start_dev<<<1, 64, 0, s>>>(ctl->cnt, tile_pos + ntiles);
    GC_LAUNCH_CHECK();
    for (int32_t rd = 0; rd < rounds; ++rd) {
      int32_t *fr = buf[rd & 1], *nx = buf[(rd + 1) & 1];
      int32_t *cf = &ctl->cnt[rd % 3], *cn = &ctl->cnt[(rd + 1) % 3], *cz = &ctl->cnt[(rd + 2) % 3];
      k_peel<<<peel_blocks, PBLK, 0, s>>>(c, fr, cf, thr, sup, state, nx, cn, nullptr, lb_min);
      k_advance<<<1024, 256, 0, s>>>(fr, cf, nx, cn, cz, state, c.eid, nullptr, kk - 1, ctl->st,
                                     nullptr);
      GC_LAUNCH_CHECK();
    }
    // the frontier the next round would take: 0 if the level has ended
    k_copy_i32<<<1, 64, 0, s>>>(&ctl->cnt[rounds % 3], &ctl->leftover[kk - 3]);
    GC_LAUNCH_CHECK();
    // next level: the round buffers start over from buf[0]
  }
  k_fill_u8<<<gsz(m), 256, 0, s>>>(mask, m, 0);
  k_mask_live<<<grid_for(m, 256, 4096), 256, 0, s>>>(state, c.eid, m, mask);
  GC_LAUNCH_CHECK();
  return GC_OK;
}

gc_status decomposition_peel(gc_graph *g, int32_t *tau, int32_t *h_kmax, hipStream_t s,
                             int32_t k_stop, uint8_t *mask, int64_t *h_mk) {
  const int32_t m = (int32_t)g->m;
  if (mask && m > 0) GC_HIP(hipMemsetAsync(mask, 0, (size_t)m, s));
  if (h_mk) *h_mk = 0;
  if (m == 0) {
    if (h_kmax) *h_kmax = 0;
    return GC_OK;
  }
  PeelState ps;
  for (int i = 0; i < 2; ++i) {
    GC_TRY(dalloc(ps.sup[i], sizeof(int32_t) * ((size_t)m + 1)));
    GC_TRY(dalloc(ps.state[i], (size_t)m + 1));
    GC_TRY(dalloc(ps.front[i], sizeof(int32_t) * ((size_t)m + 1)));
  }
  GC_TRY(dalloc(ps.flag, sizeof(int32_t) * ((size_t)m + 1)));
  // (m + 2 for the scans over slots; the level start also keeps four arrays
  // of per-tile values there, 4 * (ceil(m / CT_TILE) + 1) <= m + 64 entries)
  GC_TRY(dalloc(ps.pos, sizeof(int32_t) * ((size_t)m + 64)));
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
  // frontier buffers: a level collects into buf[0]; round r reads buf[r & 1]
  // and appends the next frontier to buf[(r + 1) & 1]
  int32_t *buf[2] = {static_cast<int32_t *>(ps.front[0].ptr),
                     static_cast<int32_t *>(ps.front[1].ptr)};
  int next_store = 0;
  int32_t kmax = 2;
  // 56 waves per CU, twice the 28 resident at 7 waves per SIMD: rounds hand
  // out their work to waves statically, and the second half lets the
  // dispatcher even out the end (R-MAT scale 24: 1,275 ms, against 1,293 at
  // 48, 1,288 at 64 and 1,280 at 84 waves per CU)
  const int64_t peel_waves = kPeelWaves;
  const unsigned peel_blocks = (unsigned)(peel_waves / (PBLK / 64));
  // smallest frontier for the lane-balanced batches (GC_PEEL_LB_MIN; below
  // it, or below one edge per wave, each edge gets whole waves)
  int32_t lb_min = (int32_t)peel_waves;
  if (const char *ev = getenv("GC_PEEL_LB_MIN")) lb_min = (int32_t)strtol(ev, nullptr, 10);
  // a level's first frontier is sorted by higher endpoint when it holds at
  // least sort_min edges (GC_PEEL_SORT_MIN; 0: never), so that the waves of
  // a batch search the same lists
  int64_t sort_min = 100000;
  if (const char *ev = getenv("GC_PEEL_SORT_MIN")) sort_min = strtoll(ev, nullptr, 10);
  // frontier fr[0, nf) in order of higher endpoint (stable: ties keep their order)
  auto sort_front = [&](int32_t *fr, int32_t nf) -> gc_status {
    const size_t need = 2 * abytes<uint64_t>(nf) + 2 * abytes<uint32_t>(nf) +
                        sort_scratch_bytes(nf) + 1024;
    GC_TRY(g->ws.reserve(need));
    uint64_t *ka = g->ws.take<uint64_t>(nf), *kb = g->ws.take<uint64_t>(nf);
    uint32_t *va = g->ws.take<uint32_t>(nf), *vb = g->ws.take<uint32_t>(nf);
    void *sscr = g->ws.take<char>(sort_scratch_bytes(nf));
    k_front_keys<<<gsz(nf), 256, 0, s>>>(fr, nf, c.col, ka, va);
    GC_LAUNCH_CHECK();
    uint64_t *ks;
    uint32_t *vs;
    GC_TRY(radix_sort(ka, kb, va, vb, nf, g->bits, sscr, s, &ks, &vs));
    k_front_store<<<gsz(nf), 256, 0, s>>>(vs, nf, fr);
    GC_LAUNCH_CHECK();
    return GC_OK;
  };
  int64_t *stats = g->peel_stats;
  for (int i = 0; i < 41; ++i) stats[i] = 0;
  // per-wave work counters (candidates, searches, triangles), summed at the end
  GC_TRY(dalloc(ps.work, sizeof(unsigned long long) * 4 * (size_t)peel_waves + 64));
  unsigned long long *work = static_cast<unsigned long long *>(ps.work.ptr);
  GC_HIP(hipMemsetAsync(work, 0, sizeof(unsigned long long) * (4 * (size_t)peel_waves + 8), s));
  // round control in device memory: three frontier counters (round r reads
  // cnt[r % 3], appends to cnt[(r + 1) % 3]) and the round statistics
  struct Ctl {
    int32_t cnt[16];
    long long st[40];
  };
  GC_TRY(dalloc(ps.ctl, sizeof(Ctl)));
  Ctl *ctl = static_cast<Ctl *>(ps.ctl.ptr);
  GC_HIP(hipMemsetAsync(ctl, 0, sizeof(Ctl), s));
  // host copies of the counters, in pinned memory (fast device-to-host
  // reads), and a mailbox the level-start and retire kernels write directly
  // (host-mapped, coherent: the stores bypass the GPU caches, so they are
  // visible once the stream wait returns, with no copy launched)
  struct Pinned {
    void *p = nullptr;
    ~Pinned() { if (p) (void)hipHostFree(p); }
  } pin;
  GC_HIP(hipHostMalloc(&pin.p, 4096, hipHostMallocMapped | hipHostMallocCoherent));
  Ctl &h_ctl = *static_cast<Ctl *>(pin.p);
  // hq: [0] min support, [1] live edges, [2] first frontier size; hb: [0]
  // next frontier size, [1..2] edges removed (low, high 32 bits)
  volatile int32_t *hq = reinterpret_cast<int32_t *>(static_cast<char *>(pin.p) + 2048);
  volatile int32_t *hb = hq + 16;
  int32_t *dq = nullptr;  // the mailbox as the device addresses it
  GC_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&dq), const_cast<int32_t *>(hq), 0));
  int32_t *db = dq + 16;
  auto removed_so_far = [&]() -> long long {
    return (long long)(uint32_t)hb[1] | ((long long)hb[2] << 32);
  };
  long long removed_base = 0;  // edges removed when live was last counted
  int32_t thr_prev = 0;        // threshold of the last level (0 before the first)

  for (;;) {
    int32_t *sup = static_cast<int32_t *>(ps.sup[ps.cur].ptr);
    uint8_t *state = static_cast<uint8_t *>(ps.state[ps.cur].ptr);
    // ---- level start, one tiled pass over the slots of the current CSR
    // (at least three quarters of them live: it is compacted below that):
    // minimum support and number of the live edges, and the edges of support
    // thr_prev (every live edge has at least that support when a level ends,
    // so if the minimum is thr_prev they are the next level's first frontier;
    // otherwise none is taken).  Tiles are compacted in slot order into flag,
    // placed by a scan of their counts and copied to buf[0]. ----
    int32_t nf = 0;
    auto collect = [&](int32_t t, int32_t *dmin, int32_t *dalive) -> gc_status {
      const int32_t ntiles = (int32_t)(((int64_t)c.m + CT_TILE - 1) / CT_TILE);
      int32_t *tile_cnt = pos, *tile_pos = pos + ntiles + 1;
      int32_t *tile_min = pos + 2 * (ntiles + 1), *tile_live = pos + 3 * (ntiles + 1);
      k_collect_tiles<<<ntiles, 256, 0, s>>>(c.m, t, state, sup, flag, tile_cnt,
                                             dmin ? tile_min : nullptr, tile_live);
      GC_LAUNCH_CHECK();
      if (dmin) {
        k_min_live<<<1, 1024, 0, s>>>(tile_min, tile_live, ntiles, dmin, dalive, dq);
        GC_LAUNCH_CHECK();
      }
      GC_TRY(g->ws.reserve(scan_scratch_bytes((int64_t)ntiles + 1)));
      GC_TRY(exclusive_scan(tile_cnt, tile_pos, ntiles,
                            g->ws.take<char>(scan_scratch_bytes((int64_t)ntiles + 1)), s));
      k_gather_tiles<<<grid_for(ntiles, 1, 4096), 256, 0, s>>>(flag, tile_cnt, tile_pos, ntiles,
                                                               buf[0], dq + 2);
      GC_LAUNCH_CHECK();
      return GC_OK;
    };
    const int32_t thr_spec = thr_prev + 1;
    k_set_i32<<<1, 64, 0, s>>>(misc, 0x7fffffff, 0);
    GC_LAUNCH_CHECK();
    GC_TRY(collect(thr_spec, misc, misc + 1));
    GC_HIP(hipStreamSynchronize(s));
    nf = hq[2];
    const int32_t alive = hq[1];
    if (alive == 0) break;
    const int32_t k = hq[0] + 3;   // first level that removes something
    const int32_t thr = k - 2;
    if (thr != thr_spec && nf != 0) {
      set_error("decomposition: live edge below the previous level's threshold");
      return GC_EDEVICE;
    }
    if (k > k_stop) {
      // every live edge survives the levels up to k_stop: the k_stop-truss
      if (mask) {
        k_mask_live<<<grid_for(c.m, 256, 4096), 256, 0, s>>>(state, c.eid, c.m, mask);
        GC_LAUNCH_CHECK();
      }
      if (h_mk) *h_mk = alive;
      break;
    }
    if ((int64_t)alive * 4 < (int64_t)c.m * 3) {
      // compact the CSR when a quarter of it is dead (dead entries cost the
      // peel candidates and longer searches; compacting at 1/2, 0.6 or 0.85
      // live measured slower)
      GC_TRY(compact_peel(g, ps, c, next_store, buf[0], nf, s));
      sup = static_cast<int32_t *>(ps.sup[ps.cur].ptr);
      state = static_cast<uint8_t *>(ps.state[ps.cur].ptr);
    }
    if (thr != thr_spec) {
      // the minimum is above thr_prev: collect the live edges with support
      // < k - 2 now
      GC_TRY(collect(thr, nullptr, nullptr));
      GC_HIP(hipStreamSynchronize(s));
      nf = hq[2];
    }
    thr_prev = thr;
    int batch = 1;
    if (sort_min > 0 && nf >= sort_min) GC_TRY(sort_front(buf[0], nf));
    k_level_start<<<1, 64, 0, s>>>(ctl->cnt, nf);
    GC_LAUNCH_CHECK();
    ++stats[0];
    kmax = k - 1 > kmax ? k - 1 : kmax;
    int64_t live = alive;  // live edges at the level start (or last compaction)
    // ---- rounds of level k, queued in batches without waiting for their
    // sizes (a round whose frontier is empty does nothing); the host looks at
    // the counters between batches, to stop and to compact ----
    int r = 0;
    int32_t nfront = 0;
    for (;;) {
      for (int i = 0; i < batch; ++i, ++r) {
        int32_t *fr = buf[r & 1], *nx = buf[(r + 1) & 1];
        int32_t *cf = &ctl->cnt[r % 3], *cn = &ctl->cnt[(r + 1) % 3], *cz = &ctl->cnt[(r + 2) % 3];
        k_peel<<<peel_blocks, PBLK, 0, s>>>(c, fr, cf, thr, sup, state, nx, cn, work, lb_min);
        GC_LAUNCH_CHECK();
        k_advance<<<1024, 256, 0, s>>>(fr, cf, nx, cn, cz, state, c.eid, tau, k - 1, ctl->st,
                                       i + 1 == batch ? db : nullptr);
        GC_LAUNCH_CHECK();
      }
      GC_HIP(hipStreamSynchronize(s));
      nfront = hb[0];  // the last retire of the batch left the next size
      if (nfront == 0) break;
      if ((live - (removed_so_far() - removed_base)) * 4 < (int64_t)c.m * 3) {
        GC_TRY(compact_peel(g, ps, c, next_store, buf[r & 1], nfront, s));
        sup = static_cast<int32_t *>(ps.sup[ps.cur].ptr);
        state = static_cast<uint8_t *>(ps.state[ps.cur].ptr);
        live = c.m;
        removed_base = removed_so_far();
      }
      batch = batch < 16 ? batch * 2 : 16;
    }
    removed_base = removed_so_far();
  }
  GC_HIP(hipMemcpyAsync(&h_ctl, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  GC_HIP(hipStreamSynchronize(s));
  stats[1] = h_ctl.st[0];
  stats[2] = h_ctl.st[1];
  stats[3] = h_ctl.st[2];
  for (int i = 0; i < 32; ++i) stats[5 + i] = h_ctl.st[3 + i];
  unsigned long long *wsum = work + 4 * (size_t)peel_waves;
  k_sum_work<<<1, 256, 0, s>>>(work, peel_waves, wsum);
  GC_LAUNCH_CHECK();
  unsigned long long hw[4] = {0, 0, 0, 0};
  GC_HIP(hipMemcpyAsync(hw, wsum, sizeof(hw), hipMemcpyDeviceToHost, s));
  GC_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < 4; ++i) stats[37 + i] = (int64_t)hw[i];
  if (h_kmax) *h_kmax = kmax;
  return GC_OK;
}

}  // namespace gc
