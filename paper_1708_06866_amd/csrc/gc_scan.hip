// gc_scan.hip -- device exclusive prefix sum (reduce-then-scan).
//
// Used for every offset computation of the build (unique-edge positions, row
// pointers, radix-sort digit offsets) and for compaction of the k-truss edge
// list.  Three phases: per-tile sums, a scan of the tile sums (recursive), and
// a per-tile scan that adds the tile's base.  No inter-block waiting, so no
// forward-progress assumptions.
#include "gc_common.h"

namespace gc {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;  // 2048

// Block-wide exclusive scan of one value per thread; returns the exclusive
// prefix and writes the block total to *total.
template <class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *smem4, T *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) smem4[wave] = inc;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < SCAN_BLOCK / 64; ++w) {
    const T s = smem4[w];
    base += (w < wave) ? s : T(0);
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

// Per-tile sums, accumulated in the output type.
template <class In, class Acc>
__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_sums(const In *in, int64_t n, Acc *sums) {
  __shared__ Acc sm[SCAN_BLOCK / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  Acc acc = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    int64_t i = base + (int64_t)j * SCAN_BLOCK + threadIdx.x;
    if (i < n) acc += (Acc)in[i];
  }
  Acc tot;
  (void)block_exclusive_scan<Acc>(acc, sm, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Scan each tile (thread t owns the contiguous items t*ITEMS .. +ITEMS-1) and
// add the tile base from `bases` (exclusive-scanned tile sums).  If `total` is
// non-null the last tile writes the grand total there.
template <class In, class Acc>
__global__ __launch_bounds__(SCAN_BLOCK) void k_tile_scan(const In *in, Acc *out, int64_t n,
                                                          const Acc *bases, Acc *total) {
  __shared__ Acc sm[SCAN_BLOCK / 64];
  __shared__ Acc tile[SCAN_TILE];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  // coalesced load into LDS
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    int idx = j * SCAN_BLOCK + threadIdx.x;
    int64_t i = base + idx;
    tile[idx] = (i < n) ? (Acc)in[i] : Acc(0);
  }
  __syncthreads();
  Acc x[SCAN_ITEMS];
  Acc acc = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    x[j] = tile[threadIdx.x * SCAN_ITEMS + j];
    acc += x[j];
  }
  Acc tot;
  Acc pre = block_exclusive_scan<Acc>(acc, sm, &tot);
  const Acc tb = bases ? bases[blockIdx.x] : Acc(0);
  pre += tb;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    tile[threadIdx.x * SCAN_ITEMS + j] = pre;
    pre += x[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    int idx = j * SCAN_BLOCK + threadIdx.x;
    int64_t i = base + idx;
    if (i < n) out[i] = tile[idx];
  }
  if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = tb + tot;
}

static int64_t num_tiles(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

template <class Acc>
static size_t scratch_bytes(int64_t n) {
  size_t b = 0;
  int64_t t = num_tiles(n);
  while (t > 1) {
    b += abytes<Acc>(t + 1);
    t = num_tiles(t);
  }
  return b + 256;
}

size_t scan_scratch_bytes(int64_t n) { return scratch_bytes<int64_t>(n); }

template <class In, class Acc>
static gc_status scan_rec(const In *in, Acc *out, int64_t n, Acc *total, char *scratch,
                          hipStream_t s) {
  if (n <= 0) {
    if (total) GC_HIP(hipMemsetAsync(total, 0, sizeof(Acc), s));
    return GC_OK;
  }
  int64_t t = num_tiles(n);
  if (t == 1) {
    k_tile_scan<In, Acc><<<1, SCAN_BLOCK, 0, s>>>(in, out, n, nullptr, total);
    GC_LAUNCH_CHECK();
    return GC_OK;
  }
  Acc *sums = reinterpret_cast<Acc *>(scratch);
  scratch += abytes<Acc>(t + 1);
  k_tile_sums<In, Acc><<<(unsigned)t, SCAN_BLOCK, 0, s>>>(in, n, sums);
  GC_LAUNCH_CHECK();
  GC_TRY((scan_rec<Acc, Acc>(sums, sums, t, nullptr, scratch, s)));
  k_tile_scan<In, Acc><<<(unsigned)t, SCAN_BLOCK, 0, s>>>(in, out, n, sums, total);
  GC_LAUNCH_CHECK();
  return GC_OK;
}

gc_status exclusive_scan(const int32_t *in, int32_t *out, int64_t n, void *scratch,
                         hipStream_t s) {
  return scan_rec<int32_t, int32_t>(in, out, n, out + n, static_cast<char *>(scratch), s);
}

gc_status exclusive_scan64(const int32_t *in, int64_t *out, int64_t n, void *scratch,
                           hipStream_t s) {
  return scan_rec<int32_t, int64_t>(in, out, n, out + n, static_cast<char *>(scratch), s);
}

}  // namespace gc
