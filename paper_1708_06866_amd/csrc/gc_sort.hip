// gc_sort.hip -- stable LSD radix sort of 64-bit keys with an optional 32-bit
// payload, 8-bit digits, only as many passes as the key has significant bits.
//
// One pass = (1) per-tile digit histograms, (2) an exclusive scan of the
// digit-major histogram matrix [digit][tile], which yields every (digit, tile)
// output base, and (3) a scatter in which each tile ranks its keys stably,
// reorders them through LDS and writes each digit run contiguously.
//
// Tile = 4 waves x 16 rows x 64 lanes = 4096 keys.  Wave w owns the contiguous
// sub-range [w*1024, (w+1)*1024) of the tile and walks it in 16 rows of 64, so
// tile order = (wave, row, lane).  A key's rank among equal digits inside its
// wave comes from a ballot-based match over the 8 digit bits plus a running
// per-wave digit count kept in LDS; ranks across waves come from a per-digit
// prefix over the four waves.  All of this preserves input order, so the sort
// is stable and its output is deterministic.
#include "gc_common.h"

namespace gc {

constexpr int RS_BLOCK = 256;
constexpr int RS_WAVES = RS_BLOCK / 64;
constexpr int RS_ROWS = 16;
constexpr int RS_WAVE_SPAN = 64 * RS_ROWS;        // 1024
constexpr int RS_TILE = RS_WAVES * RS_WAVE_SPAN;  // 4096
constexpr int RS_DIGITS = 256;

__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const uint64_t *__restrict__ keys,
                                                      int64_t n, int shift,
                                                      int32_t *__restrict__ hist,
                                                      int64_t ntiles) {
  __shared__ int32_t cnt[RS_WAVES][RS_DIGITS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int w = 0; w < RS_WAVES; ++w) cnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE + (int64_t)wave * RS_WAVE_SPAN;
#pragma unroll 4
  for (int r = 0; r < RS_ROWS; ++r) {
    int64_t i = base + r * 64 + lane;
    if (i < n) {
      uint32_t d = (uint32_t)(keys[i] >> shift) & 0xFF;
      atomicAdd(&cnt[wave][d], 1);
    }
  }
  __syncthreads();
  int32_t c = 0;
#pragma unroll
  for (int w = 0; w < RS_WAVES; ++w) c += cnt[w][threadIdx.x];
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = c;
}

template <bool VALS>
__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift,
    const int32_t *__restrict__ offs, int64_t ntiles) {
  __shared__ uint64_t s_keys[RS_TILE];
  __shared__ uint32_t s_vals[VALS ? RS_TILE : 1];
  __shared__ int32_t s_wcnt[RS_WAVES][RS_DIGITS];
  __shared__ int32_t s_dstart[RS_DIGITS];
  __shared__ int32_t s_gbase[RS_DIGITS];
  __shared__ int32_t s_red[RS_WAVES];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int w = 0; w < RS_WAVES; ++w) s_wcnt[w][threadIdx.x] = 0;
  s_gbase[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
  __syncthreads();

  const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
  const int64_t wbase = tbase + (int64_t)wave * RS_WAVE_SPAN;
  const uint64_t ltmask = lanemask_lt();
  uint64_t k[RS_ROWS];
  uint32_t val[RS_ROWS];
  int32_t rank[RS_ROWS];

#pragma unroll
  for (int r = 0; r < RS_ROWS; ++r) {
    const int64_t i = wbase + r * 64 + lane;
    const bool valid = i < n;
    k[r] = valid ? kin[i] : 0;
    if (VALS) val[r] = valid ? vin[i] : 0;
    const uint32_t d = (uint32_t)(k[r] >> shift) & 0xFF;
    // lanes of this row holding the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int before = __popcll(peers & ltmask);
    const int cnt = __popcll(peers);
    const int32_t old = valid ? s_wcnt[wave][d] : 0;
    rank[r] = old + before;
    // ordering: every lane read its digit's count above before the single
    // writer per digit (the lowest peer) updates it
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) s_wcnt[wave][d] = old + cnt;
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // per digit: prefix over waves, and the tile's digit starts
  {
    const int d = threadIdx.x;
    int32_t c[RS_WAVES], tot = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) { c[w] = s_wcnt[w][d]; tot += c[w]; }
    int32_t acc = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) { s_wcnt[w][d] = acc; acc += c[w]; }
    // exclusive scan of tot over the 256 digits
    const int32_t inc = wave_inclusive_scan(tot);
    if (lane == 63) s_red[wave] = inc;
    __syncthreads();
    int32_t b = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) b += (w < wave) ? s_red[w] : 0;
    s_dstart[d] = b + inc - tot;
  }
  __syncthreads();

#pragma unroll
  for (int r = 0; r < RS_ROWS; ++r) {
    const int64_t i = wbase + r * 64 + lane;
    if (i < n) {
      const uint32_t d = (uint32_t)(k[r] >> shift) & 0xFF;
      const int pos = s_dstart[d] + s_wcnt[wave][d] + rank[r];
      s_keys[pos] = k[r];
      if (VALS) s_vals[pos] = val[r];
    }
  }
  __syncthreads();

  const int64_t rem = n - tbase;
  const int tcount = rem < RS_TILE ? (int)rem : RS_TILE;
  for (int p = threadIdx.x; p < tcount; p += RS_BLOCK) {
    const uint64_t kk = s_keys[p];
    const uint32_t d = (uint32_t)(kk >> shift) & 0xFF;
    const int64_t o = (int64_t)s_gbase[d] + (p - s_dstart[d]);
    kout[o] = kk;
    if (VALS) vout[o] = s_vals[p];
  }
}

static int64_t rs_tiles(int64_t n) { return (n + RS_TILE - 1) / RS_TILE; }

size_t sort_scratch_bytes(int64_t n) {
  const int64_t h = rs_tiles(n) * RS_DIGITS;
  return abytes<int32_t>(h + 1) + scan_scratch_bytes(h);
}

gc_status radix_sort(uint64_t *keys, uint64_t *alt, uint32_t *vals, uint32_t *valt,
                     int64_t n, int bits, void *scratch, hipStream_t s,
                     uint64_t **keys_out, uint32_t **vals_out) {
  *keys_out = keys;
  if (vals_out) *vals_out = vals;
  if (n <= 1 || bits <= 0) return GC_OK;
  const int64_t nt = rs_tiles(n);
  const int64_t h = nt * RS_DIGITS;
  if (h >= INT32_MAX) {
    set_error("radix_sort: too many keys");
    return GC_EOVERFLOW;
  }
  int32_t *hist = static_cast<int32_t *>(scratch);
  void *sscratch = static_cast<char *>(scratch) + abytes<int32_t>(h + 1);
  uint64_t *ka = keys, *kb = alt;
  uint32_t *va = vals, *vb = valt;
  for (int shift = 0; shift < bits; shift += 8) {
    k_rs_hist<<<(unsigned)nt, RS_BLOCK, 0, s>>>(ka, n, shift, hist, nt);
    GC_LAUNCH_CHECK();
    GC_TRY(exclusive_scan(hist, hist, h, sscratch, s));
    if (va) {
      k_rs_scatter<true><<<(unsigned)nt, RS_BLOCK, 0, s>>>(ka, va, kb, vb, n, shift, hist, nt);
    } else {
      k_rs_scatter<false><<<(unsigned)nt, RS_BLOCK, 0, s>>>(ka, nullptr, kb, nullptr, n, shift,
                                                            hist, nt);
    }
    GC_LAUNCH_CHECK();
    uint64_t *tk = ka; ka = kb; kb = tk;
    uint32_t *tv = va; va = vb; vb = tv;
  }
  *keys_out = ka;
  if (vals_out) *vals_out = va;
  return GC_OK;
}

}  // namespace gc
