// gc_common.h -- internal helpers shared by the libgc HIP sources (not part of
// the public ABI): status handling, a grow-only device workspace, and
// wavefront primitives for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <exception>
#include <string>

#include "gc.h"

namespace gc {

// --------------------------------------------------------------------------
// Status handling
// --------------------------------------------------------------------------
void set_error(const std::string &msg);
void clear_error();

// Evaluate a HIP call; on failure record the message and return GC_EDEVICE
// (or GC_ENOMEM for allocation failures) from the enclosing function.
#define GC_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      ::gc::set_error(std::string(#call) + ": " + hipGetErrorString(e_));   \
      return e_ == hipErrorOutOfMemory ? GC_ENOMEM : GC_EDEVICE;            \
    }                                                                       \
  } while (0)

// Propagate a gc_status from a helper.
#define GC_TRY(expr)                 \
  do {                               \
    gc_status s_ = (expr);           \
    if (s_ != GC_OK) return s_;      \
  } while (0)

// Check the last kernel launch.
#define GC_LAUNCH_CHECK() GC_HIP(hipGetLastError())

// Entry points that allocate host memory or start threads keep C++ exceptions
// from crossing the C ABI: a failed host allocation or thread start becomes
// GC_ENOMEM, with the exception's text as the last error.
void note_host_failure(const char *where, const char *what) noexcept;

template <class F>
inline gc_status guard_host(const char *where, F &&body) noexcept {
  try {
    return body();
  } catch (const std::exception &e) {
    note_host_failure(where, e.what());
  } catch (...) {
    note_host_failure(where, "unknown exception");
  }
  return GC_ENOMEM;
}

// --------------------------------------------------------------------------
// Device memory: a tracked allocation and a grow-only bump workspace.
// --------------------------------------------------------------------------
struct DeviceBuffer {
  void *ptr = nullptr;
  size_t bytes = 0;
  hipStream_t ord = nullptr;  // stream-ordered allocation: released on this stream
  bool ordered = false;
};

gc_status dalloc(DeviceBuffer &b, size_t bytes);  // (re)allocates if too small
void dfree(DeviceBuffer &b);

// Stream-ordered device memory for the calling thread.  hipFree waits for
// the whole device, and while it waits other threads' launches stall too.
// While an AllocScope is alive, dalloc takes memory with hipMallocAsync on
// the scope's stream, and such a buffer is later released with hipFreeAsync:
// on the stream it was allocated on, or on the stream of a FreeScope alive
// at the time of release (for buffers that no work in flight uses any more).
// Neither waits for work on other streams.  Outside any scope dalloc / dfree
// use hipMalloc / hipFree.  The streams must outlive the buffers.
struct AllocScope {
  hipStream_t prev;
  explicit AllocScope(hipStream_t s);
  ~AllocScope();
};
struct FreeScope {
  hipStream_t prev;
  explicit FreeScope(hipStream_t s);
  ~FreeScope();
};

// Device memory an allocation holds: the HIP allocator rounds buffers above
// 2 MiB up to 2 MiB multiples, and smaller ones up to 4 KiB pages plus a
// header (measured on MI355X: 256 B takes 10.2 KiB, 64 KiB takes 71.7 KiB,
// 1 MiB takes 1 MiB, 3 MiB takes 4 MiB).
inline size_t held_bytes(const DeviceBuffer &b) {
  if (!b.ptr) return 0;
  constexpr size_t kBig = size_t(2) << 20, kPage = 4096, kHeader = 8192;
  return b.bytes > kBig ? (b.bytes + kBig - 1) / kBig * kBig
                        : (b.bytes + kPage - 1) / kPage * kPage + kHeader;
}

// Carves 256-byte aligned sub-buffers out of one allocation.  reserve() grows
// the backing allocation (only between calls; contents are not preserved).
struct Workspace {
  DeviceBuffer buf;
  size_t off = 0;
  Workspace() = default;
  Workspace(const Workspace &) = delete;
  Workspace &operator=(const Workspace &) = delete;
  ~Workspace() { dfree(buf); }
  gc_status reserve(size_t bytes) { off = 0; return dalloc(buf, bytes); }
  template <class T>
  T *take(size_t count) {
    size_t b = (count * sizeof(T) + 255) & ~size_t(255);
    T *p = reinterpret_cast<T *>(static_cast<char *>(buf.ptr) + off);
    off += b;
    return p;
  }
};

template <class T>
inline size_t abytes(size_t count) {
  return (count * sizeof(T) + 255) & ~size_t(255);
}

inline int ceil_log2_u64(uint64_t x) {  // smallest b with 2^b >= x
  int b = 0;
  while (b < 63 && (uint64_t(1) << b) < x) ++b;
  return b;
}

inline unsigned grid_for(int64_t work, int per_block, int64_t cap = 1 << 20) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// --------------------------------------------------------------------------
// Scans and sort (gc_scan.hip, gc_sort.hip)
// --------------------------------------------------------------------------

// Scratch needed by exclusive_scan or exclusive_scan64 for n elements.
size_t scan_scratch_bytes(int64_t n);
// out[i] = sum_{j<i} in[i] for i < n, and out[n] = total (out holds n+1).
// In-place (out == in) is allowed.  n < 2^31, total < 2^31.
gc_status exclusive_scan(const int32_t *in, int32_t *out, int64_t n,
                         void *scratch, hipStream_t s);
// The same with 64-bit sums: out (n+1 entries) may total beyond 2^31.
gc_status exclusive_scan64(const int32_t *in, int64_t *out, int64_t n,
                           void *scratch, hipStream_t s);

// Scratch needed by radix_sort for n keys.
size_t sort_scratch_bytes(int64_t n);
// Stable LSD radix sort of keys (and optional 32-bit payload) on their low
// `bits` bits.  keys/alt (and vals/valt) are ping-pong buffers of n entries;
// on return *keys_out / *vals_out point at whichever buffer holds the result.
gc_status radix_sort(uint64_t *keys, uint64_t *alt, uint32_t *vals,
                     uint32_t *valt, int64_t n, int bits, void *scratch,
                     hipStream_t s, uint64_t **keys_out, uint32_t **vals_out);

// --------------------------------------------------------------------------
// Wavefront primitives (wave64)
// --------------------------------------------------------------------------
#ifdef __HIP_DEVICE_COMPILE__
#define GC_DEVICE_INLINE __device__ __forceinline__
#else
#define GC_DEVICE_INLINE __device__ inline
#endif

// Sum over the 64 lanes with DPP row operations, then the two cross-row
// broadcasts; every active lane must participate.  Result returned to all
// lanes via readlane 63.
GC_DEVICE_INLINE int32_t wave_sum_i32(int32_t v) {
  // within quads
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  // within rows of 16
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row_mirror
  // across rows: lane 15 of row r -> row r+1, then lane 31 -> rows 2, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast31
  return __builtin_amdgcn_readlane(v, 63);
}

GC_DEVICE_INLINE uint64_t lanemask_lt() {
  const unsigned lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Inclusive scan over the wave (shuffles).
GC_DEVICE_INLINE int32_t wave_inclusive_scan(int32_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Append `take` (per lane) to a global list with one atomic per wave: returns
// this lane's slot (valid where take is true).  Works with any set of active
// lanes: the ballot only sees active lanes.
GC_DEVICE_INLINE int32_t wave_append(bool take, int32_t *counter) {
  const uint64_t mask = __ballot(take);
  if (mask == 0) return -1;
  const int leader = __ffsll((long long)mask) - 1;
  int32_t base = 0;
  if ((int)__lane_id() == leader) base = atomicAdd(counter, (int32_t)__popcll(mask));
  base = __shfl(base, leader, 64);
  return base + (int32_t)__popcll(mask & lanemask_lt());
}

// counts[key] += number of lanes holding `key`, for keys sorted along the
// wave (equal keys in consecutive lanes): one atomic per run of equal keys.
// Every lane of the wave must call this; lanes with valid == false add
// nothing.
GC_DEVICE_INLINE void wave_run_count(bool valid, int32_t key, int32_t *counts) {
  const int lane = (int)__lane_id();
  const int32_t k = valid ? key : -1;
  const int32_t prev = __shfl_up(k, 1, 64);
  const uint64_t bounds = __ballot(lane == 0 || k != prev);
  if (valid && (lane == 0 || k != prev)) {
    const uint64_t after = lane == 63 ? 0ull : (bounds >> (lane + 1));
    const int len = after ? __ffsll((long long)after) : 64 - lane;
    atomicAdd(&counts[k], len);
  }
}

}  // namespace gc
