// Shared host/device helpers of the graphlet library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "graphlet.h"

namespace gc {

typedef unsigned long long u64;
typedef unsigned __int128 u128;
typedef __int128 i128;

constexpr int kWave = 64;

// ---------------------------------------------------------------- errors

void set_error(const char *fmt, ...);
void clear_error();

#define GC_TRY_HIP(call)                                                         \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ::gc::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),     \
                      __FILE__, __LINE__);                                       \
      return GC_EHIP;                                                            \
    }                                                                            \
  } while (0)

#define GC_TRY(expr)          \
  do {                        \
    int rc_ = (expr);         \
    if (rc_ != GC_OK) return rc_; \
  } while (0)

// ---------------------------------------------------------------- arena
// Bump allocator over one device workspace.  In measuring mode (base ==
// nullptr) it only records the high-water mark, so the size query and the
// real run walk the same allocation sequence.
struct Arena {
  char *base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  size_t peak = 0;
  bool overflow = false;

  template <class T>
  T *take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    size_t o = off;
    off += bytes;
    if (off > peak) peak = off;
    if (!base) return nullptr;
    if (off > cap) {
      overflow = true;
      return nullptr;
    }
    return reinterpret_cast<T *>(base + o);
  }
  size_t mark() const { return off; }
  void release(size_t m) { off = m; }
  bool measuring() const { return base == nullptr; }
};

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ u64 lanemask_lt() {
  return (lane_id() == 0) ? 0ull : ((~0ull) >> (64 - lane_id()));
}

// Unsigned 128-bit atomic add of a 128-bit value stored as {lo, hi}.
__device__ __forceinline__ void atomic_add_u128(u64 *p, u128 v) {
  u64 lo = (u64)v, hi = (u64)(v >> 64);
  u64 old = atomicAdd(p, lo);
  if (old + lo < old) hi += 1;
  if (hi) atomicAdd(p + 1, hi);
}

__device__ __forceinline__ u128 wave_sum_u128(u128 v) {
  for (int off = 32; off > 0; off >>= 1) {
    u64 lo = __shfl_xor((u64)v, off, kWave);
    u64 hi = __shfl_xor((u64)(v >> 64), off, kWave);
    v += ((u128)hi << 64) | lo;
  }
  return v;
}

__device__ __forceinline__ u64 wave_sum_u64(u64 v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block-wide sum of a u128 (blockDim.x a multiple of 64, <= 1024); result
// valid in thread 0.  `scratch` holds 2 * 16 u64.
__device__ __forceinline__ u128 block_sum_u128(u128 v, u64 *scratch) {
  v = wave_sum_u128(v);
  int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();
  if (lane_id() == 0) {
    scratch[2 * w] = (u64)v;
    scratch[2 * w + 1] = (u64)(v >> 64);
  }
  __syncthreads();
  u128 r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; i++) r += ((u128)scratch[2 * i + 1] << 64) | scratch[2 * i];
  __syncthreads();
  return r;
}

template <class T>
__device__ __forceinline__ int lower_bound_dev(const T *a, int n, T x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Largest i in [0, n) with a[i] <= x (a non-decreasing, a[0] <= x).
template <class T>
__device__ __forceinline__ int upper_index_dev(const T *a, int n, T x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

static inline int bits_for(u64 v) {  // number of bits to hold values < v+1
  int b = 0;
  while (b < 64 && (v >> b) != 0) b++;
  return b;
}

}  // namespace gc
