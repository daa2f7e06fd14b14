// Device-wide exclusive scan and stable LSD radix sort (own kernels).
#pragma once

#include "common.h"

namespace gc {

// out[i] = sum_{j<i} in[i]; in == out allowed.  Temporaries come from the
// arena and are released before returning.  T: int32_t, int64_t, uint32_t, u64.
template <class T>
int scan_exclusive(const T *in, T *out, int64_t n, Arena &a, hipStream_t s);

// Stable sort of 64-bit keys on bits [lo, lo + bits).  Sorts keys[0..n)
// using alt[0..n) as the second buffer; returns the buffer that holds the
// result (keys or alt) through *result.
int radix_sort_u64(u64 *keys, u64 *alt, int64_t n, int bits, u64 **result, Arena &a,
                   hipStream_t s, int lo = 0);

// Fill n elements with a value (a kernel, never a memset node).
template <class T>
int fill(T *p, T v, int64_t n, hipStream_t s);

}  // namespace gc
