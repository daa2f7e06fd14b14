// Device-wide scan and radix sort used by the prepass (relabelling by degree).
#include "primitives.h"

namespace gc {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanIpt = 8;
constexpr int kScanTile = kScanBlock * kScanIpt;

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_tile(const T *in, T *out, T *sums, int64_t n) {
  __shared__ T s[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIpt;
  T v[kScanIpt];
  T tot = 0;
#pragma unroll
  for (int k = 0; k < kScanIpt; k++) {
    int64_t i = base + k;
    v[k] = i < n ? in[i] : T(0);
    tot += v[k];
  }
  s[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    T t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : T(0);
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  T run = s[threadIdx.x] - tot;
  if (threadIdx.x == kScanBlock - 1 && sums) sums[blockIdx.x] = s[kScanBlock - 1];
#pragma unroll
  for (int k = 0; k < kScanIpt; k++) {
    int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_add(T *out, const T *offs, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) out[i] += offs[i / kScanTile];
}

template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// ------------------------------------------------------------------ radix sort
constexpr int kRsBlock = 256;
constexpr int kRsIpt = 16;
constexpr int kRsTile = kRsBlock * kRsIpt;

__global__ __launch_bounds__(kRsBlock) void k_rs_hist(const u64 *keys, int64_t n, int shift,
                                                      uint32_t *hist, int64_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll 4
  for (int r = 0; r < kRsIpt; r++) {
    int64_t i = base + (int64_t)r * kRsBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: keys of a tile keep their order within a digit.  Rounds
// of 256 keys go in index order; inside a round, a key's rank among equal
// digits is (keys of earlier rounds) + (keys of lower waves) + (lower lanes
// of its own wave, found with eight ballots).
__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(const u64 *in, u64 *out, int64_t n,
                                                         int shift, const uint32_t *offs,
                                                         int64_t ntiles) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kRsBlock / kWave][256];
  const int tid = threadIdx.x, wave = tid / kWave;
  run[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  const u64 lt = lanemask_lt();
  for (int r = 0; r < kRsIpt; r++) {
#pragma unroll
    for (int w = 0; w < kRsBlock / kWave; w++) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t i = base + (int64_t)r * kRsBlock + tid;
    const bool valid = i < n;
    const u64 key = valid ? in[i] : 0ull;
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    u64 peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const bool bit = (d >> b) & 1u;
      const u64 bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t lrank = (uint32_t)__popcll(peers & lt);
    if (valid && lrank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    {
      uint32_t acc = run[tid];
#pragma unroll
      for (int w = 0; w < kRsBlock / kWave; w++) {
        uint32_t c = wcnt[w][tid];
        wcnt[w][tid] = acc;
        acc += c;
      }
      run[tid] = acc;
    }
    __syncthreads();
    if (valid) out[wcnt[wave][d] + lrank] = key;
    __syncthreads();
  }
}

inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65535 * 16) g = 65535 * 16;
  return (int)g;
}

}  // namespace

template <class T>
int scan_exclusive(const T *in, T *out, int64_t n, Arena &a, hipStream_t s) {
  if (n <= 0) return GC_OK;
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  size_t m = a.mark();
  T *sums = tiles > 1 ? a.take<T>(tiles) : nullptr;
  T *offs = tiles > 1 ? a.take<T>(tiles) : nullptr;
  if (!a.measuring()) {
    if (a.overflow) return GC_ENOMEM;
    k_scan_tile<T><<<(unsigned)tiles, kScanBlock, 0, s>>>(in, out, sums, n);
    GC_TRY_HIP(hipGetLastError());
  }
  if (tiles > 1) {
    GC_TRY(scan_exclusive<T>(sums, offs, tiles, a, s));
    if (!a.measuring()) {
      k_scan_add<T><<<(unsigned)((n + kScanBlock - 1) / kScanBlock), kScanBlock, 0, s>>>(out, offs,
                                                                                         n);
      GC_TRY_HIP(hipGetLastError());
    }
  }
  a.release(m);
  return GC_OK;
}

template int scan_exclusive<int32_t>(const int32_t *, int32_t *, int64_t, Arena &, hipStream_t);
template int scan_exclusive<int64_t>(const int64_t *, int64_t *, int64_t, Arena &, hipStream_t);
template int scan_exclusive<uint32_t>(const uint32_t *, uint32_t *, int64_t, Arena &, hipStream_t);
template int scan_exclusive<u64>(const u64 *, u64 *, int64_t, Arena &, hipStream_t);

template <class T>
int fill(T *p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return GC_OK;
  k_fill<T><<<grid_for(n, 256) > 4096 ? 4096 : grid_for(n, 256), 256, 0, s>>>(p, v, n);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

template int fill<int32_t>(int32_t *, int32_t, int64_t, hipStream_t);
template int fill<uint32_t>(uint32_t *, uint32_t, int64_t, hipStream_t);
template int fill<u64>(u64 *, u64, int64_t, hipStream_t);
template int fill<int64_t>(int64_t *, int64_t, int64_t, hipStream_t);

int radix_sort_u64(u64 *keys, u64 *alt, int64_t n, int bits, u64 **result, Arena &a,
                   hipStream_t s, int lo) {
  *result = keys;
  if (n <= 1 || bits <= 0) return GC_OK;
  const int64_t ntiles = (n + kRsTile - 1) / kRsTile;
  size_t m = a.mark();
  uint32_t *hist = a.take<uint32_t>((size_t)ntiles * 256);
  if (a.measuring()) {
    GC_TRY(scan_exclusive<uint32_t>(hist, hist, ntiles * 256, a, s));
    a.release(m);
    return GC_OK;
  }
  if (a.overflow) return GC_ENOMEM;
  u64 *src = keys, *dst = alt;
  for (int shift = lo; shift < lo + bits; shift += 8) {
    k_rs_hist<<<(unsigned)ntiles, kRsBlock, 0, s>>>(src, n, shift, hist, ntiles);
    GC_TRY_HIP(hipGetLastError());
    GC_TRY(scan_exclusive<uint32_t>(hist, hist, ntiles * 256, a, s));
    k_rs_scatter<<<(unsigned)ntiles, kRsBlock, 0, s>>>(src, dst, n, shift, hist, ntiles);
    GC_TRY_HIP(hipGetLastError());
    u64 *t = src;
    src = dst;
    dst = t;
  }
  *result = src;
  a.release(m);
  return GC_OK;
}

}  // namespace gc
