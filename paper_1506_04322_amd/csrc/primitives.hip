// Device-wide scan and radix sort used by the prepass (relabelling by degree).
#include "primitives.h"

namespace gc {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanIpt = 8;
constexpr int kScanTile = kScanBlock * kScanIpt;

// A tile of kScanTile elements, kScanIpt consecutive ones per thread: the
// thread totals are scanned within each wave by shuffles, the wave totals
// through LDS after one barrier.
template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_tile(const T *in, T *out, T *sums, int64_t n) {
  __shared__ T wsum[kScanBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIpt;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  T v[kScanIpt];
  T tot = 0;
#pragma unroll
  for (int k = 0; k < kScanIpt; k++) {
    int64_t i = base + k;
    v[k] = i < n ? in[i] : T(0);
    tot += v[k];
  }
  T incl = tot;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const T t = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += t;
  }
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kScanBlock / kWave; w++) {
    if (w < wave) before += wsum[w];
    all += wsum[w];
  }
  T run = before + incl - tot;
  if (threadIdx.x == kScanBlock - 1 && sums) sums[blockIdx.x] = all;
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

// Stable scatter: keys of a tile keep their order within a digit.  The tile
// is first put in digit order in LDS: a key's place is the tile's start of
// its digit, plus the keys of that digit in earlier rounds of 256 (a running
// count), in lower waves and in lower lanes of its own wave (eight ballots).
// Then the tile is written out in that order, so that consecutive threads
// write consecutive addresses within each digit's run.
__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(const u64 *in, u64 *out, int64_t n,
                                                         int shift, const uint32_t *offs,
                                                         int64_t ntiles) {
  __shared__ u64 stage[kRsTile];
  __shared__ uint32_t run[256], lstart[256], goff[256];
  __shared__ uint32_t wcnt[kRsBlock / kWave][256];
  const int tid = threadIdx.x, wave = tid / kWave;
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  const int cnt = (int)(n - base < kRsTile ? n - base : kRsTile);
  goff[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
  run[tid] = 0;
  __syncthreads();
  u64 key[kRsIpt];
#pragma unroll
  for (int r = 0; r < kRsIpt; r++) {
    const int i = r * kRsBlock + tid;
    key[r] = i < cnt ? in[base + i] : 0ull;
    if (i < cnt) atomicAdd(&run[(uint32_t)(key[r] >> shift) & 255u], 1u);
  }
  __syncthreads();
  // the tile's start of each digit: an exclusive scan of its counts
  {
    const uint32_t c = run[tid];
    uint32_t incl = c;
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t t = __shfl_up(incl, off, kWave);
      if (lane_id() >= off) incl += t;
    }
    if (lane_id() == kWave - 1) wcnt[0][wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; w++) before += wcnt[0][w];
    lstart[tid] = before + incl - c;
    run[tid] = before + incl - c;  // running place of the next key of each digit
    __syncthreads();
  }
  const u64 lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < kRsIpt; r++) {
#pragma unroll
    for (int w = 0; w < kRsBlock / kWave; w++) wcnt[w][tid] = 0;
    __syncthreads();
    const int i = r * kRsBlock + tid;
    const bool valid = i < cnt;
    const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
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
        const uint32_t c = wcnt[w][tid];
        wcnt[w][tid] = acc;
        acc += c;
      }
      run[tid] = acc;
    }
    __syncthreads();
    if (valid) stage[wcnt[wave][d] + lrank] = key[r];
    __syncthreads();  // wcnt is cleared by the next round
  }
  for (int i = tid; i < cnt; i += kRsBlock) {
    const u64 k = stage[i];
    const uint32_t d = (uint32_t)(k >> shift) & 255u;
    out[goff[d] + (i - lstart[d])] = k;
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
