// Many small graphs in one launch (graph classification workloads of the
// paper, Section 6: each graph described by its k = 2, 3, 4 counts).
//
// One workgroup per graph.  The graph's adjacency lives in LDS as n rows of
// ceil(n/64) 64-bit words, so Step 1 of the method (Tri_e, Star_u, Star_v of
// every edge, Section 3) is an AND + popcount of two rows.  Step 2 needs only
// the totals here: 4-cliques are listed once each from their lowest edge
// (three rows ANDed), and 4-cycles come from the identity
//   sum_e C4_e = 4 (C4ni - sum_e C(T_e, 2) + 3 K4),
// where C4ni, the number of 4-cycles with chords allowed, is half the sum
// over vertex pairs {a, b} of C(|N(a) n N(b)|, 2).  Step 3 accumulates the
// unrestricted counts in int64 (every count of a graph with n <= 1024 fits)
// and Step 4 applies the Lemmas of Section 4.3 on the device.
#include <algorithm>
#include <vector>

#include "common.h"
#include "primitives.h"

namespace gc {

int batched(const gc_batch *b, int64_t *out, hipStream_t s, uint32_t flags);

namespace {

constexpr int kBBlock = 256;
constexpr int kBAcc = 15;  // 11 unrestricted sums + K4 + C4ni + T check + error

enum BAcc {
  B_T = 0, B_S, B_I, B_TT, B_SUSV, B_TS, B_SS, B_TI, B_SI, B_II, B_II1, B_K4, B_C4NI, B_ERR
};

__device__ __forceinline__ long long ch2(long long c) { return c * (c - 1) / 2; }

__device__ bool exact(long long a, long long d, long long *q) {
  if (a % d != 0) return false;
  *q = a / d;
  return true;
}

// Step 4 in int64 for one graph; returns false on a remainder or a negative count.
__device__ bool finalize_i64(const long long *A, long long n, long long m, long long *g) {
  const long long c2 = n * (n - 1) / 2;
  const long long c3 = n >= 3 ? c2 * (n - 2) / 3 : 0;
  const long long c4 = n >= 4 ? c3 * (n - 3) / 4 : 0;
  g[0] = m;
  g[1] = c2 - m;
  if (!exact(A[B_T], 3, &g[2])) return false;
  if (!exact(A[B_S], 2, &g[3])) return false;
  g[4] = A[B_I];
  g[5] = c3 - g[2] - g[3] - g[4];
  g[6] = A[B_K4];
  g[7] = A[B_TT] - 6 * g[6];
  g[9] = A[B_C4NI] - A[B_TT] + 3 * g[6];  // sum_e C4_e / 4
  g[11] = A[B_SUSV] - 4 * g[9];
  if (!exact(A[B_TS] - 4 * g[7], 2, &g[8])) return false;
  if (!exact(A[B_SS] - g[8], 3, &g[10])) return false;
  if (!exact(A[B_TI] - g[8], 3, &g[12])) return false;
  if (!exact(A[B_SI] - 2 * g[11], 2, &g[13])) return false;
  long long t = A[B_II1] - (6 * g[6] + 4 * g[7] + 2 * g[8]) - (4 * g[9] + 2 * g[11]);
  if (!exact(t, 2, &g[14])) return false;
  g[15] = A[B_II] - 2 * g[14];
  t = 0;
  for (int i = 6; i <= 15; i++) t += g[i];
  g[16] = c4 - t;
  for (int i = 0; i < 17; i++)
    if (g[i] < 0) return false;
  return true;
}

template <int WORDS>
__global__ __launch_bounds__(kBBlock) void k_batched(const int64_t *node_off, const int32_t *rp,
                                                     const int32_t *col, int64_t G, int nmin_words,
                                                     int64_t *out, int32_t *err) {
  extern __shared__ u64 R[];  // n * WORDS
  __shared__ long long red[kBBlock / kWave][kBAcc];
  const int tid = threadIdx.x;
  for (int64_t gi = blockIdx.x; gi < G; gi += gridDim.x) {
    const int64_t r0 = node_off[gi];
    const int n = (int)(node_off[gi + 1] - r0);
    const int words = (n + 63) / 64;
    if (words > WORDS || words < nmin_words) continue;  // another size class takes it
    const int64_t e0 = rp[r0];
    for (int w = tid; w < n * WORDS; w += kBBlock) R[w] = 0;
    __syncthreads();
    // rows: each row written by one thread
    for (int i = tid; i < n; i += kBBlock) {
      u64 *Ri = R + i * WORDS;
      for (int64_t p = rp[r0 + i]; p < rp[r0 + i + 1]; p++) {
        const int j = col[p];
        Ri[j >> 6] |= 1ull << (j & 63);
      }
    }
    __syncthreads();
    long long A[kBAcc];
#pragma unroll
    for (int k = 0; k < kBAcc; k++) A[k] = 0;
    const long long nn = n;
    const long long m = (rp[r0 + n] - e0) / 2;
    // Steps 1-3 per edge (i, j), i < j, one thread per CSR entry.
    const int64_t nnz = rp[r0 + n] - e0;
    for (int64_t t = tid; t < nnz; t += kBBlock) {
      const int64_t p = e0 + t;
      const int j = col[p];
      // row of entry p
      int lo = 0, hi = n;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (rp[r0 + mid + 1] <= p) lo = mid + 1;
        else hi = mid;
      }
      const int i = lo;
      if (j <= i) continue;
      const u64 *Ri = R + i * WORDS, *Rj = R + j * WORDS;
      long long T = 0;
      for (int w = 0; w < words; w++) T += __popcll(Ri[w] & Rj[w]);
      const long long du = rp[r0 + i + 1] - rp[r0 + i], dv = rp[r0 + j + 1] - rp[r0 + j];
      const long long Su = du - 1 - T, Sv = dv - 1 - T, S = Su + Sv;
      const long long I = nn - du - dv + T;
      A[B_T] += T;
      A[B_S] += S;
      A[B_I] += I;
      A[B_TT] += ch2(T);
      A[B_SUSV] += Su * Sv;
      A[B_TS] += T * S;
      A[B_SS] += ch2(Su) + ch2(Sv);
      A[B_TI] += T * I;
      A[B_SI] += S * I;
      A[B_II] += I > 0 ? ch2(I) : 0;
      A[B_II1] += m - du - dv + 1;
      // 4-cliques {i, j, k, l} with i < j < k < l, found from edge (i, j)
      for (int w = (j + 1) >> 6; w < words; w++) {
        u64 tri = Ri[w] & Rj[w];
        if (w == ((j + 1) >> 6)) tri &= (~0ull) << ((j + 1) & 63);
        while (tri) {
          const int k = (w << 6) + __ffsll((long long)tri) - 1;
          tri &= tri - 1;
          const u64 *Rk = R + k * WORDS;
          for (int z = (k + 1) >> 6; z < words; z++) {
            u64 q = Ri[z] & Rj[z] & Rk[z];
            if (z == ((k + 1) >> 6)) q &= (~0ull) << ((k + 1) & 63);
            A[B_K4] += __popcll(q);
          }
        }
      }
    }
    // 4-cycles with chords allowed: pairs {a, b} with c common neighbours
    // close C(c, 2) cycles on the diagonal a-b; each cycle has two diagonals.
    for (int a = 0; a < n; a++) {
      const u64 *Ra = R + a * WORDS;
      for (int bb = a + 1 + tid; bb < n; bb += kBBlock) {
        const u64 *Rb = R + bb * WORDS;
        long long c = 0;
        for (int w = 0; w < words; w++) c += __popcll(Ra[w] & Rb[w]);
        A[B_C4NI] += ch2(c);
      }
    }
    // block reduction
#pragma unroll
    for (int k = 0; k < kBAcc; k++) {
      long long v = A[k];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
      if (lane_id() == 0) red[tid / kWave][k] = v;
    }
    __syncthreads();
    if (tid == 0) {
      long long S[kBAcc];
      for (int k = 0; k < kBAcc; k++) {
        S[k] = 0;
        for (int w = 0; w < kBBlock / kWave; w++) S[k] += red[w][k];
      }
      if (S[B_C4NI] % 2 != 0) atomicMin(err, GC_EINTERNAL);
      S[B_C4NI] /= 2;
      long long g[17];
      if (!finalize_i64(S, nn, m, g)) {
        atomicMin(err, GC_EINTERNAL);
        for (int k = 0; k < 17; k++) out[gi * 17 + k] = -1;
      } else {
        for (int k = 0; k < 17; k++) out[gi * 17 + k] = g[k];
      }
    }
    __syncthreads();
  }
}

// Sets bit (-code) of *err per violation; the host reports the lowest bit.
__device__ __forceinline__ void bflag(int32_t *err, int code) { atomicOr(err, 1 << (-code)); }

__global__ void k_batch_check(const int64_t *node_off, const int32_t *rp, const int32_t *col,
                              int64_t G, int validate, int32_t *err) {
  int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= G) return;
  const int64_t a = node_off[gi], b = node_off[gi + 1];
  if (b < a) {
    bflag(err, GC_EINVAL);
    return;
  }
  if (b - a > GC_BATCH_MAX_N) {
    bflag(err, GC_EOVERFLOW);
    return;
  }
  if (!validate) return;
  const int n = (int)(b - a);
  for (int i = 0; i < n; i++) {
    const int32_t p0 = rp[a + i], p1 = rp[a + i + 1];
    if (p1 < p0) {
      bflag(err, GC_EINVAL);
      return;
    }
    for (int32_t p = p0; p < p1; p++) {
      const int j = col[p];
      if (j < 0 || j >= n) {
        bflag(err, GC_EASYMMETRIC);
        return;
      }
      if (j == i) bflag(err, GC_ESELFLOOP);
      if (p > p0 && col[p - 1] >= j) bflag(err, GC_ENOTSORTED);
      const int32_t q0 = rp[a + j], q1 = rp[a + j + 1];
      int lo = q0, hi = q1;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (col[mid] < i) lo = mid + 1;
        else hi = mid;
      }
      if (lo >= q1 || col[lo] != i) bflag(err, GC_EASYMMETRIC);
    }
  }
}

}  // namespace

int batched(const gc_batch *b, int64_t *out, hipStream_t s, uint32_t flags) {
  if (!b || b->graphs < 0 || (b->graphs > 0 && (!b->node_off || !b->row_ptr || !out))) {
    set_error("invalid batch arguments");
    return GC_EINVAL;
  }
  const int64_t G = b->graphs;
  if (G == 0) return GC_OK;
  int32_t *err = nullptr;
  GC_TRY_HIP(hipMallocAsync((void **)&err, 4, s));
  int32_t h = 0;
  hipError_t e = hipMemcpyAsync(err, &h, 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    k_batch_check<<<(unsigned)((G + 255) / 256), 256, 0, s>>>(b->node_off, b->row_ptr, b->col, G,
                                                              (flags & GC_VALIDATE) ? 1 : 0, err);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&h, err, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && h != 0) {
    (void)hipFreeAsync(err, s);
    const int code = -(__builtin_ffs(h) - 1);
    if (code == GC_EOVERFLOW) set_error("a graph has more than GC_BATCH_MAX_N vertices");
    else set_error("batch CSR contract violated (code %d)", code);
    return code;
  }
  static bool attr_set = false;
  if (e == hipSuccess && !attr_set) {
    e = hipFuncSetAttribute((const void *)k_batched<10>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, 640 * 10 * 8);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void *)k_batched<16>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 1024 * 16 * 8);
    attr_set = e == hipSuccess;
  }
  if (e == hipSuccess) {
    const unsigned grid = (unsigned)std::min<int64_t>(G, 65536);
    // three size classes by words per row: <= 4 (n <= 256), <= 10 (n <= 640), <= 16
    k_batched<4><<<grid, kBBlock, 256 * 4 * sizeof(u64), s>>>(b->node_off, b->row_ptr, b->col, G,
                                                              0, out, err);
    k_batched<10><<<grid, kBBlock, 640 * 10 * sizeof(u64), s>>>(b->node_off, b->row_ptr, b->col,
                                                                G, 5, out, err);
    k_batched<16><<<grid, kBBlock, 1024 * 16 * sizeof(u64), s>>>(b->node_off, b->row_ptr, b->col,
                                                                 G, 11, out, err);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&h, err, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipError_t f = hipFreeAsync(err, s);
  if (e == hipSuccess) e = f;
  if (e != hipSuccess) {
    set_error("batched: %s", hipGetErrorString(e));
    return GC_EHIP;
  }
  if (h != 0) {
    set_error("exact identity check failed for a graph of the batch (internal error)");
    return h;
  }
  return GC_OK;
}

}  // namespace gc

extern "C" int graphlet_count_batched(const gc_batch *b, int64_t *out, void *stream,
                                      uint32_t flags) {
  gc::clear_error();
  try {
    return gc::batched(b, out, (hipStream_t)stream, flags);
  } catch (...) {
    gc::set_error("unexpected exception");
    return GC_EINTERNAL;
  }
}
