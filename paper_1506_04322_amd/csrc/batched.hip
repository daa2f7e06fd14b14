// Many small graphs per launch (graph classification workloads of the
// paper, Section 6: each graph described by its k = 2, 3, 4 counts).
//
// Graphs are binned by size class (64-bit words per adjacency row); each
// class is counted by one persistent grid-stride launch over its graphs,
// costliest first, with the LDS of the largest graph in the class.  A plan
// (classes, order, workgroup size, grids) is made once per batch and its
// launches are captured into a HIP graph that each run replays; the
// autotuner times candidate class sets and workgroup sizes on the batch.
//
// One workgroup per graph.  The graph's adjacency lives in LDS as n rows of
// ceil(n/64) 64-bit words, so Step 1 of the method (Tri_e, Star_u, Star_v of
// every edge, Section 3) is an AND + popcount of two rows.  Step 2 needs only
// the totals here: 4-cliques are listed once each from their lowest edge
// (three rows ANDed), and 4-cycles come from the identity
//   sum_e C4_e = 4 (C4ni - sum_e C(T_e, 2) + 3 K4),
// where C4ni, the number of 4-cycles with chords allowed, is half the sum
// over vertex pairs {a, b} of C(|N(a) n N(b)|, 2) (over all pairs for a dense
// graph, over pairs two steps apart for a sparse one).  Step 3 accumulates the
// unrestricted counts in int64 (every count of a graph with n <= 1024 fits)
// and Step 4 applies the Lemmas of Section 4.3 on the device.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace gc {

namespace {

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

// Registers held for 4 waves per SIMD at 512 threads and 5 at 256 (two
// workgroups of 512 per compute unit when LDS allows).
template <int WORDS, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(BLOCK == 512 ? 4 : 5)))
void k_batched(const int64_t *node_off, const int32_t *rp, const int32_t *col,
               const int32_t *list, int count, int64_t *out, int32_t *err) {
  // row i at R + i * SW: an odd stride (in 64-bit words) spreads the rows
  // that the lanes of a wave read at once over all LDS banks
  constexpr int SW = WORDS | 1;
  extern __shared__ u64 R[];  // n * SW
  __shared__ long long red[BLOCK / kWave][kBAcc];
  __shared__ unsigned long long s_sq;  // sum of squared degrees of the graph
  const int tid = threadIdx.x;
  for (int qi = blockIdx.x; qi < count; qi += gridDim.x) {
    const int64_t gi = list[qi];
    const int64_t r0 = node_off[gi];
    const int n = (int)(node_off[gi + 1] - r0);
    const int words = (n + 63) / 64;
    if (words > WORDS) {  // the batch changed since the plan was made
      if (tid == 0) atomicMin(err, GC_EINVAL);
      continue;
    }
    const int64_t e0 = rp[r0];
    for (int w = tid; w < n * SW; w += BLOCK) R[w] = 0;
    if (tid == 0) s_sq = 0;
    __syncthreads();
    // rows: each row written by one thread
    unsigned long long sq = 0;
    for (int i = tid; i < n; i += BLOCK) {
      u64 *Ri = R + i * SW;
      const int64_t pa = rp[r0 + i], pb = rp[r0 + i + 1];
      for (int64_t p = pa; p < pb; p++) {
        const int j = col[p];
        Ri[j >> 6] |= 1ull << (j & 63);
      }
      sq += (unsigned long long)((pb - pa) * (pb - pa));
    }
    if (sq) atomicAdd(&s_sq, sq);
    __syncthreads();
    long long A[kBAcc];
#pragma unroll
    for (int k = 0; k < kBAcc; k++) A[k] = 0;
    const long long nn = n;
    const long long m = (rp[r0 + n] - e0) / 2;
    // Steps 1-3 per edge (i, j), i < j, one thread per CSR entry.
    const int64_t nnz = rp[r0 + n] - e0;
    for (int64_t t = tid; t < nnz; t += BLOCK) {
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
      const u64 *Ri = R + i * SW, *Rj = R + j * SW;
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
          const u64 *Rk = R + k * SW;
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
    // Only pairs at distance two have c > 0.  A sparse graph takes, for each
    // a, the union of its neighbours' rows (the vertices two steps away, a
    // itself included) and the pairs with b > a in it: about
    // sum_v deg(v)^2 row reads instead of n^2 / 2 (the same sum).
    if (s_sq + (unsigned long long)nnz < (unsigned long long)n * (unsigned long long)n / 2) {
      for (int a = tid; a < n; a += BLOCK) {
        const u64 *Ra = R + a * SW;
        const int64_t pa = rp[r0 + a], pb = rp[r0 + a + 1];
        const int wa = (a + 1) >> 6;
        for (int w = wa; w < words; w++) {  // a word of the union at a time
          u64 t = 0;
          for (int64_t p = pa; p < pb; p++) t |= R[col[p] * SW + w];
          if (w == wa) t &= (~0ull) << ((a + 1) & 63);
          while (t) {
            const int b = (w << 6) + __ffsll((long long)t) - 1;
            t &= t - 1;
            const u64 *Rb = R + b * SW;
            long long c = 0;
            for (int z = 0; z < words; z++) c += __popcll(Ra[z] & Rb[z]);
            A[B_C4NI] += ch2(c);
          }
        }
      }
    } else {
      for (int a = 0; a < n; a++) {
        const u64 *Ra = R + a * SW;
        for (int bb = a + 1 + tid; bb < n; bb += BLOCK) {
          const u64 *Rb = R + bb * SW;
          long long c = 0;
          for (int w = 0; w < words; w++) c += __popcll(Ra[w] & Rb[w]);
          A[B_C4NI] += ch2(c);
        }
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
        for (int w = 0; w < BLOCK / kWave; w++) S[k] += red[w][k];
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


// Graphlet frequency distributions (Section 6.1): per graph and per size k,
// each count over the sum of the counts of that size (all classes, whose sum
// is C(n, k), or the connected ones only).  Counts of graphs with n <= 1024
// are below 2^53, so the operands are exact doubles and the quotient is the
// correctly rounded one.
__global__ void k_batch_gfd(const int64_t *counts, int64_t G, double *out, int connected) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= G) return;
  const int64_t *c = counts + gi * 17;
  double *o = out + gi * 17;
  // [first, end) of each size and the end of its connected classes
  const int lo[3] = {0, 2, 6}, hi[3] = {2, 6, 17}, hc[3] = {1, 4, 12};
  for (int k = 0; k < 3; k++) {
    const int top = connected ? hc[k] : hi[k];
    int64_t sum = 0;
    for (int i = lo[k]; i < top; i++) sum += c[i];
    for (int i = lo[k]; i < hi[k]; i++)
      o[i] = (i < top && sum > 0) ? (double)c[i] / (double)sum : 0.0;
  }
}

__global__ void k_batch_reset(int32_t *err) {
  if (threadIdx.x == 0) *err = 0;
}

__global__ void k_batch_sizes(const int64_t *node_off, const int32_t *rp, int64_t G,
                              int64_t *sizes) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= G) return;
  const int64_t a = node_off[gi], b = node_off[gi + 1];
  sizes[2 * gi] = b - a;
  sizes[2 * gi + 1] = (b >= a) ? (int64_t)rp[b] - rp[a] : -1;
}

// ------------------------------------------------------------------ host

// Size classes: a class of W words holds graphs with at most 64 W vertices.
constexpr int kWords[] = {1, 2, 4, 6, 8, 10, 12, 16};
constexpr int kNumWords = 8;
constexpr int kBlocks[] = {256, 512};

typedef void (*KernelFn)(const int64_t *, const int32_t *, const int32_t *, const int32_t *, int,
                         int64_t *, int32_t *);

template <int BLOCK>
KernelFn kernel_w(int words) {
  switch (words) {
    case 1: return k_batched<1, BLOCK>;
    case 2: return k_batched<2, BLOCK>;
    case 4: return k_batched<4, BLOCK>;
    case 6: return k_batched<6, BLOCK>;
    case 8: return k_batched<8, BLOCK>;
    case 10: return k_batched<10, BLOCK>;
    case 12: return k_batched<12, BLOCK>;
    default: return k_batched<16, BLOCK>;
  }
}

KernelFn kernel_for(int block, int words) {
  return block == 256 ? kernel_w<256>(words) : kernel_w<512>(words);
}

std::string error_text(int code) {
  switch (code) {
    case GC_EOVERFLOW: return "a graph has more than GC_BATCH_MAX_N vertices";
    case GC_EINTERNAL: return "exact identity check failed for a graph of the batch (internal error)";
    case GC_EINVAL: return "batch CSR malformed, or changed since the plan was made";
    default: return "batch CSR contract violated";
  }
}

struct BatchShape {
  int block = 256;
  unsigned classes = 0;  // bit i: a class of kWords[i] words
};

struct ClassLaunch {
  int words = 0, count = 0, offset = 0, grid = 0, per_cu = 0;
  size_t lds = 0;
};

}  // namespace
}  // namespace gc

struct gc_batch_plan {
  gc_batch b{};
  int64_t *out = nullptr;
  gc::BatchShape shape;
  std::vector<gc::ClassLaunch> launches;
  double tuned_ms = 0;
  int candidates = 0;
  std::vector<int64_t> sizes;  // host copy: (n, nnz) per graph
  int32_t *dbuf = nullptr;     // class lists (G ints), then err
  int32_t *err = nullptr;
  int32_t *herr = nullptr;     // pinned (plans), or &hval (one-shot calls)
  int32_t hval = 0;
  bool stream_owned = false;   // dbuf from hipMallocAsync on the call's stream
  bool borrowed = false;       // dbuf is the caller's (not freed with the plan)
  hipStream_t owner = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace gc {
namespace {

std::mutex g_tune_mu;
std::unordered_map<uint64_t, BatchShape> g_tuned;

uint64_t signature(const std::vector<int64_t> &sizes) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    h ^= v;
    h *= 1099511628211ull;
  };
  const size_t G = sizes.size() / 2;
  mix(G);
  uint64_t hist[33] = {0};
  int64_t nnz = 0;
  for (size_t i = 0; i < G; i++) {
    hist[std::min<int64_t>(32, sizes[2 * i] / 32)]++;
    nnz += sizes[2 * i + 1];
  }
  for (uint64_t v : hist) mix(v);
  mix((uint64_t)(nnz >> 16));
  return h;
}

// Estimated work of one graph: row building, per-edge Steps 1-3, the
// all-pairs pass and the 4-clique listing.
double cost_of(int64_t n, int64_t nnz) {
  const double w = (double)((n + 63) / 64);
  // vertex pairs of the 4-cycle pass: all of them, or about sum deg^2 (taken
  // as nnz^2 / n) for a sparse graph
  const double all = 0.5 * (double)n * (double)(n - 1);
  const double pairs =
      std::min(all, n > 0 ? (double)nnz * (double)nnz / (double)n + (double)nnz : 0.0);
  const double rho = n > 1 ? (double)nnz / ((double)n * (double)(n - 1)) : 0.0;
  const double tri = all * (double)(n - 2) / 3.0 * rho * rho * rho;
  return pairs * w + 1.5 * tri * w + (double)nnz * (8.0 + w) + 2000.0;
}

int words_of(int64_t n) { return (int)((n + 63) / 64); }

int max_words(const std::vector<int64_t> &sizes) {
  int mw = 1;
  for (size_t i = 0; i < sizes.size() / 2; i++) mw = std::max(mw, words_of(sizes[2 * i]));
  return mw;
}

// Assigns every graph to the smallest class of the shape that holds it and
// orders each class costliest first; false if no class holds some graph.
bool layout(gc_batch_plan *p, const BatchShape &sh, std::vector<int32_t> *order) {
  const int64_t G = p->b.graphs;
  std::vector<std::vector<std::pair<double, int32_t>>> bins(kNumWords);
  std::vector<int64_t> nmax(kNumWords, 0);
  for (int64_t i = 0; i < G; i++) {
    const int64_t n = p->sizes[2 * i], nnz = p->sizes[2 * i + 1];
    const int w = words_of(n);
    int c = -1;
    for (int k = 0; k < kNumWords; k++)
      if ((sh.classes >> k & 1u) && kWords[k] >= w) {
        c = k;
        break;
      }
    if (c < 0) return false;
    bins[c].push_back({cost_of(n, nnz), (int32_t)i});
    nmax[c] = std::max(nmax[c], n);
  }
  auto desc = [](const std::pair<double, int32_t> &x, const std::pair<double, int32_t> &y) {
    return x.first > y.first || (x.first == y.first && x.second < y.second);
  };
  order->clear();
  std::vector<ClassLaunch> L;
  for (int k = 0; k < kNumWords; k++) {
    if (bins[k].empty()) continue;
    std::sort(bins[k].begin(), bins[k].end(), desc);
    ClassLaunch c;
    c.words = kWords[k];
    c.count = (int)bins[k].size();
    c.offset = (int)order->size();
    c.lds = std::max<size_t>((size_t)nmax[k] * (kWords[k] | 1) * sizeof(u64), 8);  // odd row stride
    for (auto &x : bins[k]) order->push_back(x.second);
    L.push_back(c);
  }
  p->shape = sh;
  p->launches.swap(L);
  return true;
}

int drop_graph(gc_batch_plan *p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  return GC_OK;
}

// Error reset, then one launch per class.
hipError_t launch(gc_batch_plan *p, hipStream_t s) {
  k_batch_reset<<<1, 64, 0, s>>>(p->err);
  hipError_t e = hipGetLastError();
  for (const ClassLaunch &c : p->launches) {
    if (e != hipSuccess) break;
    KernelFn k = kernel_for(p->shape.block, c.words);
    k<<<c.grid, p->shape.block, c.lds, s>>>(p->b.node_off, p->b.row_ptr, p->b.col,
                                            p->dbuf + c.offset, c.count, p->out, p->err);
    e = hipGetLastError();
  }
  return e;
}

// Uploads the class lists, sizes each persistent grid and, with `capture`,
// records the launches into a HIP graph.
int prepare(gc_batch_plan *p, const std::vector<int32_t> &order, hipStream_t s, bool capture) {
  drop_graph(p);
  const int64_t G = p->b.graphs;
  GC_TRY_HIP(hipMemcpyAsync(p->dbuf, order.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, s));
  GC_TRY_HIP(hipStreamSynchronize(s));
  int dev = 0, cus = 0;
  GC_TRY_HIP(hipGetDevice(&dev));
  GC_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  for (ClassLaunch &c : p->launches) {
    KernelFn k = kernel_for(p->shape.block, c.words);
    GC_TRY_HIP(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)c.lds));
    int per_cu = 0;
    GC_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k,
                                                            p->shape.block, c.lds));
    if (per_cu <= 0) {
      set_error("batched kernel does not fit on a compute unit (LDS %zu bytes)", c.lds);
      return GC_ENOMEM;
    }
    c.per_cu = per_cu;
    c.grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)per_cu * cus, c.count));
  }
  if (!capture) return GC_OK;
  hipStream_t cs = nullptr;
  GC_TRY_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t e1 = launch(p, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &p->graph);
    e = e1 != hipSuccess ? e1 : e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    drop_graph(p);
    set_error("batched graph capture: %s", hipGetErrorString(e));
    return GC_EHIP;
  }
  return GC_OK;
}

int run_plan(gc_batch_plan *p, hipStream_t s) {
  if (p->b.graphs == 0) return GC_OK;
  if (p->exec) GC_TRY_HIP(hipGraphLaunch(p->exec, s));
  else GC_TRY_HIP(launch(p, s));
  GC_TRY_HIP(hipMemcpyAsync(p->herr, p->err, 4, hipMemcpyDeviceToHost, s));
  GC_TRY_HIP(hipStreamSynchronize(s));
  const int h = *p->herr;
  if (h != 0) {
    set_error("%s", error_text(h).c_str());
    return h;
  }
  return GC_OK;
}

int time_plan(gc_batch_plan *p, hipStream_t s, double *ms) {
  hipEvent_t a, b;
  GC_TRY_HIP(hipEventCreate(&a));
  GC_TRY_HIP(hipEventCreate(&b));
  int rc = run_plan(p, s);
  double best = 1e30;
  for (int it = 0; it < 3 && rc == GC_OK; it++) {
    hipError_t e = hipEventRecord(a, s);
    if (e == hipSuccess) e = p->exec ? hipGraphLaunch(p->exec, s) : launch(p, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (e != hipSuccess) {
      set_error("batched timing: %s", hipGetErrorString(e));
      rc = GC_EHIP;
    }
    best = std::min(best, (double)t);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = best;
  return rc;
}

}  // namespace

// Validates a batch (GC_VALIDATE: the full CSR contract of every graph) and
// returns, per graph, its vertex count and its adjacency-list length.  Shared
// with the batched per-vertex entry point.
int check_batch(const gc_batch *b, int64_t *out, hipStream_t s, uint32_t flags,
                std::vector<int64_t> *sizes, int32_t *err_buf, int64_t *sizes_buf) {
  if (!b || b->graphs < 0 || b->graphs > (1ll << 30) ||
      (b->graphs > 0 && (!b->node_off || !b->row_ptr || !out))) {
    set_error("invalid batch arguments");
    return GC_EINVAL;
  }
  const int64_t G = b->graphs;
  sizes->assign(2 * G, 0);
  if (G == 0) return GC_OK;
  // the caller's buffers (the allocation-free entry point), else stream-ordered ones
  const bool own = err_buf == nullptr;
  int32_t *err = err_buf;
  int64_t *dsz = sizes_buf;
  hipError_t e = hipSuccess;
  if (own) {
    GC_TRY_HIP(hipMallocAsync((void **)&err, 4, s));
    e = hipMallocAsync((void **)&dsz, sizeof(int64_t) * 2 * G, s);
  }
  int32_t h = 0;
  if (e == hipSuccess) {
    k_batch_reset<<<1, 64, 0, s>>>(err);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const unsigned grid = (unsigned)((G + 255) / 256);
    k_batch_check<<<grid, 256, 0, s>>>(b->node_off, b->row_ptr, b->col, G,
                                       (flags & GC_VALIDATE) ? 1 : 0, err);
    k_batch_sizes<<<grid, 256, 0, s>>>(b->node_off, b->row_ptr, G, dsz);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&h, err, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sizes->data(), dsz, sizeof(int64_t) * 2 * G, hipMemcpyDeviceToHost, s);
  if (own) {
    if (dsz) (void)hipFreeAsync(dsz, s);
    (void)hipFreeAsync(err, s);
  }
  hipError_t f = hipStreamSynchronize(s);
  if (e == hipSuccess) e = f;
  if (e != hipSuccess) {
    set_error("batched: %s", hipGetErrorString(e));
    return GC_EHIP;
  }
  if (h != 0) {
    const int code = -(__builtin_ffs(h) - 1);
    set_error("%s", error_text(code).c_str());
    return code;
  }
  return GC_OK;
}

namespace {

void destroy_plan(gc_batch_plan *p) {
  if (!p) return;
  drop_graph(p);
  if (p->borrowed) {
    // nothing of the plan's own on the device
  } else if (p->stream_owned) {
    if (p->dbuf) (void)hipFreeAsync(p->dbuf, p->owner);
  } else {
    if (p->dbuf) (void)hipFree(p->dbuf);
    if (p->herr) (void)hipHostFree(p->herr);
  }
  delete p;
}

// Candidate class sets: one class for everything (a single launch), or
// classes at every power-of-two-ish step up to the largest graph.
std::vector<unsigned> class_sets(int mw) {
  int top = 0;
  while (top < kNumWords - 1 && kWords[top] < mw) top++;
  const unsigned topbit = 1u << top;
  std::vector<unsigned> sets = {topbit};
  const unsigned masks[] = {0x04u /*4*/, 0x05u /*1,4*/, 0x24u /*4,10*/, 0x14u /*4,8*/,
                            0x2Au /*2,6,10*/, 0xFFu /*all*/};
  for (unsigned m : masks) {
    const unsigned s = (m & (topbit - 1)) | topbit;
    if (std::find(sets.begin(), sets.end(), s) == sets.end()) sets.push_back(s);
  }
  return sets;
}

// Classes of 4 and 10 words and one for the largest graphs.
BatchShape default_shape(int mw) {
  int top = 0;
  while (top < kNumWords - 1 && kWords[top] < mw) top++;
  const unsigned topbit = 1u << top;
  return BatchShape{256, (0x24u & (topbit - 1)) | topbit};
}

// Device buffers a call brings in instead of allocating: the error word, the
// per-graph sizes (2 G int64) and the class lists (G + 8 int32).
struct BatchScratch {
  int32_t *err;
  int64_t *sizes;
  int32_t *dbuf;
};

int create_plan(const gc_batch *b, int64_t *out, int tune, bool capture, hipStream_t s,
                uint32_t flags, gc_batch_plan **result, const BatchScratch *bs = nullptr) {
  if (!result) {
    set_error("null plan pointer");
    return GC_EINVAL;
  }
  *result = nullptr;
  std::vector<int64_t> sizes;
  GC_TRY(check_batch(b, out, s, flags, &sizes, bs ? bs->err : nullptr, bs ? bs->sizes : nullptr));
  gc_batch_plan *p = new (std::nothrow) gc_batch_plan();
  if (!p) return GC_ENOMEM;
  p->b = *b;
  p->out = out;
  p->sizes.swap(sizes);
  const int64_t G = b->graphs;
  hipError_t e;
  if (bs) {  // one call on the caller's scratch: nothing allocated
    p->borrowed = true;
    p->herr = &p->hval;
    p->dbuf = bs->dbuf;
    e = hipSuccess;
  } else if (capture) {
    e = hipMalloc((void **)&p->dbuf, sizeof(int32_t) * (G + 8));
    if (e == hipSuccess) e = hipHostMalloc((void **)&p->herr, 64, hipHostMallocDefault);
  } else {  // one call: stream-ordered scratch, freed when the call ends
    p->stream_owned = true;
    p->owner = s;
    p->herr = &p->hval;
    e = hipMallocAsync((void **)&p->dbuf, sizeof(int32_t) * (G + 8), s);
  }
  if (e != hipSuccess) {
    destroy_plan(p);
    set_error("batched plan allocation: %s", hipGetErrorString(e));
    return GC_ENOMEM;
  }
  p->err = p->dbuf + ((G + 1) & ~int64_t(1));
  if (G == 0) {
    *result = p;
    return GC_OK;
  }
  const int mw = max_words(p->sizes);
  const uint64_t sig = signature(p->sizes);
  BatchShape sh = default_shape(mw);
  bool known = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(sig);
    if (it != g_tuned.end()) {
      sh = it->second;
      known = true;
    }
  }
  std::vector<int32_t> order;
  int rc = GC_OK;
  if (tune && !known) {
    double best = 1e30;
    BatchShape best_sh = sh;
    bool any = false;
    for (int blk : kBlocks)
      for (unsigned cls : class_sets(mw)) {
        BatchShape c{blk, cls};
        if (!layout(p, c, &order)) continue;
        rc = prepare(p, order, s, true);
        double ms = 0;
        if (rc == GC_OK) rc = time_plan(p, s, &ms);
        if (rc != GC_OK) break;
        p->candidates++;
        if (ms < best) {
          best = ms;
          best_sh = c;
          any = true;
        }
      }
    if (rc == GC_OK && any) {
      sh = best_sh;
      p->tuned_ms = best;
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tuned[sig] = sh;
    }
  }
  if (rc == GC_OK && !layout(p, sh, &order)) {
    set_error("no size class holds the largest graph of the batch");
    rc = GC_EINTERNAL;
  }
  if (rc == GC_OK) rc = prepare(p, order, s, capture);
  if (rc != GC_OK) {
    destroy_plan(p);
    return rc;
  }
  *result = p;
  return GC_OK;
}

}  // namespace
}  // namespace gc

// Scratch of graphlet_count_batched_noalloc, one copy per device (each GPU the
// library runs on holds it until the process ends): the error word (padded to
// 256 bytes), then (n, nnz) of each graph, then the class-ordered graph list.
constexpr size_t kNaErrBytes = 256;
constexpr size_t kNaSizesBytes = sizeof(int64_t) * 2 * GC_NOALLOC_MAX_GRAPHS;
constexpr size_t kNaListBytes = sizeof(int32_t) * (GC_NOALLOC_MAX_GRAPHS + 8);
constexpr size_t kNaBytes = kNaErrBytes + kNaSizesBytes + kNaListBytes;
static_assert(kNaSizesBytes % 256 == 0, "list stays aligned");
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace gc {
namespace {

constexpr int kNaMaxDevices = 64;
// Per device: the device address of `scratch` (host code never uses the
// array's own name, a host-side stand-in) and the lock that makes calls on
// that device take turns with the array.
unsigned char *g_na_ptr[kNaMaxDevices];
std::mutex g_na_mu[kNaMaxDevices];

}  // namespace
}  // namespace gc

extern "C" {

int graphlet_batch_plan_create(const gc_batch *b, int64_t *out, int tune, void *stream,
                               uint32_t flags, gc_batch_plan **plan) {
  gc::clear_error();
  try {
    return gc::create_plan(b, out, tune, true, (hipStream_t)stream, flags, plan);
  } catch (...) {
    gc::set_error("unexpected exception");
    return GC_EINTERNAL;
  }
}

int graphlet_batch_plan_run(gc_batch_plan *p, void *stream) {
  gc::clear_error();
  if (!p) {
    gc::set_error("null plan");
    return GC_EINVAL;
  }
  return gc::run_plan(p, (hipStream_t)stream);
}

int graphlet_batch_plan_info(const gc_batch_plan *p, gc_batch_plan_info *o) {
  gc::clear_error();
  if (!p || !o) {
    gc::set_error("null argument");
    return GC_EINVAL;
  }
  std::memset(o, 0, sizeof(*o));
  o->block = p->shape.block;
  o->classes = (int)p->launches.size();
  for (size_t i = 0; i < p->launches.size() && i < 8; i++) {
    o->class_words[i] = p->launches[i].words;
    o->class_graphs[i] = p->launches[i].count;
    o->class_grid[i] = p->launches[i].grid;
    o->class_lds[i] = p->launches[i].lds;
  }
  o->candidates = p->candidates;
  o->tuned_ms = p->tuned_ms;
  return GC_OK;
}

int graphlet_batch_plan_reshape(gc_batch_plan *p, int block, uint32_t class_words_mask,
                                void *stream) {
  gc::clear_error();
  if (!p || (block != 256 && block != 512)) {
    gc::set_error("block must be 256 or 512");
    return GC_EINVAL;
  }
  if (p->b.graphs == 0) return GC_OK;
  try {
    // the batch may hold new graphs of other sizes: re-read them
    int rc = gc::check_batch(&p->b, p->out, (hipStream_t)stream, 0, &p->sizes, nullptr, nullptr);
    if (rc != GC_OK) return rc;
    unsigned cls = 0;
    for (int k = 0; k < gc::kNumWords; k++)
      if (class_words_mask >> (gc::kWords[k] - 1) & 1u) cls |= 1u << k;
    std::vector<int32_t> order;
    if (cls == 0 || !gc::layout(p, gc::BatchShape{block, cls}, &order)) {
      gc::set_error("the classes do not hold every graph of the batch");
      return GC_EINVAL;
    }
    return gc::prepare(p, order, (hipStream_t)stream, true);
  } catch (...) {
    gc::set_error("unexpected exception");
    return GC_EINTERNAL;
  }
}

void graphlet_batch_plan_destroy(gc_batch_plan *p) { gc::destroy_plan(p); }

int graphlet_batch_gfd(const int64_t *counts, int64_t graphs, double *out, int connected_only,
                       void *stream) {
  gc::clear_error();
  if (graphs < 0 || (graphs > 0 && (!counts || !out))) {
    gc::set_error("invalid arguments");
    return GC_EINVAL;
  }
  if (graphs == 0) return GC_OK;
  hipStream_t s = (hipStream_t)stream;
  gc::k_batch_gfd<<<(unsigned)((graphs + 255) / 256), 256, 0, s>>>(counts, graphs, out,
                                                                  connected_only ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    gc::set_error("gfd: %s", hipGetErrorString(e));
    return GC_EHIP;
  }
  return GC_OK;
}

int graphlet_count_batched(const gc_batch *b, int64_t *out, void *stream, uint32_t flags) {
  gc::clear_error();
  try {
    gc_batch_plan *p = nullptr;
    int rc = gc::create_plan(b, out, 0, false, (hipStream_t)stream, flags, &p);
    if (rc != GC_OK) return rc;
    rc = gc::run_plan(p, (hipStream_t)stream);
    gc::destroy_plan(p);
    return rc;
  } catch (...) {
    gc::set_error("unexpected exception");
    return GC_EINTERNAL;
  }
}


int graphlet_count_batched_noalloc(const gc_batch *b, int64_t *out, void *stream,
                                   uint32_t flags) {
  gc::clear_error();
  if (!b) {
    gc::set_error("invalid batch arguments");
    return GC_EINVAL;
  }
  if (b->graphs > GC_NOALLOC_MAX_GRAPHS) {
    gc::set_error("batch of %lld graphs exceeds the allocation-free limit of %d graphs",
                  (long long)b->graphs, GC_NOALLOC_MAX_GRAPHS);
    return GC_EINVAL;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    gc::set_error("hipGetDevice: %s", hipGetErrorString(e));
    return GC_EHIP;
  }
  if (dev < 0 || dev >= gc::kNaMaxDevices) {
    gc::set_error("device %d beyond the allocation-free entry point's %d devices", dev,
                  gc::kNaMaxDevices);
    return GC_EINVAL;
  }
  try {
    std::lock_guard<std::mutex> lk(gc::g_na_mu[dev]);
    if (!gc::g_na_ptr[dev]) {  // first call on this device, which is current
      unsigned char *ptr = nullptr;
      e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        gc::set_error("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        return GC_EHIP;
      }
      gc::g_na_ptr[dev] = ptr;
    }
    unsigned char *base = gc::g_na_ptr[dev];
    gc::BatchScratch bs;
    bs.err = reinterpret_cast<int32_t *>(base);
    bs.sizes = reinterpret_cast<int64_t *>(base + kNaErrBytes);
    bs.dbuf = reinterpret_cast<int32_t *>(base + kNaErrBytes + kNaSizesBytes);
    const hipStream_t s = (hipStream_t)stream;
    gc_batch_plan *p = nullptr;
    int rc = gc::create_plan(b, out, 0, false, s, flags, &p, &bs);
    if (rc != GC_OK) return rc;
    rc = gc::run_plan(p, s);
    gc::destroy_plan(p);
    return rc;
  } catch (...) {
    gc::set_error("unexpected exception");
    return GC_EINTERNAL;
  }
}

}  // extern "C"
