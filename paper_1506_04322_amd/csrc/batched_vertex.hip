// Per-vertex counts of every graph of a batch: the node-level counts of the
// single-graph path (for each vertex, the k-subsets containing it by class)
// for the many small graphs of graph classification (Section 6).
//
// One workgroup per graph, its adjacency as LDS bitmap rows.  The per-edge
// K4, C4, D and B terms enter a vertex's counts only through their sums over
// its edges, and those sums reduce to quantities that are cheap on bitmaps:
//   sum_e B_e  = sum_{w in N(v)} deg(w) |Tri_(v,w)|
//   sum_e D_e  = sum_e |Tri_e|^2 + 2 OPP(v) - 4 t_v,  OPP(v) = the sum of
//                |Tri_(w,a)| over the triangles {v, w, a} at v (the edge
//                opposite v)
//   sum_e K4_e = 3 (4-cliques at v)
//   sum_e C4_e = 2 Q(v) - sum_e D_e + 2 sum_e K4_e,  Q(v) = the 4-cycles
//                through v, induced or not = sum_{x != v} C(|N(v) & N(x)|, 2)
// (the non-induced 4-cycles through an edge are its induced ones plus the
// chorded ones, D_e - 2 K4_e).  Passes:
//   1. per undirected edge e = (v, w), v < w (a wave per row v, a lane per
//      edge): |Tri_e| and the other end's degree added to both ends' sums,
//      |Tri_e| added to OPP of every member of Tri_e, and the 4-cliques
//      whose two smallest vertices are v and w (the edges inside M = Tri_e
//      above w) credited to their four vertices: x in M is in |N(x) & M| of
//      them, v and w in half the sum; every triangle is visited once, at its
//      two smallest vertices
//   2. per vertex, over all x: c = |N(v) & N(x)| (x adjacent: the edge terms
//      of (v, x); any x != v: Q(v)); then the per-vertex algebra shared with
//      the single-graph kernel.
// Graphs are binned by row width (64-bit words) into classes, one launch per
// class with the LDS of its largest graph; workgroups take the graphs of a
// class costliest first from a counter.  Row reads load the class width
// unconditionally (the words past a graph's own width are masked), so they
// issue back to back instead of one branch and one wait per word.  Rows
// have an odd stride, so lanes reading the same word of different rows
// spread over the LDS banks; the loop of pass 2 is the same on every lane,
// so its row reads are broadcasts.  Graphs have at most GC_BATCH_MAX_N
// vertices, so every count and LDS sum fits its type.
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.h"
#include "vertex_terms.h"

namespace gc {

int check_batch(const gc_batch *b, int64_t *out, hipStream_t s, uint32_t flags,
                std::vector<int64_t> *sizes, int32_t *err_buf, int64_t *sizes_buf);

namespace {

constexpr int kBvBlock = 512;
constexpr int kBvVertexBytes = 20;  // deg, tv2, sv, opp, k4 per vertex
// size classes in 64-bit words per row (class W holds graphs of at most 64 W
// vertices)
constexpr int kBvWords[] = {1, 2, 4, 6, 8, 10, 12, 16};
constexpr int kBvClasses = 8;

// word q of a register row, with every index a compile-time constant
template <int W>
__device__ __forceinline__ u64 pick(const u64 (&r)[W], int q) {
  u64 x = 0;
#pragma unroll
  for (int i = 0; i < W; i++)
    if (i == q) x = r[i];
  return x;
}

template <int W>
__device__ __forceinline__ int and_pop(const u64 (&r)[W], const u64 *row) {
  int c = 0;
#pragma unroll
  for (int i = 0; i < W; i++) c += __popcll(r[i] & row[i]);
  return c;
}

template <int W>
__global__ __launch_bounds__(kBvBlock) void k_batch_vertex(const int64_t *node_off,
                                                           const int32_t *rp, const int32_t *col,
                                                           const int32_t *list, int count,
                                                           int32_t *next, u64 *out) {
  extern __shared__ u64 smem[];
  __shared__ u64 red[kBvBlock / kWave][2];
  __shared__ u64 tot[2];
  __shared__ int cur, vnext;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) cur = atomicAdd(next, 1);
    __syncthreads();
    const int qi = cur;
    if (qi >= count) break;  // the same on every thread
    const int64_t gi = list[qi];
    const int64_t r0 = node_off[gi];
    const int n = (int)(node_off[gi + 1] - r0);
    const int words = (n + 63) / 64;  // <= W (the host bins by size)
    const int S = words | 1;          // row stride
    u64 *R = smem;
    int32_t *deg = reinterpret_cast<int32_t *>(smem + (size_t)n * S);
    uint32_t *tv2 = reinterpret_cast<uint32_t *>(deg + n);  // twice the triangles
    uint32_t *sv = tv2 + n;                                  // neighbour-degree sums
    uint32_t *opp = sv + n;                                  // OPP(v)
    uint32_t *k4 = opp + n;                                  // 4-cliques at v
    for (int w = tid; w < n * S; w += kBvBlock) R[w] = 0;
    for (int v = tid; v < n; v += kBvBlock) tv2[v] = sv[v] = opp[v] = k4[v] = 0;
    if (tid == 0) vnext = 0;
    __syncthreads();
    for (int v = tid; v < n; v += kBvBlock) {
      u64 *Rv = R + (size_t)v * S;
      const int64_t a = rp[r0 + v], b = rp[r0 + v + 1];
      for (int64_t p = a; p < b; p++) {
        const int j = col[p];
        Rv[j >> 6] |= 1ull << (j & 63);
      }
      deg[v] = (int32_t)(b - a);
    }
    __syncthreads();
    // pass 1: one row per wave, rows handed out in id order (the heaviest
    // first: row v holds the edges to the larger ids), its edges (v, w),
    // w > v, one per lane
    u64 t6 = 0, p2 = 0;
    const int lane = lane_id();
    for (;;) {
      int v = 0;
      if (lane == 0) v = atomicAdd(&vnext, 1);
      v = __builtin_amdgcn_readfirstlane(v);
      if (v >= n) break;
      // W words of the row: those past the graph's width (read past the row's
      // end, inside the padded allocation) are cleared, and every AND below
      // involves this row or a mask taken from it
      const u64 *Rrow = R + (size_t)v * S;
      u64 Rv[W];
      const int qv = v >> 6;
      const u64 below = (1ull << (v & 63)) - 1;
      int lower = 0;
#pragma unroll
      for (int i = 0; i < W; i++) {
        Rv[i] = Rrow[i] & (i < words ? ~0ull : 0ull);
        lower += __popcll(Rv[i] & (i < qv ? ~0ull : (i == qv ? below : 0ull)));
      }
      const int dv = deg[v], upper = dv - lower;
      const int64_t first = (int64_t)rp[r0 + v] + lower;  // the edges to larger ids
      if (lane == 0) p2 += vx_c2((u64)dv);
      uint32_t tv = 0, sw = 0, k4v = 0;
      for (int k0 = 0; k0 < upper; k0 += kWave) {
        const int k = k0 + lane;
        if (k >= upper) break;
        const int w = col[first + k];
        const u64 *Rw = R + (size_t)w * S;
        u64 tri_m[W];
        int T = 0;
#pragma unroll
        for (int i = 0; i < W; i++) {
          tri_m[i] = Rv[i] & Rw[i];
          T += __popcll(tri_m[i]);
        }
        tv += (uint32_t)T;
        sw += (uint32_t)deg[w];
        atomicAdd(&sv[w], (uint32_t)dv);
        if (T == 0) continue;
        atomicAdd(&tv2[w], (uint32_t)T);
        // 4-cliques whose two smallest vertices are v and w: the edges inside
        // M = Tri_e above w; x in M is in popcount(M & N(x)) of them
        const int qw = (w + 1) >> 6;
        const u64 lowcut = ~0ull << ((w + 1) & 63);
        uint32_t kw = 0;
        for (int q = 0; q < words; q++) {
          u64 tb = pick(tri_m, q);
          while (tb) {
            const int a = (q << 6) + __ffsll((long long)tb) - 1;
            tb &= tb - 1;
            atomicAdd(&opp[a], (uint32_t)T);
            if (a < w) continue;
            const u64 *Ra = R + (size_t)a * S;
            uint32_t c = 0;
#pragma unroll
            for (int i = 0; i < W; i++) {
              const u64 keep = i < qw ? 0ull : (i == qw ? lowcut : ~0ull);
              c += (uint32_t)__popcll(tri_m[i] & keep & Ra[i]);
            }
            if (c) {
              atomicAdd(&k4[a], c);
              kw += c;
            }
          }
        }
        kw /= 2;
        if (kw) {
          k4v += kw;
          atomicAdd(&k4[w], kw);
        }
      }
      // the row's own sums, once per wave
      tv = (uint32_t)wave_sum_u64(tv);
      sw = (uint32_t)wave_sum_u64(sw);
      k4v = (uint32_t)wave_sum_u64(k4v);
      if (lane == 0) {
        atomicAdd(&tv2[v], tv);
        atomicAdd(&sv[v], sw);
        if (k4v) atomicAdd(&k4[v], k4v);
        t6 += 2 * (u64)tv;  // each edge's triangles at both ends
      }
    }
    t6 = wave_sum_u64(t6);
    p2 = wave_sum_u64(p2);
    if (lane_id() == 0) {
      red[tid / kWave][0] = t6;
      red[tid / kWave][1] = p2;
    }
    __syncthreads();
    if (tid == 0) {
      u64 a = 0, b = 0;
      for (int w = 0; w < kBvBlock / kWave; w++) {
        a += red[w][0];
        b += red[w][1];
      }
      tot[0] = a / 6;            // triangles: each counted twice at each of its 3 vertices
      tot[1] = b - 3 * (a / 6);  // induced 2-stars
    }
    __syncthreads();
    // pass 2
    const u64 nn = (u64)n, m = (u64)((rp[r0 + n] - rp[r0]) / 2), tri = tot[0], star = tot[1];
    for (int v = tid; v < n; v += kBvBlock) {
      const u64 *Rrow = R + (size_t)v * S;
      u64 Rv[W];
#pragma unroll
      for (int i = 0; i < W; i++) Rv[i] = Rrow[i] & (i < words ? ~0ull : 0ull);
      const u64 d = (u64)deg[v], t = tv2[v] / 2, s = sv[v];
      u64 acc[kVxAcc];
#pragma unroll
      for (int k = 0; k < kVxAcc; k++) acc[k] = 0;
      u64 Q = 0;
      for (int q = 0; q < words; q++) {
        const u64 bits = pick(Rv, q);
        const int xe = min(64, n - (q << 6));
        for (int b = 0; b < xe; b++) {
          const int x = (q << 6) + b;
          const u64 c = (u64)and_pop(Rv, R + (size_t)x * S);
          if ((bits >> b) & 1) {
            vx_add_edge_tri(acc, c, d, (u64)deg[x], nn);
            vx_add_edge_other(acc, tv2[x] / 2, sv[x], t, s, m);
          }
          if (x != v) Q += vx_c2(c);
        }
      }
      const u64 sK4 = 3 * (u64)k4[v], sT2 = acc[1], sB = acc[9];
      const u64 sD = sT2 + 2 * (u64)opp[v] - 4 * t;
      const u64 sC4 = 2 * Q - sD + 2 * sK4;
      vx_add_edge_sums(acc, sK4, sC4, sD, sB);
      u64 r[17];
      vx_counts(acc, d, t, s, nn, m, tri, star, r);
      u64 *o = out + (size_t)(r0 + v) * 17;
#pragma unroll
      for (int k = 0; k < 17; k++) o[k] = r[k];
    }
    __syncthreads();
  }
}

using BvKernel = void (*)(const int64_t *, const int32_t *, const int32_t *, const int32_t *, int,
                          int32_t *, u64 *);

BvKernel bv_kernel(int cls) {
  switch (cls) {
    case 0: return k_batch_vertex<1>;
    case 1: return k_batch_vertex<2>;
    case 2: return k_batch_vertex<4>;
    case 3: return k_batch_vertex<6>;
    case 4: return k_batch_vertex<8>;
    case 5: return k_batch_vertex<10>;
    case 6: return k_batch_vertex<12>;
    default: return k_batch_vertex<16>;
  }
}

// Streams on which the size classes run side by side (default priority,
// created once per device and kept for the process), and the lock that
// makes one call's fork and join a unit.
constexpr int kBvMaxDevices = 64;
std::mutex g_bv_mu;
hipStream_t g_bv_streams[kBvMaxDevices][kBvClasses];
bool g_bv_ready[kBvMaxDevices];

hipError_t class_streams(int dev, hipStream_t **out) {
  if (dev < 0 || dev >= kBvMaxDevices) return hipErrorInvalidDevice;
  if (!g_bv_ready[dev]) {
    for (int c = 0; c < kBvClasses; c++) {
      const hipError_t e = hipStreamCreateWithFlags(&g_bv_streams[dev][c], hipStreamNonBlocking);
      if (e != hipSuccess) {
        for (int k = 0; k < c; k++) (void)hipStreamDestroy(g_bv_streams[dev][k]);
        return e;
      }
    }
    g_bv_ready[dev] = true;
  }
  *out = g_bv_streams[dev];
  return hipSuccess;
}

// Estimated work of one graph: the all-pairs pass, the triangle visits and
// the per-edge row intersections.
double bv_cost(int64_t n, int64_t nnz) {
  const double w = (double)((n + 63) / 64);
  const double pairs = 0.5 * (double)n * (double)(n - 1);
  const double rho = n > 1 ? (double)nnz / ((double)n * (double)(n - 1)) : 0.0;
  const double tri = pairs * (double)(n - 2) / 3.0 * rho * rho * rho;
  return 2.0 * pairs * w + tri * (w + 3.0) + (double)nnz * (4.0 + w) + 2000.0;
}

}  // namespace
}  // namespace gc

extern "C" int graphlet_batch_vertex(const gc_batch *b, uint64_t *out, void *stream,
                                     uint32_t flags) {
  gc::clear_error();
  try {
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> sizes;
    // the validation, the size check (GC_BATCH_MAX_N) and the sizes
    int rc = gc::check_batch(b, reinterpret_cast<int64_t *>(out), s, flags, &sizes, nullptr,
                             nullptr);
    if (rc != GC_OK) return rc;
    const int64_t G = b->graphs;
    // bin the graphs with vertices by row width, each class costliest first
    std::vector<std::vector<std::pair<double, int32_t>>> bins(gc::kBvClasses);
    std::vector<int64_t> nmax(gc::kBvClasses, 0);
    for (int64_t g = 0; g < G; g++) {
      const int64_t n = sizes[2 * g];
      if (n == 0) continue;
      const int64_t w = (n + 63) / 64;
      int c = 0;
      while (gc::kBvWords[c] < w) c++;  // n <= GC_BATCH_MAX_N: within the table
      bins[c].push_back({-gc::bv_cost(n, sizes[2 * g + 1]), (int32_t)g});
      nmax[c] = std::max(nmax[c], n);
    }
    std::vector<int32_t> list;
    std::vector<int> first(gc::kBvClasses, 0);
    for (int c = 0; c < gc::kBvClasses; c++) {
      std::sort(bins[c].begin(), bins[c].end());
      first[c] = (int)list.size();
      for (const auto &x : bins[c]) list.push_back(x.second);
    }
    if (list.empty()) return GC_OK;  // no vertices: nothing to write
    // device: the graph order, then one counter per class
    int32_t *dlist = nullptr;
    const size_t bytes = sizeof(int32_t) * (list.size() + gc::kBvClasses);
    GC_TRY_HIP(hipMallocAsync((void **)&dlist, bytes, s));
    int32_t *dnext = dlist + list.size();
    hipError_t e = hipMemcpyAsync(dlist, list.data(), sizeof(int32_t) * list.size(),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(dnext, 0, sizeof(int32_t) * gc::kBvClasses, s);
    int dev = 0, cus = 256;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // the classes run on streams of their own, after the uploads on s, and s
    // waits for all of them (largest class first, so its tail overlaps the
    // rest).  The lock covers the stream pool and each call's attribute,
    // launch and event sequence, not the wait for the results: calls from
    // several threads queue their launches in turn and overlap on the device.
    hipStream_t *cs = nullptr;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> done;
    std::vector<int> launched;
    std::unique_lock<std::mutex> lk(gc::g_bv_mu);
    if (e == hipSuccess) e = gc::class_streams(dev, &cs);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(fork, s);
    for (int c = gc::kBvClasses - 1; c >= 0 && e == hipSuccess; c--) {
      const int count = (int)bins[c].size();
      if (count == 0) continue;
      const int W = gc::kBvWords[c];
      const int64_t Smax = ((nmax[c] + 63) / 64) | 1;
      // rows, per-vertex arrays, and W words of padding for the class-width
      // reads past the last row
      const size_t lds = (size_t)nmax[c] * ((size_t)Smax * sizeof(gc::u64) + gc::kBvVertexBytes) +
                         (size_t)W * sizeof(gc::u64);
      gc::BvKernel k = gc::bv_kernel(c);
      e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
      int per_cu = 1;
      if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k, gc::kBvBlock,
                                                         lds);
      if (e != hipSuccess) break;
      const int grid = std::max(1, std::min(count, cus * std::max(per_cu, 1)));
      hipEvent_t ev = nullptr;
      e = hipStreamWaitEvent(cs[c], fork, 0);
      if (e != hipSuccess) break;
      k<<<grid, gc::kBvBlock, lds, cs[c]>>>(b->node_off, b->row_ptr, b->col, dlist + first[c],
                                            count, dnext + c, reinterpret_cast<gc::u64 *>(out));
      e = hipGetLastError();
      if (e == hipSuccess) launched.push_back(c);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) {
        done.push_back(ev);
        e = hipEventRecord(ev, cs[c]);
      }
      if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
    }
    lk.unlock();
    // on an error part way, the classes already launched finish before the
    // order and counters are freed
    if (e != hipSuccess)
      for (int c : launched) (void)hipStreamSynchronize(cs[c]);
    (void)hipFreeAsync(dlist, s);
    const hipError_t f = hipStreamSynchronize(s);
    if (e == hipSuccess) e = f;
    for (hipEvent_t ev : done) (void)hipEventDestroy(ev);
    if (fork) (void)hipEventDestroy(fork);
    if (e != hipSuccess) {
      gc::set_error("batched vertex counts: %s", hipGetErrorString(e));
      return GC_EHIP;
    }
    return GC_OK;
  } catch (...) {
    gc::set_error("unexpected exception");
    return GC_EINTERNAL;
  }
}
