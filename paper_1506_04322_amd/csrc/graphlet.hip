// Per-edge graphlet decomposition (k = 2, 3, 4) of one graph on an MI355X.
//
// The method (Ahmed et al., arXiv 1506.04322, Sections 3-4): for every edge
// e = (u, v) find Tri_e, Star_u, Star_v (Step 1), count the 4-cliques and
// induced 4-cycles containing e (Step 2), accumulate the unrestricted counts
// of Equations "comb_n_ai_ai"/"comb_n_ai_aj" (Step 3), and derive all 17
// counts with the Lemmas of Section 4.3 and Equations "g_4_9", "g_4_11"
// (Step 4).
//
// How the steps map onto the GPU (the paper's CPU loop order is not kept;
// every per-edge quantity is the same number):
//
//  prepass   vertices relabelled by (degree, id) with a stable radix sort, and
//            every neighbour list re-sorted in the new ids, so that for each
//            vertex x its lower neighbours L(x) and upper neighbours U(x)
//            are contiguous.  |U(x)| <= sqrt(2m) for every x.
//  Step 1+2a one workgroup per vertex u builds, in LDS, the adjacency bitmap
//            of the subgraph induced by U(u).  Every bit (i, j) is a triangle
//            {u, U_i, U_j} seen from its lowest vertex u: it adds one to
//            |Tri| of edge (U_i, U_j) (a global atomic) and row popcounts
//            give |Tri| of the edges (u, U_i).  AND+popcount of two rows
//            counts the 4-cliques through u; per-edge 4-clique counts come
//            from the same rows in a second pass.
//  Step 2b   4-cycles through an edge: C4_e = C4ni_e - D_e + 2 K4_e, where
//            C4ni_e counts 4-cycles through e that may have chords and
//            D_e = sum_{w in Tri_e} (|Tri_(u,w)| + |Tri_(v,w)| - 2).  The
//            chordless cycles of Corollary "cyc" (N_{Su,Sv,1}) are what is
//            left after removing cycles with a chord through a triangle
//            vertex (each such chorded cycle is counted by D_e, cycles with
//            both chords twice, hence + 2 K4_e).  C4ni is found by wedge
//            aggregation: each 4-cycle has one highest vertex x, and is two
//            paths x - v - y with v, y below x; counters per (x, y) live in
//            an LDS hash (light x) or in y-range chunks of LDS counters
//            (heavy x).  Summed over all edges, sum_e D_e = 4 sum_e C(T_e,2).
//  Step 3    one thread per edge computes T, Su, Sv, I and the eleven
//            unrestricted terms, reduced exactly in 128 bits.
//  Step 4    host, 128-bit, with every division checked for a remainder.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "primitives.h"

namespace gc {

namespace {
thread_local std::string t_err;
thread_local bool t_timing = false;
thread_local gc_timing t_last_timing;
}

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
}
void clear_error() { t_err.clear(); }
const char *last_error() { return t_err.c_str(); }

namespace {

// Number of Step-3 accumulators.
constexpr int kAcc = 13;
enum AccIdx {
  A_T = 0,    // sum |Tri_e|
  A_S,        // sum |Star_u| + |Star_v|
  A_I,        // sum I_e = |V| - |N(u) u N(v)|
  A_TT,       // sum C(T, 2)                      N_{T,T}
  A_SUSV,     // sum Su Sv                        N_{Su,Sv}
  A_TS,       // sum T (Su + Sv)                  N_{T,Su v Sv}
  A_SS,       // sum C(Su,2) + C(Sv,2)            N_{S.,S.}
  A_TI,       // sum T I                          N_{T,I}
  A_SI,       // sum (Su + Sv) I                  N_{Su v Sv,I}
  A_II,       // sum C(I, 2)                      N_{I,I}
  A_II1,      // sum |E| - d_u - d_v + 1           (N_{I,I,1} before the subtractions)
  A_K4,       // sum 4-cliques through e           N_{T,T,1}
  A_C4        // sum induced 4-cycles through e    N_{Su,Sv,1}
};

// Device accumulator block layout (u64 words).
struct DevAcc {
  u64 k4x3[2];  // 3 x (number of 4-cliques), from the clique pass
  u64 c4ni[2];  // number of 4-cycles, chords allowed, from the wedge pass
  u64 step3[kAcc][2];
  int32_t err;  // validation error code (0 = ok)
  int32_t pad;
  u64 queue;    // work-queue head for persistent kernels
  u64 queue2;
};

constexpr int kTkBins = 4;
struct Counters {
  int32_t tk_cnt[kTkBins];
  int32_t c4_light;
  int32_t c4_heavy;
  int32_t max_ucnt;
  int32_t max_lcnt_heavy;
  int32_t max_deg;
  int32_t pad[7];
  u64 wedges_light;
  u64 wedges_heavy;
  u64 clique_entries;
  u64 pad2;
};

// Bin limits for the clique kernel: |U(u)| <= 64, 256, 512, larger.
constexpr int kTkLim0 = 64, kTkLim1 = 256, kTkLim2 = 512;
// Light wedge vertices: at most this many wedges (hash of <= 2048 slots).
constexpr u64 kLightWedges = 1024;
constexpr int kHashSlots = 2048;
// Heavy wedge vertices: LDS counter chunk, 64 KiB.
constexpr int kChunkWords = 16384;
// Target wedges per heavy work item.
constexpr u64 kPieceWork = u64(1) << 21;
constexpr int kTk3Slots = 64;     // concurrent workgroups for |U(u)| > 512
constexpr int kC4HeavyBlock = 512;

inline unsigned grid1d(int64_t n, int block, int64_t cap = 1 << 20) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ================================================================ validation

// Validation sets bit (-code) of *err for every violation it finds; the host
// reports the most basic one (lowest bit).
__device__ __forceinline__ void flag_err(int32_t *err, int code) { atomicOr(err, 1 << (-code)); }

__global__ void k_validate(const int32_t *rp, const int32_t *col, int64_t n, int64_t nnz,
                           int32_t *err) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; u < n; u += stride) {
    int64_t a = rp[u], b = rp[u + 1];
    if (a < 0 || b < a || b > nnz) {
      flag_err(err, GC_EINVAL);
      continue;
    }
    for (int64_t j = a; j < b; j++) {
      int64_t v = col[j];
      if (v < 0 || v >= n) {
        flag_err(err, GC_EASYMMETRIC);
        break;
      }
      if (v == u) flag_err(err, GC_ESELFLOOP);
      if (j > a && col[j - 1] >= v) flag_err(err, GC_ENOTSORTED);
      int64_t c = rp[v], d = rp[v + 1];
      if (c < 0 || d < c || d > nnz) continue;
      int pos = lower_bound_dev<int32_t>(col + c, (int)(d - c), (int32_t)u);
      if (pos >= d - c || col[c + pos] != u) flag_err(err, GC_EASYMMETRIC);
    }
  }
}

__global__ void k_check_rowptr_ends(const int32_t *rp, int64_t n, int64_t nnz, int32_t *err) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    if (rp[0] != 0 || rp[n] != nnz) flag_err(err, GC_EINVAL);
}

// ================================================================ prepass

// deg[u] and the key (deg << B | u) that orders vertices by (degree, id).
__global__ void k_degree_keys(const int32_t *rp, int64_t n, int B, int32_t *deg, u64 *key,
                              int32_t *max_deg) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int mx = 0;
  if (u < n) {
    int d = rp[u + 1] - rp[u];
    deg[u] = d;
    if (key) key[u] = ((u64)d << B) | (u64)u;
    mx = d;
  }
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, kWave));
  if (lane_id() == 0) atomicMax(max_deg, mx);
}

// order[x] = old id of new vertex x; rank[old] = x; deg2[x] = degree.
__global__ void k_rank(const u64 *sorted, int64_t n, int B, int32_t *order, int32_t *rank,
                       int32_t *deg2) {
  int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  u64 k = sorted[x];
  int32_t old = (int32_t)(k & ((1ull << B) - 1));
  order[x] = old;
  rank[old] = (int32_t)x;
  deg2[x] = (int32_t)(k >> B);
}

// One wave per original row: keys (rank[u] << B | rank[w]) for every entry.
// An id outside [0, n) (a broken contract without GC_VALIDATE) is flagged and
// never used as an index.
__global__ void k_edge_keys(const int32_t *rp, const int32_t *col, int64_t n, int B,
                            const int32_t *rank, u64 *ekeys, int32_t *err) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int lane = lane_id();
  for (int64_t u = wave; u < n; u += nwaves) {
    const u64 ru = (u64)rank[u] << B;
    for (int64_t j = rp[u] + lane; j < rp[u + 1]; j += kWave) {
      int32_t w = col[j];
      if (w < 0 || w >= n) {
        flag_err(err, GC_EASYMMETRIC);
        w = (int32_t)u;
      }
      ekeys[j] = ru | (u64)rank[w];
    }
  }
}

__global__ void k_split_keys(const u64 *ekeys, int64_t nnz, int B, int32_t *col2) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnz) col2[p] = (int32_t)(ekeys[p] & ((1ull << B) - 1));
}

// lcnt[x] = |L(x)|, ucnt[x] = |U(x)|, ustart[x] = first upper position.
__global__ void k_split_rows(const int32_t *rp2, const int32_t *col2, int64_t n, int32_t *lcnt,
                             int32_t *ucnt, int32_t *ustart, int32_t *max_ucnt) {
  int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int mx = 0;
  if (x < n) {
    int a = rp2[x], d = rp2[x + 1] - a;
    int l = lower_bound_dev<int32_t>(col2 + a, d, (int32_t)x);
    lcnt[x] = l;
    ucnt[x] = d - l;
    ustart[x] = a + l;
    mx = d - l;
  }
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, kWave));
  if (lane_id() == 0) atomicMax(max_ucnt, mx);
}

// tpos[p] = position of the reverse entry (x in the list of y).  Every
// position is written; a missing reverse entry or a self-loop (broken
// contract) is flagged and points at p itself.
__global__ void k_tpos(const u64 *ekeys, const int32_t *col2, const int32_t *rp2,
                       const int32_t *lcnt, int64_t nnz, int B, int32_t *tpos, int32_t *err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const int32_t x = (int32_t)(ekeys[p] >> B);
  const int32_t y = col2[p];
  int a, len;
  if (y > x) {  // x sits in the lower part of y's list
    a = rp2[y];
    len = lcnt[y];
  } else {      // x sits in the upper part
    a = rp2[y] + lcnt[y];
    len = rp2[y + 1] - a;
  }
  const int q = a + lower_bound_dev<int32_t>(col2 + a, len, x);
  if (y == x || q >= a + len || col2[q] != x) {
    flag_err(err, y == x ? GC_ESELFLOOP : GC_EASYMMETRIC);
    tpos[p] = (int32_t)p;
    return;
  }
  tpos[p] = q;
}

// W[x] = number of wedges x - v - y with v, y < x: sum over v in L(x) of
// the length of the prefix of N(v) below x, which ends at the position of x
// in N(v), tpos[q].  One thread per lower position; wave-aggregated atomics.
// Also counts the entries the clique pass will scan: vertex v reads U(x)
// for every x in U(v), i.e. |U(x)| per lower position (x, v).
__global__ void k_wedges(const u64 *ekeys, const int32_t *col2, const int32_t *rp2,
                         const int32_t *tpos, const int32_t *ucnt, int64_t nnz, int B, u64 *W,
                         u64 *clique_entries) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t x = -1;
  u64 len = 0, ce = 0;
  if (p < nnz) {
    int32_t r = (int32_t)(ekeys[p] >> B);
    int32_t v = col2[p];
    if (v < r) {
      x = r;
      len = (u64)(tpos[p] - rp2[v]);
      ce = (u64)ucnt[r];
    }
  }
  ce = wave_sum_u64(ce);
  if (lane_id() == 0 && ce) atomicAdd(clique_entries, ce);
  const int32_t x0 = __shfl(x, 0, kWave);
  const bool same = __all(x == x0);
  if (same) {
    u64 s = wave_sum_u64(len);
    if (lane_id() == 0 && x0 >= 0 && s) atomicAdd(&W[x0], s);
  } else if (x >= 0 && len) {
    atomicAdd(&W[x], len);
  }
}

// Work lists.  tk lists: vertices with |U(u)| >= 2 by size class; c4 lists:
// vertices with wedges, light (LDS hash) or heavy (chunked counters).
__global__ void k_bins(const int32_t *ucnt, const int32_t *lcnt, const u64 *W, int64_t n,
                       int32_t *tk0, int32_t *tk1, int32_t *tk2, int32_t *tk3, int32_t *c4l,
                       int32_t *c4h, Counters *cnt) {
  int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  int k = ucnt[x];
  if (k >= 2) {
    if (k <= kTkLim0) tk0[atomicAdd(&cnt->tk_cnt[0], 1)] = (int32_t)x;
    else if (k <= kTkLim1) tk1[atomicAdd(&cnt->tk_cnt[1], 1)] = (int32_t)x;
    else if (k <= kTkLim2) tk2[atomicAdd(&cnt->tk_cnt[2], 1)] = (int32_t)x;
    else tk3[atomicAdd(&cnt->tk_cnt[3], 1)] = (int32_t)x;
  }
  u64 w = W[x];
  u64 wl = 0, wh = 0;
  if (w >= 2) {  // fewer than two wedges cannot close a cycle
    if (w <= kLightWedges) {
      c4l[atomicAdd(&cnt->c4_light, 1)] = (int32_t)x;
      wl = w;
    } else {
      c4h[atomicAdd(&cnt->c4_heavy, 1)] = (int32_t)x;
      atomicMax(&cnt->max_lcnt_heavy, lcnt[x]);
      wh = w;
    }
  }
  if (wl) atomicAdd(&cnt->wedges_light, wl);
  if (wh) atomicAdd(&cnt->wedges_heavy, wh);
}

// ================================================================ Steps 1 + 2a
// Triangles and 4-cliques, one workgroup per vertex u (the lowest vertex of
// every triangle / clique it reports).

struct TkArgs {
  const int32_t *col2;
  const int32_t *ustart;
  const int32_t *ucnt;
  const int32_t *list;
  int nlist;
  uint32_t *T;    // |Tri| per upper position
  u64 *K4w;       // per-edge pass: 4-cliques per upper position
  u64 *Dw;        // per-edge pass: D_e per upper position
  u64 *k4x3;      // total 3 x 4-cliques (128-bit)
  // global storage for the largest class, per workgroup slot
  u64 *gR;
  int32_t *gI;    // 3 * kmax int32 per slot: U, V, P (+1)
  u64 *gA;        // 2 * kmax u64 per slot (per-edge accumulators)
  int kmax;
};

// Exclusive scan of A[0..k) in place, writes the total to A[k].  BLOCK threads.
template <int BLOCK>
__device__ void block_scan_excl(int32_t *A, int k, int32_t *sums) {
  const int tid = threadIdx.x;
  const int per = (k + BLOCK - 1) / BLOCK;
  const int a = min(k, tid * per), b = min(k, a + per);
  int32_t s = 0;
  for (int i = a; i < b; i++) s += A[i];
  sums[tid] = s;
  __syncthreads();
  for (int off = 1; off < BLOCK; off <<= 1) {
    int32_t t = tid >= off ? sums[tid - off] : 0;
    __syncthreads();
    sums[tid] += t;
    __syncthreads();
  }
  int32_t run = sums[tid] - s;
  for (int i = a; i < b; i++) {
    int32_t v = A[i];
    A[i] = run;
    run += v;
  }
  if (tid == BLOCK - 1) A[k] = sums[BLOCK - 1];
  __syncthreads();
}

// Body shared by all size classes.  U, V, P: int32 arrays (k, k, k+1),
// R: k * words u64 rows, Tu/ACC1/ACC2 only in the per-edge pass.
template <int BLOCK, bool PER_EDGE>
__device__ void tk_vertex(const TkArgs &g, int u, int32_t *U, int32_t *V, int32_t *P, u64 *R,
                          int words, int32_t *sums, u64 *A1, u64 *A2, uint32_t *Tu,
                          u64 *red, u128 &k4acc) {
  const int tid = threadIdx.x;
  const int k = g.ucnt[u];
  const int base = g.ustart[u];
  for (int i = tid; i < k; i += BLOCK) U[i] = g.col2[base + i];
  for (int w = tid; w < k * words; w += BLOCK) R[w] = 0;
  __syncthreads();
  for (int i = tid; i < k; i += BLOCK) {
    int v = U[i];
    V[i] = g.ustart[v];
    P[i] = g.ucnt[v];
    if (PER_EDGE) {
      Tu[i] = g.T[base + i];
      A1[i] = 0;
      A2[i] = 0;
    }
  }
  __syncthreads();
  block_scan_excl<BLOCK>(P, k, sums);
  const int total = P[k];
  // Build the rows: entry x of U(U_i) that is also in U(u) is a triangle.
  for (int t = tid; t < total; t += BLOCK) {
    int i = upper_index_dev<int32_t>(P, k, t);
    int pos = V[i] + (t - P[i]);
    int x = g.col2[pos];
    int j = i + 1 + lower_bound_dev<int32_t>(U + i + 1, k - i - 1, x);
    if (j < k && U[j] == x) {
      atomicOr(&R[(size_t)i * words + (j >> 6)], 1ull << (j & 63));
      atomicOr(&R[(size_t)j * words + (i >> 6)], 1ull << (i & 63));
      if (!PER_EDGE) atomicAdd(&g.T[pos], 1u);
    }
  }
  __syncthreads();
  if (!PER_EDGE) {
    // |Tri| of edges (u, U_i) from third vertices in U(u); 3 x cliques.
    u64 acc = 0;
    for (int i = tid; i < k; i += BLOCK) {
      const u64 *Ri = R + (size_t)i * words;
      uint32_t c = 0;
      for (int w = 0; w < words; w++) c += (uint32_t)__popcll(Ri[w]);
      if (c) atomicAdd(&g.T[base + i], c);
      for (int w = (i + 1) >> 6; w < words; w++) {
        u64 bits = Ri[w];
        if (w == ((i + 1) >> 6)) bits &= (~0ull) << ((i + 1) & 63);
        while (bits) {
          int j = (w << 6) + __ffsll((long long)bits) - 1;
          bits &= bits - 1;
          const u64 *Rj = R + (size_t)j * words;
          for (int z = 0; z < words; z++) acc += (u64)__popcll(Ri[z] & Rj[z]);
        }
      }
    }
    k4acc += (u128)acc;
  } else {
    // Per local edge (i, j): 4-cliques {u, U_i, U_j, x} and D terms.
    for (int t = tid; t < total; t += BLOCK) {
      int i = upper_index_dev<int32_t>(P, k, t);
      int pos = V[i] + (t - P[i]);
      int x = g.col2[pos];
      int j = i + 1 + lower_bound_dev<int32_t>(U + i + 1, k - i - 1, x);
      if (j < k && U[j] == x) {
        const u64 *Ri = R + (size_t)i * words, *Rj = R + (size_t)j * words;
        u64 c = 0;
        for (int z = 0; z < words; z++) c += (u64)__popcll(Ri[z] & Rj[z]);
        const u64 tij = g.T[pos];
        if (c) atomicAdd(&g.K4w[pos], c);
        atomicAdd(&g.Dw[pos], (u64)Tu[i] + Tu[j] - 2);
        if (c) {
          atomicAdd(&A1[i], c);
          atomicAdd(&A1[j], c);
        }
        atomicAdd(&A2[i], (u64)Tu[j] + tij - 2);
        atomicAdd(&A2[j], (u64)Tu[i] + tij - 2);
      }
    }
    __syncthreads();
    for (int i = tid; i < k; i += BLOCK) {
      if (A1[i]) atomicAdd(&g.K4w[base + i], A1[i] / 2);
      if (A2[i]) atomicAdd(&g.Dw[base + i], A2[i]);
    }
  }
  __syncthreads();
}

template <int BLOCK, int KMAX, bool PER_EDGE>
__global__ __launch_bounds__(BLOCK) void k_tk_lds(TkArgs g) {
  constexpr int WORDS = (KMAX + 63) / 64;
  __shared__ int32_t U[KMAX], V[KMAX], P[KMAX + 1], sums[BLOCK];
  __shared__ u64 R[KMAX * WORDS];
  __shared__ u64 A1[PER_EDGE ? KMAX : 1], A2[PER_EDGE ? KMAX : 1];
  __shared__ uint32_t Tu[PER_EDGE ? KMAX : 1];
  __shared__ u64 red[32];
  u128 k4acc = 0;
  for (int it = blockIdx.x; it < g.nlist; it += gridDim.x) {
    const int u = g.list[it];
    const int words = (g.ucnt[u] + 63) / 64;
    tk_vertex<BLOCK, PER_EDGE>(g, u, U, V, P, R, words, sums, A1, A2, Tu, red, k4acc);
  }
  if (!PER_EDGE) {
    u128 s = block_sum_u128(k4acc, red);
    if (threadIdx.x == 0 && s) atomic_add_u128(g.k4x3, s);
  }
}

template <int BLOCK, bool PER_EDGE>
__global__ __launch_bounds__(BLOCK) void k_tk_global(TkArgs g) {
  __shared__ int32_t sums[BLOCK];
  __shared__ u64 red[32];
  const size_t kmax = (size_t)g.kmax;
  const size_t wmax = (kmax + 63) / 64;
  u64 *R = g.gR + (size_t)blockIdx.x * kmax * wmax;
  int32_t *I = g.gI + (size_t)blockIdx.x * (3 * kmax + 1);
  int32_t *U = I, *V = I + kmax, *P = I + 2 * kmax;
  u64 *A1 = g.gA + (size_t)blockIdx.x * 3 * kmax;
  u64 *A2 = A1 + kmax;
  uint32_t *Tu = reinterpret_cast<uint32_t *>(A2 + kmax);
  u128 k4acc = 0;
  for (int it = blockIdx.x; it < g.nlist; it += gridDim.x) {
    const int u = g.list[it];
    const int words = (g.ucnt[u] + 63) / 64;
    tk_vertex<BLOCK, PER_EDGE>(g, u, U, V, P, R, words, sums, A1, A2, Tu, red, k4acc);
    __threadfence_block();
  }
  if (!PER_EDGE) {
    u128 s = block_sum_u128(k4acc, red);
    if (threadIdx.x == 0 && s) atomic_add_u128(g.k4x3, s);
  }
}

// ================================================================ Step 2b
// 4-cycles (chords allowed) by wedge aggregation.

struct C4Args {
  const int32_t *col2;
  const int32_t *rp2;
  const int32_t *lcnt;
  const int32_t *tpos;
  const u64 *W;
  const int32_t *list;
  int nlist;
  u64 *c4ni;   // total (128-bit)
  u64 *C4w;    // per-edge pass: 4-cycles (chords allowed) per upper position
  // heavy items
  const int4 *items;  // (x, y_begin, y_end, unused)
  int nitems;
  u64 *queue;
  int32_t *gcur;      // per slot: cursor per lower neighbour
  int32_t *gbeg;      // per slot (per-edge): cursor at chunk start
  u64 *gacc;          // per slot (per-edge): credit for edge (x, v)
  int lmax;
};

__device__ __forceinline__ u64 choose2(u64 c) { return c * (c - 1) / 2; }

// Upper position of the undirected edge stored at position p of N(v).
__device__ __forceinline__ int upper_pos(const int32_t *col2, const int32_t *tpos, int p, int v) {
  return col2[p] > v ? p : tpos[p];
}

// Light x: one 64-lane workgroup per vertex, counters in an LDS hash.
template <bool PER_EDGE>
__global__ __launch_bounds__(kWave) void k_c4_light(C4Args g) {
  __shared__ int32_t hkey[kHashSlots];
  __shared__ uint32_t hcnt[kHashSlots];
  __shared__ int32_t sIncl[kWave], sStart[kWave], sLen[kWave], sQ[kWave], sV[kWave];
  __shared__ u64 red[32];
  const int lane = threadIdx.x;
  for (int h = lane; h < kHashSlots; h += kWave) {
    hkey[h] = -1;
    hcnt[h] = 0;
  }
  __syncthreads();
  u128 acc = 0;
  for (int it = blockIdx.x; it < g.nlist; it += gridDim.x) {
    const int x = g.list[it];
    const u64 w = g.W[x];
    int hs = 64;
    while ((u64)hs < 2 * w) hs <<= 1;
    const uint32_t mask = (uint32_t)hs - 1;
    const int hbits = __ffs(hs) - 1;
    const int Lx = g.rp2[x], nL = g.lcnt[x];
    for (int pass = 0; pass < (PER_EDGE ? 2 : 1); pass++) {
      for (int b = 0; b < nL; b += kWave) {
        const int i = b + lane;
        int len = 0;
        if (i < nL) {
          const int q = Lx + i;
          const int v = g.col2[q];
          const int s = g.rp2[v];
          len = g.tpos[q] - s;
          sStart[lane] = s;
          sQ[lane] = q;
          sV[lane] = v;
        }
        int incl = len;
        for (int off = 1; off < kWave; off <<= 1) {
          int t = __shfl_up(incl, off, kWave);
          if (lane >= off) incl += t;
        }
        sIncl[lane] = incl;
        sLen[lane] = len;
        __syncthreads();
        const int total = sIncl[kWave - 1];
        for (int t = lane; t < total; t += kWave) {
          // owner: first lane whose inclusive prefix exceeds t
          int lo = 0, hi = kWave - 1;
          while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (sIncl[mid] > t) hi = mid;
            else lo = mid + 1;
          }
          const int p = sStart[lo] + (t - (sIncl[lo] - sLen[lo]));
          const int y = g.col2[p];
          uint32_t h = ((uint32_t)y * 2654435761u) >> (32 - hbits);
          if (pass == 0) {
            while (true) {
              int old = atomicCAS(&hkey[h], -1, y);
              if (old == -1 || old == y) {
                atomicAdd(&hcnt[h], 1u);
                break;
              }
              h = (h + 1) & mask;
            }
          } else {
            while (hkey[h] != y) h = (h + 1) & mask;
            const u64 c = hcnt[h];
            if (c >= 2) {
              atomicAdd(&g.C4w[upper_pos(g.col2, g.tpos, p, sV[lo])], c - 1);
              atomicAdd(&g.C4w[g.tpos[sQ[lo]]], c - 1);
            }
          }
        }
        __syncthreads();
      }
    }
    for (int h = lane; h < hs; h += kWave) {
      if (hkey[h] != -1) {
        acc += (u128)choose2(hcnt[h]);
        hkey[h] = -1;
        hcnt[h] = 0;
      }
    }
    __syncthreads();
  }
  u128 s = block_sum_u128(acc, red);
  if (threadIdx.x == 0 && s) atomic_add_u128(g.c4ni, s);
}

// Heavy x: persistent workgroups take items (x, y range) from a queue.  The
// y range is walked in chunks of LDS counters (2 x 16-bit per word when
// |L(x)| < 65536, else 32-bit); every lower neighbour v keeps a cursor into
// the sorted N(v) so each wedge is read once per pass.
template <bool PER_EDGE>
__global__ __launch_bounds__(kC4HeavyBlock) void k_c4_heavy(C4Args g) {
  __shared__ uint32_t cnt[kChunkWords];
  __shared__ u64 red[32];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  int32_t *cur = g.gcur + (size_t)blockIdx.x * g.lmax;
  int32_t *beg = PER_EDGE ? g.gbeg + (size_t)blockIdx.x * g.lmax : nullptr;
  u64 *cacc = PER_EDGE ? g.gacc + (size_t)blockIdx.x * g.lmax : nullptr;
  u128 acc = 0;
  while (true) {
    if (tid == 0) s_item = (int)atomicAdd(g.queue, 1ull);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= g.nitems) break;
    const int4 it = g.items[item];
    const int x = it.x, ya = it.y, yb = it.z;
    const int Lx = g.rp2[x], nL = g.lcnt[x];
    const bool packed = nL < 65536;
    const int K = packed ? 2 * kChunkWords : kChunkWords;
    for (int i = tid; i < nL; i += kC4HeavyBlock) {
      const int q = Lx + i;
      const int v = g.col2[q];
      const int s = g.rp2[v];
      const int e = g.tpos[q];
      cur[i] = s + lower_bound_dev<int32_t>(g.col2 + s, e - s, ya);
      if (PER_EDGE) cacc[i] = 0;
    }
    __syncthreads();
    for (int c0 = ya; c0 < yb; c0 += K) {
      const int c1 = min(c0 + K, yb);
      for (int w = tid; w < kChunkWords; w += kC4HeavyBlock) cnt[w] = 0;
      __syncthreads();
      for (int i = tid; i < nL; i += kC4HeavyBlock) {
        const int q = Lx + i;
        const int e = g.tpos[q];
        int p = cur[i];
        if (PER_EDGE) beg[i] = p;
        for (; p < e; p++) {
          const int y = g.col2[p];
          if (y >= c1) break;
          const int d = y - c0;
          if (packed) atomicAdd(&cnt[d >> 1], (d & 1) ? 65536u : 1u);
          else atomicAdd(&cnt[d], 1u);
        }
        cur[i] = p;
      }
      __syncthreads();
      if (PER_EDGE) {
        for (int i = tid; i < nL; i += kC4HeavyBlock) {
          const int q = Lx + i;
          const int v = g.col2[q];
          u64 credit = 0;
          for (int p = beg[i]; p < cur[i]; p++) {
            const int y = g.col2[p];
            const int d = y - c0;
            const u64 c = packed ? ((cnt[d >> 1] >> ((d & 1) * 16)) & 0xffffu) : cnt[d];
            if (c >= 2) {
              atomicAdd(&g.C4w[upper_pos(g.col2, g.tpos, p, v)], c - 1);
              credit += c - 1;
            }
          }
          cacc[i] += credit;
        }
        __syncthreads();
      }
      u64 part = 0;
      for (int w = tid; w < kChunkWords; w += kC4HeavyBlock) {
        const uint32_t val = cnt[w];
        if (packed) part += choose2(val & 0xffffu) + choose2(val >> 16);
        else part += choose2(val);
      }
      acc += (u128)part;
      __syncthreads();
    }
    if (PER_EDGE) {
      for (int i = tid; i < nL; i += kC4HeavyBlock)
        if (cacc[i]) atomicAdd(&g.C4w[g.tpos[Lx + i]], cacc[i]);
    }
    __syncthreads();
  }
  u128 s = block_sum_u128(acc, red);
  if (threadIdx.x == 0 && s) atomic_add_u128(g.c4ni, s);
}

// ================================================================ Step 3

struct S3Args {
  const u64 *ekeys;
  const int32_t *col2;
  const int32_t *deg2;
  const uint32_t *T;
  const u64 *K4w, *C4w, *Dw;  // per-edge mode only
  int64_t nnz, n, m;
  int B;
  u64 *partials;  // [gridDim][kAcc][2]
  // per-edge output mapping
  const int32_t *order;
  const int32_t *rp;   // original row_ptr
  const int32_t *col;  // original col
  const int64_t *cu;   // exclusive scan of upper counts (original ids)
  int64_t *out;        // [3][m]
};

template <bool PER_EDGE>
__global__ __launch_bounds__(256) void k_step3(S3Args g) {
  __shared__ u64 red[32];
  u128 a[kAcc];
#pragma unroll
  for (int i = 0; i < kAcc; i++) a[i] = 0;
  const u64 n = (u64)g.n, m = (u64)g.m;
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; p < g.nnz; p += stride) {
    const int32_t x = (int32_t)(g.ekeys[p] >> g.B);
    const int32_t y = g.col2[p];
    if (y <= x) continue;
    const u64 du = (u64)g.deg2[x], dv = (u64)g.deg2[y];
    const u64 T = g.T[p];
    const u64 Su = du - 1 - T, Sv = dv - 1 - T;
    const u64 I = n - du - dv + T;  // |V| - |N(u) u N(v)|, the union holding u and v
    const u64 S = Su + Sv;
    a[A_T] += T;
    a[A_S] += S;
    a[A_I] += I;
    a[A_TT] += choose2(T);
    a[A_SUSV] += (u128)Su * Sv;
    a[A_TS] += (u128)T * S;
    a[A_SS] += (u128)choose2(Su) + choose2(Sv);
    a[A_TI] += (u128)T * I;
    a[A_SI] += (u128)S * I;
    a[A_II] += (u128)I * (I - (I > 0)) / 2;
    a[A_II1] += m - du - dv + 1;
    if (PER_EDGE) {
      const u64 k4 = g.K4w[p];
      const u64 c4 = g.C4w[p] - g.Dw[p] + 2 * k4;
      a[A_K4] += k4;
      a[A_C4] += c4;
      // canonical id of the edge in the caller's numbering
      int32_t ua = g.order[x], ub = g.order[y];
      int32_t lo = ua < ub ? ua : ub, hi = ua < ub ? ub : ua;
      const int32_t r0 = g.rp[lo], r1 = g.rp[lo + 1];
      const int split = lower_bound_dev<int32_t>(g.col + r0, r1 - r0, lo);
      const int pos = lower_bound_dev<int32_t>(g.col + r0, r1 - r0, hi);
      const int64_t id = g.cu[lo] + (pos - split);
      g.out[id] = (int64_t)T;
      g.out[g.m + id] = (int64_t)k4;
      g.out[2 * g.m + id] = (int64_t)c4;
    }
  }
  for (int i = 0; i < kAcc; i++) {
    u128 s = block_sum_u128(a[i], red);
    if (threadIdx.x == 0) {
      g.partials[((size_t)blockIdx.x * kAcc + i) * 2] = (u64)s;
      g.partials[((size_t)blockIdx.x * kAcc + i) * 2 + 1] = (u64)(s >> 64);
    }
  }
}

__global__ void k_step3_final(const u64 *partials, int nblocks, DevAcc *acc) {
  // one wave per accumulator
  const int i = blockIdx.x;
  u128 s = 0;
  for (int b = threadIdx.x; b < nblocks; b += kWave)
    s += ((u128)partials[((size_t)b * kAcc + i) * 2 + 1] << 64) | partials[((size_t)b * kAcc + i) * 2];
  s = wave_sum_u128(s);
  if (threadIdx.x == 0) {
    acc->step3[i][0] = (u64)s;
    acc->step3[i][1] = (u64)(s >> 64);
  }
}

// Upper-neighbour counts in the caller's ids (for canonical edge numbering).
__global__ void k_orig_upper(const int32_t *rp, const int32_t *col, int64_t n, int64_t *up) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int a = rp[u], d = rp[u + 1] - a;
  up[u] = d - lower_bound_dev<int32_t>(col + a, d, (int32_t)u);
}

__global__ void k_gather_heavy(const int32_t *list, int nh, const u64 *W, const int32_t *lcnt,
                               int4 *info) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nh) return;
  int x = list[i];
  u64 w = W[x];
  info[i] = make_int4(x, lcnt[x], (int)(w & 0xffffffffu), (int)(w >> 32));
}

// ================================================================ Step 4 (host)

struct Plan {
  int64_t n = 0, nnz = 0, m = 0;
  int B = 1;
  bool per_edge = false;
  int max_deg = 0;   // known before the prepass (workspace sizing)
  int max_ucnt = 0;  // bound on |U(x)| used for sizing
};

inline u128 choose_h(u128 n, int k) {
  if (n < (u128)k) return 0;
  u128 r = 1;
  for (int i = 0; i < k; i++) r = r * (n - i) / (u128)(i + 1);
  return r;
}

// Divide exactly or flag an internal error.
inline bool exact_div(i128 a, int d, i128 *q) {
  if (a % d != 0) return false;
  *q = a / d;
  return true;
}

int finalize(const u128 A[kAcc], int64_t n_, int64_t m_, gc_u128 out[17]) {
  const i128 n = (i128)n_, m = (i128)m_;
  i128 g[17];
  i128 t;
  g[0] = m;                                                  // g2_1
  g[1] = (i128)choose_h((u128)n, 2) - m;                     // g2_2
  if (!exact_div((i128)A[A_T], 3, &g[2])) goto bad;          // Eq. "triangle"
  if (!exact_div((i128)A[A_S], 2, &g[3])) goto bad;          // Eq. "2-star"
  g[4] = (i128)A[A_I];                                       // Eq. "g3_3"
  g[5] = (i128)choose_h((u128)n, 3) - g[2] - g[3] - g[4];    // Eq. "g3_4"
  if (!exact_div((i128)A[A_K4], 6, &g[6])) goto bad;         // Cor. "cliq": 6 edges each
  if (!exact_div((i128)A[A_C4], 4, &g[9])) goto bad;         // Cor. "cyc": 4 edges each
  g[7] = (i128)A[A_TT] - 6 * g[6];                           // Lemma "rel-cliq-chcy"
  g[11] = (i128)A[A_SUSV] - 4 * g[9];                        // Lemma "rel-cyc-path"
  if (!exact_div((i128)A[A_TS] - 4 * g[7], 2, &g[8])) goto bad;   // Lemma "rel-ttri-chcy2"
  if (!exact_div((i128)A[A_SS] - g[8], 3, &g[10])) goto bad;      // Lemma "rel-ttri-3star"
  if (!exact_div((i128)A[A_TI] - g[8], 3, &g[12])) goto bad;      // Lemma "rel-4node-tri-ttri"
  if (!exact_div((i128)A[A_SI] - 2 * g[11], 2, &g[13])) goto bad; // Lemma "rel-4node-2star-path"
  t = (i128)A[A_II1] - (6 * g[6] + 4 * g[7] + 2 * g[8]) - (4 * g[9] + 2 * g[11]);
  if (!exact_div(t, 2, &g[14])) goto bad;                    // Eq. "g_4_9"
  g[15] = (i128)A[A_II] - 2 * g[14];                         // Lemma "rel-4node-2edge-1edge"
  t = 0;
  for (int i = 6; i <= 15; i++) t += g[i];
  g[16] = (i128)choose_h((u128)n, 4) - t;                    // Eq. "g_4_11"
  for (int i = 0; i < 17; i++)
    if (g[i] < 0) goto bad;
  for (int i = 0; i < 17; i++) {
    out[i].lo = (uint64_t)(u128)g[i];
    out[i].hi = (uint64_t)((u128)g[i] >> 64);
  }
  return GC_OK;
bad:
  set_error("exact identity check failed in the final step (internal error)");
  return GC_EINTERNAL;
}

// ================================================================ pipeline

struct Buffers {
  DevAcc *acc;
  Counters *cnt;
  int32_t *deg, *order, *rank, *deg2, *rp2, *col2, *lcnt, *ucnt, *ustart, *tpos;
  u64 *rkeys, *rkeys_alt, *ekeys, *ekeys_alt, *W;
  uint32_t *T;
  u64 *K4w, *C4w, *Dw;
  int32_t *tk[kTkBins], *c4l, *c4h;
  int64_t *cu;
  u64 *partials;
  int nstep3;
};

constexpr int kStep3Grid = 2048;

// Allocates every buffer of the plan (measuring or real).
void alloc_fixed(Arena &a, const Plan &P, Buffers &b) {
  const int64_t n = P.n, nnz = P.nnz;
  b.acc = a.take<DevAcc>(1);
  b.cnt = a.take<Counters>(1);
  b.deg = a.take<int32_t>(n);
  b.order = a.take<int32_t>(n);
  b.rank = a.take<int32_t>(n);
  b.deg2 = a.take<int32_t>(n);
  b.rp2 = a.take<int32_t>(n + 1);
  b.lcnt = a.take<int32_t>(n);
  b.ucnt = a.take<int32_t>(n);
  b.ustart = a.take<int32_t>(n);
  b.W = a.take<u64>(n);
  b.rkeys = a.take<u64>(n);
  b.rkeys_alt = a.take<u64>(n);
  b.ekeys = a.take<u64>(nnz);
  b.ekeys_alt = a.take<u64>(nnz);
  b.col2 = a.take<int32_t>(nnz);
  b.tpos = a.take<int32_t>(nnz);
  b.T = a.take<uint32_t>(nnz);
  for (int i = 0; i < kTkBins; i++) b.tk[i] = a.take<int32_t>(n);
  b.c4l = a.take<int32_t>(n);
  b.c4h = a.take<int32_t>(n);
  b.nstep3 = (int)std::min<int64_t>(kStep3Grid, std::max<int64_t>(1, (nnz + 255) / 256));
  b.partials = a.take<u64>((size_t)b.nstep3 * kAcc * 2);
  if (P.per_edge) {
    b.K4w = a.take<u64>(nnz);
    b.C4w = a.take<u64>(nnz);
    b.Dw = a.take<u64>(nnz);
    b.cu = a.take<int64_t>(n + 1);
  } else {
    b.K4w = b.C4w = b.Dw = nullptr;
    b.cu = nullptr;
  }
}

// Scratch for the two kernels that keep per-workgroup state in global memory.
struct Scratch {
  u64 *gR;
  int32_t *gI;
  u64 *gA;
  int32_t *gcur, *gbeg;
  u64 *gacc;
  int4 *items;
  int tk3_slots, c4_slots;
};

void alloc_scratch(Arena &a, const Plan &P, int kmax, int lmax, int64_t nitems, int c4_slots,
                   Scratch &s) {
  const size_t km = (size_t)std::max(kmax, 1), wm = (km + 63) / 64;
  s.tk3_slots = kTk3Slots;
  s.gR = a.take<u64>((size_t)kTk3Slots * km * wm);
  s.gI = a.take<int32_t>((size_t)kTk3Slots * (3 * km + 1));
  s.gA = a.take<u64>((size_t)kTk3Slots * 3 * km);
  s.c4_slots = c4_slots;
  const size_t lm = (size_t)std::max(lmax, 1);
  s.gcur = a.take<int32_t>((size_t)c4_slots * lm);
  if (P.per_edge) {
    s.gbeg = a.take<int32_t>((size_t)c4_slots * lm);
    s.gacc = a.take<u64>((size_t)c4_slots * lm);
  } else {
    s.gbeg = nullptr;
    s.gacc = nullptr;
  }
  s.items = a.take<int4>((size_t)std::max<int64_t>(nitems, 1));
}

int device_cu_count(int *out) {
  static int cached = 0;
  if (!cached) {
    int dev = 0;
    GC_TRY_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    GC_TRY_HIP(hipGetDeviceProperties(&prop, dev));
    cached = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  }
  *out = cached;
  return GC_OK;
}

int c4_slots_for(int lmax_bound) {
  (void)lmax_bound;
  int cus = 256;
  device_cu_count(&cus);
  return 2 * cus;  // two 512-thread workgroups per CU with 64 KiB LDS each
}

// Upper bounds that size the per-workgroup scratch before the prepass runs.
void scratch_bounds(const Plan &P, int *kmax, int *lmax, int64_t *items) {
  // |U(x)| <= sqrt(2m) under the degree order, and <= max degree.
  int64_t sq = 0;
  while ((sq + 1) * (sq + 1) <= 2 * P.m) sq++;
  *kmax = (int)std::min<int64_t>(P.max_ucnt > 0 ? P.max_ucnt : sq, P.max_deg);
  *lmax = P.max_deg;
  // pieces: at most (W / piece) + 1 per heavy vertex, and W sums to at most
  // sum_v d_v * |U(v)| <= 2m * kmax
  int64_t wsum_bound = P.nnz * (int64_t)std::max(*kmax, 1);
  *items = wsum_bound / (int64_t)kPieceWork + P.n + 1;
}

// HIP events at the phase boundaries of one call (only when timing is on).
struct PhaseEvents {
  static constexpr int kN = 8;
  hipEvent_t e[kN] = {};
  bool on = false;
  int init() {
    on = t_timing;
    if (!on) return GC_OK;
    for (int i = 0; i < kN; i++) GC_TRY_HIP(hipEventCreate(&e[i]));
    return GC_OK;
  }
  void record(int i, hipStream_t s) {
    if (on) (void)hipEventRecord(e[i], s);
  }
  ~PhaseEvents() {
    if (on)
      for (int i = 0; i < kN; i++)
        if (e[i]) (void)hipEventDestroy(e[i]);
  }
  float span(int a, int b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e[a], e[b]) != hipSuccess) return 0.f;
    return ms;
  }
};

int run_pipeline(const gc_csr *G, gc_u128 out17[17], int64_t *per_edge_out, Arena &a,
                 hipStream_t s, uint32_t flags, Plan &P) {
  Buffers b;
  alloc_fixed(a, P, b);
  int kmax_b, lmax_b;
  int64_t items_b;
  scratch_bounds(P, &kmax_b, &lmax_b, &items_b);
  const int c4_slots = c4_slots_for(lmax_b);
  Scratch sc;
  alloc_scratch(a, P, kmax_b, lmax_b, items_b, c4_slots, sc);
  if (a.measuring()) {
    // temporaries of the scans and sorts
    size_t m0 = a.mark();
    u64 *dummy;
    GC_TRY(radix_sort_u64(nullptr, nullptr, P.nnz, 2 * P.B, &dummy, a, s));
    a.release(m0);
    GC_TRY(radix_sort_u64(nullptr, nullptr, P.n, P.B + 32, &dummy, a, s));
    a.release(m0);
    GC_TRY(scan_exclusive<int32_t>(nullptr, nullptr, P.n + 1, a, s));
    a.release(m0);
    GC_TRY(scan_exclusive<int64_t>(nullptr, nullptr, P.n + 1, a, s));
    a.release(m0);
    return GC_OK;
  }
  if (a.overflow) {
    set_error("workspace too small");
    return GC_ENOMEM;
  }
  const int64_t n = P.n, nnz = P.nnz, m = P.m;
  const int B = P.B;
  PhaseEvents ev;
  GC_TRY(ev.init());
  for (int i = 0; i < PhaseEvents::kN; i++) ev.record(i, s);  // all valid even if a phase is empty

  // -- zero accumulators and counters (fill kernels, no memset nodes)
  GC_TRY(fill<u64>(reinterpret_cast<u64 *>(b.acc), 0ull, sizeof(DevAcc) / 8, s));
  GC_TRY(fill<int32_t>(reinterpret_cast<int32_t *>(b.cnt), 0, sizeof(Counters) / 4, s));
  GC_TRY(fill<u64>(b.W, 0ull, n, s));
  GC_TRY(fill<uint32_t>(b.T, 0u, nnz, s));
  if (P.per_edge) {
    GC_TRY(fill<u64>(b.K4w, 0ull, nnz, s));
    GC_TRY(fill<u64>(b.C4w, 0ull, nnz, s));
    GC_TRY(fill<u64>(b.Dw, 0ull, nnz, s));
  }

  // -- prepass: degree order, relabelled sorted lists
  ev.record(0, s);
  k_degree_keys<<<grid1d(n, 256), 256, 0, s>>>(G->row_ptr, n, B, b.deg, b.rkeys, &b.cnt->max_deg);
  GC_TRY_HIP(hipGetLastError());
  u64 *rsorted;
  GC_TRY(radix_sort_u64(b.rkeys, b.rkeys_alt, n, B + bits_for((u64)nnz), &rsorted, a, s));
  k_rank<<<grid1d(n, 256), 256, 0, s>>>(rsorted, n, B, b.order, b.rank, b.deg2);
  GC_TRY_HIP(hipGetLastError());
  GC_TRY(scan_exclusive<int32_t>(b.deg2, b.rp2, n, a, s));
  // rp2[n] = nnz
  {
    int32_t nz = (int32_t)nnz;
    GC_TRY(fill<int32_t>(b.rp2 + n, nz, 1, s));
  }
  k_edge_keys<<<grid1d(n * kWave, 256, 65536), 256, 0, s>>>(G->row_ptr, G->col, n, B, b.rank,
                                                           b.ekeys, &b.acc->err);
  GC_TRY_HIP(hipGetLastError());
  u64 *esorted;
  GC_TRY(radix_sort_u64(b.ekeys, b.ekeys_alt, nnz, 2 * B, &esorted, a, s));
  k_split_keys<<<grid1d(nnz, 256), 256, 0, s>>>(esorted, nnz, B, b.col2);
  k_split_rows<<<grid1d(n, 256), 256, 0, s>>>(b.rp2, b.col2, n, b.lcnt, b.ucnt, b.ustart,
                                               &b.cnt->max_ucnt);
  k_tpos<<<grid1d(nnz, 256), 256, 0, s>>>(esorted, b.col2, b.rp2, b.lcnt, nnz, B, b.tpos,
                                           &b.acc->err);
  k_wedges<<<grid1d(nnz, 256), 256, 0, s>>>(esorted, b.col2, b.rp2, b.tpos, b.ucnt, nnz, B, b.W,
                                            &b.cnt->clique_entries);
  k_bins<<<grid1d(n, 256), 256, 0, s>>>(b.ucnt, b.lcnt, b.W, n, b.tk[0], b.tk[1], b.tk[2],
                                        b.tk[3], b.c4l, b.c4h, b.cnt);
  GC_TRY_HIP(hipGetLastError());
  ev.record(1, s);
  Counters hc;
  int32_t perr = 0;
  GC_TRY_HIP(hipMemcpyAsync(&hc, b.cnt, sizeof hc, hipMemcpyDeviceToHost, s));
  GC_TRY_HIP(hipMemcpyAsync(&perr, &b.acc->err, 4, hipMemcpyDeviceToHost, s));
  GC_TRY_HIP(hipStreamSynchronize(s));
  if (perr != 0) {
    const int code = -(__builtin_ffs(perr) - 1);
    set_error("CSR contract violated (code %d); run with GC_VALIDATE for details", code);
    return code;
  }
  if (hc.max_ucnt > kmax_b || hc.max_lcnt_heavy > lmax_b) {
    set_error("internal sizing bound exceeded (kmax %d > %d or lmax %d > %d)", hc.max_ucnt,
              kmax_b, hc.max_lcnt_heavy, lmax_b);
    return GC_EINTERNAL;
  }

  // -- heavy wedge items (x, y range), largest first
  std::vector<int4> items;
  if (hc.c4_heavy > 0) {
    int4 *info = sc.items;  // reuse as staging, items are rebuilt below
    std::vector<int4> hinfo(hc.c4_heavy);
    k_gather_heavy<<<grid1d(hc.c4_heavy, 256), 256, 0, s>>>(b.c4h, hc.c4_heavy, b.W, b.lcnt,
                                                           info);
    GC_TRY_HIP(hipGetLastError());
    GC_TRY_HIP(hipMemcpyAsync(hinfo.data(), info, sizeof(int4) * hc.c4_heavy,
                              hipMemcpyDeviceToHost, s));
    GC_TRY_HIP(hipStreamSynchronize(s));
    struct It {
      int x, ya, yb;
      u64 w;
    };
    std::vector<It> v;
    for (const int4 &h : hinfo) {
      const int x = h.x, nL = h.y;
      const u64 w = (u64)(uint32_t)h.z | ((u64)(uint32_t)h.w << 32);
      const int K = nL < 65536 ? 2 * kChunkWords : kChunkWords;
      const int64_t nchunks = ((int64_t)x + K - 1) / K;
      int64_t S = (int64_t)((w + kPieceWork - 1) / kPieceWork);
      S = std::max<int64_t>(1, std::min<int64_t>(S, nchunks));
      for (int64_t sidx = 0; sidx < S; sidx++) {
        int64_t c0 = nchunks * sidx / S, c1 = nchunks * (sidx + 1) / S;
        int ya = (int)(c0 * K), yb = (int)std::min<int64_t>(c1 * K, x);
        if (yb > ya) v.push_back({x, ya, yb, w / (u64)S});
      }
    }
    std::sort(v.begin(), v.end(), [](const It &p, const It &q) { return p.w > q.w; });
    if ((int64_t)v.size() > items_b) {
      set_error("internal sizing bound exceeded (items)");
      return GC_EINTERNAL;
    }
    items.resize(v.size());
    for (size_t i = 0; i < v.size(); i++) items[i] = make_int4(v[i].x, v[i].ya, v[i].yb, 0);
    GC_TRY_HIP(hipMemcpyAsync(sc.items, items.data(), sizeof(int4) * items.size(),
                              hipMemcpyHostToDevice, s));
  }

  // -- Steps 1 + 2a: triangles and 4-cliques
  ev.record(2, s);
  TkArgs tk{};
  tk.col2 = b.col2;
  tk.ustart = b.ustart;
  tk.ucnt = b.ucnt;
  tk.T = b.T;
  tk.K4w = b.K4w;
  tk.Dw = b.Dw;
  tk.k4x3 = b.acc->k4x3;
  tk.gR = sc.gR;
  tk.gI = sc.gI;
  tk.gA = sc.gA;
  tk.kmax = kmax_b;
  auto launch_tk = [&](bool per_edge) -> int {
    for (int bin = 0; bin < kTkBins; bin++) {
      const int cntb = hc.tk_cnt[bin];
      if (cntb == 0) continue;
      tk.list = b.tk[bin];
      tk.nlist = cntb;
      if (bin == 0) {
        unsigned grid = (unsigned)std::min(cntb, 65536);
        if (per_edge) k_tk_lds<64, kTkLim0, true><<<grid, 64, 0, s>>>(tk);
        else k_tk_lds<64, kTkLim0, false><<<grid, 64, 0, s>>>(tk);
      } else if (bin == 1) {
        unsigned grid = (unsigned)std::min(cntb, 16384);
        if (per_edge) k_tk_lds<256, kTkLim1, true><<<grid, 256, 0, s>>>(tk);
        else k_tk_lds<256, kTkLim1, false><<<grid, 256, 0, s>>>(tk);
      } else if (bin == 2) {
        unsigned grid = (unsigned)std::min(cntb, 4096);
        if (per_edge) k_tk_lds<256, kTkLim2, true><<<grid, 256, 0, s>>>(tk);
        else k_tk_lds<256, kTkLim2, false><<<grid, 256, 0, s>>>(tk);
      } else {
        unsigned grid = (unsigned)std::min(cntb, sc.tk3_slots);
        if (per_edge) k_tk_global<256, true><<<grid, 256, 0, s>>>(tk);
        else k_tk_global<256, false><<<grid, 256, 0, s>>>(tk);
      }
      GC_TRY_HIP(hipGetLastError());
    }
    return GC_OK;
  };
  GC_TRY(launch_tk(false));
  ev.record(3, s);

  // -- Step 2b: 4-cycles by wedges
  C4Args c4{};
  c4.col2 = b.col2;
  c4.rp2 = b.rp2;
  c4.lcnt = b.lcnt;
  c4.tpos = b.tpos;
  c4.W = b.W;
  c4.c4ni = b.acc->c4ni;
  c4.C4w = b.C4w;
  c4.lmax = lmax_b;
  c4.gcur = sc.gcur;
  c4.gbeg = sc.gbeg;
  c4.gacc = sc.gacc;
  if (hc.c4_light > 0) {
    c4.list = b.c4l;
    c4.nlist = hc.c4_light;
    unsigned grid = (unsigned)std::min(hc.c4_light, 65536);
    if (P.per_edge) k_c4_light<true><<<grid, kWave, 0, s>>>(c4);
    else k_c4_light<false><<<grid, kWave, 0, s>>>(c4);
    GC_TRY_HIP(hipGetLastError());
  }
  ev.record(4, s);
  if (!items.empty()) {
    c4.items = sc.items;
    c4.nitems = (int)items.size();
    c4.queue = &b.acc->queue;
    unsigned grid = (unsigned)std::min<int64_t>((int64_t)items.size(), sc.c4_slots);
    if (P.per_edge) k_c4_heavy<true><<<grid, kC4HeavyBlock, 0, s>>>(c4);
    else k_c4_heavy<false><<<grid, kC4HeavyBlock, 0, s>>>(c4);
    GC_TRY_HIP(hipGetLastError());
  }

  ev.record(5, s);
  // -- per-edge 4-cliques and D_e (needs final |Tri|)
  if (P.per_edge) GC_TRY(launch_tk(true));
  ev.record(6, s);

  // -- Step 3
  S3Args s3{};
  s3.ekeys = esorted;
  s3.col2 = b.col2;
  s3.deg2 = b.deg2;
  s3.T = b.T;
  s3.K4w = b.K4w;
  s3.C4w = b.C4w;
  s3.Dw = b.Dw;
  s3.nnz = nnz;
  s3.n = n;
  s3.m = m;
  s3.B = B;
  s3.partials = b.partials;
  if (P.per_edge) {
    k_orig_upper<<<grid1d(n, 256), 256, 0, s>>>(G->row_ptr, G->col, n, b.cu);
    GC_TRY_HIP(hipGetLastError());
    GC_TRY(scan_exclusive<int64_t>(b.cu, b.cu, n, a, s));
    s3.order = b.order;
    s3.rp = G->row_ptr;
    s3.col = G->col;
    s3.cu = b.cu;
    s3.out = per_edge_out;
    k_step3<true><<<b.nstep3, 256, 0, s>>>(s3);
  } else {
    k_step3<false><<<b.nstep3, 256, 0, s>>>(s3);
  }
  GC_TRY_HIP(hipGetLastError());
  k_step3_final<<<kAcc, kWave, 0, s>>>(b.partials, b.nstep3, b.acc);
  GC_TRY_HIP(hipGetLastError());
  ev.record(7, s);

  DevAcc h;
  GC_TRY_HIP(hipMemcpyAsync(&h, b.acc, sizeof h, hipMemcpyDeviceToHost, s));
  GC_TRY_HIP(hipStreamSynchronize(s));
  if (ev.on) {
    gc_timing &t = t_last_timing;
    t.ms[0] = ev.span(0, 1);
    t.ms[1] = ev.span(2, 3);
    t.ms[2] = ev.span(3, 4);
    t.ms[3] = ev.span(4, 5);
    t.ms[4] = ev.span(5, 6);
    t.ms[5] = ev.span(6, 7);
    t.clique_entries = hc.clique_entries;
    t.wedges_light = hc.wedges_light;
    t.wedges_heavy = hc.wedges_heavy;
    t.heavy_items = (int64_t)items.size();
  }
  u128 A[kAcc];
  for (int i = 0; i < kAcc; i++) A[i] = ((u128)h.step3[i][1] << 64) | h.step3[i][0];
  if (!P.per_edge) {
    // sum_e K4_e = 6 x cliques; sum_e C4_e = 4 C4ni - sum_e D_e + 2 sum_e K4_e
    // with sum_e D_e = 4 sum_e C(T_e, 2).
    const u128 k4x3 = ((u128)h.k4x3[1] << 64) | h.k4x3[0];
    const u128 c4ni = ((u128)h.c4ni[1] << 64) | h.c4ni[0];
    A[A_K4] = 2 * k4x3;
    const i128 c4 = 4 * (i128)c4ni - 4 * (i128)A[A_TT] + 2 * (i128)A[A_K4];
    if (c4 < 0) {
      set_error("negative 4-cycle total (internal error)");
      return GC_EINTERNAL;
    }
    A[A_C4] = (u128)c4;
  }
  return finalize(A, n, m, out17);
}

__global__ void k_max_deg(const int32_t *rp, int64_t n, int32_t *out) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int mx = 0;
  if (u < n) mx = rp[u + 1] - rp[u];
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, kWave));
  if (lane_id() == 0) atomicMax(out, mx);
}

// max over vertices of |U(x)|: neighbours later in the (degree, id) order.
__global__ void k_max_ucnt(const int32_t *rp, const int32_t *col, int64_t n, int32_t *out) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int lane = lane_id();
  for (int64_t u = wave; u < n; u += nwaves) {
    const int a = rp[u], b = rp[u + 1], du = b - a;
    int c = 0;
    for (int j = a + lane; j < b; j += kWave) {
      const int w = col[j];
      if (w < 0 || w >= n) continue;  // broken contract: never used as an index
      const int dw = rp[w + 1] - rp[w];
      c += (dw > du || (dw == du && w > u)) ? 1 : 0;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, kWave);
    if (lane == 0) atomicMax(out, c);
  }
}

// Reads the maximum degree and maximum |U(x)| (two small kernels, one sync).
int probe_graph(const gc_csr *g, hipStream_t s, int *max_deg, int *max_ucnt) {
  *max_deg = 0;
  *max_ucnt = 0;
  if (g->n == 0 || g->nnz == 0) return GC_OK;
  int32_t *d = nullptr;
  GC_TRY_HIP(hipMallocAsync((void **)&d, 8, s));
  int32_t h[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(d, h, 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    k_max_deg<<<grid1d(g->n, 256), 256, 0, s>>>(g->row_ptr, g->n, d);
    k_max_ucnt<<<grid1d(g->n * kWave, 256, 65536), 256, 0, s>>>(g->row_ptr, g->col, g->n, d + 1);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h, d, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipError_t f = hipFreeAsync(d, s);
  if (e == hipSuccess) e = f;
  if (e != hipSuccess) {
    set_error("probe: %s", hipGetErrorString(e));
    return GC_EHIP;
  }
  *max_deg = h[0];
  *max_ucnt = h[1];
  return GC_OK;
}

int check_args(const gc_csr *g) {
  if (!g) {
    set_error("null graph");
    return GC_EINVAL;
  }
  if (g->n < 0 || g->nnz < 0 || g->n > 2147483646LL || g->nnz > 2147483646LL || (g->nnz & 1)) {
    set_error("invalid sizes n=%lld nnz=%lld", (long long)g->n, (long long)g->nnz);
    return GC_EINVAL;
  }
  if (!g->row_ptr || (g->nnz > 0 && !g->col)) {
    set_error("null CSR array");
    return GC_EINVAL;
  }
  return GC_OK;
}

// Counts of a graph with no edges: only the independent classes.
void counts_no_edges(int64_t n, gc_u128 out[17]) {
  memset(out, 0, sizeof(gc_u128) * 17);
  u128 c2 = choose_h((u128)n, 2), c3 = choose_h((u128)n, 3), c4 = choose_h((u128)n, 4);
  out[1].lo = (uint64_t)c2;
  out[1].hi = (uint64_t)(c2 >> 64);
  out[5].lo = (uint64_t)c3;
  out[5].hi = (uint64_t)(c3 >> 64);
  out[16].lo = (uint64_t)c4;
  out[16].hi = (uint64_t)(c4 >> 64);
}

}  // namespace

size_t workspace_size(const gc_csr *g, int per_edge, hipStream_t s, int *rc) {
  *rc = check_args(g);
  if (*rc) return 0;
  Plan P;
  P.n = g->n;
  P.nnz = g->nnz;
  P.m = g->nnz / 2;
  P.per_edge = per_edge != 0;
  P.B = std::max(1, bits_for((u64)std::max<int64_t>(g->n - 1, 1)));
  if (P.n == 0 || P.nnz == 0) return 256;
  *rc = probe_graph(g, s, &P.max_deg, &P.max_ucnt);
  if (*rc) return 0;
  Arena a;
  *rc = run_pipeline(g, nullptr, nullptr, a, s, 0, P);
  if (*rc) return 0;
  return a.peak + 4096;
}

int count(const gc_csr *g, gc_u128 out[17], int64_t *per_edge_out, void *ws, size_t ws_bytes,
          hipStream_t s, uint32_t flags) {
  GC_TRY(check_args(g));
  if (!out) {
    set_error("null output");
    return GC_EINVAL;
  }
  if (g->nnz == 0) {
    if ((flags & GC_VALIDATE) && g->n > 0) {
      // row_ptr must be all zeros
      std::vector<int32_t> h(g->n + 1);
      GC_TRY_HIP(hipMemcpyAsync(h.data(), g->row_ptr, sizeof(int32_t) * (g->n + 1),
                                hipMemcpyDeviceToHost, s));
      GC_TRY_HIP(hipStreamSynchronize(s));
      for (int32_t v : h)
        if (v != 0) {
          set_error("row_ptr inconsistent with nnz = 0");
          return GC_EINVAL;
        }
    }
    counts_no_edges(g->n, out);
    return GC_OK;
  }
  Plan P;
  P.n = g->n;
  P.nnz = g->nnz;
  P.m = g->nnz / 2;
  P.per_edge = per_edge_out != nullptr;
  P.B = std::max(1, bits_for((u64)std::max<int64_t>(g->n - 1, 1)));
  if (flags & GC_VALIDATE) {
    // bounds checks before anything dereferences the lists
    Arena va;
    int32_t *e = nullptr;
    GC_TRY_HIP(hipMallocAsync((void **)&e, 4, s));
    int32_t zero = 0, err = 0;
    hipError_t he = hipMemcpyAsync(e, &zero, 4, hipMemcpyHostToDevice, s);
    if (he == hipSuccess) {
      k_check_rowptr_ends<<<1, 64, 0, s>>>(g->row_ptr, g->n, g->nnz, e);
      k_validate<<<grid1d(g->n, 256, 16384), 256, 0, s>>>(g->row_ptr, g->col, g->n, g->nnz, e);
      he = hipGetLastError();
    }
    if (he == hipSuccess) he = hipMemcpyAsync(&err, e, 4, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    (void)hipFreeAsync(e, s);
    if (he != hipSuccess) {
      set_error("validation: %s", hipGetErrorString(he));
      return GC_EHIP;
    }
    if (err != 0) {
      const int code = -(__builtin_ffs(err) - 1);
      set_error("CSR contract violated (code %d)", code);
      return code;
    }
    flags &= ~GC_VALIDATE;
  }
  GC_TRY(probe_graph(g, s, &P.max_deg, &P.max_ucnt));
  Arena meas;
  GC_TRY(run_pipeline(g, nullptr, nullptr, meas, s, 0, P));
  const size_t need = meas.peak + 4096;
  void *own = nullptr;
  if (!ws) {
    hipError_t e = hipMallocAsync(&own, need, s);
    if (e != hipSuccess) {
      set_error("device allocation of %zu bytes failed: %s", need, hipGetErrorString(e));
      return GC_ENOMEM;
    }
    ws = own;
    ws_bytes = need;
  } else if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    return GC_ENOMEM;
  }
  Arena a;
  a.base = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(ws) + 255) & ~uintptr_t(255));
  a.cap = ws_bytes - (size_t)(a.base - reinterpret_cast<char *>(ws));
  int rc = run_pipeline(g, out, per_edge_out, a, s, flags, P);
  if (own) {
    hipError_t e = hipFreeAsync(own, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (rc == GC_OK && e != hipSuccess) {
      set_error("hipFreeAsync: %s", hipGetErrorString(e));
      rc = GC_EHIP;
    }
  }
  return rc;
}

}  // namespace gc

// ================================================================ C ABI

extern "C" {

size_t graphlet_workspace_size(const gc_csr *g, int per_edge, void *stream) {
  gc::clear_error();
  int rc = 0;
  try {
    return gc::workspace_size(g, per_edge, (hipStream_t)stream, &rc);
  } catch (...) {
    gc::set_error("unexpected exception");
    return 0;
  }
}

int graphlet_count(const gc_csr *g, gc_u128 out_counts[17], int64_t *per_edge_out,
                   void *workspace, size_t ws_bytes, void *stream, uint32_t flags) {
  gc::clear_error();
  try {
    return gc::count(g, out_counts, per_edge_out, workspace, ws_bytes, (hipStream_t)stream, flags);
  } catch (...) {
    gc::set_error("unexpected exception");
    return GC_EINTERNAL;
  }
}

const char *graphlet_last_error(void) { return gc::last_error(); }

void graphlet_timing_enable(int on) { gc::t_timing = on != 0; }

int graphlet_last_timing(gc_timing *out) {
  if (!out) return GC_EINVAL;
  *out = gc::t_last_timing;
  return GC_OK;
}

const char *graphlet_version(void) { return "graphlet-mi355x 0.1"; }

}  // extern "C"
