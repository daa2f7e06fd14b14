// Per-vertex graphlet counts: for every vertex v and each of the 17 classes of
// Table 1, the number of induced k-subsets S with v in S whose induced
// subgraph is that class.
//
// The per-edge local 4-node vectors of Section 4.2 count, for an edge e =
// (v, w), the 4-sets {v, w, a, b} by the types of a and b relative to e (T:
// adjacent to both ends, S_v / S_w: to one end, I: to neither) and by whether
// a and b are adjacent.  Every class and every position of v in it (its
// degree inside S) corresponds to a fixed set of these types, so a subset in
// which v has degree delta > 0 is seen delta times over v's incident edges.
// The terms that tell the two ends of e apart come from two sums over v's
// edges, using A_v(e) = sum over a in Tri_e of |Tri_(v,a)|:
//   sum_e A_v(e) = sum_e |Tri_e|^2     (a in N(v) is in Tri_e for |Tri_(v,a)| edges)
//   sum_e A_w(e) = sum_e (D_e + 2|Tri_e|) - sum_e |Tri_e|^2
// with D_e = A_v + A_w - 2|Tri_e| the per-edge sum the clique pass keeps.
// Directed terms (w the other end; t_x triangles at x, s_x sum of the degrees
// of x's neighbours, B_e sum of degrees over Tri_e, C4 induced 4-cycles of e):
//   N_{T,Sv,1} = A_v - T - 2K4            N_{T,Sw,1} = A_w - T - 2K4
//   N_{Sv,Sv,1} = t_v - A_v + K4          N_{Sw,Sw,1} = t_w - A_w + K4
//   N_{Sv,I,1} = s_v - d_w - B - Sv - N_{T,Sv,1} - 2 N_{Sv,Sv,1} - C4
// (the degrees of the S_v vertices split into v, T, S_v, S_w and I
// neighbours), and the other ends' terms are the undirected ones.
//
// Subsets in which v has no neighbour (g2_2, g3_3, g3_4, g4_7, g4_8, g4_10,
// g4_11) need the (k-1)-node graphlets of G minus the closed neighbourhood
// N[v].  By inclusion and exclusion over the vertices of a triangle (or an
// induced 2-star) that lie in N[v]:
//   triangles touching N[v] = sum_{x in N[v]} t_x - sum over pairs in N[v]
//                              + those inside N[v]
//   triangles avoiding N[v] = t - sum_{w in N(v)} t_w + X - K4(v)
// where X = sum of |Tri| over the edges inside N(v) = sum_e A_w(e) / 2, and
// for induced 2-stars the pair term uses |S_x| + |S_y| for adjacent pairs and
// the common-neighbour count for the others (whose total over pairs in N(v)
// is C(d_v, 2) plus the non-induced 4-cycles through v).  The 1-edge
// 3-subsets of the rest follow from edges(R)(|R| - 2) - 2 stars - 3 triangles
// and g4_11 closes the C(n-1, 3) subsets containing v.
//
// All per-vertex arithmetic is modulo 2^64: every result is exact when
// C(n-1, 3) < 2^64 (checked by the host), and each division is applied to a
// sum whose true value is a non-negative multiple of the divisor below that
// bound.
#include "kernels.h"
#include "vertex_terms.h"

namespace gc {
namespace {

constexpr int kVxBlock = 256;

__global__ __launch_bounds__(kVxBlock) void k_vertex_counts(VxArgs g) {
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * (kVxBlock / kWave);
  const u64 n = (u64)g.n, m = (u64)g.m;
  for (int64_t i = (int64_t)blockIdx.x * (kVxBlock / kWave) + threadIdx.x / kWave; i < g.n;
       i += waves) {
    // highest ranks (largest degrees) first, so the long rows start early
    const int32_t x = (int32_t)(g.n - 1 - i);
    const int32_t r0 = g.rp2[x], r1 = g.rp2[x + 1], nl = g.lcnt[x];
    const u64 d = (u64)(r1 - r0), t = g.tv[x] / 2, s = g.sv[x];
    u64 a[kVxAcc];
#pragma unroll
    for (int k = 0; k < kVxAcc; k++) a[k] = 0;
    for (int q = r0 + lane; q < r1; q += kWave) {
      const int32_t y = g.col2[q];
      const int64_t p = (q - r0 < nl) ? g.tpos[q] : q;  // upper position of the edge
      const u64 T = g.T[p], K4 = g.K4w[p], D = g.Dw[p], B = g.Bw[p];
      const u64 C4 = g.C4w[p] - D + 2 * K4;  // induced 4-cycles; wraps cancel
      vx_add_edge(a, T, K4, C4, D, B, d, t, s, (u64)g.deg2[y], g.tv[y] / 2, g.sv[y], n, m);
    }
#pragma unroll
    for (int k = 0; k < kVxAcc; k++) a[k] = wave_sum_u64(a[k]);
    u64 r[17];
    vx_counts(a, d, t, s, n, m, g.tri, g.star, r);
    const int64_t id = g.order[x];
    if (lane < 17) {
      u64 v = r[0];
#pragma unroll
      for (int k = 1; k < 17; k++)
        if (lane == k) v = r[k];
      g.out[(int64_t)lane * g.n + id] = v;
    }
  }
}

}  // namespace

int launch_vertex_counts(const VxArgs &g, hipStream_t s) {
  if (g.n <= 0) return GC_OK;
  const int64_t blocks = (g.n + kVxBlock / kWave - 1) / (kVxBlock / kWave);
  const unsigned grid = (unsigned)std::min<int64_t>(blocks, 8192);
  k_vertex_counts<<<grid, kVxBlock, 0, s>>>(g);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

}  // namespace gc
