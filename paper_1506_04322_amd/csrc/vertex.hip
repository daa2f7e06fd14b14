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

namespace gc {
namespace {

constexpr int kVxBlock = 256;
constexpr int kVxAcc = 19;

__device__ __forceinline__ u64 c2(u64 x) { return x * (x - 1) / 2 * (x > 1); }

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
      const u64 dw = (u64)g.deg2[y], tw = g.tv[y] / 2, sw = g.sv[y];
      const u64 Sv = d - 1 - T, Sw = dw - 1 - T, I = n - d - dw + T;
      // I-I adjacent pairs of the edge (the undirected local-vector term)
      const u64 TS1 = D - 4 * K4, SS1 = t + tw + 2 * K4 - D - 2 * T;
      const u64 eX = 1 + 2 * T + Sv + Sw + K4 + TS1 + SS1 + C4;
      a[0] += K4;
      a[1] += T * T;
      a[2] += c2(T);
      a[3] += D;
      a[4] += C4;
      a[5] += B;
      a[6] += tw;
      a[7] += c2(dw) + sw - dw - 3 * tw;  // induced 2-stars at w
      a[8] += sw;
      a[9] += dw * T;
      a[10] += c2(Sv);
      a[11] += c2(Sw);
      a[12] += Sv * Sw;
      a[13] += T * I;
      a[14] += Sv * I;
      a[15] += Sw * I;
      a[16] += c2(I);
      a[17] += m - (s + sw - B) + eX;
      a[18] += I;
    }
#pragma unroll
    for (int k = 0; k < kVxAcc; k++) a[k] = wave_sum_u64(a[k]);
    const u64 sK4 = a[0], sT2 = a[1], sTC2 = a[2], sD = a[3], sC4 = a[4], sB = a[5];
    const u64 stw = a[6], sg32w = a[7], ssw = a[8], sY = a[9], sSvC2 = a[10], sSwC2 = a[11];
    const u64 sSvSw = a[12], sTI = a[13], sSvI = a[14], sSwI = a[15], sIC2 = a[16];
    const u64 sII1 = a[17], sI = a[18];

    const u64 K4v = sK4 / 3;
    const u64 TSown1 = sT2 - 2 * t - 2 * sK4;
    const u64 Aw = sD + 4 * t - sT2;  // sum_e A_w(e)
    const u64 TSoth1 = Aw - 2 * t - 2 * sK4;
    const u64 SSown1 = d * t - sT2 + sK4;
    const u64 SSoth1 = stw - Aw + sK4;
    const u64 TI1 = sB - 4 * t + 2 * sK4 - sD;
    const u64 SSown0 = sSvC2 - SSown1, SSoth0 = sSwC2 - SSoth1;
    const u64 SvSw0 = sSvSw - sC4;
    const u64 sumSw = s - d - 2 * t, sumSv = d * (d - 1) - 2 * t;
    const u64 SothI1 = ssw - d * d - sB - sumSw - TSoth1 - 2 * SSoth1 - sC4;
    const u64 SownI1 = d * s - s - sB - sumSv - TSown1 - 2 * SSown1 - sC4;
    const u64 TI0 = sTI - TI1;
    const u64 SownI0 = sSvI - SownI1, SothI0 = sSwI - SothI1;
    // the rest R = V \ N[v]
    const u64 X = Aw / 2;
    const u64 tri_far = g.tri - stw + X - K4v;
    const u64 g32v = c2(d) + s - d - 3 * t;
    const u64 c4ni = (sC4 + sD - 2 * sK4) / 2;  // non-induced 4-cycles through v
    const u64 q1 = g32v + sg32w;
    const u64 q2 = (d * d + s - 2 * d - 4 * t) + (sY - 2 * t - 2 * X) + (c2(d) + c4ni - X);
    const u64 q3 = (c2(d) - t) + sTC2 - 3 * K4v;
    const u64 star_far = g.star - (q1 - q2 + q3);
    const u64 mR = m - s + t, nR = n - 1 - d;
    const u64 e1_far = mR * (nR - 2) - 2 * star_far - 3 * tri_far;

    u64 r[17];
    r[0] = d;
    r[1] = n - 1 - d;
    r[2] = t;
    r[3] = g32v;
    r[4] = sI + mR;
    r[5] = c2(n - 1) - r[2] - r[3] - r[4];
    r[6] = K4v;
    r[7] = (sTC2 - sK4) + TSoth1 / 2;
    r[8] = SSown1 + SSoth1 + TI1;
    r[9] = sC4 / 2;
    r[10] = SSown0 / 3 + SSoth0;
    r[11] = SvSw0 + SothI1;
    r[12] = TI0 / 2 + tri_far;
    r[13] = SownI0 / 2 + SothI0 + star_far;
    r[14] = sII1;
    r[15] = (sIC2 - sII1) + e1_far;
    // C(n-1, 3) modulo 2^64: one of three consecutive integers is divisible by 3
    u64 a0 = n - 1, a1 = n - 2, a2 = n - 3;
    if (n < 4) a0 = a1 = a2 = 0;
    if (a0 % 3 == 0) a0 /= 3;
    else if (a1 % 3 == 0) a1 /= 3;
    else a2 /= 3;
    if (a0 % 2 == 0) a0 /= 2;
    else a1 /= 2;
    u64 rest = a0 * a1 * a2;
#pragma unroll
    for (int k = 6; k < 16; k++) rest -= r[k];
    r[16] = rest;
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
