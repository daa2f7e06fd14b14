// Per-vertex counts from per-edge terms: the algebra shared by the
// single-graph per-vertex kernel and the batched one.  See vertex.hip for
// the derivation.  Everything is modulo 2^64; results are exact while every
// per-vertex count is below 2^64 (each division is applied to a sum whose
// true value is a non-negative multiple of the divisor).
#pragma once

#include "common.h"

namespace gc {

constexpr int kVxAcc = 19;

__device__ __forceinline__ u64 vx_c2(u64 x) { return x * (x - 1) / 2 * (x > 1); }

// The terms of one edge (v, w) of vertex v fall into three groups, each
// summed over v's edges: those that depend only on |Tri_e| = T, the two
// degrees d, dw and n; those linear in w's triangles tw and neighbour-degree
// sum sw (with v's own t, s and m); and those linear in the per-edge K4
// (4-cliques through e), C4 (induced 4-cycles through e), D (sum over a in
// Tri_e of |Tri_(v,a)| + |Tri_(w,a)| - 2) and B (sum of degrees over Tri_e).
// The last group may be given the sums of K4, C4, D and B over v's edges in
// one call.
__device__ __forceinline__ void vx_add_edge_tri(u64 (&a)[kVxAcc], u64 T, u64 d, u64 dw, u64 n) {
  const u64 Sv = d - 1 - T, Sw = dw - 1 - T, I = n - d - dw + T;
  a[1] += T * T;
  a[2] += vx_c2(T);
  a[7] += vx_c2(dw) - dw;
  a[9] += dw * T;
  a[10] += vx_c2(Sv);
  a[11] += vx_c2(Sw);
  a[12] += Sv * Sw;
  a[13] += T * I;
  a[14] += Sv * I;
  a[15] += Sw * I;
  a[16] += vx_c2(I);
  a[17] += 1 + Sv + Sw;
  a[18] += I;
}

__device__ __forceinline__ void vx_add_edge_other(u64 (&a)[kVxAcc], u64 tw, u64 sw, u64 t, u64 s,
                                                  u64 m) {
  a[6] += tw;
  a[7] += sw - 3 * tw;  // with the degree part: induced 2-stars at w
  a[8] += sw;
  a[17] += m - s - sw + t + tw;
}

__device__ __forceinline__ void vx_add_edge_sums(u64 (&a)[kVxAcc], u64 K4, u64 C4, u64 D, u64 B) {
  a[0] += K4;
  a[3] += D;
  a[4] += C4;
  a[5] += B;
  // I-I adjacent pairs of the edge: m minus the edges touching {v, w} or
  // Tri_e, S_v, S_w; only these parts are linear in K4, C4, D, B
  a[17] += B + C4 - K4;
}

// All terms of one edge (v, w) of vertex v; (d, t, s) of v and (dw, tw, sw)
// of w are degree, triangles and neighbour-degree sum.
__device__ __forceinline__ void vx_add_edge(u64 (&a)[kVxAcc], u64 T, u64 K4, u64 C4, u64 D,
                                            u64 B, u64 d, u64 t, u64 s, u64 dw, u64 tw, u64 sw,
                                            u64 n, u64 m) {
  vx_add_edge_tri(a, T, d, dw, n);
  vx_add_edge_other(a, tw, sw, t, s, m);
  vx_add_edge_sums(a, K4, C4, D, B);
}

// The 17 counts of vertex v (order g2_1 .. g4_11) from its summed edge terms,
// its (d, t, s), and the graph's n, m, triangles and induced 2-stars.
__device__ __forceinline__ void vx_counts(const u64 (&a)[kVxAcc], u64 d, u64 t, u64 s, u64 n,
                                          u64 m, u64 tri, u64 star, u64 (&r)[17]) {
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
  const u64 tri_far = tri - stw + X - K4v;
  const u64 g32v = vx_c2(d) + s - d - 3 * t;
  const u64 c4ni = (sC4 + sD - 2 * sK4) / 2;  // non-induced 4-cycles through v
  const u64 q1 = g32v + sg32w;
  const u64 q2 = (d * d + s - 2 * d - 4 * t) + (sY - 2 * t - 2 * X) + (vx_c2(d) + c4ni - X);
  const u64 q3 = (vx_c2(d) - t) + sTC2 - 3 * K4v;
  const u64 star_far = star - (q1 - q2 + q3);
  const u64 mR = m - s + t, nR = n - 1 - d;
  const u64 e1_far = mR * (nR - 2) - 2 * star_far - 3 * tri_far;
  r[0] = d;
  r[1] = n - 1 - d;
  r[2] = t;
  r[3] = g32v;
  r[4] = sI + mR;
  r[5] = vx_c2(n - 1) - r[2] - r[3] - r[4];
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
}

}  // namespace gc
