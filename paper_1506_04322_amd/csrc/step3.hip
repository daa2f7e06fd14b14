// Step 3: per edge, the unrestricted counts of Section 4.2 in constant time,
// summed exactly.
//
// For e = (u, v) with T = |Tri_e|, Su = |Star_u| = d_u - 1 - T,
// Sv = |Star_v| = d_v - 1 - T and I = |V| - |N(u) u N(v)| = n - d_u - d_v + T
// (the union holds u and v themselves), Equations "comb_n_ai_ai" and
// "comb_n_ai_aj" give N_{T,T} = C(T,2), N_{Su,Sv} = Su Sv, ..., N_{I,I} =
// C(I,2), and the graphlet counting algorithm adds |E| - d_u - d_v + 1 toward
// N_{I,I,1}.  Every per-edge term fits 64 bits (each factor is below 2^31);
// the sums do not (C(I,2) summed over R-MAT scale 22 is ~5e20), so each
// thread accumulates in 128 bits and blocks reduce exactly.
#include "kernels.h"

namespace gc {

namespace {

__device__ __forceinline__ u64 choose2(u64 c) { return c * (c - 1) / 2; }

// The per-edge local 4-node vector of e = (x, y) (Section 4.2): the
// unrestricted counts N_{a,b} from T, Su, Sv, I, and the restricted ones
// N_{a,b,1} from per-edge and per-vertex sums.  With A_u = sum over w in
// Tri_e of |Tri_(u,w)|, D = A_u + A_v - 2T, B = sum over Tri_e of deg(w),
// t_u the triangles at u and s_u the degree sum over N(u):
//   N_{T,S,1}  = D - 4 K4           (each w in Tri_e sees |Tri_(u,w)| - 1
//                                     vertices of N(u) - v, 2 K4 of them in Tri_e)
//   N_{S,S,1}  = t_u + t_v + 2 K4 - D - 2T   (edges inside N(u) by kind)
//   N_{T,I,1}  = B - 2T - 2K4 - N_{T,S,1}     (degrees of the Tri_e vertices)
//   N_{S,I,1}  = s_u + s_v - d_u - d_v - 2B - (Su + Sv) - (D - 4K4)
//                - 2 N_{S,S,1} - 2 C4         (degrees of the star vertices)
//   N_{I,I,1}  = m - (s_u + s_v - B) + e(X), X = N(u) u N(v) holding
//                e(X) = 1 + 2T + Su + Sv + K4 + N_{T,S,1} + N_{S,S,1} + C4
// and N_{a,b,0} = N_{a,b} - N_{a,b,1}.  Output order as the oracle's.
__device__ __forceinline__ void write_local(const S3Args &g, int64_t id, int64_t p, int32_t x,
                                            int32_t y, int64_t T, int64_t K4, int64_t C4) {
  const int64_t n = g.n, m = g.m;
  const int64_t du = g.deg2[x], dv = g.deg2[y];
  const int64_t Su = du - 1 - T, Sv = dv - 1 - T, S = Su + Sv, I = n - du - dv + T;
  const int64_t D = (int64_t)g.Dw[p], B = (int64_t)g.Bw[p];
  const int64_t tu = (int64_t)(g.tv[x] / 2), tw = (int64_t)(g.tv[y] / 2);
  const int64_t su = (int64_t)g.sv[x], sw = (int64_t)g.sv[y];
  const int64_t TS1 = D - 4 * K4;
  const int64_t SS1 = tu + tw + 2 * K4 - D - 2 * T;
  const int64_t TI1 = B - 2 * T - 2 * K4 - TS1;
  const int64_t SI1 = su + sw - du - dv - 2 * B - S - (D - 4 * K4) - 2 * SS1 - 2 * C4;
  const int64_t eX = 1 + 2 * T + S + K4 + TS1 + SS1 + C4;
  const int64_t II1 = m - (su + sw - B) + eX;
  const int64_t v[kLocal] = {T,
                             S,
                             I,
                             K4,
                             T * (T - 1) / 2 - K4,
                             TS1,
                             T * S - TS1,
                             TI1,
                             SS1,
                             C4,
                             Su * (Su - 1) / 2 + Sv * (Sv - 1) / 2 - SS1,
                             Su * Sv - C4,
                             SI1,
                             T * I - TI1,
                             S * I - SI1,
                             II1,
                             I * (I - 1) / 2 - II1};
#pragma unroll
  for (int k = 0; k < kLocal; k++) g.local[(int64_t)k * m + id] = v[k];
}

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
    if (y <= x) continue;  // each undirected edge once, at its upper position
    const u64 du = (u64)g.deg2[x], dv = (u64)g.deg2[y];
    const u64 T = g.T[p];
    const u64 Su = du - 1 - T, Sv = dv - 1 - T, S = Su + Sv;
    const u64 I = n - du - dv + T;
    a[A_T] += T;
    a[A_S] += S;
    a[A_I] += I;
    a[A_TT] += choose2(T);
    a[A_SUSV] += (u128)Su * Sv;
    a[A_TS] += (u128)T * S;
    a[A_SS] += (u128)choose2(Su) + choose2(Sv);
    a[A_TI] += (u128)T * I;
    a[A_SI] += (u128)S * I;
    a[A_II] += I ? (u128)choose2(I) : (u128)0;
    a[A_II1] += m - du - dv + 1;
    if (PER_EDGE) {
      const u64 k4 = g.K4w[p];
      const u64 c4 = g.C4w[p] - g.Dw[p] + 2 * k4;  // non-negative; wraps cancel
      a[A_K4] += k4;
      a[A_C4] += c4;
      // canonical id of the edge in the caller's numbering: lo's upper
      // entries start at cu[lo], and its list ends with them (cu[lo + 1] -
      // cu[lo] of them), so hi is found among those alone
      const int32_t ua = g.order[x], ub = g.order[y];
      const int32_t lo = ua < ub ? ua : ub, hi = ua < ub ? ub : ua;
      const int64_t c0 = g.cu[lo];
      const int nup = (int)(g.cu[lo + 1] - c0);
      const int32_t r1 = g.rp[lo + 1];
      const int64_t id = c0 + lower_bound_dev<int32_t>(g.col + (r1 - nup), nup, hi);
      if (g.out) {
        g.out[id] = (int64_t)T;
        g.out[g.m + id] = (int64_t)k4;
        g.out[2 * g.m + id] = (int64_t)c4;
      }
      if (g.local) write_local(g, id, p, x, y, (int64_t)T, (int64_t)k4, (int64_t)c4);
    }
  }
  for (int i = 0; i < kAcc; i++) {
    const u128 s = block_sum_u128(a[i], red);
    if (threadIdx.x == 0) {
      g.partials[((size_t)blockIdx.x * kAcc + i) * 2] = (u64)s;
      g.partials[((size_t)blockIdx.x * kAcc + i) * 2 + 1] = (u64)(s >> 64);
    }
  }
}

// One wave per accumulator sums the block partials.
__global__ void k_step3_final(const u64 *partials, int nblocks, DevAcc *acc) {
  const int i = blockIdx.x;
  u128 s = 0;
  for (int b = threadIdx.x; b < nblocks; b += kWave)
    s += ((u128)partials[((size_t)b * kAcc + i) * 2 + 1] << 64) |
         partials[((size_t)b * kAcc + i) * 2];
  s = wave_sum_u128(s);
  if (threadIdx.x == 0) {
    acc->step3[i][0] = (u64)s;
    acc->step3[i][1] = (u64)(s >> 64);
  }
}

// One wave per vertex x: tv[x] = sum of |Tri_e| over x's edges (read at each
// edge's upper position), sv[x] = sum of the neighbours' degrees.
__global__ __launch_bounds__(256) void k_vertex_sums(const int32_t *rp2, const int32_t *col2,
                                                     const int32_t *lcnt, const int32_t *tpos,
                                                     const uint32_t *T, const int32_t *deg2,
                                                     int64_t n, u64 *tv, u64 *sv) {
  const int64_t waves = (int64_t)gridDim.x * (256 / kWave);
  for (int64_t x = (int64_t)blockIdx.x * (256 / kWave) + threadIdx.x / kWave; x < n;
       x += waves) {
    const int32_t r0 = rp2[x], r1 = rp2[x + 1], nl = lcnt[x];
    u64 t = 0, d = 0;
    for (int q = r0 + lane_id(); q < r1; q += kWave) {
      d += (u64)deg2[col2[q]];
      t += T[q - r0 < nl ? tpos[q] : q];
    }
    t = wave_sum_u64(t);
    d = wave_sum_u64(d);
    if (lane_id() == 0) {
      tv[x] = t;
      sv[x] = d;
    }
  }
}

// Upper-neighbour counts in the caller's ids (canonical edge numbering).
// up[u] = neighbours of u above u in the caller's numbering; up[n] = 0 (the
// exclusive scan then ends with the edge count).
__global__ void k_orig_upper(const int32_t *rp, const int32_t *col, int64_t n, int64_t *up) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u > n) return;
  if (u == n) {
    up[n] = 0;
    return;
  }
  const int a = rp[u], d = rp[u + 1] - a;
  up[u] = d - lower_bound_dev<int32_t>(col + a, d, (int32_t)u);
}

}  // namespace

int launch_step3(S3Args g, int grid, bool per_edge, hipStream_t s) {
  if (per_edge) k_step3<true><<<grid, 256, 0, s>>>(g);
  else k_step3<false><<<grid, 256, 0, s>>>(g);
  GC_TRY_HIP(hipGetLastError());
  k_step3_final<<<kAcc, kWave, 0, s>>>(g.partials, grid, g.acc);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

int launch_vertex_sums(const int32_t *rp2, const int32_t *col2, const int32_t *lcnt,
                       const int32_t *tpos, const uint32_t *T, const int32_t *deg2, int64_t n,
                       u64 *tv, u64 *sv, hipStream_t s) {
  if (n <= 0) return GC_OK;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 3) / 4, 16384);
  k_vertex_sums<<<grid, 256, 0, s>>>(rp2, col2, lcnt, tpos, T, deg2, n, tv, sv);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

int launch_orig_upper(const int32_t *rp, const int32_t *col, int64_t n, int64_t *up,
                      hipStream_t s) {
  k_orig_upper<<<grid1d(n + 1, 256), 256, 0, s>>>(rp, col, n, up);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

}  // namespace gc
