// Localized update of the 17 counts when one edge is inserted or deleted
// (the localized dynamic updates of Section 6.3, interactive graphlet
// mining: counts updated from the edge's neighbourhood instead of a full
// recount).  Only subsets that
// hold both endpoints change class.  For e = (u, v) present, the local
// vector of e (the N_{a,b}, N_{a,b,1}, N_{a,b,0} terms of Section 4.2) says
// how many subsets of each kind contain e; removing e turns each kind into
// one other graphlet (a 4-clique into a chordal cycle, a 4-cycle into a
// 4-path, ...), so the counts move by the terms of that vector alone.
//
// The local vector needs, around u and v only: |Tri_e|, the edges inside
// Tri_e (4-cliques), the edges between Star_u and Star_v (4-cycles), the
// triangle counts of the edges (u, w) and (v, w) for w in Tri_e, the degree
// sum over Tri_e, the triangle counts t_u, t_v and the neighbour-degree sums
// s_u, s_v.  All come from one pass over the lists of the neighbours of u
// and v, with membership in N(u) and N(v) read from two bitmaps.
#include <algorithm>
#include <cstring>
#include <vector>

#include "kernels.h"
#include "primitives.h"

namespace gc {

namespace {

// Accumulators of the pass (u64 each).
enum UpdAcc { U_T = 0, U_K4X2, U_C4, U_AU, U_AV, U_B, U_TU2, U_TV2, U_SU, U_SV, U_N };

__global__ void k_mark(const int32_t *rp, const int32_t *col, int32_t x, uint32_t *bits, int set) {
  const int a = rp[x], b = rp[x + 1];
  for (int p = a + blockIdx.x * blockDim.x + threadIdx.x; p < b; p += gridDim.x * blockDim.x) {
    const int32_t y = col[p];
    if (set) atomicOr(&bits[y >> 5], 1u << (y & 31));
    else bits[y >> 5] = 0;
  }
}

__device__ __forceinline__ bool bit(const uint32_t *bits, int32_t x) {
  return (bits[x >> 5] >> (x & 31)) & 1u;
}

// One wave per neighbour w of u or v (w from N(u), then N(v) minus N(u)).
__global__ __launch_bounds__(256) void k_two_hop(const int32_t *rp, const int32_t *col, int32_t u,
                                                 int32_t v, const uint32_t *bu,
                                                 const uint32_t *bv, u64 *acc) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int au = rp[u], du = rp[u + 1] - au, av = rp[v], dv = rp[v + 1] - av;
  u64 a[U_N];
  for (int i = 0; i < U_N; i++) a[i] = 0;
  for (int64_t k = wave; k < (int64_t)du + dv; k += nwaves) {
    const int32_t w = k < du ? col[au + k] : col[av + (k - du)];
    const bool wu = bit(bu, w), wv = bit(bv, w);
    if (k >= du && wu) continue;  // already taken from N(u)
    const int aw = rp[w], dw = rp[w + 1] - aw;
    u64 cu = 0, cv = 0, cuv = 0, cstar = 0;
    for (int p = aw + lane; p < aw + dw; p += kWave) {
      const int32_t x = col[p];
      const bool xu = bit(bu, x), xv = bit(bv, x);
      cu += xu;
      cv += xv;
      cuv += xu && xv;
      cstar += xv && !xu && x != u;
    }
    cu = wave_sum_u64(cu);
    cv = wave_sum_u64(cv);
    cuv = wave_sum_u64(cuv);
    cstar = wave_sum_u64(cstar);
    if (lane == 0) {
      const bool tri = wu && wv, star_u = wu && !wv && w != v;
      if (wu) {
        a[U_SU] += (u64)dw;
        a[U_TU2] += cu;  // |N(u) n N(w)|: twice t_u over all w in N(u)
      }
      if (wv) {
        a[U_SV] += (u64)dw;
        a[U_TV2] += cv;
      }
      if (tri) {
        a[U_T] += 1;
        a[U_B] += (u64)dw;
        a[U_AU] += cu;
        a[U_AV] += cv;
        a[U_K4X2] += cuv;  // edges inside Tri_e, each seen from both ends
      }
      if (star_u) a[U_C4] += cstar;  // edges from Star_u to Star_v
    }
  }
  if (lane == 0)
    for (int i = 0; i < U_N; i++)
      if (a[i]) atomicAdd(&acc[i], a[i]);
}

// Row offsets after inserting (sign 1) or deleting (sign -1) the edge
// (a, b), a < b: rows after a gain or lose one entry, rows after b two.
__global__ void k_shift_rows(const int32_t *rp, int64_t n, int32_t a, int32_t b, int sign,
                             int32_t *rp_out) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x > n) return;
  rp_out[x] = rp[x] + sign * ((x > a) + (x > b));
}

// The two new entries of an insertion.
__global__ void k_put2(int32_t *col, int64_t i1, int32_t v1, int64_t i2, int32_t v2) {
  if (threadIdx.x == 0) {
    col[i1] = v1;
    col[i2] = v2;
  }
}

__global__ void k_zero(u64 *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

struct Local {
  int64_t T, S, I, K4, TS1, SS1, TI1, C4, SI1, II1;
  int64_t Su, Sv;
};

// The local vector of the edge (u, v) in the graph that holds it, from the
// raw sums of the pass (same identities as the per-edge local vectors).
Local local_of(int64_t n, int64_t m, int64_t du, int64_t dv, int64_t T, int64_t K4, int64_t C4,
               int64_t D, int64_t B, int64_t tu, int64_t tv, int64_t su, int64_t sv) {
  Local L{};
  L.T = T;
  L.Su = du - 1 - T;
  L.Sv = dv - 1 - T;
  L.S = L.Su + L.Sv;
  L.I = n - du - dv + T;
  L.K4 = K4;
  L.C4 = C4;
  L.TS1 = D - 4 * K4;
  L.SS1 = tu + tv + 2 * K4 - D - 2 * T;
  L.TI1 = B - 2 * T - 2 * K4 - L.TS1;
  L.SI1 = su + sv - du - dv - 2 * B - L.S - (D - 4 * K4) - 2 * L.SS1 - 2 * C4;
  const int64_t eX = 1 + 2 * T + L.S + K4 + L.TS1 + L.SS1 + C4;
  L.II1 = m - (su + sv - B) + eX;
  return L;
}

int update_edge(const gc_csr *g, int32_t u, int32_t v, int insert, gc_u128 counts[17],
                hipStream_t s) {
  if (!g || !counts || !g->row_ptr || (g->nnz > 0 && !g->col) || g->n < 0 || g->nnz < 0 ||
      (g->nnz & 1) || u < 0 || v < 0 || u >= g->n || v >= g->n || u == v) {
    set_error("invalid arguments (null pointer, endpoint out of range, or u == v)");
    return GC_EINVAL;
  }
  const int64_t n = g->n, m = g->nnz / 2;
  const size_t words = (size_t)(n + 31) / 32;
  char *buf = nullptr;
  const size_t bytes = 2 * words * 4 + 256 + U_N * 8;
  GC_TRY_HIP(hipMallocAsync((void **)&buf, bytes, s));
  uint32_t *bu = reinterpret_cast<uint32_t *>(buf), *bv = bu + words;
  u64 *acc = reinterpret_cast<u64 *>(buf + ((2 * words * 4 + 255) & ~size_t(255)));
  int32_t h_rp[4];
  u64 h[U_N];
  hipError_t e = hipSuccess;
  // zero the bitmaps (a fill kernel, no memset) and the accumulators
  int rc = fill<uint32_t>(bu, 0u, 2 * (int64_t)words, s);
  if (rc == GC_OK) {
    k_zero<<<1, 64, 0, s>>>(acc, U_N);
    e = hipGetLastError();
  }
  if (rc == GC_OK && e == hipSuccess) {
    e = hipMemcpyAsync(&h_rp[0], g->row_ptr + u, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h_rp[2], g->row_ptr + v, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (rc == GC_OK && e == hipSuccess) {
    const int64_t du = h_rp[1] - h_rp[0], dv = h_rp[3] - h_rp[2];
    const unsigned gu = (unsigned)std::max<int64_t>(1, std::min<int64_t>((du + 255) / 256, 1024));
    const unsigned gv = (unsigned)std::max<int64_t>(1, std::min<int64_t>((dv + 255) / 256, 1024));
    k_mark<<<gu, 256, 0, s>>>(g->row_ptr, g->col, u, bu, 1);
    k_mark<<<gv, 256, 0, s>>>(g->row_ptr, g->col, v, bv, 1);
    const int64_t waves = du + dv;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((waves + 3) / 4, 65536));
    k_two_hop<<<grid, 256, 0, s>>>(g->row_ptr, g->col, u, v, bu, bv, acc);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h, acc, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  (void)hipFreeAsync(buf, s);
  if (rc != GC_OK) return rc;
  if (e != hipSuccess) {
    set_error("edge update: %s", hipGetErrorString(e));
    return GC_EHIP;
  }
  const int64_t du0 = h_rp[1] - h_rp[0], dv0 = h_rp[3] - h_rp[2];
  // is (u, v) an edge of g?  (a search of the sorted list N(u))
  int32_t found = 0;
  {
    std::vector<int32_t> lu((size_t)du0);
    if (du0 > 0 &&
        hipMemcpy(lu.data(), g->col + h_rp[0], sizeof(int32_t) * du0, hipMemcpyDeviceToHost) !=
            hipSuccess) {
      set_error("edge update: reading N(u) failed");
      return GC_EHIP;
    }
    found = std::binary_search(lu.begin(), lu.end(), v) ? 1 : 0;
  }
  if (insert && found) {
    set_error("edge (%d, %d) is already in the graph", u, v);
    return GC_EINVAL;
  }
  if (!insert && !found) {
    set_error("edge (%d, %d) is not in the graph", u, v);
    return GC_EINVAL;
  }
  const int64_t T = (int64_t)h[U_T], K4x2 = (int64_t)h[U_K4X2];
  if (K4x2 % 2 || h[U_TU2] % 2 || h[U_TV2] % 2) {
    set_error("edge update: odd pair count (internal error)");
    return GC_EINTERNAL;
  }
  const int64_t K4 = K4x2 / 2, C4 = (int64_t)h[U_C4], B = (int64_t)h[U_B];
  int64_t Au = (int64_t)h[U_AU], Av = (int64_t)h[U_AV];
  int64_t tu = (int64_t)h[U_TU2] / 2, tv = (int64_t)h[U_TV2] / 2;
  int64_t su = (int64_t)h[U_SU], sv = (int64_t)h[U_SV];
  int64_t du = du0, dv = dv0, mm = m;
  if (insert) {  // the same quantities in the graph with the edge added
    Au += T;  // v is now a common neighbour of u and every w in Tri_e
    Av += T;
    tu += T;
    tv += T;
    su += dv0 + 1;
    sv += du0 + 1;
    du += 1;
    dv += 1;
    mm += 1;
  }
  const int64_t D = Au + Av - 2 * T;
  const Local L = local_of(n, mm, du, dv, T, K4, C4, D, B, tu, tv, su, sv);
  // terms of the local vector: (count, class with e, class without e)
  const int64_t TT = T * (T - 1) / 2, TS = T * L.S, TI = T * L.I, SuSv = L.Su * L.Sv;
  const int64_t SS = L.Su * (L.Su - 1) / 2 + L.Sv * (L.Sv - 1) / 2, SI = L.S * L.I;
  const int64_t II = L.I * (L.I - 1) / 2;
  struct Move {
    int64_t c;
    int with, without;
  } mv[] = {
      {1, 0, 1},                  // the pair {u, v}
      {T, 2, 3},                  // triangle / 2-star
      {L.S, 3, 4},                // 2-star / 3-node-1-edge
      {L.I, 4, 5},                // 3-node-1-edge / independent
      {K4, 6, 7},                 // 4-clique / chordal cycle
      {TT - K4, 7, 9},            // chordal cycle (e the chord) / 4-cycle
      {L.TS1, 7, 8},              // chordal cycle (e on the cycle) / tailed triangle
      {TS - L.TS1, 8, 11},        // tailed triangle / 4-path
      {L.TI1, 8, 10},             // tailed triangle / 3-star
      {L.SS1, 8, 12},             // tailed triangle (e the tail) / 4-node-1-triangle
      {C4, 9, 11},                // 4-cycle / 4-path
      {SS - L.SS1, 10, 13},       // 3-star / 4-node-2-star
      {SuSv - C4, 11, 14},        // 4-path (e in the middle) / 4-node-2-edge
      {L.SI1, 11, 13},            // 4-path (e at an end) / 4-node-2-star
      {TI - L.TI1, 12, 13},       // 4-node-1-triangle / 4-node-2-star
      {SI - L.SI1, 13, 15},       // 4-node-2-star / 4-node-1-edge
      {L.II1, 14, 15},            // 4-node-2-edge / 4-node-1-edge
      {II - L.II1, 15, 16},       // 4-node-1-edge / 4-node-independent
  };
  i128 cnt[17];
  for (int i = 0; i < 17; i++) cnt[i] = (i128)(((u128)counts[i].hi << 64) | counts[i].lo);
  for (const Move &x : mv) {
    if (x.c < 0) {
      set_error("edge update: negative term (internal error)");
      return GC_EINTERNAL;
    }
    const i128 d = insert ? (i128)x.c : -(i128)x.c;
    cnt[x.with] += d;
    cnt[x.without] -= d;
  }
  for (int i = 0; i < 17; i++)
    if (cnt[i] < 0) {
      set_error("edge update: the given counts are not those of the graph (count %d < 0)", i);
      return GC_EINVAL;
    }
  for (int i = 0; i < 17; i++) {
    counts[i].lo = (uint64_t)(u128)cnt[i];
    counts[i].hi = (uint64_t)((u128)cnt[i] >> 64);
  }
  return GC_OK;
}

}  // namespace

// Writes the CSR of g with the edge (u, v) inserted (insert = 1) or deleted
// into rp_out (n + 1 entries) and col_out (nnz + 2 resp. nnz - 2 entries),
// which must not overlap g's arrays.  Rows stay sorted: the entry goes to
// its place in N(u) and N(v), found on host copies of the two rows.  The
// edge must be absent (insert) or present (delete), else GC_EINVAL.
int csr_apply_edge(const gc_csr *g, int32_t u, int32_t v, int insert, int32_t *rp_out,
                   int32_t *col_out, hipStream_t s) {
  if (!g || !rp_out || !col_out || u < 0 || v < 0 || u >= g->n || v >= g->n || u == v) {
    set_error("invalid arguments");
    return GC_EINVAL;
  }
  const int32_t a = std::min(u, v), b = std::max(u, v);
  int32_t ra[2], rb[2];
  GC_TRY_HIP(hipMemcpyAsync(ra, g->row_ptr + a, 8, hipMemcpyDeviceToHost, s));
  GC_TRY_HIP(hipMemcpyAsync(rb, g->row_ptr + b, 8, hipMemcpyDeviceToHost, s));
  GC_TRY_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> la((size_t)(ra[1] - ra[0])), lb((size_t)(rb[1] - rb[0]));
  if (!la.empty())
    GC_TRY_HIP(hipMemcpyAsync(la.data(), g->col + ra[0], 4 * la.size(), hipMemcpyDeviceToHost, s));
  if (!lb.empty())
    GC_TRY_HIP(hipMemcpyAsync(lb.data(), g->col + rb[0], 4 * lb.size(), hipMemcpyDeviceToHost, s));
  GC_TRY_HIP(hipStreamSynchronize(s));
  // pa: position of b in row a (or where it would go), pb: of a in row b
  const int64_t ia = std::lower_bound(la.begin(), la.end(), b) - la.begin();
  const int64_t ib = std::lower_bound(lb.begin(), lb.end(), a) - lb.begin();
  const bool has = ia < (int64_t)la.size() && la[ia] == b;
  const bool has_b = ib < (int64_t)lb.size() && lb[ib] == a;
  if (has != has_b) {
    set_error("CSR is not symmetric at (%d, %d)", a, b);
    return GC_EASYMMETRIC;
  }
  if (insert == has) {
    set_error(insert ? "edge (%d, %d) is already in the graph" : "edge (%d, %d) is not in the graph",
              u, v);
    return GC_EINVAL;
  }
  const int64_t pa = ra[0] + ia, pb = rb[0] + ib, nnz = g->nnz;  // pa < pb
  auto copy = [&](int64_t dst, int64_t src, int64_t len) -> hipError_t {
    if (len <= 0) return hipSuccess;
    return hipMemcpyAsync(col_out + dst, g->col + src, 4 * (size_t)len, hipMemcpyDeviceToDevice,
                          s);
  };
  if (insert) {
    GC_TRY_HIP(copy(0, 0, pa));
    GC_TRY_HIP(copy(pa + 1, pa, pb - pa));
    GC_TRY_HIP(copy(pb + 2, pb, nnz - pb));
    k_put2<<<1, 64, 0, s>>>(col_out, pa, b, pb + 1, a);
  } else {
    GC_TRY_HIP(copy(0, 0, pa));
    GC_TRY_HIP(copy(pa, pa + 1, pb - pa - 1));
    GC_TRY_HIP(copy(pb - 1, pb + 1, nnz - pb - 1));
  }
  GC_TRY_HIP(hipGetLastError());
  k_shift_rows<<<grid1d(g->n + 1, 256), 256, 0, s>>>(g->row_ptr, g->n, a, b, insert ? 1 : -1,
                                                      rp_out);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

}  // namespace gc

extern "C" int graphlet_update_edge(const gc_csr *g, int32_t u, int32_t v, int insert,
                                    gc_u128 counts[17], void *stream) {
  gc::clear_error();
  try {
    return gc::update_edge(g, u, v, insert, counts, (hipStream_t)stream);
  } catch (...) {
    gc::set_error("unexpected exception");
    return GC_EINTERNAL;
  }
}
