// Steps 1 and 2a: |Tri_e| of every edge and the 4-cliques.
//
// One workgroup per vertex u with k = |U(u)| >= 2 upper neighbours (in the
// degree order).  The subgraph induced by U(u) is built in LDS as a bitmap:
// bit (i, j) means U_j is in U(U_i), i.e. {u, U_i, U_j} is a triangle whose
// lowest vertex is u.  Each triangle is therefore found exactly once, which
// replaces the marking array X of the paper's triad census (Section 3) by a
// per-vertex bitmap:
//   * |Tri| of edge (U_i, U_j) gains one (global atomic at its position);
//   * |Tri| of edge (u, U_i) is the number of local neighbours of U_i;
//   * the 4-cliques with lowest vertex u are the triangles of the local
//     graph: AND + popcount of two rows (CliqueCount of Section 4.4, which
//     marks Tri_e and scans neighbour lists, reads the same adjacencies).
//
// Global mode keeps only the upper half of the local adjacency (bit j > i in
// row i), packed triangularly; a column counter per local vertex gives the
// lower half's contribution to |Tri|.  U(u) is indexed by an LDS hash, with
// a bit filter in front of it: most candidates are not in U(u), and one LDS
// read turns them away before the probe.  Per-edge mode keeps symmetric
// rows, so that every local edge can read its common-neighbour count
// (4-cliques through that edge); rows of up to 896 local vertices stay in
// LDS, larger ones (up to 1088) use a per-workgroup slot in global memory.
#include <algorithm>

#include "kernels.h"

namespace gc {

namespace {

// Exclusive scan of A[0..k) in place; total in A[k].  BLOCK threads.
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
    const int32_t t = tid >= off ? sums[tid - off] : 0;
    __syncthreads();
    sums[tid] += t;
    __syncthreads();
  }
  int32_t run = sums[tid] - s;
  for (int i = a; i < b; i++) {
    const int32_t v = A[i];
    A[i] = run;
    run += v;
  }
  if (tid == BLOCK - 1) A[k] = sums[BLOCK - 1];
  __syncthreads();
}

__device__ __forceinline__ uint32_t hslot(int32_t x, int hbits) {
  return ((uint32_t)x * 2654435761u) >> (32 - hbits);
}

// Local index of vertex x in U(u), or -1.  H holds index + 1 (0 = empty).
__device__ __forceinline__ int hfind(const int32_t *H, const int32_t *U, uint32_t mask, int hbits,
                                     int32_t x) {
  uint32_t h = hslot(x, hbits);
  while (true) {
    const int v = H[h];
    if (v == 0) return -1;
    if (U[v - 1] == x) return v - 1;
    h = (h + 1) & mask;
  }
}

// Candidate entries (the upper lists of the kept rows, concatenated; row o
// starts at P[o] and reads list position V[o]) are taken in slabs of
// kWave * RUN per wave: in step r, lane L takes candidate s0 + r * kWave + L,
// so the lanes of each load and of each per-entry atomic touch consecutive
// entries.  The rows of the slab's first and last candidates are found by
// galloping forward from a cursor (a wave's slabs advance through the rows),
// each lane finds the row of its first candidate by binary search between
// them, then follows its later candidates forward (rows are long on
// average: most steps stay in the row).  pos[r] = -1 past the end.

// Largest o in [from, n) with P[o] <= x, given P[from] <= x (P increasing).
__device__ __forceinline__ int gallop_row(const int32_t *P, int n, int from, int x) {
  int lo = from, hi = from + 1, step = 1;
  while (hi < n && P[hi] <= x) {
    lo = hi;
    step <<= 1;
    hi = lo + step;
  }
  hi = min(hi, n);  // P[lo] <= x, and hi == n or P[hi] > x
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (P[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int RUN>
__device__ __forceinline__ void slab_positions(const int32_t *P, const int32_t *V,
                                               const int32_t *rid, int nr, int total, int s0,
                                               int &cursor, int (&pos)[RUN], int (&row)[RUN]) {
  const int lane = lane_id();
  const int ia = gallop_row(P, nr, cursor, s0);
  const int ib = gallop_row(P, nr, ia, min(s0 + kWave * RUN, total) - 1) + 1;
  cursor = ia;
  int lo = ia;  // P[lo] <= t < P[lo + 1] for the lane's current candidate t
  if (s0 + lane < total) {
    int hi = ib;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (P[mid] <= s0 + lane) lo = mid;
      else hi = mid;
    }
  }
  // the current row's start, end, list position and id, reloaded only when a
  // candidate crosses into a later row
  int p_lo = P[lo], p_next = lo + 1 < ib ? P[lo + 1] : total, v_lo = V[lo], r_lo = rid[lo];
#pragma unroll
  for (int r = 0; r < RUN; r++) {
    const int t = s0 + r * kWave + lane;
    pos[r] = -1;
    if (t < total) {
      if (t >= p_next) {
        do {
          lo++;
        } while (lo + 1 < ib && P[lo + 1] <= t);
        p_lo = P[lo];
        p_next = lo + 1 < ib ? P[lo + 1] : total;
        v_lo = V[lo];
        r_lo = rid[lo];
      }
      pos[r] = v_lo + (t - p_lo);
      row[r] = r_lo;
    }
  }
}

// Bit filter of the hashed set: one bit per 2^FLOG slot of the same
// multiplicative hash; a candidate whose bit is clear is not in the set.
template <int FLOG>
__device__ __forceinline__ uint32_t fslot(int32_t x) {
  return ((uint32_t)x * 2654435761u) >> (32 - FLOG);
}

// Row i of the triangular layout holds words [i >> 6, W) of the upper half.
__device__ __forceinline__ int tri_off(int i, int W) {
  const int q = i >> 6;
  return i * W - (32 * q * (q - 1) + q * (i - 64 * q));
}

// ------------------------------------------------------------ global mode

// The three smaller shapes fit 8 waves per SIMD by LDS; their registers are
// held to 64 per lane so that they do (the issue of VALU work bounds them).
template <int BLOCK, int KCAP, int HS>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(BLOCK <= 512 ? 8 : 1))) void k_tk_up(TkArgs g) {
  constexpr int WC = (KCAP + 63) / 64;
  constexpr int RWORDS = 32 * WC * (WC + 1);  // tri_off(64 WC, WC)
  // candidates per lane per slab, all loaded before any is probed; the
  // 1024-thread shape is held to 4 waves per SIMD by LDS, not registers, so
  // it keeps four times as many loads in flight (24 still fits in 128 VGPRs)
  constexpr int RUN = BLOCK == 1024 ? 24 : 6;
  // filter of U(u): 8 bits per hash slot (4 for the two largest tables),
  // so at most 1 in 32 candidates outside U(u) reaches the hash table
  constexpr int FLOG = (31 - __builtin_clz(HS)) + (HS <= 1024 ? 3 : 2);
  constexpr int FW = (1 << FLOG) / 32;
  __shared__ int32_t U[KCAP], V[KCAP], P[KCAP + 1], rid[KCAP], H[HS], sums[BLOCK];
  __shared__ uint32_t colcnt[KCAP], F[FW];
  __shared__ u64 R[RWORDS];
  __shared__ u64 red[32];
  __shared__ int next, nrows;
  const int tid = threadIdx.x;
  u128 k4acc = 0;
  for (int it = blockIdx.x; it < g.nlist; it += gridDim.x) {
    const int u = g.list[it];
    const int k = g.ucnt[u];
    const int base = g.ustart[u];
    const int W = (k + 63) >> 6;
    int hs = 64;  // load factor <= 1/4: most misses stop at the first slot
    while (hs < 4 * k && hs < HS) hs <<= 1;
    const int hbits = __ffs(hs) - 1;
    const uint32_t mask = (uint32_t)hs - 1;
    const int rwords = tri_off(k, W);
    for (int i = tid; i < k; i += BLOCK) {
      U[i] = g.col2[base + i];
      colcnt[i] = 0;
    }
    for (int h = tid; h < hs; h += BLOCK) H[h] = 0;
    for (int w = tid; w < FW; w += BLOCK) F[w] = 0;
    for (int w = tid; w < rwords; w += BLOCK) R[w] = 0;
    if (tid == 0) {
      next = 0;
      nrows = 0;
    }
    __syncthreads();
    // hash U(u); keep only the rows whose vertex has upper neighbours
    for (int i0 = 0; i0 < k; i0 += BLOCK) {
      const int i = i0 + tid;
      int len = 0, v = 0;
      if (i < k) {
        v = U[i];
        len = g.ucnt[v];
        uint32_t h = hslot(v, hbits);
        while (atomicCAS(&H[h], 0, i + 1) != 0) h = (h + 1) & mask;
        const uint32_t f = fslot<FLOG>(v);
        atomicOr(&F[f >> 5], 1u << (f & 31));
      }
      const bool keep = len > 0;
      const u64 m = __ballot(keep);
      int b = 0;
      if (lane_id() == 0 && m) b = atomicAdd(&nrows, __popcll(m));
      b = __shfl(b, 0, kWave);
      if (keep) {
        const int o = b + __popcll(m & lanemask_lt());
        rid[o] = i;
        V[o] = g.ustart[v];
        P[o] = len;
      }
    }
    __syncthreads();
    const int nr = nrows;
    block_scan_excl<BLOCK>(P, nr, sums);
    const int total = P[nr];
    // Build: every entry x of U(U_i) that lies in U(u) is a triangle.  Each
    // thread takes RUN consecutive entries: positions first, then all loads,
    // then the filter, so RUN reads are in flight per thread.  The few
    // candidates that pass the filter are packed, as candidate indices, into
    // the wave's queue (the scan's scratch, free here) and probed 64 at a time,
    // so the probe and the atomics run on full waves instead of once per
    // candidate slot with most lanes idle; a queued index finds its row by
    // binary search and its entry again (just read: a cache hit).
    int32_t *qt = sums + (tid / kWave) * kWave;
    int qn = 0;  // entries in the wave's queue (the same on every lane)
    auto probe = [&](int cnt) {  // the queue's first cnt entries, one per lane
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int l = lane_id();
      if (l < cnt) {
        const int t = qt[l];
        const int o = upper_index_dev<int32_t>(P, nr, t);
        const int pos = V[o] + (t - P[o]);
        const int j = hfind(H, U, mask, hbits, g.col2[pos]);
        if (j >= 0) {
          const int ir = rid[o];
          atomicOr(&R[tri_off(ir, W) + (j >> 6) - (ir >> 6)], 1ull << (j & 63));
          atomicAdd(&colcnt[j], 1u);
          atomicAdd(&g.T[pos], 1u);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    int cursor = 0;  // row at or before the wave's next slab
    for (int s0 = (tid / kWave) * kWave * RUN; s0 < total; s0 += BLOCK * RUN) {
      int pos[RUN], row[RUN], xv[RUN];
      slab_positions<RUN>(P, V, rid, nr, total, s0, cursor, pos, row);
#pragma unroll
      for (int r = 0; r < RUN; r++) xv[r] = g.col2[pos[r] >= 0 ? pos[r] : 0];
#pragma unroll
      for (int r = 0; r < RUN; r++) {
        const uint32_t f = fslot<FLOG>(xv[r]);
        const bool ok = pos[r] >= 0 && ((F[f >> 5] >> (f & 31)) & 1u);
        if (BLOCK == 1024) {
          // the largest U(u) are dense: most slots pass, so probe in place
          if (ok) {
            const int j = hfind(H, U, mask, hbits, xv[r]);
            if (j >= 0) {
              const int ir = row[r];
              atomicOr(&R[tri_off(ir, W) + (j >> 6) - (ir >> 6)], 1ull << (j & 63));
              atomicAdd(&colcnt[j], 1u);
              atomicAdd(&g.T[pos[r]], 1u);
            }
          }
          continue;
        }
        const u64 b = __ballot(ok);
        const int cnt = __popcll(b);
        if (qn + cnt > kWave) {  // the same on every lane
          probe(qn);
          qn = 0;
        }
        if (ok) qt[qn + __popcll(b & lanemask_lt())] = s0 + r * kWave + lane_id();
        qn += cnt;
      }
    }
    if (qn > 0) probe(qn);
    __syncthreads();
    // |Tri| of edges (u, U_i); 4-cliques u < U_i < U_j < U_l, each once.
    // Row i stays in registers (word z of the row, zero below word qi), so
    // each AND reads only row j from LDS.
    u64 acc = 0;
    for (int i = atomicAdd(&next, 1); i < k; i = atomicAdd(&next, 1)) {
      const u64 *Ri = R + tri_off(i, W);
      const int qi = i >> 6;
      u64 ri[WC];
#pragma unroll
      for (int z = 0; z < WC; z++) ri[z] = (z >= qi && z < W) ? Ri[z - qi] : 0ull;
      uint32_t c = colcnt[i];
#pragma unroll
      for (int z = 0; z < WC; z++) c += (uint32_t)__popcll(ri[z]);
      if (c) atomicAdd(&g.T[base + i], c);
      if (!g.k4) continue;  // per-edge mode: its own pass counts the 4-cliques
#pragma unroll
      for (int w = 0; w < WC; w++) {
        u64 bits = ri[w];
        while (bits) {
          const int j = (w << 6) + __ffsll((long long)bits) - 1;
          bits &= bits - 1;
          const u64 *Rj = R + tri_off(j, W) - (j >> 6);  // Rj[z] = word z of row j
#pragma unroll
          for (int z = w; z < WC; z++)
            if (z < W) acc += (u64)__popcll(ri[z] & Rj[z]);
        }
      }
    }
    k4acc += (u128)acc;
    __syncthreads();
  }
  const u128 s = block_sum_u128(k4acc, red);
  if (threadIdx.x == 0 && s && g.k4) atomic_add_u128(g.k4, s);
}

// ------------------------------------------------------------ per-edge mode

// Per-edge pass (|Tri| is final): the 4-cliques through every local edge and
// the D_e terms, with U(u) hashed and candidates read RUN at a time as in
// k_tk_up.  Pass 1 builds the symmetric local adjacency (rows of W words,
// in LDS, or in a per-workgroup global slot when GR); pass 2 revisits the
// candidates and, for every local edge (U_i, U_j):
//   c = |N(U_i) n N(U_j) n U(u)| (AND + popcount of the two rows) goes to
//     the edge itself, and (halved at the end: each clique {u, U_i, U_j, U_l}
//     is seen from two local edges at U_i) to edges (u, U_i) and (u, U_j);
//   |Tri(u,U_i)| + |Tri(u,U_j)| - 2 goes to D of the edge, and
//   |Tri(u,U_j)| + |Tri(U_i,U_j)| - 2 to D of (u, U_i) (and symmetrically).
// Vertices of the list with k <= KMIN (or k > KCAP) are left to another
// launch over the same list.  With HBITS > 0, pass 1 marks its hits in an LDS
// bitmap over the candidate indices (when there are at most HBITS
// candidates), and pass 2 walks the marked candidates only: about one
// candidate in ten is a triangle.
// The 64-thread shape is held to 64 VGPRs, and its bitmap to 480 bytes, so
// that it runs 8 waves per SIMD.
template <int BLOCK, int KCAP, int HS, bool GR, int KMIN = 0, int HBITS = 0>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(BLOCK == 64 ? 8 : 1))) void k_tk_pe(TkArgs g) {
  constexpr int WC = (KCAP + 63) / 64;
  constexpr int RUN = 6;
  constexpr int FLOG = (31 - __builtin_clz(HS)) + (HS <= 1024 ? 3 : 2);  // as in k_tk_up
  constexpr int FW = (1 << FLOG) / 32;
  constexpr int HBW = HBITS > 0 ? HBITS / 32 : 1;
  __shared__ int32_t U[KCAP], V[KCAP], P[KCAP + 1], rid[KCAP], H[HS], sums[BLOCK];
  __shared__ uint32_t Tu[KCAP], A1[KCAP], F[FW], HB[HBW];
  __shared__ u64 A2[KCAP], B2[KCAP];  // B2: degree sums for edges (u, U_i)
  __shared__ u64 Rl[GR ? 1 : KCAP * WC];
  __shared__ int nrows;
  const int tid = threadIdx.x;
  u64 *R = Rl;
  if (GR) {
    const size_t km = (size_t)g.kmax;
    R = g.gR + (size_t)blockIdx.x * km * ((km + 63) / 64);
  }
  for (int it = blockIdx.x; it < g.nlist; it += gridDim.x) {
    const int u = g.list[it];
    const int k = g.ucnt[u];
    if (k <= KMIN || k > KCAP) continue;  // the same on every thread
    const int base = g.ustart[u];
    const int W = (k + 63) >> 6;
    int hs = 64;
    while (hs < 4 * k && hs < HS) hs <<= 1;
    const int hbits = __ffs(hs) - 1;
    const uint32_t mask = (uint32_t)hs - 1;
    for (int i = tid; i < k; i += BLOCK) {
      U[i] = g.col2[base + i];
      Tu[i] = g.T[base + i];
      A1[i] = 0;
      A2[i] = 0;
      B2[i] = 0;
    }
    for (int h = tid; h < hs; h += BLOCK) H[h] = 0;
    for (int w = tid; w < FW; w += BLOCK) F[w] = 0;
    for (int w = tid; w < k * W; w += BLOCK) R[w] = 0;
    if (tid == 0) nrows = 0;
    __syncthreads();
    for (int i0 = 0; i0 < k; i0 += BLOCK) {
      const int i = i0 + tid;
      int len = 0, v = 0;
      if (i < k) {
        v = U[i];
        len = g.ucnt[v];
        uint32_t h = hslot(v, hbits);
        while (atomicCAS(&H[h], 0, i + 1) != 0) h = (h + 1) & mask;
        const uint32_t f = fslot<FLOG>(v);
        atomicOr(&F[f >> 5], 1u << (f & 31));
      }
      const bool keep = len > 0;
      const u64 m = __ballot(keep);
      int b = 0;
      if (lane_id() == 0 && m) b = atomicAdd(&nrows, __popcll(m));
      b = __shfl(b, 0, kWave);
      if (keep) {
        const int o = b + __popcll(m & lanemask_lt());
        rid[o] = i;
        V[o] = g.ustart[v];
        P[o] = len;
      }
    }
    __syncthreads();
    const int nr = nrows;
    block_scan_excl<BLOCK>(P, nr, sums);
    const int total = P[nr];
    const bool hits = HBITS > 0 && total <= HBITS;  // the same on every thread
    const int nhw = (total + 31) >> 5;
    if (hits) {
      for (int w = tid; w < nhw; w += BLOCK) HB[w] = 0;
      __syncthreads();
    }
    // Candidates past the bit filter are packed per wave (as candidate
    // indices, in the scan's scratch) and probed 64 at a time, as in k_tk_up.
    int32_t *qt = sums + (tid / kWave) * kWave;
    for (int pass = 0; pass < 2; pass++) {
      int qn = 0;  // entries in the wave's queue (the same on every lane)
      auto probe = [&](int cnt) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int l = lane_id();
        if (l < cnt) {
          const int t = qt[l];
          const int o = upper_index_dev<int32_t>(P, nr, t);
          const int p = V[o] + (t - P[o]);
          const int j = hfind(H, U, mask, hbits, g.col2[p]);
          const int ir = rid[o];  // j > ir: U(U_i) lies above U_i
          if (j >= 0 && pass == 0) {
            atomicOr(&R[(size_t)ir * W + (j >> 6)], 1ull << (j & 63));
            atomicOr(&R[(size_t)j * W + (ir >> 6)], 1ull << (ir & 63));
            if (hits) atomicOr(&HB[t >> 5], 1u << (t & 31));
          } else if (j >= 0) {
            const u64 *Ri = R + (size_t)ir * W, *Rj = R + (size_t)j * W;
            uint32_t c = 0;
            for (int z = 0; z < W; z++) c += (uint32_t)__popcll(Ri[z] & Rj[z]);
            const u64 tij = g.T[p];
            if (c) {
              atomicAdd(&g.K4w[p], (u64)c);
              atomicAdd(&A1[ir], c);
              atomicAdd(&A1[j], c);
            }
            atomicAdd(&g.Dw[p], (u64)Tu[ir] + Tu[j] - 2);
            atomicAdd(&A2[ir], (u64)Tu[j] + tij - 2);
            atomicAdd(&A2[j], (u64)Tu[ir] + tij - 2);
            if (g.Bw) {  // local vectors: degrees of the third vertex of the triangle
              atomicAdd(&g.Bw[p], (u64)g.deg2[u]);
              atomicAdd(&B2[ir], (u64)g.deg2[U[j]]);
              atomicAdd(&B2[j], (u64)g.deg2[U[ir]]);
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      };
      if (pass == 1 && hits) {
        // the marked candidates: each lane takes one word of the bitmap and
        // hands out one of its bits per round (hits are sparse here, so the
        // queue's entries, spread over 64 words, rarely share lines anyway)
        for (int w0 = (tid / kWave) * kWave; w0 < nhw; w0 += BLOCK) {
          const int w = w0 + lane_id();
          uint32_t bits = w < nhw ? HB[w] : 0u;
          while (__ballot(bits != 0)) {  // the same on every lane
            const bool ok = bits != 0;
            const int t = (w << 5) + (ok ? __ffs(bits) - 1 : 0);
            bits &= bits - 1;
            const u64 b = __ballot(ok);
            const int cnt = __popcll(b);
            if (qn + cnt > kWave) {
              probe(qn);
              qn = 0;
            }
            if (ok) qt[qn + __popcll(b & lanemask_lt())] = t;
            qn += cnt;
          }
        }
      } else {
        int cursor = 0;  // row at or before the wave's next slab
        for (int s0 = (tid / kWave) * kWave * RUN; s0 < total; s0 += BLOCK * RUN) {
          int pos[RUN], row[RUN], xv[RUN];
          slab_positions<RUN>(P, V, rid, nr, total, s0, cursor, pos, row);
#pragma unroll
          for (int r = 0; r < RUN; r++) xv[r] = g.col2[pos[r] >= 0 ? pos[r] : 0];
#pragma unroll
          for (int r = 0; r < RUN; r++) {
            const uint32_t f = fslot<FLOG>(xv[r]);
            const bool ok = pos[r] >= 0 && ((F[f >> 5] >> (f & 31)) & 1u);
            const u64 b = __ballot(ok);
            const int cnt = __popcll(b);
            if (qn + cnt > kWave) {  // the same on every lane
              probe(qn);
              qn = 0;
            }
            if (ok) qt[qn + __popcll(b & lanemask_lt())] = s0 + r * kWave + lane_id();
            qn += cnt;
          }
        }
      }
      if (qn > 0) probe(qn);
      __syncthreads();
    }
    for (int i = tid; i < k; i += BLOCK) {
      if (A1[i]) atomicAdd(&g.K4w[base + i], (u64)(A1[i] / 2));
      if (A2[i]) atomicAdd(&g.Dw[base + i], A2[i]);
      if (B2[i]) atomicAdd(&g.Bw[base + i], B2[i]);  // zero unless g.Bw
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ symmetric rows

template <int BLOCK, bool PER_EDGE>
__device__ void tk_vertex(const TkArgs &g, int u, int32_t *U, int32_t *V, int32_t *P, u64 *R,
                          int words, int32_t *sums, u64 *A1, u64 *A2, uint32_t *Tu,
                          u128 &k4acc) {
  const int tid = threadIdx.x;
  const int k = g.ucnt[u];
  const int base = g.ustart[u];
  for (int i = tid; i < k; i += BLOCK) U[i] = g.col2[base + i];
  for (int w = tid; w < k * words; w += BLOCK) R[w] = 0;
  __syncthreads();
  for (int i = tid; i < k; i += BLOCK) {
    const int v = U[i];
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
  for (int t = tid; t < total; t += BLOCK) {
    const int i = upper_index_dev<int32_t>(P, k, t);
    const int pos = V[i] + (t - P[i]);
    const int x = g.col2[pos];
    const int j = i + 1 + lower_bound_dev<int32_t>(U + i + 1, k - i - 1, x);
    if (j < k && U[j] == x) {
      atomicOr(&R[(size_t)i * words + (j >> 6)], 1ull << (j & 63));
      atomicOr(&R[(size_t)j * words + (i >> 6)], 1ull << (i & 63));
      if (!PER_EDGE) atomicAdd(&g.T[pos], 1u);
    }
  }
  __syncthreads();
  if (!PER_EDGE) {
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
          const int j = (w << 6) + __ffsll((long long)bits) - 1;
          bits &= bits - 1;
          const u64 *Rj = R + (size_t)j * words;
          for (int z = 0; z < words; z++) acc += (u64)__popcll(Ri[z] & Rj[z]);
        }
      }
    }
    k4acc += (u128)acc;
  } else {
    // Per local edge (i, j): 4-cliques {u, U_i, U_j, x}, x in U(u), and the
    // D_e terms of the 4-cycle identity (|Tri| is final here).
    for (int t = tid; t < total; t += BLOCK) {
      const int i = upper_index_dev<int32_t>(P, k, t);
      const int pos = V[i] + (t - P[i]);
      const int x = g.col2[pos];
      const int j = i + 1 + lower_bound_dev<int32_t>(U + i + 1, k - i - 1, x);
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
        if (g.Bw) {  // local vectors: degrees of the third vertex of the triangle
          atomicAdd(&g.Bw[pos], (u64)g.deg2[u]);
          atomicAdd(&g.Bw[base + i], (u64)g.deg2[U[j]]);
          atomicAdd(&g.Bw[base + j], (u64)g.deg2[U[i]]);
        }
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

// Fallback for large k: rows and arrays in global memory, one slot per block.
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
    tk_vertex<BLOCK, PER_EDGE>(g, u, U, V, P, R, words, sums, A1, A2, Tu, k4acc);
  }
  if (!PER_EDGE) {
    const u128 s = block_sum_u128(k4acc, red);
    if (threadIdx.x == 0 && s) atomic_add_u128(g.k4x3, s);
  }
}

}  // namespace

int launch_cliques(TkArgs g, int bin, bool per_edge, hipStream_t s) {
  if (g.nlist <= 0) return GC_OK;
  auto grid = [&](int cap) { return (unsigned)std::min(g.nlist, cap); };
  if (!per_edge) {
    switch (bin) {
      case 0: k_tk_up<64, kTkLim0, 256><<<grid(65536), 64, 0, s>>>(g); break;
      case 1: k_tk_up<256, kTkLim1, 1024><<<grid(16384), 256, 0, s>>>(g); break;
      case 2: k_tk_up<512, kTkLim2, 2048><<<grid(8192), 512, 0, s>>>(g); break;
      case 3: k_tk_up<1024, kTkLim3, 4096><<<grid(4096), 1024, 0, s>>>(g); break;
      default: k_tk_global<256, false><<<grid(kTkGlobalSlots), 256, 0, s>>>(g); break;
    }
  } else {
    switch (bin) {
      // the smallest class keeps a hit bitmap of 3840 candidates (three
      // quarters of its candidates on the Chung-Lu graph, one in ten a
      // triangle); for the larger classes the second pass is dominated by
      // the probes and their atomics, and a bitmap measured no gain
      case 0: k_tk_pe<64, kTkLim0, 256, false, 0, 3840><<<grid(65536), 64, 0, s>>>(g); break;
      case 1: k_tk_pe<256, kTkLim1, 1024, false><<<grid(16384), 256, 0, s>>>(g); break;
      case 2: k_tk_pe<512, kTkLim2, 2048, false><<<grid(8192), 512, 0, s>>>(g); break;
      // symmetric rows of up to 896 vertices (98 KB) fit beside the lists;
      // those of up to 1088 (148 KB) take a global slot
      case 3:
        k_tk_pe<1024, kTkPeLds, 4096, false><<<grid(4096), 1024, 0, s>>>(g);
        GC_TRY_HIP(hipGetLastError());
        k_tk_pe<1024, kTkLim3, 4096, true, kTkPeLds><<<grid(kTkGlobalSlots), 1024, 0, s>>>(g);
        break;
      default: k_tk_global<256, true><<<grid(kTkGlobalSlots), 256, 0, s>>>(g); break;
    }
  }
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

}  // namespace gc
