// Step 2b: 4-cycles through every edge.
//
// The paper's CycleCount (Section 4.4) marks Star_v and scans N(w) for every
// w in Star_u: O(|E| Delta S_max) reads, about 1.5e14 on R-MAT scale 22.
// Here the same per-edge numbers come from
//     C4_e = C4ni_e - D_e + 2 K4_e,
// where C4ni_e counts the 4-cycles through e whether or not they have chords,
// D_e = sum_{w in Tri_e} (|Tri_(u,w)| + |Tri_(v,w)| - 2) counts the chorded
// ones through each chord-carrying triangle vertex, and the 4-cycles with both
// chords (4-cliques) are subtracted twice by D_e, hence + 2 K4_e.  C4ni comes
// from wedge aggregation: a 4-cycle has one highest vertex x (degree order)
// and is the union of two paths x - v - y with v, y below x, so with c(x, y)
// the number of such paths, the cycles through x as highest vertex are
// C(c(x, y), 2) per y.  In the per-edge pass, each wedge x - v - y lies on
// c(x, y) - 1 cycles, credited to its two edges.
//
// Light x (few wedges): one wavefront, c(x, .) in an LDS hash.
// Heavy x: work items (x, y range); the range is walked in chunks of LDS
// counters, and every lower neighbour v of x keeps a cursor into its sorted
// list, so each wedge entry is read once per pass.
#include <algorithm>

#include "kernels.h"

namespace gc {

namespace {

__device__ __forceinline__ u64 choose2(u64 c) { return c * (c - 1) / 2; }


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
          const int t = __shfl_up(incl, off, kWave);
          if (lane >= off) incl += t;
        }
        sIncl[lane] = incl;
        sLen[lane] = len;
        __syncthreads();
        const int total = sIncl[kWave - 1];
        for (int t = lane; t < total; t += kWave) {
          int lo = 0, hi = kWave - 1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sIncl[mid] > t) hi = mid;
            else lo = mid + 1;
          }
          const int p = sStart[lo] + (t - (sIncl[lo] - sLen[lo]));
          const int y = g.col2[p];
          uint32_t h = ((uint32_t)y * 2654435761u) >> (32 - hbits);
          if (pass == 0) {
            while (true) {
              const int old = atomicCAS(&hkey[h], -1, y);
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
              atomicAdd(&g.C4w[p], c - 1);       // edge (v, y) at v's entry for y
              atomicAdd(&g.C4w[sQ[lo]], c - 1);  // edge (x, v) at x's entry for v
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
  const u128 s = block_sum_u128(acc, red);
  if (threadIdx.x == 0 && s) atomic_add_u128(g.c4ni, s);
}

// Exclusive scan of A[0..k) in place, total in A[k]; BLOCK threads, three
// barriers (wave scans by shuffles, one wave scans the wave totals).
template <int BLOCK>
__device__ void scan_excl(int32_t *A, int k, int32_t *wsum) {
  constexpr int NW = BLOCK / kWave;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int per = (k + BLOCK - 1) / BLOCK;
  const int a = min(k, tid * per), b = min(k, a + per);
  int32_t s = 0;
  for (int i = a; i < b; i++) s += A[i];
  int32_t incl = s;
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t t = __shfl_up(incl, off, kWave);
    if (lane >= off) incl += t;
  }
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    int32_t v = lane < NW ? wsum[lane] : 0;
    int32_t vi = v;
    for (int off = 1; off < kWave; off <<= 1) {
      const int32_t t = __shfl_up(vi, off, kWave);
      if (lane >= off) vi += t;
    }
    if (lane < NW) wsum[lane] = vi - v;
    if (lane == NW - 1) wsum[NW] = vi;
  }
  __syncthreads();
  int32_t run = wsum[wave] + incl - s;
  for (int i = a; i < b; i++) {
    const int32_t v = A[i];
    A[i] = run;
    run += v;
  }
  if (tid == 0) A[k] = wsum[NW];
  __syncthreads();
}

// Medium x: one workgroup per vertex, c(x, .) in an LDS hash of
// kMediumSlots slots (keys, and 16-bit counts packed two per word: every
// count is at most W(x) <= kMediumWedges < 2^16); wedges enumerated flat over
// batches of lower neighbours so every thread reads a share of each batch.
// Per-edge mode walks the wedges a second time once the counts are final:
// wedge x - v - y adds c(x, y) - 1 to edge (v, y) and, summed over the
// wedges of v, to edge (x, v).
template <bool PER_EDGE>
__global__ __launch_bounds__(kMediumBlock) void k_c4_medium(C4Args g) {
  __shared__ int32_t hkey[kMediumSlots];
  __shared__ uint32_t hcnt[kMediumSlots / 2];
  __shared__ int32_t sPre[kMediumBlock + 1], sStart[kMediumBlock], sums[kMediumBlock / kWave + 1];
  __shared__ u64 credit[PER_EDGE ? kMediumBlock : 1];
  __shared__ u64 red[32];
  const int tid = threadIdx.x;
  for (int h = tid; h < kMediumSlots; h += kMediumBlock) hkey[h] = -1;
  for (int h = tid; h < kMediumSlots / 2; h += kMediumBlock) hcnt[h] = 0;
  __syncthreads();
  u128 acc = 0;
  for (int it = blockIdx.x; it < g.nlist; it += gridDim.x) {
    const int x = g.list[it];
    const u64 w = g.W[x];
    // table size: a multiple of 64 above W(x) >= distinct endpoints (load < 3/4)
    const int hs = (int)min<u64>((u64)kMediumSlots, ((3 * w / 2) + 64) & ~63ull);
    const int Lx = g.rp2[x], nL = g.lcnt[x];
    for (int b = 0; b < nL; b += kMediumBlock) {
      const int nb = min(kMediumBlock, nL - b);
      if (tid < nb) {
        const int q = Lx + b + tid;
        const int s = g.rp2[g.col2[q]];
        sStart[tid] = s;
        sPre[tid] = g.tpos[q] - s;
      }
      __syncthreads();
      scan_excl<kMediumBlock>(sPre, nb, sums);
      const int total = sPre[nb];
      // each thread takes a contiguous range of the wedges: one search for
      // the list of its first, then a cursor
      const int per = (total + kMediumBlock - 1) / kMediumBlock;
      const int t0 = tid * per, t1 = min(total, t0 + per);
      if (t0 < t1) {
        int o = upper_index_dev<int32_t>(sPre, nb, t0);
        int lo = sPre[o], next = sPre[o + 1];
        for (int t = t0; t < t1; t++) {
          while (t >= next) {  // ends: t < total = sPre[nb]
            o++;
            lo = next;
            next = sPre[o + 1];
          }
          const int y = g.col2[sStart[o] + (t - lo)];
          int h = (int)(((u64)((uint32_t)y * 2654435761u) * (u64)hs) >> 32);
          while (true) {
            const int old = atomicCAS(&hkey[h], -1, y);
            if (old == -1 || old == y) {
              atomicAdd(&hcnt[h >> 1], (h & 1) ? 65536u : 1u);
              break;
            }
            h = h + 1 == hs ? 0 : h + 1;
          }
        }
      }
      __syncthreads();
    }
    if (PER_EDGE) {
      for (int b = 0; b < nL; b += kMediumBlock) {
        const int nb = min(kMediumBlock, nL - b);
        if (tid < nb) {
          const int q = Lx + b + tid;
          const int s = g.rp2[g.col2[q]];
          sStart[tid] = s;
          sPre[tid] = g.tpos[q] - s;
          credit[tid] = 0;
        }
        __syncthreads();
        scan_excl<kMediumBlock>(sPre, nb, sums);
        const int total = sPre[nb];
        // contiguous ranges and a list cursor, as in the count above; the
        // credits of edge (x, v) gather in a register while the list lasts
        const int per = (total + kMediumBlock - 1) / kMediumBlock;
        const int t0 = tid * per, t1 = min(total, t0 + per);
        if (t0 < t1) {
          int o = upper_index_dev<int32_t>(sPre, nb, t0);
          int lo = sPre[o], next = sPre[o + 1];
          u64 cr = 0;
          for (int t = t0; t < t1; t++) {
            while (t >= next) {  // ends: t < total = sPre[nb]
              if (cr) atomicAdd(&credit[o], cr);
              cr = 0;
              o++;
              lo = next;
              next = sPre[o + 1];
            }
            const int p = sStart[o] + (t - lo);
            const int y = g.col2[p];
            int h = (int)(((u64)((uint32_t)y * 2654435761u) * (u64)hs) >> 32);
            while (hkey[h] != y) h = h + 1 == hs ? 0 : h + 1;  // y was inserted above
            const uint32_t c = (hcnt[h >> 1] >> ((h & 1) * 16)) & 0xffffu;
            if (c >= 2) {
              atomicAdd(&g.C4w[p], (u64)(c - 1));
              cr += c - 1;
            }
          }
          if (cr) atomicAdd(&credit[o], cr);
        }
        __syncthreads();
        if (tid < nb && credit[tid]) atomicAdd(&g.C4w[Lx + b + tid], credit[tid]);
        __syncthreads();
      }
    }
    u64 part = 0;
    for (int h = tid; h < hs; h += kMediumBlock) {
      if (hkey[h] != -1) {
        const uint32_t pair = hcnt[h >> 1];
        part += choose2((h & 1) ? (pair >> 16) : (pair & 0xffffu));
        hkey[h] = -1;
      }
    }
    __syncthreads();
    for (int h = tid; h < (hs + 1) / 2; h += kMediumBlock) hcnt[h] = 0;
    acc += (u128)part;
    __syncthreads();
  }
  const u128 s = block_sum_u128(acc, red);
  if (threadIdx.x == 0 && s) atomic_add_u128(g.c4ni, s);
}


// Counter bands of the heavy chunks.  c(x, y) <= min(nL, deg y), and degrees
// do not decrease with rank, so the counters of a chunk of low-degree
// endpoints need few bits: a chunk's counters are 2^lb-bit fields packed
// 2^(5-lb) to a 32-bit word (lb = 1: 2 bits, ..., lb = 5: 32 bits), and a
// chunk is as wide as CW words of its fields (kChunkWords, or kChunkWordsPE
// in per-edge mode), so the y range of an
// item is walked in fewer chunks where its endpoints have low degrees.  No
// field can overflow into its neighbour.
__device__ __forceinline__ void band_add(uint32_t *cnt, int lb, int d) {
  const int fl = 5 - lb;
  atomicAdd(&cnt[d >> fl], 1u << ((d & ((1 << fl) - 1)) << lb));
}

__device__ __forceinline__ uint32_t band_mask(int lb) {
  return lb == 5 ? 0xffffffffu : (1u << (1 << lb)) - 1u;
}

__device__ __forceinline__ uint32_t band_get(const uint32_t *cnt, int lb, int d) {
  const int fl = 5 - lb;
  return (cnt[d >> fl] >> ((d & ((1 << fl) - 1)) << lb)) & band_mask(lb);
}

// Sum of C(c, 2) over the counters of four consecutive words (one 16-byte
// LDS read of the sweep).  Byte counters: sum c^2 - sum c from byte dot
// products (4-bit counters split into two byte sets); 2-bit: popcounts.
__device__ __forceinline__ u64 band_quad_pairs(uint4 v, int lb) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  if (lb == 1) {  // c in 0..3: C(c, 2) = 0, 0, 1, 3
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const uint32_t hi = (w[i] >> 1) & 0x55555555u, lo = w[i] & 0x55555555u;
      s += (uint32_t)__popc(hi & ~lo) + 3u * (uint32_t)__popc(hi & lo);
    }
    return s;
  }
  if (lb <= 3) {  // at most 32 counters of 15, or 16 of 255: the sums fit 32 bits
    uint32_t sq = 0, sm = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      if (lb == 2) {
        const uint32_t lo = w[i] & 0x0f0f0f0fu, hi = (w[i] >> 4) & 0x0f0f0f0fu;
        sq = __builtin_amdgcn_udot4(lo, lo, sq, false);
        sq = __builtin_amdgcn_udot4(hi, hi, sq, false);
        sm = __builtin_amdgcn_udot4(lo, 0x01010101u, sm, false);
        sm = __builtin_amdgcn_udot4(hi, 0x01010101u, sm, false);
      } else {
        sq = __builtin_amdgcn_udot4(w[i], w[i], sq, false);
        sm = __builtin_amdgcn_udot4(w[i], 0x01010101u, sm, false);
      }
    }
    return (sq - sm) / 2;
  }
  u64 s = 0;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    if (lb == 4) s += choose2(w[i] & 0xffffu) + choose2(w[i] >> 16);
    else s += choose2(w[i]);
  }
  return s;
}

// This thread's share of the chunk's sum of C(c, 2), its counters cleared.
template <int CW>
__device__ __forceinline__ u64 band_sweep(uint32_t *cnt, int lb) {
  u64 part = 0;
  uint4 *c4 = reinterpret_cast<uint4 *>(cnt);
  for (int w = threadIdx.x; w < CW / 4; w += blockDim.x) {
    const uint4 v = c4[w];
    if (v.x | v.y | v.z | v.w) {
      c4[w] = make_uint4(0u, 0u, 0u, 0u);
      part += band_quad_pairs(v, lb);
    }
  }
  return part;
}

// Ranks bounding the bands: R[j] (j = 0..3) is the first rank whose degree
// exceeds the largest count of 2^(j+1)-bit fields (3, 15, 255, 65535); R[4]
// is the first rank of degree at least 2 (endpoints of degree 1 close no
// 4-cycle: c(x, y) <= 1).  Computed by threads 0..4, one binary search each.
__device__ void band_ranks(const int32_t *deg2, int64_t n, int32_t *R) {
  const int t = threadIdx.x;
  if (t < 5) {
    const int64_t lim = t == 4 ? 1 : (int64_t)band_mask(t + 1);
    int64_t lo = 0, hi = n;  // first rank with deg2 > lim
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)deg2[mid] > lim) hi = mid;
      else lo = mid + 1;
    }
    R[t] = (int32_t)lo;
  }
}

// The next chunk [c0, c1) of an item and its field width 2^lb: the widest
// chunk whose counters fit (the same on every thread).
template <int CW>
__device__ __forceinline__ int band_chunk(int c0, int yb, int nL, const int32_t *R, int *lb_out) {
  int64_t best = -1;
  int blb = 5;
  for (int lb = 1; lb <= 5; lb++) {
    int64_t c1 = min((int64_t)yb, (int64_t)c0 + ((int64_t)CW << (5 - lb)));
    if ((uint32_t)nL > band_mask(lb)) {
      if (c0 >= R[lb - 1]) continue;
      c1 = min(c1, (int64_t)R[lb - 1]);
    }
    if (c1 > best) {
      best = c1;
      blb = lb;
    }
  }
  *lb_out = blb;
  return (int)best;
}

// Per-edge credits of heavy wedges: wedge x - v - y adds c(x, y) - 1 to
// edge (v, y) at v's entry b for y.  With C4h (every entry's credit total
// fits 32 bits) the entries b, b + 1 (b even) share one 64-bit atomic add;
// otherwise each entry takes its own, into C4w.
__device__ __forceinline__ void credit_pair(const C4Args &g, int b, uint32_t lo, uint32_t hi) {
  if (g.C4h) {
    if (lo | hi)
      atomicAdd(reinterpret_cast<unsigned long long *>(g.C4h + b),
                (unsigned long long)(((u64)hi << 32) | lo));
  } else {
    if (lo) atomicAdd(&g.C4w[b], (u64)lo);
    if (hi) atomicAdd(&g.C4w[b + 1], (u64)hi);
  }
}

__device__ __forceinline__ void credit_one(const C4Args &g, int b, uint32_t v) {
  if (!v) return;
  if (g.C4h) atomicAdd(g.C4h + b, v);
  else atomicAdd(&g.C4w[b], (u64)v);
}

// The chunk's counts are complete: credits of one thread's run [st, en) of a
// list (entries below c0 take none), read PF at a time from an even entry;
// returns their sum, which also goes to edge (x, v).
template <int PF>
__device__ __forceinline__ u64 credit_run_thread(const C4Args &g, const uint32_t *cnt, int lb, int c0,
                                                 int st, int en) {
  static_assert(PF % 2 == 0, "pairs");
  u64 cr = 0;
  for (int b = st & ~1; b < en; b += PF) {
    int yv[PF];
#pragma unroll
    for (int k = 0; k < PF; k++) yv[k] = b + k >= st && b + k < en ? g.col2[b + k] : -1;
    uint32_t cv[PF];
#pragma unroll
    for (int k = 0; k < PF; k++) {
      cv[k] = yv[k] >= c0 ? band_get(cnt, lb, yv[k] - c0) - 1 : 0u;  // c >= 1: the wedge itself
      cr += cv[k];
    }
#pragma unroll
    for (int k = 0; k < PF; k += 2) credit_pair(g, b + k, cv[k], cv[k + 1]);
  }
  return cr;
}

// The same for a run read by a whole wave, 64 consecutive entries at a time;
// an even entry's lane adds its odd neighbour's credit with its own.  Returns
// the run's total on every lane.
__device__ __forceinline__ u64 credit_run_wave(const C4Args &g, const uint32_t *cnt, int lb, int c0,
                                               int st, int en) {
  const int lane = lane_id();
  u64 cr = 0;
  for (int b0 = st; b0 < en; b0 += kWave) {  // the same trip count on every lane
    const int b = b0 + lane;
    uint32_t cv = 0;
    if (b < en) {
      const int y = g.col2[b];
      if (y >= c0) cv = band_get(cnt, lb, y - c0) - 1;
    }
    cr += cv;
    const uint32_t next = __shfl_down(cv, 1, kWave);  // zero past the run
    if (b < en) {
      if (!(b & 1)) {
        if (lane < kWave - 1) credit_pair(g, b, cv, next);
        else credit_one(g, b, cv);  // b + 1 is lane 0's of the next round
      } else if (lane == 0) {
        credit_one(g, b, cv);  // its even neighbour is not in this round
      }
    }
  }
  return wave_sum_u64(cr);
}

// One heavy item by walking: list i of the item (the part of N(v_i) below x)
// is owned by thread i mod block, at most LPT per thread, with its cursor and
// the next PF entries in registers (nL <= kWalkLists, kWalkListsPE in
// per-edge mode, and the run queue holds every list).  Per chunk, each thread
// counts the buffered entries below the chunk's end and reloads its buffer
// from the new cursor (the loads of the next chunk are in flight while the
// chunk is summed); a run that continues past the buffer takes up to three
// more rounds of 8 entries (all of the thread's lists at once), and one
// longer still is queued (in LDS) and read by a whole wave, two runs at a
// time, two rows of 64 consecutive entries of each per round.  The chunk's
// counters are summed and cleared by a sweep of the LDS words, 16 bytes per
// read.  Entries below the first counted rank (endpoints of degree <= 1,
// which close no 4-cycle) are passed over in the first chunk.  Per-edge mode
// (PE) credits each wedge once the chunk's counts are complete, before the
// sweep.  Two to four barriers per chunk, no global cursor state.
template <int LPT, int PF, int XR, bool PE, int CW>
__device__ __forceinline__ void heavy_walk_item(const C4Args &g, int Lx, int nL, int ya_item,
                                                int yb, uint32_t *cnt, const int32_t *R,
                                                int32_t *qpos, int32_t *qend, int32_t *qstart,
                                                int32_t *qid, int *s_nq, u128 &acc) {
  constexpr int NW = kC4HeavyBlock / kWave;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int ys = max(ya_item, R[4]);
  if (tid == 0) s_nq[0] = s_nq[1] = 0;
  int p[LPT], e[LPT], buf[LPT][PF];
#pragma unroll
  for (int r = 0; r < LPT; r++) {
    const int i = tid + r * kC4HeavyBlock;
    p[r] = 0;
    e[r] = 0;
    if (i < nL) {
      const int q = Lx + i;
      const int s = g.rp2[g.col2[q]];
      e[r] = g.tpos[q];
      p[r] = ya_item > 0 ? s + lower_bound_dev<int32_t>(g.col2 + s, e[r] - s, ys) : s;
    }
  }
#pragma unroll
  for (int r = 0; r < LPT; r++)
#pragma unroll
    for (int k = 0; k < PF; k++) buf[r][k] = p[r] + k < e[r] ? g.col2[p[r] + k] : INT32_MAX;
  __syncthreads();
  int par = 0;
  for (int c0 = ys, c1; c0 < yb; c0 = c1, par ^= 1) {
    int lb;
    c1 = band_chunk<CW>(c0, yb, nL, R, &lb);
    int qs[LPT];  // queue slot of a list whose run goes on past what it read, or -1
    int q[LPT];   // cursor after the entries read so far in this chunk
    int ps[LPT];  // per-edge: the cursor at the chunk's start
    bool run[LPT];
#pragma unroll
    for (int r = 0; r < LPT; r++) {
      ps[r] = p[r];
      int taken = 0;
      bool live = true;
#pragma unroll
      for (int k = 0; k < PF; k++) {
        live = live && buf[r][k] < c1;
        if (live) {
          if (buf[r][k] >= c0) band_add(cnt, lb, buf[r][k] - c0);
          taken++;
        }
      }
      q[r] = p[r] + taken;
      run[r] = taken == PF && q[r] < e[r];
    }
    // runs longer than the buffer: up to three more rounds of XR entries
    // here, the loads of all the thread's lists in flight together
#pragma unroll
    for (int round = 0; round < 3; round++) {
      bool any = false;
#pragma unroll
      for (int r = 0; r < LPT; r++) any = any || run[r];
      if (!any) break;
      int yv[LPT][XR];
#pragma unroll
      for (int r = 0; r < LPT; r++)
#pragma unroll
        for (int k = 0; k < XR; k++)
          yv[r][k] = run[r] && q[r] + k < e[r] ? g.col2[q[r] + k] : INT32_MAX;
#pragma unroll
      for (int r = 0; r < LPT; r++) {
        int t = 0;
        bool lv = run[r];
#pragma unroll
        for (int k = 0; k < XR; k++) {
          lv = lv && yv[r][k] < c1;
          if (lv) {
            if (yv[r][k] >= c0) band_add(cnt, lb, yv[r][k] - c0);
            t++;
          }
        }
        q[r] += t;
        run[r] = run[r] && t == XR && q[r] < e[r];
      }
    }
#pragma unroll
    for (int r = 0; r < LPT; r++) {
      qs[r] = -1;
      if (run[r]) {
        // each list is queued at most once per chunk: the queue holds them all
        const int slot = atomicAdd(&s_nq[par], 1);
        qpos[slot] = q[r];
        qend[slot] = e[r];
        if (PE) {
          qstart[slot] = q[r];
          qid[slot] = tid + r * kC4HeavyBlock;
        }
        qs[r] = slot;
      } else if (q[r] != p[r]) {
        p[r] = q[r];
#pragma unroll
        for (int k = 0; k < PF; k++) buf[r][k] = p[r] + k < e[r] ? g.col2[p[r] + k] : INT32_MAX;
      }
    }
    __syncthreads();
    const int nq = s_nq[par];
    if (tid == 0) s_nq[par ^ 1] = 0;  // the next chunk's queue
    if (nq > 0) {  // the same on every thread
      // a wave reads QR runs at once, two rows of 64 entries of each per round
      constexpr int QR = 2;
      for (int q0 = wave * QR; q0 < nq; q0 += NW * QR) {
        int pos[QR], qe[QR];
        bool go[QR];  // the same on the wave: from LDS, then from ballots
#pragma unroll
        for (int r = 0; r < QR; r++) {
          go[r] = q0 + r < nq;
          pos[r] = go[r] ? qpos[q0 + r] : 0;
          qe[r] = go[r] ? qend[q0 + r] : 0;
        }
        while (go[0] || go[1]) {
          int y0[QR], y1[QR];
#pragma unroll
          for (int r = 0; r < QR; r++) {
            const int p0 = pos[r] + lane, p1 = pos[r] + kWave + lane;
            y0[r] = go[r] && p0 < qe[r] ? g.col2[p0] : INT32_MAX;
            y1[r] = go[r] && p1 < qe[r] ? g.col2[p1] : INT32_MAX;
          }
#pragma unroll
          for (int r = 0; r < QR; r++) {
            if (!go[r]) continue;
            const bool in0 = y0[r] < c1, in1 = y1[r] < c1;
            if (in0 && y0[r] >= c0) band_add(cnt, lb, y0[r] - c0);
            if (in1 && y1[r] >= c0) band_add(cnt, lb, y1[r] - c0);
            const u64 b0 = __ballot(!in0), b1 = __ballot(!in1);
            if (b0) {
              pos[r] += __ffsll((long long)b0) - 1;
              go[r] = false;
            } else if (b1) {
              pos[r] += kWave + __ffsll((long long)b1) - 1;
              go[r] = false;
            } else {
              pos[r] += 2 * kWave;
            }
          }
        }
        if (lane == 0) {
#pragma unroll
          for (int r = 0; r < QR; r++)
            if (q0 + r < nq) qpos[q0 + r] = pos[r];
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < LPT; r++)
        if (qs[r] >= 0) {
          p[r] = qpos[qs[r]];
#pragma unroll
          for (int k = 0; k < PF; k++) buf[r][k] = p[r] + k < e[r] ? g.col2[p[r] + k] : INT32_MAX;
        }
    }
    if (PE) {
      // The chunk's counts are complete: wedge x - v - y adds c(x, y) - 1 to
      // edge (v, y) (v's entry for y) and, summed per list, to edge (x, v)
      // (x's entry for v).  Each thread rereads its own part of its runs,
      // each wave the queued parts it read.
#pragma unroll
      for (int r = 0; r < LPT; r++) {
        const u64 cr = credit_run_thread<PF>(g, cnt, lb, c0, ps[r], q[r]);
        if (cr) atomicAdd(&g.C4w[Lx + tid + r * kC4HeavyBlock], cr);
      }
      for (int qi = wave; qi < nq; qi += NW) {
        const u64 cr = credit_run_wave(g, cnt, lb, c0, qstart[qi], qpos[qi]);
        if (lane == 0 && cr) atomicAdd(&g.C4w[Lx + qid[qi]], cr);
      }
      __syncthreads();  // the counters are read before the sweep clears them
    }
    acc += (u128)band_sweep<CW>(cnt, lb);
    __syncthreads();
  }
  __syncthreads();  // s_item is rewritten next
}

// One heavy item with more lists than the registers of the walking path hold:
// the same walk, over groups of 2 x block lists in turn within each chunk,
// each list's cursor and end kept in the workgroup's slot of global memory
// (cur, end) between groups and chunks, and its first PF entries read when
// its group comes up.  The run queue is emptied per group.
template <bool PE, int CW>
__device__ __forceinline__ void heavy_walk_groups(const C4Args &g, int Lx, int nL, int ya_item,
                                                  int yb, uint32_t *cnt, const int32_t *R,
                                                  int32_t *qpos, int32_t *qend, int32_t *qstart,
                                                  int32_t *qid, int *s_nq, int32_t *cur,
                                                  int32_t *end, int32_t *cb, u128 &acc) {
  constexpr int LPT = 2, PF = 8, XR = 8, GS = LPT * kC4HeavyBlock;
  constexpr int NW = kC4HeavyBlock / kWave;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int ys = max(ya_item, R[4]);
  for (int i = tid; i < nL; i += kC4HeavyBlock) {
    const int q = Lx + i;
    const int s = g.rp2[g.col2[q]];
    const int e = g.tpos[q];
    cur[i] = ya_item > 0 ? s + lower_bound_dev<int32_t>(g.col2 + s, e - s, ys) : s;
    end[i] = e;
  }
  if (tid == 0) s_nq[0] = s_nq[1] = 0;
  __syncthreads();
  int par = 0;
  for (int c0 = ys, c1; c0 < yb; c0 = c1) {
    int lb;
    c1 = band_chunk<CW>(c0, yb, nL, R, &lb);
    for (int g0 = 0; g0 < nL; g0 += GS, par ^= 1) {
      int p[LPT], e[LPT], q[LPT], qs[LPT];
      bool run[LPT];
      int buf[LPT][PF];
#pragma unroll
      for (int r = 0; r < LPT; r++) {
        const int i = g0 + tid + r * kC4HeavyBlock;
        p[r] = i < nL ? cur[i] : 0;
        e[r] = i < nL ? end[i] : 0;
        if (PE && i < nL) cb[i] = p[r];  // where the list's run in this chunk starts
      }
#pragma unroll
      for (int r = 0; r < LPT; r++)
#pragma unroll
        for (int k = 0; k < PF; k++) buf[r][k] = p[r] + k < e[r] ? g.col2[p[r] + k] : INT32_MAX;
#pragma unroll
      for (int r = 0; r < LPT; r++) {
        int taken = 0;
        bool live = true;
#pragma unroll
        for (int k = 0; k < PF; k++) {
          live = live && buf[r][k] < c1;
          if (live) {
            if (buf[r][k] >= c0) band_add(cnt, lb, buf[r][k] - c0);
            taken++;
          }
        }
        q[r] = p[r] + taken;
        run[r] = taken == PF && q[r] < e[r];
      }
#pragma unroll
      for (int round = 0; round < 3; round++) {
        bool any = false;
#pragma unroll
        for (int r = 0; r < LPT; r++) any = any || run[r];
        if (!any) break;
        int yv[LPT][XR];
#pragma unroll
        for (int r = 0; r < LPT; r++)
#pragma unroll
          for (int k = 0; k < XR; k++)
            yv[r][k] = run[r] && q[r] + k < e[r] ? g.col2[q[r] + k] : INT32_MAX;
#pragma unroll
        for (int r = 0; r < LPT; r++) {
          int t = 0;
          bool lv = run[r];
#pragma unroll
          for (int k = 0; k < XR; k++) {
            lv = lv && yv[r][k] < c1;
            if (lv) {
              if (yv[r][k] >= c0) band_add(cnt, lb, yv[r][k] - c0);
              t++;
            }
          }
          q[r] += t;
          run[r] = run[r] && t == XR && q[r] < e[r];
        }
      }
#pragma unroll
      for (int r = 0; r < LPT; r++) {
        const int i = g0 + tid + r * kC4HeavyBlock;
        qs[r] = -1;
        if (run[r]) {
          const int slot = atomicAdd(&s_nq[par], 1);  // at most GS per group
          qpos[slot] = q[r];
          qend[slot] = e[r];
          qs[r] = slot;
        } else if (i < nL && q[r] != p[r]) {
          cur[i] = q[r];
        }
      }
      __syncthreads();
      const int nq = s_nq[par];
      if (tid == 0) s_nq[par ^ 1] = 0;  // the next group's queue
      if (nq > 0) {  // the same on every thread
        for (int qi = wave; qi < nq; qi += NW) {
          int pos = qpos[qi];
          const int qe = qend[qi];
          while (true) {  // every exit is decided by a ballot: the same on the wave
            const int p0 = pos + lane, p1 = pos + kWave + lane;
            const int y0 = p0 < qe ? g.col2[p0] : INT32_MAX;
            const int y1 = p1 < qe ? g.col2[p1] : INT32_MAX;
            const bool in0 = y0 < c1, in1 = y1 < c1;
            if (in0 && y0 >= c0) band_add(cnt, lb, y0 - c0);
            if (in1 && y1 >= c0) band_add(cnt, lb, y1 - c0);
            const u64 b0 = __ballot(!in0), b1 = __ballot(!in1);
            if (b0) {
              pos += __ffsll((long long)b0) - 1;
              break;
            }
            if (b1) {
              pos += kWave + __ffsll((long long)b1) - 1;
              break;
            }
            pos += 2 * kWave;
          }
          if (lane == 0) qpos[qi] = pos;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < LPT; r++)
          if (qs[r] >= 0) cur[g0 + tid + r * kC4HeavyBlock] = qpos[qs[r]];
      }
      __syncthreads();  // the queue is rewritten by the next group
    }
    if (PE) {
      // The chunk's counts are complete: each list's run in it is
      // [cb, cur).  Group by group, a thread credits the short runs of its
      // lists itself and queues the longer ones for whole waves.
      for (int g0 = 0; g0 < nL; g0 += GS, par ^= 1) {
#pragma unroll
        for (int r = 0; r < LPT; r++) {
          const int i = g0 + tid + r * kC4HeavyBlock;
          if (i >= nL) continue;
          const int st = cb[i], en = cur[i];
          if (en - st > PF + 3 * XR) {
            const int slot = atomicAdd(&s_nq[par], 1);
            qstart[slot] = st;
            qpos[slot] = en;
            qid[slot] = i;
            continue;
          }
          const u64 cr = credit_run_thread<PF>(g, cnt, lb, c0, st, en);
          if (cr) atomicAdd(&g.C4w[Lx + i], cr);
        }
        __syncthreads();
        const int nq = s_nq[par];
        if (tid == 0) s_nq[par ^ 1] = 0;
        for (int qi = wave; qi < nq; qi += NW) {
          const u64 cr = credit_run_wave(g, cnt, lb, c0, qstart[qi], qpos[qi]);
          if (lane == 0 && cr) atomicAdd(&g.C4w[Lx + qid[qi]], cr);
        }
        __syncthreads();  // the queue is rewritten by the next group
      }
    }
    acc += (u128)band_sweep<CW>(cnt, lb);
    __syncthreads();
  }
  __syncthreads();  // s_item is rewritten next
}

// Heavy x: work items (x, y range) taken from a queue, one workgroup each,
// walked chunk by chunk (heavy_walk_item, or heavy_walk_groups for more
// lists than the registers hold).  In per-edge mode each wedge x - v - y
// adds c(x, y) - 1 to edge (v, y) and to edge (x, v), each at a directed
// entry (folded into the edge's upper position afterwards).
template <bool PER_EDGE>
__global__ __launch_bounds__(kC4HeavyBlock) void k_c4_heavy_bal(C4Args g) {
  constexpr int CW = PER_EDGE ? kChunkWordsPE : kChunkWords;
  __shared__ __align__(16) uint32_t cnt[CW];
  // the run queue, a slot per list of a walk or a group: position and end,
  // and per-edge the start and the list
  constexpr int QL = PER_EDGE ? kWalkListsPE : kWalkLists;
  static_assert(QL >= 2 * kC4HeavyBlock, "a group's lists fit the queue");
  __shared__ int32_t qpos[QL], qend[QL];
  __shared__ int32_t qid[PER_EDGE ? QL : 1], qstart[PER_EDGE ? QL : 1];
  __shared__ u64 red[32];
  __shared__ int s_item, s_nq[2];
  __shared__ int32_t s_R[5];
  const int tid = threadIdx.x;
  band_ranks(g.deg2, g.n, s_R);
  const int64_t nitems = *g.nitems;
  // per-slot list state of heavy_walk_groups: cursor, end, and per-edge the
  // cursor where the current chunk began
  int32_t *cur = g.gcur + (size_t)blockIdx.x * g.lmax;
  int32_t *end = g.gbeg + (size_t)blockIdx.x * g.lmax;
  int32_t *cb = PER_EDGE ? g.gcb + (size_t)blockIdx.x * g.lmax : nullptr;
  for (int w = tid; w < CW; w += kC4HeavyBlock) cnt[w] = 0;
  u128 acc = 0;
  while (true) {
    if (tid == 0) s_item = (int)atomicAdd(g.queue, 1ull);
    __syncthreads();
    const int item = s_item;
    if (item >= nitems) break;
    const int4 it = g.items[item];
    const int x = it.x, yb = it.z;
    const int Lx = g.rp2[x], nL = g.lcnt[x];
    if (nL <= QL) {  // the same on every thread
      if (nL <= kC4HeavyBlock) {
        heavy_walk_item<1, 8, 8, PER_EDGE, CW>(g, Lx, nL, it.y, yb, cnt, s_R, qpos, qend, qstart,
                                               qid, s_nq, acc);
      } else if constexpr (PER_EDGE) {
        heavy_walk_item<2, 8, 8, true, CW>(g, Lx, nL, it.y, yb, cnt, s_R, qpos, qend, qstart, qid,
                                           s_nq, acc);
      } else {
        if (nL <= 2 * kC4HeavyBlock)
          heavy_walk_item<2, 8, 8, false, CW>(g, Lx, nL, it.y, yb, cnt, s_R, qpos, qend, qstart,
                                              qid, s_nq, acc);
        else
          heavy_walk_item<3, 8, 8, false, CW>(g, Lx, nL, it.y, yb, cnt, s_R, qpos, qend, qstart,
                                              qid, s_nq, acc);
      }
      continue;
    }
    heavy_walk_groups<PER_EDGE, CW>(g, Lx, nL, it.y, yb, cnt, s_R, qpos, qend, qstart, qid, s_nq,
                                    cur, end, cb, acc);
  }
  const u128 s = block_sum_u128(acc, red);
  if (threadIdx.x == 0 && s) atomic_add_u128(g.c4ni, s);
}

// ------------------------------------------------------------ dense hub slabs

// Number of the slab's hubs above rank y (xs descending: a prefix).
__device__ __forceinline__ int hubs_above(const int32_t *xs, int nslab, int y) {
  int lo = 0, hi = nslab;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (xs[mid] > y) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// First rank whose degree exceeds kDenseShortDeg (degrees grow with rank).
__device__ int first_long_row(const int32_t *rp2, int64_t n) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (rp2[mid + 1] - rp2[mid] > kDenseShortDeg) hi = mid;
    else lo = mid + 1;
  }
  return (int)lo;
}

// Sets (or clears) bit k of the mask of every lower neighbour of hub k.
template <bool SET>
__global__ void k_hub_mark(HubArgs g) {
  const int k = blockIdx.x;
  if (k >= g.nslab) return;
  const int x = g.xs[k];
  const int a = g.rp2[x], nl = g.lcnt[x];
  const u64 bit = 1ull << (k & 63);
  for (int i = threadIdx.x; i < nl; i += blockDim.x) {
    const size_t v = (size_t)g.col2[a + i];
    if (SET) {
      atomicOr(&g.mask[kDenseWords * v + (k >> 6)], bit);
    } else {
      for (int w = 0; w < kDenseWords; w++) g.mask[kDenseWords * v + w] = 0;
    }
  }
}

// Adds a one-bit-per-hub mask to the bit planes (counters up to 1023).
constexpr int kShortBits = 10;
__device__ __forceinline__ void plane_add(u64 (&P)[kShortBits], u64 m) {
#pragma unroll
  for (int j = 0; j < kShortBits; j++) {
    const u64 c = P[j] & m;
    P[j] ^= m;
    m = c;
  }
}

// sum over the hubs in V of C(c_k, 2), c_k held in bit planes:
//   sum c^2 - sum c = sum_j (4^j - 2^j) |P_j & V| + 2 sum_{j<j'} 2^(j+j') |P_j & P_j' & V|.
__device__ __forceinline__ u64 planes_pairs(const u64 (&P)[kShortBits], u64 V) {
  u64 s = 0;
#pragma unroll
  for (int j = 1; j < kShortBits; j++)
    s += (((1ull << (2 * j)) - (1ull << j)) / 2) * __popcll(P[j] & V);
#pragma unroll
  for (int j = 0; j < kShortBits; j++)
#pragma unroll
    for (int jj = j + 1; jj < kShortBits; jj++) s += (1ull << (j + jj)) * __popcll(P[j] & P[jj] & V);
  return s;
}

// Rows y of degree <= kDenseShortDeg below the slab's top hub, one thread
// each (rows are in degree order, so a wave's rows have similar lengths).
__global__ __launch_bounds__(256) void k_hub_short(HubArgs g) {
  __shared__ int32_t xs[kDenseSlab];
  __shared__ u64 red[32];
  __shared__ int s_long;
  for (int k = threadIdx.x; k < g.nslab; k += blockDim.x) xs[k] = g.xs[k];
  if (threadIdx.x == 0) s_long = first_long_row(g.rp2, g.n);
  __syncthreads();
  const int ylim = min(s_long, xs[0]);
  const ulonglong2 *M = reinterpret_cast<const ulonglong2 *>(g.mask);
  constexpr int NH = kDenseWords / 2;  // 128-bit halves per vertex
  u64 acc = 0;
  for (int y = blockIdx.x * blockDim.x + threadIdx.x; y < ylim; y += gridDim.x * blockDim.x) {
    const int t = hubs_above(xs, g.nslab, y);
    if (t == 0) continue;
    u64 P[kDenseWords][kShortBits];
#pragma unroll
    for (int w = 0; w < kDenseWords; w++)
#pragma unroll
      for (int j = 0; j < kShortBits; j++) P[w][j] = 0;
    const int a = g.rp2[y], b = g.rp2[y + 1];
    int p = a;
    // pairs of entries, the next pair's masks in flight while the current
    // pair's are added to the planes
    ulonglong2 mm[2][NH];
    if (p + 2 <= b) {
#pragma unroll
      for (int r = 0; r < 2; r++) {
        const int v = g.col2[p + r];
#pragma unroll
        for (int h = 0; h < NH; h++) mm[r][h] = M[(size_t)v * NH + h];
      }
    }
    for (; p + 2 <= b; p += 2) {
      ulonglong2 cur[2][NH];
#pragma unroll
      for (int r = 0; r < 2; r++)
#pragma unroll
        for (int h = 0; h < NH; h++) cur[r][h] = mm[r][h];
      if (p + 4 <= b) {
#pragma unroll
        for (int r = 0; r < 2; r++) {
          const int v = g.col2[p + 2 + r];
#pragma unroll
          for (int h = 0; h < NH; h++) mm[r][h] = M[(size_t)v * NH + h];
        }
      }
#pragma unroll
      for (int r = 0; r < 2; r++)
#pragma unroll
        for (int h = 0; h < NH; h++) {
          if (cur[r][h].x) plane_add(P[2 * h], cur[r][h].x);
          if (cur[r][h].y) plane_add(P[2 * h + 1], cur[r][h].y);
        }
    }
    for (; p < b; p++) {
      const int v = g.col2[p];
#pragma unroll
      for (int h = 0; h < NH; h++) {
        const ulonglong2 mm = M[(size_t)v * NH + h];
        if (mm.x) plane_add(P[2 * h], mm.x);
        if (mm.y) plane_add(P[2 * h + 1], mm.y);
      }
    }
    u64 any = 0;
#pragma unroll
    for (int w = 0; w < kDenseWords; w++)
#pragma unroll
      for (int j = 0; j < kShortBits; j++) any |= P[w][j];
    if (!any) continue;
#pragma unroll
    for (int w = 0; w < kDenseWords; w++) {
      const int tw = t - 64 * w;
      const u64 V = tw >= 64 ? ~0ull : (tw > 0 ? ((1ull << tw) - 1) : 0ull);
      acc += planes_pairs(P[w], V);
    }
  }
  const u128 s = block_sum_u128((u128)acc, red);
  if (threadIdx.x == 0 && s) atomic_add_u128(g.c4ni, s);
}

// Rows y of degree > kDenseShortDeg below the slab's top hub, one
// workgroup each.  Each thread adds a contiguous chunk of at most
// kDenseShortDeg entries into bit planes, as the short rows do, then adds
// its per-hub counts into the row's LDS counters (one atomic per hub it
// saw, not one per entry and hub); rows longer than 256 chunks take several
// rounds.
__global__ __launch_bounds__(256) void k_hub_long(HubArgs g) {
  __shared__ int32_t xs[kDenseSlab];
  __shared__ uint32_t cnt[kDenseSlab];
  __shared__ u64 red[32];
  __shared__ int s_long;
  for (int k = threadIdx.x; k < g.nslab; k += blockDim.x) xs[k] = g.xs[k];
  if (threadIdx.x == 0) s_long = first_long_row(g.rp2, g.n);
  __syncthreads();
  const int y0 = s_long, ylim = xs[0];
  const ulonglong2 *M = reinterpret_cast<const ulonglong2 *>(g.mask);
  constexpr int NH = kDenseWords / 2;
  constexpr int ROUND = 256 * kDenseShortDeg;  // entries per round of the workgroup
  u128 acc = 0;
  for (int y = y0 + blockIdx.x; y < ylim; y += gridDim.x) {
    const int t = hubs_above(xs, g.nslab, y);
    if (t == 0) continue;  // uniform
    for (int k = threadIdx.x; k < kDenseSlab; k += blockDim.x) cnt[k] = 0;
    __syncthreads();
    const int a = g.rp2[y], b = g.rp2[y + 1];
    for (int r0 = a; r0 < b; r0 += ROUND) {
      const int len = min(ROUND, b - r0);
      const int L = (len + 255) / 256;  // <= kDenseShortDeg: no plane overflows
      const int c0 = r0 + (int)threadIdx.x * L, c1 = min(r0 + len, c0 + L);
      u64 P[kDenseWords][kShortBits];
#pragma unroll
      for (int w = 0; w < kDenseWords; w++)
#pragma unroll
        for (int j = 0; j < kShortBits; j++) P[w][j] = 0;
      for (int p = c0; p < c1; p++) {
        const int v = g.col2[p];
#pragma unroll
        for (int h = 0; h < NH; h++) {
          const ulonglong2 mm = M[(size_t)v * NH + h];
          if (mm.x) plane_add(P[2 * h], mm.x);
          if (mm.y) plane_add(P[2 * h + 1], mm.y);
        }
      }
#pragma unroll
      for (int w = 0; w < kDenseWords; w++) {
        const int tw = t - 64 * w;
        u64 any = 0;
#pragma unroll
        for (int j = 0; j < kShortBits; j++) any |= P[w][j];
        any &= tw >= 64 ? ~0ull : (tw > 0 ? ((1ull << tw) - 1) : 0ull);
        while (any) {
          const int bit = __builtin_ctzll(any);
          any &= any - 1;
          uint32_t c = 0;
#pragma unroll
          for (int j = 0; j < kShortBits; j++) c |= (uint32_t)((P[w][j] >> bit) & 1ull) << j;
          atomicAdd(&cnt[64 * w + bit], c);
        }
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < t; k += blockDim.x) acc += (u128)choose2(cnt[k]);
    __syncthreads();
  }
  const u128 s = block_sum_u128(acc, red);
  if (threadIdx.x == 0 && s) atomic_add_u128(g.c4ni, s);
}

// Per-edge mode: the 4-cycle credits of an edge were added at either of its
// two directed entries; the lower one is folded into the upper position,
// where the per-edge outputs are read.
__global__ void k_c4_fold(const u64 *ekeys, const int32_t *col2, const int32_t *tpos, int64_t nnz,
                          int B, u64 *C4w, const uint32_t *C4h) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const int32_t x = (int32_t)(ekeys[p] >> B);
  if (col2[p] > x) {
    const int32_t q = tpos[p];
    u64 s = C4w[q];
    if (C4h) s += (u64)C4h[p] + C4h[q];
    C4w[p] += s;
  }
}

}  // namespace

int launch_c4_fold(const u64 *ekeys, const int32_t *col2, const int32_t *tpos, int64_t nnz, int B,
                   u64 *C4w, const uint32_t *C4h, hipStream_t s) {
  if (nnz <= 0) return GC_OK;
  k_c4_fold<<<grid1d(nnz, 256), 256, 0, s>>>(ekeys, col2, tpos, nnz, B, C4w, C4h);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

int launch_dense_slab(const HubArgs &g, hipStream_t s) {
  if (g.nslab <= 0) return GC_OK;
  k_hub_mark<true><<<g.nslab, 256, 0, s>>>(g);
  GC_TRY_HIP(hipGetLastError());
  const int cus = 256;
  k_hub_short<<<cus * 8, 256, 0, s>>>(g);
  GC_TRY_HIP(hipGetLastError());
  k_hub_long<<<cus * 4, 256, 0, s>>>(g);
  GC_TRY_HIP(hipGetLastError());
  k_hub_mark<false><<<g.nslab, 256, 0, s>>>(g);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

int launch_cycles_medium(C4Args g, bool per_edge, hipStream_t s) {
  if (g.nlist <= 0) return GC_OK;
  const unsigned grid = (unsigned)std::min(g.nlist, 16384);
  if (per_edge) k_c4_medium<true><<<grid, kMediumBlock, 0, s>>>(g);
  else k_c4_medium<false><<<grid, kMediumBlock, 0, s>>>(g);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

int launch_cycles_light(C4Args g, bool per_edge, hipStream_t s) {
  if (g.nlist <= 0) return GC_OK;
  const unsigned grid = (unsigned)std::min(g.nlist, 65536);
  if (per_edge) k_c4_light<true><<<grid, kWave, 0, s>>>(g);
  else k_c4_light<false><<<grid, kWave, 0, s>>>(g);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

int launch_cycles_heavy(C4Args g, int slots, bool per_edge, hipStream_t s) {
  if (slots <= 0) return GC_OK;
  if (per_edge) k_c4_heavy_bal<true><<<slots, kC4HeavyBlock, 0, s>>>(g);
  else k_c4_heavy_bal<false><<<slots, kC4HeavyBlock, 0, s>>>(g);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

}  // namespace gc
