// Prepass: contract validation, relabelling by degree, re-sorted adjacency,
// reverse-entry positions, per-vertex work estimates and work lists.
//
// The paper's implementation orders neighbour lists and edge jobs by degree
// (Section 5.1, batches of edge jobs); here the order is the total order
// x < y iff (deg x, x) < (deg y, y), applied by relabelling every vertex with
// its rank.  Under it, every vertex has at most sqrt(2m) upper neighbours,
// which bounds the per-vertex state of the clique pass, and every 4-cycle has
// one highest vertex, which the wedge pass aggregates on.
#include <cstring>

#include "kernels.h"
#include "primitives.h"

namespace gc {

namespace {

// Sets bit (-code) of *err for every violation; the host reports the lowest.
__global__ void k_validate(const int32_t *rp, const int32_t *col, int64_t n, int64_t nnz,
                           int32_t *err) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; u < n; u += stride) {
    const int64_t a = rp[u], b = rp[u + 1];
    if (a < 0 || b < a || b > nnz) {
      flag_err(err, GC_EINVAL);
      continue;
    }
    for (int64_t j = a; j < b; j++) {
      const int64_t v = col[j];
      if (v < 0 || v >= n) {
        flag_err(err, GC_EASYMMETRIC);
        break;
      }
      if (v == u) flag_err(err, GC_ESELFLOOP);
      if (j > a && col[j - 1] >= v) flag_err(err, GC_ENOTSORTED);
      const int64_t c = rp[v], d = rp[v + 1];
      if (c < 0 || d < c || d > nnz) continue;
      const int pos = lower_bound_dev<int32_t>(col + c, (int)(d - c), (int32_t)u);
      if (pos >= d - c || col[c + pos] != u) flag_err(err, GC_EASYMMETRIC);
    }
  }
}

__global__ void k_check_rowptr_ends(const int32_t *rp, int64_t n, int64_t nnz, int32_t *err) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    if (rp[0] != 0 || rp[n] != nnz) flag_err(err, GC_EINVAL);
}

// deg[u] and the key (deg << B | u) ordering vertices by (degree, id).
// A capped grid walks the vertices, so the maxima and sums below take one
// atomic per block (a per-wave atomic on one address serialises thousands).
constexpr int kRedBlock = 256;
constexpr int kRedGrid = 2048;

template <class T, class Op>
__device__ __forceinline__ T block_reduce(T v, Op op, T *sh) {
  for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off, kWave));
  const int wave = threadIdx.x / kWave;
  __syncthreads();  // sh may still be read by an earlier call
  if (lane_id() == 0) sh[wave] = v;
  __syncthreads();
  T r = sh[0];
  for (int w = 1; w < (int)(blockDim.x / kWave); w++) r = op(r, sh[w]);
  return r;
}

struct MaxOp {
  template <class T>
  __device__ T operator()(T a, T b) const { return a > b ? a : b; }
};
struct AddOp {
  template <class T>
  __device__ T operator()(T a, T b) const { return a + b; }
};

__global__ __launch_bounds__(kRedBlock) void k_degree_keys(const int32_t *rp, int64_t n, int B,
                                                           int32_t *deg, u64 *key,
                                                           int32_t *max_deg) {
  __shared__ int sh[kRedBlock / kWave];
  int mx = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    const int d = rp[u + 1] - rp[u];
    deg[u] = d;
    key[u] = ((u64)d << B) | (u64)u;
    mx = max(mx, d);
  }
  mx = block_reduce(mx, MaxOp(), sh);
  if (threadIdx.x == 0 && mx) atomicMax(max_deg, mx);
}

// order[x] = caller's id of new vertex x; rank[old] = x; deg2[x] = degree.
__global__ void k_rank(const u64 *sorted, int64_t n, int B, int32_t *order, int32_t *rank,
                       int32_t *deg2) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const u64 k = sorted[x];
  const int32_t old = (int32_t)(k & ((1ull << B) - 1));
  order[x] = old;
  rank[old] = (int32_t)x;
  deg2[x] = (int32_t)(k >> B);
}

// Edge keys (rank[u] << B | rank[w]) for every entry, in tiles of kEkTile
// consecutive entries.  The row of each entry comes from the row starts that
// fall inside the tile, marked in LDS and carried forward by a prefix max, so
// the entries are read and the keys written in order whatever the row
// lengths.  tilerow[t] is the row that holds entry t kEkTile, and
// tilerow[ntiles] the row of the last entry, both written by k_tile_rows;
// rows, tiles and ids are clamped, so a row_ptr that breaks the
// contract (unchecked without validation) gives wrong keys, never an access
// outside the arrays.  An id outside [0, n) is flagged and never indexed.
constexpr int kEkBlock = 256;
constexpr int kEkIpt = 8;
constexpr int kEkTile = kEkBlock * kEkIpt;

__global__ void k_tile_rows(const int32_t *rp, int64_t n, int64_t nnz, int64_t ntiles,
                            int32_t *tilerow) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
    const int64_t a = rp[u], b = min((int64_t)rp[u + 1], nnz);
    if (a < 0 || a >= b) continue;
    for (int64_t t = (a + kEkTile - 1) / kEkTile; t * kEkTile < b; t++) tilerow[t] = (int32_t)u;
    if (b == nnz) tilerow[ntiles] = (int32_t)u;
  }
}

__global__ __launch_bounds__(kEkBlock) void k_edge_keys(const int32_t *rp, const int32_t *col,
                                                        int64_t n, int64_t nnz, int B,
                                                        const int32_t *rank,
                                                        const int32_t *tilerow, u64 *ekeys,
                                                        int32_t *err) {
  __shared__ int32_t rowat[kEkTile];
  __shared__ int32_t wmax[kEkBlock / kWave];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  const int64_t t = blockIdx.x, ntiles = gridDim.x;
  const int64_t jb = t * kEkTile;
  const int cnt = (int)min((int64_t)kEkTile, nnz - jb);
  const int64_t uf = min(max((int64_t)tilerow[t], (int64_t)0), n - 1);
  const int64_t ul = min(max((int64_t)tilerow[t + 1], uf), n - 1);
#pragma unroll
  for (int r = 0; r < kEkIpt; r++) rowat[r * kEkBlock + tid] = r == 0 && tid == 0 ? (int32_t)uf : -1;
  __syncthreads();
  // rows after the tile's first row that start inside the tile (an empty row
  // starts where the next row does and is skipped)
  for (int64_t u = uf + 1 + tid; u <= ul; u += kEkBlock) {
    const int64_t a = rp[u], b = rp[u + 1];
    if (a >= jb && a < jb + cnt && b > a) rowat[a - jb] = (int32_t)u;
  }
  __syncthreads();
  // inclusive prefix max over the tile: kEkIpt consecutive slots per thread
  int32_t v[kEkIpt], m = -1;
#pragma unroll
  for (int r = 0; r < kEkIpt; r++) {
    m = max(m, rowat[tid * kEkIpt + r]);
    v[r] = m;
  }
  int32_t incl = m;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t o = __shfl_up(incl, off, kWave);
    if (lane >= off) incl = max(incl, o);
  }
  if (lane == kWave - 1) wmax[wave] = incl;
  __syncthreads();
  int32_t before = __shfl_up(incl, 1, kWave);
  if (lane == 0) before = -1;
  for (int w = 0; w < wave; w++) before = max(before, wmax[w]);
#pragma unroll
  for (int r = 0; r < kEkIpt; r++) rowat[tid * kEkIpt + r] = max(v[r], before);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kEkIpt; r++) {
    const int i = r * kEkBlock + tid;
    if (i < cnt) {
      const int32_t u = rowat[i];
      int32_t w = col[jb + i];
      if (w < 0 || w >= n) {
        flag_err(err, GC_EASYMMETRIC);
        w = u;
      }
      ekeys[jb + i] = ((u64)rank[u] << B) | (u64)rank[w];
    }
  }
}

// col2 from the sorted keys; tpos starts as the identity so that every entry
// holds a valid position even where the CSR lacks a reverse entry.
__global__ void k_split_keys(const u64 *ekeys, int64_t nnz, int B, int32_t *col2, int32_t *tpos) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nnz) {
    col2[p] = (int32_t)(ekeys[p] & ((1ull << B) - 1));
    tpos[p] = (int32_t)p;
  }
}

// lcnt[x] = |L(x)|, ucnt[x] = |U(x)|, ustart[x] = first upper position.
// Also sums |L(x)| over all x (nnz / 2 for a symmetric CSR) and the entries
// the clique pass scans: vertex v reads U(x) for every x in U(v), i.e.
// |L(x)| |U(x)| summed over x.
__global__ __launch_bounds__(kRedBlock) void k_split_rows(const int32_t *rp2, const int32_t *col2,
                                                          int64_t n, int32_t *lcnt, int32_t *ucnt,
                                                          int32_t *ustart, int32_t *max_ucnt,
                                                          u64 *lower_total, u64 *clique_entries) {
  __shared__ int shm[kRedBlock / kWave];
  __shared__ u64 shs[kRedBlock / kWave];
  int mx = 0;
  u64 lsum = 0, ce = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
    const int a = rp2[x], d = rp2[x + 1] - a;
    const int l = lower_bound_dev<int32_t>(col2 + a, d, (int32_t)x);
    lcnt[x] = l;
    ucnt[x] = d - l;
    ustart[x] = a + l;
    mx = max(mx, d - l);
    lsum += (u64)l;
    ce += (u64)l * (u64)(d - l);
  }
  mx = block_reduce(mx, MaxOp(), shm);
  lsum = block_reduce(lsum, AddOp(), shs);
  ce = block_reduce(ce, AddOp(), shs);
  if (threadIdx.x == 0) {
    if (mx) atomicMax(max_ucnt, mx);
    if (lsum) atomicAdd(lower_total, lsum);
    if (ce) atomicAdd(clique_entries, ce);
  }
}

// Twin positions (tpos[p] = position of the reverse entry) by a stable sort
// instead of a search per edge.  Every upper entry p = (x, y), y >= x, gets
// the key (y << 32 | p), written at its place among the upper entries in
// CSR order (uoff: exclusive scan of |U|).  A stable sort on y then lists,
// for each y, the upper entries pointing at y by increasing x: exactly the
// order of the lower part of y's list, so the k-th of them is the twin of
// y's k-th lower entry.  The pass after the sort checks each pairing (the
// key's place lies in y's segment, loff: exclusive scan of |L|, and the
// lower entry's value is the row of p), so a CSR that is not symmetric is
// flagged, as is a self-loop (an upper entry y == x).
__global__ void k_twin_keys(const int32_t *rp2, const int32_t *col2, const int32_t *ustart,
                            const int32_t *uoff, int64_t n, u64 *keys, int32_t *err) {
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int lane = lane_id();
  for (int64_t x = wave; x < n; x += nwaves) {
    const int a = ustart[x], b = rp2[x + 1];
    const int64_t o = (int64_t)uoff[x] - a;
    for (int p = a + lane; p < b; p += kWave) {
      const int32_t y = col2[p];
      if (y == (int32_t)x) flag_err(err, GC_ESELFLOOP);
      keys[o + p] = ((u64)(uint32_t)y << 32) | (u64)(uint32_t)p;
    }
  }
}

// Both twin positions of every pair, and the wedge counts: W[y] = wedges
// y - v - w with v, w below y, the sum over v in L(y) of the length of the
// prefix of N(v) below y, which ends at p (y's own position in N(v)).  The
// keys are sorted by y, so each wave adds the lengths of a run of equal y
// first (a segmented sum by shuffles) and its first lane adds them to W[y]
// (zero on entry).
__global__ void k_twin_pairs(const u64 *sorted, int64_t nup, const int32_t *rp2,
                             const int32_t *col2, const int32_t *lcnt, const int32_t *loff,
                             int64_t n, int64_t nnz, const u64 *lower_total, int32_t *tpos,
                             u64 *W, int32_t *err) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = lane_id();
  int64_t y = -1 - lane;  // a lane without a pair is a segment of its own
  u64 len = 0;
  if (q < nup) {
    if (q == 0 && 2 * *lower_total != (u64)nnz) flag_err(err, GC_EASYMMETRIC);
    const u64 key = sorted[q];
    const int64_t yk = (int64_t)(key >> 32), p = (int64_t)(key & 0xffffffffull);
    bool ok = yk < n && p < nnz;  // else only with a count mismatch (keys left unwritten)
    int64_t k = 0;
    if (ok) {
      k = q - loff[yk];
      ok = k >= 0 && k < lcnt[yk];
    }
    int32_t lo = 0, x = 0;
    if (ok) {
      lo = rp2[yk] + (int32_t)k;
      x = col2[lo];  // y's k-th lower neighbour: the row of p if symmetric
      ok = p >= rp2[x] && p < rp2[x + 1];
    }
    if (ok) {
      tpos[lo] = (int32_t)p;
      tpos[p] = lo;
      y = yk;
      len = (u64)(p - rp2[x]);
    } else {
      flag_err(err, GC_EASYMMETRIC);
    }
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const u64 t = __shfl_down(len, off, kWave);
    const int64_t ty = __shfl_down(y, off, kWave);
    if (lane + off < kWave && ty == y) len += t;
  }
  const int64_t py = __shfl_up(y, 1, kWave);
  if (y >= 0 && (lane == 0 || py != y) && len) atomicAdd(&W[y], len);
}

// Vertex bins: the clique classes by |U(x)|, the 4-cycle classes by W[x].
// A block of kBinsBlock vertices reserves its places in each of the eight
// lists with one atomic per list (per-wave atomics on eight counters
// serialise by the thousand), and a vertex's place is the block's base plus
// the members in lower waves and lower lanes.
constexpr int kBinsBlock = 1024;
constexpr int kBinsLists = 8;

__global__ __launch_bounds__(kBinsBlock) void k_bins(const int32_t *ucnt, const int32_t *lcnt,
                                                     const u64 *W, int64_t n, int32_t *tk0,
                                                     int32_t *tk1, int32_t *tk2, int32_t *tk3,
                                                     int32_t *tk4, int32_t *c4l, int32_t *c4m,
                                                     int32_t *c4h, u64 medium_max,
                                                     Counters *cnt) {
  constexpr int NW = kBinsBlock / kWave;
  __shared__ int32_t off[kBinsLists][NW];
  __shared__ int shm[NW];
  __shared__ u64 shs[NW];
  const int wave = threadIdx.x / kWave, lane = lane_id();
  const int64_t xi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = xi < n;
  const int32_t x = (int32_t)xi;
  const int k = in ? ucnt[x] : 0;
  const u64 w = in ? W[x] : 0;
  const int cls = k >= 2 ? tk_class(k) : -1;
  const bool light = w >= 2 && w <= kLightWedges;  // one wedge cannot close a cycle
  const bool medium = w > kLightWedges && w <= medium_max;
  const bool heavy = w > medium_max && w > kLightWedges;
  // list i: clique class i for i < 5, then light, medium and heavy x
  u64 bal[kBinsLists];
#pragma unroll
  for (int i = 0; i < 5; i++) bal[i] = __ballot(cls == i);
  bal[5] = __ballot(light);
  bal[6] = __ballot(medium);
  bal[7] = __ballot(heavy);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < kBinsLists; i++) off[i][wave] = __popcll(bal[i]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kBinsLists; i++) {
    if ((int)threadIdx.x == i) {
      int sum = 0;
      for (int v = 0; v < NW; v++) {
        const int c = off[i][v];
        off[i][v] = sum;
        sum += c;
      }
      int32_t *ctr = i < 5 ? &cnt->tk_cnt[i] : i == 5 ? &cnt->c4_light : i == 6 ? &cnt->c4_medium
                                                                               : &cnt->c4_heavy;
      const int base = sum ? atomicAdd(ctr, sum) : 0;
      for (int v = 0; v < NW; v++) off[i][v] += base;
    }
  }
  __syncthreads();
  const u64 lt = lanemask_lt();
  if (cls >= 0) {
    int32_t *L = cls == 0 ? tk0 : cls == 1 ? tk1 : cls == 2 ? tk2 : cls == 3 ? tk3 : tk4;
    u64 b = bal[0];
#pragma unroll
    for (int i = 1; i < 5; i++)
      if (cls == i) b = bal[i];
    L[off[cls][wave] + __popcll(b & lt)] = x;
  }
  if (light) c4l[off[5][wave] + __popcll(bal[5] & lt)] = x;
  if (medium) c4m[off[6][wave] + __popcll(bal[6] & lt)] = x;
  if (heavy) c4h[off[7][wave] + __popcll(bal[7] & lt)] = x;
  const int gs = block_reduce((cls == 3 && k > kTkPeLds) ? 1 : 0, AddOp(), shm);
  const int ml = block_reduce(heavy ? lcnt[x] : 0, MaxOp(), shm);
  const u64 wl = block_reduce(light ? w : 0, AddOp(), shs);
  const u64 wm = block_reduce(medium ? w : 0, AddOp(), shs);
  const u64 wh = block_reduce(heavy ? w : 0, AddOp(), shs);
  if (threadIdx.x == 0) {
    if (gs) atomicAdd(&cnt->tk_pe_global, gs);
    if (ml) atomicMax(&cnt->max_lcnt_heavy, ml);
    if (wl) atomicAdd(&cnt->wedges_light, wl);
    if (wh) atomicAdd(&cnt->wedges_heavy, wh);
    if (wm) atomicAdd(&cnt->wedges_medium, wm);
  }
}

// ------------------------------------------------------------ heavy items

// Sort key: larger work first (32-bit clamped), then list index.
__global__ void k_heavy_keys(const int32_t *c4h, int nh, const u64 *W, u64 *keys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nh) return;
  const u64 w = W[c4h[i]];
  const u64 wc = w > 0xffffffffull ? 0xffffffffull : w;
  keys[i] = ((0xffffffffull - wc) << 32) | (u64)i;
}

__device__ __forceinline__ int chunk_span(int nl) { return nl < 65536 ? 2 * kChunkWords : kChunkWords; }

// Pieces of a heavy vertex.  Wedge endpoints y crowd toward x (the highest
// ranks are the highest degrees), so the y range [0, x) is cut from the top
// in pieces of 1, 1, 2, 4, 8, ... LDS chunks, the last piece taking the rest;
// at most about W / kPieceWork pieces.
__device__ __forceinline__ int64_t piece_top(int64_t k) { return k == 0 ? 0 : (int64_t)1 << (k - 1); }

__device__ int64_t piece_count(u64 w, int64_t nchunks) {
  int64_t S = (int64_t)((w + kPieceWork - 1) / kPieceWork);
  int64_t need = 1;  // pieces until the doubling sizes cover every chunk
  while (piece_top(need) < nchunks) need++;
  if (S > need) S = need;
  if (S < 1) S = 1;
  return S;
}

// Pieces per heavy vertex; the first `skip` (the costliest, counted by the
// dense hub pass instead) get none.
__global__ void k_heavy_pieces(const u64 *sorted, int nh, int skip, const int32_t *c4h,
                               const u64 *W, const int32_t *lcnt, int64_t *pcount) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nh) return;
  if (s < skip) {
    pcount[s] = 0;
    return;
  }
  const int x = c4h[(int)(sorted[s] & 0xffffffffull)];
  const int64_t K = chunk_span(lcnt[x]);
  const int64_t nchunks = ((int64_t)x + K - 1) / K;
  pcount[s] = piece_count(W[x], nchunks);
}

__global__ void k_heavy_expand(const u64 *sorted, int nh, const int32_t *c4h,
                               const int32_t *lcnt, const int64_t *poff, const int64_t *pcount,
                               int4 *items, int64_t *nitems) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nh) return;
  const int x = c4h[(int)(sorted[s] & 0xffffffffull)];
  const int64_t K = chunk_span(lcnt[x]);
  const int64_t nchunks = ((int64_t)x + K - 1) / K;
  const int64_t S = pcount[s], base = poff[s];
  if (s == nh - 1) *nitems = base + S;
  for (int64_t k = 0; k < S; k++) {
    const int64_t hi = nchunks - piece_top(k);
    int64_t lo = k == S - 1 ? 0 : nchunks - piece_top(k + 1);
    if (lo < 0) lo = 0;
    const int ya = (int)(lo * K);
    const int yb = (int)(hi * K < x ? hi * K : x);
    items[base + k] = make_int4(x, ya, yb, 0);
  }
}

// The `cnt` costliest heavy vertices: rank and wedge count.
__global__ void k_heavy_top(const u64 *sorted, int cnt, const int32_t *c4h, const u64 *W,
                            int32_t *xs, u64 *ws) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= cnt) return;
  const int x = c4h[(int)(sorted[s] & 0xffffffffull)];
  xs[s] = x;
  ws[s] = W[x];
}

__global__ void k_max_deg(const int32_t *rp, int64_t n, int32_t *out) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int mx = 0;
  if (u < n) mx = rp[u + 1] - rp[u];
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, __shfl_xor(mx, off, kWave));
  if (lane_id() == 0 && mx) atomicMax(out, mx);
}

// Max over vertices of |U(x)| (neighbours later in the (degree, id) order)
// and sum over vertices of deg(x) |U(x)|, a bound of the wedges x - v - y
// with v, y below x (each v in L(x) adds at most deg(v) of them).  One wave
// per vertex, one atomic per block.
__global__ __launch_bounds__(256) void k_max_ucnt(const int32_t *rp, const int32_t *col, int64_t n,
                                                  int32_t *out, u64 *wsum) {
  __shared__ int32_t smx[256 / kWave];
  __shared__ u64 ssum[256 / kWave];
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int lane = lane_id();
  int mx = 0;
  u64 sum = 0;
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
    mx = max(mx, c);
    sum += (u64)c * (u64)du;
  }
  if (lane == 0) {
    smx[threadIdx.x / kWave] = mx;
    ssum[threadIdx.x / kWave] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256 / kWave; w++) {
      mx = max(mx, smx[w]);
      sum += ssum[w];
    }
    if (mx) atomicMax(out, mx);
    if (sum) atomicAdd(wsum, sum);
  }
}

}  // namespace

int probe_graph(const gc_csr *g, hipStream_t s, int *max_deg, int *max_ucnt, u64 *wedge_bound) {
  *max_deg = 0;
  *max_ucnt = 0;
  *wedge_bound = 0;
  if (g->n == 0 || g->nnz == 0) return GC_OK;
  int32_t *d = nullptr;
  GC_TRY_HIP(hipMallocAsync((void **)&d, 16, s));
  int32_t h[4] = {0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(d, h, 16, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    k_max_deg<<<grid1d(g->n, 256), 256, 0, s>>>(g->row_ptr, g->n, d);
    k_max_ucnt<<<grid1d(g->n * kWave, 256, 2048), 256, 0, s>>>(g->row_ptr, g->col, g->n, d + 1,
                                                               reinterpret_cast<u64 *>(d + 2));
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h, d, 16, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const hipError_t f = hipFreeAsync(d, s);
  if (e == hipSuccess) e = f;
  if (e != hipSuccess) {
    set_error("probe: %s", hipGetErrorString(e));
    return GC_EHIP;
  }
  *max_deg = h[0];
  *max_ucnt = h[1];
  u64 w;
  std::memcpy(&w, h + 2, 8);
  *wedge_bound = w;
  return GC_OK;
}

int launch_validate(const int32_t *rp, const int32_t *col, int64_t n, int64_t nnz, int32_t *err,
                    hipStream_t s) {
  k_check_rowptr_ends<<<1, 64, 0, s>>>(rp, n, nnz, err);
  k_validate<<<grid1d(n, 256, 16384), 256, 0, s>>>(rp, col, n, nnz, err);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

int run_prepass(PrepassArgs &p, Arena &a, hipStream_t s) {
  const int64_t n = p.n, nnz = p.nnz;
  const int B = p.B;
  k_degree_keys<<<grid1d(n, kRedBlock, kRedGrid), kRedBlock, 0, s>>>(p.row_ptr, n, B, p.deg, p.rkeys,
                                                                     &p.cnt->max_deg);
  GC_TRY_HIP(hipGetLastError());
  u64 *rsorted;
  // the keys are made in id order, so a stable sort on the degree bits alone
  // orders them by (degree, id)
  GC_TRY(radix_sort_u64(p.rkeys, p.rkeys_alt, n, bits_for((u64)nnz), &rsorted, a, s, B));
  k_rank<<<grid1d(n, 256), 256, 0, s>>>(rsorted, n, B, p.order, p.rank, p.deg2);
  GC_TRY_HIP(hipGetLastError());
  GC_TRY(scan_exclusive<int32_t>(p.deg2, p.rp2, n, a, s));
  GC_TRY(fill<int32_t>(p.rp2 + n, (int32_t)nnz, 1, s));
  if (nnz > 0) {
    // the ntiles + 1 tile rows live in the sort's second key buffer (nnz
    // words of 8 bytes) until the sort
    const int64_t ntiles = (nnz + kEkTile - 1) / kEkTile;
    int32_t *tilerow = reinterpret_cast<int32_t *>(p.ekeys_alt);
    k_tile_rows<<<grid1d(n, 256), 256, 0, s>>>(p.row_ptr, n, nnz, ntiles, tilerow);
    k_edge_keys<<<(unsigned)ntiles, kEkBlock, 0, s>>>(p.row_ptr, p.col, n, nnz, B, p.rank, tilerow,
                                                      p.ekeys, &p.acc->err);
    GC_TRY_HIP(hipGetLastError());
  }
  GC_TRY(radix_sort_u64(p.ekeys, p.ekeys_alt, nnz, 2 * B, &p.esorted, a, s));
  k_split_keys<<<grid1d(nnz, 256), 256, 0, s>>>(p.esorted, nnz, B, p.col2, p.tpos);
  k_split_rows<<<grid1d(n, kRedBlock, kRedGrid), kRedBlock, 0, s>>>(
      p.rp2, p.col2, n, p.lcnt, p.ucnt, p.ustart, &p.cnt->max_ucnt, &p.cnt->lower_total,
      &p.cnt->clique_entries);
  {
    // twin positions: the upper entries sorted by target (the other edge-key
    // buffer, free after the edge sort, holds the keys and their second
    // buffer; the vertex-key buffers, free after the ranks, the offsets)
    // upper entries if the CSR is symmetric (nnz is even); a CSR with another
    // count is flagged by the count check, and its keys stay inside the
    // buffer (at most nnz upper entries)
    const int64_t nup = nnz / 2;
    int32_t *uoff = reinterpret_cast<int32_t *>(p.rkeys);
    int32_t *loff = reinterpret_cast<int32_t *>(p.rkeys_alt);
    GC_TRY(scan_exclusive<int32_t>(p.ucnt, uoff, n, a, s));
    GC_TRY(scan_exclusive<int32_t>(p.lcnt, loff, n, a, s));
    u64 *tk = p.esorted == p.ekeys ? p.ekeys_alt : p.ekeys;
    k_twin_keys<<<grid1d(n * kWave, 256, 65536), 256, 0, s>>>(p.rp2, p.col2, p.ustart, uoff, n, tk,
                                                             &p.acc->err);
    GC_TRY_HIP(hipGetLastError());
    u64 *tsorted;
    GC_TRY(radix_sort_u64(tk, tk + nup, nup, B, &tsorted, a, s, 32));
    k_twin_pairs<<<grid1d(nup, 256), 256, 0, s>>>(tsorted, nup, p.rp2, p.col2, p.lcnt, loff, n,
                                                 nnz, &p.cnt->lower_total, p.tpos, p.W,
                                                 &p.acc->err);
  }
  k_bins<<<grid1d(n, kBinsBlock), kBinsBlock, 0, s>>>(p.ucnt, p.lcnt, p.W, n, p.tk[0], p.tk[1],
                                                      p.tk[2], p.tk[3], p.tk[4], p.c4l, p.c4m,
                                                      p.c4h, p.medium_max, p.cnt);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

void measure_heavy_items(int nheavy, Arena &a) {
  size_t m0 = a.mark();
  u64 *dummy;
  (void)radix_sort_u64(nullptr, nullptr, nheavy, 64, &dummy, a, nullptr);
  (void)scan_exclusive<int64_t>(nullptr, nullptr, nheavy, a, nullptr);
  a.release(m0);
}

int sort_heavy(const PrepassArgs &p, int nh, u64 *keys, u64 *keys_alt, u64 **sorted, Arena &a,
               hipStream_t s) {
  *sorted = keys;
  if (nh <= 0) return GC_OK;
  k_heavy_keys<<<grid1d(nh, 256), 256, 0, s>>>(p.c4h, nh, p.W, keys);
  GC_TRY_HIP(hipGetLastError());
  // the key's high half is the order; the low half (the list index) is the
  // input order, which a stable sort keeps for equal costs
  GC_TRY(radix_sort_u64(keys, keys_alt, nh, 32, sorted, a, s, 32));
  return GC_OK;
}

int heavy_top(const PrepassArgs &p, const u64 *sorted, int cnt, int32_t *xs, u64 *ws,
              hipStream_t s) {
  if (cnt <= 0) return GC_OK;
  k_heavy_top<<<grid1d(cnt, 256), 256, 0, s>>>(sorted, cnt, p.c4h, p.W, xs, ws);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

int expand_heavy_items(const PrepassArgs &p, int nh, int skip, const u64 *sorted, u64 *spare,
                       int4 *items, int64_t *pcount, Arena &a, hipStream_t s) {
  if (nh <= 0) return GC_OK;
  k_heavy_pieces<<<grid1d(nh, 256), 256, 0, s>>>(sorted, nh, skip, p.c4h, p.W, p.lcnt, pcount);
  GC_TRY_HIP(hipGetLastError());
  int64_t *poff = reinterpret_cast<int64_t *>(spare);
  GC_TRY(scan_exclusive<int64_t>(pcount, poff, nh, a, s));
  k_heavy_expand<<<grid1d(nh, 256), 256, 0, s>>>(sorted, nh, p.c4h, p.lcnt, poff, pcount, items,
                                                 &p.acc->nitems);
  GC_TRY_HIP(hipGetLastError());
  return GC_OK;
}

}  // namespace gc
