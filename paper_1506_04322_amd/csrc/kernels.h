// Internal interfaces between the host pipeline and the kernel files of the
// single-graph path (not part of the ABI).
#pragma once

#include "common.h"

namespace gc {

// ---------------------------------------------------------------- constants

// Step-3 accumulators (unrestricted counts of Section 4.2, summed over edges).
constexpr int kAcc = 13;
enum AccIdx {
  A_T = 0,  // sum |Tri_e|
  A_S,      // sum |Star_u| + |Star_v|
  A_I,      // sum I_e = |V| - |N(u) u N(v)|
  A_TT,     // sum C(T, 2)                      N_{T,T}
  A_SUSV,   // sum Su Sv                        N_{Su,Sv}
  A_TS,     // sum T (Su + Sv)                  N_{T,Su v Sv}
  A_SS,     // sum C(Su,2) + C(Sv,2)            N_{S.,S.}
  A_TI,     // sum T I                          N_{T,I}
  A_SI,     // sum (Su + Sv) I                  N_{Su v Sv,I}
  A_II,     // sum C(I, 2)                      N_{I,I}
  A_II1,    // sum |E| - d_u - d_v + 1           (N_{I,I,1} before its subtractions)
  A_K4,     // sum 4-cliques through e           N_{T,T,1}
  A_C4      // sum induced 4-cycles through e    N_{Su,Sv,1}
};

// Size classes of the clique pass by k = |U(u)|.
constexpr int kTkBins = 5;
constexpr int kTkLim0 = 64, kTkLim1 = 256, kTkLim2 = 512, kTkLim3 = 1088;
// Largest k of the per-edge 1024-thread class whose symmetric rows stay in
// LDS; the class's larger vertices keep their rows in a global slot.
constexpr int kTkPeLds = 896;
static_assert(kTkLim2 < kTkPeLds && kTkPeLds < kTkLim3, "splits the 1024-thread class");
// Class of a vertex with k = |U(u)| >= 2 upper neighbours.
__host__ __device__ inline int tk_class(int k) {
  return k <= kTkLim0 ? 0 : k <= kTkLim1 ? 1 : k <= kTkLim2 ? 2 : k <= kTkLim3 ? 3 : 4;
}
// Light wedge vertices: at most this many wedges (LDS hash of <= 2048 slots).
constexpr u64 kLightWedges = 1024;
constexpr int kHashSlots = 2048;
// Medium wedge vertices: one workgroup, LDS hash of
// kMediumSlots slots (int32 key, 16-bit count) at load factor < 3/4.
constexpr u64 kMediumWedges = 16384;
constexpr int kMediumSlots = 22528;
constexpr int kMediumBlock = 1024;
// Heavy wedge vertices: LDS counter chunk of 128 KiB.
constexpr int kChunkWords = 32768;
// Per-edge mode: 112 KiB, leaving room for the run queue's four arrays.
constexpr int kChunkWordsPE = 28672;
constexpr int kC4HeavyBlock = 1024;
// Heavy items (global mode) of vertices with at most this many lower
// neighbours keep every list's cursor in registers (up to three lists per
// thread); long runs are queued for whole waves, in a queue with a slot per
// list.  Vertices with more lists walk them in groups of two per thread,
// cursors kept in global memory between groups.
constexpr int kWalkLists = 3 * kC4HeavyBlock;
constexpr int kWalkListsPE = 2 * kC4HeavyBlock;  // per-edge mode: two lists per thread
// Target wedges per heavy work item.
constexpr u64 kPieceWork = u64(1) << 21;
// Concurrent workgroups of the global-memory clique kernel.
constexpr int kTkGlobalSlots = 256;

// Device accumulators and scalars (u64 words; filled with zero per call).
struct DevAcc {
  u64 k4;       // number of 4-cliques (global mode)
  u64 k4_hi;
  u64 k4x3;     // 3 x 4-cliques (fallback kernel counts each clique 3 times)
  u64 k4x3_hi;
  u64 c4ni;     // number of 4-cycles, chords allowed
  u64 c4ni_hi;
  u64 step3[kAcc][2];
  int32_t err;  // contract violations (bit -code per kind)
  int32_t pad;
  u64 queue;    // persistent work-queue heads
  u64 queue2;
  int64_t nitems;  // heavy wedge work items
};

struct Counters {
  int32_t tk_cnt[kTkBins];
  int32_t c4_light;
  int32_t c4_heavy;
  int32_t max_ucnt;
  int32_t max_lcnt_heavy;
  int32_t max_deg;
  int32_t c4_medium;
  int32_t tk_pe_global;  // vertices with kTkPeLds < k <= kTkLim3
  int32_t pad[4];
  u64 wedges_light;
  u64 wedges_heavy;
  u64 clique_entries;
  u64 wedges_medium;
  u64 lower_total;  // sum of |L(x)|: nnz / 2 for a symmetric CSR
};

__device__ __forceinline__ void flag_err(int32_t *err, int code) { atomicOr(err, 1 << (-code)); }

// Blocks for n items of one thread each.  A cap is for kernels that loop
// over their items; without one the grid covers every item, as the
// one-thread-per-item kernels need (n < 2^31 keeps the grid below 2^32
// work-items).
inline unsigned grid1d(int64_t n, int block, int64_t cap = INT64_MAX) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ---------------------------------------------------------------- prepass

struct PrepassArgs {
  const int32_t *row_ptr, *col;  // caller's CSR
  int64_t n, nnz;
  int B;                          // bits of a vertex id
  DevAcc *acc;
  Counters *cnt;
  // outputs
  int32_t *deg, *order, *rank, *deg2, *rp2, *col2, *lcnt, *ucnt, *ustart, *tpos;
  u64 *rkeys, *rkeys_alt, *ekeys, *ekeys_alt, *W;
  int32_t *tk[kTkBins], *c4l, *c4m, *c4h;
  u64 medium_max;  // wedges of the largest medium vertex (= light limit: no medium class)
  u64 *esorted;    // set by the prepass: sorted (row << B | col) keys
};

// Maximum degree, maximum |U(x)| and sum of deg(x) |U(x)| (a bound of the
// wedges x - v - y with v, y below x) of a caller CSR (one sync on s).
int probe_graph(const gc_csr *g, hipStream_t s, int *max_deg, int *max_ucnt, u64 *wedge_bound);
int launch_validate(const int32_t *rp, const int32_t *col, int64_t n, int64_t nnz, int32_t *err,
                    hipStream_t s);
int run_prepass(PrepassArgs &p, Arena &a, hipStream_t s);
// Heavy wedge items (x, y_begin, y_end), largest first, built on the device.
// Heavy wedge vertices sorted costliest first (keys: wedge count descending).
int sort_heavy(const PrepassArgs &p, int nheavy, u64 *keys, u64 *keys_alt, u64 **sorted,
               Arena &a, hipStream_t s);
// Rank and wedge count of the first `cnt` sorted heavy vertices.
int heavy_top(const PrepassArgs &p, const u64 *sorted, int cnt, int32_t *xs, u64 *ws,
              hipStream_t s);
// Work items (x, y range) of the sorted heavy vertices after the first `skip`;
// `spare` is the other radix buffer (nheavy u64).
int expand_heavy_items(const PrepassArgs &p, int nheavy, int skip, const u64 *sorted, u64 *spare,
                       int4 *items, int64_t *pcount, Arena &a, hipStream_t s);
void measure_heavy_items(int nheavy, Arena &a);

// ---------------------------------------------------------------- cliques

struct TkArgs {
  const int32_t *col2;
  const int32_t *ustart;
  const int32_t *ucnt;
  const int32_t *list;
  int nlist;
  uint32_t *T;  // |Tri| per upper position
  u64 *K4w;     // per-edge pass: 4-cliques per upper position
  u64 *Dw;      // per-edge pass: D_e per upper position
  u64 *Bw;      // per-edge pass (local vectors): sum of deg(w) over w in Tri_e, or null
  const int32_t *deg2;  // degree by rank
  u64 *k4;      // global mode: number of 4-cliques (128-bit); null in per-edge mode
  u64 *k4x3;    // fallback kernel: 3 x 4-cliques (128-bit)
  // global storage of the fallback kernel, per workgroup slot
  u64 *gR;
  int32_t *gI;
  u64 *gA;
  int kmax;
};

// Launches the clique pass for one size class.
int launch_cliques(TkArgs g, int bin, bool per_edge, hipStream_t s);
// Whether a class needs the global-memory scratch in the given mode.
inline bool cliques_need_global(int bin, bool per_edge) { return bin == 4 || (per_edge && bin == 3); }

// ---------------------------------------------------------------- cycles

struct C4Args {
  const int32_t *col2;
  const int32_t *rp2;
  const int32_t *lcnt;
  const int32_t *tpos;
  const u64 *W;
  const int32_t *list;
  int nlist;
  u64 *c4ni;  // total (128-bit)
  u64 *C4w;   // per-edge pass: 4-cycles (chords allowed) per edge, credited at
              // either directed entry until folded into the upper position
  const int4 *items;  // (x, y_begin, y_end, -)
  const int64_t *nitems;
  u64 *queue;
  int32_t *gcur;  // per slot: cursor per lower neighbour (items of many lists)
  int32_t *gbeg;  // per slot: end of each list
  int32_t *gcb;   // per slot (per-edge): run start of each list in the chunk
  int lmax;
  const int32_t *deg2;  // degree of each rank (non-decreasing)
  int64_t n;
  // Per-edge mode: the heavy wedges' credits per directed entry in 32 bits
  // (nnz + 2 entries, folded into C4w), or null: into C4w.  Used when the
  // maximum degree is at most kC4hMaxDeg: an entry (v, y) gains at most
  // c(x, y) - 1 < deg(y) from each of the fewer than deg(v) vertices x.
  uint32_t *C4h;
};
constexpr int kC4hMaxDeg = 65535;

// Dense hub slabs (global mode).  The costliest heavy vertices are counted
// kDenseSlab at a time: every vertex v gets a mask whose bit k says that v is
// a lower neighbour of hub k, and one pass over all rows y sums, per hub, the
// mask bits of y's neighbours, which is c(x_k, y).
constexpr int kDenseSlab = 256;        // hubs per slab
constexpr int kDenseWords = kDenseSlab / 64;  // mask words per vertex
constexpr int kDenseHubMax = 8192;     // candidates examined by the host
constexpr int kDenseShortDeg = 1023;   // rows up to this degree: one thread, 10 bit planes
// Cost model of the route (picoseconds), measured on R-MAT s22: a slab pass
// reads every adjacency entry and gathers one mask per entry (2.63 ms for
// 1.28e8 entries, about 20 us of it its four launches); a heavy wedge by work
// items costs 2.84 ps.
constexpr double kDenseSlabFixedPs = 2.0e7;
constexpr double kDenseSlabEntryPs = 20.3;
constexpr double kSparseWedgePs = 2.84;
struct HubArgs {
  const int32_t *rp2, *col2, *lcnt;
  int64_t n;
  u64 *mask;          // 2 words per vertex, zero between slabs
  const int32_t *xs;  // the slab's hubs, ranks descending
  int nslab;
  u64 *c4ni;          // total (128-bit)
};
int launch_dense_slab(const HubArgs &g, hipStream_t s);

int launch_cycles_light(C4Args g, bool per_edge, hipStream_t s);
int launch_cycles_medium(C4Args g, bool per_edge, hipStream_t s);
// Per-edge mode: adds each edge's lower directed entry of C4w, and both
// entries of C4h (if not null), into its upper position of C4w.
int launch_c4_fold(const u64 *ekeys, const int32_t *col2, const int32_t *tpos, int64_t nnz, int B,
                   u64 *C4w, const uint32_t *C4h, hipStream_t s);
int launch_cycles_heavy(C4Args g, int slots, bool per_edge, hipStream_t s);

// ---------------------------------------------------------------- Step 3

struct S3Args {
  const u64 *ekeys;
  const int32_t *col2;
  const int32_t *deg2;
  const uint32_t *T;
  const u64 *K4w, *C4w, *Dw;  // per-edge mode only
  int64_t nnz, n, m;
  int B;
  u64 *partials;  // [grid][kAcc][2]
  DevAcc *acc;
  const int32_t *order;
  const int32_t *rp;
  const int32_t *col;
  const int64_t *cu;
  int64_t *out;  // [3][m], or null
  // local vectors (or null): sum of deg over Tri_e per upper position, and
  // per vertex (by rank) twice the triangle count and the sum of neighbour
  // degrees
  const u64 *Bw, *tv, *sv;
  int64_t *local;  // [kLocal][m]
};

constexpr int kLocal = 17;
// Per vertex by rank: tv = sum of T_e over incident edges (twice its
// triangles), sv = sum of the neighbours' degrees.
int launch_vertex_sums(const int32_t *rp2, const int32_t *col2, const int32_t *lcnt,
                       const int32_t *tpos, const uint32_t *T, const int32_t *deg2, int64_t n,
                       u64 *tv, u64 *sv, hipStream_t s);

// Per-vertex counts from the per-edge arrays of the local-vector pass.
struct VxArgs {
  const int32_t *rp2, *col2, *lcnt, *tpos, *deg2, *order;
  const uint32_t *T;
  const u64 *K4w, *C4w, *Dw, *Bw, *tv, *sv;
  int64_t n, m;
  u64 tri, star;  // global triangles and induced 2-stars, modulo 2^64
  u64 *out;       // [17][n] by the caller's vertex id
};
int launch_vertex_counts(const VxArgs &g, hipStream_t s);

constexpr int kStep3Grid = 2048;
int launch_step3(S3Args g, int grid, bool per_edge, hipStream_t s);
int launch_orig_upper(const int32_t *rp, const int32_t *col, int64_t n, int64_t *up,
                      hipStream_t s);

}  // namespace gc
