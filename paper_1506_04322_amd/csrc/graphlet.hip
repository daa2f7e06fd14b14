// Per-edge graphlet decomposition (k = 2, 3, 4) of one graph on an MI355X:
// host side of graphlet_count.
//
// The method (Ahmed et al., arXiv 1506.04322, Sections 3-4): for every edge
// e = (u, v) find Tri_e, Star_u, Star_v (Step 1), count the 4-cliques and
// induced 4-cycles containing e (Step 2), accumulate the unrestricted counts
// of Equations "comb_n_ai_ai"/"comb_n_ai_aj" (Step 3), and derive all 17
// counts with the Lemmas of Section 4.3 and Equations "g_4_9", "g_4_11"
// (Step 4).  The kernels: prepass.hip (degree order), cliques.hip (Steps 1
// and 2a), cycles.hip (Step 2b), step3.hip (Step 3); Step 4 is below.
//
// Workspace: a fixed part sized by n and nnz, and a part sized after the
// prepass from the actual maxima (per-workgroup state of the kernels that
// keep it in global memory, heavy work items).  graphlet_workspace_size
// bounds both from two cheap device reductions.
#include <algorithm>
#include <cmath>
#include <functional>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"
#include "primitives.h"

namespace gc {

namespace {
thread_local std::string t_err;
thread_local bool t_timing = false;
thread_local gc_timing t_last_timing;
}  // namespace

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

struct Plan {
  int64_t n = 0, nnz = 0, m = 0;
  int B = 1;
  bool per_edge = false;
  bool local = false;  // per-edge local 4-node vectors (implies per_edge)
  uint32_t flags = 0;
};

struct Fixed {
  PrepassArgs pp;
  uint32_t *T;
  u64 *K4w, *C4w, *Dw;
  uint32_t *C4h;      // per-edge: heavy wedge credits, 32 bits per entry
  u64 *Bw, *tv, *sv;  // local vectors only
  int64_t *cu;
  u64 *partials;
  int nstep3;
};

void alloc_fixed(Arena &a, const Plan &P, Fixed &f) {
  const int64_t n = P.n, nnz = P.nnz;
  PrepassArgs &p = f.pp;
  p.acc = a.take<DevAcc>(1);
  p.cnt = a.take<Counters>(1);
  p.deg = a.take<int32_t>(n);
  p.order = a.take<int32_t>(n);
  p.rank = a.take<int32_t>(n);
  p.deg2 = a.take<int32_t>(n);
  p.rp2 = a.take<int32_t>(n + 1);
  p.lcnt = a.take<int32_t>(n);
  p.ucnt = a.take<int32_t>(n);
  p.ustart = a.take<int32_t>(n);
  p.W = a.take<u64>(n);
  p.rkeys = a.take<u64>(n);
  p.rkeys_alt = a.take<u64>(n);
  p.ekeys = a.take<u64>(nnz);
  p.ekeys_alt = a.take<u64>(nnz);
  p.col2 = a.take<int32_t>(nnz);
  p.tpos = a.take<int32_t>(nnz);
  for (int i = 0; i < kTkBins; i++) p.tk[i] = a.take<int32_t>(n);
  p.c4l = a.take<int32_t>(n);
  p.c4m = a.take<int32_t>(n);
  p.c4h = a.take<int32_t>(n);
  p.medium_max = kMediumWedges;
  f.T = a.take<uint32_t>(nnz);
  f.nstep3 = (int)std::min<int64_t>(kStep3Grid, std::max<int64_t>(1, (nnz + 255) / 256));
  f.partials = a.take<u64>((size_t)f.nstep3 * kAcc * 2);
  if (P.per_edge) {
    f.K4w = a.take<u64>(nnz);
    f.C4w = a.take<u64>(nnz);
    f.Dw = a.take<u64>(nnz);
    f.C4h = a.take<uint32_t>(nnz + 2);
    f.cu = a.take<int64_t>(n + 1);
  } else {
    f.K4w = f.C4w = f.Dw = nullptr;
    f.C4h = nullptr;
    f.cu = nullptr;
  }
  if (P.local) {
    f.Bw = a.take<u64>(nnz);
    f.tv = a.take<u64>(n);
    f.sv = a.take<u64>(n);
  } else {
    f.Bw = f.tv = f.sv = nullptr;
  }
  // temporaries of the prepass sorts and scans, measured only (the real run
  // takes and releases them inside the sort and scan calls)
  if (a.measuring()) {
    const size_t m0 = a.mark();
    u64 *dummy;
    (void)radix_sort_u64(nullptr, nullptr, std::max(P.nnz, P.n), 64, &dummy, a, nullptr);
    a.release(m0);
    (void)scan_exclusive<int64_t>(nullptr, nullptr, P.n + 1, a, nullptr);
    a.release(m0);
  }
}

// Sizes of the state allotted after the prepass.
struct DynNeed {
  int kmax_global = 0;  // |U(u)| bound of the global-memory clique kernel, 0 = unused
  int lmax = 0;         // max |L(x)| of heavy wedge vertices
  int slots = 0;        // heavy wedge workgroups
  int nheavy = 0;
  int64_t items_cap = 0;
};

struct Dyn {
  u64 *gR;
  int32_t *gI;
  u64 *gA;
  int32_t *gcur, *gbeg, *gcb;
  int4 *items;
  u64 *hkeys, *hkeys_alt;
  int64_t *pcount;
  u64 *hubmask;     // dense hub slabs: kDenseWords mask words per vertex (global mode)
  int32_t *hubs;    // dense hubs, slab by slab, ranks descending in a slab
  u64 *hubw;        // wedge counts of the candidate hubs
};

void alloc_dyn(Arena &a, const Plan &P, const DynNeed &d, Dyn &y) {
  const size_t km = (size_t)d.kmax_global, wm = (km + 63) / 64;
  y.gR = km ? a.take<u64>((size_t)kTkGlobalSlots * km * wm) : nullptr;
  y.gI = km ? a.take<int32_t>((size_t)kTkGlobalSlots * (3 * km + 1)) : nullptr;
  y.gA = km ? a.take<u64>((size_t)kTkGlobalSlots * 3 * km) : nullptr;
  const size_t lm = (size_t)std::max(d.lmax, 1), sl = (size_t)std::max(d.slots, 1);
  y.gcur = a.take<int32_t>(sl * lm);
  y.gbeg = a.take<int32_t>(sl * lm);
  y.gcb = P.per_edge ? a.take<int32_t>(sl * lm) : nullptr;
  y.items = a.take<int4>((size_t)std::max<int64_t>(d.items_cap, 1));
  const size_t nh = (size_t)std::max(d.nheavy, 1);
  y.hkeys = a.take<u64>(nh);
  y.hkeys_alt = a.take<u64>(nh);
  y.pcount = a.take<int64_t>(nh);
  const bool dense = !P.per_edge && d.nheavy > 0;
  y.hubmask = dense ? a.take<u64>(kDenseWords * (size_t)P.n) : nullptr;
  y.hubs = dense ? a.take<int32_t>(kDenseHubMax) : nullptr;
  y.hubw = dense ? a.take<u64>(kDenseHubMax) : nullptr;
  if (a.measuring()) {
    measure_heavy_items(d.nheavy, a);
    if (P.per_edge) {  // scan of the canonical edge offsets
      const size_t m0 = a.mark();
      (void)scan_exclusive<int64_t>(nullptr, nullptr, P.n + 1, a, nullptr);
      a.release(m0);
    }
  }
}

int device_cus() {
  static int cached = 0;
  if (!cached) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
        prop.multiProcessorCount > 0)
      cached = prop.multiProcessorCount;
    else
      cached = 256;
  }
  return cached;
}

DynNeed dyn_need(const Plan &P, const Counters &hc) {
  DynNeed d;
  const bool global_tk = hc.tk_cnt[4] > 0 || (P.per_edge && hc.tk_cnt[3] > 0);
  d.kmax_global = global_tk ? hc.max_ucnt : 0;
  d.nheavy = hc.c4_heavy;
  d.lmax = hc.max_lcnt_heavy;
  d.items_cap = (int64_t)hc.c4_heavy + (int64_t)(hc.wedges_heavy / kPieceWork) + 1;
  d.slots = (int)std::min<int64_t>(device_cus(), std::max<int64_t>(d.items_cap, 1));
  return d;
}

// Upper bound of dyn_need before the prepass (workspace size query);
// wedge_bound bounds the wedges of all vertices (sum of deg(x) |U(x)|).
DynNeed dyn_bound(const Plan &P, int max_deg, int max_ucnt, u64 wedge_bound) {
  DynNeed d;
  const bool global_tk = max_ucnt > kTkLim3 || (P.per_edge && max_ucnt > kTkLim2);
  d.kmax_global = global_tk ? max_ucnt : 0;
  d.nheavy = (int)P.n;
  d.lmax = max_deg;
  // sum of wedges <= sum_v d_v |U(v)| <= nnz * max |U|
  const u64 wedges = std::min((u64)P.nnz * (u64)std::max(max_ucnt, 1), wedge_bound);
  d.items_cap = P.n + (int64_t)(wedges / kPieceWork) + 1;
  d.slots = device_cus();
  return d;
}

// ------------------------------------------------------------------ Step 4

inline u128 choose_h(u128 n, int k) {
  if (n < (u128)k) return 0;
  u128 r = 1;
  for (int i = 0; i < k; i++) r = r * (n - i) / (u128)(i + 1);
  return r;
}

inline bool exact_div(i128 a, int d, i128 *q) {
  if (a % d != 0) return false;
  *q = a / d;
  return true;
}

// The 17 counts from the summed per-edge quantities (all 128-bit).
int finalize(const u128 A[kAcc], int64_t n_, int64_t m_, gc_u128 out[17]) {
  const i128 n = (i128)n_, m = (i128)m_;
  i128 g[17];
  i128 t;
  g[0] = m;                                                 // g2_1
  g[1] = (i128)choose_h((u128)n, 2) - m;                    // g2_2
  if (!exact_div((i128)A[A_T], 3, &g[2])) goto bad;         // Eq. "triangle"
  if (!exact_div((i128)A[A_S], 2, &g[3])) goto bad;         // Eq. "2-star"
  g[4] = (i128)A[A_I];                                      // Eq. "g3_3"
  g[5] = (i128)choose_h((u128)n, 3) - g[2] - g[3] - g[4];   // Eq. "g3_4"
  if (!exact_div((i128)A[A_K4], 6, &g[6])) goto bad;        // Cor. "cliq": 6 edges each
  if (!exact_div((i128)A[A_C4], 4, &g[9])) goto bad;        // Cor. "cyc": 4 edges each
  g[7] = (i128)A[A_TT] - 6 * g[6];                          // Lemma "rel-cliq-chcy"
  g[11] = (i128)A[A_SUSV] - 4 * g[9];                       // Lemma "rel-cyc-path"
  if (!exact_div((i128)A[A_TS] - 4 * g[7], 2, &g[8])) goto bad;    // Lemma "rel-ttri-chcy2"
  if (!exact_div((i128)A[A_SS] - g[8], 3, &g[10])) goto bad;       // Lemma "rel-ttri-3star"
  if (!exact_div((i128)A[A_TI] - g[8], 3, &g[12])) goto bad;       // Lemma "rel-4node-tri-ttri"
  if (!exact_div((i128)A[A_SI] - 2 * g[11], 2, &g[13])) goto bad;  // Lemma "rel-4node-2star-path"
  t = (i128)A[A_II1] - (6 * g[6] + 4 * g[7] + 2 * g[8]) - (4 * g[9] + 2 * g[11]);
  if (!exact_div(t, 2, &g[14])) goto bad;                   // Eq. "g_4_9"
  g[15] = (i128)A[A_II] - 2 * g[14];                        // Lemma "rel-4node-2edge-1edge"
  t = 0;
  for (int i = 6; i <= 15; i++) t += g[i];
  g[16] = (i128)choose_h((u128)n, 4) - t;                   // Eq. "g_4_11"
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

// Counts of a graph with no edges: only the independent classes.
void counts_no_edges(int64_t n, gc_u128 out[17]) {
  memset(out, 0, sizeof(gc_u128) * 17);
  const u128 c2 = choose_h((u128)n, 2), c3 = choose_h((u128)n, 3), c4 = choose_h((u128)n, 4);
  out[1] = {(uint64_t)c2, (uint64_t)(c2 >> 64)};
  out[5] = {(uint64_t)c3, (uint64_t)(c3 >> 64)};
  out[16] = {(uint64_t)c4, (uint64_t)(c4 >> 64)};
}

// ------------------------------------------------------------------ timing

struct PhaseEvents {
  static constexpr int kN = 11;  // 0..8 the counting phases, 9..10 per-vertex counts
  hipEvent_t e[kN] = {};
  bool on = false;
  int init(hipStream_t s) {
    on = t_timing;
    if (!on) return GC_OK;
    for (int i = 0; i < kN; i++) GC_TRY_HIP(hipEventCreate(&e[i]));
    for (int i = 0; i < kN; i++) record(i, s);  // every event valid even if a phase is empty
    return GC_OK;
  }
  void record(int i, hipStream_t s) {
    if (on) (void)hipEventRecord(e[i], s);
  }
  float span(int a, int b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e[a], e[b]) != hipSuccess) return 0.f;
    return ms;
  }
  ~PhaseEvents() {
    if (on)
      for (int i = 0; i < kN; i++)
        if (e[i]) (void)hipEventDestroy(e[i]);
  }
};

// Device memory the library allocated for one call; freed stream-ordered.
struct Owned {
  std::vector<void *> ptrs;
  hipStream_t s = nullptr;
  int alloc(size_t bytes, char **out) {
    void *p = nullptr;
    hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess) {
      set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
      return GC_ENOMEM;
    }
    ptrs.push_back(p);
    *out = reinterpret_cast<char *>(p);
    return GC_OK;
  }
  ~Owned() {
    for (void *p : ptrs) (void)hipFreeAsync(p, s);
    if (!ptrs.empty()) (void)hipStreamSynchronize(s);
  }
};

inline char *align256(char *p) {
  return reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(p) + 255) & ~uintptr_t(255));
}

// ------------------------------------------------------------------ pipeline

int run(const gc_csr *G, gc_u128 out17[17], int64_t *per_edge_out, int64_t *local_out,
        u64 *vertex_out, char *ws, size_t ws_bytes, hipStream_t s, const Plan &P) {
  const int64_t n = P.n, nnz = P.nnz, m = P.m;
  Owned owned;
  owned.s = s;
  // fixed part
  Fixed f;
  Arena a;
  {
    Arena meas;
    alloc_fixed(meas, P, f);
    const size_t need = meas.peak + 256;
    if (ws) {
      if (ws_bytes < need) {
        set_error("workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
        return GC_ENOMEM;
      }
      a.base = align256(ws);
      a.cap = ws_bytes - (size_t)(a.base - ws);
    } else {
      char *p;
      GC_TRY(owned.alloc(need, &p));
      a.base = align256(p);
      a.cap = need - (size_t)(a.base - p);
    }
    alloc_fixed(a, P, f);
    if (a.overflow) {
      set_error("workspace too small");
      return GC_ENOMEM;
    }
  }
  PrepassArgs &pp = f.pp;
  pp.row_ptr = G->row_ptr;
  pp.col = G->col;
  pp.n = n;
  pp.nnz = nnz;
  pp.B = P.B;

  GC_TRY(fill<u64>(reinterpret_cast<u64 *>(pp.acc), 0ull, sizeof(DevAcc) / 8, s));
  GC_TRY(fill<int32_t>(reinterpret_cast<int32_t *>(pp.cnt), 0, sizeof(Counters) / 4, s));
  GC_TRY(fill<u64>(pp.W, 0ull, n, s));
  GC_TRY(fill<uint32_t>(f.T, 0u, nnz, s));
  if (P.per_edge) {
    GC_TRY(fill<u64>(f.K4w, 0ull, nnz, s));
    GC_TRY(fill<u64>(f.C4w, 0ull, nnz, s));
    GC_TRY(fill<u64>(f.Dw, 0ull, nnz, s));
    GC_TRY(fill<uint32_t>(f.C4h, 0u, nnz + 2, s));
    if (P.local) {
      GC_TRY(fill<u64>(f.Bw, 0ull, nnz, s));
      GC_TRY(fill<u64>(f.tv, 0ull, n, s));
      GC_TRY(fill<u64>(f.sv, 0ull, n, s));
    }
  }
  PhaseEvents ev;
  GC_TRY(ev.init(s));

  // -- prepass
  ev.record(0, s);
  GC_TRY(run_prepass(pp, a, s));
  ev.record(1, s);
  Counters hc;
  int32_t perr = 0;
  GC_TRY_HIP(hipMemcpyAsync(&hc, pp.cnt, sizeof hc, hipMemcpyDeviceToHost, s));
  GC_TRY_HIP(hipMemcpyAsync(&perr, &pp.acc->err, 4, hipMemcpyDeviceToHost, s));
  GC_TRY_HIP(hipStreamSynchronize(s));
  if (perr != 0) {
    const int code = -(__builtin_ffs(perr) - 1);
    set_error("CSR contract violated (code %d); run with GC_VALIDATE for details", code);
    return code;
  }

  // -- state sized by the prepass
  const DynNeed dn = dyn_need(P, hc);
  Dyn dy;
  Arena da;
  {
    Arena meas;
    alloc_dyn(meas, P, dn, dy);
    const size_t need = meas.peak + 256;
    if (ws) {
      da.base = align256(a.base + a.off);
      const size_t used = (size_t)(da.base - ws);
      if (used + need > ws_bytes) {
        set_error("workspace of %zu bytes is smaller than the %zu needed", ws_bytes, used + need);
        return GC_ENOMEM;
      }
      da.cap = ws_bytes - used;
    } else {
      char *p;
      GC_TRY(owned.alloc(need, &p));
      da.base = align256(p);
      da.cap = need - (size_t)(da.base - p);
    }
    alloc_dyn(da, P, dn, dy);
    if (da.overflow) {
      set_error("workspace too small for the per-workgroup state");
      return GC_ENOMEM;
    }
  }
  // Heavy wedge vertices, costliest first; the costliest go to dense hub
  // slabs while a slab's wedges cost more by the item route than one pass.
  u64 *hsorted = nullptr;
  GC_TRY(sort_heavy(pp, dn.nheavy, dy.hkeys, dy.hkeys_alt, &hsorted, da, s));
  int ndense = 0;
  u64 dense_wedges = 0;
  std::vector<int32_t> hubs;
  const bool dense_all = (P.flags & GC_DENSE_ALL) != 0, dense_off = (P.flags & GC_DENSE_OFF) != 0;
  if (dy.hubmask) {
    const int cand = std::min(dn.nheavy, kDenseHubMax);
    std::vector<int32_t> hx(cand);
    std::vector<u64> hw(cand);
    GC_TRY(heavy_top(pp, hsorted, cand, dy.hubs, dy.hubw, s));
    GC_TRY_HIP(hipMemcpyAsync(hx.data(), dy.hubs, sizeof(int32_t) * cand, hipMemcpyDeviceToHost, s));
    GC_TRY_HIP(hipMemcpyAsync(hw.data(), dy.hubw, sizeof(u64) * cand, hipMemcpyDeviceToHost, s));
    GC_TRY_HIP(hipStreamSynchronize(s));
    const double slab_ps = kDenseSlabFixedPs + kDenseSlabEntryPs * (double)nnz;
    for (int b = 0; b < cand; b += kDenseSlab) {
      const int e = std::min(cand, b + kDenseSlab);
      u64 w = 0;
      for (int i = b; i < e; i++) w += hw[i];
      if (dense_off || (!dense_all && (double)w * kSparseWedgePs < slab_ps)) break;
      std::vector<int32_t> slab(hx.begin() + b, hx.begin() + e);
      std::sort(slab.begin(), slab.end(), std::greater<int32_t>());
      hubs.insert(hubs.end(), slab.begin(), slab.end());
      dense_wedges += w;
      ndense = e;
    }
    if (ndense > 0) {
      GC_TRY_HIP(hipMemcpyAsync(dy.hubs, hubs.data(), sizeof(int32_t) * ndense,
                                hipMemcpyHostToDevice, s));
      GC_TRY(fill<u64>(dy.hubmask, 0ull, kDenseWords * n, s));
    }
  }
  GC_TRY(expand_heavy_items(pp, dn.nheavy, ndense, hsorted,
                            hsorted == dy.hkeys ? dy.hkeys_alt : dy.hkeys, dy.items, dy.pcount, da,
                            s));
  if (ndense > 0) GC_TRY_HIP(hipStreamSynchronize(s));  // the host vector goes away later

  // -- Steps 1 + 2a
  ev.record(2, s);
  TkArgs tk{};
  tk.col2 = pp.col2;
  tk.ustart = pp.ustart;
  tk.ucnt = pp.ucnt;
  tk.T = f.T;
  tk.K4w = f.K4w;
  tk.Dw = f.Dw;
  tk.k4 = P.per_edge ? nullptr : &pp.acc->k4;  // per-edge: the K4 totals come from Step 3
  tk.k4x3 = &pp.acc->k4x3;
  tk.gR = dy.gR;
  tk.gI = dy.gI;
  tk.gA = dy.gA;
  tk.kmax = dn.kmax_global;
  tk.deg2 = pp.deg2;
  tk.Bw = nullptr;  // set for the per-edge pass below
  auto cliques = [&](bool per_edge) -> int {
    for (int bin = 0; bin < kTkBins; bin++) {
      tk.list = pp.tk[bin];
      tk.nlist = hc.tk_cnt[bin];
      if (tk.nlist > 0 && cliques_need_global(bin, per_edge) && !tk.gR) {
        set_error("internal: global clique state missing");
        return GC_EINTERNAL;
      }
      GC_TRY(launch_cliques(tk, bin, per_edge, s));
    }
    return GC_OK;
  };
  GC_TRY(cliques(false));
  ev.record(3, s);

  // -- Step 2b
  C4Args c4{};
  c4.col2 = pp.col2;
  c4.rp2 = pp.rp2;
  c4.lcnt = pp.lcnt;
  c4.tpos = pp.tpos;
  c4.W = pp.W;
  c4.deg2 = pp.deg2;
  c4.n = n;
  c4.c4ni = &pp.acc->c4ni;
  c4.C4w = f.C4w;
  c4.list = pp.c4l;
  c4.nlist = hc.c4_light;
  GC_TRY(launch_cycles_light(c4, P.per_edge, s));
  if (hc.c4_medium > 0) {
    C4Args cm = c4;
    cm.list = pp.c4m;
    cm.nlist = hc.c4_medium;
    GC_TRY(launch_cycles_medium(cm, P.per_edge, s));
  }
  ev.record(4, s);
  for (int b = 0; b < ndense; b += kDenseSlab) {
    HubArgs hg{};
    hg.rp2 = pp.rp2;
    hg.col2 = pp.col2;
    hg.lcnt = pp.lcnt;
    hg.n = n;
    hg.mask = dy.hubmask;
    hg.xs = dy.hubs + b;
    hg.nslab = std::min(kDenseSlab, ndense - b);
    hg.c4ni = &pp.acc->c4ni;
    GC_TRY(launch_dense_slab(hg, s));
  }
  ev.record(5, s);
  if (dn.nheavy > 0) {
    c4.items = dy.items;
    c4.nitems = &pp.acc->nitems;
    c4.queue = &pp.acc->queue;
    c4.gcur = dy.gcur;
    c4.gbeg = dy.gbeg;
    c4.gcb = dy.gcb;
    c4.lmax = std::max(dn.lmax, 1);
    // per-edge: 32-bit credits (two entries per atomic) when no sum can overflow
    c4.C4h = hc.max_deg <= kC4hMaxDeg ? f.C4h : nullptr;
    GC_TRY(launch_cycles_heavy(c4, dn.slots, P.per_edge, s));
  }
  if (P.per_edge)
    GC_TRY(launch_c4_fold(pp.esorted, pp.col2, pp.tpos, nnz, P.B, f.C4w, c4.C4h, s));
  ev.record(6, s);

  // -- per-edge 4-cliques and D_e (needs final |Tri|)
  if (P.per_edge) {
    tk.Bw = f.Bw;
    GC_TRY(cliques(true));
  }
  if (P.local)
    GC_TRY(launch_vertex_sums(pp.rp2, pp.col2, pp.lcnt, pp.tpos, f.T, pp.deg2, n, f.tv, f.sv, s));
  ev.record(7, s);

  // -- Step 3
  S3Args s3{};
  s3.ekeys = pp.esorted;
  s3.col2 = pp.col2;
  s3.deg2 = pp.deg2;
  s3.T = f.T;
  s3.K4w = f.K4w;
  s3.C4w = f.C4w;
  s3.Dw = f.Dw;
  s3.nnz = nnz;
  s3.n = n;
  s3.m = m;
  s3.B = P.B;
  s3.partials = f.partials;
  s3.acc = pp.acc;
  if (P.per_edge) {
    GC_TRY(launch_orig_upper(G->row_ptr, G->col, n, f.cu, s));
    GC_TRY(scan_exclusive<int64_t>(f.cu, f.cu, n + 1, da, s));
    s3.order = pp.order;
    s3.rp = G->row_ptr;
    s3.col = G->col;
    s3.cu = f.cu;
    s3.out = per_edge_out;
    s3.local = local_out;
    s3.Bw = f.Bw;
    s3.tv = f.tv;
    s3.sv = f.sv;
  }
  GC_TRY(launch_step3(s3, f.nstep3, P.per_edge, s));
  ev.record(8, s);

  DevAcc h;
  GC_TRY_HIP(hipMemcpyAsync(&h, pp.acc, sizeof h, hipMemcpyDeviceToHost, s));
  GC_TRY_HIP(hipStreamSynchronize(s));
  if (ev.on) {
    gc_timing &t = t_last_timing;
    t.ms[0] = ev.span(0, 1);
    t.ms[1] = ev.span(2, 3);
    t.ms[2] = ev.span(3, 4);
    t.ms[3] = ev.span(4, 5);
    t.ms[4] = ev.span(5, 6);
    t.ms[5] = ev.span(6, 7);
    t.ms[6] = ev.span(7, 8);
    t.ms[7] = 0.0;
    t.clique_entries = hc.clique_entries;
    t.wedges_light = hc.wedges_light + hc.wedges_medium;
    t.wedges_heavy = hc.wedges_heavy - dense_wedges;
    t.heavy_items = h.nitems;
    t.wedges_dense = dense_wedges;
    t.dense_hubs = ndense;
    for (int b = 0; b < kTkBins; b++) t.clique_class[b] = hc.tk_cnt[b];
    t.clique_class[kTkBins] = hc.tk_pe_global;
  }
  u128 A[kAcc];
  for (int i = 0; i < kAcc; i++) A[i] = ((u128)h.step3[i][1] << 64) | h.step3[i][0];
  if (!P.per_edge) {
    // sum_e K4_e = 6 x cliques; sum_e C4_e = 4 C4ni - sum_e D_e + 2 sum_e K4_e
    // with sum_e D_e = 4 sum_e C(T_e, 2): over the three edges of a triangle
    // the D terms add 2 (T_a + T_b + T_c) - 6, and summed over triangles
    // that is 2 sum_e T_e^2 - 6 t = 4 sum_e C(T_e, 2).
    const u128 k4 = ((u128)h.k4_hi << 64) | h.k4;
    const u128 k4x3 = ((u128)h.k4x3_hi << 64) | h.k4x3;
    if (k4x3 % 3 != 0) {
      set_error("internal: clique total not divisible by 3");
      return GC_EINTERNAL;
    }
    const u128 c4ni = ((u128)h.c4ni_hi << 64) | h.c4ni;
    A[A_K4] = 6 * (k4 + k4x3 / 3);
    const i128 c4 = 4 * (i128)c4ni - 4 * (i128)A[A_TT] + 2 * (i128)A[A_K4];
    if (c4 < 0) {
      set_error("internal: negative 4-cycle total");
      return GC_EINTERNAL;
    }
    A[A_C4] = (u128)c4;
  }
  GC_TRY(finalize(A, n, m, out17));
  if (vertex_out) {
    VxArgs vx{};
    vx.rp2 = pp.rp2;
    vx.col2 = pp.col2;
    vx.lcnt = pp.lcnt;
    vx.tpos = pp.tpos;
    vx.deg2 = pp.deg2;
    vx.order = pp.order;
    vx.T = f.T;
    vx.K4w = f.K4w;
    vx.C4w = f.C4w;
    vx.Dw = f.Dw;
    vx.Bw = f.Bw;
    vx.tv = f.tv;
    vx.sv = f.sv;
    vx.n = n;
    vx.m = m;
    vx.tri = out17[2].lo;
    vx.star = out17[3].lo;
    vx.out = vertex_out;
    ev.record(9, s);
    GC_TRY(launch_vertex_counts(vx, s));
    ev.record(10, s);
    GC_TRY_HIP(hipStreamSynchronize(s));
    if (ev.on) t_last_timing.ms[7] = ev.span(9, 10);
  }
  return GC_OK;
}

int check_args(const gc_csr *g) {
  if (!g) {
    set_error("null graph");
    return GC_EINVAL;
  }
  if (g->n < 0 || g->nnz < 0 || g->n > 2147483646LL || g->nnz > 2147483646LL || (g->nnz & 1) ||
      (g->n == 0 && g->nnz > 0)) {
    set_error("invalid sizes n=%lld nnz=%lld", (long long)g->n, (long long)g->nnz);
    return GC_EINVAL;
  }
  if (!g->row_ptr || (g->nnz > 0 && !g->col)) {
    set_error("null CSR array");
    return GC_EINVAL;
  }
  return GC_OK;
}

Plan plan_of(const gc_csr *g, bool per_edge) {
  Plan P;
  P.n = g->n;
  P.nnz = g->nnz;
  P.m = g->nnz / 2;
  P.per_edge = per_edge;
  P.B = std::max(1, bits_for((u64)std::max<int64_t>(g->n - 1, 1)));
  return P;
}

int validate(const gc_csr *g, hipStream_t s) {
  int32_t *e = nullptr;
  GC_TRY_HIP(hipMallocAsync((void **)&e, 4, s));
  int32_t zero = 0, err = 0;
  hipError_t he = hipMemcpyAsync(e, &zero, 4, hipMemcpyHostToDevice, s);
  int rc = GC_OK;
  if (he == hipSuccess) rc = launch_validate(g->row_ptr, g->col, g->n, g->nnz, e, s);
  if (he == hipSuccess && rc == GC_OK) he = hipMemcpyAsync(&err, e, 4, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess && rc == GC_OK) he = hipStreamSynchronize(s);
  const hipError_t fe = hipFreeAsync(e, s);
  if (rc != GC_OK) return rc;
  if (he == hipSuccess) he = fe;
  if (he != hipSuccess) {
    set_error("validation: %s", hipGetErrorString(he));
    return GC_EHIP;
  }
  if (err != 0) {
    const int code = -(__builtin_ffs(err) - 1);
    set_error("CSR contract violated (code %d)", code);
    return code;
  }
  return GC_OK;
}

}  // namespace

// Workspace bound from host-side maxima (used by the server's admission).
size_t workspace_bound(int64_t n, int64_t nnz, int max_deg, int max_ucnt, bool per_edge) {
  if (n == 0 || nnz == 0) return 256;
  gc_csr g{n, nnz, nullptr, nullptr};
  const Plan P = plan_of(&g, per_edge);
  Arena a;
  Fixed f;
  alloc_fixed(a, P, f);
  Arena b;
  Dyn d;
  alloc_dyn(b, P, dyn_bound(P, max_deg, max_ucnt, ~0ull), d);
  return a.peak + b.peak + 1024;
}

// From n and nnz alone: the maximum degree is at most min(n - 1, nnz), and
// a vertex's k upper neighbours each have degree at least k, so k^2 <= nnz.
size_t workspace_bound_host(int64_t n, int64_t nnz, int per_edge, int *rc) {
  *rc = GC_OK;
  if (n < 0 || nnz < 0 || n > 2147483646LL || nnz > 2147483646LL || (nnz & 1) || per_edge < 0 ||
      per_edge > 2) {
    set_error("invalid sizes n=%lld nnz=%lld per_edge=%d", (long long)n, (long long)nnz, per_edge);
    *rc = GC_EINVAL;
    return 0;
  }
  if (n == 0 || nnz == 0) return 256;
  const int max_deg = (int)std::min<int64_t>(n - 1, nnz);
  int64_t k = (int64_t)std::sqrt((double)nnz);
  while (k * k > nnz) k--;
  while ((k + 1) * (k + 1) <= nnz) k++;
  const int max_ucnt = (int)std::min<int64_t>(k, max_deg);
  gc_csr g{n, nnz, nullptr, nullptr};
  Plan P = plan_of(&g, per_edge != 0);
  P.local = per_edge == 2;
  Arena a;
  Fixed f;
  alloc_fixed(a, P, f);
  Arena b;
  Dyn d;
  alloc_dyn(b, P, dyn_bound(P, max_deg, max_ucnt, ~0ull), d);
  return a.peak + b.peak + 1024;
}

size_t workspace_size(const gc_csr *g, int per_edge, hipStream_t s, int *rc) {
  *rc = check_args(g);
  if (*rc) return 0;
  if (per_edge < 0 || per_edge > 2) {
    *rc = GC_EINVAL;
    set_error("per_edge must be 0, 1 or 2");
    return 0;
  }
  Plan P = plan_of(g, per_edge != 0);
  P.local = per_edge == 2;
  if (P.n == 0 || P.nnz == 0) return 256;
  int max_deg = 0, max_ucnt = 0;
  u64 wedge_bound = 0;
  *rc = probe_graph(g, s, &max_deg, &max_ucnt, &wedge_bound);
  if (*rc) return 0;
  Arena a;
  Fixed f;
  alloc_fixed(a, P, f);
  Arena b;
  Dyn d;
  alloc_dyn(b, P, dyn_bound(P, max_deg, max_ucnt, wedge_bound), d);
  return a.peak + b.peak + 1024;
}

int count(const gc_csr *g, gc_u128 out[17], int64_t *per_edge_out, int64_t *local_out,
          u64 *vertex_out, void *ws, size_t ws_bytes, hipStream_t s, uint32_t flags) {
  GC_TRY(check_args(g));
  if (!out) {
    set_error("null output");
    return GC_EINVAL;
  }
  if (vertex_out && g->n >= 4 && (choose_h((u128)(g->n - 1), 3) >> 64) != 0) {
    set_error("per-vertex counts of n = %lld vertices do not fit 64 bits", (long long)g->n);
    return GC_EOVERFLOW;
  }
  if (g->nnz == 0) {
    if ((flags & GC_VALIDATE) && g->n > 0) {
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
    if (vertex_out && g->n > 0) {
      // no edges: every subset containing v is independent
      const u64 n1 = (u64)g->n - 1;
      GC_TRY(fill<u64>(vertex_out, 0ull, 17 * g->n, s));
      GC_TRY(fill<u64>(vertex_out + 1 * g->n, n1, g->n, s));
      GC_TRY(fill<u64>(vertex_out + 5 * g->n, (u64)choose_h(n1, 2), g->n, s));
      GC_TRY(fill<u64>(vertex_out + 16 * g->n, (u64)choose_h(n1, 3), g->n, s));
      GC_TRY_HIP(hipStreamSynchronize(s));
    }
    return GC_OK;
  }
  if (flags & GC_VALIDATE) GC_TRY(validate(g, s));
  Plan P = plan_of(g, per_edge_out != nullptr || local_out != nullptr || vertex_out != nullptr);
  P.local = local_out != nullptr || vertex_out != nullptr;
  P.flags = flags;
  return run(g, out, per_edge_out, local_out, vertex_out, reinterpret_cast<char *>(ws),
             ws ? ws_bytes : 0, s, P);
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

size_t graphlet_workspace_bound(int64_t n, int64_t nnz, int per_edge) {
  gc::clear_error();
  int rc = 0;
  try {
    return gc::workspace_bound_host(n, nnz, per_edge, &rc);
  } catch (...) {
    gc::set_error("unexpected exception");
    return 0;
  }
}

int graphlet_count(const gc_csr *g, gc_u128 out_counts[17], int64_t *per_edge_out,
                   void *workspace, size_t ws_bytes, void *stream, uint32_t flags) {
  gc::clear_error();
  try {
    return gc::count(g, out_counts, per_edge_out, nullptr, nullptr, workspace, ws_bytes,
                     (hipStream_t)stream, flags);
  } catch (...) {
    gc::set_error("unexpected exception");
    return GC_EINTERNAL;
  }
}

int graphlet_count_local(const gc_csr *g, gc_u128 out_counts[17], int64_t *local_out,
                         void *workspace, size_t ws_bytes, void *stream, uint32_t flags) {
  gc::clear_error();
  if (!local_out) {
    gc::set_error("null local output");
    return GC_EINVAL;
  }
  try {
    return gc::count(g, out_counts, nullptr, local_out, nullptr, workspace, ws_bytes,
                     (hipStream_t)stream, flags);
  } catch (...) {
    gc::set_error("unexpected exception");
    return GC_EINTERNAL;
  }
}

int graphlet_count_vertex(const gc_csr *g, gc_u128 out_counts[17], uint64_t *vertex_out,
                          void *workspace, size_t ws_bytes, void *stream, uint32_t flags) {
  gc::clear_error();
  if (!vertex_out) {
    gc::set_error("null per-vertex output");
    return GC_EINVAL;
  }
  try {
    return gc::count(g, out_counts, nullptr, nullptr, reinterpret_cast<gc::u64 *>(vertex_out),
                     workspace, ws_bytes,
                     (hipStream_t)stream, flags);
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

const char *graphlet_version(void) { return "graphlet-mi355x 0.5"; }

}  // extern "C"
