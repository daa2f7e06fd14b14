// Seeded synthetic graph generators.
//
// Every graph leaves here as an undirected simple graph in CSR form: int32
// row offsets (n+1) and int32 column ids (2m), each neighbour list strictly
// increasing, no self-loops, symmetric.  The paper drops weights, self-loops
// and direction from its inputs before counting (Section 5, experimental
// setup); the generators do the same by construction.
//
// This module produces inputs only.  It holds none of the counting arithmetic
// and is shared, unchanged, by the CPU oracle and the GPU path.
//
// Random numbers: xoshiro256** seeded through splitmix64 (Blackman & Vigna),
// integer draws by Lemire's multiply-shift with rejection, so a seed gives
// the same graph on every x86-64 host.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <unordered_set>
#include <vector>

namespace {

struct SplitMix64 {
  uint64_t s;
  explicit SplitMix64(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
  }
};

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

struct Xoshiro256ss {
  uint64_t s[4];
  explicit Xoshiro256ss(uint64_t seed) {
    SplitMix64 sm(seed);
    for (auto &w : s) w = sm.next();
  }
  uint64_t next() {
    const uint64_t result = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
  }
  // Uniform integer in [0, k), k >= 1 (Lemire 2019, unbiased).
  uint64_t below(uint64_t k) {
    unsigned __int128 p = (unsigned __int128)next() * k;
    uint64_t lo = (uint64_t)p;
    if (lo < k) {
      uint64_t thresh = (0 - k) % k;
      while (lo < thresh) {
        p = (unsigned __int128)next() * k;
        lo = (uint64_t)p;
      }
    }
    return (uint64_t)(p >> 64);
  }
  // Uniform double in [0, 1) with 53 random bits.
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

// LSD radix sort of 64-bit keys, 11 bits per pass, over the bits in use.
static void radix_sort_u64(std::vector<uint64_t> &keys) {
  if (keys.size() < 2) return;
  uint64_t maxk = 0;
  for (uint64_t k : keys) maxk |= k;
  int bits = 64 - __builtin_clzll(maxk | 1);
  std::vector<uint64_t> tmp(keys.size());
  const int R = 11;
  const size_t B = size_t(1) << R;
  std::vector<size_t> cnt(B);
  for (int shift = 0; shift < bits; shift += R) {
    std::fill(cnt.begin(), cnt.end(), 0);
    for (uint64_t k : keys) cnt[(k >> shift) & (B - 1)]++;
    size_t sum = 0;
    for (size_t i = 0; i < B; i++) {
      size_t c = cnt[i];
      cnt[i] = sum;
      sum += c;
    }
    for (uint64_t k : keys) tmp[cnt[(k >> shift) & (B - 1)]++] = k;
    keys.swap(tmp);
  }
}

struct Csr {
  int64_t n = 0;
  std::vector<int32_t> row_ptr;
  std::vector<int32_t> col;
};

// keys: (min << 32 | max) pairs, loops already removed.  Sorted, deduplicated,
// then expanded to a symmetric CSR whose lists come out strictly increasing:
// in key order every row x first receives its lower neighbours (pairs (w,x),
// increasing w) and then its upper ones (pairs (x,v), increasing v).
static void csr_from_keys(int64_t n, std::vector<uint64_t> &keys, Csr &g) {
  radix_sort_u64(keys);
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  g.n = n;
  g.row_ptr.assign(n + 1, 0);
  for (uint64_t k : keys) {
    g.row_ptr[(k >> 32) + 1]++;
    g.row_ptr[(k & 0xffffffffULL) + 1]++;
  }
  for (int64_t i = 0; i < n; i++) g.row_ptr[i + 1] += g.row_ptr[i];
  g.col.resize(2 * keys.size());
  std::vector<int32_t> cur(g.row_ptr.begin(), g.row_ptr.end() - 1);
  for (uint64_t k : keys) {
    uint32_t u = (uint32_t)(k >> 32), v = (uint32_t)(k & 0xffffffffULL);
    g.col[cur[u]++] = (int32_t)v;
    g.col[cur[v]++] = (int32_t)u;
  }
}

static inline uint64_t pair_key(uint64_t u, uint64_t v) {
  return u < v ? ((u << 32) | v) : ((v << 32) | u);
}

// Erdos-Renyi G(n, m): m distinct pairs drawn uniformly, one at a time with
// rejection of repeats.
static void gen_er_gnm(int64_t n, int64_t m, uint64_t seed, Csr &g) {
  Xoshiro256ss rng(seed);
  int64_t maxm = n * (n - 1) / 2;
  if (m > maxm) m = maxm;
  std::vector<uint64_t> keys;
  keys.reserve(m);
  if (m * 3 > maxm) {
    // Dense: shuffle-select over all pairs (partial Fisher-Yates on indices).
    std::vector<uint64_t> all;
    all.reserve(maxm);
    for (int64_t u = 0; u < n; u++)
      for (int64_t v = u + 1; v < n; v++) all.push_back(((uint64_t)u << 32) | (uint64_t)v);
    for (int64_t i = 0; i < m; i++) {
      uint64_t j = i + rng.below(maxm - i);
      std::swap(all[i], all[j]);
      keys.push_back(all[i]);
    }
  } else {
    std::unordered_set<uint64_t> seen;
    seen.reserve(m * 2);
    while ((int64_t)keys.size() < m) {
      uint64_t u = rng.below(n), v = rng.below(n);
      if (u == v) continue;
      uint64_t k = pair_key(u, v);
      if (seen.insert(k).second) keys.push_back(k);
    }
  }
  csr_from_keys(n, keys, g);
}

// Seeded uniform permutation of [0, n) (Fisher-Yates).
static std::vector<uint32_t> permutation(int64_t n, Xoshiro256ss &rng) {
  std::vector<uint32_t> p(n);
  for (int64_t i = 0; i < n; i++) p[i] = (uint32_t)i;
  for (int64_t i = n - 1; i > 0; i--) std::swap(p[i], p[rng.below(i + 1)]);
  return p;
}

// Chung-Lu by ball dropping: `balls` endpoint pairs, each endpoint drawn with
// probability proportional to w_i = (i + i0)^(-1/(beta-1)); loops and repeats
// dropped; vertex ids randomly permuted so degree is not tied to id.
static void gen_chung_lu(int64_t n, double beta, double i0, int64_t balls, uint64_t seed, Csr &g) {
  Xoshiro256ss rng(seed);
  const double ex = -1.0 / (beta - 1.0);
  std::vector<double> w(n);
  double tot = 0.0;
  for (int64_t i = 0; i < n; i++) {
    w[i] = std::pow((double)i + i0, ex);
    tot += w[i];
  }
  // Fixed-point cumulative table: cum[i] = floor(2^62 * sum_{j<=i} w_j / tot).
  std::vector<uint64_t> cum(n);
  double acc = 0.0;
  const double scale = 4611686018427387904.0;  // 2^62
  for (int64_t i = 0; i < n; i++) {
    acc += w[i];
    double c = acc / tot * scale;
    cum[i] = c >= scale ? (uint64_t)1 << 62 : (uint64_t)c;
  }
  cum[n - 1] = (uint64_t)1 << 62;
  auto draw = [&]() -> uint64_t {
    uint64_t r = rng.next() >> 2;  // uniform in [0, 2^62)
    return (uint64_t)(std::upper_bound(cum.begin(), cum.end(), r) - cum.begin());
  };
  std::vector<uint32_t> perm = permutation(n, rng);
  std::vector<uint64_t> keys;
  keys.reserve(balls);
  for (int64_t b = 0; b < balls; b++) {
    uint64_t u = draw(), v = draw();
    if (u == v) continue;
    keys.push_back(pair_key(perm[u], perm[v]));
  }
  csr_from_keys(n, keys, g);
}

// R-MAT (Chakrabarti, Zhan, Faloutsos 2004) without noise: each of
// edge_factor * 2^scale tuples picks one quadrant per level with
// probabilities (a, b, c, 1-a-b-c); ids are then randomly permuted
// (Graph500 style); symmetrised, deduplicated, loops dropped.
static void gen_rmat(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed,
                     Csr &g) {
  Xoshiro256ss rng(seed);
  const int64_t n = int64_t(1) << scale;
  const int64_t tuples = edge_factor * n;
  // Integer thresholds on a 32-bit draw keep the generator bit-reproducible.
  const uint64_t TA = (uint64_t)std::llround(a * 4294967296.0);
  const uint64_t TB = (uint64_t)std::llround((a + b) * 4294967296.0);
  const uint64_t TC = (uint64_t)std::llround((a + b + c) * 4294967296.0);
  std::vector<uint32_t> perm = permutation(n, rng);
  std::vector<uint64_t> keys;
  keys.reserve(tuples);
  for (int64_t t = 0; t < tuples; t++) {
    uint64_t u = 0, v = 0;
    uint64_t r = 0;
    for (int lvl = 0; lvl < scale; lvl++) {
      uint64_t x;
      if ((lvl & 1) == 0) {
        r = rng.next();
        x = r & 0xffffffffULL;
      } else {
        x = r >> 32;
      }
      uint64_t bu = 0, bv = 0;
      if (x < TA) {
      } else if (x < TB) {
        bv = 1;
      } else if (x < TC) {
        bu = 1;
      } else {
        bu = 1;
        bv = 1;
      }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    if (u == v) continue;
    keys.push_back(pair_key(perm[u], perm[v]));
  }
  csr_from_keys(n, keys, g);
}

// Random geometric graph on the unit torus: n uniform points, an edge when the
// wrap-around distance is below r.  r = sqrt(mean_deg / (pi (n-1))) gives the
// requested mean degree exactly in expectation on the torus (no boundary).
static void gen_rgg_torus(int64_t n, double mean_deg, uint64_t seed, Csr &g) {
  Xoshiro256ss rng(seed);
  std::vector<double> x(n), y(n);
  for (int64_t i = 0; i < n; i++) {
    x[i] = rng.uniform();
    y[i] = rng.uniform();
  }
  double r = n > 1 ? std::sqrt(mean_deg / (M_PI * (double)(n - 1))) : 0.0;
  double r2 = r * r;
  std::vector<uint64_t> keys;
  for (int64_t i = 0; i < n; i++)
    for (int64_t j = i + 1; j < n; j++) {
      double dx = std::fabs(x[i] - x[j]);
      double dy = std::fabs(y[i] - y[j]);
      if (dx > 0.5) dx = 1.0 - dx;
      if (dy > 0.5) dy = 1.0 - dy;
      if (dx * dx + dy * dy < r2) keys.push_back(((uint64_t)i << 32) | (uint64_t)j);
    }
  csr_from_keys(n, keys, g);
}

struct Batch {
  int64_t graphs = 0;
  std::vector<int64_t> node_off;  // G+1 offsets into the concatenated rows
  std::vector<int64_t> kind;      // 0 = ER, 1 = RGG
  Csr cat;                        // concatenated rows, per-graph local ids,
                                  // row_ptr global over the concatenation
};

// Many small graphs: node counts uniform in [nmin, nmax]; a fraction rgg_frac
// are torus RGGs of mean degree rgg_deg, the rest ER G(n, round(rho C(n,2)))
// with rho uniform in [rho_min, rho_max].  Per-graph seeds come from one
// splitmix64 stream so any graph can be regenerated alone.
static void gen_batch(int64_t G, int64_t nmin, int64_t nmax, double rho_min, double rho_max,
                      double rgg_frac, double rgg_deg, uint64_t seed, Batch &bt) {
  Xoshiro256ss rng(seed);
  bt.graphs = G;
  bt.node_off.assign(1, 0);
  bt.kind.clear();
  bt.cat.n = 0;
  bt.cat.row_ptr.assign(1, 0);
  bt.cat.col.clear();
  for (int64_t gi = 0; gi < G; gi++) {
    int64_t n = nmin + (int64_t)rng.below(nmax - nmin + 1);
    bool is_rgg = rng.uniform() < rgg_frac;
    double rho = rho_min + (rho_max - rho_min) * rng.uniform();
    uint64_t gseed = rng.next();
    Csr g;
    if (is_rgg) {
      gen_rgg_torus(n, rgg_deg, gseed, g);
    } else {
      int64_t m = (int64_t)std::llround(rho * (double)(n * (n - 1) / 2));
      gen_er_gnm(n, m, gseed, g);
    }
    int64_t base = bt.cat.row_ptr.back();
    for (int64_t i = 0; i < n; i++) bt.cat.row_ptr.push_back((int32_t)(base + g.row_ptr[i + 1]));
    bt.cat.col.insert(bt.cat.col.end(), g.col.begin(), g.col.end());
    bt.cat.n += n;
    bt.node_off.push_back(bt.cat.n);
    bt.kind.push_back(is_rgg ? 1 : 0);
  }
}

struct Handle {
  Csr g;
  Batch b;
  bool is_batch = false;
};

}  // namespace

extern "C" {

// Graph kinds for gg_make.  params (doubles) per kind:
//   1 ER G(n,m):       {n, m}
//   2 Chung-Lu:        {n, beta, i0, balls}
//   3 R-MAT:           {scale, edge_factor, a, b, c}
//   4 RGG on torus:    {n, mean_degree}
//   5 batch of graphs: {G, nmin, nmax, rho_min, rho_max, rgg_frac, rgg_deg}
// Returns an opaque handle, or NULL on bad parameters / out of memory.
void *gg_make(int kind, const double *p, uint64_t seed) {
  Handle *h = new (std::nothrow) Handle();
  if (!h) return nullptr;
  try {
    switch (kind) {
      case 1:
        if (p[0] < 0 || p[0] > 2147483647.0 || p[1] < 0) break;
        gen_er_gnm((int64_t)p[0], (int64_t)p[1], seed, h->g);
        return h;
      case 2:
        if (p[0] < 1 || p[1] <= 1.0 || p[2] < 0 || p[3] < 0) break;
        gen_chung_lu((int64_t)p[0], p[1], p[2], (int64_t)p[3], seed, h->g);
        return h;
      case 3:
        if (p[0] < 1 || p[0] > 30 || p[1] < 1) break;
        gen_rmat((int)p[0], (int64_t)p[1], p[2], p[3], p[4], seed, h->g);
        return h;
      case 4:
        if (p[0] < 0 || p[0] > 100000 || p[1] < 0) break;
        gen_rgg_torus((int64_t)p[0], p[1], seed, h->g);
        return h;
      case 5:
        if (p[0] < 0 || p[1] < 1 || p[2] < p[1] || p[2] > 100000) break;
        gen_batch((int64_t)p[0], (int64_t)p[1], (int64_t)p[2], p[3], p[4], p[5], p[6], seed,
                  h->b);
        h->is_batch = true;
        h->g = std::move(h->b.cat);
        return h;
      default:
        break;
    }
  } catch (...) {
  }
  delete h;
  return nullptr;
}

int64_t gg_n(const void *h) { return ((const Handle *)h)->g.n; }
int64_t gg_nnz(const void *h) { return (int64_t)((const Handle *)h)->g.col.size(); }
int64_t gg_graphs(const void *h) {
  const Handle *x = (const Handle *)h;
  return x->is_batch ? x->b.graphs : 1;
}

// Copies the CSR into caller buffers of n+1 and nnz int32 entries.
void gg_export(const void *h, int32_t *row_ptr, int32_t *col) {
  const Handle *x = (const Handle *)h;
  std::memcpy(row_ptr, x->g.row_ptr.data(), sizeof(int32_t) * x->g.row_ptr.size());
  if (!x->g.col.empty()) std::memcpy(col, x->g.col.data(), sizeof(int32_t) * x->g.col.size());
}

// Batch only: node offsets (G+1 int64) and kinds (G int64: 0 ER, 1 RGG).
void gg_export_batch(const void *h, int64_t *node_off, int64_t *kind) {
  const Handle *x = (const Handle *)h;
  if (!x->is_batch) return;
  std::memcpy(node_off, x->b.node_off.data(), sizeof(int64_t) * x->b.node_off.size());
  std::memcpy(kind, x->b.kind.data(), sizeof(int64_t) * x->b.kind.size());
}

void gg_free(void *h) { delete (Handle *)h; }

}  // extern "C"
