// Serving loop: graphs of mixed sizes submitted from host memory, admitted
// onto the device by HBM footprint, counted concurrently on several streams.
//
// Continuous batching: a request is admitted as soon as a worker slot is free
// and the device-memory budget can hold its footprint (CSR + workspace bound);
// requests that arrive while others are running are admitted as earlier ones
// finish and release their memory, so the work of several requests overlaps
// on the device.  Admission is first-come-first-served, but a request that
// does not fit yet does not block a later one that does.
//
// Each request's CSR stays resident on the device from admission until its
// counts are on the host; each request runs the same graphlet_count path as
// a standalone call, so its result does not depend on what else is running.
//
// Small graphs (at most GC_BATCH_MAX_N vertices) take the batch lane: one
// thread with its own stream and preallocated device and pinned host buffers
// (charged to the budget once, at creation) gathers every pending small
// request, up to the lane's capacity, into one concatenated CSR, uploads it in
// one copy and counts the whole batch with one launch per size class of the
// batched kernel (one workgroup per graph); requests arriving meanwhile form
// the next batch.  A batch that fails (a graph breaking the CSR contract
// under validation) is counted again one request at a time, so the failure
// stays with its own request.  Batched counts are the same integers as the
// single-graph path's.
//
// Resident graphs: a registered graph keeps its CSR (two buffers, the live
// one and a spare) and its counts on the device until it is unregistered.
// Edge updates against it are requests too; those of one graph run one at a
// time in submission order.  Each takes the localized update of the counts
// (graphlet_update_edge on the live CSR), then writes the changed CSR into
// the spare buffer and swaps; a failed update leaves graph and counts as
// they were.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace gc {
size_t workspace_bound(int64_t n, int64_t nnz, int max_deg, int max_ucnt, bool per_edge);
int csr_apply_edge(const gc_csr *g, int32_t u, int32_t v, int insert, int32_t *rp_out,
                   int32_t *col_out, hipStream_t s);
}

namespace {

using Clock = std::chrono::steady_clock;

enum State { PENDING = 0, RUNNING = 1, DONE = 2, FAILED = 3, CANCELLED = 4 };
enum Kind { COUNT = 0, REGISTER = 1, UPDATE = 2 };

// A registered graph.  Its id is the id of its registration request.
struct Resident {
  int64_t id = 0;
  int64_t n = 0, nnz = 0, cap = 0;  // cap: entries each col buffer holds
  int32_t *rp[2] = {nullptr, nullptr}, *col[2] = {nullptr, nullptr};
  int live = 0;
  bool ready = false;  // registration counted
  bool busy = false;   // a request on it is running
  bool gone = false;   // registration failed or unregistered
  size_t bytes = 0;    // device memory held while registered
  gc_u128 counts[17];
};

struct Request {
  int64_t id = 0;
  Kind kind = COUNT;
  Resident *g = nullptr;  // REGISTER, UPDATE
  int32_t u = 0, v = 0;
  int insert = 0;
  int64_t n = 0, nnz = 0;
  std::vector<int32_t> rp, col;
  size_t footprint = 0;
  State state = PENDING;
  bool cancel = false;
  int rc = 0;
  std::string err;
  gc_u128 out[17];
  Clock::time_point t_submit, t_start, t_done;
};

}  // namespace

namespace {

// Capacity of one batch of the batch lane.
constexpr int kLaneGraphs = 1024;
constexpr int64_t kLaneRows = int64_t(1) << 18;     // vertices
constexpr int64_t kLaneEntries = int64_t(1) << 22;  // adjacency entries

struct Lane {
  bool on = false;
  size_t bytes = 0;  // device memory, charged to the budget while the server lives
  hipStream_t st = nullptr;
  int64_t *d_off = nullptr, *h_off = nullptr;
  int32_t *d_rp = nullptr, *h_rp = nullptr;
  int32_t *d_col = nullptr, *h_col = nullptr;
  int64_t *d_out = nullptr, *h_out = nullptr;
};

}  // namespace

struct gc_server {
  size_t budget = 0;
  size_t in_use = 0;
  size_t peak = 0;
  uint32_t flags = 0;
  int device = 0;
  int slots = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> pending;
  std::unordered_map<int64_t, Request *> all;
  std::unordered_map<int64_t, Resident *> graphs;
  std::vector<std::thread> workers;
  Lane lane;
  std::thread lane_thread;
  std::condition_variable cv_lane;
  int64_t batches = 0, batched = 0;
  int64_t next_id = 1;
  bool stop = false;
  int running = 0;
  // statistics since the last reset
  int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, cancelled = 0;
  int64_t edges_done = 0;
  std::vector<double> latencies;
  Clock::time_point t_first, t_last;
  bool any = false;
};

namespace {

thread_local std::string t_srv_err;

// Completion of a request under the lock: state, statistics, wake-ups.
// `keep` bytes of its footprint stay charged (a registered graph's CSR).
void finish(gc_server *S, Request *r, int rc, const std::string &err, size_t keep) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->in_use -= r->footprint - keep;
    S->running--;
    r->t_done = Clock::now();
    r->rc = rc;
    r->err = err;
    r->rp.clear();
    r->rp.shrink_to_fit();
    r->col.clear();
    r->col.shrink_to_fit();
    if (r->g) r->g->busy = false;
    if (r->cancel) {
      r->state = CANCELLED;
      S->cancelled++;
    } else if (rc == GC_OK) {
      r->state = DONE;
      S->completed++;
      if (r->kind != UPDATE) S->edges_done += r->nnz / 2;
      S->latencies.push_back(
          std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
      S->t_last = r->t_done;
    } else {
      r->state = FAILED;
      S->failed++;
    }
  }
  S->cv_done.notify_all();
  S->cv_work.notify_all();
}

void free_resident(Resident *G) {
  for (int b = 0; b < 2; b++) {
    if (G->rp[b]) (void)hipFree(G->rp[b]);
    if (G->col[b]) (void)hipFree(G->col[b]);
    G->rp[b] = nullptr;
    G->col[b] = nullptr;
  }
}

// Registration: both CSR buffers are allocated for the graph's lifetime, the
// CSR is uploaded into one and counted.  On failure the graph is dropped and
// its pending updates fail.
void run_register(gc_server *S, Request *r, hipStream_t st) {
  Resident *G = r->g;
  int rc = GC_OK;
  std::string err;
  hipError_t e = hipSuccess;
  for (int b = 0; b < 2 && e == hipSuccess; b++) {
    e = hipMalloc((void **)&G->rp[b], sizeof(int32_t) * (size_t)(G->n + 1));
    if (e == hipSuccess) e = hipMalloc((void **)&G->col[b], sizeof(int32_t) * (size_t)G->cap);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(G->rp[0], r->rp.data(), sizeof(int32_t) * (size_t)(G->n + 1),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess && G->nnz > 0)
    e = hipMemcpyAsync(G->col[0], r->col.data(), sizeof(int32_t) * (size_t)G->nnz,
                       hipMemcpyHostToDevice, st);
  if (e != hipSuccess) {
    rc = e == hipErrorOutOfMemory ? GC_ENOMEM : GC_EHIP;
    err = hipGetErrorString(e);
  } else {
    gc_csr g{G->n, G->nnz, G->rp[0], G->col[0]};
    rc = graphlet_count(&g, r->out, nullptr, nullptr, 0, st,
                        (S->flags & ~GC_SERVE_NO_LANE) | GC_VALIDATE);
    if (rc != GC_OK) err = graphlet_last_error();
  }
  (void)hipStreamSynchronize(st);
  if (rc == GC_OK) {
    std::lock_guard<std::mutex> lk(S->mu);
    std::memcpy(G->counts, r->out, sizeof(G->counts));
    G->live = 0;
    G->ready = true;
  } else {
    free_resident(G);
    std::lock_guard<std::mutex> lk(S->mu);
    G->gone = true;
    for (auto it = S->pending.begin(); it != S->pending.end();) {
      if ((*it)->g == G) {
        (*it)->state = FAILED;
        (*it)->rc = GC_EINVAL;
        (*it)->err = "the graph's registration failed";
        (*it)->g = nullptr;
        S->failed++;
        it = S->pending.erase(it);
      } else {
        ++it;
      }
    }
  }
  finish(S, r, rc, err, rc == GC_OK ? G->bytes : 0);
}

// One edge update of a registered graph: the counts by the localized update
// on the live CSR, then the changed CSR into the spare buffer; both are
// committed together.
void run_update(gc_server *S, Request *r, hipStream_t st) {
  Resident *G = r->g;
  gc_csr cur{G->n, G->nnz, G->rp[G->live], G->col[G->live]};
  gc_u128 c[17];
  std::memcpy(c, G->counts, sizeof(c));
  std::string err;
  int rc = graphlet_update_edge(&cur, r->u, r->v, r->insert, c, st);
  if (rc != GC_OK) {
    err = graphlet_last_error();
  } else if (r->insert && G->nnz + 2 > G->cap) {
    rc = GC_ENOMEM;
    err = "the registered graph has no room for more edges";
  } else {
    const int spare = 1 - G->live;
    rc = gc::csr_apply_edge(&cur, r->u, r->v, r->insert, G->rp[spare], G->col[spare], st);
    if (rc != GC_OK) err = graphlet_last_error();
    if (hipStreamSynchronize(st) != hipSuccess && rc == GC_OK) {
      rc = GC_EHIP;
      err = "stream error after the CSR update";
    }
  }
  if (rc == GC_OK) {
    // A request cancelled while it ran is not committed: the spare buffer it
    // wrote is scratch until the swap, so graph and counts stay as they were
    // and the request ends CANCELLED.
    std::lock_guard<std::mutex> lk(S->mu);
    if (!r->cancel) {
      G->live = 1 - G->live;
      G->nnz += r->insert ? 2 : -2;
      std::memcpy(G->counts, c, sizeof(c));
      std::memcpy(r->out, c, sizeof(c));
    }
  }
  finish(S, r, rc, err, 0);
}

// A count request by the single-graph path on stream st: upload, count, free.
void count_one(gc_server *S, Request *r, hipStream_t st) {
  int rc = GC_OK;
  std::string err;
  int32_t *d_rp = nullptr, *d_col = nullptr;
  hipError_t e = hipMallocAsync((void **)&d_rp, sizeof(int32_t) * (r->n + 1), st);
  if (e == hipSuccess && r->nnz > 0)
    e = hipMallocAsync((void **)&d_col, sizeof(int32_t) * r->nnz, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_rp, r->rp.data(), sizeof(int32_t) * (r->n + 1), hipMemcpyHostToDevice,
                       st);
  if (e == hipSuccess && r->nnz > 0)
    e = hipMemcpyAsync(d_col, r->col.data(), sizeof(int32_t) * r->nnz, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) {
    rc = e == hipErrorOutOfMemory ? GC_ENOMEM : GC_EHIP;
    err = hipGetErrorString(e);
  } else {
    gc_csr g{r->n, r->nnz, d_rp, d_col};
    rc = graphlet_count(&g, r->out, nullptr, nullptr, 0, st, S->flags & ~GC_SERVE_NO_LANE);
    if (rc != GC_OK) err = graphlet_last_error();
  }
  if (d_col) (void)hipFreeAsync(d_col, st);
  if (d_rp) (void)hipFreeAsync(d_rp, st);
  (void)hipStreamSynchronize(st);
  finish(S, r, rc, err, 0);
}

// A count request for the batch lane (under the lock).
bool is_small(const gc_server *S, const Request *r) {
  return S->lane.on && r->kind == COUNT && r->n <= GC_BATCH_MAX_N && r->nnz <= kLaneEntries;
}

void worker_main(gc_server *S) {
  (void)hipSetDevice(S->device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  while (true) {
    Request *r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      while (true) {
        if (S->stop) break;
        // first pending request, in order, that fits the remaining budget;
        // an update waits for its graph's registration and for the update
        // before it (the graph is busy meanwhile)
        for (auto it = S->pending.begin(); it != S->pending.end(); ++it) {
          Request *q = *it;
          if (is_small(S, q)) continue;  // the batch lane's
          if (q->kind == UPDATE && (!q->g->ready || q->g->busy)) continue;
          if (S->in_use + q->footprint <= S->budget) {
            r = q;
            S->pending.erase(it);
            break;
          }
        }
        if (r) break;
        S->cv_work.wait(lk);
      }
      if (!r) break;
      S->in_use += r->footprint;
      S->peak = std::max(S->peak, S->in_use);
      S->running++;
      r->state = RUNNING;
      r->t_start = Clock::now();
      if (r->g) r->g->busy = true;
    }
    if (r->kind == REGISTER) {
      run_register(S, r, st);
      continue;
    }
    if (r->kind == UPDATE) {
      run_update(S, r, st);
      continue;
    }
    count_one(S, r, st);  // outside the lock
  }
  if (st) (void)hipStreamDestroy(st);
}

// The batch lane: every pending small request, up to the lane's capacity, in
// one batched call on the lane's stream.
void run_batch(gc_server *S, const std::vector<Request *> &take) {
  Lane &L = S->lane;
  const int G = (int)take.size();
  int64_t rows = 0, ents = 0;
  L.h_off[0] = 0;
  L.h_rp[0] = 0;
  for (int g = 0; g < G; g++) {
    const Request *r = take[g];
    for (int64_t i = 0; i < r->n; i++) L.h_rp[rows + i + 1] = (int32_t)(ents + r->rp[i + 1]);
    if (r->nnz) std::memcpy(L.h_col + ents, r->col.data(), sizeof(int32_t) * (size_t)r->nnz);
    rows += r->n;
    ents += r->nnz;
    L.h_off[g + 1] = rows;
  }
  hipError_t e = hipMemcpyAsync(L.d_off, L.h_off, sizeof(int64_t) * (G + 1),
                                hipMemcpyHostToDevice, L.st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(L.d_rp, L.h_rp, sizeof(int32_t) * (rows + 1), hipMemcpyHostToDevice, L.st);
  if (e == hipSuccess && ents)
    e = hipMemcpyAsync(L.d_col, L.h_col, sizeof(int32_t) * ents, hipMemcpyHostToDevice, L.st);
  int rc = e == hipSuccess ? GC_OK : GC_EHIP;
  if (rc == GC_OK) {
    gc_batch b{G, L.d_off, L.d_rp, L.d_col};
    rc = graphlet_count_batched_noalloc(&b, L.d_out, L.st, S->flags & GC_VALIDATE);
  }
  if (rc == GC_OK) {
    e = hipMemcpyAsync(L.h_out, L.d_out, sizeof(int64_t) * 17 * G, hipMemcpyDeviceToHost, L.st);
    if (e == hipSuccess) e = hipStreamSynchronize(L.st);
    if (e != hipSuccess) rc = GC_EHIP;
  } else {
    (void)hipStreamSynchronize(L.st);
  }
  if (rc == GC_OK) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->batches++;
      S->batched += G;
    }
    for (int g = 0; g < G; g++) {
      Request *r = take[g];
      for (int k = 0; k < 17; k++) {
        r->out[k].lo = (uint64_t)L.h_out[(size_t)g * 17 + k];  // non-negative
        r->out[k].hi = 0;
      }
      finish(S, r, GC_OK, std::string(), 0);
    }
    return;
  }
  // a failed batch: each request again on its own, so an error stays with its
  // request
  for (Request *r : take) count_one(S, r, L.st);
}

void lane_main(gc_server *S) {
  (void)hipSetDevice(S->device);
  while (true) {
    std::vector<Request *> take;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      while (true) {
        if (S->stop) break;
        int64_t rows = 0, ents = 0;
        for (auto it = S->pending.begin(); it != S->pending.end();) {
          Request *q = *it;
          if (is_small(S, q) && (int)take.size() < kLaneGraphs && rows + q->n <= kLaneRows &&
              ents + q->nnz <= kLaneEntries) {
            rows += q->n;
            ents += q->nnz;
            take.push_back(q);
            it = S->pending.erase(it);
          } else {
            ++it;
          }
        }
        if (!take.empty()) break;
        S->cv_lane.wait(lk);
      }
      if (take.empty()) break;
      const auto now = Clock::now();
      for (Request *q : take) {
        q->state = RUNNING;
        q->t_start = now;
        q->footprint = 0;  // the lane's buffers are charged once, at creation
        S->running++;
      }
    }
    run_batch(S, take);
  }
}

// Device and pinned host buffers of the batch lane, if the budget leaves
// room for them beside requests (it takes at most a quarter of the budget).
void lane_create(gc_server *S) {
  Lane &L = S->lane;
  const size_t dev = sizeof(int64_t) * (kLaneGraphs + 1) + sizeof(int32_t) * (kLaneRows + 1) +
                     sizeof(int32_t) * kLaneEntries + sizeof(int64_t) * 17 * kLaneGraphs;
  if ((S->flags & GC_SERVE_NO_LANE) || 4 * dev > S->budget) return;
  hipError_t e = hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc((void **)&L.d_off, sizeof(int64_t) * (kLaneGraphs + 1));
  if (e == hipSuccess) e = hipMalloc((void **)&L.d_rp, sizeof(int32_t) * (kLaneRows + 1));
  if (e == hipSuccess) e = hipMalloc((void **)&L.d_col, sizeof(int32_t) * kLaneEntries);
  if (e == hipSuccess) e = hipMalloc((void **)&L.d_out, sizeof(int64_t) * 17 * kLaneGraphs);
  if (e == hipSuccess) e = hipHostMalloc((void **)&L.h_off, sizeof(int64_t) * (kLaneGraphs + 1));
  if (e == hipSuccess) e = hipHostMalloc((void **)&L.h_rp, sizeof(int32_t) * (kLaneRows + 1));
  if (e == hipSuccess) e = hipHostMalloc((void **)&L.h_col, sizeof(int32_t) * kLaneEntries);
  if (e == hipSuccess) e = hipHostMalloc((void **)&L.h_out, sizeof(int64_t) * 17 * kLaneGraphs);
  if (e == hipSuccess) {
    L.on = true;
    L.bytes = dev;
    S->in_use += dev;
    S->peak = std::max(S->peak, S->in_use);
  } else {
    (void)hipGetLastError();
  }
}

void lane_destroy(gc_server *S) {
  Lane &L = S->lane;
  if (L.d_off) (void)hipFree(L.d_off);
  if (L.d_rp) (void)hipFree(L.d_rp);
  if (L.d_col) (void)hipFree(L.d_col);
  if (L.d_out) (void)hipFree(L.d_out);
  if (L.h_off) (void)hipHostFree(L.h_off);
  if (L.h_rp) (void)hipHostFree(L.h_rp);
  if (L.h_col) (void)hipHostFree(L.h_col);
  if (L.h_out) (void)hipHostFree(L.h_out);
  if (L.st) (void)hipStreamDestroy(L.st);
  L = Lane();
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t lo = (size_t)pos;
  const size_t hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (v[hi] - v[lo]) * (pos - (double)lo);
}

// Maximum degree and maximum number of later neighbours under the
// (degree, id) order, from a host CSR (O(nnz)); also checks the ids.
bool host_maxima(int64_t n, const int32_t *rp, const int32_t *col, int *max_deg, int *max_ucnt) {
  int md = 0, mu = 0;
  for (int64_t u = 0; u < n; u++) {
    const int64_t a = rp[u], b = rp[u + 1];
    if (b < a) return false;
    md = std::max<int>(md, (int)(b - a));
  }
  for (int64_t u = 0; u < n; u++) {
    const int64_t a = rp[u], b = rp[u + 1];
    const int64_t du = b - a;
    int c = 0;
    for (int64_t j = a; j < b; j++) {
      const int64_t w = col[j];
      if (w < 0 || w >= n) return false;
      const int64_t dw = rp[w + 1] - rp[w];
      c += (dw > du || (dw == du && w > u)) ? 1 : 0;
    }
    mu = std::max(mu, c);
  }
  *max_deg = md;
  *max_ucnt = mu;
  return true;
}

}  // namespace

extern "C" {

const char *gc_server_last_error(void) { return t_srv_err.c_str(); }

gc_server *gc_server_create(size_t hbm_budget, int slots, uint32_t flags) {
  t_srv_err.clear();
  if (slots <= 0 || slots > 64 || hbm_budget == 0) {
    t_srv_err = "slots must be in 1..64 and the budget positive";
    return nullptr;
  }
  gc_server *S = new (std::nothrow) gc_server();
  if (!S) return nullptr;
  S->budget = hbm_budget;
  S->slots = slots;
  S->flags = flags;
  if (hipGetDevice(&S->device) != hipSuccess) S->device = 0;
  lane_create(S);
  try {
    for (int i = 0; i < slots; i++) S->workers.emplace_back(worker_main, S);
    if (S->lane.on) S->lane_thread = std::thread(lane_main, S);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->cv_work.notify_all();
    S->cv_lane.notify_all();
    for (auto &t : S->workers) t.join();
    if (S->lane_thread.joinable()) S->lane_thread.join();
    lane_destroy(S);
    delete S;
    t_srv_err = "could not start worker threads";
    return nullptr;
  }
  return S;
}

int64_t gc_server_submit(gc_server *S, int64_t n, int64_t nnz, const int32_t *row_ptr,
                         const int32_t *col) {
  t_srv_err.clear();
  if (!S || n < 0 || nnz < 0 || (nnz & 1) || n > 2147483646LL || nnz > 2147483646LL ||
      !row_ptr || (nnz > 0 && !col)) {
    t_srv_err = "invalid request arguments";
    if (S) {
      std::lock_guard<std::mutex> lk(S->mu);
      S->rejected++;
    }
    return GC_EINVAL;
  }
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) {
    t_srv_err = "row_ptr does not span [0, nnz]";
    std::lock_guard<std::mutex> lk(S->mu);
    S->rejected++;
    return GC_EINVAL;
  }
  int max_deg = 0, max_ucnt = 0;
  if (!host_maxima(n, row_ptr, col, &max_deg, &max_ucnt)) {
    t_srv_err = "malformed CSR (row offsets or vertex ids)";
    std::lock_guard<std::mutex> lk(S->mu);
    S->rejected++;
    return GC_EINVAL;
  }
  const size_t fp = sizeof(int32_t) * (size_t)(n + 1 + nnz) +
                    gc::workspace_bound(n, nnz, max_deg, max_ucnt, false) + (1u << 20);
  Request *r = new (std::nothrow) Request();
  if (!r) return GC_ENOMEM;
  std::lock_guard<std::mutex> lk(S->mu);
  if (fp > S->budget) {
    delete r;
    t_srv_err = "graph footprint exceeds the server's device-memory budget";
    S->rejected++;
    return GC_ENOMEM;
  }
  r->id = S->next_id++;
  r->n = n;
  r->nnz = nnz;
  r->rp.assign(row_ptr, row_ptr + n + 1);
  if (nnz) r->col.assign(col, col + nnz);
  r->footprint = fp;
  r->t_submit = Clock::now();
  if (!S->any) {
    S->t_first = r->t_submit;
    S->any = true;
  }
  S->all[r->id] = r;
  S->pending.push_back(r);
  S->submitted++;
  if (is_small(S, r)) S->cv_lane.notify_one();
  else S->cv_work.notify_one();
  return r->id;
}

// 1: done (out filled), 0: not finished, < 0: the request's error code.
static int report(gc_server *S, Request *r, gc_u128 out[17], double *latency_ms) {
  (void)S;
  if (r->state == DONE) {
    if (out) std::memcpy(out, r->out, sizeof(r->out));
    if (latency_ms)
      *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    return 1;
  }
  if (r->state == FAILED) {
    t_srv_err = r->err;
    return r->rc < 0 ? r->rc : GC_EINTERNAL;
  }
  if (r->state == CANCELLED) {
    t_srv_err = "cancelled";
    return GC_EINVAL;
  }
  return 0;
}

int gc_server_poll(gc_server *S, int64_t id, gc_u128 out[17], double *latency_ms) {
  t_srv_err.clear();
  if (!S) return GC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end()) {
    t_srv_err = "unknown request id";
    return GC_EINVAL;
  }
  return report(S, it->second, out, latency_ms);
}

int gc_server_wait(gc_server *S, int64_t id, gc_u128 out[17], double *latency_ms) {
  t_srv_err.clear();
  if (!S) return GC_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end()) {
    t_srv_err = "unknown request id";
    return GC_EINVAL;
  }
  Request *r = it->second;
  S->cv_done.wait(lk, [&] { return r->state >= DONE; });
  return report(S, r, out, latency_ms);
}

int gc_server_cancel(gc_server *S, int64_t id) {
  t_srv_err.clear();
  if (!S) return GC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end()) {
    t_srv_err = "unknown request id";
    return GC_EINVAL;
  }
  Request *r = it->second;
  if (r->state == PENDING) {
    S->pending.erase(std::find(S->pending.begin(), S->pending.end(), r));
    r->state = CANCELLED;
    r->rp.clear();
    r->col.clear();
    S->cancelled++;
    if (r->kind == REGISTER) {
      // the graph never becomes resident: its queued updates are cancelled
      // too (it stays known until gc_server_unregister, holding no memory)
      Resident *G = r->g;
      G->gone = true;
      for (auto p = S->pending.begin(); p != S->pending.end();) {
        if ((*p)->g == G) {
          (*p)->state = CANCELLED;
          (*p)->g = nullptr;
          S->cancelled++;
          p = S->pending.erase(p);
        } else {
          ++p;
        }
      }
      r->g = nullptr;
    }
    S->cv_done.notify_all();
  } else if (r->state == RUNNING) {
    r->cancel = true;  // result discarded when the device work ends
  }
  return GC_OK;
}

int gc_server_release(gc_server *S, int64_t id) {
  if (!S) return GC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end() || it->second->state < DONE) return GC_EINVAL;
  delete it->second;
  S->all.erase(it);
  return GC_OK;
}

int gc_server_stats(gc_server *S, gc_serve_stats *o) {
  if (!S || !o) return GC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(o, 0, sizeof(*o));
  o->submitted = S->submitted;
  o->completed = S->completed;
  o->failed = S->failed;
  o->rejected = S->rejected;
  o->cancelled = S->cancelled;
  o->pending = (int64_t)S->pending.size();
  o->running = S->running;
  o->batches = S->batches;
  o->batched = S->batched;
  o->bytes_in_use = S->in_use;
  o->bytes_peak = S->peak;
  o->budget = S->budget;
  o->p50_ms = percentile(S->latencies, 0.50);
  o->p99_ms = percentile(S->latencies, 0.99);
  double sum = 0;
  for (double v : S->latencies) sum += v;
  o->mean_ms = S->latencies.empty() ? 0.0 : sum / (double)S->latencies.size();
  if (S->any && S->completed > 0) {
    const double el = std::chrono::duration<double>(S->t_last - S->t_first).count();
    o->elapsed_s = el;
    o->graphs_per_s = el > 0 ? (double)S->completed / el : 0.0;
    o->edges_per_s = el > 0 ? (double)S->edges_done / el : 0.0;
  }
  return GC_OK;
}

int gc_server_reset_stats(gc_server *S) {
  if (!S) return GC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  S->submitted = S->completed = S->failed = S->rejected = S->cancelled = 0;
  S->batches = S->batched = 0;
  S->edges_done = 0;
  S->latencies.clear();
  S->any = false;
  S->peak = S->in_use;
  return GC_OK;
}

int64_t gc_server_register(gc_server *S, int64_t n, int64_t nnz, const int32_t *row_ptr,
                           const int32_t *col) {
  t_srv_err.clear();
  if (!S || n <= 0 || nnz < 0 || (nnz & 1) || n > 2147483646LL || nnz > 2147483646LL ||
      !row_ptr || (nnz > 0 && !col) || row_ptr[0] != 0 || row_ptr[n] != nnz) {
    t_srv_err = "invalid graph arguments";
    return GC_EINVAL;
  }
  int max_deg = 0, max_ucnt = 0;
  if (!host_maxima(n, row_ptr, col, &max_deg, &max_ucnt)) {
    t_srv_err = "malformed CSR (row offsets or vertex ids)";
    return GC_EINVAL;
  }
  Resident *G = new (std::nothrow) Resident();
  Request *r = new (std::nothrow) Request();
  if (!G || !r) {
    delete G;
    delete r;
    return GC_ENOMEM;
  }
  G->n = n;
  G->nnz = nnz;
  // room for nnz / 8 more entries (at least 512 edges) before the graph is full
  G->cap = nnz + std::max<int64_t>(1024, (nnz / 8 + 1) & ~int64_t(1));
  if (G->cap > 2147483646LL) G->cap = 2147483646LL & ~int64_t(1);
  G->bytes = 2 * sizeof(int32_t) * (size_t)(n + 1 + G->cap);
  const size_t fp =
      G->bytes + gc::workspace_bound(n, nnz, max_deg, max_ucnt, false) + (1u << 20);
  std::lock_guard<std::mutex> lk(S->mu);
  if (fp > S->budget) {
    delete G;
    delete r;
    t_srv_err = "graph footprint exceeds the server's device-memory budget";
    S->rejected++;
    return GC_ENOMEM;
  }
  r->id = S->next_id++;
  r->kind = REGISTER;
  r->g = G;
  G->id = r->id;
  r->n = n;
  r->nnz = nnz;
  r->rp.assign(row_ptr, row_ptr + n + 1);
  if (nnz) r->col.assign(col, col + nnz);
  r->footprint = fp;
  r->t_submit = Clock::now();
  if (!S->any) {
    S->t_first = r->t_submit;
    S->any = true;
  }
  S->all[r->id] = r;
  S->graphs[G->id] = G;
  S->pending.push_back(r);
  S->submitted++;
  S->cv_work.notify_one();
  return G->id;
}

int64_t gc_server_update(gc_server *S, int64_t graph, int32_t u, int32_t v, int insert) {
  t_srv_err.clear();
  if (!S) return GC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->graphs.find(graph);
  if (it == S->graphs.end() || it->second->gone) {
    t_srv_err = "unknown graph";
    S->rejected++;
    return GC_EINVAL;
  }
  Resident *G = it->second;
  if (u < 0 || v < 0 || u >= G->n || v >= G->n || u == v) {
    t_srv_err = "endpoint out of range, or u == v";
    S->rejected++;
    return GC_EINVAL;
  }
  Request *r = new (std::nothrow) Request();
  if (!r) return GC_ENOMEM;
  r->id = S->next_id++;
  r->kind = UPDATE;
  r->g = G;
  r->u = u;
  r->v = v;
  r->insert = insert ? 1 : 0;
  // the two membership bitmaps and the accumulators of the update
  r->footprint = 2 * sizeof(uint32_t) * (size_t)((G->n + 31) / 32) + (1u << 16);
  r->t_submit = Clock::now();
  if (!S->any) {
    S->t_first = r->t_submit;
    S->any = true;
  }
  S->all[r->id] = r;
  S->pending.push_back(r);
  S->submitted++;
  S->cv_work.notify_one();
  return r->id;
}

int gc_server_graph_counts(gc_server *S, int64_t graph, gc_u128 out_counts[17]) {
  t_srv_err.clear();
  if (!S || !out_counts) return GC_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->graphs.find(graph);
  if (it == S->graphs.end() || it->second->gone) {
    t_srv_err = "unknown graph";
    return GC_EINVAL;
  }
  if (!it->second->ready) return 0;
  std::memcpy(out_counts, it->second->counts, sizeof(it->second->counts));
  return 1;
}

int gc_server_unregister(gc_server *S, int64_t graph) {
  t_srv_err.clear();
  if (!S) return GC_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->graphs.find(graph);
  if (it == S->graphs.end()) {
    t_srv_err = "unknown graph";
    return GC_EINVAL;
  }
  Resident *G = it->second;
  // pending requests on the graph are cancelled; a running one finishes
  for (auto p = S->pending.begin(); p != S->pending.end();) {
    if ((*p)->g == G) {
      (*p)->state = CANCELLED;
      (*p)->g = nullptr;
      (*p)->rp.clear();
      (*p)->col.clear();
      S->cancelled++;
      p = S->pending.erase(p);
    } else {
      ++p;
    }
  }
  S->cv_done.wait(lk, [&] { return !G->busy; });
  for (auto &kv : S->all)
    if (kv.second->g == G) kv.second->g = nullptr;
  if (G->ready && !G->gone) S->in_use -= G->bytes;
  S->graphs.erase(G->id);
  lk.unlock();
  (void)hipSetDevice(S->device);
  free_resident(G);
  delete G;
  S->cv_done.notify_all();
  S->cv_work.notify_all();
  return GC_OK;
}

void gc_server_destroy(gc_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    for (Request *r : S->pending) {
      r->state = CANCELLED;
    }
    S->pending.clear();
  }
  S->cv_work.notify_all();
  S->cv_lane.notify_all();
  for (auto &t : S->workers) t.join();
  if (S->lane_thread.joinable()) S->lane_thread.join();
  for (auto &kv : S->all) delete kv.second;
  (void)hipSetDevice(S->device);
  lane_destroy(S);
  for (auto &kv : S->graphs) {
    free_resident(kv.second);
    delete kv.second;
  }
  delete S;
}

}  // extern "C"
