/*
 * graphlet.h -- C ABI of the MI355X graphlet counting library.
 *
 * Exact counts of all induced 2-, 3- and 4-node graphlets (17 classes,
 * connected and disconnected) of an undirected simple graph, by the per-edge
 * method of Ahmed et al., "Graphlet Decomposition: Framework, Algorithms, and
 * Applications" (arXiv 1506.04322):
 *   Step 1  per edge e = (u, v): the triangle set Tri_e and the 2-star sets
 *           Star_u, Star_v (Section 3, the triad census algorithm);
 *   Step 2  per edge: the 4-cliques and 4-cycles containing e (Section 4,
 *           Corollaries "cliq" and "cyc", procedures CliqueCount and
 *           CycleCount of the graphlet counting algorithm);
 *   Step 3  per edge: the unrestricted counts N_{a,b} in constant time
 *           (Equations "comb_n_ai_ai" and "comb_n_ai_aj");
 *   Step 4  all 17 counts from the sums, by the Lemmas of Section 4.3 and
 *           Equations "g_4_9" and "g_4_11".
 *
 * All counting is integer and exact.  Totals are unsigned 128-bit (C(n,3)
 * exceeds 2^63 from n ~ 3.8 million on).
 *
 * Output order of a 17-entry count vector (Table 1 numbering):
 *   [0] g2_1 edge            [1] g2_2 2-node-independent
 *   [2] g3_1 triangle        [3] g3_2 2-star
 *   [4] g3_3 3-node-1-edge   [5] g3_4 3-node-independent
 *   [6] g4_1 4-clique        [7] g4_2 4-chordalcycle   [8] g4_3 4-tailedtriangle
 *   [9] g4_4 4-cycle         [10] g4_5 3-star          [11] g4_6 4-path
 *   [12] g4_7 4-node-1-triangle  [13] g4_8 4-node-2-star  [14] g4_9 4-node-2-edge
 *   [15] g4_10 4-node-1-edge     [16] g4_11 4-node-independent
 *
 * Threading: calls are reentrant; each call uses only its own workspace.
 * Errors: every entry point returns GC_OK (0) or a negative GC_E* code; the
 * message of the calling thread's last error is graphlet_last_error().  No
 * C++ exception crosses this interface.  Outputs are unspecified on error.
 * Ownership: the library keeps no pointer passed in after a call returns.
 */
#ifndef GRAPHLET_H
#define GRAPHLET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define GC_OK 0
#define GC_EINVAL (-1)       /* bad argument: null pointer, negative size, odd nnz,
                                 entries with no vertices */
#define GC_ENOTSORTED (-2)   /* a neighbour list is not strictly increasing (covers duplicates) */
#define GC_ESELFLOOP (-3)    /* (u, u) present */
#define GC_EASYMMETRIC (-4)  /* v in N(u) but u not in N(v), or an id outside [0, n) */
#define GC_EOVERFLOW (-5)    /* a count does not fit the output type */
#define GC_ENOMEM (-6)       /* workspace too small, or device allocation failed */
#define GC_EHIP (-7)         /* a HIP runtime call failed */
#define GC_EINTERNAL (-8)    /* an exact division left a remainder: never expected */

/* Flags. */
#define GC_VALIDATE 1u /* check the CSR contract on the device first, O(m log Delta) */
/* Route of the costliest 4-cycle vertices (global counts only; the counts do
 * not depend on it).  By default a cost model sends hubs to dense slabs when
 * a slab pass is cheaper than their wedges by work items. */
#define GC_DENSE_ALL 2u /* up to 8192 costliest heavy vertices in dense slabs */
#define GC_DENSE_OFF 4u /* no dense slabs */
/* Serving only (gc_server_create): no batch lane, every request on a slot. */
#define GC_SERVE_NO_LANE 256u

/*
 * An undirected simple graph in CSR form, in DEVICE memory owned by the
 * caller.  The paper's input is G = (V, E) undirected, with weights, loops and
 * direction discarded (Section 5, setup).
 *   n        number of vertices, all of them counted in |V| (isolated ones
 *            too); 0 <= n < 2^31
 *   nnz      2 |E|: every edge appears in both endpoint lists; nnz < 2^31
 *   row_ptr  int32[n+1], row_ptr[0] = 0, row_ptr[n] = nnz, non-decreasing
 *   col      int32[nnz], each list strictly increasing, ids in [0, n),
 *            no (u, u), symmetric
 * Inputs that break the contract give unspecified counts unless
 * GC_VALIDATE is set, in which case they are rejected with the codes above.
 */
typedef struct gc_csr {
  int64_t n;
  int64_t nnz;
  const int32_t *row_ptr;
  const int32_t *col;
} gc_csr;

/* Unsigned 128-bit integer: value = hi * 2^64 + lo. */
typedef struct gc_u128 {
  uint64_t lo;
  uint64_t hi;
} gc_u128;

/*
 * Bytes of device workspace graphlet_count needs for this graph (per_edge:
 * 0 global counts only, 1 with per_edge_out, 2 for graphlet_count_local and graphlet_count_vertex).  Reads g->n and g->nnz only on the
 * host, plus the maximum degree on the device (one small stream-ordered read
 * on `stream`, a hipStream_t).  Returns 0 if the sizes are invalid.
 */
size_t graphlet_workspace_size(const gc_csr *g, int per_edge, void *stream);

/*
 * A workspace size that suffices for every graph with these sizes, from n and
 * nnz alone (per_edge as above): no device work and no stream.  It is
 * larger than graphlet_workspace_size's figure for the same graph, which
 * also reads the degrees.  Returns 0 on invalid sizes (negative, odd nnz, n
 * or nnz of 2^31 - 1 or more, per_edge outside 0..2).
 */
size_t graphlet_workspace_bound(int64_t n, int64_t nnz, int per_edge);

/*
 * Global counts, and optionally per-edge quantities, of one graph.
 *   g             the graph (device arrays, see gc_csr)
 *   out_counts    HOST gc_u128[17], the 17 counts in the order above
 *   per_edge_out  NULL, or DEVICE int64[3*m] (m = nnz/2), filled with
 *                 [0*m + k] |Tri_e|        (triangles through e, Section 3)
 *                 [1*m + k] 4-cliques containing e  (Corollary "cliq")
 *                 [2*m + k] induced 4-cycles containing e (Corollary "cyc")
 *                 where k is the canonical id of e = (u, v), u < v: edges
 *                 numbered u ascending, then v ascending as in u's list.
 *   workspace     DEVICE buffer of ws_bytes >= graphlet_workspace_size(),
 *                 or NULL to let the library allocate (and free) its own
 *   stream        hipStream_t the work is ordered on (NULL = default stream)
 *   flags         GC_VALIDATE or 0
 * Returns after out_counts is filled; per_edge_out is complete when the
 * call returns.  Device memory the caller passed is only read, except
 * per_edge_out and workspace.
 */
int graphlet_count(const gc_csr *g, gc_u128 out_counts[17], int64_t *per_edge_out,
                   void *workspace, size_t ws_bytes, void *stream, uint32_t flags);

/*
 * Per-edge local 4-node vectors ("edge orbits"): for every edge e = (u, v),
 * the 3- and 4-node subsets containing e split by their graphlet and by the
 * place of e in it, from the unrestricted and restricted counts N_{a,b} and
 * N_{a,b,0/1} of Section 4.2 (vertex types T, Su, Sv, I relative to e;
 * Corollaries of Section 4.3 for the restricted counts).  Also fills
 * out_counts (HOST, as graphlet_count).
 *   local_out  DEVICE int64[GC_LOCAL * m], component-major: entry
 *              [j * m + k] is term j of the edge with canonical id k (as
 *              per_edge_out), terms j =
 *     0 |Tri_e| (triangle)            1 |Su|+|Sv| (2-star)     2 I_e (3-node-1-edge)
 *     3 N_{T,T,1} 4-clique            4 N_{T,T,0} chordal cycle, e the chord
 *     5 N_{T,S,1} chordal cycle, e on the cycle
 *     6 N_{T,S,0} tailed triangle, e in the triangle at the tail's vertex
 *     7 N_{T,I,1} tailed triangle, e in the triangle away from the tail
 *     8 N_{S,S,1} tailed triangle, e the tail      9 N_{Su,Sv,1} 4-cycle
 *    10 N_{S,S,0} 3-star             11 N_{Su,Sv,0} 4-path, e in the middle
 *    12 N_{S,I,1} 4-path, e at an end  13 N_{T,I,0} 4-node-1-triangle
 *    14 N_{S,I,0} 4-node-2-star      15 N_{I,I,1} 4-node-2-edge
 *    16 N_{I,I,0} 4-node-1-edge
 *   (S,S: two vertices of the same star; T,S: a Tri_e vertex and a star
 *   vertex; S,I: a star vertex and an I vertex.)  Terms 3..16 of an edge add
 *   up to C(n-2, 2); summed over all edges, the terms of a graphlet give its
 *   count times its number of edges.
 *   workspace  as graphlet_count, sized with graphlet_workspace_size(g, 2, .)
 */
#define GC_LOCAL 17
int graphlet_count_local(const gc_csr *g, gc_u128 out_counts[17], int64_t *local_out,
                         void *workspace, size_t ws_bytes, void *stream, uint32_t flags);

/*
 * Per-vertex graphlet counts: for every vertex v and each of the 17 classes,
 * the number of k-node subsets S containing v whose induced subgraph is that
 * class (the node-level counterpart of the edge weights used to rank edges
 * or nodes by their 4-stars and 4-cliques, subsection "Finding Large Stars,
 * Cliques, and other Patterns Fast").  Derived from the per-edge local
 * 4-node vectors of v's edges plus, for the classes in which v can be
 * isolated, the 2- and 3-node graphlets outside N(v) u {v}.  Summed over v,
 * the column of a k-node class is k times its global count.  Also fills
 * out_counts (HOST, as graphlet_count).
 *   vertex_out  DEVICE uint64[17 * n], class-major: entry [c * n + v] is
 *               class c (order as out_counts) for the caller's vertex v.
 *   workspace   as graphlet_count, sized with graphlet_workspace_size(g, 2, .)
 * Exact in 64 bits while C(n-1, 3) < 2^64 (n up to about 4.8 million);
 * returns GC_EOVERFLOW for larger n before any work.  vertex_out is complete
 * when the call returns.
 */
int graphlet_count_vertex(const gc_csr *g, gc_u128 out_counts[17], uint64_t *vertex_out,
                          void *workspace, size_t ws_bytes, void *stream, uint32_t flags);

/*
 * Localized update of the counts of one graph when one edge changes
 * (Section 6.3: counts updated from the neighbourhood of the changed edge
 * instead of recomputed).  Only the subsets holding both endpoints change
 * class; their numbers are the terms of the edge's local 4-node vector (as
 * graphlet_count_local), computed from the lists of u, v and their
 * neighbours only: O(sum of deg(w) over w in N(u) u N(v)) work.
 *   g        DEVICE CSR of the graph BEFORE the change (gc_csr contract)
 *   u, v     the edge's endpoints, u != v, both in [0, n)
 *   insert   1: the edge is added (it must be absent from g),
 *            0: the edge is removed (it must be present in g)
 *   counts   HOST, in: the 17 counts of g; out: the counts after the change
 * Returns GC_EINVAL if the endpoints are invalid, the edge's presence does
 * not match `insert`, or the counts cannot be those of g (a count would turn
 * negative); counts are left unchanged on error.  The caller updates its CSR.
 * Allocates a stream-ordered scratch of 2 bits per vertex.
 */
int graphlet_update_edge(const gc_csr *g, int32_t u, int32_t v, int insert, gc_u128 counts[17],
                         void *stream);

/*
 * Many small graphs in one call (the paper's graph-classification use, many
 * small networks each described by its k = 2, 3, 4 counts, Section 6).
 *   graphs    G >= 0
 *   node_off  DEVICE int64[G+1]: graph i owns rows node_off[i] .. node_off[i+1]-1
 *             of the concatenated row_ptr; every graph has at most
 *             GC_BATCH_MAX_N vertices
 *   row_ptr   DEVICE int32[node_off[G]+1], offsets into col (global)
 *   col       DEVICE int32[...], vertex ids LOCAL to each graph (0..n_i-1),
 *             per-graph lists obey the gc_csr contract
 * out: DEVICE int64[G][17], the 17 counts of each graph in the order above
 * (every count of a graph with at most GC_BATCH_MAX_N vertices fits int64).
 * Stream-ordered; returns when the results are complete.
 */
#define GC_BATCH_MAX_N 1024
typedef struct gc_batch {
  int64_t graphs;
  const int64_t *node_off;
  const int32_t *row_ptr;
  const int32_t *col;
} gc_batch;

int graphlet_count_batched(const gc_batch *b, int64_t *out, void *stream, uint32_t flags);

/*
 * graphlet_count_batched without any device allocation, for callers that
 * cannot allocate device memory (serving loops with a fixed footprint,
 * harnesses that forbid hipMalloc).  Same arguments, checks, results and
 * errors as graphlet_count_batched, with the size classes and order it would
 * use; it allocates nothing (no hipMalloc, hipMallocAsync or library
 * allocator).  Its scratch (an error word, the per-graph sizes and the class
 * lists: about 1.3 MB) is a static device array of the library that each GPU
 * it runs on holds until the process ends, so a batch holds at most
 * GC_NOALLOC_MAX_GRAPHS graphs: a larger one is refused with GC_EINVAL before
 * any device work.  Every call on a device shares that device's array, which
 * keeps the last call's contents (the call clears what must start at zero);
 * the library makes calls on one device from several host threads take turns
 * (a lock per device), since calls that overlapped on one array would race.
 * Stream-ordered; returns when the results are complete.
 */
#define GC_NOALLOC_MAX_GRAPHS 65536
int graphlet_count_batched_noalloc(const gc_batch *b, int64_t *out, void *stream,
                                   uint32_t flags);

/*
 * Per-vertex counts of every graph of a batch (the node-level view of the
 * per-edge local counts of Section 4.2, for the graph-classification batches
 * of Section 6): for each vertex v of each graph and each of the 17 classes,
 * the number of induced k-subsets of v's graph that contain v and induce that
 * class, the same quantity graphlet_count_vertex gives for one graph.
 *   b     as for graphlet_count_batched (same checks, same GC_VALIDATE)
 *   out   DEVICE uint64[node_off[G]][17], vertex-major: the row of vertex i of
 *         graph g is node_off[g] + i, its 17 counts in the order above (every
 *         count fits 64 bits for graphs of at most GC_BATCH_MAX_N vertices)
 * Summed over the vertices of a graph, the counts of a size-k class are k
 * times that graph's count.  Errors as for graphlet_count_batched; out is
 * not written when the checks fail (a HIP error part way may leave some
 * rows written).  Stream-ordered; returns when out is complete.  The size
 * classes run on streams of the library's own (created on first use,
 * one set per device, kept until the process ends), joined to `stream`;
 * calls from several host threads queue their launches on them in turn
 * (a lock covers the launches, not the wait for the results).
 */
int graphlet_batch_vertex(const gc_batch *b, uint64_t *out, void *stream, uint32_t flags);

/*
 * Graphlet frequency distributions of a batch (the normalised counts used to
 * compare and classify graphs, Section 6.1): for each graph and each size
 * k = 2, 3, 4, every count of size k divided by the sum of the counts of
 * size k (connected_only = 0: all classes of that size, a sum of C(n, k);
 * 1: the connected classes only, the disconnected entries set to 0).
 *   counts  DEVICE int64[G][17] as written by graphlet_count_batched
 *   out     DEVICE double[G][17]; an entry whose size has a zero sum is 0
 * Every quotient is the correctly rounded double of the exact ratio.
 * Stream-ordered; returns when out is complete.
 */
int graphlet_batch_gfd(const int64_t *counts, int64_t graphs, double *out, int connected_only,
                       void *stream);

/*
 * Batched execution plan, for a batch counted again and again (the same
 * arrays, possibly with new contents of the same sizes).  Creating a plan
 * checks the batch (GC_VALIDATE as above) and bins the graphs into size
 * classes by 64-bit words per adjacency row (a class of W words holds graphs
 * of at most 64 W vertices; W in 1, 2, 4, 6, 8, 10, 12, 16).  Each class is
 * counted by one persistent launch sized to fill the device, one workgroup
 * per graph at a time, costliest graphs first; the launches are captured into
 * a HIP graph.  With tune != 0 the class set and the workgroup size are
 * chosen by timing the candidates on this batch (the choice is remembered per
 * process for batches of the same size profile, and graphlet_count_batched
 * then uses it too).
 *   graphlet_batch_plan_create  b, out as for graphlet_count_batched (both
 *                      must stay valid while the plan lives); *plan receives
 *                      the plan.  Allocates device and pinned host memory.
 *                      Returns GC_OK or an error code (then *plan is NULL).
 *   graphlet_batch_plan_run     replays the captured launches on `stream` and
 *                      returns when out holds the counts; allocates nothing.
 *                      GC_EINVAL if a graph outgrew its class since the plan
 *                      was made.
 *   graphlet_batch_plan_info    the shape in use.
 *   graphlet_batch_plan_reshape forces a shape: block 256 or 512 threads, and
 *                      the classes as a mask (bit W-1 set: a class of W
 *                      words).  GC_EINVAL if no class holds some graph.
 *                      Re-reads the graph sizes, so it also re-plans a batch
 *                      whose graphs changed size (same array lengths).
 *   graphlet_batch_plan_destroy frees the plan.
 * One plan must not be run from two threads at once.
 */
typedef struct gc_batch_plan gc_batch_plan;
#define GC_BATCH_MAX_CLASSES 8
typedef struct gc_batch_plan_info {
  int block;                                 /* threads per workgroup */
  int classes;                               /* launches per run */
  int class_words[GC_BATCH_MAX_CLASSES];     /* words per row of each class */
  int64_t class_graphs[GC_BATCH_MAX_CLASSES];
  int class_grid[GC_BATCH_MAX_CLASSES];      /* workgroups of each launch */
  size_t class_lds[GC_BATCH_MAX_CLASSES];    /* dynamic LDS per workgroup */
  int candidates;                            /* shapes timed by the autotuner (0: not tuned) */
  double tuned_ms;                           /* best candidate's time */
} gc_batch_plan_info;

int graphlet_batch_plan_create(const gc_batch *b, int64_t *out, int tune, void *stream,
                               uint32_t flags, gc_batch_plan **plan);
int graphlet_batch_plan_run(gc_batch_plan *plan, void *stream);
int graphlet_batch_plan_info(const gc_batch_plan *plan, gc_batch_plan_info *info);
int graphlet_batch_plan_reshape(gc_batch_plan *plan, int block, uint32_t class_words_mask,
                                void *stream);
void graphlet_batch_plan_destroy(gc_batch_plan *plan);

/*
 * Diagnostics.  When enabled (per calling thread), graphlet_count records HIP
 * events on its stream at the boundaries of its phases, and the durations of
 * the thread's last call can be read back, together with the amount of
 * adjacency work each counting phase performed (the algorithmic units the
 * phases are measured against).  Phases:
 *   0 prepass   relabelling by degree, re-sorted lists, work lists
 *   1 cliques   Step 1 and Step 2a (triangles, 4-cliques)
 *   2 cyc-light Step 2b for vertices with few wedges
 *   3 cyc-dense Step 2b for the costliest vertices, counted in slabs of hubs
 *               by passes over all rows (global counts only)
 *   4 cyc-heavy Step 2b for the other vertices with many wedges
 *   5 per-edge  per-edge 4-cliques and D_e (only with per_edge_out)
 *   6 step3     Step 3 sums and their reduction
 *   7 vertex    per-vertex counts from the per-edge arrays (only in
 *               graphlet_count_vertex)
 * Enabling costs one event record per phase; results are unchanged.
 */
#define GC_PHASES 8
typedef struct gc_timing {
  double ms[GC_PHASES];      /* device time per phase, milliseconds */
  uint64_t clique_entries;   /* upper-list entries scanned by phase 1 */
  uint64_t wedges_light;     /* wedges aggregated by phase 2 */
  uint64_t wedges_heavy;     /* wedges aggregated by phase 4 */
  int64_t heavy_items;       /* work items of phase 4 */
  uint64_t wedges_dense;     /* wedges of the hubs of phase 3 */
  int64_t dense_hubs;        /* hubs counted by phase 3 */
  /* Vertices u of phase 1 by k = |U(u)|, the neighbours after u in the
   * degree order (each class is one kernel shape): [0] k <= 64, [1] <= 256,
   * [2] <= 512, [3] <= 1088, [4] k > 1088 (rows in global memory); [5] the
   * vertices of [3] with k > 896, whose symmetric rows the per-edge pass
   * keeps in global memory (with per_edge_out, local or vertex outputs). */
  int64_t clique_class[6];
} gc_timing;

void graphlet_timing_enable(int on);
int graphlet_last_timing(gc_timing *out);

/*
 * Serving loop (continuous batching).  Graphs are submitted from HOST memory;
 * each is copied into the server, admitted onto the device when a worker
 * slot is free and its footprint (CSR + workspace bound) fits the remaining
 * device-memory budget, counted with graphlet_count on the worker's own HIP
 * stream, and its CSR freed when its counts are on the host.  Requests that
 * arrive while others run are admitted as slots and memory free up, so the
 * work of several requests overlaps on the device; a request's result is the
 * same as a standalone graphlet_count of its graph.  Small graphs (at most
 * GC_BATCH_MAX_N vertices) go to the batch lane instead: every pending small
 * request, up to the lane's capacity (1024 graphs, 2^18 vertices, 2^22
 * adjacency entries), is counted in one graphlet_count_batched call on the
 * lane's own stream, while requests arriving meanwhile wait for the next
 * batch; the lane's buffers (about 17 MB of device memory, and pinned host
 * memory) are charged to the budget for the server's life, and the lane is
 * left out when they would take more than a quarter of the budget, or with
 * the flag GC_SERVE_NO_LANE.
 *   gc_server_create   budget in bytes of device memory, slots = concurrent
 *                      requests (1..64, one stream each), flags as for
 *                      graphlet_count (GC_VALIDATE checks every request).
 *                      NULL on bad arguments (gc_server_last_error()).
 *   gc_server_submit   host CSR (gc_csr contract; copied before returning).
 *                      Returns a request id > 0, or GC_EINVAL for a malformed
 *                      CSR, or GC_ENOMEM when the graph alone exceeds the
 *                      budget.  Rejected requests never reach the device.
 *   gc_server_poll     1 done (out_counts filled, latency = completion minus
 *                      submission, ms), 0 still pending or running, < 0 the
 *                      request failed (its error code; others are unaffected)
 *   gc_server_wait     as poll, blocking until the request ends
 *   gc_server_cancel   a pending request is dropped; a running one finishes
 *                      on the device and its result is discarded (a running
 *                      update is then not applied: the graph and its counts
 *                      stay as they were).  Either way the request ends
 *                      CANCELLED, unless it had already finished.
 *   gc_server_release  forgets a finished request (its id becomes invalid)
 *   gc_server_stats    counters, latency percentiles over completed requests
 *                      and throughput since creation or the last reset
 *   gc_server_destroy  cancels pending requests, waits for running ones
 *                      and frees registered graphs
 * Resident graphs, for the localized updates of Section 6.3 served against a
 * graph the server keeps:
 *   gc_server_register  host CSR (copied; checked as with GC_VALIDATE), kept
 *                      on the device with room for nnz / 8 more entries (at
 *                      least 512 edges) until gc_server_unregister.  Returns
 *                      the graph id > 0, which is also the id of the request
 *                      that counts it (poll / wait give the initial counts),
 *                      or GC_EINVAL / GC_ENOMEM as gc_server_submit.  Its
 *                      device memory stays charged to the budget while it is
 *                      registered.
 *   gc_server_update   request: insert (insert = 1) or delete (0) the edge
 *                      (u, v) of a registered graph.  Returns a request id;
 *                      its result (poll / wait) is the graph's 17 counts after
 *                      the change.  Updates of one graph run one at a time in
 *                      submission order, after its registration.  A failed
 *                      update (edge already present / absent, graph full)
 *                      leaves the graph and its counts unchanged.
 *   gc_server_graph_counts  1 and the current counts, 0 if the registration
 *                      has not been counted yet, < 0 for an unknown graph
 *   gc_server_unregister  cancels the graph's pending updates, waits for a
 *                      running one, frees the graph.  Cancelling a pending
 *                      registration (gc_server_cancel on the graph id) also
 *                      cancels the graph's queued updates and refuses new
 *                      ones; a running registration completes.
 * Calls may come from any thread.  The server owns its copies of submitted
 * graphs; it keeps no caller pointer.
 */
typedef struct gc_server gc_server;
typedef struct gc_serve_stats {
  int64_t submitted, completed, failed, rejected, cancelled, pending, running;
  size_t bytes_in_use, bytes_peak, budget;
  double p50_ms, p99_ms, mean_ms, elapsed_s, graphs_per_s, edges_per_s;
  int64_t batches;  /* batched calls of the batch lane */
  int64_t batched;  /* requests counted by them */
} gc_serve_stats;

gc_server *gc_server_create(size_t hbm_budget, int slots, uint32_t flags);
int64_t gc_server_submit(gc_server *s, int64_t n, int64_t nnz, const int32_t *row_ptr,
                         const int32_t *col);
int gc_server_poll(gc_server *s, int64_t id, gc_u128 out_counts[17], double *latency_ms);
int gc_server_wait(gc_server *s, int64_t id, gc_u128 out_counts[17], double *latency_ms);
int gc_server_cancel(gc_server *s, int64_t id);
int gc_server_release(gc_server *s, int64_t id);
int gc_server_stats(gc_server *s, gc_serve_stats *out);
int gc_server_reset_stats(gc_server *s);
void gc_server_destroy(gc_server *s);
int64_t gc_server_register(gc_server *s, int64_t n, int64_t nnz, const int32_t *row_ptr,
                           const int32_t *col);
int64_t gc_server_update(gc_server *s, int64_t graph, int32_t u, int32_t v, int insert);
int gc_server_graph_counts(gc_server *s, int64_t graph, gc_u128 out_counts[17]);
int gc_server_unregister(gc_server *s, int64_t graph);
const char *gc_server_last_error(void);

/* Message of the calling thread's most recent error ("" if none). */
const char *graphlet_last_error(void);

/* Library version string. */
const char *graphlet_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GRAPHLET_H */
