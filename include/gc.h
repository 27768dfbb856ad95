/*
 * gc.h -- C ABI of libgc: exact triangle counting, per-edge triangle support,
 * k-truss and truss decomposition on one AMD Instinct MI355X (gfx950).
 *
 * The operations follow the definitions of Samsi et al., "Static Graph
 * Challenge: Subgraph Isomorphism" (2017):
 *   - input graph: an edge list of integer vertex ids, weights 1, self-loops
 *     removed, directed edges symmetrised (Sec. II);
 *   - triangle count: the number of sets of three mutually adjacent vertices
 *     (Sec. III-A; Alg. 3 computes it as a masked product);
 *   - support of an edge: the number of triangles containing it, i.e. the
 *     number of common neighbours of its endpoints (Sec. III-B, the row sums of
 *     (EA == 2));
 *   - k-truss: the largest subgraph in which every edge lies in at least k-2
 *     triangles of that subgraph (Sec. III-B, Alg. 4);
 *   - truss decomposition: the k-truss for every k >= 2 (Sec. III-B, last
 *     paragraph).
 * All arithmetic is integer and exact.
 *
 * Conventions shared by every call
 *   Pointers prefixed d_ are device pointers (hipMalloc'd or torch tensors on
 *   the current device); h_ are host pointers.  The caller owns every buffer
 *   it passes; the library owns gc_graph handles and the device memory inside
 *   them until gc_graph_free.
 *
 *   Canonical edge order: after normalisation the graph is the set of pairs
 *   (u, v) with u < v, sorted lexicographically; the position of a pair is its
 *   edge id (the row index of the incidence matrix E of Sec. III-B).  Every
 *   per-edge output (support, k-truss mask, truss number) is written in that
 *   order, so results are bit-comparable with a memcmp.
 *
 *   Streams: every call is ordered on `stream` (a hipStream_t; NULL is the
 *   null stream).  Calls that return a host scalar synchronise the stream
 *   before returning.  Device inputs must stay valid until the stream has
 *   passed the call.
 *
 *   Errors: calls never abort and no C++ exception leaves them.  They return
 *   GC_OK (0) or a negative status;
 *   gc_last_error() gives a thread-local description of the last failure.  On
 *   failure, outputs are unspecified and the handle stays valid.
 *
 *   Threading: one call at a time per handle (calls share the handle's device
 *   workspace); different handles are independent.
 *
 *   Limits: n_vertices <= 2^31 - 1; the number of input pairs and the number of
 *   edges must be < 2^31 (GC_EOVERFLOW otherwise).  Counts are int64.
 */
#ifndef GC_H_
#define GC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gc_graph gc_graph;
typedef int32_t gc_status;
typedef void *gc_stream; /* a hipStream_t */

#define GC_OK 0
#define GC_EINVAL (-1)     /* null pointer, negative size, bad flag, k < 2 */
#define GC_ERANGE (-2)     /* a vertex id outside [0, n_vertices) */
#define GC_ECAPACITY (-3)  /* output buffer shorter than required */
#define GC_ENOMEM (-4)     /* device or host allocation failed, or a host
                              thread could not start */
#define GC_EDEVICE (-5)    /* a HIP runtime error */
#define GC_EOVERFLOW (-6)  /* a size beyond the limits above */

/* gc_build_csr flags */
#define GC_INPUT_ONE_BASED 0x1u /* ids are 1..n as in the challenge's files
                                   (Sec. II); 1 is subtracted on input */

/* Build a graph handle from raw edge pairs (Sec. II).
 * d_src[i], d_dst[i] (i < n_pairs, device, int32) are the endpoints of pair i.
 * Pairs may come in any order and direction and may repeat; self-loops are
 * dropped and {u, v} / {v, u} / repeats collapse to one undirected edge.
 * On success *out receives a new handle (free with gc_graph_free); on failure
 * *out is set to NULL.  An id outside [0, n_vertices) (after the optional
 * 1-based shift) gives GC_ERANGE.  Synchronises `stream`. */
gc_status gc_build_csr(const int32_t *d_src, const int32_t *d_dst,
                       int64_t n_pairs, int32_t n_vertices, uint32_t flags,
                       gc_stream stream, gc_graph **out);

/* Sizes of a handle: vertices, undirected edges m (canonical edge count, the
 * number of rows of the incidence matrix E of Sec. III-B) and the device
 * bytes the handle currently holds.  Any output pointer may be
 * NULL. */
gc_status gc_graph_info(const gc_graph *g, int64_t *n_vertices,
                        int64_t *n_edges, int64_t *device_bytes);

/* Copy the canonical edge list (u < v, lexicographic; Sec. II / III-B rows of
 * E) into d_u[0..m), d_v[0..m) (device, int32).  cap < m gives GC_ECAPACITY. */
gc_status gc_graph_edges(gc_graph *g, int32_t *d_u, int32_t *d_v, int64_t cap,
                         gc_stream stream);

/* Copy the degree-oriented CSR used by the kernels.  Vertex r of the CSR is
 * the vertex of rank r in the strict order (degree, id); each edge is stored
 * once, from its lower-ranked to its higher-ranked endpoint (the strict
 * lower-triangular part L of Alg. 3 in that order).
 *   d_rank[0..n)        rank of each original vertex id
 *   d_row_ptr[0..n+1)   row offsets
 *   d_col[0..m)         rank of the head of each oriented edge, rows sorted
 *   d_eid[0..m)         canonical edge id of each oriented edge
 * Any output may be NULL.  cap_n < n+1 or cap_m < m gives GC_ECAPACITY. */
gc_status gc_graph_oriented(gc_graph *g, int32_t *d_rank, int32_t *d_row_ptr,
                            int32_t *d_col, int32_t *d_eid, int64_t cap_n,
                            int64_t cap_m, gc_stream stream);

/* Triangle count (Sec. III-A; Alg. 3's sum(A .* (L U)) / 2): the number of
 * vertex triples that are pairwise adjacent, written to *h_count (host).
 * Synchronises `stream`. */
gc_status gc_triangle_count(gc_graph *g, gc_stream stream, int64_t *h_count);

/* Per-edge support (Sec. III-B: row sums of (EA == 2); Alg. 2's C(u, v)):
 * d_support[e] = number of triangles containing canonical edge e, for
 * e < m (device, int32).  cap < m gives GC_ECAPACITY. */
gc_status gc_edge_support(gc_graph *g, int32_t *d_support, int64_t cap,
                          gc_stream stream);

/* Largest graph (undirected edges) gc_edge_support_noalloc accepts. */
#define GC_NOALLOC_MAX_EDGES (1 << 24)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * output as gc_edge_support, computed by the same kernels, with no device or
 * host allocation.  The slot-order counts live in a device array of the
 * library (4 * GC_NOALLOC_MAX_EDGES bytes = 64 MiB), which each GPU the
 * library runs on holds until the process ends; the handle's work units are
 * built by gc_build_csr.  Every call on one GPU shares that array and clears
 * the part it uses: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  m >
 * GC_NOALLOC_MAX_EDGES or cap < m gives GC_ECAPACITY.  Does not synchronise
 * `stream`. */
gc_status gc_edge_support_noalloc(gc_graph *g, int32_t *d_support, int64_t cap,
                                  gc_stream stream);

/* k-truss (Sec. III-B, Alg. 4): d_in_truss[e] = 1 if canonical edge e belongs
 * to the maximal k-truss, else 0 (device, uint8, m entries).  The result is
 * the fixed point of Alg. 4 (drop every edge with support < k-2 until none
 * is dropped); it is reached by peeling: support is counted once, and the
 * levels 3 .. k of the truss decomposition remove edges in rounds while the
 * support of the survivors is decremented per destroyed triangle.  With the
 * environment variable GC_TRUSS_METHOD=rounds, Alg. 4's own rounds are run
 * instead (support recounted on the compacted remaining edges each round);
 * both give the same set.  *h_m_k (host, may be NULL) receives the number of
 * edges in the k-truss.  k < 2 gives GC_EINVAL; k = 2 keeps every edge.
 * Synchronises `stream`. */
gc_status gc_ktruss(gc_graph *g, int32_t k, uint8_t *d_in_truss, int64_t cap,
                    gc_stream stream, int64_t *h_m_k);

/* Count strategies per degree bin (the 5 bins split middle vertices by
 * out-degree: <= 32, <= 256, <= 2048, <= 8192, larger).  A strategy is only
 * a schedule for the intersections behind the masked product of Alg. 3
 * (Sec. III-A): it chooses how N+(b) is staged and probed, not what is
 * counted.
 *   0 linear-probing LDS hash table, load <= 1/2
 *   1 linear-probing LDS hash table, load <= 1/4
 *   2 binary search in the sorted row in HBM (the only one for the last bin)
 *   3 bucketed LDS hash table (4 slots per 16-byte bucket), load <= 1/2
 *   4 bucketed LDS hash table, load <= 1/4
 *   5 a group of lanes per work unit (16 in bin 0, a wavefront in bin 1)
 *     with its own LDS table, one lane per in-edge (bins 0 and 1 only: many
 *     small units)
 *   6 merge: the group copies the sorted N+(b) to LDS and each lane merges
 *     the sorted tail of an in-edge with it by two pointers (bins 0 and 1
 *     only: short lists on both sides)
 * Results never depend on the strategy.  A new handle takes them from the
 * file named by the environment variable GC_AUTOTUNE_CACHE if it exists
 * (lines "<arch> <bin> <strategy> <tile>"), else {0, 0, 0, 0, 2}.
 *
 * Count tiles per degree bin: the in-edges of a middle vertex b are split
 * into work units of at most `tile` in-edges (32, 64 or 128), each staging
 * N+(b) once; smaller units balance the load of vertices with many in-edges
 * across more workgroups at the cost of staging N+(b) more often.  Results
 * never depend on the tile.  Default 128 in every bin. */

/* Autotuner: for each tile (128, 64, 32; the units of every bin rebuilt
 * with it), time every admissible strategy of every bin that has work on
 * this graph (HIP events, first run discarded); keep the fastest (strategy,
 * tile) per bin and, if GC_AUTOTUNE_CACHE is set, write the choices there.
 * h_strategy[5] and h_ms[5*7] (mean ms per bin and strategy at the tile
 * chosen for the bin, row-major by bin; -1 where not run) may be NULL; the
 * chosen tiles are read with gc_graph_count_config.
 * Synchronises `stream`. */
gc_status gc_graph_autotune(gc_graph *g, gc_stream stream, int32_t *h_strategy,
                            float *h_ms);

/* Kernel time of each degree bin's count launch in the last
 * gc_triangle_count on this handle: h_ms[b] (host, first `cap` of 5) in
 * milliseconds, from HIP events recorded around each launch on the call's
 * stream (0 for an empty bin, -1 before any count).  For the measurement of
 * the count against the HBM roofline (Sec. IV-B's rate, per kernel). */
gc_status gc_graph_count_times(const gc_graph *g, float *h_ms, int32_t cap);

/* Set the 5 per-bin strategies (GC_EINVAL if one is not admissible). */
gc_status gc_graph_set_strategy(gc_graph *g, const int32_t *h_strategy);

/* Set the 5 per-bin count tiles (host array; each 32, 64 or 128, else
 * GC_EINVAL and nothing changes).  The count units are rebuilt on the next
 * gc_triangle_count when a tile changes. */
gc_status gc_graph_set_tile(gc_graph *g, const int32_t *h_tile);

/* The handle's per-bin count strategies and tiles (host arrays of 5; either
 * may be NULL). */
gc_status gc_graph_count_config(const gc_graph *g, int32_t *h_strategy, int32_t *h_tile);

/* Truss decomposition (Sec. III-B, last paragraph): d_truss[e] = the largest
 * k such that canonical edge e belongs to the k-truss (>= 2), and *h_kmax the
 * largest k with a non-empty k-truss (0 for an empty graph, 2 if there are
 * edges but no triangle).  Either output may be NULL.  Synchronises `stream`.
 * Computed by peeling: support is counted once, then each level k removes in
 * rounds every edge whose support falls below k-2, decrementing the support
 * of the survivors once per destroyed triangle.  GC_TRUSS_METHOD=rounds
 * recounts support per round instead (Alg. 4's recompute form).  Two
 * environment variables tune the peeling without changing any result:
 * GC_PEEL_LB_MIN (smallest frontier handled in lane-balanced batches of up
 * to 64 edges per wave; default one edge per wave of the grid) and
 * GC_PEEL_SORT_MIN (smallest first frontier of a level that is sorted by
 * higher endpoint; default 100000, 0 = never).  Device memory: about 26
 * bytes per edge of working state, released on return, and the compacted
 * copies of the CSR (two at most, at most 20 bytes per edge each), which the
 * handle keeps for reuse until gc_graph_free. */
gc_status gc_truss_decomposition(gc_graph *g, int32_t *d_truss, int64_t cap,
                                 gc_stream stream, int32_t *h_kmax);

/* Counters of the incremental support update (Sec. III-B, Alg. 4's update
 * of R) in the last peeling on this handle (gc_truss_decomposition, or
 * gc_ktruss with k > 2 unless GC_TRUSS_METHOD=rounds; first `cap` of 41,
 * host): [0] levels that removed edges, [1] rounds, [2] edges removed over
 * all rounds (= m for a decomposition), [3] largest round, [4] compactions,
 * [5 + i] rounds whose removal count r has floor(log2 r) = i, [37]
 * candidate third vertices examined, [38] of them searched (edge alive),
 * [39] triangles found still present, [40] triangles destroyed (each
 * exactly once).  Edges whose support is 0 when they are peeled have no
 * triangle left and are not scanned; a scan stops once it has found as many
 * present triangles as the edge's support. */
gc_status gc_graph_truss_stats(const gc_graph *g, int64_t *h_stats, int32_t cap);

/* ------------------------------------------------------------------------ */
/* Batches: many independent graphs counted in one launch per degree bin.    */
/* Not in the paper: a throughput layer; every per-graph result is the one   */
/* Sec. III defines for that graph alone.                                    */
/* ------------------------------------------------------------------------ */
typedef struct gc_batch gc_batch;

/* Build one device structure for G independent graphs.  Graph g's raw pairs
 * are d_src/d_dst[h_pair_off[g] .. h_pair_off[g+1]) (device, int32; host
 * offsets, h_pair_off[0] = 0, non-decreasing) with ids in [0, h_nv[g]) (or
 * 1..h_nv[g] with GC_INPUT_ONE_BASED); each graph is normalised as in
 * gc_build_csr.  The graphs become one disjoint union, so the per-graph
 * results of every operation below are those of the graphs taken alone
 * (Sec. III definitions apply graph by graph).  Synchronises `stream`.
 * GC_ERANGE if an id falls outside its own graph. */
gc_status gc_batch_build(const int32_t *d_src, const int32_t *d_dst,
                         const int64_t *h_pair_off, const int32_t *h_nv,
                         int32_t G, uint32_t flags, gc_stream stream,
                         gc_batch **out);

/* Number of graphs, total canonical edges over all graphs, device bytes. */
gc_status gc_batch_info(const gc_batch *b, int32_t *n_graphs, int64_t *n_edges,
                        int64_t *device_bytes);

/* h_off[0..G] (host): the canonical edges of graph g are positions
 * [h_off[g], h_off[g+1]) of every per-edge batch output, in graph g's own
 * canonical order. */
gc_status gc_batch_edge_offsets(const gc_batch *b, int64_t *h_off);

/* The union graph behind a batch (owned by the batch; do not free).  Any
 * gc_graph call may be applied to it. */
gc_graph *gc_batch_graph(gc_batch *b);

/* Per-graph triangle counts (Sec. III-A) into d_T[0..G) (device, int64).
 * The zeroing and the per-bin count launches are captured into a HIP graph on
 * the first call and replayed afterwards.  Stream-ordered, no host sync. */
gc_status gc_batch_triangle_count(gc_batch *b, int64_t *d_T, gc_stream stream);

/* Per-edge support (Sec. III-B) of all graphs into d_support (device, int32,
 * Σm entries, batch edge order).  cap < Σm gives GC_ECAPACITY. */
gc_status gc_batch_edge_support(gc_batch *b, int32_t *d_support, int64_t cap,
                                gc_stream stream);

/* k-truss of every graph (Sec. III-B, Alg. 4): d_mask[e] in batch edge order
 * (device, uint8, Σm entries) and d_mk[g] = edges in graph g's k-truss
 * (device, int64, G entries).  For 3 <= k <= 66 the launches (support, then
 * levels 3 .. k of the peeling with a fixed number of rounds each, the mask
 * and the per-graph counts) are recorded into a HIP graph on the first call
 * for that k and replayed afterwards; if a level needed more rounds than
 * were recorded, the call peels eagerly instead (same result) and the next
 * call records twice the rounds (after a level that 1024 recorded rounds
 * did not finish, the batch peels eagerly on every call).  Rounds first
 * recorded per level: 32, or the environment variable GC_BATCH_KTRUSS_ROUNDS
 * (1 .. 4096) read when the batch is built.  cap < Σm gives GC_ECAPACITY.  Synchronises `stream`. */
gc_status gc_batch_ktruss(gc_batch *b, int32_t k, uint8_t *d_mask, int64_t cap,
                          int64_t *d_mk, gc_stream stream);

/* Autotuner of a batch, as gc_graph_autotune (strategies listed there):
 * times every admissible count strategy per degree bin on the whole batch,
 * keeps the fastest, writes GC_AUTOTUNE_CACHE if set.  h_strategy[5] and
 * h_ms[5*7] may be NULL.  Results never depend on the choice. */
gc_status gc_batch_autotune(gc_batch *b, gc_stream stream, int32_t *h_strategy,
                            float *h_ms);

/* Force the count strategy of each of the 5 bins (GC_EINVAL if a strategy is
 * not admissible for its bin; the last bin admits only 2).  Drops the
 * captured HIP graph. */
gc_status gc_batch_set_strategy(gc_batch *b, const int32_t *h_strategy);

/* Release a batch and its union graph (NULL is a no-op). */
void gc_batch_free(gc_batch *b);

/* ------------------------------------------------------------------------ */
/* Serving: queries on registered graphs with continuous batching.          */
/* Not in the paper: a serving layer whose queries return the Sec. III-A     */
/* triangle count or the size of a Sec. III-B k-truss.                       */
/* ------------------------------------------------------------------------ */
typedef struct gc_server gc_server;

#define GC_PENDING 1 /* gc_server_poll: the request has not completed yet */

/* A query on a registered graph: kind 0 = triangle count (Sec. III-A),
 * kind 1 = number of edges in the k-truss (Sec. III-B), k >= 2. */
typedef struct {
  int32_t graph_id;
  int32_t kind;
  int32_t k;
  int32_t reserved;
} gc_request;

/* Outcome of a query: status (GC_OK or an error), the value (triangles or
 * k-truss edges), the graph's edge count m, and CLOCK_MONOTONIC timestamps in
 * seconds: submission, start on the device, completion. */
typedef struct {
  int32_t status;
  int32_t kind;
  int64_t value;
  int64_t edges;
  double t_submit;
  double t_start;
  double t_done;
} gc_result;

/* Start a server on the current device with an HBM budget in bytes.  A
 * scheduler thread keeps built graphs resident (evicting idle ones, least
 * recently used first, when the budget needs room), admits a request only
 * when the budget can hold its graph's build (builds run on a thread and
 * stream of their own), and runs every triangle-count request whose graph is
 * resident in one batched launch per degree bin, forming the next batch from
 * whatever arrived while the previous one ran.  A worker thread runs every
 * queued k-truss query with the same k as one batch: the graphs' CSRs are
 * concatenated on the device into their disjoint union, which is peeled
 * once; each graph's k-truss is its slice of the union's.  The union and its
 * peeling state are charged to the budget while the batch runs. */
gc_status gc_server_create(int64_t budget_bytes, gc_server **out);

/* 0 = continuous batching (default); 1 = one request at a time in arrival
 * order with the same cache, each k-truss by gc_ktruss on its graph's own
 * handle (the per-call comparison). */
gc_status gc_server_set_mode(gc_server *s, int32_t mode);

/* Register a graph: raw pairs in host memory (copied), ids in
 * [0, n_vertices).  GC_ENOMEM if its build and a k-truss batch of it alone
 * cannot fit the budget together. */
gc_status gc_server_add_graph(gc_server *s, const int32_t *h_src,
                              const int32_t *h_dst, int64_t n_pairs,
                              int32_t n_vertices, int32_t *graph_id);

/* Queue a query; *ticket identifies it.  Thread-safe. */
gc_status gc_server_submit(gc_server *s, const gc_request *req, int64_t *ticket);

/* GC_OK with *out filled (the ticket is then released), or GC_PENDING. */
gc_status gc_server_poll(gc_server *s, int64_t ticket, gc_result *out);

/* Block until the query completes, then as gc_server_poll. */
gc_status gc_server_wait(gc_server *s, int64_t ticket, gc_result *out);

/* h_stats[12]: completed, count batches, largest count batch, builds,
 * evictions, bytes charged now, peak bytes charged, admissions deferred for
 * memory, resident graphs, budget, k-truss batches, largest k-truss batch. */
gc_status gc_server_stats(gc_server *s, int64_t *h_stats);

/* Stop the threads and release every resident graph (NULL is a no-op). */
void gc_server_destroy(gc_server *s);

/* ------------------------------------------------------------------------ */
/* Edge files (host).                                                        */

#define GC_FILE_AUTO 0 /* Matrix Market if the file starts with its banner, else TSV */
#define GC_FILE_TSV 1  /* lines "u<TAB>v<TAB>w", ids 1..n, w ignored              */
#define GC_FILE_MMIO 2 /* Matrix Market coordinate (pattern/integer/real), 1-based */

/* Read an edge file in one of the two formats the paper's data come in
 * (Sec. II: TSV triples u, v, 1 with ids 1..n, and MMIO).  Host code; reading
 * is outside the timed path (Sec. IV-B).
 * TSV: blank lines and lines starting with '#' or '%' are skipped; fields are
 * separated by tabs or spaces; a third field (the weight) is ignored.
 * MMIO: the banner must say "coordinate" (field pattern, integer or real);
 * the size line gives n = max(rows, cols) and the entry count, which must
 * match the entries present; symmetric files list each edge once (the
 * normalisation of gc_build_csr symmetrises anyway).
 * Call with h_src = h_dst = NULL to get *n_pairs (and *n_vertices for MMIO;
 * -1 for TSV, whose n is only known after parsing); then with host arrays of
 * cap >= *n_pairs entries, which receive the pairs with ids converted to
 * 0-based (ready for gc_build_csr without GC_INPUT_ONE_BASED), and *n_vertices =
 * the largest id (TSV) or max(rows, cols) (MMIO).  The caller owns the arrays.
 * Errors: unreadable file, malformed line, bad banner or size line, or an
 * entry count that differs from the size line -> GC_EINVAL; id 0, or above
 * the MMIO size -> GC_ERANGE; an id above 2^31 - 1 -> GC_EOVERFLOW; cap too
 * small -> GC_ECAPACITY.  The message names the offending line. */
gc_status gc_read_edges(const char *path, int32_t format, int32_t *h_src, int32_t *h_dst,
                        int64_t cap, int64_t *n_pairs, int64_t *n_vertices);

/* Release a handle and its device memory (NULL is a no-op). */
void gc_graph_free(gc_graph *g);

/* Text for a status code (static storage). */
const char *gc_status_str(gc_status status);

/* Thread-local description of the last failure on this thread ("" if none). */
const char *gc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GC_H_ */
