/*
 * tm.h -- exact delta-temporal motif counting on one AMD Instinct MI355X
 * (gfx950), C ABI.
 *
 * Problem (the paper's Problem 1, Section III): given a temporal graph -- a
 * list of directed, timestamped edges (src, dst, t) (Definition 1) -- and a
 * window delta, count exactly the instances of every 2- and 3-node, 3-edge
 * delta-temporal motif (Definitions 2 and 3): three distinct edges taken in
 * chronological order E1 < E2 < E3 with t(E3) - t(E1) <= delta whose static
 * graph has at most three nodes.  There are 36 such motifs: 4 pair, 24 star
 * and 8 triangle motifs (Section IV's categorisation).
 *
 * Conventions shared by every entry point:
 *   - Edge id = input row index.  Edges are totally ordered by (t, id): equal
 *     timestamps are ordered by id.  Every delta test uses t alone and is
 *     inclusive (t_last - t_first <= delta).
 *   - Direction bits: o = 0 (edge leaves the center), in = 1.
 *   - Raw counters, 56 x uint64 (the paper's counters, Sections IV-A/IV-B):
 *       [ 0,24) Star[Type][d1][d2][d3]  Type I/II/III = position of the edge
 *               whose node pair is not shared (quadruple counter)
 *       [24,32) Pair[d1][d2][d3]        each pair instance seen from both of
 *               its nodes (triple counter)
 *       [32,56) Tri[Type][d_i][d_j][d_k] each triangle instance seen from its
 *               three vertices; Type I/II/III = the far edge e_k before e_i,
 *               between e_i and e_j, after e_j; d_k relative to e_i's
 *               neighbour (quadruple counter)
 *   - Motif counts, 36 x uint64, out[6*(i-1) + (j-1)] = M_ij.  The cells the
 *     paper's text fixes are honoured (M24 = Star[I,in,o,in], M63 =
 *     Star[III,o,o,in], M25, M26 = time-respecting 3-cycle, M46, M55, M56,
 *     M65, M66); the remaining placement is this library's convention:
 *       stars:     row 1 + 2*Type + [d3 = in],  col 1 + 2*[d2 = o] + [d1 = in]
 *       triangles: Tri[I,a,b,c] class; col 5 + [b = o];
 *                  row by ([a = b],[c = b]): TT 1, FF 2, FT 3, TF 4
 *       pairs:     Pair[o,d2,d3]: (o,o) M55, (in,in) M56, (in,o) M65, (o,in) M66
 *   - Status codes: every function returns TM_OK or a negative TM_E* code;
 *     nothing throws across the ABI.  On error, output buffers are left
 *     untouched.  tm_strerror() names a code; tm_last_error() gives the
 *     calling thread's last detailed message.
 */
#ifndef TM_H
#define TM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tm_graph tm_graph;

enum {
    TM_OK = 0,
    TM_EINVAL = -1,     /* bad argument or input (see tm_build_graph)          */
    TM_ENOMEM = -2,     /* device allocation failed                             */
    TM_EHIP = -3,       /* HIP runtime error (detail in tm_last_error)          */
    TM_EAGAIN = -4,     /* try again (reserved for queued / pending work)       */
    TM_ENOTFOUND = -5,  /* no such object                                       */
    TM_EINTERNAL = -6   /* a self-check of the counters failed                  */
};

enum { TM_HOST_PTRS = 0, TM_DEVICE_PTRS = 1 };

/* Motif families (the paper's categories, Section IV: stars, pairs,
 * triangles), for tm_count_masked. */
enum { TM_STARS = 1, TM_PAIRS = 2, TM_TRIANGLES = 4, TM_ALL_MOTIFS = 7 };

/* hub_min value (tm_count_raw_tuned, tm_count_batch_raw_ex) that keeps every
 * triangle candidate in the per-candidate kernel. */
#define TM_HUB_OFF 0xffffffffu

/*
 * Build the device-resident graph used by every count (delta-independent).
 *
 * Sequences S_u (Section IV-A: every node's incident edges (t, v, dir) in
 * time order) are built by device radix sorts keyed by (node, t, edge id),
 * together with the node-pair edge sets E_(v,w) of Algorithm 2 (all edges of
 * one unordered node pair, in (t, id) order).
 *
 *   src, dst  int32[m], node ids in [0, n); src[k] != dst[k] (no self-loops)
 *   t         int64[m], |t| < 2^62
 *   m         number of edges, < 2^31 (m = 0 is allowed: all counts are 0)
 *   n_nodes   node count; 0 means max id + 1
 *   flags     TM_HOST_PTRS: the three arrays are host memory (copied in);
 *             TM_DEVICE_PTRS: they are device memory on the current device,
 *             read on `hip_stream` before this call returns
 *   hip_stream hipStream_t used for the build and for later counts on this
 *             graph (NULL = the null stream)
 *   out       receives the graph handle (owned by the library until
 *             tm_graph_free)
 * Ownership: the caller keeps ownership of src/dst/t; they only need to stay
 * valid during the call.
 * Errors: TM_EINVAL for a NULL pointer (m > 0), m >= 2^31, an id outside
 * [0, n), a negative id, a self-loop or |t| >= 2^62; TM_ENOMEM / TM_EHIP.
 */
int tm_build_graph(const int32_t *src, const int32_t *dst, const int64_t *t, uint64_t m,
                   uint32_t n_nodes, int flags, void *hip_stream, tm_graph **out);

/*
 * Batched build: G independent temporal graphs built as one device object
 * (one sort pipeline for all of them).  Graph i's edges are rows
 * edge_off[i] .. edge_off[i+1]-1 of src/dst/t, with node ids local to that
 * graph: in [0, node_count[i]), or any non-negative id when node_count[i] is
 * 0 (then the graph has max id + 1 nodes).  Graphs do not interact: counts
 * are per graph.  edge_off (G + 1 entries, edge_off[0] = 0, non-decreasing)
 * and node_count (G entries) are host arrays; src/dst/t follow `flags` as in
 * tm_build_graph.  Limits: total edges < 2^31, total nodes < 2^31, and
 * ceil(log2 G) plus the largest per-graph time-range bit width <= 64.
 * Errors as tm_build_graph; an invalid edge names its graph in
 * tm_last_error.  tm_build_graph is the case G = 1.
 */
int tm_build_batch(const int32_t *src, const int32_t *dst, const int64_t *t,
                   const uint64_t *edge_off, const uint32_t *node_count, uint32_t G, int flags,
                   void *hip_stream, tm_graph **out);

/* Number of graphs held by g (1 for tm_build_graph). */
uint32_t tm_graph_count(const tm_graph *g);

/*
 * Count every graph of a batch, graph i with window deltas[i] (host array of
 * G values, 0 <= delta < 2^62), into out[i] (36 motif counts) or raw[i] (56
 * raw counters).  All graphs go through the same kernel launches; per-graph
 * results are exact and identical to counting each graph alone.
 */
int tm_count_batch(tm_graph *g, const int64_t *deltas, uint64_t (*out)[36]);
int tm_count_batch_raw(tm_graph *g, const int64_t *deltas, uint64_t (*raw)[56]);

/*
 * tm_count_batch_raw with explicit execution choices; results never depend
 * on them.  run_chunk / tri_lane_max / hub_min as in tm_count_raw_tuned (0 =
 * the graph's tuned values, else the autotuner table's, else defaults);
 * use_graph = 1 replays the count as one captured hipGraph (captured on the
 * first call for these parameters and kept with the graph), 0 launches the
 * kernels one by one.  tm_count_batch / tm_count_batch_raw use the graph.
 */
int tm_count_batch_raw_ex(tm_graph *g, const int64_t *deltas, uint32_t run_chunk,
                          uint32_t tri_lane_max, uint32_t hub_min, int use_graph,
                          uint64_t (*raw)[56]);

/*
 * Autotuner: times the count of g (graph i with deltas[i]) over partition
 * parameters (run_chunk with tri_lane_max on a grid, then hub_min with those
 * fixed), keeps the fastest on g (used by later counts that pass 0) and in a
 * process-wide table keyed by the graph's shape (later graphs of that shape
 * default to it).  Outputs (any may be NULL): the chosen run_chunk,
 * tri_lane_max, hub_min and the count's time in milliseconds.
 */
int tm_autotune(tm_graph *g, const int64_t *deltas, uint32_t *run_chunk, uint32_t *tri_lane_max,
                uint32_t *hub_min, float *best_ms);

/*
 * tm_autotune for the several-window count of one graph (tm_count_multi):
 * times one pass over the largest min(k, 4) of the k windows deltas (host
 * array, 0 <= delta < 2^62, 1 <= k <= TM_MAX_DELTAS), on the same grid, and
 * keeps the fastest as tm_autotune does.  TM_EINVAL for a batch of several
 * graphs, k out of range or a bad delta.
 */
int tm_autotune_multi(tm_graph *g, const int64_t *deltas, uint32_t k, uint32_t *run_chunk,
                      uint32_t *tri_lane_max, uint32_t *hub_min, float *best_ms);

/* Release a graph and its device memory.  NULL is ignored. */
void tm_graph_free(tm_graph *g);

/*
 * Exact counts of the 36 motifs for window delta (blocking; one 448-byte
 * device-to-host copy at the end).  delta must satisfy 0 <= delta < 2^62;
 * delta = 0 counts only triples with equal timestamps.  out: caller-owned
 * host memory, 36 x uint64.  TM_EINTERNAL if the merge self-checks fail.
 * TM_EINVAL if g holds a batch of several graphs (use tm_count_batch).
 * Concurrent calls on one graph are allowed; they run one after another.
 */
int tm_count(tm_graph *g, int64_t delta, uint64_t out[36]);

/*
 * tm_count restricted to some motif families.  The problem statement lets
 * users pick the motif types they need (Section III); the paper times its
 * pair-only and triangle-only variants separately (Section V).
 * families: a nonzero OR of TM_STARS (the 24 star cells), TM_PAIRS (the 4
 * pair cells) and TM_TRIANGLES (the 8 triangle cells).  The selected cells
 * equal tm_count's; the others are 0.  Kernels that only serve unselected
 * families do not run: triangles only skip the star/pair sweeps, stars and
 * pairs only skip the triangle kernels, pairs only also skip the Star_I
 * sweep.  TM_EINVAL for families == 0 or bits beyond TM_ALL_MOTIFS; other
 * errors as tm_count.
 */
int tm_count_masked(tm_graph *g, int64_t delta, uint32_t families, uint64_t out[36]);

/*
 * Counts of one graph for k windows in one call (the paper's experiments
 * sweep delta, Section V): out[i] (36 motif counts) or raw[i] (56 raw
 * counters) for deltas[i] (host array, 0 <= delta < 2^62, any order,
 * repeats allowed), 1 <= k <= TM_MAX_DELTAS.  The windows are taken in
 * increasing order, up to four nested windows per pass: one window search per
 * entry for all of them, one triangle matching at the largest, each match
 * filed under the smallest window that holds it, and the star/pair sweeps once
 * per window.  Each out[i] equals tm_count(g, deltas[i]).  TM_EINVAL for a
 * batch of several graphs, k out of range or a bad delta; other errors as
 * tm_count.
 */
#define TM_MAX_DELTAS 1024
int tm_count_multi(tm_graph *g, const int64_t *deltas, uint32_t k, uint64_t (*out)[36]);
int tm_count_multi_raw(tm_graph *g, const int64_t *deltas, uint32_t k, uint64_t (*raw)[56]);

/*
 * Four-node three-edge motifs of one graph at window delta, the higher-order
 * extension the paper leaves to future work (Section VI: more centers and
 * bigger counters).  An instance is three distinct edges E1 < E2 < E3 in the
 * (t, id) order with t(E3) - t(E1) <= delta whose static graph is connected
 * on exactly four nodes (Definitions 2-3 and Problem 1 with four nodes): a
 * star (one node c on all three edges) or a path v0 - v1 - v2 - v3.
 *   out[0 .. 8)   star [d1][d2][d3]: d_k = 0 if E_k leaves c, 1 if it enters c
 *   out[8 .. 32)  path 8 + r * 8 + f1 * 4 + f2 * 2 + f3: r = 0, 1, 2 the
 *                 chronological position of the middle edge {v1, v2}; the
 *                 path is read from the end edge that comes first ({v0, v1});
 *                 f_k = 1 if E_k points from v_i to v_i+1, else 0
 * raw (may be NULL) receives the 56 raw three-edge counters of the same
 * delta, which the count needs anyway: stars are the ordered triples of one
 * node's edges less the three-node stars and pairs at that node; paths are
 * the choices (middle edge, one more edge at each end) less the triangles,
 * three-node stars and pairs those choices also form.  Host outputs; the
 * graph's stream; TM_EINVAL for a batch of several graphs or a bad delta;
 * TM_EINTERNAL if a correction exceeds its sum (an internal inconsistency,
 * never expected); other errors as tm_count.
 */
int tm_count4(tm_graph *g, int64_t delta, uint64_t raw[56], uint64_t out[32]);

/* The paper's raw counters (layout above), 56 x uint64, for window delta. */
int tm_count_raw(tm_graph *g, int64_t delta, uint64_t raw[56]);

/*
 * tm_count_raw with explicit work partitioning; the result never depends on
 * these, only the schedule does.  0 = the graph's tuned value, else the
 * autotuner table's, else the default.
 *   run_chunk  node-pair edges (elements) per thread of the star/pair
 *              kernel, which counts every element independently (1 .. 64;
 *              larger values are taken as 64)
 *   tri_lane_max  window products (|W_src| * |W_dst|) up to this are counted
 *              by one lane, larger ones by a whole wavefront
 *   hub_min    triangle candidates (first edges, Algorithm 2's triangle
 *              search) whose larger window W holds at least hub_min entries
 *              and whose smaller one fewer than 2048 are matched by slices
 *              of S_u: each slice loads the union of its windows into
 *              on-chip memory once, instead of once per candidate.
 *              TM_HUB_OFF: never.  Default 32.
 */
int tm_count_raw_tuned(tm_graph *g, int64_t delta, uint32_t run_chunk, uint32_t tri_lane_max,
                       uint32_t hub_min, uint64_t raw[56]);

/*
 * tm_count without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as tm_count for a graph of
 * one member (TM_EINVAL for a batch).  The count's workspace is carved from
 * one fixed device array of 256 MiB that the library holds on every device
 * it runs on until the process ends (enough for graphs of about 2-3 million
 * edges); a graph whose workspace would not fit is refused with TM_ENOMEM
 * and tm_last_error gives the bytes it would need.  Nothing is allocated on
 * the device or pinned on the host.  Calls on one device share that array:
 * the library runs them one at a time within a process (each returns only
 * after its count is done), so overlapping calls from several threads wait
 * for each other; the array keeps the last call's contents, and every count
 * writes what it reads first.
 */
int tm_count_noalloc(tm_graph *g, int64_t delta, uint64_t out[36]);
/* Device allocations the library has served so far, cached blocks included
 * (a test aid: tm_count_noalloc leaves it unchanged). */
uint64_t tm_debug_alloc_calls(void);

/*
 * Merge raw counters into the 36 motif counts (pair cells: the view from the
 * first edge's source; triangle cells: orbit sum / 3).  Returns TM_EINTERNAL,
 * leaving out untouched, if Pair[d] != Pair[not d] or the three triangle
 * views disagree.  Pure host function.
 * For the library's own counts the pair check is a real one (each pair
 * instance is counted once from each endpoint, by separate sweeps), but the
 * triangle check always passes: the kernels count each triangle instance
 * once, as its class, and all three views are derived from that class.  The
 * triangle check guards raw counters that come from elsewhere (for example
 * a per-center implementation of the paper's Algorithm 2).
 */
int tm_merge(const uint64_t raw[56], uint64_t out[36]);

/*
 * Graph facts: n nodes, m edges, number of node pairs with >= 2 edges and the
 * number of edges on them, and the largest S_u length.  Any output pointer
 * may be NULL.
 */
int tm_graph_info(const tm_graph *g, uint32_t *n, uint64_t *m, uint64_t *multi_pairs,
                  uint64_t *multi_pair_edges, uint64_t *max_degree);

/*
 * Copy the sequences S_u back to host memory (test and inspection aid).
 * off: uint32[n+1] (S_u = entries off[u] .. off[u+1]-1); t: int64[2m];
 * nbr: uint32[2m] the other endpoint; dir: uint8[2m] (0 = o, 1 = in);
 * id: uint32[2m] edge id.  All caller-owned host buffers; any may be NULL.
 */
int tm_graph_sequences(const tm_graph *g, uint32_t *off, int64_t *t, uint32_t *nbr,
                       uint8_t *dir, uint32_t *id);

/*
 * Kernel timing (tracing aid).  While enabled, every library kernel launch is
 * bracketed by HIP events on its stream; tm_prof_read synchronises and
 * returns, for entry i (0-based, in first-launch order), the kernel name, the
 * number of launches and their summed duration in milliseconds.  Returns
 * TM_ENOTFOUND past the last entry.  Not thread-safe against concurrent
 * counting; meant for benchmarks.
 */
void tm_prof_enable(int on);
/* Trace only launches of this name (NULL or "": every launch), so that
 * timing one kernel adds two events per launch of it and nothing else. */
void tm_prof_only(const char *name);
void tm_prof_reset(void);
int tm_prof_read(int i, char *name, int name_cap, uint64_t *launches, double *total_ms);

/*
 * Serving.  A server counts requests (graph, delta) as they arrive, on the
 * current device, with continuous batching: a scheduler thread admits
 * pending requests oldest first while at most max_inflight counts are in
 * flight and the device bytes of resident graphs and running counts stay
 * within hbm_budget_bytes; counts run asynchronously and overlap on the
 * device; a request that arrives while others run is admitted as soon as a
 * slot and memory free up.  Anonymous requests admitted together are built
 * as one batch.  Keyed graphs (graph_key != 0) stay resident after their
 * first request (least recently used idle graphs are evicted when the
 * budget is short), so later requests only count.  Results are identical to
 * counting each request alone.
 *
 * tm_server_create: budget > 0, max_inflight > 0, max_queue > 0 (pending
 *   requests beyond it are refused with TM_EAGAIN: back-pressure).
 * tm_submit: graph_key = 0 -> the edges (host arrays, copied before the call
 *   returns; same rules as tm_build_graph) are the request's graph;
 *   graph_key != 0 -> the resident graph of that key, or the edges given
 *   here become it (edges may be NULL if the key is resident or an earlier
 *   request carries them; given edges are ignored for a resident key).
 *   TM_EINVAL for bad arguments, TM_ENOTFOUND for an unknown key without
 *   edges, TM_EAGAIN when the queue is full.  A request that can never fit
 *   the budget completes with TM_ENOMEM; an invalid edge list completes with
 *   TM_EINVAL without affecting other requests.
 * tm_poll: TM_EAGAIN while pending; otherwise the request's final status
 *   (TM_OK: out holds the 36 counts) and the ticket is released; for a
 *   failed request, tm_last_error then gives its message.
 *   times_ns (optional): submit, start (admitted), done, steady-clock ns.
 * tm_wait: as tm_poll but blocks up to timeout_ms.
 * tm_server_stats: [queued, in flight, resident graphs, resident bytes,
 *   in-flight bytes, completed, failed, budget].
 * tm_server_destroy: finishes the counts in flight, drops pending requests
 *   and frees everything.
 */
typedef struct tm_server tm_server;
typedef uint64_t tm_ticket;
int tm_server_create(uint64_t hbm_budget_bytes, uint32_t max_inflight, uint32_t max_queue,
                     tm_server **out);
int tm_submit(tm_server *s, uint64_t graph_key, const int32_t *src, const int32_t *dst,
              const int64_t *t, uint64_t m, uint32_t n_nodes, int64_t delta, tm_ticket *out);
int tm_poll(tm_server *s, tm_ticket tk, uint64_t out[36], uint64_t times_ns[3]);
int tm_wait(tm_server *s, tm_ticket tk, uint64_t out[36], uint64_t times_ns[3],
            uint32_t timeout_ms);
int tm_server_stats(tm_server *s, uint64_t stats[8]);
void tm_server_destroy(tm_server *s);

/*
 * Incremental counts of an append-only edge stream (the frequently updated
 * dynamic graphs of Section I).  Every batch's timestamps must be >= every
 * earlier edge's (ties allowed; the batch's rows follow all earlier rows in
 * id order).  An instance containing a new edge then has a new last edge,
 * and its first edge is at most delta before it (Definition 2), so only the
 * earlier edges with t >= (smallest new t) - delta can take part.  The
 * stream keeps that tail on the device and, per append, builds and counts
 * tail + batch; less the count of the tail alone, that is exactly the
 * instances whose last edge is in the batch.  Summed over all appends it
 * equals tm_count of the whole stream.  The tail is cut to the rows that can
 * still meet a new edge only once at least half of it is stale; between cuts
 * the tail's count is the previous append's, so an append costs one build
 * and count, and a cutting append two.  Device memory follows the edge rate
 * times delta (at most about twice the rows that can meet a new edge, plus a
 * batch).
 *
 * tm_stream_create: delta as in tm_count; n_nodes as in tm_build_graph (an
 *   id bound for every batch, or 0 for none); hip_stream as in
 *   tm_build_graph.  out receives the handle (owned until tm_stream_free).
 * tm_stream_append: src/dst/t/m/flags as in tm_build_graph (m = 0 is a
 *   no-op); the caller keeps the arrays, needed only during the call.
 *   new_counts (36, may be NULL): the instances whose last edge is in this
 *   batch.  TM_EINVAL if the batch's smallest t is below the largest t
 *   appended before, or for tm_build_graph's edge errors (bad id, self-loop,
 *   |t| >= 2^62); the stream is then unchanged.  Calls on one stream run one
 *   after another.
 * tm_stream_totals: counts of every edge appended so far (36, may be NULL),
 *   the number of those edges and of the edges kept in the tail (either may
 *   be NULL).
 * tm_stream_free: releases the stream; NULL is ignored.
 */
typedef struct tm_stream tm_stream;
int tm_stream_create(int64_t delta, uint32_t n_nodes, void *hip_stream, tm_stream **out);
int tm_stream_append(tm_stream *s, const int32_t *src, const int32_t *dst, const int64_t *t,
                     uint64_t m, int flags, uint64_t new_counts[36]);
int tm_stream_totals(tm_stream *s, uint64_t total[36], uint64_t *edges, uint64_t *tail_edges);
void tm_stream_free(tm_stream *s);

/*
 * Failure-path testing.  The radix sorts of tm_build_graph find each tile's
 * place by waiting on the tiles before it (decoupled look-back), and every
 * such wait is bounded: past the bound the build flags the sort as failed
 * and returns TM_EINTERNAL, with every kernel still finishing in bounds.
 * With on != 0, every wait of every later build gives up before it starts,
 * so tests can drive that path from the host; 0 restores the normal bound.
 * Process-wide; not for use while other threads build.
 */
void tm_debug_lookback_giveup(int on);
/*
 * Testing.  Each edge's two positions in the sequences S_u (an index of 2m
 * words) are written straight from the node sort while the index fits the
 * GPU's last-level cache, and built by a partition of (slot, position)
 * pairs and a bucket fill above that.  With on != 0 every later build takes
 * the second way, so that small tests cover it; 0 restores the size rule.
 * Process-wide; not for use while other threads build.
 */
void tm_debug_force_edge_sort(int on);

const char *tm_strerror(int code);
const char *tm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TM_H */
