// Internal declarations of the HIP motif-counting library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "tm.h"

namespace tmc {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per block in the streaming kernels
constexpr int kItems = 16;         // items per thread in a streaming tile
constexpr int kTile = kBlock * kItems;

// Positions inside S_u and the ranks of edges are 32-bit: m < 2^31, 2m < 2^32.
constexpr uint32_t kOrientBit = 0x80000000u;  // pair-list element: src is the smaller node

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
// This thread's last error message.
const std::string &last_error();

#define TM_HIP_TRY(expr)                                                              \
    do {                                                                              \
        hipError_t _e = (expr);                                                       \
        if (_e != hipSuccess) {                                                       \
            ::tmc::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));      \
            return _e == hipErrorOutOfMemory ? TM_ENOMEM : TM_EHIP;                   \
        }                                                                             \
    } while (0)

// ---------------------------------------------------------------- profiler
// Kernel launches go through prof_begin/prof_end so that the optional tracer
// can bracket them with events on their stream.
void prof_begin(const char *name, hipStream_t s);
void prof_end(hipStream_t s);
// While a stream is being captured into a hipGraph the tracer stays silent.
void set_capturing(bool on);
// Launches made while a ProfRow is alive are traced as "<row>:<name>", the
// row naming the step of the counting path they belong to (validate, S_u
// build, pair lists, star/pair, triangles, reduction).
struct ProfRow {
    const char *prev;
    explicit ProfRow(const char *row);
    ~ProfRow();
};

#define TM_LAUNCH(name, kernel, grid, block, shm, stream, ...)                       \
    do {                                                                              \
        ::tmc::prof_begin(name, stream);                                               \
        hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);            \
        ::tmc::prof_end(stream);                                                       \
        hipError_t _le = hipGetLastError();                                           \
        if (_le != hipSuccess) {                                                      \
            ::tmc::set_error(std::string("launch ") + name + ": " + hipGetErrorString(_le)); \
            return TM_EHIP;                                                           \
        }                                                                             \
    } while (0)

// ------------------------------------------------------- device memory
// Caching allocator (mem.hip): blocks are reused across calls; a block freed
// on one stream and reused on another is ordered by an event.
int dev_alloc(void **out, size_t bytes, hipStream_t s);
void dev_free(void *p, hipStream_t s);

// A bump allocator over one cached block; everything taken from it is
// released together (to the cache) at scope exit.
struct Scratch {
    hipStream_t stream = nullptr;
    char *base = nullptr;
    size_t cap = 0, used = 0;
    bool owned = true;  // false: base is fixed device memory, not from the cache
    ~Scratch();
    int reserve(size_t bytes, hipStream_t s);
    template <typename T>
    T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        if (used + bytes > cap) return nullptr;
        T *p = reinterpret_cast<T *>(base + used);
        used += bytes;
        return p;
    }
};

// -------------------------------------------------------------- primitives
// Exclusive scan of n values produced by a loader; out[n] receives the total.
// tmp must hold scan_tmp_count(n) elements of T.
size_t scan_tmp_count(uint64_t n);
int scan_u32_array(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp, hipStream_t s);
int scan_dirbits(const uint32_t *ent_nd, uint32_t *out, uint64_t n, uint32_t *tmp, hipStream_t s);
// Each edge once, from its entry of S at the smaller node, in S order:
// key[i] = the larger node, val[i] = (smaller node, rank | orientation).
int lower_side_pairs(const uint32_t *ent_c, const uint32_t *ent_nd, const uint32_t *ent_r,
                     uint64_t n, uint32_t *key, uint2 *val, uint32_t *tmp, hipStream_t s);
// Stable sort of (larger node, (smaller node, rank | orientation)) pairs on
// key bits [0, bits); *keys / *vals point at the sorted data on return.
int radix_sort_pairs(uint32_t **keys, uint32_t **keys_alt, uint2 **vals, uint2 **vals_alt,
                     uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s);
// Exclusive prefix sums of the two bits of n flag bytes at once: bit 0's in
// the low word of out[i], bit 1's in the high word; out[n] = the totals.
int scan_flag_pairs(const uint8_t *f, uint64_t n, uint64_t *out, uint64_t *tmp, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on bits [0, bits), 8 bits per
// pass, ping-ponging between the two buffers; *keys / *vals point at the
// sorted data on return.  tmp: radix_tmp_bytes(n) bytes, 8-byte aligned.
// err: a device flag the sort sets (and never clears) when a wait of its
// look-back gave up; the sorted data are then invalid.
size_t radix_tmp_bytes(uint64_t n);
// Failure-path testing: make every later look-back wait give up at once.
void set_lookback_giveup(bool on);
// Testing: build every edge-position index by edge_positions, whatever its size.
void set_force_edge_sort(bool on);
// A range [b, e) of work items that all belong to graph g of a batch.
struct Tile {
    uint32_t g, b, e;
};

// An edge carried through the time sort: endpoints and input index.
struct EdgeVal {
    uint32_t src, dst, id;
};

// An incident entry carried through the node sort: timestamp, edge rank and
// (other endpoint << 1 | dir).
struct NodeVal {
    int64_t t;
    uint32_t r, nd;
};
// The same with the timestamp as an offset from a base, used when every
// timestamp of the build lies within 2^32 of the smallest: 12 bytes an
// entry instead of 16 through the node sort's passes.
struct NodeVal32 {
    uint32_t dt, r, nd;
};

// Where the node sort's last pass writes: the sequence arrays S_u directly,
// plus either each edge's two positions (epos[2r + dir], a random write per
// entry: used while epos fits the last-level cache) or, with epos null,
// each entry's slot 2r + dir in entry order, from which edge_positions
// builds epos.
struct SeqOut {
    uint32_t *ent_c;
    int64_t *ent_t;
    uint32_t *ent_nd;
    uint32_t *ent_r;
    uint32_t *epos;
    uint32_t *slot;
    uint64_t n;     // entries (epos slots)
    int64_t tbase;  // NodeVal32: t = tbase + dt
};

// Where the time sort's last pass writes: the arrays by edge rank r (rank =
// position in (graph, t, input index) order): t_r, perm (input index) and
// the two incident entries to sort by node (slot 2r: at src, out; 2r + 1: at
// dst, in).
struct RankOut {
    const int64_t *tmin;  // per graph
    int tbits;            // time bits of the key (>= 64: one graph, no graph bits)
    int64_t *t_r;
    uint32_t *perm;
    uint32_t *nkey;
    NodeVal *nval;      // with nval32 null
    NodeVal32 *nval32;  // else, t - tbase
    int64_t tbase;
};

// hist_name / scatter_name label the sort's kernels for the tracer.
#define TM_RADIX_DECL(NAME, K, V)                                                                \
    int NAME(K **keys, K **keys_alt, V **vals, V **vals_alt, uint64_t n, int bits, void *tmp,   \
             uint32_t *err, hipStream_t s, const char *hist_name, const char *scatter_name);
TM_RADIX_DECL(radix_sort_u64, uint64_t, uint32_t)
#undef TM_RADIX_DECL
// Time sort: (graph | t key, EdgeVal) pairs on bits [0, bits); the last pass
// writes RankOut (at least one pass always runs).
int radix_sort_time_u32(uint32_t *keys, uint32_t *keys_alt, EdgeVal *vals, EdgeVal *vals_alt,
                        uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s, RankOut out);
int radix_sort_time_u64(uint64_t *keys, uint64_t *keys_alt, EdgeVal *vals, EdgeVal *vals_alt,
                        uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s, RankOut out);
// The time sort of one graph read straight from the input arrays (key
// t - tmin[0], value (src, dst, input index)); keys / vals are only the
// ping-pong buffers.
int radix_sort_time_direct_u32(const int32_t *src, const int32_t *dst, const int64_t *t,
                               uint32_t *keys, uint32_t *keys_alt, EdgeVal *vals, EdgeVal *vals_alt,
                               uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s,
                               RankOut out);
int radix_sort_time_direct_u64(const int32_t *src, const int32_t *dst, const int64_t *t,
                               uint64_t *keys, uint64_t *keys_alt, EdgeVal *vals, EdgeVal *vals_alt,
                               uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s,
                               RankOut out);
// An edge's time and its two entry positions in S (source, destination).
struct alignas(16) EdgeRec {
    int64_t t;
    uint32_t p_src, p_dst;
};
static_assert(sizeof(EdgeRec) == 16 && offsetof(EdgeRec, p_src) == 8, "EdgeRec layout");

// epos[slot] = position of slot, from the slots in entry order (a
// permutation of [0, n)); k0, v0, k1, v1: n words each of scratch, none of
// them aliasing slot; tmp as for the radix sorts.  With erec (n even):
// erec[r] = (t_r[r], epos[2r], epos[2r + 1]) for the n / 2 edges as well.
int edge_positions(const uint32_t *slot, uint64_t n, uint32_t *k0, uint32_t *v0, uint32_t *k1,
                   uint32_t *v1, void *tmp, uint32_t *err, hipStream_t s, uint32_t *epos,
                   const int64_t *t_r = nullptr, EdgeRec *erec = nullptr);
// Node sort: (node, NodeVal) pairs on bits [0, bits); the last pass writes
// SeqOut instead of the ping-pong buffers (at least one pass always runs).
int radix_sort_nodes(uint32_t *keys, uint32_t *keys_alt, NodeVal *vals, NodeVal *vals_alt,
                     uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s, SeqOut out);
int radix_sort_nodes(uint32_t *keys, uint32_t *keys_alt, NodeVal32 *vals, NodeVal32 *vals_alt,
                     uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s, SeqOut out);


}  // namespace tmc

// ------------------------------------------------------------------ graph
namespace tmc {
struct Plan;
// Partition parameters of a count; the counts never depend on them.  0 in a
// call means: the graph's tuned value, else the autotuner table's, else the
// default.  hub_min = TM_HUB_OFF keeps every triangle candidate in the
// per-candidate kernel.
struct Params {
    uint32_t run_chunk = 0, tri_lane_max = 0, hub_min = 0;
    bool operator==(const Params &o) const {
        return run_chunk == o.run_chunk && tri_lane_max == o.tri_lane_max && hub_min == o.hub_min;
    }
};
}

struct tm_graph {
    // A graph is a batch of G independent temporal graphs stored as one union
    // graph: graph i's nodes are [node_base[i], node_base[i+1]), its edge
    // ranks (time order within the graph) [eoff[i], eoff[i+1]).
    uint32_t G = 1;
    std::vector<uint64_t> h_eoff;
    std::vector<uint32_t> h_node_base, h_ent_off, h_mpb, h_me_off;
    uint32_t *d_eoff = nullptr;       // G + 1 edge-rank bounds
    uint32_t *d_node_base = nullptr;  // G + 1
    uint32_t *d_mpb = nullptr;        // G + 1 multi-edge pair bounds
    int64_t *d_tmin = nullptr;        // G
    tmc::Tile *t_entries = nullptr;   // S_u entries, per graph
    tmc::Tile *t_elems = nullptr;     // multi-pair element sides (2 per element), per graph
    uint32_t n_t_entries = 0, n_t_elems = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;  // counts on one graph run one at a time
    // captured count sequence for repeated counts (see count.hip)
    tmc::Plan *plan = nullptr;
    // partition parameters picked by the autotuner (0 = not tuned)
    tmc::Params tuned;
    uint32_t n = 0;
    uint64_t m = 0;
    uint64_t max_degree = 0;
    bool max_degree_known = false;
    std::vector<void *> allocs;  // every device buffer below (stream-ordered allocations)
    // S_u for all u, (u, t, id) order: 2m entries
    uint32_t *off = nullptr;     // n + 1
    int64_t *ent_t = nullptr;    // timestamp
    uint32_t *ent_nd = nullptr;  // (other endpoint << 1) | dir
    uint32_t *ent_r = nullptr;   // edge rank in the global (t, id) order
    uint32_t *ent_c = nullptr;   // the center u the entry belongs to
    uint32_t *X = nullptr;       // 2m + 1: exclusive prefix count of dir = in entries
    uint32_t *epos = nullptr;    // 2m: position of edge rank r's src entry (2r) and dst entry (2r+1)
    uint32_t *perm = nullptr;    // m: edge id of rank r
    // node pairs with at least two edges (the only ones that hold pair or star
    // instances), ordered by (larger node, smaller node), and their edges
    // ("elements"), pair by pair in (t, id) order
    uint64_t n_multi = 0, n_me = 0;
    uint32_t *mp_start = nullptr;  // n_multi + 1: first element of each pair
    uint32_t *mp_lo = nullptr;     // n_multi: smaller node
    uint32_t *mp_hi = nullptr;     // n_multi: larger node
    int64_t *me_t = nullptr;       // n_me: timestamp
    uint2 *me_p = nullptr;         // n_me: position in S_lo, in S_hi
    uint4 *me_a = nullptr;         // n_me: (#o, #in) entries before it in S_lo, then in S_hi
    uint8_t *me_o = nullptr;       // n_me: bit 0 the edge leaves the smaller node, bit 1 first of its pair
};

namespace tmc {
// Builds G graphs at once: edges of graph i are rows [eoff[i], eoff[i+1]) of
// src/dst/t with node ids local to the graph (< ncount[i], or any id when
// ncount[i] == 0).  eoff and ncount are host arrays.
int build_graph_device(tm_graph *g, const int32_t *src, const int32_t *dst, const int64_t *t,
                       const uint64_t *eoff, const uint32_t *ncount, uint32_t G, hipStream_t s);
// Largest S_u length (computed on first use).
int graph_max_degree(tm_graph *g, uint64_t *out);
// Counts into raw[56] (host), see tm.h for the layout.
// Counts every graph of the batch with its own delta (host array of G) into
// raw[G * 56] (host).  use_graph: replay the count as a captured hipGraph
// (captured on first use for these partition parameters, then reused).
// families: TM_STARS | TM_PAIRS | TM_TRIANGLES; the raw counters of the
// others are zero.
int count_graph(tm_graph *g, const int64_t *deltas, Params pr, uint64_t *raw, bool use_graph,
                uint32_t families = TM_ALL_MOTIFS);
// Raw counters of one graph (G == 1) with the count's workspace carved from
// the library's fixed device array instead of the allocator (nothing is
// allocated); TM_ENOMEM if the workspace would not fit that array.
int count_graph_noalloc(tm_graph *g, int64_t delta, uint64_t *raw);
// Device allocations served so far (cache hits included), for tests.
uint64_t dev_alloc_calls();
// Raw counters of one graph (G == 1) for k windows, raw[k * 56].
int count_graph_multi(tm_graph *g, const int64_t *deltas, uint32_t k, Params pr, uint64_t *raw);
// Four-node three-edge motif counts of one graph (G == 1) into out32 (host),
// with the three-edge raw counters of the same delta into raw56 (host).
int count4_graph(tm_graph *g, int64_t delta, uint64_t *raw56, uint64_t *out32);
void plan_release(tm_graph *g);
void raw_from_counters(const uint64_t *res40, uint32_t G, uint64_t *raw);
int count_graph_async(tm_graph *g, const int64_t *pinned_deltas, uint64_t *pinned_res,
                      hipEvent_t done);
// Capture the plan count_graph_async replays (no-op when it is current).
int count_plan_prepare(tm_graph *g);
// Device bytes held by a graph (its buffers; not the per-count workspace).
size_t graph_bytes(const tm_graph *g);
// Device bytes one count of g needs for its workspace.
size_t count_workspace_bytes(const tm_graph *g);
// Upper bound of device bytes a build of m edges uses at its peak.
size_t build_peak_bytes(uint64_t m, uint64_t n, uint32_t G);
// Autotuner (count.hip) and its process-wide table (api.hip).
int autotune(tm_graph *g, const int64_t *deltas, uint32_t k, Params *best, float *best_ms);
void tune_table_lookup(const tm_graph *g, Params *p);
void tune_table_store(const tm_graph *g, const Params &p);
}  // namespace tmc
