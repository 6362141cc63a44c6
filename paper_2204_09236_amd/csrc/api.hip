// C ABI of the motif-counting library: graph lifecycle, counting entry points,
// the merge of the paper's counters into the 36 motifs, errors and tracing.
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tm_internal.h"

namespace tmc {

// ----------------------------------------------------------------- errors
static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const std::string &last_error() { return g_last_error; }

// ---------------------------------------------------------------- scratch
Scratch::~Scratch() {
    if (base && owned) dev_free(base, stream);
}

int Scratch::reserve(size_t bytes, hipStream_t s) {
    stream = s;
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    const int rc = dev_alloc(&p, bytes, s);
    if (rc) return rc;
    base = static_cast<char *>(p);
    cap = bytes;
    used = 0;
    return TM_OK;
}

// ------------------------------------------------------- autotuner table
namespace {
std::mutex g_tune_mu;
std::map<uint64_t, tmc::Params> g_tune;

int ilog2(uint64_t x) {
    int b = 0;
    while (x > 1) {
        x >>= 1;
        b++;
    }
    return b;
}

uint64_t shape_key(const tm_graph *g) {
    return ((uint64_t)ilog2(g->m + 1) << 16) | ((uint64_t)ilog2(g->n_me + 1) << 8) |
           (uint64_t)ilog2(g->G);
}
}  // namespace

void tune_table_lookup(const tm_graph *g, Params *p) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(shape_key(g));
    if (it != g_tune.end()) *p = it->second;
}

void tune_table_store(const tm_graph *g, const Params &p) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[shape_key(g)] = p;
}

// --------------------------------------------------------------- profiler
namespace {
struct ProfRec {
    std::string name;
    hipEvent_t start, stop;
    hipStream_t stream;
};
struct ProfSum {
    std::string name;
    uint64_t launches = 0;
    double ms = 0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::string g_prof_only;  // trace only launches of this name (empty: all)
std::vector<ProfRec> g_pending;
std::vector<ProfSum> g_sums;
std::vector<hipEvent_t> g_event_pool;  // recycled events (creation is slow)

hipEvent_t take_event() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
thread_local hipEvent_t g_cur_start = nullptr;
thread_local std::string g_cur_name;
thread_local const char *g_row = nullptr;  // step of the counting path the launches belong to
thread_local bool g_capturing = false;

void prof_drain_locked() {
    for (ProfRec &r : g_pending) {
        (void)hipEventSynchronize(r.stop);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, r.start, r.stop);
        g_event_pool.push_back(r.start);
        g_event_pool.push_back(r.stop);
        ProfSum *slot = nullptr;
        for (ProfSum &s : g_sums)
            if (s.name == r.name) slot = &s;
        if (!slot) {
            g_sums.push_back(ProfSum{r.name, 0, 0});
            slot = &g_sums.back();
        }
        slot->launches += 1;
        slot->ms += ms;
    }
    g_pending.clear();
}
}  // namespace

void set_capturing(bool on) { g_capturing = on; }

ProfRow::ProfRow(const char *row) : prev(g_row) { g_row = row; }
ProfRow::~ProfRow() { g_row = prev; }

void prof_begin(const char *name, hipStream_t s) {
    if (!g_prof_on || g_capturing) return;
    std::string full = g_row ? std::string(g_row) + ":" + name : std::string(name);
    if (!g_prof_only.empty() && g_prof_only != full) return;
    g_cur_name = std::move(full);
    g_cur_start = take_event();
    if (g_cur_start) (void)hipEventRecord(g_cur_start, s);
}

void prof_end(hipStream_t s) {
    if (!g_prof_on || g_capturing || !g_cur_start) return;
    hipEvent_t stop = take_event();
    if (!stop) return;
    (void)hipEventRecord(stop, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_pending.push_back(ProfRec{g_cur_name, g_cur_start, stop, s});
    g_cur_start = nullptr;
}

}  // namespace tmc

// ===================================================================== C ABI
extern "C" {

const char *tm_strerror(int code) {
    switch (code) {
        case TM_OK: return "ok";
        case TM_EINVAL: return "invalid argument or input";
        case TM_ENOMEM: return "out of device memory";
        case TM_EHIP: return "HIP runtime error";
        case TM_EAGAIN: return "try again";
        case TM_ENOTFOUND: return "not found";
        case TM_EINTERNAL: return "internal self-check failed";
        default: return "unknown status";
    }
}

const char *tm_last_error(void) { return tmc::g_last_error.c_str(); }

void tm_debug_lookback_giveup(int on) { tmc::set_lookback_giveup(on != 0); }

void tm_debug_force_edge_sort(int on) { tmc::set_force_edge_sort(on != 0); }

uint32_t tm_graph_count(const tm_graph *g) { return g ? g->G : 0; }

void tm_graph_free(tm_graph *g) {
    if (!g) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    tmc::plan_release(g);
    for (void *p : g->allocs) tmc::dev_free(p, g->stream);
    if (cur != g->device) (void)hipSetDevice(cur);
    delete g;
}

static int build_common(const int32_t *src, const int32_t *dst, const int64_t *t,
                        const uint64_t *edge_off, const uint32_t *node_count, uint32_t G, int flags,
                        void *hip_stream, tm_graph **out) {
    if (!out) {
        tmc::set_error("out is NULL");
        return TM_EINVAL;
    }
    if (G == 0 || !edge_off || !node_count) {
        tmc::set_error("a batch needs G >= 1 graphs and its edge offsets and node counts");
        return TM_EINVAL;
    }
    if (edge_off[0] != 0) {
        tmc::set_error("edge offsets must start at 0");
        return TM_EINVAL;
    }
    for (uint32_t i = 0; i < G; i++) {
        if (edge_off[i + 1] < edge_off[i]) {
            tmc::set_error("edge offsets must be non-decreasing");
            return TM_EINVAL;
        }
        if (node_count[i] >= 0x80000000u) {
            tmc::set_error("node counts must be below 2^31");
            return TM_EINVAL;
        }
    }
    const uint64_t m = edge_off[G];
    if (m > 0 && (!src || !dst || !t)) {
        tmc::set_error("NULL edge array");
        return TM_EINVAL;
    }
    if (m >= (1ull << 31)) {
        tmc::set_error("the number of edges must be below 2^31");
        return TM_EINVAL;
    }
    if (flags != TM_HOST_PTRS && flags != TM_DEVICE_PTRS) {
        tmc::set_error("flags must be TM_HOST_PTRS or TM_DEVICE_PTRS");
        return TM_EINVAL;
    }
    tm_graph *g = new (std::nothrow) tm_graph();
    if (!g) return TM_ENOMEM;
    g->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&g->device);
    const int32_t *ds = src, *dd = dst;
    const int64_t *dt = t;
    void *own = nullptr;
    int rc = TM_OK;
    if (flags == TM_HOST_PTRS && m > 0) {
        rc = tmc::dev_alloc(&own, m * 16, g->stream);
        if (rc == TM_OK) {
            int32_t *os = static_cast<int32_t *>(own);
            int32_t *od = os + m;
            int64_t *ot = reinterpret_cast<int64_t *>(od + m);
            hipStream_t s = g->stream;
            if (hipMemcpyAsync(os, src, m * 4, hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(od, dst, m * 4, hipMemcpyHostToDevice, s) ||
                hipMemcpyAsync(ot, t, m * 8, hipMemcpyHostToDevice, s)) {
                tmc::set_error("host-to-device copy failed");
                rc = TM_EHIP;
            }
            ds = os;
            dd = od;
            dt = ot;
        }
    }
    if (rc == TM_OK) rc = tmc::build_graph_device(g, ds, dd, dt, edge_off, node_count, G, g->stream);
    if (own) tmc::dev_free(own, g->stream);
    if (rc != TM_OK) {
        (void)hipStreamSynchronize(g->stream);
        tm_graph_free(g);
        return rc;
    }
    *out = g;
    return TM_OK;
}

int tm_build_graph(const int32_t *src, const int32_t *dst, const int64_t *t, uint64_t m,
                   uint32_t n_nodes, int flags, void *hip_stream, tm_graph **out) {
    if (m >= (1ull << 31)) {
        tmc::set_error("m must be below 2^31");
        return TM_EINVAL;
    }
    const uint64_t eoff[2] = {0, m};
    const uint32_t ncount[1] = {n_nodes};
    return build_common(src, dst, t, eoff, ncount, 1, flags, hip_stream, out);
}

int tm_build_batch(const int32_t *src, const int32_t *dst, const int64_t *t,
                   const uint64_t *edge_off, const uint32_t *node_count, uint32_t G, int flags,
                   void *hip_stream, tm_graph **out) {
    return build_common(src, dst, t, edge_off, node_count, G, flags, hip_stream, out);
}

static int count_common(tm_graph *g, const int64_t *deltas, const tmc::Params &pr, uint64_t *raw,
                        bool use_graph, uint32_t families = TM_ALL_MOTIFS) {
    if (!g || !raw || !deltas) {
        tmc::set_error("NULL graph, deltas or output");
        return TM_EINVAL;
    }
    for (uint32_t i = 0; i < g->G; i++)
        if (deltas[i] < 0 || deltas[i] >= ((int64_t)1 << 62)) {
            tmc::set_error("delta must satisfy 0 <= delta < 2^62");
            return TM_EINVAL;
        }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    std::vector<uint64_t> tmp((size_t)g->G * 56);
    int rc;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        rc = tmc::count_graph(g, deltas, pr, tmp.data(), use_graph, families);
    }
    if (cur != g->device) (void)hipSetDevice(cur);
    if (rc) return rc;
    for (size_t i = 0; i < tmp.size(); i++) raw[i] = tmp[i];
    return TM_OK;
}

static tmc::Params params(uint32_t run_chunk, uint32_t tri_lane_max, uint32_t hub_min) {
    tmc::Params p;
    p.run_chunk = run_chunk;
    p.tri_lane_max = tri_lane_max;
    p.hub_min = hub_min;
    return p;
}

int tm_count_batch_raw_ex(tm_graph *g, const int64_t *deltas, uint32_t run_chunk,
                          uint32_t tri_lane_max, uint32_t hub_min, int use_graph,
                          uint64_t (*raw)[56]) {
    return count_common(g, deltas, params(run_chunk, tri_lane_max, hub_min),
                        raw ? &raw[0][0] : nullptr, use_graph != 0);
}

int tm_autotune(tm_graph *g, const int64_t *deltas, uint32_t *run_chunk, uint32_t *tri_lane_max,
                uint32_t *hub_min, float *best_ms) {
    if (!g || !deltas) {
        tmc::set_error("NULL graph or deltas");
        return TM_EINVAL;
    }
    for (uint32_t i = 0; i < g->G; i++)
        if (deltas[i] < 0 || deltas[i] >= ((int64_t)1 << 62)) {
            tmc::set_error("delta must satisfy 0 <= delta < 2^62");
            return TM_EINVAL;
        }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    int rc;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        tmc::Params best;
        rc = tmc::autotune(g, deltas, 1, &best, best_ms);
        if (rc == TM_OK) {
            if (run_chunk) *run_chunk = best.run_chunk;
            if (tri_lane_max) *tri_lane_max = best.tri_lane_max;
            if (hub_min) *hub_min = best.hub_min;
        }
    }
    if (cur != g->device) (void)hipSetDevice(cur);
    return rc;
}

int tm_autotune_multi(tm_graph *g, const int64_t *deltas, uint32_t k, uint32_t *run_chunk,
                      uint32_t *tri_lane_max, uint32_t *hub_min, float *best_ms) {
    if (!g || !deltas) {
        tmc::set_error("NULL graph or deltas");
        return TM_EINVAL;
    }
    if (g->G != 1) {
        tmc::set_error("a batch of several graphs is tuned with tm_autotune");
        return TM_EINVAL;
    }
    if (k == 0 || k > TM_MAX_DELTAS) {
        tmc::set_error("k must be in [1, TM_MAX_DELTAS]");
        return TM_EINVAL;
    }
    for (uint32_t i = 0; i < k; i++)
        if (deltas[i] < 0 || deltas[i] >= ((int64_t)1 << 62)) {
            tmc::set_error("delta must satisfy 0 <= delta < 2^62");
            return TM_EINVAL;
        }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    int rc;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        tmc::Params best;
        rc = tmc::autotune(g, deltas, k, &best, best_ms);
        if (rc == TM_OK) {
            if (run_chunk) *run_chunk = best.run_chunk;
            if (tri_lane_max) *tri_lane_max = best.tri_lane_max;
            if (hub_min) *hub_min = best.hub_min;
        }
    }
    if (cur != g->device) (void)hipSetDevice(cur);
    return rc;
}

int tm_count_batch_raw(tm_graph *g, const int64_t *deltas, uint64_t (*raw)[56]) {
    return count_common(g, deltas, tmc::Params(), raw ? &raw[0][0] : nullptr, true);
}

int tm_count_batch(tm_graph *g, const int64_t *deltas, uint64_t (*out)[36]) {
    if (!g || !out) {
        tmc::set_error("NULL graph or output");
        return TM_EINVAL;
    }
    std::vector<uint64_t> raw((size_t)g->G * 56);
    int rc = count_common(g, deltas, tmc::Params(), raw.data(), true);
    if (rc) return rc;
    std::vector<uint64_t> res((size_t)g->G * 36);
    for (uint32_t i = 0; i < g->G; i++) {
        rc = tm_merge(raw.data() + (size_t)i * 56, res.data() + (size_t)i * 36);
        if (rc) return rc;
    }
    for (uint32_t i = 0; i < g->G; i++)
        for (int c = 0; c < 36; c++) out[i][c] = res[(size_t)i * 36 + c];
    return TM_OK;
}

int tm_count_raw_tuned(tm_graph *g, int64_t delta, uint32_t run_chunk, uint32_t tri_lane_max,
                       uint32_t hub_min, uint64_t raw[56]) {
    if (g && g->G != 1) {
        tmc::set_error("a batch of several graphs is counted with tm_count_batch");
        return TM_EINVAL;
    }
    return count_common(g, &delta, params(run_chunk, tri_lane_max, hub_min), raw, false);
}

int tm_count_raw(tm_graph *g, int64_t delta, uint64_t raw[56]) {
    return tm_count_raw_tuned(g, delta, 0, 0, 0, raw);
}

// 36-cell layout: out[6*(row-1) + (col-1)] = M_{row,col}
static int cell(int row, int col) { return 6 * (row - 1) + (col - 1); }

int tm_merge(const uint64_t raw[56], uint64_t out[36]) {
    if (!raw || !out) return TM_EINVAL;
    uint64_t res[36] = {0};
    for (int ty = 0; ty < 3; ty++)
        for (int d1 = 0; d1 < 2; d1++)
            for (int d2 = 0; d2 < 2; d2++)
                for (int d3 = 0; d3 < 2; d3++) {
                    const int row = 1 + 2 * ty + (d3 == 1);
                    const int col = 1 + 2 * (d2 == 0) + (d1 == 1);
                    res[cell(row, col)] += raw[ty * 8 + d1 * 4 + d2 * 2 + d3];
                }
    for (int i = 0; i < 8; i++)
        if (raw[24 + i] != raw[24 + (7 - i)]) {
            tmc::set_error("pair counters are not symmetric");
            return TM_EINTERNAL;
        }
    // pair classes seen from the first edge's source (d1 = o)
    res[cell(5, 5)] += raw[24 + 0];  // (o,o,o)
    res[cell(5, 6)] += raw[24 + 3];  // (o,in,in)
    res[cell(6, 5)] += raw[24 + 2];  // (o,in,o)
    res[cell(6, 6)] += raw[24 + 1];  // (o,o,in)
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int c = 0; c < 2; c++) {
                const uint64_t x = raw[32 + a * 4 + b * 2 + c];
                const uint64_t y = raw[40 + (1 - c) * 4 + (1 - b) * 2 + (1 - a)];
                const uint64_t z = raw[48 + c * 4 + (1 - a) * 2 + (1 - b)];
                if (x != y || y != z) {
                    tmc::set_error("triangle views disagree");
                    return TM_EINTERNAL;
                }
                const int col = 5 + (b == 0);
                const bool ab = a == b, cb = c == b;
                const int row = ab ? (cb ? 1 : 4) : (cb ? 3 : 2);
                res[cell(row, col)] += (x + y + z) / 3;
            }
    for (int i = 0; i < 36; i++) out[i] = res[i];
    return TM_OK;
}

int tm_count_noalloc(tm_graph *g, int64_t delta, uint64_t out[36]) {
    if (!g || !out) {
        tmc::set_error("NULL graph or output");
        return TM_EINVAL;
    }
    if (g->G != 1) {
        tmc::set_error("a batch of several graphs is counted with tm_count_batch");
        return TM_EINVAL;
    }
    if (delta < 0 || delta >= ((int64_t)1 << 62)) {
        tmc::set_error("delta must satisfy 0 <= delta < 2^62");
        return TM_EINVAL;
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    uint64_t raw[56];
    int rc;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        rc = tmc::count_graph_noalloc(g, delta, raw);
    }
    if (cur != g->device) (void)hipSetDevice(cur);
    if (rc) return rc;
    return tm_merge(raw, out);
}

uint64_t tm_debug_alloc_calls(void) { return tmc::dev_alloc_calls(); }

int tm_count(tm_graph *g, int64_t delta, uint64_t out[36]) {
    if (!out) {
        tmc::set_error("NULL output");
        return TM_EINVAL;
    }
    uint64_t raw[56];
    int rc = tm_count_raw(g, delta, raw);
    if (rc) return rc;
    return tm_merge(raw, out);
}

int tm_count_masked(tm_graph *g, int64_t delta, uint32_t families, uint64_t out[36]) {
    if (!out) {
        tmc::set_error("NULL output");
        return TM_EINVAL;
    }
    if (families == 0 || (families & ~(uint32_t)TM_ALL_MOTIFS)) {
        tmc::set_error("families must be a nonzero OR of TM_STARS, TM_PAIRS, TM_TRIANGLES");
        return TM_EINVAL;
    }
    if (g && g->G != 1) {
        tmc::set_error("a batch of several graphs is counted with tm_count_batch");
        return TM_EINVAL;
    }
    uint64_t raw[56];
    int rc = count_common(g, &delta, tmc::Params(), raw, false, families);
    if (rc) return rc;
    return tm_merge(raw, out);
}

int tm_count4(tm_graph *g, int64_t delta, uint64_t raw[56], uint64_t out[32]) {
    if (!g || !out) {
        tmc::set_error("NULL graph or output");
        return TM_EINVAL;
    }
    if (g->G != 1) {
        tmc::set_error("four-node motifs are counted on a single graph, not a batch");
        return TM_EINVAL;
    }
    if (delta < 0 || delta >= ((int64_t)1 << 62)) {
        tmc::set_error("delta must satisfy 0 <= delta < 2^62");
        return TM_EINVAL;
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    uint64_t r56[56], o32[32];
    int rc;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        rc = tmc::count4_graph(g, delta, r56, o32);
    }
    if (cur != g->device) (void)hipSetDevice(cur);
    if (rc) return rc;
    if (raw)
        for (int i = 0; i < 56; i++) raw[i] = r56[i];
    for (int i = 0; i < 32; i++) out[i] = o32[i];
    return TM_OK;
}

int tm_count_multi_raw(tm_graph *g, const int64_t *deltas, uint32_t k, uint64_t (*raw)[56]) {
    if (!g || !deltas || !raw) {
        tmc::set_error("NULL graph, deltas or output");
        return TM_EINVAL;
    }
    if (g->G != 1) {
        tmc::set_error("a batch of several graphs is counted with tm_count_batch");
        return TM_EINVAL;
    }
    if (k == 0 || k > TM_MAX_DELTAS) {
        tmc::set_error("k must be in [1, TM_MAX_DELTAS]");
        return TM_EINVAL;
    }
    for (uint32_t i = 0; i < k; i++)
        if (deltas[i] < 0 || deltas[i] >= ((int64_t)1 << 62)) {
            tmc::set_error("delta must satisfy 0 <= delta < 2^62");
            return TM_EINVAL;
        }
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != g->device) (void)hipSetDevice(g->device);
    std::vector<uint64_t> tmp((size_t)k * 56);
    int rc;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        rc = tmc::count_graph_multi(g, deltas, k, tmc::Params(), tmp.data());
    }
    if (cur != g->device) (void)hipSetDevice(cur);
    if (rc) return rc;
    for (uint32_t i = 0; i < k; i++)
        for (int c = 0; c < 56; c++) raw[i][c] = tmp[(size_t)i * 56 + c];
    return TM_OK;
}

int tm_count_multi(tm_graph *g, const int64_t *deltas, uint32_t k, uint64_t (*out)[36]) {
    if (!out) {
        tmc::set_error("NULL output");
        return TM_EINVAL;
    }
    if (k == 0 || k > TM_MAX_DELTAS) {
        tmc::set_error("k must be in [1, TM_MAX_DELTAS]");
        return TM_EINVAL;
    }
    std::vector<uint64_t> raw((size_t)k * 56);
    int rc = tm_count_multi_raw(g, deltas, k, reinterpret_cast<uint64_t(*)[56]>(raw.data()));
    if (rc) return rc;
    std::vector<uint64_t> res((size_t)k * 36);
    for (uint32_t i = 0; i < k; i++) {
        rc = tm_merge(raw.data() + (size_t)i * 56, res.data() + (size_t)i * 36);
        if (rc) return rc;
    }
    for (uint32_t i = 0; i < k; i++)
        for (int c = 0; c < 36; c++) out[i][c] = res[(size_t)i * 36 + c];
    return TM_OK;
}

int tm_graph_info(const tm_graph *g, uint32_t *n, uint64_t *m, uint64_t *multi_pairs,
                  uint64_t *multi_pair_edges, uint64_t *max_degree) {
    if (!g) return TM_EINVAL;
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (multi_pairs) *multi_pairs = g->n_multi;
    if (multi_pair_edges) *multi_pair_edges = g->n_me;
    if (max_degree) {
        const int rc = tmc::graph_max_degree(const_cast<tm_graph *>(g), max_degree);
        if (rc) return rc;
    }
    return TM_OK;
}

int tm_graph_sequences(const tm_graph *g, uint32_t *off, int64_t *t, uint32_t *nbr, uint8_t *dir,
                       uint32_t *id) {
    if (!g) return TM_EINVAL;
    const uint64_t len = 2 * g->m;
    hipStream_t s = g->stream;
    if (off)
        TM_HIP_TRY(hipMemcpyAsync(off, g->off, ((uint64_t)g->n + 1) * sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, s));
    if (t && len) TM_HIP_TRY(hipMemcpyAsync(t, g->ent_t, len * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    std::vector<uint32_t> nd, rk, perm;
    if ((nbr || dir || id) && len) {
        nd.resize(len);
        TM_HIP_TRY(hipMemcpyAsync(nd.data(), g->ent_nd, len * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    }
    if (id && len) {
        rk.resize(len);
        perm.resize(g->m);
        TM_HIP_TRY(hipMemcpyAsync(rk.data(), g->ent_r, len * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TM_HIP_TRY(hipMemcpyAsync(perm.data(), g->perm, g->m * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    }
    TM_HIP_TRY(hipStreamSynchronize(s));
    for (uint64_t p = 0; p < len; p++) {
        if (nbr) nbr[p] = nd[p] >> 1;
        if (dir) dir[p] = (uint8_t)(nd[p] & 1u);
        if (id) id[p] = perm[rk[p]];
    }
    return TM_OK;
}

void tm_prof_enable(int on) {
    std::lock_guard<std::mutex> lk(tmc::g_prof_mu);
    tmc::g_prof_on = on != 0;
}

void tm_prof_only(const char *name) {
    std::lock_guard<std::mutex> lk(tmc::g_prof_mu);
    tmc::g_prof_only = name ? name : "";
}

void tm_prof_reset(void) {
    std::lock_guard<std::mutex> lk(tmc::g_prof_mu);
    tmc::prof_drain_locked();
    tmc::g_sums.clear();
}

int tm_prof_read(int i, char *name, int name_cap, uint64_t *launches, double *total_ms) {
    std::lock_guard<std::mutex> lk(tmc::g_prof_mu);
    tmc::prof_drain_locked();
    if (i < 0 || i >= (int)tmc::g_sums.size()) return TM_ENOTFOUND;
    const tmc::ProfSum &s = tmc::g_sums[i];
    if (name && name_cap > 0) {
        size_t k = 0;
        for (; k + 1 < (size_t)name_cap && k < s.name.size(); k++) name[k] = s.name[k];
        name[k] = 0;
    }
    if (launches) *launches = s.launches;
    if (total_ms) *total_ms = s.ms;
    return TM_OK;
}

}  // extern "C"
