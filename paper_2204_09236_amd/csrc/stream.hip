// Incremental counts of an append-only edge stream.
//
// Each append brings a batch whose timestamps are all >= every earlier edge's
// (ties allowed; the batch's rows follow all earlier rows in id order, so a
// tie orders the earlier edge first).  An instance that contains a new edge
// then has a new last edge, and its first edge lies at most delta before that
// (Definition 2: t_last - t_first <= delta), so it only involves new edges and
// earlier edges with t >= (smallest new t) - delta.  The stream keeps that
// tail on the device; per append it counts tail + batch and the tail alone
// with the full path (build, then count) and takes the difference of the raw
// counters: exactly the instances whose last edge is new.  The raw counters
// are sums over instances, so the difference merges like any count, and the
// running sum over all appends equals the count of the whole stream.
//
// Rows older than (smallest new t) - delta can no longer meet a new edge.
// Keeping a few of them costs nothing in exactness: the instances among the
// tail's own rows cancel in the difference.  So the tail is cut (an
// order-preserving compaction) only once at least half of it is certainly
// stale, judged from each batch's largest t kept on the host.  Between cuts,
// tail + batch of one append is the whole tail of the next, whose count is
// then already known: one build and count per append instead of two.  Device
// memory still follows the edge rate times delta (at most about twice the
// rows that can meet a new edge, plus a batch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <mutex>
#include <vector>

#include "tm_internal.h"

namespace {

constexpr int kRangeBlock = 256;

__global__ void k_range_init(int64_t *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[0] = LLONG_MAX;
        out[1] = LLONG_MIN;
    }
}

// Smallest and largest t of the batch (block reduction, then one atomic per
// block).
__global__ void __launch_bounds__(kRangeBlock) k_range(const int64_t *t, uint64_t m, int64_t *out) {
    __shared__ int64_t lo_s[kRangeBlock], hi_s[kRangeBlock];
    int64_t lo = LLONG_MAX, hi = LLONG_MIN;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t v = t[i];
        lo = min(lo, v);
        hi = max(hi, v);
    }
    lo_s[threadIdx.x] = lo;
    hi_s[threadIdx.x] = hi;
    __syncthreads();
    for (uint32_t o = kRangeBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            lo_s[threadIdx.x] = min(lo_s[threadIdx.x], lo_s[threadIdx.x + o]);
            hi_s[threadIdx.x] = max(hi_s[threadIdx.x], hi_s[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMin(reinterpret_cast<long long *>(&out[0]), (long long)lo_s[0]);
        atomicMax(reinterpret_cast<long long *>(&out[1]), (long long)hi_s[0]);
    }
}

// Rows of the tail that stay: t >= cut.
__global__ void k_keep_flags(const int64_t *t, uint64_t len, int64_t cut, uint32_t *flag) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (uint64_t)gridDim.x * blockDim.x)
        flag[i] = t[i] >= cut ? 1u : 0u;
}

// Kept rows to their scanned slots (input order preserved).
__global__ void k_keep_scatter(const int32_t *src, const int32_t *dst, const int64_t *t,
                               const uint32_t *flag, const uint32_t *idx, uint64_t len,
                               int32_t *nsrc, int32_t *ndst, int64_t *nt) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (!flag[i]) continue;
        const uint32_t j = idx[i];
        nsrc[j] = src[i];
        ndst[j] = dst[i];
        nt[j] = t[i];
    }
}

dim3 grid_of(uint64_t n) {
    return dim3((unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 4096)));
}

// Raw counters of the graph on rows [0, len) of the device arrays.
int count_rows(const int32_t *src, const int32_t *dst, const int64_t *t, uint64_t len, uint32_t n,
               int64_t delta, hipStream_t s, uint64_t raw[56]) {
    tm_graph *g = nullptr;
    int rc = tm_build_graph(src, dst, t, len, n, TM_DEVICE_PTRS, s, &g);
    if (rc) return rc;
    rc = tm_count_raw(g, delta, raw);
    tm_graph_free(g);
    return rc;
}

}  // namespace

struct tm_stream {
    int64_t delta = 0;
    uint32_t n = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    // the kept tail: rows [0, len) of these device arrays, in id order
    int32_t *src = nullptr, *dst = nullptr;
    int64_t *t = nullptr;
    uint64_t len = 0;
    bool any = false;    // an edge has been appended
    int64_t tmax = 0;    // largest t so far
    uint64_t edges = 0;  // edges appended so far
    uint64_t total[56] = {};
    uint64_t last[56] = {};    // raw counters of the current tail (rows [0, len))
    // (largest t, rows) of each batch in the tail, in order; after a cut the
    // kept rows count as one batch with the largest t seen so far
    std::vector<std::pair<int64_t, uint64_t>> spans;
    int64_t *range = nullptr;  // device scratch: batch min and max t
    std::mutex mu;
};

namespace {

void free_tail(tm_stream *s) {
    tmc::dev_free(s->src, s->stream);
    tmc::dev_free(s->dst, s->stream);
    tmc::dev_free(s->t, s->stream);
    s->src = s->dst = nullptr;
    s->t = nullptr;
}

int batch_range(tm_stream *s, const int64_t *t, uint64_t m, int flags, int64_t *lo, int64_t *hi) {
    if (flags == TM_HOST_PTRS) {
        int64_t a = t[0], b = t[0];
        for (uint64_t i = 1; i < m; i++) {
            a = std::min(a, t[i]);
            b = std::max(b, t[i]);
        }
        *lo = a;
        *hi = b;
        return TM_OK;
    }
    TM_LAUNCH("stream_range_init", k_range_init, dim3(1), dim3(64), 0, s->stream, s->range);
    const uint64_t blocks = std::min<uint64_t>((m + kRangeBlock - 1) / kRangeBlock, 1024);
    TM_LAUNCH("stream_range", k_range, dim3((unsigned)blocks), dim3(kRangeBlock), 0, s->stream, t, m,
              s->range);
    int64_t h[2];
    TM_HIP_TRY(hipMemcpyAsync(h, s->range, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    TM_HIP_TRY(hipStreamSynchronize(s->stream));
    *lo = h[0];
    *hi = h[1];
    return TM_OK;
}

// Number of tail rows with t >= cut (flags and their scan into flag / idx,
// which the caller owns).
int count_kept(tm_stream *s, int64_t cut, uint32_t *flag, uint32_t *idx, uint32_t *tmp,
               uint64_t *kept) {
    TM_LAUNCH("stream_keep_flags", k_keep_flags, grid_of(s->len), dim3(256), 0, s->stream, s->t,
              s->len, cut, flag);
    const int rc = tmc::scan_u32_array(flag, idx, s->len, tmp, s->stream);
    if (rc) return rc;
    uint32_t h = 0;
    TM_HIP_TRY(hipMemcpyAsync(&h, idx + s->len, 4, hipMemcpyDeviceToHost, s->stream));
    TM_HIP_TRY(hipStreamSynchronize(s->stream));
    *kept = h;
    return TM_OK;
}

int keep_scatter(tm_stream *s, const uint32_t *flag, const uint32_t *idx, int32_t *nsrc,
                 int32_t *ndst, int64_t *nt) {
    TM_LAUNCH("stream_keep_scatter", k_keep_scatter, grid_of(s->len), dim3(256), 0, s->stream,
              s->src, s->dst, s->t, flag, idx, s->len, nsrc, ndst, nt);
    return TM_OK;
}

int append_locked(tm_stream *s, const int32_t *src, const int32_t *dst, const int64_t *t,
                  uint64_t m, int flags, uint64_t *diff) {
    int64_t lo = 0, hi = 0;
    int rc = batch_range(s, t, m, flags, &lo, &hi);
    if (rc) return rc;
    if (s->any && lo < s->tmax) {
        tmc::set_error("appended edges must not precede earlier ones (smallest new t < largest t so far)");
        return TM_EINVAL;
    }
    if (lo <= -((int64_t)1 << 62) || hi >= ((int64_t)1 << 62)) {
        tmc::set_error("timestamps must satisfy |t| < 2^62");
        return TM_EINVAL;
    }
    // tail rows with t < lo - delta cannot meet the new edges
    const int64_t cut = lo - s->delta;
    // rows certainly below the cut: whole batches whose largest t is
    uint64_t stale = 0;
    for (const auto &b : s->spans)
        if (b.first < cut) stale += b.second;
    const bool trim = s->len && 2 * stale >= s->len;
    uint32_t *flag = nullptr, *idx = nullptr, *tmp = nullptr;
    auto free_scan = [&]() {
        tmc::dev_free(flag, s->stream);
        tmc::dev_free(idx, s->stream);
        tmc::dev_free(tmp, s->stream);
    };
    uint64_t kept = s->len;
    if (trim) {
        rc = tmc::dev_alloc(reinterpret_cast<void **>(&flag), s->len * 4, s->stream);
        if (!rc) rc = tmc::dev_alloc(reinterpret_cast<void **>(&idx), (s->len + 1) * 4, s->stream);
        if (!rc) rc = tmc::dev_alloc(reinterpret_cast<void **>(&tmp), tmc::scan_tmp_count(s->len) * 4, s->stream);
        if (rc) {
            free_scan();
            return rc;
        }
        rc = count_kept(s, cut, flag, idx, tmp, &kept);
        if (rc) {
            free_scan();
            return rc;
        }
    }
    const uint64_t len = kept + m;
    if (len >= (1ull << 31)) {
        free_scan();
        tmc::set_error("tail plus batch must stay below 2^31 edges");
        return TM_EINVAL;
    }
    // new tail buffers: kept rows, then the batch
    int32_t *nsrc = nullptr, *ndst = nullptr;
    int64_t *nt = nullptr;
    rc = tmc::dev_alloc(reinterpret_cast<void **>(&nsrc), len * 4, s->stream);
    if (!rc) rc = tmc::dev_alloc(reinterpret_cast<void **>(&ndst), len * 4, s->stream);
    if (!rc) rc = tmc::dev_alloc(reinterpret_cast<void **>(&nt), len * 8, s->stream);
    auto fail = [&](int code) {
        free_scan();
        tmc::dev_free(nsrc, s->stream);
        tmc::dev_free(ndst, s->stream);
        tmc::dev_free(nt, s->stream);
        return code;
    };
    if (rc) return fail(rc);
    if (trim && kept) {
        rc = keep_scatter(s, flag, idx, nsrc, ndst, nt);
        if (rc) return fail(rc);
    } else if (kept) {
        hipError_t ce = hipMemcpyAsync(nsrc, s->src, kept * 4, hipMemcpyDeviceToDevice, s->stream);
        if (ce == hipSuccess) ce = hipMemcpyAsync(ndst, s->dst, kept * 4, hipMemcpyDeviceToDevice, s->stream);
        if (ce == hipSuccess) ce = hipMemcpyAsync(nt, s->t, kept * 8, hipMemcpyDeviceToDevice, s->stream);
        if (ce != hipSuccess) {
            tmc::set_error(std::string("stream tail copy: ") + hipGetErrorString(ce));
            return fail(TM_EHIP);
        }
    }
    const hipMemcpyKind kind = flags == TM_HOST_PTRS ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    hipError_t e = hipMemcpyAsync(nsrc + kept, src, m * 4, kind, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ndst + kept, dst, m * 4, kind, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(nt + kept, t, m * 8, kind, s->stream);
    if (e != hipSuccess) {
        tmc::set_error(std::string("stream copy: ") + hipGetErrorString(e));
        return fail(TM_EHIP);
    }
    // tail + batch, then the tail alone (the build validates the new rows)
    uint64_t with[56] = {}, without[56] = {};
    rc = count_rows(nsrc, ndst, nt, len, s->n, s->delta, s->stream, with);
    if (rc) return fail(rc);
    if (kept == s->len) {
        // nothing was cut: the tail is the last append's tail + batch
        for (int i = 0; i < 56; i++) without[i] = s->last[i];
    } else if (kept) {
        rc = count_rows(nsrc, ndst, nt, kept, s->n, s->delta, s->stream, without);
        if (rc) return fail(rc);
    }
    for (int i = 0; i < 56; i++) {
        if (with[i] < without[i]) {
            tmc::set_error("stream: a counter of tail + batch is below the tail's");
            return fail(TM_EINTERNAL);
        }
        diff[i] = with[i] - without[i];
    }
    // commit
    free_scan();
    free_tail(s);
    s->src = nsrc;
    s->dst = ndst;
    s->t = nt;
    s->len = len;
    if (trim) {
        s->spans.clear();
        if (kept) s->spans.emplace_back(s->tmax, kept);
    }
    s->spans.emplace_back(hi, m);
    for (int i = 0; i < 56; i++) s->last[i] = with[i];
    s->any = true;
    s->tmax = std::max(s->tmax, hi);
    s->edges += m;
    for (int i = 0; i < 56; i++) s->total[i] += diff[i];
    return TM_OK;
}

}  // namespace

extern "C" {

int tm_stream_create(int64_t delta, uint32_t n_nodes, void *hip_stream, tm_stream **out) {
    if (!out) {
        tmc::set_error("out is NULL");
        return TM_EINVAL;
    }
    if (delta < 0 || delta >= ((int64_t)1 << 62)) {
        tmc::set_error("delta must satisfy 0 <= delta < 2^62");
        return TM_EINVAL;
    }
    if (n_nodes >= 0x80000000u) {
        tmc::set_error("n_nodes must be below 2^31");
        return TM_EINVAL;
    }
    tm_stream *s = new (std::nothrow) tm_stream();
    if (!s) return TM_ENOMEM;
    s->delta = delta;
    s->n = n_nodes;
    s->stream = static_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&s->device);
    int rc = tmc::dev_alloc(reinterpret_cast<void **>(&s->range), 2 * sizeof(int64_t), s->stream);
    if (rc) {
        delete s;
        return rc;
    }
    *out = s;
    return TM_OK;
}

int tm_stream_append(tm_stream *s, const int32_t *src, const int32_t *dst, const int64_t *t,
                     uint64_t m, int flags, uint64_t new_counts[36]) {
    if (!s) {
        tmc::set_error("NULL stream");
        return TM_EINVAL;
    }
    if (flags != TM_HOST_PTRS && flags != TM_DEVICE_PTRS) {
        tmc::set_error("flags must be TM_HOST_PTRS or TM_DEVICE_PTRS");
        return TM_EINVAL;
    }
    if (m > 0 && (!src || !dst || !t)) {
        tmc::set_error("NULL edge array");
        return TM_EINVAL;
    }
    if (m >= (1ull << 31)) {
        tmc::set_error("m must be below 2^31");
        return TM_EINVAL;
    }
    uint64_t diff[56] = {};
    int rc = TM_OK;
    if (m > 0) {
        std::lock_guard<std::mutex> lk(s->mu);
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != s->device) (void)hipSetDevice(s->device);
        rc = append_locked(s, src, dst, t, m, flags, diff);
        if (cur != s->device) (void)hipSetDevice(cur);
    }
    if (rc) return rc;
    if (new_counts) {
        uint64_t cells[36];
        rc = tm_merge(diff, cells);
        if (rc) return rc;
        for (int i = 0; i < 36; i++) new_counts[i] = cells[i];
    }
    return TM_OK;
}

int tm_stream_totals(tm_stream *s, uint64_t total[36], uint64_t *edges, uint64_t *tail_edges) {
    if (!s) {
        tmc::set_error("NULL stream");
        return TM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (total) {
        uint64_t cells[36];
        const int rc = tm_merge(s->total, cells);
        if (rc) return rc;
        for (int i = 0; i < 36; i++) total[i] = cells[i];
    }
    if (edges) *edges = s->edges;
    if (tail_edges) *tail_edges = s->len;
    return TM_OK;
}

void tm_stream_free(tm_stream *s) {
    if (!s) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != s->device) (void)hipSetDevice(s->device);
    free_tail(s);
    tmc::dev_free(s->range, s->stream);
    (void)hipStreamSynchronize(s->stream);
    if (cur != s->device) (void)hipSetDevice(cur);
    delete s;
}

}  // extern "C"
