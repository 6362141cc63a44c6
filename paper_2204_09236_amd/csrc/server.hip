// Serving: a request loop that counts many temporal graphs as requests
// arrive, with continuous batching on one GPU.
//
// A request is (graph, delta).  Graphs are either keyed -- built once and kept
// resident on the device under their key, so later requests for the same key
// only count -- or anonymous (edges come with the request, freed afterwards).
// One scheduler thread repeats:
//   1. retire: in-flight counts whose completion event has fired are turned
//      into motif counts; their tickets complete and their device bytes are
//      released from the budget;
//   2. admit: pending requests, oldest first, while the number of counts in
//      flight and the device-byte budget allow.  A keyed graph that is not
//      resident is built first (evicting idle resident graphs, least
//      recently used first, when the budget is short); anonymous requests
//      admitted together are built as one union batch and counted together;
//   3. launch: every admitted count is issued asynchronously (captured count
//      graph replayed on the graph's own stream, counters copied to pinned
//      host memory, completion event), so counts of different requests
//      overlap on the device and a request that arrives while others run is
//      admitted as soon as a slot and memory are free.
// The budget is an admission bound on the bytes the server's graphs and
// counts need (estimated before a build, measured after); the device
// allocator caches freed blocks for reuse.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "tm_internal.h"

namespace tmc {
namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    tm_ticket ticket = 0;
    uint64_t key = 0;  // 0: anonymous
    std::vector<int32_t> src, dst;
    std::vector<int64_t> t;
    uint32_t n = 0;
    uint64_t m = 0;
    bool has_edges = false;
    int64_t delta = 0;
    int status = TM_EAGAIN;  // final status once done
    uint64_t out[36] = {0};
    uint64_t t_submit = 0, t_start = 0, t_done = 0;
};

struct Resident {
    tm_graph *g = nullptr;
    size_t bytes = 0;  // graph buffers + its count workspace
    uint64_t last_use = 0;
    int inflight = 0;  // counts running on it
    int queued = 0;    // queued requests that rely on it (submitted without edges)
};

struct Pinned {
    void *p = nullptr;
    size_t bytes = 0;
};

// One asynchronous count in flight: a resident graph (one request) or an
// anonymous union batch (member i answers reqs[i]).
struct Flight {
    std::vector<Request *> reqs;
    tm_graph *g = nullptr;
    bool owned = false;
    uint64_t key = 0;
    hipEvent_t done = nullptr;
    Pinned deltas, res;
    size_t footprint = 0;  // bytes charged to the budget while in flight
};

}  // namespace
}  // namespace tmc

struct tm_server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<tmc::Request *> pending;
    std::unordered_map<tm_ticket, tmc::Request *> tickets;
    bool stop = false;
    uint64_t next_ticket = 1;
    uint64_t budget = 0;
    uint32_t max_inflight = 0, max_queue = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    std::thread worker;
    // scheduler-thread state (read for stats under mu)
    std::unordered_map<uint64_t, tmc::Resident> resident;
    // keys whose graph is being built from an admitted request (under mu)
    std::unordered_set<uint64_t> building;
    std::vector<tmc::Flight> flights;
    std::vector<tmc::Pinned> pinned_pool;
    size_t resident_bytes = 0, flight_bytes = 0;
    uint64_t completed = 0, failed = 0, clock = 0;
};

namespace tmc {
namespace {

int take_pinned(tm_server *S, size_t bytes, Pinned *out) {
    for (size_t i = 0; i < S->pinned_pool.size(); i++)
        if (S->pinned_pool[i].bytes >= bytes) {
            *out = S->pinned_pool[i];
            S->pinned_pool.erase(S->pinned_pool.begin() + (long)i);
            return TM_OK;
        }
    size_t cap = 4096;
    while (cap < bytes) cap <<= 1;
    void *p = nullptr;
    TM_HIP_TRY(hipHostMalloc(&p, cap, hipHostMallocDefault));
    *out = Pinned{p, cap};
    return TM_OK;
}

void give_pinned(tm_server *S, Pinned &p) {
    if (p.p) S->pinned_pool.push_back(p);
    p = Pinned{};
}

void finish(tm_server *S, Request *r, int status) {
    std::lock_guard<std::mutex> lk(S->mu);
    r->status = status;
    r->t_done = now_ns();
    if (status == TM_OK) S->completed++;
    else S->failed++;
    S->cv_done.notify_all();
}

size_t budget_used(const tm_server *S) { return S->resident_bytes + S->flight_bytes; }

// Free idle resident graphs, least recently used first, until `need` more
// bytes fit in the budget.  Returns whether they fit.
bool make_room(tm_server *S, size_t need) {
    while (budget_used(S) + need > S->budget) {
        tm_graph *victim_g = nullptr;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            uint64_t victim = 0, oldest = ~0ull;
            for (auto &kv : S->resident)
                if (kv.second.inflight == 0 && kv.second.queued == 0 && kv.second.last_use < oldest) {
                    oldest = kv.second.last_use;
                    victim = kv.first;
                }
            if (oldest == ~0ull) return false;
            Resident &rg = S->resident[victim];
            victim_g = rg.g;
            S->resident_bytes -= rg.bytes;
            S->resident.erase(victim);
        }
        tm_graph_free(victim_g);
    }
    return true;
}

int launch(tm_server *S, Flight &f) {
    const uint32_t G = f.g->G;
    int rc = take_pinned(S, (size_t)G * 8, &f.deltas);
    if (!rc) rc = take_pinned(S, (size_t)G * 40 * 8, &f.res);
    if (rc) return rc;
    int64_t *d = static_cast<int64_t *>(f.deltas.p);
    for (uint32_t i = 0; i < G; i++) d[i] = f.reqs[i]->delta;
    TM_HIP_TRY(hipEventCreateWithFlags(&f.done, hipEventDisableTiming));
    std::lock_guard<std::mutex> lk(f.g->mu);
    return count_graph_async(f.g, d, static_cast<uint64_t *>(f.res.p), f.done);
}

void release_flight(tm_server *S, Flight &f) {
    if (f.done) (void)hipEventDestroy(f.done);
    f.done = nullptr;
    give_pinned(S, f.deltas);
    give_pinned(S, f.res);
    S->flight_bytes -= f.footprint;
    if (f.owned) {
        tm_graph_free(f.g);
    } else {
        auto it = S->resident.find(f.key);
        if (it != S->resident.end()) {
            it->second.inflight--;
            it->second.last_use = ++S->clock;
        }
    }
}

// Retire finished flights; returns how many were retired.
int retire(tm_server *S, bool wait_all) {
    int n = 0;
    for (size_t i = 0; i < S->flights.size();) {
        Flight &f = S->flights[i];
        hipError_t q = wait_all ? hipEventSynchronize(f.done) : hipEventQuery(f.done);
        if (q == hipErrorNotReady) {
            i++;
            continue;
        }
        const uint32_t G = f.g->G;
        if (q == hipSuccess) {
            std::vector<uint64_t> raw((size_t)G * 56);
            raw_from_counters(static_cast<const uint64_t *>(f.res.p), G, raw.data());
            for (uint32_t k = 0; k < G; k++) {
                uint64_t out[36];
                const int rc = tm_merge(raw.data() + (size_t)k * 56, out);
                if (rc == TM_OK)
                    for (int c = 0; c < 36; c++) f.reqs[k]->out[c] = out[c];
                finish(S, f.reqs[k], rc);
            }
        } else {
            set_error(std::string("count failed: ") + hipGetErrorString(q));
            for (Request *r : f.reqs) finish(S, r, TM_EHIP);
        }
        release_flight(S, f);
        S->flights.erase(S->flights.begin() + (long)i);
        n++;
    }
    return n;
}

int build_one(tm_server *S, Request *r, tm_graph **g) {
    return tm_build_graph(r->src.data(), r->dst.data(), r->t.data(), r->m, r->n, TM_HOST_PTRS,
                          S->stream, g);
}

// Admit and launch pending requests while slots and budget allow.
void admit(tm_server *S) {
    std::vector<Request *> anon;
    size_t anon_need = 0;
    while (true) {
        Request *r = nullptr;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->pending.empty()) break;
            r = S->pending.front();
        }
        if (S->flights.size() + (anon.empty() ? 0 : 1) >= S->max_inflight) break;
        bool is_resident = false;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            is_resident = r->key && S->resident.count(r->key);
        }
        if (is_resident) {
            Resident *rgp;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->pending.pop_front();
                rgp = &S->resident[r->key];
                if (!r->has_edges) rgp->queued--;
            }
            Resident &rg = *rgp;
            Flight f;
            f.reqs.push_back(r);
            f.g = rg.g;
            f.key = r->key;
            r->t_start = now_ns();
            rg.inflight++;
            const int rc = launch(S, f);
            S->flights.push_back(f);
            if (rc) {
                finish(S, r, rc);
                release_flight(S, S->flights.back());
                S->flights.pop_back();
            }
            continue;
        }
        const size_t need = build_peak_bytes(r->m, r->n, 1);
        if (need > S->budget) {
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->pending.pop_front();
            }
            set_error("request needs more device memory than the server budget");
            finish(S, r, TM_ENOMEM);
            continue;
        }
        if (r->key && !r->has_edges) {
            // its graph was to come from an earlier request that failed
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->pending.pop_front();
            }
            set_error("graph key is not resident and the request carries no edges");
            finish(S, r, TM_ENOTFOUND);
            continue;
        }
        if (r->key) {
            if (!make_room(S, need + anon_need)) break;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                S->pending.pop_front();
                S->building.insert(r->key);
            }
            r->t_start = now_ns();
            tm_graph *g = nullptr;
            int rc = build_one(S, r, &g);
            if (rc) {
                {
                    std::lock_guard<std::mutex> lk(S->mu);
                    S->building.erase(r->key);
                }
                finish(S, r, rc);
                continue;
            }
            Resident rg;
            rg.g = g;
            rg.bytes = graph_bytes(g) + count_workspace_bytes(g);
            rg.last_use = ++S->clock;
            rg.inflight = 1;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                // queued requests for this key that came without edges need it
                for (Request *q : S->pending)
                    if (q->key == r->key && !q->has_edges) rg.queued++;
                S->resident[r->key] = rg;
                S->building.erase(r->key);
            }
            S->resident_bytes += rg.bytes;
            r->src.clear();
            r->src.shrink_to_fit();
            r->dst.clear();
            r->dst.shrink_to_fit();
            r->t.clear();
            r->t.shrink_to_fit();
            Flight f;
            f.reqs.push_back(r);
            f.g = g;
            f.key = r->key;
            rc = launch(S, f);
            S->flights.push_back(f);
            if (rc) {
                finish(S, r, rc);
                release_flight(S, S->flights.back());
                S->flights.pop_back();
            }
            continue;
        }
        // anonymous: join the union batch of this admission cycle
        if (!make_room(S, anon_need + need)) break;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->pending.pop_front();
        }
        r->t_start = now_ns();
        anon.push_back(r);
        anon_need += need;
    }
    if (anon.empty()) return;
    // one union build for the anonymous requests of this admission cycle
    const uint32_t G = (uint32_t)anon.size();
    std::vector<uint64_t> eoff(G + 1, 0);
    std::vector<uint32_t> ncount(G);
    for (uint32_t i = 0; i < G; i++) {
        eoff[i + 1] = eoff[i] + anon[i]->m;
        ncount[i] = anon[i]->n;
    }
    std::vector<int32_t> src(eoff[G]), dst(eoff[G]);
    std::vector<int64_t> t(eoff[G]);
    for (uint32_t i = 0; i < G; i++) {
        std::copy(anon[i]->src.begin(), anon[i]->src.end(), src.begin() + (long)eoff[i]);
        std::copy(anon[i]->dst.begin(), anon[i]->dst.end(), dst.begin() + (long)eoff[i]);
        std::copy(anon[i]->t.begin(), anon[i]->t.end(), t.begin() + (long)eoff[i]);
    }
    tm_graph *g = nullptr;
    int rc = tm_build_batch(src.data(), dst.data(), t.data(), eoff.data(), ncount.data(), G,
                            TM_HOST_PTRS, S->stream, &g);
    if (rc == TM_EINVAL && G > 1) {
        // an invalid member must not fail the others: isolate it
        std::vector<Request *> good;
        for (Request *r : anon) {
            tm_graph *one = nullptr;
            const int r1 = build_one(S, r, &one);
            if (r1) finish(S, r, r1);
            else {
                good.push_back(r);
                tm_graph_free(one);
            }
        }
        anon.swap(good);
        if (anon.empty()) return;
        const uint32_t G2 = (uint32_t)anon.size();
        eoff.assign(G2 + 1, 0);
        ncount.assign(G2, 0);
        src.clear();
        dst.clear();
        t.clear();
        for (uint32_t i = 0; i < G2; i++) {
            eoff[i + 1] = eoff[i] + anon[i]->m;
            ncount[i] = anon[i]->n;
            src.insert(src.end(), anon[i]->src.begin(), anon[i]->src.end());
            dst.insert(dst.end(), anon[i]->dst.begin(), anon[i]->dst.end());
            t.insert(t.end(), anon[i]->t.begin(), anon[i]->t.end());
        }
        rc = tm_build_batch(src.data(), dst.data(), t.data(), eoff.data(), ncount.data(), G2,
                            TM_HOST_PTRS, S->stream, &g);
    }
    if (rc) {
        for (Request *r : anon) finish(S, r, rc);
        return;
    }
    Flight f;
    f.reqs = anon;
    f.g = g;
    f.owned = true;
    f.footprint = graph_bytes(g) + count_workspace_bytes(g);
    S->flight_bytes += f.footprint;
    rc = launch(S, f);
    S->flights.push_back(f);
    if (rc) {
        for (Request *r : f.reqs) finish(S, r, rc);
        release_flight(S, S->flights.back());
        S->flights.pop_back();
    }
}

void worker_main(tm_server *S) {
    (void)hipSetDevice(S->device);
    while (true) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->flights.empty() && S->pending.empty() && !S->stop)
                S->cv_work.wait(lk, [S] { return S->stop || !S->pending.empty(); });
            if (S->stop) break;
        }
        const int retired = retire(S, false);
        admit(S);
        if (retired == 0 && !S->flights.empty()) {
            // counts in flight and nothing finished yet: brief back-off
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait_for(lk, std::chrono::microseconds(50));
        }
    }
    retire(S, true);
}

}  // namespace
}  // namespace tmc

extern "C" {

int tm_server_create(uint64_t hbm_budget_bytes, uint32_t max_inflight, uint32_t max_queue,
                     tm_server **out) {
    if (!out || hbm_budget_bytes == 0 || max_inflight == 0 || max_queue == 0) {
        tmc::set_error("server needs an output handle, a budget, max_inflight and max_queue > 0");
        return TM_EINVAL;
    }
    tm_server *S = new (std::nothrow) tm_server();
    if (!S) return TM_ENOMEM;
    S->budget = hbm_budget_bytes;
    S->max_inflight = max_inflight;
    S->max_queue = max_queue;
    (void)hipGetDevice(&S->device);
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
        tmc::set_error("hipStreamCreate failed");
        delete S;
        return TM_EHIP;
    }
    S->worker = std::thread(tmc::worker_main, S);
    *out = S;
    return TM_OK;
}

static int enqueue(tm_server *S, tmc::Request *r, tmc::Resident *rg, tm_ticket *out);

int tm_submit(tm_server *S, uint64_t graph_key, const int32_t *src, const int32_t *dst,
              const int64_t *t, uint64_t m, uint32_t n_nodes, int64_t delta, tm_ticket *out) {
    if (!S || !out) {
        tmc::set_error("NULL server or ticket");
        return TM_EINVAL;
    }
    if (delta < 0 || delta >= ((int64_t)1 << 62)) {
        tmc::set_error("delta must satisfy 0 <= delta < 2^62");
        return TM_EINVAL;
    }
    auto *r = new (std::nothrow) tmc::Request();
    if (!r) return TM_ENOMEM;
    r->key = graph_key;
    r->delta = delta;
    r->n = n_nodes;
    // A known key (resident, being built, or carried by a pending request)
    // needs no edges: the request is queued in the same critical section
    // that found the key, so the graph cannot be evicted, or become resident
    // without counting this request, in between.
    if (graph_key) {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->resident.find(graph_key);
        bool known = it != S->resident.end() || S->building.count(graph_key);
        for (tmc::Request *q : S->pending)
            if (!known && q->key == graph_key && q->has_edges) known = true;
        if (known) return enqueue(S, r, it != S->resident.end() ? &it->second : nullptr, out);
    }
    if (graph_key && !src) {
        delete r;
        tmc::set_error("unknown graph key and no edges given");
        return TM_ENOTFOUND;
    }
    if (m > 0 && (!src || !dst || !t)) {
        delete r;
        tmc::set_error("NULL edge array");
        return TM_EINVAL;
    }
    if (m >= (1ull << 31)) {
        delete r;
        tmc::set_error("m must be below 2^31");
        return TM_EINVAL;
    }
    r->m = m;
    r->has_edges = true;
    if (m) {
        r->src.assign(src, src + m);
        r->dst.assign(dst, dst + m);
        r->t.assign(t, t + m);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    return enqueue(S, r, nullptr, out);
}

// Queue a request (caller holds S->mu).  rg: the resident graph an
// edge-less keyed request relies on, which must then stay resident until
// the request runs.
static int enqueue(tm_server *S, tmc::Request *r, tmc::Resident *rg, tm_ticket *out) {
    if (S->stop) {
        delete r;
        tmc::set_error("server is shutting down");
        return TM_EINVAL;
    }
    if (S->pending.size() >= S->max_queue) {
        delete r;
        tmc::set_error("server queue is full");
        return TM_EAGAIN;
    }
    if (rg) rg->queued++;
    r->ticket = S->next_ticket++;
    r->t_submit = tmc::now_ns();
    S->tickets[r->ticket] = r;
    S->pending.push_back(r);
    *out = r->ticket;
    S->cv_work.notify_one();
    return TM_OK;
}

static int collect(tm_server *S, tm_ticket tk, uint64_t out[36], uint64_t times_ns[3],
                   std::unique_lock<std::mutex> &lk) {
    auto it = S->tickets.find(tk);
    if (it == S->tickets.end()) return TM_ENOTFOUND;
    tmc::Request *r = it->second;
    if (r->status == TM_EAGAIN) return TM_EAGAIN;
    const int st = r->status;
    if (st == TM_OK && out)
        for (int c = 0; c < 36; c++) out[c] = r->out[c];
    if (times_ns) {
        times_ns[0] = r->t_submit;
        times_ns[1] = r->t_start;
        times_ns[2] = r->t_done;
    }
    S->tickets.erase(it);
    lk.unlock();
    delete r;
    return st;
}

int tm_poll(tm_server *S, tm_ticket tk, uint64_t out[36], uint64_t times_ns[3]) {
    if (!S) return TM_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    return collect(S, tk, out, times_ns, lk);
}

int tm_wait(tm_server *S, tm_ticket tk, uint64_t out[36], uint64_t times_ns[3],
            uint32_t timeout_ms) {
    if (!S) return TM_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    const auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms);
    while (true) {
        auto it = S->tickets.find(tk);
        if (it == S->tickets.end()) return TM_ENOTFOUND;
        if (it->second->status != TM_EAGAIN) return collect(S, tk, out, times_ns, lk);
        if (S->cv_done.wait_until(lk, until) == std::cv_status::timeout) return TM_EAGAIN;
    }
}

int tm_server_stats(tm_server *S, uint64_t stats[8]) {
    if (!S || !stats) return TM_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    stats[0] = S->pending.size();
    stats[1] = S->flights.size();
    stats[2] = S->resident.size();
    stats[3] = S->resident_bytes;
    stats[4] = S->flight_bytes;
    stats[5] = S->completed;
    stats[6] = S->failed;
    stats[7] = S->budget;
    return TM_OK;
}

void tm_server_destroy(tm_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->device);
    for (auto &kv : S->resident) tm_graph_free(kv.second.g);
    for (tmc::Pinned &p : S->pinned_pool) (void)hipHostFree(p.p);
    for (auto &kv : S->tickets) delete kv.second;
    if (S->stream) (void)hipStreamDestroy(S->stream);
    delete S;
}

}  // extern "C"
