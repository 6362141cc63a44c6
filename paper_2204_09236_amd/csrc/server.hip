// Serving: a request loop that counts many temporal graphs as requests
// arrive, with continuous batching on one GPU.
//
// A request is (graph, delta).  Graphs are either keyed -- built once and kept
// resident on the device under their key, so later requests for the same key
// only count -- or anonymous (edges come with the request, freed afterwards).
// Two threads share the work:
// * the scheduler repeats
//   1. retire: in-flight counts whose completion event has fired are turned
//      into motif counts; their tickets complete and their device bytes are
//      released from the budget;
//   2. take built graphs from the builder: a keyed graph becomes resident, an
//      anonymous union batch becomes a flight, and each count is launched;
//   3. admit: pending requests, oldest first, while the number of counts in
//      flight or being built and the device-byte budget allow.  A request for
//      a resident graph is launched at once; one for a key whose graph is
//      still being built waits in the queue (later requests are admitted past
//      it); a keyed graph that is not resident is handed to the builder
//      (evicting idle resident graphs, least recently used first, when the
//      budget is short); anonymous requests admitted together go to the
//      builder as one union batch;
// * the builder builds those graphs one after another on its own stream, so
//   a large build never stalls retiring, launching and admitting the others.
// Counts are issued asynchronously (captured count graph replayed on the
// graph's own stream, counters copied to pinned host memory, completion
// event), so counts of different requests overlap on the device and a
// request that arrives while others run is admitted as soon as a slot and
// memory are free.  The budget is an admission bound on the bytes the
// server's graphs, builds and counts need (estimated before a build,
// measured after); the device allocator caches freed blocks for reuse.
#include <algorithm>
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
    std::string error;       // the failing call's message (status != TM_OK)
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

// A graph for the builder: one keyed request's graph, or the union batch of
// anonymous requests admitted together (member i answers reqs[i]).
struct BuildJob {
    std::vector<Request *> reqs;
    uint64_t key = 0;     // 0: anonymous union batch
    size_t need = 0;      // bytes charged to the budget while it builds
    tm_graph *g = nullptr;
    int rc = TM_OK;
    std::string error;    // the builder's message when rc != TM_OK
    Pinned deltas, res;   // a union batch's count buffers, taken by the builder
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
    hipStream_t stream = nullptr;        // counts
    hipStream_t build_stream = nullptr;  // builds (builder thread)
    std::thread worker, builder;
    std::condition_variable cv_build;
    std::deque<tmc::BuildJob *> build_q;  // to the builder (under mu)
    std::deque<tmc::BuildJob *> built_q;  // back to the scheduler (under mu)
    // jobs handed to the builder and not yet taken back, and their budget
    // charge (changed by the scheduler under mu)
    uint32_t builds = 0;
    size_t build_bytes = 0;
    // scheduler-thread state (read for stats under mu)
    std::unordered_map<uint64_t, tmc::Resident> resident;
    // keys whose graph is being built from an admitted request (under mu)
    std::unordered_set<uint64_t> building;
    std::vector<tmc::Flight> flights;
    std::mutex pin_mu;  // the pinned pool is shared by the scheduler and the builder
    std::vector<tmc::Pinned> pinned_pool;
    size_t resident_bytes = 0, flight_bytes = 0;
    uint64_t completed = 0, failed = 0, clock = 0;
};

namespace tmc {
namespace {

// A pinned host buffer of at least `bytes` from the pool, allocated when none
// fits.  The scheduler's flights of one request take the 4 KiB buffers the
// server allocates up front; larger ones (union batches) are taken by the
// builder before it hands a batch over, so pinned allocations (which are not
// allowed while another thread captures a stream) only happen there.
int take_pinned(tm_server *S, size_t bytes, Pinned *out) {
    {
        std::lock_guard<std::mutex> lk(S->pin_mu);
        for (size_t i = 0; i < S->pinned_pool.size(); i++)
            if (S->pinned_pool[i].bytes >= bytes) {
                *out = S->pinned_pool[i];
                S->pinned_pool.erase(S->pinned_pool.begin() + (long)i);
                return TM_OK;
            }
    }
    size_t cap = 4096;
    while (cap < bytes) cap <<= 1;
    void *p = nullptr;
    TM_HIP_TRY(hipHostMalloc(&p, cap, hipHostMallocDefault));
    *out = Pinned{p, cap};
    return TM_OK;
}

void give_pinned(tm_server *S, Pinned &p) {
    if (p.p) {
        std::lock_guard<std::mutex> lk(S->pin_mu);
        S->pinned_pool.push_back(p);
    }
    p = Pinned{};
}

void finish(tm_server *S, Request *r, int status) {
    std::lock_guard<std::mutex> lk(S->mu);
    r->status = status;
    if (status != TM_OK) r->error = last_error();  // of this (scheduler or builder) thread
    r->t_done = now_ns();
    if (status == TM_OK) S->completed++;
    else S->failed++;
    S->cv_done.notify_all();
}

size_t budget_used(const tm_server *S) {
    return S->resident_bytes + S->flight_bytes + S->build_bytes;
}

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
    int rc = f.deltas.p ? TM_OK : take_pinned(S, (size_t)G * 8, &f.deltas);
    if (!rc && !f.res.p) rc = take_pinned(S, (size_t)G * 40 * 8, &f.res);
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
                          S->build_stream, g);
}

void drop_edges(Request *r) {
    r->src.clear();
    r->src.shrink_to_fit();
    r->dst.clear();
    r->dst.shrink_to_fit();
    r->t.clear();
    r->t.shrink_to_fit();
}

// Builder thread: one job at a time.  An invalid member of a union batch
// must not fail the others, so a batch whose build is refused as invalid is
// retried without its invalid members (found by building each alone); they
// complete here with their error.  The finished graph then counts on the
// scheduler's stream (its build is complete, every build ends by
// synchronising its stream).
void build_job(tm_server *S, BuildJob *job) {
    tm_graph *g = nullptr;
    int rc;
    if (job->key) {
        rc = build_one(S, job->reqs[0], &g);
    } else {
        auto union_build = [&](const std::vector<Request *> &rs) {
            const uint32_t G = (uint32_t)rs.size();
            std::vector<uint64_t> eoff(G + 1, 0);
            std::vector<uint32_t> ncount(G);
            for (uint32_t i = 0; i < G; i++) {
                eoff[i + 1] = eoff[i] + rs[i]->m;
                ncount[i] = rs[i]->n;
            }
            std::vector<int32_t> src(eoff[G]), dst(eoff[G]);
            std::vector<int64_t> t(eoff[G]);
            for (uint32_t i = 0; i < G; i++) {
                std::copy(rs[i]->src.begin(), rs[i]->src.end(), src.begin() + (long)eoff[i]);
                std::copy(rs[i]->dst.begin(), rs[i]->dst.end(), dst.begin() + (long)eoff[i]);
                std::copy(rs[i]->t.begin(), rs[i]->t.end(), t.begin() + (long)eoff[i]);
            }
            return tm_build_batch(src.data(), dst.data(), t.data(), eoff.data(), ncount.data(), G,
                                  TM_HOST_PTRS, S->build_stream, &g);
        };
        rc = union_build(job->reqs);
        if (rc == TM_EINVAL && job->reqs.size() > 1) {
            std::vector<Request *> good;
            for (Request *r : job->reqs) {
                tm_graph *one = nullptr;
                const int r1 = build_one(S, r, &one);
                if (r1) finish(S, r, r1);
                else {
                    good.push_back(r);
                    tm_graph_free(one);
                }
            }
            job->reqs.swap(good);
            rc = job->reqs.empty() ? TM_OK : union_build(job->reqs);
        }
    }
    if (g) {
        g->stream = S->stream;
        // the count plan is captured here too: captures and builds then never
        // overlap (some calls a build makes are not allowed while another
        // thread captures a stream), and the scheduler only replays plans
        if (rc == TM_OK) rc = count_plan_prepare(g);
        if (rc == TM_OK && !job->key) {
            // at least 8 KiB: the 4 KiB buffers stay for the scheduler
            rc = take_pinned(S, std::max<size_t>((size_t)g->G * 8, 8192), &job->deltas);
            if (rc == TM_OK) rc = take_pinned(S, std::max<size_t>((size_t)g->G * 40 * 8, 8192), &job->res);
        }
        if (rc) {
            tm_graph_free(g);
            g = nullptr;
        }
    }
    job->g = g;
    job->rc = rc;
    if (rc) job->error = last_error();
}

void builder_main(tm_server *S) {
    (void)hipSetDevice(S->device);
    while (true) {
        BuildJob *job = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_build.wait(lk, [S] { return S->stop || !S->build_q.empty(); });
            if (S->build_q.empty()) break;  // stopping, nothing left to build
            job = S->build_q.front();
            S->build_q.pop_front();
        }
        build_job(S, job);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->built_q.push_back(job);
        }
        S->cv_work.notify_all();
    }
}

void launch_flight(tm_server *S, Flight &f) {
    const int rc = launch(S, f);
    S->flights.push_back(f);
    if (rc) {
        for (Request *r : f.reqs) finish(S, r, rc);
        release_flight(S, S->flights.back());
        S->flights.pop_back();
    }
}

// Take finished builds back: keyed graphs become resident and count their
// request; union batches count as one flight.  Returns how many.
int take_built(tm_server *S) {
    std::deque<BuildJob *> done;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        done.swap(S->built_q);
    }
    for (BuildJob *job : done) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->builds--;
            S->build_bytes -= job->need;
        }
        if (job->key) {
            Request *r = job->reqs[0];
            if (job->rc) {
                {
                    std::lock_guard<std::mutex> lk(S->mu);
                    S->building.erase(job->key);
                }
                set_error(job->error);
                finish(S, r, job->rc);
                delete job;
                continue;
            }
            Resident rg;
            rg.g = job->g;
            rg.bytes = graph_bytes(job->g) + count_workspace_bytes(job->g);
            rg.last_use = ++S->clock;
            rg.inflight = 1;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                // queued requests for this key that came without edges need it
                for (Request *q : S->pending)
                    if (q->key == job->key && !q->has_edges) rg.queued++;
                S->resident[job->key] = rg;
                S->building.erase(job->key);
            }
            S->resident_bytes += rg.bytes;
            drop_edges(r);
            Flight f;
            f.reqs.push_back(r);
            f.g = job->g;
            f.key = job->key;
            launch_flight(S, f);
        } else if (job->rc) {
            set_error(job->error);
            for (Request *r : job->reqs) finish(S, r, job->rc);
        } else if (!job->reqs.empty()) {
            for (Request *r : job->reqs) drop_edges(r);
            Flight f;
            f.reqs = job->reqs;
            f.g = job->g;
            f.owned = true;
            f.deltas = job->deltas;
            f.res = job->res;
            job->deltas = job->res = Pinned{};
            f.footprint = graph_bytes(job->g) + count_workspace_bytes(job->g);
            S->flight_bytes += f.footprint;
            launch_flight(S, f);
        }
        give_pinned(S, job->deltas);
        give_pinned(S, job->res);
        delete job;
    }
    return (int)done.size();
}

// Admit pending requests, oldest first, while slots and budget allow.  A
// request for a key that is still being built stays queued and later ones
// are admitted past it.
void admit(tm_server *S) {
    std::vector<Request *> anon;
    size_t anon_need = 0;
    auto slots_used = [&]() { return S->flights.size() + S->builds + (anon.empty() ? 0 : 1); };
    std::vector<Request *> order;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        order.assign(S->pending.begin(), S->pending.end());
    }
    auto remove_locked = [&](Request *r) {  // caller holds S->mu
        for (auto it = S->pending.begin(); it != S->pending.end(); ++it)
            if (*it == r) {
                S->pending.erase(it);
                break;
            }
    };
    auto take = [&](Request *r) {  // remove r from the queue
        std::lock_guard<std::mutex> lk(S->mu);
        remove_locked(r);
    };
    for (Request *r : order) {
        if (slots_used() >= S->max_inflight) break;
        bool is_resident = false, is_building = false;
        Resident *rgp = nullptr;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (r->key) {
                auto it = S->resident.find(r->key);
                is_resident = it != S->resident.end();
                if (is_resident) rgp = &it->second;
                is_building = S->building.count(r->key) != 0;
            }
        }
        if (is_resident) {
            take(r);
            {
                std::lock_guard<std::mutex> lk(S->mu);
                if (!r->has_edges) rgp->queued--;
            }
            if (r->has_edges) drop_edges(r);
            Flight f;
            f.reqs.push_back(r);
            f.g = rgp->g;
            f.key = r->key;
            r->t_start = now_ns();
            rgp->inflight++;
            launch_flight(S, f);
            continue;
        }
        if (is_building) continue;  // its graph comes with a build in progress
        const size_t need = build_peak_bytes(r->m, r->n, 1);
        if (need > S->budget) {
            take(r);
            set_error("request needs more device memory than the server budget");
            finish(S, r, TM_ENOMEM);
            continue;
        }
        if (r->key && !r->has_edges) {
            // its graph was to come from an earlier request that failed
            take(r);
            set_error("graph key is not resident and the request carries no edges");
            finish(S, r, TM_ENOTFOUND);
            continue;
        }
        if (r->key) {
            if (!make_room(S, need + anon_need)) break;
            r->t_start = now_ns();
            auto *job = new BuildJob();
            job->reqs.push_back(r);
            job->key = r->key;
            job->need = need;
            {
                // leaving the queue and becoming "being built" in one
                // critical section: a submit in between would otherwise find
                // the key nowhere
                std::lock_guard<std::mutex> lk(S->mu);
                remove_locked(r);
                S->builds++;
                S->build_bytes += need;
                S->building.insert(r->key);
                S->build_q.push_back(job);
            }
            S->cv_build.notify_one();
            continue;
        }
        // anonymous: join the union batch of this admission cycle
        if (!make_room(S, anon_need + need)) break;
        take(r);
        r->t_start = now_ns();
        anon.push_back(r);
        anon_need += need;
    }
    if (anon.empty()) return;
    auto *job = new BuildJob();
    job->reqs = anon;
    job->need = anon_need;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->builds++;
        S->build_bytes += anon_need;
        S->build_q.push_back(job);
    }
    S->cv_build.notify_one();
}

void worker_main(tm_server *S) {
    (void)hipSetDevice(S->device);
    while (true) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->flights.empty() && S->built_q.empty() && S->builds == 0 && S->pending.empty() &&
                !S->stop)
                S->cv_work.wait(lk, [S] {
                    return S->stop || !S->pending.empty() || !S->built_q.empty();
                });
            if (S->stop) break;
        }
        const int retired = retire(S, false);
        const int built = take_built(S);
        admit(S);
        if (retired == 0 && built == 0 && (!S->flights.empty() || S->builds > 0)) {
            // counts in flight or builds running and nothing finished yet:
            // brief back-off (a finished build wakes it at once)
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->built_q.empty()) S->cv_work.wait_for(lk, std::chrono::microseconds(50));
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
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&S->build_stream, hipStreamNonBlocking) != hipSuccess) {
        tmc::set_error("hipStreamCreate failed");
        if (S->stream) (void)hipStreamDestroy(S->stream);
        delete S;
        return TM_EHIP;
    }
    // pinned buffers for the flights of single requests, allocated before
    // any thread can capture a stream
    {
        std::vector<tmc::Pinned> held(2 * (max_inflight + 1));
        for (tmc::Pinned &p : held)
            if (tmc::take_pinned(S, 4096, &p) != TM_OK) break;
        for (tmc::Pinned &p : held) tmc::give_pinned(S, p);
    }
    S->worker = std::thread(tmc::worker_main, S);
    S->builder = std::thread(tmc::builder_main, S);
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
    if (st != TM_OK) tmc::set_error(r->error);  // readable by tm_last_error in the caller
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
    stats[1] = S->flights.size() + S->builds;
    stats[2] = S->resident.size();
    stats[3] = S->resident_bytes;
    stats[4] = S->flight_bytes + S->build_bytes;
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
    {
        // builds not started are dropped; the one running finishes first
        std::lock_guard<std::mutex> lk(S->mu);
        for (tmc::BuildJob *job : S->build_q) delete job;
        S->build_q.clear();
    }
    S->cv_build.notify_all();
    if (S->builder.joinable()) S->builder.join();
    (void)hipSetDevice(S->device);
    for (tmc::BuildJob *job : S->built_q) {
        if (job->g) tm_graph_free(job->g);
        tmc::give_pinned(S, job->deltas);
        tmc::give_pinned(S, job->res);
        delete job;
    }
    for (auto &kv : S->resident) tm_graph_free(kv.second.g);
    for (tmc::Pinned &p : S->pinned_pool) (void)hipHostFree(p.p);
    for (auto &kv : S->tickets) delete kv.second;
    if (S->stream) (void)hipStreamDestroy(S->stream);
    if (S->build_stream) (void)hipStreamDestroy(S->build_stream);
    delete S;
}

}  // extern "C"
