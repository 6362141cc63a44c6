// Caching device allocator.
//
// Graph buffers and per-count scratch are taken from per-device free lists
// instead of hipMalloc / hipFree (whose host-side cost is tens of
// microseconds per call and which synchronise the device).  A freed block
// keeps the stream it was freed on and an event recorded there; reusing it on
// the same stream is ordered by the stream itself, reusing it on another
// stream first makes that stream wait for the event.  Blocks stay cached
// until the process ends or an allocation fails, in which case the cache is
// released and the allocation retried once.
#include <atomic>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "tm_internal.h"

namespace tmc {

namespace {

struct FreeBlock {
    void *p;
    size_t size;
    hipStream_t stream;
    hipEvent_t ready;
};

struct DeviceCache {
    std::multimap<size_t, FreeBlock> free_blocks;
    std::unordered_map<void *, size_t> live;
    std::vector<hipEvent_t> events;
};

std::mutex g_mu;
std::unordered_map<int, DeviceCache> g_cache;
std::atomic<uint64_t> g_alloc_calls{0};

size_t round_size(size_t bytes) {
    if (bytes == 0) bytes = 1;
    const size_t small = 512, big = (size_t)2 << 20;
    return bytes <= ((size_t)1 << 20) ? (bytes + small - 1) / small * small
                                      : (bytes + big - 1) / big * big;
}

hipEvent_t take_event(DeviceCache &c) {
    if (!c.events.empty()) {
        hipEvent_t e = c.events.back();
        c.events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// Release every cached block of this device (caller holds g_mu).
void release_cached(DeviceCache &c) {
    for (auto &kv : c.free_blocks) {
        if (kv.second.ready) {
            (void)hipEventSynchronize(kv.second.ready);
            c.events.push_back(kv.second.ready);
        }
        (void)hipFree(kv.second.p);
    }
    c.free_blocks.clear();
}

}  // namespace

uint64_t dev_alloc_calls() { return g_alloc_calls.load(); }

int dev_alloc(void **out, size_t bytes, hipStream_t s) {
    *out = nullptr;
    g_alloc_calls.fetch_add(1);
    int dev = 0;
    (void)hipGetDevice(&dev);
    const size_t size = round_size(bytes);
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache &c = g_cache[dev];
    // best fit among cached blocks, without wasting more than half of a block
    auto it = c.free_blocks.lower_bound(size);
    if (it != c.free_blocks.end() && it->first <= 2 * size + ((size_t)4 << 20)) {
        FreeBlock b = it->second;
        c.free_blocks.erase(it);
        if (b.ready) {
            if (b.stream != s) (void)hipStreamWaitEvent(s, b.ready, 0);
            c.events.push_back(b.ready);
        }
        c.live[b.p] = b.size;
        *out = b.p;
        return TM_OK;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, size);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release_cached(c);
        e = hipMalloc(&p, size);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error(std::string("hipMalloc(") + std::to_string(size) + "): " + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? TM_ENOMEM : TM_EHIP;
    }
    c.live[p] = size;
    *out = p;
    return TM_OK;
}

size_t dev_block_size(void *p) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache &c = g_cache[dev];
    auto it = c.live.find(p);
    return it == c.live.end() ? 0 : it->second;
}

size_t graph_bytes(const tm_graph *g) {
    size_t b = 0;
    for (void *p : g->allocs) b += dev_block_size(p);
    return b;
}

size_t build_peak_bytes(uint64_t m, uint64_t n, uint32_t G) {
    // scratch (sort buffers, ranks, scans) + the graph's own arrays, both
    // bounded per edge; see the buffer layout of the build
    return (size_t)m * 240 + (size_t)n * 8 + (size_t)G * 64 + ((size_t)64 << 20);
}

void dev_free(void *p, hipStream_t s) {
    if (!p) return;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceCache &c = g_cache[dev];
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    const size_t size = it->second;
    c.live.erase(it);
    hipEvent_t ev = take_event(c);
    if (ev) (void)hipEventRecord(ev, s);
    c.free_blocks.emplace(size, FreeBlock{p, size, s, ev});
}

}  // namespace tmc
