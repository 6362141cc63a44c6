// Internal declarations of the HIP motif-counting library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

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

// ------------------------------------------------------- device workspace
// A bump allocator over one stream-ordered allocation; everything taken from
// it is released together.
struct Scratch {
    hipStream_t stream = nullptr;
    char *base = nullptr;
    size_t cap = 0, used = 0;
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

// Stable LSD radix sort of (key, value) pairs on bits [0, bits), 8 bits per
// pass, ping-ponging between the two buffers; *keys / *vals point at the
// sorted data on return.  tmp must hold radix_tmp_count(n) u32.
size_t radix_tmp_count(uint64_t n);
// hist_name / scatter_name label the two kernels of each pass for the tracer.
int radix_sort_u32(uint32_t **keys, uint32_t **keys_alt, uint32_t **vals, uint32_t **vals_alt,
                   uint64_t n, int bits, uint32_t *tmp, hipStream_t s, const char *hist_name,
                   const char *scatter_name);
int radix_sort_u64(uint64_t **keys, uint64_t **keys_alt, uint32_t **vals, uint32_t **vals_alt,
                   uint64_t n, int bits, uint32_t *tmp, hipStream_t s, const char *hist_name,
                   const char *scatter_name);

int fill_iota(uint32_t *p, uint64_t n, hipStream_t s);

}  // namespace tmc

// ------------------------------------------------------------------ graph
struct tm_graph {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t n = 0;
    uint64_t m = 0;
    uint64_t max_degree = 0;
    // S_u for all u, (u, t, id) order: 2m entries
    uint32_t *off = nullptr;     // n + 1
    int64_t *ent_t = nullptr;    // timestamp
    uint32_t *ent_nd = nullptr;  // (other endpoint << 1) | dir
    uint32_t *ent_r = nullptr;   // edge rank in the global (t, id) order
    uint32_t *X = nullptr;       // 2m + 1: exclusive prefix count of dir = in entries
    uint32_t *epos = nullptr;    // 2m: position of edge rank r's src entry (2r) and dst entry (2r+1)
    uint32_t *perm = nullptr;    // m: edge id of rank r
    // node-pair edge sets: all edges sorted by (min node, max node, t, id)
    uint32_t *pair_el = nullptr;  // m: rank | kOrientBit if src is the smaller node
    // node pairs with at least two edges (the only ones that hold pair or star instances)
    uint64_t n_multi = 0;
    uint32_t *mp_start = nullptr;  // n_multi: first index in pair_el
    uint32_t *mp_end = nullptr;    // n_multi: one past the last
    uint32_t *mp_lo = nullptr;     // n_multi: smaller node
    uint32_t *mp_hi = nullptr;     // n_multi: larger node
};

namespace tmc {
int build_graph_device(tm_graph *g, const int32_t *src, const int32_t *dst, const int64_t *t,
                       uint64_t m, uint32_t n_nodes, hipStream_t s);
// Counts into raw[56] (host), see tm.h for the layout.
int count_graph(tm_graph *g, int64_t delta, uint32_t run_chunk, uint32_t tri_lane_max,
                uint64_t raw[56]);
}  // namespace tmc
