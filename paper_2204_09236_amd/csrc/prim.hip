// Device primitives: exclusive scan and a stable LSD radix sort, written for
// 64-wide CDNA wavefronts (ballot-based digit matching, no block barriers in
// the ranking loop).
#include <algorithm>
#include <atomic>
#include <type_traits>
#include <utility>

#include "tm_internal.h"

namespace tmc {

namespace {

__device__ inline uint64_t lanemask_lt(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

template <typename T>
__device__ inline T wave_incl_scan(T v, int lane) {
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(v, o, kWave);
        if (lane >= o) v += y;
    }
    return v;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Inclusive scan over the NT threads of the block; *total receives the
// block sum; lds4 holds NT / 64 values.
template <typename T, int NT = kBlock>
__device__ inline T block_incl_scan(T v, T *total, T *lds4) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    T s = wave_incl_scan(v, lane);
    if (lane == kWave - 1) lds4[w] = s;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / kWave; i++) {
        T x = lds4[i];
        if (i < w) pre += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return s + pre;
}

template <typename T>
__device__ inline T block_sum(T v, T *lds4) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    T s = wave_sum(v);
    if (lane == 0) lds4[w] = s;
    __syncthreads();
    T tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; i++) tot += lds4[i];
    __syncthreads();
    return tot;
}

// A scan's input: ld(i) is element i's value, of type L::value_type.
struct LoadArray {
    using value_type = uint32_t;
    const uint32_t *p;
    __device__ uint32_t operator()(uint64_t i) const { return p[i]; }
};
struct LoadDirBit {
    using value_type = uint32_t;
    const uint32_t *nd;
    __device__ uint32_t operator()(uint64_t i) const { return nd[i] & 1u; }
};
// 1 for an entry of S seen from the smaller node of its edge
struct LoadLowerSide {
    using value_type = uint32_t;
    const uint32_t *c, *nd;
    __device__ uint32_t operator()(uint64_t i) const { return (nd[i] >> 1) > c[i] ? 1u : 0u; }
};
// A flag byte (bit 0 to the low word, bit 1 to the high word)
struct LoadFlagPair {
    using value_type = uint64_t;
    const uint8_t *f;
    __device__ uint64_t operator()(uint64_t i) const {
        const uint32_t b = f[i];
        return (uint64_t)(b & 1u) | ((uint64_t)(b >> 1) << 32);
    }
};

template <typename L>
__global__ void __launch_bounds__(kBlock) k_tile_sum(L ld, uint64_t n, typename L::value_type *part) {
    using T = typename L::value_type;
    __shared__ T lds[kBlock / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    T acc = 0;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        const uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
        if (idx < n) acc += ld(idx);
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// One block of kPartsThreads: exclusive scan of np partial sums in place;
// part[np] = total.  Each thread takes kPartsPer consecutive sums a round.
constexpr int kPartsThreads = 1024;
constexpr int kPartsPer = 8;

template <typename T>
__global__ void __launch_bounds__(kPartsThreads) k_scan_parts(T *part, uint32_t np) {
    __shared__ T lds[kPartsThreads / kWave];
    T carry = 0;
    for (uint64_t b = 0; b < np; b += (uint64_t)kPartsThreads * kPartsPer) {
        const uint64_t i0 = b + (uint64_t)threadIdx.x * kPartsPer;
        T x[kPartsPer];
        T sum = 0;
#pragma unroll
        for (int k = 0; k < kPartsPer; k++) {
            x[k] = i0 + k < np ? part[i0 + k] : T(0);
            sum += x[k];
        }
        T tot;
        const T inc = block_incl_scan<T, kPartsThreads>(sum, &tot, lds);
        T run = carry + inc - sum;
#pragma unroll
        for (int k = 0; k < kPartsPer; k++) {
            if (i0 + k < np) part[i0 + k] = run;
            run += x[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) part[np] = carry;
}

// Where a scan's results go: wr(i, exclusive prefix, value) per element and
// wr.total(n, total) once.  ArrayWrite stores the prefixes (out[n] = total).
// kLoads: the writer reads memory of its own per element; such a scan keeps
// every element's load, scan and write in one round of the block (barriers
// between rounds), so that the writer's loads of different rounds overlap
// with other blocks' work rather than waiting one after another.
template <typename T>
struct ArrayWriteT {
    static constexpr bool kLoads = false;
    T *out;
    __device__ void operator()(uint64_t i, T ex, T) const { out[i] = ex; }
    __device__ void total(uint64_t n, T t) const { out[n] = t; }
};
using ArrayWrite = ArrayWriteT<uint32_t>;

// The pair sort's input: each edge once, from its entry at the smaller node
// (S order: smaller node, then (t, id)), as key = the larger node, value =
// (smaller node, rank | orientation), compacted by the scan of LoadLowerSide.
// A stable sort by the key then groups every node pair, its edges in (t, id)
// order, pairs by (larger, smaller).
struct LowerSideWrite {
    static constexpr bool kLoads = true;
    const uint32_t *c, *nd, *r;
    uint32_t *key;
    uint2 *val;
    __device__ void operator()(uint64_t i, uint32_t ex, uint32_t v) const {
        if (!v) return;
        const uint32_t e = nd[i];
        key[ex] = e >> 1;
        // direction bit 0: the edge leaves the center, so its source is the smaller node
        val[ex] = make_uint2(c[i], r[i] | ((e & 1u) ? 0u : kOrientBit));
    }
    __device__ void total(uint64_t, uint32_t) const {}
};

// One tile of a scan, kTile elements from base.  Returns the tile's total.
// Without writer loads: wave w owns the contiguous run [base + w * kItems *
// 64, ...) and walks it in kItems rounds of 64 lanes, so (wave, round, lane)
// is input order; all loads are issued first, each round is scanned within
// the wave with a running carry, and one barrier exchanges the wave totals.
// With writer loads: kItems rounds of kBlock elements, each scanned over the
// block.
template <typename L, typename W>
__device__ __forceinline__ typename L::value_type scan_tile_body(L ld, uint64_t n, uint64_t base,
                                                        typename L::value_type start, W wr,
                                                        typename L::value_type *wsum) {
    using T = typename L::value_type;
    if constexpr (W::kLoads) {
        T carry = start;
        for (int i = 0; i < kItems; i++) {
            const uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
            const T v = idx < n ? ld(idx) : T(0);
            T tot;
            const T inc = block_incl_scan(v, &tot, wsum);
            if (idx < n) wr(idx, carry + inc - v, v);
            carry += tot;
        }
        return carry - start;
    } else {
        const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
        const uint64_t wbase = base + (uint64_t)w * kItems * kWave;
        T v[kItems];
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            const uint64_t idx = wbase + (uint64_t)i * kWave + lane;
            v[i] = idx < n ? ld(idx) : T(0);
        }
        T ex[kItems];
        T carry = 0;
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            const T inc = wave_incl_scan(v[i], lane);
            ex[i] = carry + inc - v[i];
            carry += __shfl(inc, kWave - 1, kWave);
        }
        if (lane == 0) wsum[w] = carry;
        __syncthreads();
        T off = start, tot = start;
#pragma unroll
        for (int j = 0; j < kBlock / kWave; j++) {
            const T x = wsum[j];
            off += j < w ? x : T(0);
            tot += x;
        }
#pragma unroll
        for (int i = 0; i < kItems; i++) {
            const uint64_t idx = wbase + (uint64_t)i * kWave + lane;
            if (idx < n) wr(idx, off + ex[i], v[i]);
        }
        return tot - start;
    }
}

template <typename L, typename W>
__global__ void __launch_bounds__(kBlock) k_tile_scan(L ld, uint64_t n,
                                                      const typename L::value_type *part,
                                                      uint32_t np, W wr) {
    using T = typename L::value_type;
    __shared__ T wsum[kBlock / kWave];
    scan_tile_body(ld, n, (uint64_t)blockIdx.x * kTile, part[blockIdx.x], wr, wsum);
    if (blockIdx.x == 0 && threadIdx.x == 0) wr.total(n, part[np]);
}

// The whole scan when the input fits one tile: one launch instead of three.
template <typename L, typename W>
__global__ void __launch_bounds__(kBlock) k_scan_one(L ld, uint64_t n, W wr) {
    using T = typename L::value_type;
    __shared__ T wsum[kBlock / kWave];
    const T tot = scan_tile_body(ld, n, 0, T(0), wr, wsum);
    if (threadIdx.x == 0) wr.total(n, tot);
}

template <typename W>
__global__ void k_scan_empty(W wr) { wr.total(0, 0); }

// tmp: scan_tmp_count(n) elements of L::value_type.
// Trace names of the tile-sum and tile-scan launches: sum_name, tile_name.
template <typename L, typename W = ArrayWrite>
int scan_impl(L ld, W wr, uint64_t n, typename L::value_type *tmp, hipStream_t s,
              const char *sum_name = "scan_tile_sum", const char *tile_name = "scan_tile") {
    using T = typename L::value_type;
    const uint64_t nb = (n + kTile - 1) / kTile;
    if (nb == 0) {
        // a kernel, not a memset: this may run inside a captured graph
        TM_LAUNCH("scan_empty", k_scan_empty<W>, dim3(1), dim3(1), 0, s, wr);
        return TM_OK;
    }
    if (nb == 1) {
        TM_LAUNCH("scan_one", (k_scan_one<L, W>), dim3(1), dim3(kBlock), 0, s, ld, n, wr);
        return TM_OK;
    }
    TM_LAUNCH(sum_name, (k_tile_sum<L>), dim3(nb), dim3(kBlock), 0, s, ld, n, tmp);
    TM_LAUNCH("scan_parts", k_scan_parts<T>, dim3(1), dim3(kPartsThreads), 0, s, tmp, (uint32_t)nb);
    TM_LAUNCH(tile_name, (k_tile_scan<L, W>), dim3(nb), dim3(kBlock), 0, s, ld, n, tmp,
              (uint32_t)nb, wr);
    return TM_OK;
}

// ------------------------------------------------------------ radix sort
// Stable LSD radix sort, 8-bit digits, one kernel per digit pass.
//
// A histogram kernel reads the keys once and counts the digits of every
// pass.  In a pass, each block takes the next tile in input order from a
// counter, ranks its keys (wave w owns the contiguous run
// [w * ITEMS * 64, (w + 1) * ITEMS * 64) of the tile and walks it in ITEMS
// rounds of 64, so tile order = (wave, round, lane) = input order and a
// per-wave running digit count gives stable ranks without block barriers),
// publishes its 256 digit counts, and adds up the counts of all earlier
// tiles by decoupled look-back: each earlier tile's word holds either its
// own count (aggregate) or the count of itself and everything before it
// (inclusive), and the walk stops at the first inclusive word.  The tile is
// then staged in LDS in digit order so that each digit's run is written to
// HBM contiguously.
constexpr int kOsThreads = 512;
constexpr int kOsWaves = kOsThreads / kWave;
constexpr int kMaxPasses = 8;
constexpr int kHistItems = 4;
constexpr uint64_t kStAgg = 1ull << 62;
constexpr uint64_t kStInc = 2ull << 62;
constexpr uint64_t kStVal = (1ull << 62) - 1;
// A look-back wait polls at most this many times (about a second) before it
// gives up, flags the error and lets the kernel finish.
constexpr uint32_t kSpinLimit = 1u << 20;
std::atomic<uint32_t> g_spin_limit{kSpinLimit};
uint32_t lookback_spin_limit() { return g_spin_limit.load(std::memory_order_relaxed); }
constexpr uint64_t kMinTile = (uint64_t)kOsThreads * 6;

// Block size and items per thread of a pass, by element type: the node
// sort's 20-byte elements run in 1024-thread blocks with 6144-element tiles
// (one block per CU, 141 KiB of LDS), its 16-byte ones (NodeVal32) with
// 8192-element tiles (145 KiB); the others in 512-thread blocks with
// 3072-5120-element tiles (two blocks per CU).  Measured on gfx950: longer
// digit runs per tile pay more than occupancy for the node sort.
template <typename K, typename V>
constexpr int os_threads() {
    return (std::is_same<V, NodeVal>::value || std::is_same<V, NodeVal32>::value) && sizeof(K) == 4
               ? 1024
               : kOsThreads;
}

template <typename K, typename V>
constexpr int os_items() {
    return sizeof(K) + sizeof(V) <= 12 ? 10 : (sizeof(K) + sizeof(V) <= 16 ? 8 : 6);
}

// Digit of a key and the lanes of this wave that share it (ballot matching).
template <typename K>
__device__ inline uint64_t digit_peers(K key, int shift, bool valid, uint32_t *digit) {
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    *digit = d;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        peers &= bit ? bb : ~bb;
    }
    return peers;
}

// Exclusive scan of one value per digit, held by threads [0, 256) of a
// block of at least 256 threads; every thread of the block must call it.
__device__ inline uint32_t digit_excl_scan(uint32_t v, uint32_t *lds4) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t s = wave_incl_scan(v, lane);
    if (w < 4 && lane == kWave - 1) lds4[w] = s;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (int i = 0; i < 3; i++)
        if (i < w) pre += lds4[i];
    __syncthreads();
    return s + pre - v;
}

// Zero the digit counts and tile counters of every pass and the first
// pass's look-back words.
__global__ void k_os_init(uint32_t *counts, uint32_t n_counts, uint64_t *status, uint64_t n_status) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_counts; i += stride)
        counts[i] = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_status; i += stride)
        status[i] = 0;
}

// Where a sort's first pass (and its histogram) reads its elements: plain
// arrays, or elements built on the fly from arrays another kernel wrote, so
// that no separate kernel has to write them out first.
template <typename K, typename V>
struct ArrayIn {
    const K *k;
    const V *v;
    __device__ inline K key(uint64_t i) const { return k[i]; }
    __device__ inline void load(uint64_t i, K &key, V &val) const {
        key = k[i];
        val = v[i];
    }
};

// Time sort of one graph from the input arrays: key t - tmin, value
// (src, dst, input index).
template <typename K>
struct TimeIn {
    const int32_t *src, *dst;
    const int64_t *t;
    const int64_t *tmin;  // one value, on the device
    __device__ inline K key(uint64_t i) const { return (K)(uint64_t)(t[i] - *tmin); }
    __device__ inline void load(uint64_t i, K &key, EdgeVal &val) const {
        key = (K)(uint64_t)(t[i] - *tmin);
        val = EdgeVal{(uint32_t)src[i], (uint32_t)dst[i], (uint32_t)i};
    }
};

// Digit counts of every pass over all keys: per-block LDS counters (plain
// LDS atomics: counting needs no ranks), each block writing its own row
// part[block][pass][digit]; no global atomics here, since thousands of blocks
// adding into the same 256 words serialise across the XCDs.
constexpr uint32_t kHistBlocks = 512;
constexpr uint32_t kHistSumSplit = 16;

template <typename K, typename In>
__global__ void __launch_bounds__(kOsThreads) k_os_hist(In in, uint64_t n, int passes, int shift0,
                                                        uint32_t *part) {
    __shared__ uint32_t h[kMaxPasses][256];
    for (int i = threadIdx.x; i < kMaxPasses * 256; i += kOsThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint64_t chunk = (uint64_t)kOsThreads * kHistItems;
    for (uint64_t base = (uint64_t)blockIdx.x * chunk; base < n; base += (uint64_t)gridDim.x * chunk) {
        K key[kHistItems];
#pragma unroll
        for (int i = 0; i < kHistItems; i++) {
            const uint64_t idx = base + (uint64_t)i * kOsThreads + threadIdx.x;
            key[i] = idx < n ? in.key(idx) : K(0);
        }
#pragma unroll
        for (int i = 0; i < kHistItems; i++) {
            if (base + (uint64_t)i * kOsThreads + threadIdx.x < n) {
                for (int p = 0; p < passes; p++)
                    atomicAdd(&h[p][(uint32_t)(key[i] >> (shift0 + 8 * p)) & 255u], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < passes * 256; i += kOsThreads)
        part[(uint64_t)blockIdx.x * passes * 256 + i] = (&h[0][0])[i];
}

// ghist[pass][digit] += the rows of blocks y, y + split, ... (grid: pass x
// split); a handful of global adds per counter.
__global__ void __launch_bounds__(256) k_os_hist_sum(const uint32_t *part, uint32_t nblocks,
                                                     int passes, uint32_t *ghist) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    uint32_t s = 0;
    for (uint32_t b = blockIdx.y; b < nblocks; b += gridDim.y) s += part[(uint64_t)b * passes * 256 + i];
    if (s) atomicAdd(&ghist[i], s);
}

// Digit counts of every pass when the keys are exactly 0 .. n-1 in some
// order (the edge slots): in pass p (bits [shift0 + 8p, +8)), digit d holds
// n / 2^(sh+8) full runs of 2^sh keys plus what the last, partial cycle
// gives it.  Grid: one block of 256 per pass.
__global__ void __launch_bounds__(256) k_os_hist_iota(uint64_t n, int shift0, uint32_t *ghist) {
    const int p = blockIdx.x, d = threadIdx.x;
    const int sh = shift0 + 8 * p;
    const uint64_t w = 1ull << sh, cyc = w << 8;
    const uint64_t rem = n % cyc, lo = (uint64_t)d * w;
    const uint64_t extra = rem > lo ? min(rem - lo, w) : 0ull;
    ghist[256 * p + d] = (uint32_t)((n / cyc) * w + extra);
}

template <typename K, typename V>
struct PairOut {
    K *kout;
    V *vout;
    __device__ inline void operator()(uint32_t pos, K k, const V &v) const {
        kout[pos] = k;
        vout[pos] = v;
    }
};

__device__ inline int64_t node_time(const NodeVal &v, int64_t) { return v.t; }
__device__ inline int64_t node_time(const NodeVal32 &v, int64_t base) {
    return base + (int64_t)v.dt;
}

template <typename V>
struct SeqWrite {
    SeqOut o;
    __device__ inline void operator()(uint32_t pos, uint32_t k, const V &v) const {
        o.ent_c[pos] = k;
        o.ent_t[pos] = node_time(v, o.tbase);
        o.ent_nd[pos] = v.nd;
        o.ent_r[pos] = v.r;
        // the entry's slot: 2r at the source, 2r + 1 at the destination
        const uint32_t slot = 2 * v.r + (v.nd & 1u);
        if (o.epos) {
            // a slot outside [0, n) only after an abandoned look-back (flagged)
            if (slot < o.n) o.epos[slot] = pos;
        } else {
            o.slot[pos] = slot;  // in entry order, for edge_positions
        }
    }
};

// Slots in entry order as sort input: key = slot, value = its position.
struct SlotIn {
    const uint32_t *slot;
    __device__ inline uint32_t key(uint64_t i) const { return slot[i]; }
    __device__ inline void load(uint64_t i, uint32_t &key, uint32_t &val) const {
        key = slot[i];
        val = (uint32_t)i;
    }
};

template <typename K>
struct RankWrite {
    RankOut o;
    __device__ inline void operator()(uint32_t r, K key, const EdgeVal &ev) const {
        const uint64_t k = (uint64_t)key;
        const uint32_t gi = o.tbits >= 64 ? 0u : (uint32_t)(k >> o.tbits);
        const uint64_t tmask = o.tbits >= 64 ? ~0ull : ((1ull << o.tbits) - 1);
        const int64_t te = (int64_t)((k & tmask) + (uint64_t)o.tmin[gi]);
        o.t_r[r] = te;
        o.perm[r] = ev.id;
        o.nkey[2 * (uint64_t)r] = ev.src;
        o.nkey[2 * (uint64_t)r + 1] = ev.dst;
        if (o.nval32) {
            const uint32_t dt = (uint32_t)(te - o.tbase);
            o.nval32[2 * (uint64_t)r] = NodeVal32{dt, r, ev.dst << 1};
            o.nval32[2 * (uint64_t)r + 1] = NodeVal32{dt, r, (ev.src << 1) | 1u};
        } else {
            o.nval[2 * (uint64_t)r] = NodeVal{te, r, ev.dst << 1};
            o.nval[2 * (uint64_t)r + 1] = NodeVal{te, r, (ev.src << 1) | 1u};
        }
    }
};

// One digit pass.  ghist: this pass's 256 digit counts over all keys;
// status: this pass's look-back words (tile x 256, zero on entry);
// status_next: the next pass's words, whose row for this tile is cleared
// here (null on the last pass); ticket: tile counter (zero on entry).
template <typename K, typename V, typename In, typename Out, int THREADS, int ITEMS>
__global__ void __launch_bounds__(THREADS) k_os_scatter(In in, Out out,
                                                           uint64_t n, int shift,
                                                           const uint32_t *ghist, uint64_t *status,
                                                           uint64_t *status_next, uint32_t *ticket,
                                                           uint32_t *err, uint32_t spin_limit) {
    constexpr uint32_t kT = (uint32_t)THREADS * ITEMS;
    constexpr int kWv = THREADS / kWave;
    __shared__ V s_val[kT];
    __shared__ K s_key[kT];
    __shared__ uint32_t wh[kWv][256];
    __shared__ uint32_t blk_off[256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t lds4[4];
    __shared__ uint32_t s_tile;
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int i = threadIdx.x; i < kWv * 256; i += THREADS) (&wh[0][0])[i] = 0;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (status_next && threadIdx.x < 256) status_next[(uint64_t)tile * 256 + threadIdx.x] = 0;
    const uint64_t tile0 = (uint64_t)tile * kT;
    const uint64_t base = tile0 + (uint64_t)w * (ITEMS * kWave);
    const uint64_t lt = lanemask_lt(lane);
    // values travel in registers as 32-bit words (struct-typed register
    // arrays are not promoted and would spill)
    static_assert(sizeof(V) % 4 == 0, "value size must be a multiple of 4 bytes");
    constexpr int kVW = (int)(sizeof(V) / 4);
    K key[ITEMS];
    uint32_t val[ITEMS][kVW];
    uint32_t rank[ITEMS];
    uint32_t dig[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const uint64_t idx = base + (uint64_t)i * kWave + lane;
        key[i] = K(0);
#pragma unroll
        for (int j = 0; j < kVW; j++) val[i][j] = 0;
        if (idx < n) {
            V v;
            in.load(idx, key[i], v);
            __builtin_memcpy(&val[i][0], &v, sizeof(V));
        }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const bool valid = base + (uint64_t)i * kWave + lane < n;
        uint32_t d;
        const uint64_t peers = digit_peers(key[i], shift, valid, &d);
        dig[i] = d;
        const uint32_t below = __popcll(peers & lt);
        const uint32_t cnt = __popcll(peers);
        uint32_t run = 0;
        if (valid) run = wh[w][d];
        __builtin_amdgcn_wave_barrier();
        rank[i] = run + below;
        if (valid && below == 0) wh[w][d] = run + cnt;
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    const int d = threadIdx.x;
    uint32_t c[kWv];
    uint32_t tot = 0;
    if (d < 256) {
#pragma unroll
        for (int q = 0; q < kWv; q++) {
            c[q] = wh[q][d];
            tot += c[q];
        }
    }
    const uint32_t excl = digit_excl_scan(tot, lds4);
    const uint32_t gex = digit_excl_scan(d < 256 ? ghist[d] : 0u, lds4);
    if (d < 256) {
        blk_off[d] = excl;
        uint32_t run = excl;
#pragma unroll
        for (int q = 0; q < kWv; q++) {
            wh[q][d] = run;
            run += c[q];
        }
        uint64_t *mine = status + (uint64_t)tile * 256 + d;
        uint64_t prefix = 0;
        if (tile == 0) {
            __hip_atomic_store(mine, kStInc | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(mine, kStAgg | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t k = tile - 1;
            uint32_t spins = 0;
            // a limit of 0 (set from the host by the failure-path tests)
            // gives up before the first wait
            if (spin_limit == 0) atomicOr(err, 1u);
            while (spin_limit != 0) {
                const uint64_t v = __hip_atomic_load(status + (uint64_t)k * 256 + d, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t st = v & ~kStVal;
                if (st == 0) {
                    if (++spins >= spin_limit) {
                        atomicOr(err, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                prefix += v & kStVal;
                if (st == kStInc || k == 0) break;
                k--;
            }
            __hip_atomic_store(mine, kStInc | (prefix + tot), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        gbase[d] = gex + (uint32_t)prefix;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        if (base + (uint64_t)i * kWave + lane < n) {
            const uint32_t x = wh[w][dig[i]] + rank[i];
            s_key[x] = key[i];
            __builtin_memcpy(&s_val[x], &val[i][0], sizeof(V));
        }
    }
    __syncthreads();
    const uint32_t cnt_tile = (uint32_t)min<uint64_t>((uint64_t)kT, n - tile0);
    for (uint32_t x = threadIdx.x; x < cnt_tile; x += THREADS) {
        const K k = s_key[x];
        const uint32_t dk = (uint32_t)(k >> shift) & 255u;
        const uint32_t pos = gbase[dk] + (x - blk_off[dk]);
        // only an abandoned look-back can place an element outside [0, n)
        if (pos < n) out(pos, k, s_val[x]);
        else atomicOr(err, 2u);
    }
}

// Layout of the sort's scratch: digit counts and tile counters of every
// pass, two look-back word arrays (passes alternate between them), and the
// histogram blocks' rows.
struct OsTmp {
    uint32_t *ghist;    // kMaxPasses x 256
    uint32_t *tickets;  // kMaxPasses
    uint64_t *status[2];
    uint32_t *part;     // kHistBlocks x kMaxPasses x 256
};

inline OsTmp os_tmp(void *tmp, uint64_t ntiles) {
    OsTmp t;
    t.ghist = static_cast<uint32_t *>(tmp);
    t.tickets = t.ghist + kMaxPasses * 256;
    t.status[0] = reinterpret_cast<uint64_t *>(t.tickets + kMaxPasses);  // 8-byte aligned
    t.status[1] = t.status[0] + ntiles * 256;
    t.part = reinterpret_cast<uint32_t *>(t.status[1] + ntiles * 256);
    return t;
}

// In0: where the histogram and the first pass read the elements (the later
// passes read the ping-pong buffers *keys / *vals).
// Sorts on key bits [shift0, bits).
template <typename K, typename V, typename Final, typename In0>
int radix_impl(K **keys, K **keys_alt, V **vals, V **vals_alt, uint64_t n, int bits, void *tmp,
               uint32_t *err, hipStream_t s, const char *hist_name, const char *scatter_name,
               const Final *fin, const In0 &in0, int shift0 = 0, bool iota_keys = false) {
    constexpr int kItems_ = os_items<K, V>();
    constexpr int kThr = os_threads<K, V>();
    constexpr uint64_t kT = (uint64_t)kThr * kItems_;
    const int passes = (bits - shift0 + 7) / 8;
    if (passes < 1 || passes > kMaxPasses || shift0 + 8 * (passes - 1) >= (int)sizeof(K) * 8) {
        set_error("radix sort: key bits out of range");
        return TM_EINTERNAL;
    }
    const uint64_t ntiles = (n + kT - 1) / kT;
    const OsTmp t = os_tmp(tmp, ntiles);
    const uint64_t n_status = ntiles * 256;
    TM_LAUNCH("sort_init", k_os_init, dim3((unsigned)std::min<uint64_t>((n_status + kBlock - 1) / kBlock + 1, 4096)),
              dim3(kBlock), 0, s, t.ghist, (uint32_t)(kMaxPasses * 257), t.status[0], n_status);
    if (iota_keys) {
        // keys 0 .. n-1: the digit counts follow from n alone
        TM_LAUNCH(hist_name, k_os_hist_iota, dim3((unsigned)passes), dim3(256), 0, s, n, shift0,
                  t.ghist);
    } else {
        const uint64_t hchunk = (uint64_t)kOsThreads * kHistItems;
        const uint32_t hblocks = (uint32_t)std::min<uint64_t>((n + hchunk - 1) / hchunk, kHistBlocks);
        TM_LAUNCH(hist_name, (k_os_hist<K, In0>), dim3(hblocks), dim3(kOsThreads), 0, s, in0, n,
                  passes, shift0, t.part);
        TM_LAUNCH("sort_hist_sum", k_os_hist_sum, dim3((unsigned)passes, kHistSumSplit), dim3(256), 0,
                  s, t.part, hblocks, passes, t.ghist);
    }
    const uint32_t spin = lookback_spin_limit();
    // the pass that writes the final arrays is traced under its own name
    const std::string last_name = std::string(scatter_name) + "_last";
    for (int p = 0; p < passes; p++) {
        uint64_t *st = t.status[p & 1];
        uint64_t *st_next = p + 1 < passes ? t.status[(p + 1) & 1] : nullptr;
        const ArrayIn<K, V> arr{*keys, *vals};
        const bool last = fin && p + 1 == passes;
        if (p == 0 && last) {
            TM_LAUNCH(last_name.c_str(), (k_os_scatter<K, V, In0, Final, kThr, kItems_>),
                      dim3((unsigned)ntiles), dim3(kThr), 0, s, in0, *fin, n, shift0 + 8 * p,
                      t.ghist + 256 * p, st, st_next, t.tickets + p, err, spin);
        } else if (last) {
            TM_LAUNCH(last_name.c_str(), (k_os_scatter<K, V, ArrayIn<K, V>, Final, kThr, kItems_>),
                      dim3((unsigned)ntiles), dim3(kThr), 0, s, arr, *fin, n, shift0 + 8 * p,
                      t.ghist + 256 * p, st, st_next, t.tickets + p, err, spin);
        } else {
            const PairOut<K, V> po{*keys_alt, *vals_alt};
            if (p == 0)
                TM_LAUNCH(scatter_name, (k_os_scatter<K, V, In0, PairOut<K, V>, kThr, kItems_>),
                          dim3((unsigned)ntiles), dim3(kThr), 0, s, in0, po, n, shift0 + 8 * p,
                          t.ghist + 256 * p, st, st_next, t.tickets + p, err, spin);
            else
                TM_LAUNCH(scatter_name,
                          (k_os_scatter<K, V, ArrayIn<K, V>, PairOut<K, V>, kThr, kItems_>),
                          dim3((unsigned)ntiles), dim3(kThr), 0, s, arr, po, n, shift0 + 8 * p,
                          t.ghist + 256 * p, st, st_next, t.tickets + p, err, spin);
            std::swap(*keys, *keys_alt);
            std::swap(*vals, *vals_alt);
        }
    }
    return TM_OK;
}

}  // namespace

void set_lookback_giveup(bool on) { g_spin_limit.store(on ? 0u : kSpinLimit); }

size_t scan_tmp_count(uint64_t n) { return (n + kTile - 1) / kTile + 2; }

size_t radix_tmp_bytes(uint64_t n) {
    const uint64_t ntiles = (n + kMinTile - 1) / kMinTile;
    return (size_t)kMaxPasses * 257 * 4 + 2 * ntiles * 256 * 8 + (size_t)kHistBlocks * kMaxPasses * 256 * 4 + 64;
}

int scan_u32_array(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp, hipStream_t s) {
    return scan_impl(LoadArray{in}, ArrayWrite{out}, n, tmp, s);
}

int scan_dirbits(const uint32_t *ent_nd, uint32_t *out, uint64_t n, uint32_t *tmp, hipStream_t s) {
    return scan_impl(LoadDirBit{ent_nd}, ArrayWrite{out}, n, tmp, s);
}

int scan_flag_pairs(const uint8_t *f, uint64_t n, uint64_t *out, uint64_t *tmp, hipStream_t s) {
    return scan_impl(LoadFlagPair{f}, ArrayWriteT<uint64_t>{out}, n, tmp, s, "scan_flags_sum",
                     "scan_flags_tile");
}

int lower_side_pairs(const uint32_t *ent_c, const uint32_t *ent_nd, const uint32_t *ent_r,
                     uint64_t n, uint32_t *key, uint2 *val, uint32_t *tmp, hipStream_t s) {
    return scan_impl(LoadLowerSide{ent_c, ent_nd}, LowerSideWrite{ent_c, ent_nd, ent_r, key, val},
                     n, tmp, s, "scan_lower_sum", "scan_lower_tile");
}

int radix_sort_pairs(uint32_t **keys, uint32_t **keys_alt, uint2 **vals, uint2 **vals_alt,
                     uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s) {
    if (n == 0 || bits <= 0) return TM_OK;
    const ArrayIn<uint32_t, uint2> in0{*keys, *vals};
    return radix_impl<uint32_t, uint2, PairOut<uint32_t, uint2>>(
        keys, keys_alt, vals, vals_alt, n, bits, tmp, err, s, "sort_pair_hist", "sort_pair_scatter",
        nullptr, in0);
}

int radix_sort_u64(uint64_t **keys, uint64_t **keys_alt, uint32_t **vals, uint32_t **vals_alt,
                   uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s,
                   const char *hist_name, const char *scatter_name) {
    if (n == 0 || bits <= 0) return TM_OK;
    const ArrayIn<uint64_t, uint32_t> in0{*keys, *vals};
    return radix_impl<uint64_t, uint32_t, PairOut<uint64_t, uint32_t>>(
        keys, keys_alt, vals, vals_alt, n, bits, tmp, err, s, hist_name, scatter_name, nullptr, in0);
}

int radix_sort_time_u32(uint32_t *keys, uint32_t *keys_alt, EdgeVal *vals, EdgeVal *vals_alt,
                        uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s, RankOut ro) {
    if (n == 0) return TM_OK;
    const RankWrite<uint32_t> fin{ro};
    const ArrayIn<uint32_t, EdgeVal> in0{keys, vals};
    return radix_impl<uint32_t, EdgeVal, RankWrite<uint32_t>>(
        &keys, &keys_alt, &vals, &vals_alt, n, bits < 1 ? 1 : bits, tmp, err, s, "sort_time_hist",
        "sort_time_scatter", &fin, in0);
}

int radix_sort_time_u64(uint64_t *keys, uint64_t *keys_alt, EdgeVal *vals, EdgeVal *vals_alt,
                        uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s, RankOut ro) {
    if (n == 0) return TM_OK;
    const RankWrite<uint64_t> fin{ro};
    const ArrayIn<uint64_t, EdgeVal> in0{keys, vals};
    return radix_impl<uint64_t, EdgeVal, RankWrite<uint64_t>>(
        &keys, &keys_alt, &vals, &vals_alt, n, bits < 1 ? 1 : bits, tmp, err, s, "sort_time_hist",
        "sort_time_scatter", &fin, in0);
}

template <typename K>
static int time_direct(const int32_t *src, const int32_t *dst, const int64_t *t, K *keys,
                       K *keys_alt, EdgeVal *vals, EdgeVal *vals_alt, uint64_t n, int bits,
                       void *tmp, uint32_t *err, hipStream_t s, RankOut ro) {
    if (n == 0) return TM_OK;
    const RankWrite<K> fin{ro};
    const TimeIn<K> in0{src, dst, t, ro.tmin};
    return radix_impl<K, EdgeVal, RankWrite<K>>(&keys, &keys_alt, &vals, &vals_alt, n,
                                                bits < 1 ? 1 : bits, tmp, err, s,
                                                "sort_time_hist", "sort_time_scatter", &fin, in0);
}

int radix_sort_time_direct_u32(const int32_t *src, const int32_t *dst, const int64_t *t,
                               uint32_t *keys, uint32_t *keys_alt, EdgeVal *vals, EdgeVal *vals_alt,
                               uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s,
                               RankOut ro) {
    return time_direct<uint32_t>(src, dst, t, keys, keys_alt, vals, vals_alt, n, bits, tmp, err, s, ro);
}

int radix_sort_time_direct_u64(const int32_t *src, const int32_t *dst, const int64_t *t,
                               uint64_t *keys, uint64_t *keys_alt, EdgeVal *vals, EdgeVal *vals_alt,
                               uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s,
                               RankOut ro) {
    return time_direct<uint64_t>(src, dst, t, keys, keys_alt, vals, vals_alt, n, bits, tmp, err, s, ro);
}

// ------------------------------------------------------- edge positions
// epos[slot] = the entry position of slot (2r at the source of edge rank r,
// 2r + 1 at its destination): the inverse of the node sort's permutation.
// Written directly it is one random 4-byte write per entry, which costs a
// partial-line write each once the index outgrows the last-level cache.
// Instead, (slot, position) pairs in entry order are partitioned by the
// slot's bits above kSlotBucketBits (radix passes, coalesced writes), and
// then each block fills one bucket of 2^kSlotBucketBits slots: slots are a
// permutation of [0, n), so bucket b is exactly sorted positions
// [b * 2^kSlotBucketBits, ...); the block places them in LDS by their low
// bits and writes the bucket out in order.
constexpr int kSlotBucketBits = 15;  // 128 KiB of LDS per bucket
constexpr uint32_t kSlotBucket = 1u << kSlotBucketBits;

// key: slots; val: their positions (null: position = index, the unsorted case).
// With erec, also each edge's record (t, both positions) for the edges of
// the bucket: a bucket starts at an even slot and n is even, so it holds
// both slots of each of its edges.
__global__ void __launch_bounds__(1024) k_epos_fill(const uint32_t *key, const uint32_t *val,
                                                    uint64_t n, uint32_t *epos,
                                                    const int64_t *t_r, EdgeRec *erec) {
    __shared__ uint32_t buf[kSlotBucket];
    for (uint64_t b = blockIdx.x; b * kSlotBucket < n; b += gridDim.x) {
        const uint64_t lo = b * kSlotBucket;
        const uint32_t cnt = (uint32_t)min<uint64_t>(kSlotBucket, n - lo);
        for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x)
            buf[key[lo + i] & (kSlotBucket - 1)] = val ? val[lo + i] : (uint32_t)(lo + i);
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) epos[lo + i] = buf[i];
        if (erec) {
            const uint64_t r0 = lo / 2;
            for (uint32_t i = threadIdx.x; i < cnt / 2; i += blockDim.x)
                erec[r0 + i] = EdgeRec{t_r[r0 + i], buf[2 * i], buf[2 * i + 1]};
        }
        __syncthreads();
    }
}

int edge_positions(const uint32_t *slot, uint64_t n, uint32_t *k0, uint32_t *v0, uint32_t *k1,
                   uint32_t *v1, void *tmp, uint32_t *err, hipStream_t s, uint32_t *epos,
                   const int64_t *t_r, EdgeRec *erec) {
    if (n == 0) return TM_OK;
    if (erec && n % 2) return TM_EINTERNAL;
    int bits = 0;
    while (bits < 32 && ((n - 1) >> bits) != 0) bits++;
    const uint32_t *key = slot, *val = nullptr;
    if (bits > kSlotBucketBits) {
        uint32_t *keys = k0, *keys_alt = k1, *vals = v0, *vals_alt = v1;
        const SlotIn in0{slot};
        const int rc = radix_impl<uint32_t, uint32_t, PairOut<uint32_t, uint32_t>>(
            &keys, &keys_alt, &vals, &vals_alt, n, bits, tmp, err, s, "sort_slot_hist",
            "sort_slot_scatter", nullptr, in0, kSlotBucketBits, /*iota_keys=*/true);
        if (rc) return rc;
        key = keys;
        val = vals;
    }
    const uint64_t nb = std::min<uint64_t>((n + kSlotBucket - 1) / kSlotBucket, 8192);
    TM_LAUNCH("epos_fill", k_epos_fill, dim3((unsigned)nb), dim3(1024), 0, s, key, val, n, epos,
              t_r, erec);
    return TM_OK;
}

template <typename V>
static int node_sort(uint32_t *keys, uint32_t *keys_alt, V *vals, V *vals_alt, uint64_t n,
                     int bits, void *tmp, uint32_t *err, hipStream_t s, SeqOut so) {
    if (n == 0) return TM_OK;
    const SeqWrite<V> fin{so};
    const ArrayIn<uint32_t, V> in0{keys, vals};
    return radix_impl<uint32_t, V, SeqWrite<V>>(&keys, &keys_alt, &vals, &vals_alt, n,
                                                bits < 1 ? 1 : bits, tmp, err, s, "sort_node_hist",
                                                "sort_node_scatter", &fin, in0);
}

int radix_sort_nodes(uint32_t *keys, uint32_t *keys_alt, NodeVal *vals, NodeVal *vals_alt,
                     uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s, SeqOut so) {
    return node_sort(keys, keys_alt, vals, vals_alt, n, bits, tmp, err, s, so);
}

int radix_sort_nodes(uint32_t *keys, uint32_t *keys_alt, NodeVal32 *vals, NodeVal32 *vals_alt,
                     uint64_t n, int bits, void *tmp, uint32_t *err, hipStream_t s, SeqOut so) {
    return node_sort(keys, keys_alt, vals, vals_alt, n, bits, tmp, err, s, so);
}

}  // namespace tmc
