// Device primitives: exclusive scan and a stable LSD radix sort, written for
// 64-wide CDNA wavefronts (ballot-based digit matching, no block barriers in
// the ranking loop).
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

// Inclusive scan over the kBlock threads; *total receives the block sum.
template <typename T>
__device__ inline T block_incl_scan(T v, T *total, T *lds4) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    T s = wave_incl_scan(v, lane);
    if (lane == kWave - 1) lds4[w] = s;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; i++) {
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

struct LoadArray {
    const uint32_t *p;
    __device__ uint32_t operator()(uint64_t i) const { return p[i]; }
};
struct LoadDirBit {
    const uint32_t *nd;
    __device__ uint32_t operator()(uint64_t i) const { return nd[i] & 1u; }
};

template <typename L>
__global__ void __launch_bounds__(kBlock) k_tile_sum(L ld, uint64_t n, uint32_t *part) {
    __shared__ uint32_t lds[kBlock / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
        if (idx < n) acc += ld(idx);
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// One block: exclusive scan of np partial sums in place; part[np] = total.
__global__ void __launch_bounds__(kBlock) k_scan_parts(uint32_t *part, uint32_t np) {
    __shared__ uint32_t lds[kBlock / kWave];
    uint32_t carry = 0;
    for (uint32_t b = 0; b < np; b += kBlock) {
        uint32_t i = b + threadIdx.x;
        uint32_t v = i < np ? part[i] : 0;
        uint32_t tot;
        uint32_t inc = block_incl_scan(v, &tot, lds);
        if (i < np) part[i] = carry + inc - v;
        carry += tot;
    }
    if (threadIdx.x == 0) part[np] = carry;
}

template <typename L>
__global__ void __launch_bounds__(kBlock) k_tile_scan(L ld, uint64_t n, const uint32_t *part,
                                                      uint32_t np, uint32_t *out) {
    __shared__ uint32_t lds[kBlock / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    uint32_t carry = part[blockIdx.x];
    for (int i = 0; i < kItems; i++) {
        uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
        uint32_t v = idx < n ? ld(idx) : 0;
        uint32_t tot;
        uint32_t inc = block_incl_scan(v, &tot, lds);
        if (idx < n) out[idx] = carry + inc - v;
        carry += tot;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = part[np];
}

__global__ void k_set_zero(uint32_t *p) { *p = 0; }

template <typename L>
int scan_impl(L ld, uint32_t *out, uint64_t n, uint32_t *tmp, hipStream_t s) {
    const uint64_t nb = (n + kTile - 1) / kTile;
    if (nb == 0) {
        // a kernel, not a memset: this may run inside a captured graph
        TM_LAUNCH("scan_empty", k_set_zero, dim3(1), dim3(1), 0, s, out);
        return TM_OK;
    }
    TM_LAUNCH("scan_tile_sum", (k_tile_sum<L>), dim3(nb), dim3(kBlock), 0, s, ld, n, tmp);
    TM_LAUNCH("scan_parts", k_scan_parts, dim3(1), dim3(kBlock), 0, s, tmp, (uint32_t)nb);
    TM_LAUNCH("scan_tile", (k_tile_scan<L>), dim3(nb), dim3(kBlock), 0, s, ld, n, tmp,
              (uint32_t)nb, out);
    return TM_OK;
}

// ------------------------------------------------------------ radix sort
// Tile of kRadixTile elements per block; wave w owns the contiguous quarter
// [w*1024, (w+1)*1024) of the tile and walks it in 16 rounds of 64, so the
// order inside the tile is (wave, round, lane) = input order and a per-wave
// running digit count gives stable ranks without block barriers.
constexpr int kRadixItems = 8;
constexpr int kRadixTile = kBlock * kRadixItems;
constexpr int kWaves = kBlock / kWave;
static_assert(kBlock == 256, "radix kernels map one thread to each 8-bit digit");

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

// Per-block digit histogram.  Each wave keeps its own sub-histogram; the
// lowest lane of every group of equal digits adds the group size, so no two
// lanes of a wave touch one counter (skewed keys, e.g. a hub's node id, do
// not serialise on LDS atomics).
template <typename K>
__global__ void __launch_bounds__(kBlock) k_radix_hist(const K *keys, uint64_t n, int shift,
                                                       uint32_t *hist, uint32_t nb) {
    __shared__ uint32_t h[kWaves][256];
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int i = threadIdx.x; i < kWaves * 256; i += kBlock) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRadixTile + (uint64_t)w * (kRadixItems * kWave);
    const uint64_t lt = lanemask_lt(lane);
#pragma unroll 4
    for (int i = 0; i < kRadixItems; i++) {
        const uint64_t idx = base + (uint64_t)i * kWave + lane;
        const bool valid = idx < n;
        const K key = valid ? keys[idx] : K(0);
        uint32_t d;
        const uint64_t peers = digit_peers(key, shift, valid, &d);
        if (valid && __popcll(peers & lt) == 0) h[w][d] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kWaves; q++) s += h[q][threadIdx.x];
    hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = s;
}

// Stable scatter of one digit pass.  Ranks come from per-wave running digit
// counts (tile order = (wave, round, lane) = input order); the tile is then
// staged in LDS in digit order so that the global writes of each digit's run
// are contiguous.
template <typename K, typename V>
struct PairOut {
    K *kout;
    V *vout;
    __device__ inline void operator()(uint32_t pos, K k, const V &v) const {
        kout[pos] = k;
        vout[pos] = v;
    }
};

struct SeqWrite {
    SeqOut o;
    __device__ inline void operator()(uint32_t pos, uint32_t k, const NodeVal &v) const {
        o.ent_c[pos] = k;
        o.ent_t[pos] = v.t;
        o.ent_nd[pos] = v.nd;
        o.ent_r[pos] = v.r;
        o.epos[2 * (uint64_t)v.r + (v.nd & 1u)] = pos;
    }
};

template <typename K, typename V, typename Out>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const K *kin, const V *vin, Out out,
                                                          uint64_t n, int shift,
                                                          const uint32_t *offs, uint32_t nb) {
    __shared__ uint32_t wh[kWaves][256];
    __shared__ uint32_t blk_off[256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t scan_lds[kBlock / kWave];
    __shared__ K s_key[kRadixTile];
    __shared__ V s_val[kRadixTile];
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int i = threadIdx.x; i < kWaves * 256; i += kBlock) (&wh[0][0])[i] = 0;
    __syncthreads();
    const uint64_t tile0 = (uint64_t)blockIdx.x * kRadixTile;
    const uint64_t base = tile0 + (uint64_t)w * (kRadixItems * kWave);
    const uint64_t lt = lanemask_lt(lane);
    K key[kRadixItems];
    uint32_t rank[kRadixItems];
    uint32_t dig[kRadixItems];
#pragma unroll
    for (int i = 0; i < kRadixItems; i++) {
        const uint64_t idx = base + (uint64_t)i * kWave + lane;
        const bool valid = idx < n;
        key[i] = valid ? kin[idx] : K(0);
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
    // digit totals of the tile -> exclusive prefix over digits (one thread per digit)
    {
        const int d = threadIdx.x;
        uint32_t c[kWaves];
        uint32_t tot = 0;
#pragma unroll
        for (int q = 0; q < kWaves; q++) {
            c[q] = wh[q][d];
            tot += c[q];
        }
        uint32_t total;
        const uint32_t excl = block_incl_scan(tot, &total, scan_lds) - tot;
        blk_off[d] = excl;
        gbase[d] = offs[(uint64_t)d * nb + blockIdx.x];
        uint32_t run = excl;
#pragma unroll
        for (int q = 0; q < kWaves; q++) {
            wh[q][d] = run;
            run += c[q];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRadixItems; i++) {
        const uint64_t idx = base + (uint64_t)i * kWave + lane;
        if (idx < n) {
            // values are not held in registers: read straight into their slot
            const uint32_t x = wh[w][dig[i]] + rank[i];
            s_key[x] = key[i];
            s_val[x] = vin[idx];
        }
    }
    __syncthreads();
    const uint32_t cnt_tile = (uint32_t)min<uint64_t>((uint64_t)kRadixTile, n - tile0);
    for (uint32_t x = threadIdx.x; x < cnt_tile; x += kBlock) {
        const K k = s_key[x];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint32_t pos = gbase[d] + (x - blk_off[d]);
        out(pos, k, s_val[x]);
    }
}

template <typename K, typename V>
int radix_impl(K **keys, K **keys_alt, V **vals, V **vals_alt, uint64_t n, int bits,
               uint32_t *tmp, hipStream_t s, const char *hist_name, const char *scatter_name) {
    if (n <= 1 || bits <= 0) return TM_OK;
    const uint64_t nb = (n + kRadixTile - 1) / kRadixTile;
    const uint64_t nh = nb * 256;
    uint32_t *hist = tmp;                      // nh + 1
    uint32_t *stmp = tmp + nh + 1;             // scan partials
    for (int shift = 0; shift < bits; shift += 8) {
        TM_LAUNCH(hist_name, k_radix_hist<K>, dim3(nb), dim3(kBlock), 0, s, *keys, n, shift,
                  hist, (uint32_t)nb);
        int rc = scan_impl(LoadArray{hist}, hist, nh, stmp, s);
        if (rc) return rc;
        TM_LAUNCH(scatter_name, (k_radix_scatter<K, V, PairOut<K, V>>), dim3(nb), dim3(kBlock), 0, s,
                  *keys, *vals, (PairOut<K, V>{*keys_alt, *vals_alt}), n, shift, hist, (uint32_t)nb);
        K *tk = *keys;
        *keys = *keys_alt;
        *keys_alt = tk;
        V *tv = *vals;
        *vals = *vals_alt;
        *vals_alt = tv;
    }
    return TM_OK;
}

__global__ void k_iota(uint32_t *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
}

}  // namespace

size_t scan_tmp_count(uint64_t n) { return (n + kTile - 1) / kTile + 2; }

size_t radix_tmp_count(uint64_t n) {
    const uint64_t nb = (n + kRadixTile - 1) / kRadixTile;
    const uint64_t nh = nb * 256;
    return nh + 1 + scan_tmp_count(nh) + 4;
}

int scan_u32_array(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp, hipStream_t s) {
    return scan_impl(LoadArray{in}, out, n, tmp, s);
}

int scan_dirbits(const uint32_t *ent_nd, uint32_t *out, uint64_t n, uint32_t *tmp, hipStream_t s) {
    return scan_impl(LoadDirBit{ent_nd}, out, n, tmp, s);
}

#define TM_RADIX_INST(NAME, K, V)                                                             \
    int NAME(K **keys, K **keys_alt, V **vals, V **vals_alt, uint64_t n, int bits, uint32_t *tmp, \
             hipStream_t s, const char *hist_name, const char *scatter_name) {                    \
        return radix_impl<K, V>(keys, keys_alt, vals, vals_alt, n, bits, tmp, s, hist_name,      \
                                scatter_name);                                                   \
    }
TM_RADIX_INST(radix_sort_u32, uint32_t, uint32_t)
TM_RADIX_INST(radix_sort_u64, uint64_t, uint32_t)
TM_RADIX_INST(radix_sort_u32_v64, uint32_t, uint64_t)
TM_RADIX_INST(radix_sort_u32_edge, uint32_t, EdgeVal)
TM_RADIX_INST(radix_sort_u64_edge, uint64_t, EdgeVal)
#undef TM_RADIX_INST

int radix_sort_nodes(uint32_t *keys, uint32_t *keys_alt, NodeVal *vals, NodeVal *vals_alt,
                     uint64_t n, int bits, uint32_t *tmp, hipStream_t s, SeqOut so) {
    if (n == 0) return TM_OK;
    if (bits < 1) bits = 1;
    const uint64_t nb = (n + kRadixTile - 1) / kRadixTile;
    const uint64_t nh = nb * 256;
    uint32_t *hist = tmp;
    uint32_t *stmp = tmp + nh + 1;
    for (int shift = 0; shift < bits; shift += 8) {
        TM_LAUNCH("sort_node_hist", k_radix_hist<uint32_t>, dim3(nb), dim3(kBlock), 0, s, keys, n,
                  shift, hist, (uint32_t)nb);
        int rc = scan_impl(LoadArray{hist}, hist, nh, stmp, s);
        if (rc) return rc;
        if (shift + 8 >= bits) {
            TM_LAUNCH("sort_node_scatter", (k_radix_scatter<uint32_t, NodeVal, SeqWrite>), dim3(nb),
                      dim3(kBlock), 0, s, keys, vals, SeqWrite{so}, n, shift, hist, (uint32_t)nb);
        } else {
            TM_LAUNCH("sort_node_scatter", (k_radix_scatter<uint32_t, NodeVal, PairOut<uint32_t, NodeVal>>),
                      dim3(nb), dim3(kBlock), 0, s, keys, vals,
                      (PairOut<uint32_t, NodeVal>{keys_alt, vals_alt}), n, shift, hist, (uint32_t)nb);
            uint32_t *tk = keys;
            keys = keys_alt;
            keys_alt = tk;
            NodeVal *tv = vals;
            vals = vals_alt;
            vals_alt = tv;
        }
    }
    return TM_OK;
}

int fill_iota(uint32_t *p, uint64_t n, hipStream_t s) {
    if (n == 0) return TM_OK;
    uint64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 65536) nb = 65536;
    TM_LAUNCH("iota", k_iota, dim3(nb), dim3(kBlock), 0, s, p, n);
    return TM_OK;
}

}  // namespace tmc
