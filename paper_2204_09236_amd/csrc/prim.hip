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

template <typename L>
int scan_impl(L ld, uint32_t *out, uint64_t n, uint32_t *tmp, hipStream_t s) {
    const uint64_t nb = (n + kTile - 1) / kTile;
    if (nb == 0) {
        TM_HIP_TRY(hipMemsetAsync(out, 0, sizeof(uint32_t), s));
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
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kBlock * kRadixItems;
constexpr int kWaves = kBlock / kWave;

template <typename K>
__global__ void __launch_bounds__(kBlock) k_radix_hist(const K *keys, uint64_t n, int shift,
                                                       uint32_t *hist, uint32_t nb) {
    __shared__ uint32_t h[kWaves][256];
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int i = threadIdx.x; i < kWaves * 256; i += kBlock) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRadixTile + (uint64_t)w * (kRadixItems * kWave);
#pragma unroll 4
    for (int i = 0; i < kRadixItems; i++) {
        uint64_t idx = base + (uint64_t)i * kWave + lane;
        if (idx < n) {
            uint32_t d = (uint32_t)(keys[idx] >> shift) & 255u;
            atomicAdd(&h[w][d], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < 256) {
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < kWaves; q++) s += h[q][threadIdx.x];
        hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = s;
    }
}

template <typename K>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const K *kin, const uint32_t *vin,
                                                          K *kout, uint32_t *vout, uint64_t n,
                                                          int shift, const uint32_t *offs,
                                                          uint32_t nb) {
    __shared__ uint32_t wh[kWaves][256];
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    for (int i = threadIdx.x; i < kWaves * 256; i += kBlock) (&wh[0][0])[i] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRadixTile + (uint64_t)w * (kRadixItems * kWave);
    const uint64_t lt = lanemask_lt(lane);
    K key[kRadixItems];
    uint32_t val[kRadixItems];
    uint32_t rank[kRadixItems];
    uint32_t dig[kRadixItems];
#pragma unroll
    for (int i = 0; i < kRadixItems; i++) {
        const uint64_t idx = base + (uint64_t)i * kWave + lane;
        const bool valid = idx < n;
        key[i] = valid ? kin[idx] : K(0);
        val[i] = valid ? vin[idx] : 0u;
        const uint32_t d = (uint32_t)(key[i] >> shift) & 255u;
        dig[i] = d;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
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
    // exclusive prefix over waves, offset by this block's global digit base
    if (threadIdx.x < 256) {
        uint32_t run = offs[(uint64_t)threadIdx.x * nb + blockIdx.x];
#pragma unroll
        for (int q = 0; q < kWaves; q++) {
            uint32_t c = wh[q][threadIdx.x];
            wh[q][threadIdx.x] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRadixItems; i++) {
        const uint64_t idx = base + (uint64_t)i * kWave + lane;
        if (idx < n) {
            const uint32_t pos = wh[w][dig[i]] + rank[i];
            kout[pos] = key[i];
            vout[pos] = val[i];
        }
    }
}

template <typename K>
int radix_impl(K **keys, K **keys_alt, uint32_t **vals, uint32_t **vals_alt, uint64_t n, int bits,
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
        TM_LAUNCH(scatter_name, k_radix_scatter<K>, dim3(nb), dim3(kBlock), 0, s, *keys, *vals,
                  *keys_alt, *vals_alt, n, shift, hist, (uint32_t)nb);
        K *tk = *keys;
        *keys = *keys_alt;
        *keys_alt = tk;
        uint32_t *tv = *vals;
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

int radix_sort_u32(uint32_t **keys, uint32_t **keys_alt, uint32_t **vals, uint32_t **vals_alt,
                   uint64_t n, int bits, uint32_t *tmp, hipStream_t s, const char *hist_name,
                   const char *scatter_name) {
    return radix_impl<uint32_t>(keys, keys_alt, vals, vals_alt, n, bits, tmp, s, hist_name,
                                scatter_name);
}

int radix_sort_u64(uint64_t **keys, uint64_t **keys_alt, uint32_t **vals, uint32_t **vals_alt,
                   uint64_t n, int bits, uint32_t *tmp, hipStream_t s, const char *hist_name,
                   const char *scatter_name) {
    return radix_impl<uint64_t>(keys, keys_alt, vals, vals_alt, n, bits, tmp, s, hist_name,
                                scatter_name);
}

int fill_iota(uint32_t *p, uint64_t n, hipStream_t s) {
    if (n == 0) return TM_OK;
    uint64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 65536) nb = 65536;
    TM_LAUNCH("iota", k_iota, dim3(nb), dim3(kBlock), 0, s, p, n);
    return TM_OK;
}

}  // namespace tmc
