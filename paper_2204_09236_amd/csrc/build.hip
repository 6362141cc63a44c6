// Graph build: the per-node time-ordered sequences S_u (the paper's Section
// IV-A input to FAST-Star; Algorithm 1 "get S_u") and the node-pair edge sets
// E_(v,w) of Algorithm 2, both produced by stable device radix sorts.
//
//   1. validate the edge list, find min/max t and max node id
//   2. sort edges by t (stable, so ties stay in id order): rank r -> edge id
//   3. emit two incident entries per edge in rank order and sort them by node
//      (stable): S_u in (u, t, id) order, offsets from the sorted node keys
//   4. sort edges (in rank order) by (min node, max node) (stable): every
//      unordered node pair's edges become one run in (t, id) order; runs with
//      at least two edges are indexed (only they can hold pair or star
//      instances: both need two edges on one node pair)
#include <algorithm>
#include <vector>

#include "tm_internal.h"

namespace tmc {

namespace {

constexpr int64_t kTLimit = (int64_t)1 << 62;

struct Stat {
    uint32_t bad;        // bit 0: id out of range / negative, bit 1: self-loop, bit 2: |t| too big
    uint32_t max_id;
    uint64_t tmin_key;   // t ^ sign bit, so unsigned order = signed order
    uint64_t tmax_key;
};

__global__ void __launch_bounds__(kBlock) k_validate(const int32_t *src, const int32_t *dst,
                                                     const int64_t *t, uint64_t m,
                                                     uint32_t n_limit, Stat *st) {
    uint32_t bad = 0, mx = 0;
    uint64_t tmin = ~0ull, tmax = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const int32_t a = src[e], b = dst[e];
        const int64_t te = t[e];
        if (a < 0 || b < 0 || (uint32_t)a >= n_limit || (uint32_t)b >= n_limit) bad |= 1u;
        if (a == b) bad |= 2u;
        if (te >= kTLimit || te <= -kTLimit) bad |= 4u;
        mx = max(mx, (uint32_t)max(a, b));
        const uint64_t k = (uint64_t)te ^ 0x8000000000000000ull;
        tmin = min(tmin, k);
        tmax = max(tmax, k);
    }
    // wave reduction, then one atomic per wave (flags and extrema, not counts)
    for (int o = kWave / 2; o > 0; o >>= 1) {
        bad |= __shfl_xor(bad, o, kWave);
        mx = max(mx, (uint32_t)__shfl_xor(mx, o, kWave));
        tmin = min(tmin, (uint64_t)__shfl_xor(tmin, o, kWave));
        tmax = max(tmax, (uint64_t)__shfl_xor(tmax, o, kWave));
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (bad) atomicOr(&st->bad, bad);
        atomicMax(&st->max_id, mx);
        atomicMin((unsigned long long *)&st->tmin_key, (unsigned long long)tmin);
        atomicMax((unsigned long long *)&st->tmax_key, (unsigned long long)tmax);
    }
}

template <typename K>
__global__ void k_time_keys(const int64_t *t, uint64_t m, int64_t tmin, K *keys, uint32_t *vals) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        keys[e] = (K)(uint64_t)(t[e] - tmin);
        vals[e] = (uint32_t)e;
    }
}

// Incident entries in rank order: slot 2r = src side (dir o), 2r+1 = dst side (dir in).
__global__ void k_entries(const int32_t *src, const int32_t *dst, const uint32_t *perm, uint64_t m,
                          uint32_t *nkey, uint32_t *nval) {
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t e = perm[r];
        nkey[2 * r] = (uint32_t)src[e];
        nkey[2 * r + 1] = (uint32_t)dst[e];
        nval[2 * r] = (uint32_t)(2 * r);
        nval[2 * r + 1] = (uint32_t)(2 * r + 1);
    }
}

// off[u] = first position of node u in the node-sorted keys, atomic-free:
// each boundary between consecutive keys fills the offsets of the (absent)
// nodes it skips over, up to kGapFill of them; longer runs of absent nodes are
// left marked and resolved by k_offsets_gaps with a binary search.
constexpr uint32_t kGapFill = 64;
constexpr uint32_t kUnset = 0xffffffffu;

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_offsets(const uint32_t *skey, uint64_t len, uint32_t n, uint32_t *off) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= len;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t prev = p == 0 ? -1 : (int64_t)skey[p - 1];
        const int64_t cur = p == len ? (int64_t)n : (int64_t)skey[p];
        if (cur == prev) continue;
        off[cur] = (uint32_t)p;
        const int64_t stop = min(cur - 1, prev + (int64_t)kGapFill);
        for (int64_t u = prev + 1; u <= stop; u++) off[u] = (uint32_t)p;
    }
}

__global__ void k_offsets_gaps(const uint32_t *skey, uint64_t len, uint32_t n, uint32_t *off) {
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n;
         u += (uint64_t)gridDim.x * blockDim.x) {
        if (off[u] != kUnset) continue;
        uint64_t a = 0, b = len;  // lower bound of u
        while (a < b) {
            const uint64_t mid = a + (b - a) / 2;
            if (skey[mid] < u) a = mid + 1;
            else b = mid;
        }
        off[u] = (uint32_t)a;
    }
}

__global__ void k_fill_seq(const int32_t *src, const int32_t *dst, const int64_t *t,
                           const uint32_t *perm, const uint32_t *sval, uint64_t len,
                           int64_t *ent_t, uint32_t *ent_nd, uint32_t *ent_r, uint32_t *epos) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < len;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t slot = sval[p];
        const uint32_t r = slot >> 1, side = slot & 1u;
        const uint32_t e = perm[r];
        const uint32_t nbr = side ? (uint32_t)src[e] : (uint32_t)dst[e];
        ent_t[p] = t[e];
        ent_nd[p] = (nbr << 1) | side;
        ent_r[p] = r;
        epos[slot] = (uint32_t)p;
    }
}

__global__ void k_pair_keys(const int32_t *src, const int32_t *dst, const uint32_t *perm,
                            uint64_t m, uint64_t n, uint64_t *pkey, uint32_t *pval) {
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t e = perm[r];
        const uint32_t a = (uint32_t)src[e], b = (uint32_t)dst[e];
        const uint32_t lo = min(a, b), hi = max(a, b);
        pkey[r] = (uint64_t)lo * n + hi;
        pval[r] = (uint32_t)r | (a == lo ? kOrientBit : 0u);
    }
}

// Head of a run with at least two edges.
__global__ void k_multi_heads(const uint64_t *pkey, uint64_t m, uint32_t *flag) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < m;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const bool head = g == 0 || pkey[g] != pkey[g - 1];
        const bool multi = g + 1 < m && pkey[g + 1] == pkey[g];
        flag[g] = (head && multi) ? 1u : 0u;
    }
}

__global__ void k_multi_fill(const uint64_t *pkey, uint64_t m, uint64_t n, const uint32_t *flag,
                             const uint32_t *idx, uint32_t *mp_start, uint32_t *mp_end,
                             uint32_t *mp_lo, uint32_t *mp_hi) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < m;
         g += (uint64_t)gridDim.x * blockDim.x) {
        if (!flag[g]) continue;
        const uint32_t k = idx[g];
        const uint64_t key = pkey[g];
        // end of the run: upper bound of key in the sorted keys
        uint64_t lo = g + 1, hi = m;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (pkey[mid] <= key) lo = mid + 1;
            else hi = mid;
        }
        mp_start[k] = (uint32_t)g;
        mp_end[k] = (uint32_t)lo;
        mp_lo[k] = (uint32_t)(key / n);
        mp_hi[k] = (uint32_t)(key % n);
    }
}

__global__ void k_max_degree(const uint32_t *off, uint32_t n, uint32_t *out) {
    uint32_t mx = 0;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (uint64_t)gridDim.x * blockDim.x)
        mx = max(mx, off[u + 1] - off[u]);
    for (int o = kWave / 2; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o, kWave));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, mx);
}

int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) b++;
    return b;
}

dim3 grid_for(uint64_t n) {
    uint64_t nb = (n + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    if (nb > 16384) nb = 16384;
    return dim3((unsigned)nb);
}

template <typename T>
int dmalloc(T **p, size_t count) {
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? TM_ENOMEM : TM_EHIP;
    }
    return TM_OK;
}

}  // namespace

#define TRY(x)                 \
    do {                       \
        int _rc = (x);         \
        if (_rc) return _rc;   \
    } while (0)

int build_graph_device(tm_graph *g, const int32_t *src, const int32_t *dst, const int64_t *t,
                       uint64_t m, uint32_t n_nodes, hipStream_t s) {
    g->m = m;
    // ---- 1. validation
    Stat h_st{0, 0, ~0ull, 0};
    Stat *d_st = nullptr;
    TRY(dmalloc(&d_st, 1));
    struct FreeSt {
        Stat *p;
        ~FreeSt() { (void)hipFree(p); }
    } free_st{d_st};
    TM_HIP_TRY(hipMemcpyAsync(d_st, &h_st, sizeof(Stat), hipMemcpyHostToDevice, s));
    if (m > 0) {
        TM_LAUNCH("validate", k_validate, grid_for(m), dim3(kBlock), 0, s, src, dst, t, m,
                  n_nodes ? n_nodes : 0x7fffffffu, d_st);
    }
    TM_HIP_TRY(hipMemcpyAsync(&h_st, d_st, sizeof(Stat), hipMemcpyDeviceToHost, s));
    TM_HIP_TRY(hipStreamSynchronize(s));
    if (h_st.bad) {
        set_error(std::string("invalid edge list:") + ((h_st.bad & 1) ? " node id out of range" : "") +
                  ((h_st.bad & 2) ? " self-loop" : "") + ((h_st.bad & 4) ? " |t| >= 2^62" : ""));
        return TM_EINVAL;
    }
    uint64_t n = n_nodes ? n_nodes : (m ? (uint64_t)h_st.max_id + 1 : 0);
    if (n > 0x7fffffffull) {
        set_error("node count must be below 2^31");
        return TM_EINVAL;
    }
    g->n = (uint32_t)n;
    const uint64_t len = 2 * m;
    TRY(dmalloc(&g->off, n + 1));
    TRY(dmalloc(&g->ent_t, len));
    TRY(dmalloc(&g->ent_nd, len));
    TRY(dmalloc(&g->ent_r, len));
    TRY(dmalloc(&g->X, len + 1));
    TRY(dmalloc(&g->epos, len));
    TRY(dmalloc(&g->perm, m));
    TRY(dmalloc(&g->pair_el, m));
    if (m == 0) {
        TM_HIP_TRY(hipMemsetAsync(g->off, 0, (n + 1) * sizeof(uint32_t), s));
        TM_HIP_TRY(hipMemsetAsync(g->X, 0, sizeof(uint32_t), s));
        TM_HIP_TRY(hipStreamSynchronize(s));
        return TM_OK;
    }
    const int64_t tmin = (int64_t)(h_st.tmin_key ^ 0x8000000000000000ull);
    const int64_t tmax = (int64_t)(h_st.tmax_key ^ 0x8000000000000000ull);
    const int tbits = bits_for((uint64_t)(tmax - tmin));

    // scratch: two key buffers (u64 of 2m) and two value buffers (u32 of 2m)
    uint64_t *k64a = nullptr, *k64b = nullptr;
    uint32_t *va = nullptr, *vb = nullptr, *tmp = nullptr;
    struct FreeAll {
        std::vector<void *> ps;
        ~FreeAll() {
            for (void *p : ps) (void)hipFree(p);
        }
    } fa;
    TRY(dmalloc(&k64a, len));
    fa.ps.push_back(k64a);
    TRY(dmalloc(&k64b, len));
    fa.ps.push_back(k64b);
    TRY(dmalloc(&va, len));
    fa.ps.push_back(va);
    TRY(dmalloc(&vb, len));
    fa.ps.push_back(vb);
    const size_t ntmp = std::max(radix_tmp_count(len), scan_tmp_count(len)) + 16;
    TRY(dmalloc(&tmp, ntmp));
    fa.ps.push_back(tmp);

    // ---- 2. sort edges by t (stable): perm[r] = edge id of rank r
    uint32_t *vals = va, *vals_alt = vb;
    if (tbits <= 32) {
        uint32_t *keys = reinterpret_cast<uint32_t *>(k64a);
        uint32_t *keys_alt = reinterpret_cast<uint32_t *>(k64b);
        TM_LAUNCH("time_keys", k_time_keys<uint32_t>, grid_for(m), dim3(kBlock), 0, s, t, m, tmin,
                  keys, vals);
        TRY(radix_sort_u32(&keys, &keys_alt, &vals, &vals_alt, m, tbits, tmp, s, "sort_time_hist",
                           "sort_time_scatter"));
    } else {
        uint64_t *keys = k64a, *keys_alt = k64b;
        TM_LAUNCH("time_keys", k_time_keys<uint64_t>, grid_for(m), dim3(kBlock), 0, s, t, m, tmin,
                  keys, vals);
        TRY(radix_sort_u64(&keys, &keys_alt, &vals, &vals_alt, m, tbits, tmp, s, "sort_time_hist",
                           "sort_time_scatter"));
    }
    TM_HIP_TRY(hipMemcpyAsync(g->perm, vals, m * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));

    // ---- 3. incident entries sorted by node (stable over rank order)
    {
        uint32_t *keys = reinterpret_cast<uint32_t *>(k64a);
        uint32_t *keys_alt = reinterpret_cast<uint32_t *>(k64b);
        uint32_t *v = va, *v_alt = vb;
        TM_LAUNCH("entries", k_entries, grid_for(m), dim3(kBlock), 0, s, src, dst, g->perm, m, keys,
                  v);
        TRY(radix_sort_u32(&keys, &keys_alt, &v, &v_alt, len, bits_for(n - 1), tmp, s,
                           "sort_node_hist", "sort_node_scatter"));
        TM_LAUNCH("offsets_fill", k_fill_u32, grid_for(n + 1), dim3(kBlock), 0, s, g->off, n + 1,
                  kUnset);
        TM_LAUNCH("offsets", k_offsets, grid_for(len + 1), dim3(kBlock), 0, s, keys, len,
                  (uint32_t)n, g->off);
        TM_LAUNCH("offsets_gaps", k_offsets_gaps, grid_for(n + 1), dim3(kBlock), 0, s, keys, len,
                  (uint32_t)n, g->off);
        TM_LAUNCH("fill_seq", k_fill_seq, grid_for(len), dim3(kBlock), 0, s, src, dst, t, g->perm, v,
                  len, g->ent_t, g->ent_nd, g->ent_r, g->epos);
        TRY(scan_dirbits(g->ent_nd, g->X, len, tmp, s));
    }

    // ---- 4. node-pair edge sets
    {
        uint64_t *keys = k64a, *keys_alt = k64b;
        uint32_t *v = va, *v_alt = vb;
        TM_LAUNCH("pair_keys", k_pair_keys, grid_for(m), dim3(kBlock), 0, s, src, dst, g->perm, m,
                  n, keys, v);
        TRY(radix_sort_u64(&keys, &keys_alt, &v, &v_alt, m, bits_for(n * n - 1), tmp, s,
                           "sort_pair_hist", "sort_pair_scatter"));
        TM_HIP_TRY(hipMemcpyAsync(g->pair_el, v, m * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        uint32_t *flag = v_alt;            // free value buffer
        uint32_t *idx = reinterpret_cast<uint32_t *>(keys_alt);  // free key buffer (>= m + 1 u32)
        TM_LAUNCH("multi_heads", k_multi_heads, grid_for(m), dim3(kBlock), 0, s, keys, m, flag);
        TRY(scan_u32_array(flag, idx, m, tmp, s));
        uint32_t n_multi = 0;
        TM_HIP_TRY(hipMemcpyAsync(&n_multi, idx + m, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TM_HIP_TRY(hipStreamSynchronize(s));
        g->n_multi = n_multi;
        TRY(dmalloc(&g->mp_start, n_multi));
        TRY(dmalloc(&g->mp_end, n_multi));
        TRY(dmalloc(&g->mp_lo, n_multi));
        TRY(dmalloc(&g->mp_hi, n_multi));
        if (n_multi) {
            TM_LAUNCH("multi_fill", k_multi_fill, grid_for(m), dim3(kBlock), 0, s, keys, m, n, flag,
                      idx, g->mp_start, g->mp_end, g->mp_lo, g->mp_hi);
        }
    }
    // ---- facts
    {
        uint32_t *d_mx = tmp;
        TM_HIP_TRY(hipMemsetAsync(d_mx, 0, sizeof(uint32_t), s));
        TM_LAUNCH("max_degree", k_max_degree, grid_for(n), dim3(kBlock), 0, s, g->off, (uint32_t)n,
                  d_mx);
        uint32_t mx = 0;
        TM_HIP_TRY(hipMemcpyAsync(&mx, d_mx, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TM_HIP_TRY(hipStreamSynchronize(s));
        g->max_degree = mx;
    }
    return TM_OK;
}

}  // namespace tmc
