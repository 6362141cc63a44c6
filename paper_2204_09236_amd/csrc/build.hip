// Graph build: the per-node time-ordered sequences S_u (Section IV-A: every
// node's incident edges (t, v, dir) in time order, the input of FAST-Star and
// FAST-Tri) and the node-pair edge sets E_(v,w) of Algorithm 2, produced by
// stable device radix sorts.  Everything here is delta-independent.
//
//   1. validate the edge list; min/max t and max node id
//   2. sort edges by t, carrying (src, dst, id): stable, so equal timestamps
//      stay in id order -> edge rank r in the (t, id) order
//   3. two incident entries per edge, in rank order, sorted by node (stable),
//      carrying (r, other endpoint, dir): S_u in (u, t, id) order
//   4. edges (in rank order) sorted by (smaller node, larger node) (stable):
//      each unordered node pair's edges in (t, id) order.  Only pairs with at
//      least two edges can hold pair or star instances (both need two edges
//      on one node pair); their edges are gathered into compact per-pair
//      arrays with, for each of the two nodes, the edge's position in S_u and
//      the number of dir-o / dir-in entries before it.
#include <algorithm>
#include <atomic>
#include <vector>

#include "tm_internal.h"

namespace tmc {

namespace {

constexpr int64_t kTLimit = (int64_t)1 << 62;
constexpr uint32_t kGapFill = 64;
constexpr uint32_t kUnset = 0xffffffffu;
constexpr uint32_t kMaxStatBlocks = 4096;
constexpr uint64_t kEntryTile = 8192, kElemTile = 1024;
// The edge-position index is scattered straight from the node sort while it
// fits MI355X's 256 MiB last-level cache (random 4-byte writes merge there);
// larger ones are built by edge_positions.
constexpr uint64_t kDirectEposBytes = (uint64_t)256 << 20;
std::atomic<bool> g_force_edge_sort{false};  // tests: build every index by edge_positions
// a single graph's entry tiles start at multiples of 64: the count's window
// kernel then writes whole 64-entry words of the window bit planes
static_assert(kEntryTile % 64 == 0, "entry tiles must be 64-aligned");

struct Stat {
    uint32_t bad;        // bit 0: id out of range / negative, bit 1: self-loop, bit 2: |t| too big
    uint32_t max_id;
    uint64_t tmin_key;   // t ^ sign bit, so unsigned order = signed order
    uint64_t tmax_key;
};

// Flags and extrema (not counts) per graph.  Edge tiles lie inside one graph;
// each block reduces its tile, then updates its graph's record atomically.
__global__ void __launch_bounds__(kBlock) k_validate(const int32_t *src, const int32_t *dst,
                                                     const int64_t *t, const Tile *tiles,
                                                     uint32_t n_tiles, const uint32_t *n_limit,
                                                     Stat *st) {
    __shared__ Stat ws[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
        const Tile tl = tiles[ti];
        const uint32_t lim = n_limit[tl.g];
        uint32_t bad = 0, mx = 0;
        uint64_t tmin = ~0ull, tmax = 0;
        for (uint64_t e = tl.b + threadIdx.x; e < tl.e; e += blockDim.x) {
            const int32_t a = src[e], b = dst[e];
            const int64_t te = t[e];
            if (a < 0 || b < 0 || (uint32_t)a >= lim || (uint32_t)b >= lim) bad |= 1u;
            if (a == b) bad |= 2u;
            if (te >= kTLimit || te <= -kTLimit) bad |= 4u;
            mx = max(mx, (uint32_t)max(a, b));
            const uint64_t k = (uint64_t)te ^ 0x8000000000000000ull;
            tmin = min(tmin, k);
            tmax = max(tmax, k);
        }
        for (int o = kWave / 2; o > 0; o >>= 1) {
            bad |= __shfl_xor(bad, o, kWave);
            mx = max(mx, (uint32_t)__shfl_xor(mx, o, kWave));
            tmin = min(tmin, (uint64_t)__shfl_xor(tmin, o, kWave));
            tmax = max(tmax, (uint64_t)__shfl_xor(tmax, o, kWave));
        }
        if (lane == 0) ws[w] = Stat{bad, mx, tmin, tmax};
        __syncthreads();
        if (threadIdx.x == 0) {
            Stat r = ws[0];
            for (int i = 1; i < kBlock / kWave; i++) {
                r.bad |= ws[i].bad;
                r.max_id = max(r.max_id, ws[i].max_id);
                r.tmin_key = min(r.tmin_key, ws[i].tmin_key);
                r.tmax_key = max(r.tmax_key, ws[i].tmax_key);
            }
            Stat *d = st + tl.g;
            if (r.bad) atomicOr(&d->bad, r.bad);
            atomicMax(&d->max_id, r.max_id);
            atomicMin((unsigned long long *)&d->tmin_key, (unsigned long long)r.tmin_key);
            atomicMax((unsigned long long *)&d->tmax_key, (unsigned long long)r.tmax_key);
        }
        __syncthreads();
    }
}

// Time-sort key = (graph << tbits) | (t - tmin of the graph); the value
// carries the endpoints as union-graph node ids (local id + graph's node base).
template <typename K>
__global__ void k_time_keys(const int32_t *src, const int32_t *dst, const int64_t *t,
                            const Tile *tiles, uint32_t n_tiles, const int64_t *tmin,
                            const uint32_t *node_base, int tbits, K *keys, EdgeVal *vals) {
    for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
        const Tile tl = tiles[ti];
        const int64_t t0 = tmin[tl.g];
        const uint32_t nb = node_base[tl.g];
        const uint64_t gk = (uint64_t)tl.g << tbits;
        for (uint64_t e = tl.b + threadIdx.x; e < tl.e; e += blockDim.x) {
            keys[e] = (K)(gk | (uint64_t)(t[e] - t0));
            vals[e] = EdgeVal{(uint32_t)src[e] + nb, (uint32_t)dst[e] + nb, (uint32_t)e};
        }
    }
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// off[u] = first position of node u in the node-sorted keys, atomic-free:
// each boundary between consecutive keys fills the offsets of the (absent)
// nodes it skips over, up to kGapFill of them; longer runs of absent nodes are
// left marked and resolved by k_offsets_gaps with a binary search.  Keys are
// below n after a sound sort; a key >= n can only be left over where a sort's
// look-back gave up (some positions then keep stale contents), so such a
// boundary writes nothing and raises the sort's error flag instead.
__global__ void k_offsets(const uint32_t *skey, uint64_t len, uint32_t n, uint32_t *off,
                          uint32_t *err) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= len;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t prev = p == 0 ? -1 : (int64_t)skey[p - 1];
        const int64_t cur = p == len ? (int64_t)n : (int64_t)skey[p];
        if (cur == prev) continue;
        if (cur > (int64_t)n || prev >= (int64_t)n) {
            atomicOr(err, 4u);
            continue;
        }
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

// Element g of the pair-sorted edges: bit 0 if its node pair has >= 2
// edges, bit 1 if it is also the first of its pair.
__global__ void k_pair_flags(const uint32_t *pkey, const uint2 *pval, uint64_t m, uint8_t *f) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < m;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t k = pkey[g], lo = pval[g].x;
        const bool same_prev = g > 0 && pkey[g - 1] == k && pval[g - 1].x == lo;
        const bool same_next = g + 1 < m && pkey[g + 1] == k && pval[g + 1].x == lo;
        f[g] = (uint8_t)((same_prev || same_next ? 1u : 0u) | (!same_prev && same_next ? 2u : 0u));
    }
}

struct MultiOut {
    uint32_t *mp_start, *mp_lo, *mp_hi;
    int64_t *me_t;
    uint2 *me_p;
    uint4 *me_a;
    uint8_t *me_o;  // bit 0: leaves the smaller node, bit 1: first of its pair
};

// pre: scan_flag_pairs of k_pair_flags (m + 1 entries): element g
// is in a pair with >= 2 edges iff the low words of pre[g] and pre[g + 1]
// differ, the first of its pair iff the high words do, and the low and high
// words of pre[g] are its element index and pair index.  An edge's time and
// positions come from erec when it is given (one line per edge), else from
// t_r and epos.
__global__ void k_multi_fill(const uint32_t *pkey, const uint2 *pval, uint64_t m,
                             const uint64_t *pre, const EdgeRec *erec, const int64_t *t_r,
                             const uint32_t *epos, const uint32_t *X, const uint32_t *off,
                             uint64_t n_multi, uint64_t n_me, MultiOut o) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < m;
         g += (uint64_t)gridDim.x * blockDim.x) {
        if (g == 0) o.mp_start[n_multi] = (uint32_t)n_me;
        const uint64_t a = pre[g], b = pre[g + 1];
        if ((uint32_t)a == (uint32_t)b) continue;
        const bool head = (a >> 32) != (b >> 32);
        const uint32_t k = (uint32_t)a;
        const uint2 pv = pval[g];
        const uint32_t lo = pv.x, hi = pkey[g];
        if (head) {
            const uint32_t q = (uint32_t)(a >> 32);
            o.mp_start[q] = k;
            o.mp_lo[q] = lo;
            o.mp_hi[q] = hi;
        }
        const uint32_t el = pv.y;
        const uint32_t r = el & ~kOrientBit;
        const uint32_t src_is_lo = el >> 31;
        // entry of this edge at lo / at hi: the src entry sits at 2r, the dst entry at 2r+1
        int64_t te;
        uint32_t p_src, p_dst;
        if (erec) {
            const EdgeRec e = erec[r];
            te = e.t;
            p_src = e.p_src;
            p_dst = e.p_dst;
        } else {
            te = t_r[r];
            p_src = epos[2 * (uint64_t)r];
            p_dst = epos[2 * (uint64_t)r + 1];
        }
        const uint32_t p_lo = src_is_lo ? p_src : p_dst;
        const uint32_t p_hi = src_is_lo ? p_dst : p_src;
        const uint32_t s_lo = off[lo], s_hi = off[hi];
        const uint32_t a1_lo = X[p_lo] - X[s_lo], a1_hi = X[p_hi] - X[s_hi];
        o.me_t[k] = te;
        o.me_p[k] = make_uint2(p_lo, p_hi);
        o.me_a[k] = make_uint4(p_lo - s_lo - a1_lo, a1_lo, p_hi - s_hi - a1_hi, a1_hi);
        // bit 0: the edge leaves the smaller node; bit 1: first element of its pair
        o.me_o[k] = (uint8_t)(src_is_lo | (head ? 2u : 0u));
    }
}

// Per graph: first S_u position, first multi-edge pair and its first element
// (pairs are ordered by their larger node, which lies in their graph).
__global__ void k_graph_ranges(const uint32_t *off, const uint32_t *node_base, uint32_t G,
                               const uint32_t *mp_hi, uint64_t n_multi, const uint32_t *mp_start,
                               uint32_t *ent_off, uint32_t *mpb, uint32_t *me_off) {
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= G;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t nb = node_base[g];
        ent_off[g] = off[nb];
        uint64_t a = 0, b = n_multi;  // first pair whose larger node is >= nb
        while (a < b) {
            const uint64_t mid = a + (b - a) / 2;
            if (mp_hi[mid] < nb) a = mid + 1;
            else b = mid;
        }
        mpb[g] = (uint32_t)a;
        me_off[g] = mp_start[a];
    }
}

__global__ void __launch_bounds__(kBlock) k_max_degree(const uint32_t *off, uint32_t n,
                                                       uint32_t *out) {
    uint32_t mx = 0;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (uint64_t)gridDim.x * blockDim.x)
        mx = max(mx, off[u + 1] - off[u]);
    for (int o = kWave / 2; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o, kWave));
    __shared__ uint32_t ws[kBlock / kWave];
    if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / kWave; i++) mx = max(mx, ws[i]);
        atomicMax(out, mx);
    }
}

}  // namespace

void set_force_edge_sort(bool on) { g_force_edge_sort.store(on); }

namespace {

int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) b++;
    return b;
}

dim3 grid_for(uint64_t n, uint64_t cap = 16384) {
    uint64_t nb = (n + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    if (nb > cap) nb = cap;
    return dim3((unsigned)nb);
}

}  // namespace

#define TRY(x)                 \
    do {                       \
        int _rc = (x);         \
        if (_rc) return _rc;   \
    } while (0)

int graph_alloc(tm_graph *g, void **p, size_t bytes) {
    const int rc = dev_alloc(p, bytes ? bytes : 256, g->stream);
    if (rc) return rc;
    g->allocs.push_back(*p);
    return TM_OK;
}

template <typename T>
static int galloc(tm_graph *g, T **p, size_t count) {
    return graph_alloc(g, (void **)p, count * sizeof(T));
}

// Tiles of at most `cap` items over per-graph ranges [bound[g], bound[g+1]).
static std::vector<Tile> make_tiles(const std::vector<uint64_t> &bound, uint64_t cap) {
    std::vector<Tile> tiles;
    for (size_t gi = 0; gi + 1 < bound.size(); gi++)
        for (uint64_t b = bound[gi]; b < bound[gi + 1]; b += cap)
            tiles.push_back(Tile{(uint32_t)gi, (uint32_t)b, (uint32_t)std::min(bound[gi + 1], b + cap)});
    return tiles;
}

static int upload_tiles(tm_graph *g, const std::vector<Tile> &tiles, Tile **out, uint32_t *count,
                        hipStream_t s) {
    *count = (uint32_t)tiles.size();
    TRY(galloc(g, out, std::max<size_t>(tiles.size(), 1)));
    if (!tiles.empty())
        TM_HIP_TRY(hipMemcpyAsync(*out, tiles.data(), tiles.size() * sizeof(Tile),
                                  hipMemcpyHostToDevice, s));
    return TM_OK;
}

int build_graph_device(tm_graph *g, const int32_t *src, const int32_t *dst, const int64_t *t,
                       const uint64_t *eoff, const uint32_t *ncount, uint32_t G, hipStream_t s) {
    const uint64_t m = eoff[G];
    g->m = m;
    g->G = G;
    g->h_eoff.assign(eoff, eoff + G + 1);
    // ---- 1. per-graph validation
    std::vector<Stat> h_st(G, Stat{0, 0, ~0ull, 0});
    std::vector<uint32_t> h_lim(G);
    for (uint32_t i = 0; i < G; i++) h_lim[i] = ncount[i] ? ncount[i] : 0x7fffffffu;
    const std::vector<Tile> etiles = make_tiles(g->h_eoff, 1u << 13);
    {
        ProfRow row_a1("a1");
        Scratch vs;
        TRY(vs.reserve(G * sizeof(Stat) + G * 4 + etiles.size() * sizeof(Tile) + 1024, s));
        Stat *d_st = vs.take<Stat>(G);
        uint32_t *d_lim = vs.take<uint32_t>(G);
        Tile *d_et = vs.take<Tile>(std::max<size_t>(etiles.size(), 1));
        TM_HIP_TRY(hipMemcpyAsync(d_st, h_st.data(), G * sizeof(Stat), hipMemcpyHostToDevice, s));
        TM_HIP_TRY(hipMemcpyAsync(d_lim, h_lim.data(), G * 4, hipMemcpyHostToDevice, s));
        if (!etiles.empty()) {
            TM_HIP_TRY(hipMemcpyAsync(d_et, etiles.data(), etiles.size() * sizeof(Tile),
                                      hipMemcpyHostToDevice, s));
            TM_LAUNCH("validate", k_validate,
                      dim3((unsigned)std::min<size_t>(etiles.size(), kMaxStatBlocks)), dim3(kBlock), 0,
                      s, src, dst, t, d_et, (uint32_t)etiles.size(), d_lim, d_st);
        }
        TM_HIP_TRY(hipMemcpyAsync(h_st.data(), d_st, G * sizeof(Stat), hipMemcpyDeviceToHost, s));
        TM_HIP_TRY(hipStreamSynchronize(s));
    }
    std::vector<uint32_t> node_base(G + 1, 0);
    std::vector<int64_t> tmin_g(G, 0);
    int tbits = 0;
    bool any_t = false;
    int64_t t_lo = 0, t_hi = 0;  // over all graphs
    for (uint32_t i = 0; i < G; i++) {
        if (h_st[i].bad) {
            const uint32_t bad = h_st[i].bad;
            set_error(std::string("invalid edge list") + (G > 1 ? " (graph " + std::to_string(i) + ")" : "") +
                      ":" + ((bad & 1) ? " node id out of range" : "") + ((bad & 2) ? " self-loop" : "") +
                      ((bad & 4) ? " |t| >= 2^62" : ""));
            return TM_EINVAL;
        }
        const bool has_edges = eoff[i + 1] > eoff[i];
        const uint64_t ni = ncount[i] ? ncount[i] : (has_edges ? (uint64_t)h_st[i].max_id + 1 : 0);
        if ((uint64_t)node_base[i] + ni > 0x7fffffffull) {
            set_error("total node count must be below 2^31");
            return TM_EINVAL;
        }
        node_base[i + 1] = node_base[i] + (uint32_t)ni;
        if (has_edges) {
            const int64_t lo = (int64_t)(h_st[i].tmin_key ^ 0x8000000000000000ull);
            const int64_t hi = (int64_t)(h_st[i].tmax_key ^ 0x8000000000000000ull);
            tmin_g[i] = lo;
            tbits = std::max(tbits, bits_for((uint64_t)(hi - lo)));
            t_lo = any_t ? std::min(t_lo, lo) : lo;
            t_hi = any_t ? std::max(t_hi, hi) : hi;
            any_t = true;
        }
    }
    const int gbits = bits_for(G - 1);
    if (gbits + tbits > 64) {
        set_error("graph index and time range do not fit one 64-bit sort key");
        return TM_EINVAL;
    }
    const uint64_t n = node_base[G];
    g->n = (uint32_t)n;
    g->h_node_base = node_base;
    const uint64_t len = 2 * m;
    TRY(galloc(g, &g->off, n + 1));
    TRY(galloc(g, &g->ent_t, len));
    TRY(galloc(g, &g->ent_nd, len));
    TRY(galloc(g, &g->ent_r, len));
    TRY(galloc(g, &g->ent_c, len));
    TRY(galloc(g, &g->X, len + 1));
    TRY(galloc(g, &g->epos, len));
    TRY(galloc(g, &g->perm, m));
    TRY(galloc(g, &g->d_eoff, G + 1));
    {
        std::vector<uint32_t> e32(G + 1);
        for (uint32_t i = 0; i <= G; i++) e32[i] = (uint32_t)eoff[i];
        TM_HIP_TRY(hipMemcpyAsync(g->d_eoff, e32.data(), (G + 1) * 4, hipMemcpyHostToDevice, s));
    }
    if (m == 0) {
        TM_HIP_TRY(hipMemsetAsync(g->off, 0, (n + 1) * sizeof(uint32_t), s));
        TM_HIP_TRY(hipMemsetAsync(g->X, 0, sizeof(uint32_t), s));
        TRY(galloc(g, &g->mp_start, 1));
        TM_HIP_TRY(hipMemsetAsync(g->mp_start, 0, sizeof(uint32_t), s));
        TRY(galloc(g, &g->d_mpb, G + 1));
        TM_HIP_TRY(hipMemsetAsync(g->d_mpb, 0, (G + 1) * sizeof(uint32_t), s));
        g->h_ent_off.assign(G + 1, 0);
        g->h_mpb.assign(G + 1, 0);
        g->h_me_off.assign(G + 1, 0);
        TM_HIP_TRY(hipStreamSynchronize(s));
        return TM_OK;
    }
    const int kbits = gbits + tbits;
    uint32_t *d_nb = nullptr;
    TRY(galloc(g, &d_nb, G + 1));
    g->d_node_base = d_nb;
    TM_HIP_TRY(hipMemcpyAsync(d_nb, node_base.data(), (G + 1) * 4, hipMemcpyHostToDevice, s));
    TRY(galloc(g, &g->d_tmin, G));
    TM_HIP_TRY(hipMemcpyAsync(g->d_tmin, tmin_g.data(), G * 8, hipMemcpyHostToDevice, s));
    Tile *d_etiles = nullptr;
    uint32_t n_etiles = 0;
    TRY(upload_tiles(g, etiles, &d_etiles, &n_etiles, s));

    // ---- scratch (stream-ordered, released when this function returns)
    // KA, KB: 8 bytes x 2m each   (time keys, node keys; later the pair
    //                              flags' prefix (KA) and bytes (KB))
    // VA, VB: 16 bytes x 2m each  (EdgeVal of m, NodeVal(32) of 2m; later the
    //                              slots and the EdgeRec of m)
    // PKA, PKB: 8 bytes x m; PVA, PVB: u32 x m   (pair sort values, keys)
    // TR: i64 x m                 (timestamps by rank)
    // TMP: scan / histogram scratch (the flag scan's u64 partials too)
    const size_t ntmp =
        std::max({radix_tmp_bytes(len) / 4 + 1, scan_tmp_count(len), 2 * scan_tmp_count(m),
                  (size_t)3 * (G + 1)}) + 16;
    Scratch sc;
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t bytes = 2 * up(8 * len) + 2 * up(16 * len) + 2 * up(8 * m) + 2 * up(4 * m) +
                         up(8 * m) + up(4 * ntmp) + up(4);
    TRY(sc.reserve(bytes, s));
    char *KA = sc.take<char>(8 * len), *KB = sc.take<char>(8 * len);
    char *VA = sc.take<char>(16 * len), *VB = sc.take<char>(16 * len);
    uint64_t *PKA = sc.take<uint64_t>(m), *PKB = sc.take<uint64_t>(m);
    uint32_t *PVA = sc.take<uint32_t>(m), *PVB = sc.take<uint32_t>(m);
    int64_t *TR = sc.take<int64_t>(m);
    uint32_t *tmp = sc.take<uint32_t>(ntmp);
    uint32_t *sort_err = sc.take<uint32_t>(1);
    TM_LAUNCH("sort_err_clear", k_fill_u32, dim3(1), dim3(kBlock), 0, s, sort_err, 1, 0u);

    // trace rows: a2 the sequences S_u (time sort, node sort, offsets,
    // direction prefix), a3 the node-pair lists
    ProfRow row_a2("a2");
    // ---- 2. time sort carrying (src, dst, id); its last pass writes the
    // rank-ordered arrays.  Pass i writes the (KB, VB) set when i is even, so
    // the last pass reads (KA, VA) when the pass count is odd and the node
    // keys and values go to the set it does not read.  One graph: the first
    // pass reads the input arrays themselves; a batch adds the graph index
    // and the node base in k_time_keys first.
    // timestamps within 2^32 of the smallest go through the node sort as
    // 32-bit offsets (|t| < 2^62, so the difference fits an int64)
    const bool t32 = (uint64_t)(t_hi - t_lo) <= 0xffffffffull;
    uint32_t *nkey = nullptr;
    NodeVal *nval = nullptr;
    EdgeRec *erec = nullptr;  // per-edge (t, positions), built with the bucketed index
    {
        const int tpasses = (std::max(kbits, 1) + 7) / 8;
        const bool to_b = (tpasses % 2) == 1;
        nkey = reinterpret_cast<uint32_t *>(to_b ? KB : KA);
        nval = reinterpret_cast<NodeVal *>(to_b ? VB : VA);
        const RankOut ro{g->d_tmin, G > 1 ? tbits : 64, TR, g->perm, nkey, t32 ? nullptr : nval,
                         t32 ? reinterpret_cast<NodeVal32 *>(nval) : nullptr, t_lo};
        EdgeVal *ev = reinterpret_cast<EdgeVal *>(VA), *ev_alt = reinterpret_cast<EdgeVal *>(VB);
        const dim3 tgrid((unsigned)std::min<uint32_t>(n_etiles, 4096));
        if (kbits <= 32) {
            uint32_t *k = reinterpret_cast<uint32_t *>(KA), *k_alt = reinterpret_cast<uint32_t *>(KB);
            if (G == 1) {
                TRY(radix_sort_time_direct_u32(src, dst, t, k, k_alt, ev, ev_alt, m, kbits, tmp,
                                               sort_err, s, ro));
            } else {
                TM_LAUNCH("time_keys", k_time_keys<uint32_t>, tgrid, dim3(kBlock), 0, s, src, dst, t,
                          d_etiles, n_etiles, g->d_tmin, d_nb, tbits, k, ev);
                TRY(radix_sort_time_u32(k, k_alt, ev, ev_alt, m, kbits, tmp, sort_err, s, ro));
            }
        } else {
            uint64_t *k = reinterpret_cast<uint64_t *>(KA), *k_alt = reinterpret_cast<uint64_t *>(KB);
            if (G == 1) {
                TRY(radix_sort_time_direct_u64(src, dst, t, k, k_alt, ev, ev_alt, m, kbits, tmp,
                                               sort_err, s, ro));
            } else {
                TM_LAUNCH("time_keys", k_time_keys<uint64_t>, tgrid, dim3(kBlock), 0, s, src, dst, t,
                          d_etiles, n_etiles, g->d_tmin, d_nb, tbits, k, ev);
                TRY(radix_sort_time_u64(k, k_alt, ev, ev_alt, m, kbits, tmp, sort_err, s, ro));
            }
        }
    }

    // ---- 3. node sort -> S_u (the last pass writes the sequence arrays and epos)
    {
        uint32_t *k_alt = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(nkey) == KA ? KB : KA);
        NodeVal *v_alt = reinterpret_cast<NodeVal *>(reinterpret_cast<char *>(nval) == VA ? VB : VA);
        // the last pass reads (nkey, nval) after an odd number of passes,
        // else (k_alt, v_alt); the slots it writes go to the other value
        // buffer, and the edge positions are then sorted through the two
        // key buffers (8 bytes per entry each, both free by then)
        const int node_passes = (std::max(bits_for(n - 1), 1) + 7) / 8;
        char *k_read = reinterpret_cast<char *>(node_passes % 2 ? nkey : k_alt);
        char *k_free = reinterpret_cast<char *>(node_passes % 2 ? k_alt : nkey);
        uint32_t *slots = reinterpret_cast<uint32_t *>(node_passes % 2 ? (void *)v_alt : (void *)nval);
        // an index that fits the last-level cache is scattered directly
        const bool direct = len * sizeof(uint32_t) <= kDirectEposBytes && !g_force_edge_sort.load();
        const SeqOut so{g->ent_c, g->ent_t, g->ent_nd, g->ent_r, direct ? g->epos : nullptr, slots,
                        (uint64_t)len, t_lo};
        if (t32)
            TRY(radix_sort_nodes(nkey, k_alt, reinterpret_cast<NodeVal32 *>(nval),
                                 reinterpret_cast<NodeVal32 *>(v_alt), len, bits_for(n - 1), tmp,
                                 sort_err, s, so));
        else
            TRY(radix_sort_nodes(nkey, k_alt, nval, v_alt, len, bits_for(n - 1), tmp, sort_err, s, so));
        if (!direct) {
            uint32_t *k0 = reinterpret_cast<uint32_t *>(k_read), *v0 = k0 + len;
            uint32_t *k1 = reinterpret_cast<uint32_t *>(k_free), *v1 = k1 + len;
            // the edge records go to the value buffer the last pass read
            erec = reinterpret_cast<EdgeRec *>(node_passes % 2 ? (void *)nval : (void *)v_alt);
            TRY(edge_positions(slots, len, k0, v0, k1, v1, tmp, sort_err, s, g->epos, TR, erec));
        }
        TM_LAUNCH("offsets_fill", k_fill_u32, grid_for(n + 1), dim3(kBlock), 0, s, g->off, n + 1,
                  kUnset);
        TM_LAUNCH("offsets", k_offsets, grid_for(len + 1), dim3(kBlock), 0, s, g->ent_c, len,
                  (uint32_t)n, g->off, sort_err);
        TM_LAUNCH("offsets_gaps", k_offsets_gaps, grid_for(n + 1), dim3(kBlock), 0, s, g->ent_c, len,
                  (uint32_t)n, g->off);
        TRY(scan_dirbits(g->ent_nd, g->X, len, tmp, s));
    }

    // ---- 4. node-pair edge sets; the edges of pairs with >= 2 edges
    {
        ProfRow row_a3("a3");
        // each edge once, from its entry at the smaller node, in S order
        uint32_t *k = PVA, *k_alt = PVB;
        uint2 *v = reinterpret_cast<uint2 *>(PKA), *v_alt = reinterpret_cast<uint2 *>(PKB);
        TRY(lower_side_pairs(g->ent_c, g->ent_nd, g->ent_r, len, k, v, tmp, s));
        TRY(radix_sort_pairs(&k, &k_alt, &v, &v_alt, m, bits_for(n - 1), tmp, sort_err, s));
        // flag bytes, then the element and pair indices of the pairs with >=
        // 2 edges, in the (now free) node-sort key buffers; tmp holds the
        // scan's u64 partials
        uint8_t *flags = reinterpret_cast<uint8_t *>(KB);
        uint64_t *pre = reinterpret_cast<uint64_t *>(KA);
        TM_LAUNCH("pair_flags", k_pair_flags, grid_for(m), dim3(kBlock), 0, s, k, v, m, flags);
        TRY(scan_flag_pairs(flags, m, pre, reinterpret_cast<uint64_t *>(tmp), s));
        uint64_t totals = 0;
        uint32_t err = 0;
        TM_HIP_TRY(hipMemcpyAsync(&totals, pre + m, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        TM_HIP_TRY(hipMemcpyAsync(&err, sort_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TM_HIP_TRY(hipStreamSynchronize(s));
        if (err) {
            set_error("radix sort: a look-back wait gave up (device graph not built)");
            return TM_EINTERNAL;
        }
        g->n_me = (uint32_t)totals;
        g->n_multi = (uint32_t)(totals >> 32);
        TRY(galloc(g, &g->mp_start, g->n_multi + 1));
        TRY(galloc(g, &g->mp_lo, g->n_multi));
        TRY(galloc(g, &g->mp_hi, g->n_multi));
        TRY(galloc(g, &g->me_t, g->n_me));
        TRY(galloc(g, &g->me_p, g->n_me));
        TRY(galloc(g, &g->me_a, g->n_me));
        TRY(galloc(g, &g->me_o, g->n_me));
        MultiOut o{g->mp_start, g->mp_lo, g->mp_hi, g->me_t, g->me_p, g->me_a, g->me_o};
        TM_LAUNCH("multi_fill", k_multi_fill, grid_for(m), dim3(kBlock), 0, s, k, v, m, pre, erec,
                  TR, g->epos, g->X, g->off, g->n_multi, g->n_me, o);
    }

    // ---- 5. per-graph ranges and the static work tiles
    {
        uint32_t *r3 = tmp;  // 3 x (G + 1)
        TRY(galloc(g, &g->d_mpb, G + 1));
        TM_LAUNCH("graph_ranges", k_graph_ranges, grid_for(G + 1), dim3(kBlock), 0, s, g->off, d_nb, G,
                  g->mp_hi, g->n_multi, g->mp_start, r3, g->d_mpb, r3 + 2 * (G + 1));
        std::vector<uint32_t> h(3 * (G + 1));
        if (G == 1) {
            // one graph: its ranges are the whole arrays, known here already
            h = {0u, (uint32_t)len, 0u, (uint32_t)g->n_multi, 0u, (uint32_t)g->n_me};
        } else {
            TM_HIP_TRY(hipMemcpyAsync(h.data(), r3, (G + 1) * 4, hipMemcpyDeviceToHost, s));
            TM_HIP_TRY(hipMemcpyAsync(h.data() + (G + 1), g->d_mpb, (G + 1) * 4, hipMemcpyDeviceToHost, s));
            TM_HIP_TRY(hipMemcpyAsync(h.data() + 2 * (G + 1), r3 + 2 * (G + 1), (G + 1) * 4,
                                      hipMemcpyDeviceToHost, s));
            TM_HIP_TRY(hipStreamSynchronize(s));
        }
        g->h_ent_off.assign(h.begin(), h.begin() + (G + 1));
        g->h_mpb.assign(h.begin() + (G + 1), h.begin() + 2 * (G + 1));
        g->h_me_off.assign(h.begin() + 2 * (G + 1), h.end());
        std::vector<uint64_t> eb(G + 1), mb(G + 1);
        for (uint32_t i = 0; i <= G; i++) {
            eb[i] = g->h_ent_off[i];
            mb[i] = 2 * (uint64_t)g->h_me_off[i];  // element sides
        }
        TRY(upload_tiles(g, make_tiles(eb, kEntryTile), &g->t_entries, &g->n_t_entries, s));
        TRY(upload_tiles(g, make_tiles(mb, kElemTile), &g->t_elems, &g->n_t_elems, s));
        TM_HIP_TRY(hipStreamSynchronize(s));
    }

    return TM_OK;
}

int graph_max_degree(tm_graph *g, uint64_t *out) {
    if (!g->max_degree_known) {
        hipStream_t s = g->stream;
        Scratch sc;
        TRY(sc.reserve(256, s));
        uint32_t *d_mx = sc.take<uint32_t>(1);
        TM_HIP_TRY(hipMemsetAsync(d_mx, 0, sizeof(uint32_t), s));
        if (g->n) {
            TM_LAUNCH("max_degree", k_max_degree, grid_for(g->n, kMaxStatBlocks), dim3(kBlock), 0, s,
                      g->off, g->n, d_mx);
        }
        uint32_t mx = 0;
        TM_HIP_TRY(hipMemcpyAsync(&mx, d_mx, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TM_HIP_TRY(hipStreamSynchronize(s));
        g->max_degree = mx;
        g->max_degree_known = true;
    }
    *out = g->max_degree;
    return TM_OK;
}

}  // namespace tmc
