// Four-node three-edge delta-temporal motifs.
//
// The paper leaves higher-order motifs to future work (Section VI) and names
// the route: more centers and bigger counters.  A four-node instance (three
// distinct edges in (t, id) order, t(E3) - t(E1) <= delta, connected, four
// nodes) is a star, one node on all three edges, or a path v0-v1-v2-v3; the
// 32 classes are laid out in tm.h (tm_count4).  Both shapes are counted from
// sums over S_u (the S_u sequences, direction prefix X and edge positions of
// the graph build) and then corrected with the 36 three-edge classes:
//
//  stars  Every entry p of S_c, taken as E1, with the ordered pairs of later
//         entries of S_c inside delta split by direction: O(1) per entry from
//         X and Q(x) = the sum of X over the out-entries before x.  Summed
//         over centers this is every triple of one node's edges: the
//         four-node stars, the three-node stars at their center and each pair
//         instance once from each of its nodes (the paper's Star and Pair
//         counters), which are subtracted.
//  paths  Every edge e = s -> d, taken as the middle edge, with one more
//         edge x at s and one more edge y at d inside delta, classified by
//         chronological position and direction as a path is.  Of the two
//         windows that pair up, the smaller one is walked and each of its
//         entries binary-searches the other.  Besides the paths this counts
//         every triangle three times, every three-node star twice and every
//         pair six times, each into classes fixed by its own class; those are
//         subtracted with a table the library builds by running the same
//         classification over one instance of each of the 36 classes.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "tm_internal.h"

namespace tmc {
namespace {

constexpr uint32_t kQItems = 16;
constexpr uint32_t kQTile = kBlock * kQItems;
constexpr uint32_t kPartsBlock = 1024;
constexpr uint32_t kStarGrid = 4096;
constexpr uint32_t kPathGrid = 4096;

// ------------------------------------------------------------ block helpers
__device__ inline uint64_t wave_sum(uint64_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Exclusive scan of one value per thread over the block; *total = block sum.
// lds: blockDim.x / kWave entries.
__device__ inline uint64_t block_exclusive_scan(uint64_t v, uint64_t *lds, uint64_t *total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint64_t inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t n = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += n;
    }
    if (lane == kWave - 1) lds[w] = inc;
    __syncthreads();
    uint64_t before = 0, tot = 0;
    const int nw = blockDim.x / kWave;
    for (int i = 0; i < nw; i++) {
        const uint64_t x = lds[i];
        before += (i < w) ? x : 0;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

// Sum N per-thread counters over the block into row[0, N).
template <int N>
__device__ inline void block_rows(const uint64_t (&acc)[N], uint64_t (*red)[N], uint64_t *row) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int i = 0; i < N; i++) {
        const uint64_t v = wave_sum(acc[i]);
        if (lane == 0) red[w][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        uint64_t s = 0;
        for (int q = 0; q < kBlock / kWave; q++) s += red[q][threadIdx.x];
        row[threadIdx.x] = s;
    }
}

// ------------------------------------------------------- u64 prefix sums
// Exclusive prefix sums of len values given by a loader, out[len] = total, in
// three launches: tile sums, a one-block scan of them, the tiles.
// value of entry y in Q: X[y] if the entry leaves its center, else 0
struct QLoad {
    const uint32_t *nd, *X;
    __device__ inline uint64_t operator()(uint64_t y) const {
        return (nd[y] & 1u) ? 0ull : (uint64_t)X[y];
    }
};

template <class L>
__global__ void __launch_bounds__(kBlock) k_u64_tile_sum(L ld, uint64_t len, uint64_t *part) {
    __shared__ uint64_t red[kBlock / kWave][1];
    const uint64_t base = (uint64_t)blockIdx.x * kQTile;
    uint64_t acc[1] = {0};
    for (uint32_t k = threadIdx.x; k < kQTile; k += kBlock) {
        const uint64_t y = base + k;
        if (y < len) acc[0] += ld(y);
    }
    block_rows<1>(acc, red, part + blockIdx.x);
}

// Exclusive scan of part[0, np) in place, part[np] = total; one block.
__global__ void __launch_bounds__(kPartsBlock) k_u64_parts(uint64_t *part, uint32_t np) {
    __shared__ uint64_t lds[kPartsBlock / kWave];
    const uint32_t per = (np + kPartsBlock - 1) / kPartsBlock;
    const uint32_t b = min(np, threadIdx.x * per), e = min(np, b + per);
    uint64_t s = 0;
    for (uint32_t i = b; i < e; i++) s += part[i];
    uint64_t total;
    uint64_t run = block_exclusive_scan(s, lds, &total);
    for (uint32_t i = b; i < e; i++) {
        const uint64_t v = part[i];
        part[i] = run;
        run += v;
    }
    if (threadIdx.x == 0) part[np] = total;
}

// out[y] for y in the block's tile (each thread kQItems consecutive values);
// the block holding len also writes out[len].
template <class L>
__global__ void __launch_bounds__(kBlock) k_u64_tile_scan(L ld, uint64_t len, const uint64_t *part,
                                                          uint64_t *Q) {
    __shared__ uint64_t lds[kBlock / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kQTile + (uint64_t)threadIdx.x * kQItems;
    uint64_t v[kQItems];
    uint64_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kQItems; k++) {
        const uint64_t y = base + k;
        v[k] = y < len ? ld(y) : 0;
        s += v[k];
    }
    uint64_t total;
    uint64_t run = part[blockIdx.x] + block_exclusive_scan(s, lds, &total);
#pragma unroll
    for (uint32_t k = 0; k < kQItems; k++) {
        const uint64_t y = base + k;
        if (y <= len) Q[y] = run;
        run += v[k];
    }
}

// ------------------------------------------------------------ window search
// Last x in [p, hi) with T[x] <= lim, given T[p] <= lim (gallop, bisect).
__device__ inline uint32_t last_le_from(const int64_t *T, uint32_t p, uint32_t hi, int64_t lim) {
    int64_t lo = p, top = hi;
    uint64_t step = 1;
    while (true) {
        const int64_t probe = lo + (int64_t)step;
        if (probe >= top) break;
        if (T[probe] <= lim) {
            lo = probe;
            step <<= 1;
        } else {
            top = probe;
            break;
        }
    }
    while (top - lo > 1) {
        const int64_t mid = lo + (top - lo) / 2;
        if (T[mid] <= lim) lo = mid;
        else top = mid;
    }
    return (uint32_t)lo;
}

// First x in [lo, p] with T[x] >= lim, given T[p] >= lim (gallop backwards).
__device__ inline uint32_t first_ge_back(const int64_t *T, uint32_t lo, uint32_t p, int64_t lim) {
    int64_t hi = p, bot = (int64_t)lo - 1;
    uint64_t step = 1;
    while (true) {
        const int64_t probe = hi - (int64_t)step;
        if (probe <= bot) break;
        if (T[probe] >= lim) {
            hi = probe;
            step <<= 1;
        } else {
            bot = probe;
            break;
        }
    }
    while (hi - bot > 1) {
        const int64_t mid = bot + (hi - bot) / 2;
        if (T[mid] >= lim) hi = mid;
        else bot = mid;
    }
    return (uint32_t)hi;
}

// First i in [lo, hi) with A[i] >= v, else hi.
__device__ inline uint32_t lower_rank(const uint32_t *A, uint32_t lo, uint32_t hi, uint32_t v) {
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (A[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// First i in [lo, hi) with T[i] > v, else hi.
__device__ inline uint32_t upper_time(const int64_t *T, uint32_t lo, uint32_t hi, int64_t v) {
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (T[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// First i in [lo, hi) with T[i] >= v, else hi.
__device__ inline uint32_t lower_time(const int64_t *T, uint32_t lo, uint32_t hi, int64_t v) {
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (T[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------- stars
// Per entry p of S_c as E1: ordered pairs (k < l) of entries in (p, R] with
// R the last entry of S_c at t <= t_p + delta, by (dir k, dir l):
//   n1 = in-entries, n0 = out-entries of the window [a, b) = [p + 1, R + 1)
//   (in, in) = C(n1, 2), (out, out) = C(n0, 2),
//   (in, out) = sum over out-entries l in [a, b) of (X[l] - X[a])
//             = Q[b] - Q[a] - n0 X[a],  (out, in) = n0 n1 - (in, out).
// Counter [d1][d2][d3], d = 0 for out (the paper's o), 1 for in.
// The same pass writes each entry's window sizes for the paths: w[p] = (later
// entries of S_c inside delta, earlier ones).
__global__ void __launch_bounds__(kBlock) k_star4(const int64_t *T, const uint32_t *nd,
                                                  const uint32_t *C, const uint32_t *off,
                                                  const uint32_t *X, const uint64_t *Q,
                                                  uint64_t len, int64_t delta, uint64_t *rows,
                                                  uint2 *w) {
    __shared__ uint64_t red[kBlock / kWave][8];
    uint64_t acc[8];
#pragma unroll
    for (int i = 0; i < 8; i++) acc[i] = 0;
    for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < len;
         p += (uint64_t)gridDim.x * kBlock) {
        const uint32_t c = C[p];
        const int64_t tp = T[p];
        const uint32_t R = last_le_from(T, (uint32_t)p, off[c + 1], tp + delta);
        const uint32_t L = first_ge_back(T, off[c], (uint32_t)p, tp - delta);
        w[p] = make_uint2(R - (uint32_t)p, (uint32_t)p - L);
        if (R <= p + 1) continue;  // fewer than two later entries
        const uint32_t a = (uint32_t)p + 1, b = R + 1;
        const uint64_t xa = X[a];
        const uint64_t n1 = X[b] - xa, n0 = (uint64_t)(b - a) - n1;
        const uint64_t s11 = n1 * (n1 - (n1 > 0)) / 2, s00 = n0 * (n0 - (n0 > 0)) / 2;
        const uint64_t s10 = Q[b] - Q[a] - n0 * xa;
        const uint64_t s01 = n0 * n1 - s10;
        const bool d1 = nd[p] & 1u;
        acc[0] += d1 ? 0 : s00;
        acc[1] += d1 ? 0 : s01;
        acc[2] += d1 ? 0 : s10;
        acc[3] += d1 ? 0 : s11;
        acc[4] += d1 ? s00 : 0;
        acc[5] += d1 ? s01 : 0;
        acc[6] += d1 ? s10 : 0;
        acc[7] += d1 ? s11 : 0;
    }
    block_rows<8>(acc, red, rows + (uint64_t)blockIdx.x * 8);
}

// ------------------------------------------------------------------- paths
// Path classes (within the 24 path counters): r * 8 + f1 * 4 + f2 * 2 + f3,
// r = chronological position of the middle edge, f = 1 for an edge pointing
// away from the end whose end edge comes first.  With e = s -> d in the
// middle, x at s (dx = 1 if x enters s), y at d (dy = 1 if y enters d):
//   e first,  x < y:  4 + 2 dx + (1 - dy)     e first,  y < x:  2 dy + (1 - dx)
//   e second, x < y:  8 + 4 dx + 2 + (1 - dy) e second, y < x:  8 + 4 dy + (1 - dx)
//   e last,   x < y: 16 + 4 dx + 2 (1 - dy) + 1
//   e last,   y < x: 16 + 4 dy + 2 (1 - dx)
// Each update below adds a count of entries of one direction (in, out) of the
// searched window to the counter its class picks, selected by the walked
// entry's direction bit b: I0 when b = 0, I1 when b = 1.
template <int I0, int I1>
__device__ inline void sel_add(uint64_t (&acc)[24], uint32_t b, uint64_t v) {
    acc[I0] += b ? 0 : v;
    acc[I1] += b ? v : 0;
}

struct Range {
    uint32_t lo, hi;  // [lo, hi)
    __device__ inline uint32_t size() const { return hi - lo; }
};

struct PathArgs {
    const int64_t *T;
    const uint32_t *nd, *rk, *C, *X, *off, *epos;
    uint64_t m;
    int64_t delta;
};

// in-entries of [a, b) (a <= b)
__device__ inline uint64_t ins(const uint32_t *X, uint32_t a, uint32_t b) { return X[b] - X[a]; }

// Window sizes of edge r as the middle edge e = s -> d, e at ps in S_s and
// pd in S_d: (|As|, |Ad|, |Bs|, |Bd|) with As = (ps, R_s], Ad = (pd, R_d] the
// later entries inside delta and Bs = [L_s, ps), Bd = [L_d, pd) the earlier
// ones, gathered from the per-entry sizes.
__global__ void __launch_bounds__(kBlock) k_path_prep(const uint32_t *epos, const uint2 *w,
                                                      uint64_t m, uint4 *sz) {
    for (uint64_t r = (uint64_t)blockIdx.x * kBlock + threadIdx.x; r < m;
         r += (uint64_t)gridDim.x * kBlock) {
        const uint2 pp = reinterpret_cast<const uint2 *>(epos)[r];
        const uint2 a = w[pp.x], b = w[pp.y];
        sz[r] = make_uint4(a.x, b.x, a.y, b.y);
    }
}

// The four pairings walk the smaller window: e first (As, Ad), e last (Bs,
// Bd), e second with x first (Bs, Ad) and with y first (Bd, As).
__device__ inline void path_costs(uint4 z, uint32_t (&c)[4]) {
    c[0] = min(z.x, z.y);
    c[1] = min(z.z, z.w);
    c[2] = min(z.z, z.y);
    c[3] = min(z.w, z.x);
}

struct CostLoad {
    const uint4 *sz;
    __device__ inline uint64_t operator()(uint64_t r) const {
        uint32_t c[4];
        path_costs(sz[r], c);
        return (uint64_t)c[0] + c[1] + c[2] + c[3];
    }
};

// Items are numbered edge by edge (io = exclusive prefix of the costs); a
// wave takes 64 consecutive items.  ce[c] = the edge of item 64c (the last
// edge for the chunk past the end).
__global__ void __launch_bounds__(kBlock) k_chunk_edges(const uint64_t *io, uint64_t m,
                                                        uint64_t n_items, uint64_t n_chunks,
                                                        uint32_t *ce) {
    for (uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x; c <= n_chunks;
         c += (uint64_t)gridDim.x * kBlock) {
        const uint64_t item = min(c * kWave, n_items - 1);
        uint64_t lo = 0, hi = m;  // largest r with io[r] <= item
        while (hi - lo > 1) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (io[mid] <= item) lo = mid;
            else hi = mid;
        }
        ce[c] = (uint32_t)lo;
    }
}

// Per walked set (which window is walked against which), the counters of the
// searched window's entries, indexed [slot * 2 + b] for the walked entry's
// direction bit b; rank walks have four slots (in / out before it, in / out
// after it), time walks two (in / out inside delta).
template <int A0, int A1, int B0, int B1, int C0, int C1, int D0, int D1>
__device__ inline void add_rank(uint64_t (&acc)[24], uint32_t b, uint64_t il, uint64_t ol,
                                uint64_t ih, uint64_t oh) {
    sel_add<A0, A1>(acc, b, il);
    sel_add<B0, B1>(acc, b, ol);
    sel_add<C0, C1>(acc, b, ih);
    sel_add<D0, D1>(acc, b, oh);
}

// One item: the j-th walked entry of one pairing of edge r's windows.
__device__ inline void path_item(const PathArgs &g, const uint4 *sz, uint64_t r, uint64_t j,
                                 uint64_t (&acc)[24]) {
    const uint4 z = sz[r];
    uint32_t c[4];
    path_costs(z, c);
    const uint32_t ps = g.epos[2 * r], pd = g.epos[2 * r + 1];
    const Range As{ps + 1, ps + 1 + z.x}, Ad{pd + 1, pd + 1 + z.y};
    const Range Bs{ps - z.z, ps}, Bd{pd - z.w, pd};
    int set;
    Range W, V;
    if (j < c[0]) {
        const bool wx = z.x <= z.y;
        set = wx ? 0 : 1;
        W = wx ? As : Ad;
        V = wx ? Ad : As;
    } else if ((j -= c[0]) < c[1]) {
        const bool wx = z.z <= z.w;
        set = wx ? 2 : 3;
        W = wx ? Bs : Bd;
        V = wx ? Bd : Bs;
    } else if ((j -= c[1]) < c[2]) {
        const bool wx = z.z <= z.y;
        set = wx ? 4 : 5;
        W = wx ? Bs : Ad;
        V = wx ? Ad : Bs;
    } else {
        j -= c[2];
        const bool wy = z.w <= z.x;
        set = wy ? 6 : 7;
        W = wy ? Bd : As;
        V = wy ? As : Bd;
    }
    const uint32_t w = W.lo + (uint32_t)j;
    const uint32_t b = g.nd[w] & 1u;
    uint64_t il, ol, ih = 0, oh = 0;
    if (set < 4) {
        // by rank: entries of V before w and after w (an entry of the same
        // edge, a parallel edge seen from both ends, is in neither)
        const uint32_t rw = g.rk[w];
        const uint32_t lb = lower_rank(g.rk, V.lo, V.hi, rw);
        const uint32_t ub = lb + ((lb < V.hi && g.rk[lb] == rw) ? 1u : 0u);
        il = ins(g.X, V.lo, lb);
        ol = (lb - V.lo) - il;
        ih = ins(g.X, ub, V.hi);
        oh = (V.hi - ub) - ih;
    } else if (set == 4 || set == 6) {
        // W earlier than V: V's entries with t <= t_w + delta
        const uint32_t u = upper_time(g.T, V.lo, V.hi, g.T[w] + g.delta);
        il = ins(g.X, V.lo, u);
        ol = (u - V.lo) - il;
    } else {
        // W later than V: V's entries with t >= t_w - delta
        const uint32_t l = lower_time(g.T, V.lo, V.hi, g.T[w] - g.delta);
        il = ins(g.X, l, V.hi);
        ol = (V.hi - l) - il;
    }
    switch (set) {
        case 0: add_rank<3, 2, 1, 0, 4, 6, 5, 7>(acc, b, il, ol, ih, oh); break;          // x in As
        case 1: add_rank<7, 6, 5, 4, 0, 2, 1, 3>(acc, b, il, ol, ih, oh); break;          // y in Ad
        case 2: add_rank<22, 20, 18, 16, 17, 21, 19, 23>(acc, b, il, ol, ih, oh); break;  // x in Bs
        case 3: add_rank<23, 21, 19, 17, 16, 20, 18, 22>(acc, b, il, ol, ih, oh); break;  // y in Bd
        case 4: sel_add<10, 14>(acc, b, il); sel_add<11, 15>(acc, b, ol); break;          // x in Bs
        case 5: sel_add<15, 14>(acc, b, il); sel_add<11, 10>(acc, b, ol); break;          // y in Ad
        case 6: sel_add<8, 12>(acc, b, il); sel_add<9, 13>(acc, b, ol); break;            // y in Bd
        default: sel_add<13, 12>(acc, b, il); sel_add<9, 8>(acc, b, ol); break;           // x in As
    }
}

__global__ void __launch_bounds__(kBlock) k_path_items(PathArgs g, const uint4 *sz,
                                                       const uint64_t *io, const uint32_t *ce,
                                                       uint64_t n_items, uint64_t n_chunks,
                                                       uint64_t *rows) {
    __shared__ uint64_t red[kBlock / kWave][24];
    uint64_t acc[24];
#pragma unroll
    for (int i = 0; i < 24; i++) acc[i] = 0;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (uint64_t)gridDim.x * (kBlock / kWave);
    for (uint64_t c = (uint64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; c < n_chunks;
         c += waves) {
        const uint64_t item = c * kWave + lane;
        if (item >= n_items) continue;
        // the item's edge: the largest r in [ce[c], ce[c + 1]] with io[r] <= item
        uint64_t lo = ce[c], hi = (uint64_t)ce[c + 1] + 1;
        while (hi - lo > 1) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (io[mid] <= item) lo = mid;
            else hi = mid;
        }
        path_item(g, sz, lo, item - io[lo], acc);
    }
    block_rows<24>(acc, red, rows + (uint64_t)blockIdx.x * 24);
}

// out[c] = sum of rows[i * ncol + c] over i < nrow; one block per column.
__global__ void __launch_bounds__(kBlock) k_sum_rows(const uint64_t *rows, uint32_t nrow,
                                                     uint32_t ncol, uint64_t *out) {
    __shared__ uint64_t red[kBlock / kWave][1];
    uint64_t acc[1] = {0};
    for (uint32_t i = threadIdx.x; i < nrow; i += kBlock) acc[0] += rows[(uint64_t)i * ncol + blockIdx.x];
    block_rows<1>(acc, red, out + blockIdx.x);
}

// -------------------------------------------------- the correction tables
// Direction convention of the paper's raw counters: 0 = the edge leaves the
// node it is seen from (o), 1 = it enters it.
struct E3 {
    int s, d;  // endpoints; edges are listed in chronological order
};

// The path counters the kernel's enumeration adds for one three-edge
// instance: every middle edge e, x != e at src(e), y != e, x at dst(e),
// classified with the rules of path_item.
void path_choices(const E3 (&ed)[3], uint64_t (&h)[24]) {
    for (int e = 0; e < 3; e++) {
        const int s = ed[e].s, d = ed[e].d;
        for (int x = 0; x < 3; x++) {
            if (x == e || (ed[x].s != s && ed[x].d != s)) continue;
            const int dx = ed[x].d == s ? 1 : 0;
            for (int y = 0; y < 3; y++) {
                if (y == e || y == x || (ed[y].s != d && ed[y].d != d)) continue;
                const int dy = ed[y].d == d ? 1 : 0;
                int k;
                if (x > e && y > e)
                    k = x < y ? 4 + 2 * dx + (1 - dy) : 2 * dy + (1 - dx);
                else if (x < e && y < e)
                    k = x < y ? 16 + 4 * dx + 2 * (1 - dy) + 1 : 16 + 4 * dy + 2 * (1 - dx);
                else if (x < e)
                    k = 8 + 4 * dx + 2 + (1 - dy);
                else
                    k = 8 + 4 * dy + (1 - dx);
                h[k] += 1;
            }
        }
    }
}

struct Tables {
    uint64_t star[24][24];  // per raw Star[type][d1][d2][d3] cell
    uint64_t pair[4][24];   // per pair class (d2, d3), seen from src(E1)
    uint64_t tri[8][24];    // per triangle class [a][b][c], seen from the node not on E1
};

const Tables &tables() {
    static Tables t;
    static std::once_flag once;
    std::call_once(once, [] {
        std::memset(&t, 0, sizeof(t));
        // star: center 0, leaf 1 on two edges, leaf 2 on the edge at position ty
        for (int ty = 0; ty < 3; ty++)
            for (int c = 0; c < 8; c++) {
                E3 ed[3];
                for (int k = 0; k < 3; k++) {
                    const int dir = (c >> (2 - k)) & 1;
                    const int leaf = k == ty ? 2 : 1;
                    ed[k] = dir == 0 ? E3{0, leaf} : E3{leaf, 0};
                }
                path_choices(ed, t.star[ty * 8 + c]);
            }
        // pair: nodes 0, 1; E1 leaves 0
        for (int c = 0; c < 4; c++) {
            E3 ed[3] = {E3{0, 1}, ((c >> 1) & 1) ? E3{1, 0} : E3{0, 1}, (c & 1) ? E3{1, 0} : E3{0, 1}};
            path_choices(ed, t.pair[c]);
        }
        // triangle seen from x = 0 (not on E1): E2 = {0, 1} (dir a at 0),
        // E3 = {0, 2} (dir b at 0), E1 = {1, 2} (dir c at 1 = E2's other node)
        for (int c = 0; c < 8; c++) {
            const int a = (c >> 2) & 1, b = (c >> 1) & 1, k = c & 1;
            E3 ed[3] = {k == 0 ? E3{1, 2} : E3{2, 1}, a == 0 ? E3{0, 1} : E3{1, 0},
                        b == 0 ? E3{0, 2} : E3{2, 0}};
            path_choices(ed, t.tri[c]);
        }
    });
    return t;
}

}  // namespace

int count4_graph(tm_graph *g, int64_t delta, uint64_t *raw56, uint64_t *out32) {
    if (g->G != 1) {
        set_error("four-node motifs are counted on a single graph, not a batch");
        return TM_EINVAL;
    }
    Params pr;
    int rc = count_graph(g, &delta, pr, raw56, false);
    if (rc) return rc;
    uint64_t sums[32] = {0};
    const uint64_t len = 2 * g->m;
    if (g->m >= 3) {
        hipStream_t s = g->stream;
        const uint64_t m = g->m;
        const uint32_t npq = (uint32_t)(len / kQTile + 1);  // tiles covering [0, len]
        const uint32_t npc = (uint32_t)(m / kQTile + 1);    // tiles covering [0, m]
        const uint32_t gs = (uint32_t)std::min<uint64_t>(kStarGrid, (len + kBlock - 1) / kBlock);
        const uint32_t gp = (uint32_t)std::min<uint64_t>(kPathGrid, (m + kBlock - 1) / kBlock);
        auto rnd = [](size_t b) { return (b + 255) & ~size_t(255); };
        const size_t bytes = rnd((len + 1) * 8) + rnd((size_t)(std::max(npq, npc) + 1) * 8) +
                             rnd((size_t)gs * 64) + rnd((size_t)kPathGrid * 192) + rnd(32 * 8) +
                             rnd(m * 16) + rnd((m + 1) * 8) + rnd(len * 8);
        Scratch sc;
        rc = sc.reserve(bytes, s);
        if (rc) return rc;
        uint64_t *Q = sc.take<uint64_t>(len + 1);
        uint64_t *part = sc.take<uint64_t>(std::max(npq, npc) + 1);
        uint64_t *srows = sc.take<uint64_t>((size_t)gs * 8);
        uint64_t *prows = sc.take<uint64_t>((size_t)kPathGrid * 24);
        uint64_t *dsum = sc.take<uint64_t>(32);
        uint4 *sz = sc.take<uint4>(m);
        uint64_t *io = sc.take<uint64_t>(m + 1);
        uint2 *wfb = sc.take<uint2>(len);
        if (!Q || !part || !srows || !prows || !dsum || !sz || !io || !wfb) {
            set_error("four-node workspace carve");
            return TM_EINTERNAL;
        }
        ProfRow row("f4");
        // stars
        const QLoad ql{g->ent_nd, g->X};
        TM_LAUNCH("q_tile_sum", k_u64_tile_sum<QLoad>, dim3(npq), dim3(kBlock), 0, s, ql, len, part);
        TM_LAUNCH("q_parts", k_u64_parts, dim3(1), dim3(kPartsBlock), 0, s, part, npq);
        TM_LAUNCH("q_tile_scan", k_u64_tile_scan<QLoad>, dim3(npq), dim3(kBlock), 0, s, ql, len, part, Q);
        TM_LAUNCH("star4", k_star4, dim3(gs), dim3(kBlock), 0, s, g->ent_t, g->ent_nd, g->ent_c,
                  g->off, g->X, Q, len, delta, srows, wfb);
        TM_LAUNCH("sum_rows", k_sum_rows, dim3(8), dim3(kBlock), 0, s, srows, gs, 8u, dsum);
        // paths: window sizes, item numbering, items
        const PathArgs pa{g->ent_t, g->ent_nd, g->ent_r, g->ent_c, g->X, g->off, g->epos, m, delta};
        TM_LAUNCH("path_prep", k_path_prep, dim3(gp), dim3(kBlock), 0, s, g->epos, wfb, m, sz);
        const CostLoad cl{sz};
        TM_LAUNCH("cost_tile_sum", k_u64_tile_sum<CostLoad>, dim3(npc), dim3(kBlock), 0, s, cl, m, part);
        TM_LAUNCH("cost_parts", k_u64_parts, dim3(1), dim3(kPartsBlock), 0, s, part, npc);
        TM_LAUNCH("cost_tile_scan", k_u64_tile_scan<CostLoad>, dim3(npc), dim3(kBlock), 0, s, cl, m,
                  part, io);
        uint64_t n_items = 0;
        TM_HIP_TRY(hipMemcpyAsync(&n_items, io + m, 8, hipMemcpyDeviceToHost, s));
        TM_HIP_TRY(hipStreamSynchronize(s));
        uint32_t gi = 1;
        if (n_items) {
            const uint64_t n_chunks = (n_items + kWave - 1) / kWave;
            Scratch sc2;
            rc = sc2.reserve(rnd((n_chunks + 1) * 4), s);
            if (rc) return rc;
            uint32_t *ce = sc2.take<uint32_t>(n_chunks + 1);
            if (!ce) {
                set_error("four-node workspace carve");
                return TM_EINTERNAL;
            }
            TM_LAUNCH("chunk_edges", k_chunk_edges,
                      dim3((unsigned)std::min<uint64_t>(16384, n_chunks / kBlock + 1)), dim3(kBlock), 0,
                      s, io, m, n_items, n_chunks, ce);
            gi = (uint32_t)std::min<uint64_t>(kPathGrid, n_chunks / (kBlock / kWave) + 1);
            TM_LAUNCH("path_items", k_path_items, dim3(gi), dim3(kBlock), 0, s, pa, sz, io, ce, n_items,
                      n_chunks, prows);
            TM_LAUNCH("sum_rows", k_sum_rows, dim3(24), dim3(kBlock), 0, s, prows, gi, 24u, dsum + 8);
        } else {
            TM_HIP_TRY(hipMemsetAsync(dsum + 8, 0, 24 * 8, s));
        }
        TM_HIP_TRY(hipMemcpyAsync(sums, dsum, sizeof(sums), hipMemcpyDeviceToHost, s));
        TM_HIP_TRY(hipStreamSynchronize(s));
    }
    // corrections by the three-edge counts (raw layout of tm.h)
    const Tables &tb = tables();
    uint64_t sub[32] = {0};
    for (int c = 0; c < 8; c++) sub[c] = raw56[c] + raw56[8 + c] + raw56[16 + c] + raw56[24 + c];
    for (int cell = 0; cell < 24; cell++)
        for (int k = 0; k < 24; k++) sub[8 + k] += raw56[cell] * tb.star[cell][k];
    for (int c = 0; c < 4; c++)
        for (int k = 0; k < 24; k++) sub[8 + k] += raw56[24 + c] * tb.pair[c][k];
    for (int c = 0; c < 8; c++)
        for (int k = 0; k < 24; k++) sub[8 + k] += raw56[32 + c] * tb.tri[c][k];
    for (int k = 0; k < 32; k++) {
        if (sub[k] > sums[k]) {
            set_error("four-node counts: a correction exceeds its sum (internal inconsistency)");
            return TM_EINTERNAL;
        }
        out32[k] = sums[k] - sub[k];
    }
    return TM_OK;
}

}  // namespace tmc
