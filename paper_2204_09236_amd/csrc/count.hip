// Counting kernels for one window delta.
//
// Star and pair motifs (the paper's FAST-Star, Section IV-A / Algorithm 1).
// Algorithm 1 scans, for every first edge e1 of S_u, all third edges e3 inside
// delta and reads per-neighbour counts of the edges in between.  Summed over
// e3, its four counter updates are sums over the window W = (i, R(i)] of S_u
// (R(i) = last position with t <= t_i + delta) that only involve the edges to
// e1's own neighbour v -- the node-pair edge set E_(u,v) -- plus prefix counts
// of directions along S_u.  With P_d(x) = number of dir-d entries of S_u at
// positions <= x, and, over the E_(u,v) edges inside W:
//   in[d]      = how many have dir d
//   S2[d][d']  = ordered pairs k < j of them with dirs (d, d')
//   sPm[d'][d] = sum over those with dir d' of P_d(position - 1)
// the contributions of e1 = i (dir d_i) are, for all d, d':
//   Pair    [d_i][d][d'] += S2[d][d']
//   Star_II [d_i][d][d'] += sPm[d'][d] - in[d'] * P_d(i) - S2[d][d']
//   Star_III[d_i][d][d'] += in[d] * P_d'(R) - (sPm[d][d'] + [d = d'] in[d]) - S2[d][d']
// Star_I (e2 and e3 share the neighbour w != v) is the time mirror of Star_III
// and is summed per third edge j instead, over the window [L(j), j) with
// L(j) = first position with t >= t_j - delta, using the E_(u,w) edges there:
//   Star_I[d1][d2][d_j] += sPm'[d2][d1] - in'[d2] * P_d1(L - 1) - S2'[d1][d2]
// Each edge of E_(u,v) enters and leaves these windows once (two pointers), so
// a node pair's work is linear in its edge count.  Only node pairs with at
// least two edges contribute (all four sums vanish otherwise), and every such
// pair is swept from both of its nodes.  Long pairs are cut into chunks that
// each own a range of e1 (or e3) positions and first load the delta-window
// that reaches into the chunk (hub splitting); every instance is counted by
// the one chunk that owns its first (or, for Star_I, its last) edge.
//
// Triangle motifs (FAST-Tri, Section IV-B / Algorithm 2).  Every triangle
// instance is counted once, by its earliest edge E1 = (s -> d): E2 and E3 are
// the edges to the third node r inside the windows after E1 at s and at d, so
// the instances owned by E1 are the pairs (a in W_s, b in W_d) with equal
// neighbour r.  The class is the Type-I view at r (the vertex not on E1):
//   a before b: Tri[I][not dir_s(a)][not dir_d(b)][o]
//   b before a: Tri[I][not dir_d(b)][not dir_s(a)][in]
// The paper's center-based counter Tri[3][2][2][2] counts each instance once
// per vertex; its three views follow from the class exactly (orbit map in the
// host merge), so no instance is enumerated three times.
//
// Per-lane uint64 accumulators are reduced per block, then all block partials
// are summed by one deterministic tree reduction (no atomics on counts).
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "tm_internal.h"

namespace tmc {

namespace {

struct SeqView {
    const int64_t *t;      // ent_t
    const uint32_t *nd;    // ent_nd
    const uint32_t *rk;    // ent_r
    const uint32_t *c;     // ent_c
    const uint32_t *X;     // exclusive prefix of dir = in
    const uint32_t *off;
    const uint32_t *epos;
};

// Largest x in [p, hi) with t[x] <= lim, given t[p] <= lim (gallop, then bisect).
__device__ inline uint32_t window_end(const int64_t *T, uint32_t p, uint32_t hi, int64_t lim) {
    uint32_t lo = p, top = hi;
    uint64_t step = 1;
    while (true) {
        const uint64_t probe = (uint64_t)lo + step;
        if (probe >= hi) {
            top = hi;
            break;
        }
        if (T[probe] <= lim) {
            lo = (uint32_t)probe;
            step <<= 1;
        } else {
            top = (uint32_t)probe;
            break;
        }
    }
    while (top - lo > 1) {
        const uint32_t mid = lo + (top - lo) / 2;
        if (T[mid] <= lim) lo = mid;
        else top = mid;
    }
    return lo;
}

// Order this wave's LDS writes before its later LDS reads (all lanes).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ------------------------------------------------------------ window sizes
// Wf[p] = R(p) - p: how many later entries of the same S_u lie within delta
// (the delta of the graph the entry belongs to; tiles never straddle graphs).
// A wave takes 64 consecutive entries at a time and keeps the (center, t)
// keys of those and of the next 64 in a 128-slot ring in its LDS, refilled
// 64 keys per step from coalesced loads issued one step ahead.  Entries are
// sorted by (center, t), so "key <= (c_p, t_p + delta)" holds on a prefix of
// the entries after p: each lane finds the end of that prefix by binary
// search over the ring (one 16-byte LDS read per step), and only a window
// that runs past the 128 keys continues with a gallop in global memory.
// With `bits` non-null (one graph: tiles and wave spans start at multiples
// of 64, so each step covers one 64-entry word) the step also writes the
// window bit planes that k_wlevels would write.
//
// With `recR` / `recL` non-null (stars or pairs are counted) it also
// writes, per entry p, what the star/pair sweeps need about p's window in
// S_u: recR[p] = (W(p), number of dir-in entries in [p, R(p)]) and recL[p]
// = (p - L(p), number of dir-in entries in [L(p), p)), where L(p) = the
// first entry of S_u with t >= t_p - delta.  A record is written only when
// its window is not empty: the sweeps read it only for an element with
// another edge of its pair inside that window.  R(q) = q + Wf[q] never
// decreases along the whole array and never leaves q's S_u, so L(p) =
// min{q : R(q) >= p}: the entries p in (R(q - 1), R(q)] start their windows
// at q.  A step owns the entries in (R(base - 1), R(base + 63)]; its lanes
// write them in coalesced rounds of 64, each finding its q by bisection over
// the step's 64 window ends kept in LDS.  A wave span finds R of the entry
// before it with one gallop.  The direction prefix X is read next to p, R
// and L, which the wave walks in order, so these reads stay in cache; the
// sweeps then read one record per element instead of gathering X around
// each element's position.
//
// Several windows at once (K nested deltas, ascending; one graph): every step
// searches the same ring once per window, each search starting where the
// previous (smaller) window ended, and writes Wf of window i at i * len + p
// and its records at recR / recL[2 (i * len + p)] (level-major, the two
// records of an entry side by side: a window's stores cover whole lines
// together, and the sweeps find both records of an entry in one line).
// The bit planes describe the largest window.
constexpr uint32_t kRing = 2 * kWave;
constexpr uint32_t kHubCap = 2048;  // window entries per LDS segment of the hub pass
constexpr int kMaxLevels = 4;       // windows counted in one pass

template <int K>
__global__ void __launch_bounds__(kBlock) k_windows(SeqView S, const Tile *tiles, uint32_t n_tiles,
                                                    uint64_t len, const int64_t *deltas,
                                                    uint32_t *Wf, uint32_t hub_min, uint64_t *planes,
                                                    uint2 *recR, uint2 *recL) {
    // key j of the ring: (center, unused, t low, t high)
    __shared__ uint4 ring[kBlock / kWave][kRing];
    __shared__ uint32_t rend[kBlock / kWave][kWave];  // the step's window ends R
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    uint4 *rg = ring[wv];
    auto key_at = [&](uint64_t q) -> uint4 {
        if (q >= len) return make_uint4(0xffffffffu, 0u, 0u, 0u);  // matches no center
        const uint64_t t = (uint64_t)S.t[q];
        return make_uint4(S.c[q], 0u, (uint32_t)t, (uint32_t)(t >> 32));
    };
    for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
        const Tile tl = tiles[ti];
        int64_t delta[K];
#pragma unroll
        for (int i = 0; i < K; i++) delta[i] = deltas[(uint64_t)tl.g * K + i];
        // each wave walks its own contiguous span of the tile in steps of 64
        const uint32_t span = ((tl.e - tl.b + nw - 1) / nw + kWave - 1) / kWave * kWave;
        const uint32_t w_b = tl.b + wv * span, w_e = min(tl.e, w_b + span);
        if (w_b >= w_e) continue;
        // first entry whose window start this wave writes: R(w_b - 1) + 1
        uint32_t p_next[K];
#pragma unroll
        for (int i = 0; i < K; i++) {
            p_next[i] = w_b;
            if (recL && w_b > 0) {
                const uint32_t q0 = w_b - 1, c0 = S.c[q0];
                if (c0 == S.c[w_b])
                    p_next[i] = window_end(S.t, q0, S.off[c0 + 1], S.t[q0] + delta[i]) + 1;
            }
        }
        rg[lane] = key_at((uint64_t)w_b + lane);
        uint4 next = key_at((uint64_t)w_b + kWave + lane);
        uint32_t half = 0;  // ring half holding the current 64 keys
        for (uint32_t base = w_b; base < w_e; base += kWave) {
            rg[(half ^ 1) * kWave + lane] = next;
            next = key_at((uint64_t)base + 2 * kWave + lane);  // in flight during the search
            wave_lds_sync();
            const uint4 me = rg[half * kWave + lane];
            const uint32_t ca = me.x;
            const int64_t tme = (int64_t)(((uint64_t)me.w << 32) | me.z);
            const uint64_t qa = (uint64_t)base + lane;
            const uint32_t xq = recR && qa < w_e ? S.X[qa] : 0u;
            uint32_t Wtop = 0;
            uint32_t lo = (uint32_t)lane;  // a window contains the previous (smaller) one
#pragma unroll
            for (int i = 0; i < K; i++) {
                const int64_t lim = tme + delta[i];
                // last k in [lo, 128) with key(base + k) <= (ca, lim)
                uint32_t hi = kRing;
#pragma unroll
                for (int step = 0; step < 7; step++) {
                    const uint32_t mid = (lo + hi) / 2;
                    const uint4 km = rg[(half * kWave + mid) & (kRing - 1)];
                    const int64_t tm = (int64_t)(((uint64_t)km.w << 32) | km.z);
                    const bool ok = km.x < ca || (km.x == ca && tm <= lim);
                    if (hi - lo > 1) {
                        if (ok) lo = mid;
                        else hi = mid;
                    }
                }
                uint32_t W = 0, Rq = 0;
                if (qa < w_e) {
                    uint64_t R = (uint64_t)base + lo;
                    if (lo == kRing - 1)  // the window may run past the ring
                        R = window_end(S.t, (uint32_t)R, S.off[ca + 1], lim);
                    W = (uint32_t)(R - qa);
                    Wf[i * len + qa] = W;
                    Rq = (uint32_t)R;
                    // only read for a non-empty window
                    if (recR && W) recR[2 * (i * len + qa)] = make_uint2(W, S.X[R + 1] - xq);
                }
                if (i == K - 1) Wtop = W;
                if (recL) {
                    const uint32_t nvalid = min<uint32_t>(kWave, w_e - base);
                    const uint32_t r_last = __shfl(Rq, (int)nvalid - 1, kWave);
                    wave_lds_sync();  // the previous window's reads of rend are done
                    // lanes past the span own no entries
                    rend[wv][lane] = qa < w_e ? Rq : r_last;
                    wave_lds_sync();
                    for (uint32_t p0 = p_next[i]; p0 <= r_last; p0 += kWave) {
                        const uint32_t p = p0 + (uint32_t)lane;
                        if (p <= r_last) {
                            // first step entry j with R >= p (R of entry nvalid - 1 is r_last >= p)
                            uint32_t a = 0, b = nvalid - 1;
                            while (a < b) {
                                const uint32_t mid = (a + b) / 2;
                                if (rend[wv][mid] >= p) b = mid;
                                else a = mid + 1;
                            }
                            const uint32_t L = base + a;
                            // only read for a non-empty window
                            if (L < p) recL[2 * (i * len + p)] = make_uint2(p - L, S.X[p] - S.X[L]);
                        }
                    }
                    p_next[i] = r_last + 1;
                }
            }
            if (planes) {
                const uint32_t t2 = min(hub_min, kHubCap), t3 = max(hub_min, kHubCap);
                const uint64_t b = __ballot(Wtop != 0);
                const uint64_t b2 = __ballot(Wtop >= t2);
                const uint64_t b3 = __ballot(Wtop >= t3);
                if (lane == 0) {
                    uint64_t *pw = planes + 3 * (uint64_t)(base / kWave);
                    pw[0] = b;
                    pw[1] = b2;
                    pw[2] = b3;
                }
            }
            wave_lds_sync();  // the next step overwrites this half
            half ^= 1;
        }
    }
}

// --------------------------------------------------------------- star/pair
// Alg. 1 counts, for every edge e of S_c, the ordered pairs of later edges
// inside delta by their node pairs and directions.  Here the instances with
// two or three edges on one node pair are counted from the pair's side: per
// element q (an edge of a node pair with >= 2 edges) and side (center c =
// smaller / larger node), the other edges of its pair inside q's forward
// window (q, j) give the Pair, Star_II and Star_III instances whose first
// edge is q, and those inside its backward window [f, q) give the Star_I
// instances whose last edge is q.  Besides the window's own edges each needs
// the prefix counts P_0, P_1 of S_c at q's window end R (forward) or just
// before its window start L (backward), which k_windows records per entry.
//
// Window state over edges of one node pair.
struct Win {
    uint64_t in[2];
    uint64_t S2[2][2];   // S2[d][d']: ordered pairs k < j, dir k = d, dir j = d'
    uint64_t sPm[2][2];  // sPm[d'][e]: sum over dir-d' edges of P_e(position - 1)
    __device__ inline void clear() {
        in[0] = in[1] = 0;
        S2[0][0] = S2[0][1] = S2[1][0] = S2[1][1] = 0;
        sPm[0][0] = sPm[0][1] = sPm[1][0] = sPm[1][1] = 0;
    }
    // append a later edge (dir d, prefix counts a0, a1)
    __device__ inline void push(uint32_t d, uint32_t a0, uint32_t a1) {
        const uint64_t m1 = 0ull - (uint64_t)d, m0 = ~m1;
        S2[0][0] += in[0] & m0;
        S2[1][0] += in[1] & m0;
        S2[0][1] += in[0] & m1;
        S2[1][1] += in[1] & m1;
        in[0] += 1 & m0;
        in[1] += 1 & m1;
        sPm[0][0] += a0 & m0;
        sPm[0][1] += a1 & m0;
        sPm[1][0] += a0 & m1;
        sPm[1][1] += a1 & m1;
    }
    // prepend an earlier edge (dir d, prefix counts a0, a1)
    __device__ inline void push_front(uint32_t d, uint32_t a0, uint32_t a1) {
        const uint64_t m1 = 0ull - (uint64_t)d, m0 = ~m1;
        S2[0][0] += in[0] & m0;
        S2[0][1] += in[1] & m0;
        S2[1][0] += in[0] & m1;
        S2[1][1] += in[1] & m1;
        in[0] += 1 & m0;
        in[1] += 1 & m1;
        sPm[0][0] += a0 & m0;
        sPm[0][1] += a1 & m0;
        sPm[1][0] += a0 & m1;
        sPm[1][1] += a1 & m1;
    }
};

__device__ inline void add_sel(uint64_t &lo_cell, uint64_t &hi_cell, uint64_t v, uint64_t m1) {
    lo_cell += v & ~m1;
    hi_cell += v & m1;
}

// One element of a pair seen from one side: direction relative to the
// center and the prefix counts (#o, #in) of S_c before its entry.
struct El {
    uint32_t dir, a0, a1;
};
__device__ inline El elem(uint8_t o, uint4 a, uint32_t side) {
    El e;
    e.dir = 1u - ((o & 1u) ^ side);  // side 0: center = smaller node
    e.a0 = side ? a.z : a.x;
    e.a1 = side ? a.w : a.y;
    return e;
}

struct StarArgs {
    const uint32_t *mp_start;
    const int64_t *me_t;
    const uint8_t *me_o;     // bit 0: leaves the smaller node; bit 1: first of its pair
    const uint4 *me_a;
    const uint2 *me_p;       // element positions in S_lo, S_hi
    const uint2 *recR, *recL;  // window records of entry p: [2 (level * n_ent + p)]
    uint64_t n_ent;          // entries of S (2m)
    uint32_t K;              // windows of the pass; each tile runs all of them
    uint64_t part_stride;    // partial rows of window i start at partial + i * part_stride
    const uint32_t *mpb;     // G + 1: multi-edge pair bounds per graph
    const uint32_t *tfirst;  // G + 1: first element tile of each graph
    uint32_t G;
    const int64_t *deltas;   // K == 1: per graph; K > 1 (one graph): per window
    uint32_t per;            // elements per thread; a tile holds per * kBlock elements
    int star_i;              // count Star_I (stars requested)
};

// Largest i in [0, n) with a[i] <= x, for ascending a with a[0] <= x.
__device__ inline uint32_t last_le(const uint32_t *a, uint32_t n, uint32_t x) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (a[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Sum a block's N counters per thread into row[c0, c0 + N): wave sums, then
// one thread per counter adds the waves.
template <int N>
__device__ inline void star_flush(const uint64_t (&acc)[N], int c0, uint64_t (*red)[32],
                                  uint64_t *row) {
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    __syncthreads();  // the previous flush has read red
#pragma unroll
    for (int i = 0; i < N; i++) {
        uint64_t v = acc[i];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
        if (lane == 0) red[wv][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        uint64_t s = 0;
#pragma unroll
        for (int q = 0; q < kBlock / kWave; q++) s += red[q][threadIdx.x];
        row[c0 + threadIdx.x] = s;
    }
}

// One block per element tile (per * kBlock consecutive elements of one
// graph, neighbouring lanes on neighbouring elements); one partial row of 32
// counters per tile and window.  Every element is independent: its windows
// hold only the few other edges of its pair inside delta, found by walking
// its neighbours in element order up to the pair's ends (bit 1 of me_o).
// The tile and kStageHalo elements on each side (time, flags, prefix counts)
// are first copied into LDS with coalesced loads, so those walks read LDS;
// elements outside the staged range are read from global memory, so the
// result does not depend on the staging.  The windows of a pass are counted
// one after another on the staged tile, so an entry's records (side by side
// for all windows) are read again while their line is still cached.
constexpr uint32_t kStageHalo = 64;
constexpr uint32_t kStageCap = 2048;  // 51 KiB of LDS: three blocks per CU

struct ElemView {
    uint32_t lo, hi;  // staged element range
    const int64_t *st;
    const uint8_t *so;
    const uint4 *sa;
    const int64_t *gt;
    const uint8_t *go;
    const uint4 *ga;
    __device__ inline bool staged(uint32_t k) const { return k - lo < hi - lo; }
    __device__ inline int64_t t(uint32_t k) const { return staged(k) ? st[k - lo] : gt[k]; }
    __device__ inline uint8_t o(uint32_t k) const { return staged(k) ? so[k - lo] : go[k]; }
    __device__ inline uint4 a(uint32_t k) const { return staged(k) ? sa[k - lo] : ga[k]; }
};

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_star_pair(StarArgs a, uint64_t *partial) {
  __shared__ int64_t s_t[kStageCap];
  __shared__ uint4 s_a[kStageCap];
  __shared__ uint8_t s_o[kStageCap];
  __shared__ uint64_t red[kBlock / kWave][32];
  const uint32_t n_tiles = a.tfirst[a.G];
  const uint32_t tile = a.per * kBlock;
  for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
    const uint32_t gi = last_le(a.tfirst, a.G + 1, ti);
    const uint32_t gb = a.mp_start[a.mpb[gi]], ge = a.mp_start[a.mpb[gi + 1]];
    const uint32_t eb = gb + (ti - a.tfirst[gi]) * tile;
    const uint32_t ee = min(ge, eb + tile);
    const uint32_t lo = eb - min(eb - gb, kStageHalo);
    const uint32_t hi = min(min(ge, ee + kStageHalo), lo + kStageCap);
    __syncthreads();  // the previous tile is done with the stage
    for (uint32_t k = lo + threadIdx.x; k < hi; k += kBlock) {
        s_t[k - lo] = a.me_t[k];
        s_o[k - lo] = a.me_o[k];
        s_a[k - lo] = a.me_a[k];
    }
    __syncthreads();
    const ElemView V{lo, hi, s_t, s_o, s_a, a.me_t, a.me_o, a.me_a};
    for (uint32_t level = 0; level < a.K; level++) {
      const int64_t delta = a.deltas[gi + level];
      uint64_t *row = partial + level * a.part_stride + (uint64_t)ti * 32;
      {
        // ---- phase 1: Pair, Star_II, Star_III with first edge q (cell c -> A[c - 8])
        uint64_t A[24];
#pragma unroll
        for (int i = 0; i < 24; i++) A[i] = 0;
        for (uint32_t u = 0; u < a.per; u++) {
          const uint32_t q = eb + threadIdx.x + u * kBlock;
          if (q >= ee) break;
          const int64_t tq = V.t(q);
          // the pair's other edges inside q's forward window (q, jf)
          uint32_t jf = q + 1;
          while (jf < ge && !(V.o(jf) & 2u) && V.t(jf) <= tq + delta) jf++;
          if (jf == q + 1) continue;
          const uint8_t oq = V.o(q);
          const uint4 aq = V.a(q);
          const uint2 pq = a.me_p[q];
          for (uint32_t side = 0; side < 2; side++) {
            const El eq = elem(oq, aq, side);
            const uint64_t m1 = 0ull - (uint64_t)eq.dir;
            Win W;
            W.clear();
            for (uint32_t j = q + 1; j < jf; j++) {
                const El ej = elem(V.o(j), V.a(j), side);
                W.push(ej.dir, ej.a0, ej.a1);
            }
            // P_0, P_1 of S_c at q's window end R from q's record: with
            // (a0, a1) the counts before q, P_1(R) = a1 + dir-in entries in
            // [q, R], P_0(R) = entries up to R - P_1(R)
            const uint2 r = a.recR[2 * (level * a.n_ent + (side ? pq.y : pq.x))];
            const uint32_t p1 = eq.a1 + r.y;
            const uint64_t rp[2] = {(uint64_t)(eq.a0 + eq.a1 + r.x + 1 - p1), (uint64_t)p1};
            const uint64_t pin[2] = {(uint64_t)eq.a0 + (eq.dir == 0), (uint64_t)eq.a1 + (eq.dir == 1)};
#pragma unroll
            for (int d = 0; d < 2; d++) {
#pragma unroll
                for (int dp = 0; dp < 2; dp++) {
                    const uint64_t s2 = W.S2[d][dp];
                    // Pair[d_q][d][d']
                    add_sel(A[16 + d * 2 + dp], A[20 + d * 2 + dp], s2, m1);
                    // Star_II[d_q][d][d']
                    const uint64_t v2 = W.sPm[dp][d] - W.in[dp] * pin[d] - s2;
                    add_sel(A[0 + d * 2 + dp], A[4 + d * 2 + dp], v2, m1);
                    // Star_III[d_q][d][d']
                    const uint64_t sp = W.sPm[d][dp] + (d == dp ? W.in[d] : 0ull);
                    const uint64_t v3 = W.in[d] * rp[dp] - sp - s2;
                    add_sel(A[8 + d * 2 + dp], A[12 + d * 2 + dp], v3, m1);
                }
            }
          }
        }
        star_flush<24>(A, 8, red, row);
      }
      {
        // ---- phase 2: Star_I with last edge q (cells 0..7)
        uint64_t A[8];
#pragma unroll
        for (int i = 0; i < 8; i++) A[i] = 0;
        for (uint32_t u = 0; u < a.per && a.star_i; u++) {
          const uint32_t q = eb + threadIdx.x + u * kBlock;
          if (q >= ee) break;
          const int64_t tq = V.t(q);
          // the pair's other edges inside q's backward window [fb, q)
          uint32_t fb = q;
          while (fb > gb && !(V.o(fb) & 2u) && V.t(fb - 1) >= tq - delta) fb--;
          if (fb == q) continue;
          const uint8_t oq = V.o(q);
          const uint4 aq = V.a(q);
          const uint2 pq = a.me_p[q];
          for (uint32_t side = 0; side < 2; side++) {
            const El eq = elem(oq, aq, side);
            const uint64_t m1 = 0ull - (uint64_t)eq.dir;
            Win W;
            W.clear();
            for (uint32_t f = q; f > fb; f--) {
                const El ef = elem(V.o(f - 1), V.a(f - 1), side);
                W.push_front(ef.dir, ef.a0, ef.a1);
            }
            // P_0, P_1 of S_c just before q's window start L:
            // P_1(L - 1) = a1 - dir-in entries in [L, q), P_0 = L - start - P_1
            const uint2 r = a.recL[2 * (level * a.n_ent + (side ? pq.y : pq.x))];
            const uint32_t p1 = eq.a1 - r.y;
            const uint64_t lp[2] = {(uint64_t)(eq.a0 + eq.a1 - r.x - p1), (uint64_t)p1};
#pragma unroll
            for (int d1 = 0; d1 < 2; d1++) {
#pragma unroll
                for (int d2 = 0; d2 < 2; d2++) {
                    const uint64_t v1 = W.sPm[d2][d1] - W.in[d2] * lp[d1] - W.S2[d1][d2];
                    // Star_I[d1][d2][d3 = dir of q]
                    add_sel(A[d1 * 4 + d2 * 2 + 0], A[d1 * 4 + d2 * 2 + 1], v1, m1);
                }
            }
          }
        }
        star_flush<8>(A, 0, red, row);
      }
    }
  }
}

// ---------------------------------------------------------------- triangles
// Candidates whose larger window holds at least hub_min entries, and whose
// smaller one fewer than kHubCap, go to the slice kernel k_tri_hub below;
// the rest to the per-candidate kernel k_triangles.
constexpr uint32_t kHubSlice = 512;          // S positions per hub tile
constexpr uint32_t kHubBlock = 512;          // threads of a k_tri_hub block
constexpr uint32_t kHubPer = kHubSlice / kHubBlock;  // positions per thread
static_assert(kHubSlice % kHubBlock == 0, "hub slice");
constexpr uint32_t kHubSlots = 2 * kHubCap;  // hash slots (load factor <= 1/2)
constexpr uint32_t kHubBits = 12;            // log2(kHubSlots)
static_assert((1u << kHubBits) == kHubSlots, "hub table size");

// Window bit planes of the entries (largest window): for entries 64g ..
// 64g+63, planes[3g] holds W >= 1, planes[3g + 1] and planes[3g + 2] hold
// W >= t2 and W >= t3, where (t2, t3) are hub_min and kHubCap in increasing
// order.  The three words of a group lie side by side (3 len / 64 words in
// all, kept in cache), so an edge's candidate test at each of its two
// unrelated entries fetches one line, not one of Wf from HBM.
__global__ void k_wlevels(const uint32_t *Wf, uint64_t len, uint32_t hub_min, uint64_t *planes) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t t2 = min(hub_min, kHubCap), t3 = max(hub_min, kHubCap);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // the loop bound is rounded up to whole waves so every lane takes part in the ballots
    const uint64_t lim = (len + kWave - 1) / kWave * kWave;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < lim; p += stride) {
        const uint32_t w = p < len ? Wf[p] : 0u;
        const uint64_t b = __ballot(w != 0);
        const uint64_t b2 = __ballot(w >= t2);
        const uint64_t b3 = __ballot(w >= t3);
        if (lane == 0) {
            uint64_t *pw = planes + 3 * (p / kWave);
            pw[0] = b;
            pw[1] = b2;
            pw[2] = b3;
        }
    }
}

// W >= 1 at entry p
__device__ inline bool wbit(const uint64_t *planes, uint32_t p) {
    return (planes[3 * (uint64_t)(p / kWave)] >> (p % kWave)) & 1ull;
}

// (W >= 1, W >= t2, W >= t3) of entry p as bits 0, 1 and 2
__device__ inline uint32_t wplanes(const uint64_t *planes, uint32_t p) {
    const uint64_t *pw = planes + 3 * (uint64_t)(p / kWave);
    const uint32_t sh = p % kWave;
    return (uint32_t)((pw[0] >> sh) & 1ull) | ((uint32_t)((pw[1] >> sh) & 1ull) << 1) |
           ((uint32_t)((pw[2] >> sh) & 1ull) << 2);
}

// Bits of 64 entries (group g of the planes) with W >= hub_min.
__device__ inline uint64_t hub_word(const uint64_t *planes, uint64_t g, bool hub_first) {
    return planes[3 * g + (hub_first ? 1 : 2)];
}

// Candidate first edges for k_triangles: both windows after the edge (at its
// source and at its destination) hold at least one entry, and the edge is
// not one of k_tri_hub's (larger window >= hub_min, smaller < kHubCap).
__global__ void k_tri_flags(const uint2 *epos2, const uint64_t *planes, uint32_t hub_min,
                            uint64_t m, uint32_t *flag) {
    // bit of wplanes() that holds W >= hub_min, and the one with W >= kHubCap
    const uint32_t bh = hub_min <= kHubCap ? 2u : 4u, bc = hub_min <= kHubCap ? 4u : 2u;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint2 e = epos2[r];
        uint32_t f = 0;
        // the hub planes only for edges with both windows non-empty (their
        // words share the line of the first plane's)
        if (wbit(planes, e.x) && wbit(planes, e.y)) {
            const uint32_t ls = wplanes(planes, e.x), ld = wplanes(planes, e.y);
            const bool hub = ((ls | ld) & bh) && !(ls & ld & bc);
            f = hub ? 0u : 1u;
        }
        flag[r] = f;
    }
}

// Wf: the window sizes to record, entry p's at Wf[p * stride].
__global__ void k_tri_compact(const uint2 *epos2, const uint32_t *Wf, uint32_t stride,
                              const uint32_t *flag, const uint32_t *idx, uint64_t m, uint4 *cand) {
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m;
         r += (uint64_t)gridDim.x * blockDim.x) {
        if (!flag[r]) continue;
        const uint2 e = epos2[r];
        cand[idx[r]] = make_uint4(e.x, e.y, Wf[(uint64_t)e.x * stride], Wf[(uint64_t)e.y * stride]);
    }
}

// Triangle counters of one wave, in LDS: class (a, b, c) = Tri[I][a][b][c]
// of window level l at index 8 l + class.  Matches are rare next to the
// neighbour comparisons, so each adds to its counter with an LDS atomic
// instead of keeping 8 K accumulators live in every lane.
__device__ inline void tri_add(unsigned long long *cnt, uint32_t idx) { atomicAdd(&cnt[idx], 1ull); }

// class of a matched pair: a from W_s (dir relative to s), b from W_d
__device__ inline uint32_t tri_class(uint32_t ra, uint32_t da, uint32_t rb, uint32_t db) {
    return ra < rb ? ((1u - da) * 4 + (1u - db) * 2 + 0u) : ((1u - db) * 4 + (1u - da) * 2 + 1u);
}

// Window level of a matched instance when K nested windows are counted in
// one pass: the matching runs on the largest window, and the instance
// belongs to every window that holds both of its later edges, i.e. to the
// windows from index `level` up, where `level` = the number of smaller
// windows that miss one of them.  oa, ob: the later edges' offsets after
// the first edge's entries ps (at its source) and pd (at its destination);
// Wf holds the size of window i at entry p at i * len + p.  Matches are rare
// next to the comparisons, so the sizes are read here, on a match.
template <int K>
__device__ inline uint32_t tri_level(const uint32_t *Wf, uint64_t len, uint32_t ps, uint32_t oa,
                                     uint32_t pd, uint32_t ob) {
    uint32_t l = 0;
#pragma unroll
    for (int i = 0; i + 1 < K; i++)
        l += (oa > Wf[i * len + ps] || ob > Wf[i * len + pd]) ? 1u : 0u;
    return l;
}

// One block per candidate tile (kCandTile candidates of one graph); waves
// take 64 candidates at a time; one partial row of 8 counters per tile.
constexpr uint32_t kCandTile = 256;
constexpr uint32_t kTriRowsPerTile = kBlock / kWave;  // one partial row per wave
constexpr int kRegWin = 8;
// Wide candidates whose smaller window exceeds kHashMin entries are joined
// through an LDS hash table of at most 2 * kHashChunk slots per wave (load
// factor <= 1/2, so every probe sequence ends at an empty slot).
constexpr uint32_t kHashMin = 32;
constexpr uint32_t kHashChunk = 256;
constexpr uint32_t kEmptyKey = 0xffffffffu;  // node ids are below 2^31
constexpr uint32_t kHashMul = 2654435761u;   // Knuth's multiplicative constant

// K windows: the candidates and their windows are those of the largest one,
// each match is filed under its level (Wf: window i of entry p at i * len +
// p), and level l's rows go to partial + l * lvl_stride.
template <int K>
__global__ void __launch_bounds__(kBlock) k_triangles(SeqView S, const uint4 *cand,
                                                      const uint32_t *tidx, const uint32_t *eoff,
                                                      const uint32_t *ctfirst, uint32_t G,
                                                      uint32_t lane_max, const uint32_t *Wf,
                                                      uint64_t len, uint64_t lvl_stride,
                                                      uint64_t *partial) {
  const uint32_t n_tiles = ctfirst[G];
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t wv = threadIdx.x / kWave;
  __shared__ uint32_t hkey[kBlock / kWave][2 * kHashChunk];
  __shared__ uint32_t hval[kBlock / kWave][2 * kHashChunk];
  __shared__ unsigned long long tcnt[kBlock / kWave][8 * K];
  unsigned long long *T = tcnt[wv];
  for (uint32_t ti = blockIdx.x; ti < n_tiles; ti += gridDim.x) {
    const uint32_t gi = last_le(ctfirst, G + 1, ti);
    const uint32_t cb = tidx[eoff[gi]] + (ti - ctfirst[gi]) * kCandTile;
    const uint32_t ce = min(tidx[eoff[gi + 1]], cb + kCandTile);
    if (lane < 8 * K) T[lane] = 0;
    wave_lds_sync();
    for (uint32_t base = cb + wv * kWave; base < ce; base += kBlock) {
        const uint32_t ci = base + lane;
        uint32_t ps = 0, pd = 0, ws = 0, wd = 0;
        const bool active = ci < ce;
        if (active) {
            const uint4 c = cand[ci];
            ps = c.x;
            pd = c.y;
            ws = c.z;
            wd = c.w;
        }
        const bool small = active && (uint64_t)ws * wd <= lane_max;
        if (small) {
            // the smaller window, if it has at most kRegWin entries, is held in
            // registers and the larger one streamed once
            const bool s_reg = ws <= wd;
            const uint32_t rp = s_reg ? ps : pd, rw = s_reg ? ws : wd;
            const uint32_t lp = s_reg ? pd : ps, lw = s_reg ? wd : ws;
            if (rw <= kRegWin) {
                uint32_t rn[kRegWin], rr[kRegWin];
#pragma unroll
                for (int k = 0; k < kRegWin; k++) {
                    const bool v = (uint32_t)k < rw;
                    rn[k] = v ? S.nd[rp + 1 + k] : 0xffffffffu;  // matches no neighbour
                    rr[k] = v ? S.rk[rp + 1 + k] : 0u;
                }
                for (uint32_t b = lp + 1; b <= lp + lw; b++) {
                    const uint32_t ndb = S.nd[b];
#pragma unroll
                    for (int k = 0; k < kRegWin; k++) {
                        if ((rn[k] >> 1) == (ndb >> 1)) {
                            const uint32_t rb = S.rk[b];  // ranks only on a (rare) match
                            const uint32_t cls = s_reg ? tri_class(rr[k], rn[k] & 1u, rb, ndb & 1u)
                                                       : tri_class(rb, ndb & 1u, rr[k], rn[k] & 1u);
                            const uint32_t oreg = (uint32_t)k + 1, ostr = b - lp;
                            const uint32_t l = s_reg ? tri_level<K>(Wf, len, ps, oreg, pd, ostr)
                                                     : tri_level<K>(Wf, len, ps, ostr, pd, oreg);
                            tri_add(T, l * 8 + cls);
                        }
                    }
                }
            } else {
                for (uint32_t a = ps + 1; a <= ps + ws; a++) {
                    const uint32_t nda = S.nd[a];
                    for (uint32_t b = pd + 1; b <= pd + wd; b++) {
                        const uint32_t ndb = S.nd[b];
                        if ((ndb >> 1) == (nda >> 1)) {
                            const uint32_t cls = tri_class(S.rk[a], nda & 1u, S.rk[b], ndb & 1u);
                            tri_add(T, tri_level<K>(Wf, len, ps, a - ps, pd, b - pd) * 8 + cls);
                        }
                    }
                }
            }
        }
        // large windows: the whole wave takes one edge at a time
        uint64_t big = __ballot(active && !small);
        while (big) {
            const int L = __ffsll((unsigned long long)big) - 1;
            big &= big - 1;
            const uint32_t bps = __shfl(ps, L, kWave), bws = __shfl(ws, L, kWave);
            const uint32_t bpd = __shfl(pd, L, kWave), bwd = __shfl(wd, L, kWave);
            const bool s_outer = bws <= bwd;
            const uint32_t o_base = s_outer ? bps : bpd, i_base = s_outer ? bpd : bps;
            const uint32_t o_lo = o_base + 1, o_hi = s_outer ? bps + bws : bpd + bwd;
            const uint32_t i_lo = i_base + 1, i_hi = s_outer ? bpd + bwd : bps + bws;
            if (o_hi - o_lo + 1 > kHashMin) {
                // hash join: the smaller window, kHashChunk entries at a time,
                // goes into an open-addressing table in this wave's LDS (one
                // slot per entry, key = neighbour, value = its position);
                // every entry of the larger window probes it.  Work is linear in
                // the two windows plus the matches instead of their product.
                uint32_t *hk = hkey[wv], *hv = hval[wv];
                for (uint32_t cb = o_lo; cb <= o_hi; cb += kHashChunk) {
                    const uint32_t ce = min(o_hi, cb + kHashChunk - 1);
                    uint32_t hbits = 6;
                    while ((1u << hbits) < 2 * (ce - cb + 1)) hbits++;
                    const uint32_t hmask = (1u << hbits) - 1, hshift = 32 - hbits;
                    for (uint32_t q = lane; q <= hmask; q += kWave) hk[q] = kEmptyKey;
                    wave_lds_sync();
                    for (uint32_t y = cb + lane; y <= ce; y += kWave) {
                        const uint32_t nd = S.nd[y];
                        const uint32_t key = nd >> 1;
                        uint32_t h = (key * kHashMul) >> hshift;
                        while (atomicCAS(&hk[h], kEmptyKey, key) != kEmptyKey) h = (h + 1) & hmask;
                        hv[h] = y;  // its rank and direction are read on a match
                    }
                    wave_lds_sync();
                    for (uint32_t x = i_lo + lane; x <= i_hi; x += kWave) {
                        const uint32_t nd = S.nd[x];
                        const uint32_t key = nd >> 1;
                        for (uint32_t h = (key * kHashMul) >> hshift;; h = (h + 1) & hmask) {
                            const uint32_t k = hk[h];
                            if (k == kEmptyKey) break;
                            if (k == key) {
                                const uint32_t y = hv[h], rx = S.rk[x], ry = S.rk[y];
                                const uint32_t dy = S.nd[y] & 1u;
                                const uint32_t cls = s_outer ? tri_class(ry, dy, rx, nd & 1u)
                                                             : tri_class(rx, nd & 1u, ry, dy);
                                uint32_t l = 0;
                                if (K > 1) {
                                    const uint32_t oo = y - o_base, oi = x - i_base;
                                    l = s_outer ? tri_level<K>(Wf, len, bps, oo, bpd, oi)
                                                : tri_level<K>(Wf, len, bps, oi, bpd, oo);
                                }
                                tri_add(T, l * 8 + cls);
                            }
                        }
                    }
                    wave_lds_sync();
                }
                continue;
            }
            // both windows travel in 64-entry chunks, one coalesced load each;
            // the outer chunk's entries are broadcast from registers
            for (uint32_t ib = i_lo; ib <= i_hi; ib += kWave) {
                const uint32_t x = ib + lane;
                const bool valid = x <= i_hi;
                const uint32_t ndx = valid ? S.nd[x] : 0xffffffffu;
                for (uint32_t ob = o_lo; ob <= o_hi; ob += kWave) {
                    const uint32_t y = ob + lane;
                    const uint32_t ndy = y <= o_hi ? S.nd[y] : 0u;
                    const uint32_t cnt = min((uint32_t)kWave, o_hi - ob + 1);
                    for (uint32_t k = 0; k < cnt; k++) {
                        const uint32_t ndo = (uint32_t)__builtin_amdgcn_readlane((int)ndy, (int)k);
                        if (valid && (ndx >> 1) == (ndo >> 1)) {
                            // ranks are read on a (rare) match only
                            const uint32_t ro = S.rk[ob + k], rx = S.rk[x];
                            const uint32_t cls = s_outer ? tri_class(ro, ndo & 1u, rx, ndx & 1u)
                                                         : tri_class(rx, ndx & 1u, ro, ndo & 1u);
                            const uint32_t oo = ob + k - o_base, oi = x - i_base;
                            const uint32_t l = s_outer ? tri_level<K>(Wf, len, bps, oo, bpd, oi)
                                                       : tri_level<K>(Wf, len, bps, oi, bpd, oo);
                            tri_add(T, l * 8 + cls);
                        }
                    }
                }
            }
        }
    }
    // one row per wave and level (no block barrier: a wave with a wide hub
    // window does not hold the others of its block at the end of each tile)
    wave_lds_sync();
    if (lane < 8 * K)
        partial[(uint64_t)(lane / 8) * lvl_stride + ((uint64_t)ti * kTriRowsPerTile + wv) * 8 + lane % 8] =
            T[lane];
    wave_lds_sync();  // the next tile clears the row
  }
}

// ------------------------------------------------------------ hub triangles
// A hub candidate (larger window >= hub_min, smaller < kHubCap) belongs to
// its "owner" position p: the side with the larger window, the source side
// on a tie.  Its triangles are the pairs (entry of W(p), entry of the other
// window) with equal neighbours, exactly the pairs k_triangles would match.
// Consecutive positions of one S_u have overlapping windows, so rather than
// reading the large window once per candidate, each tile (kHubSlice
// positions of S) loads the union of its owners' windows into an LDS hash
// table keyed by neighbour, one kHubCap-entry segment at a time, and every
// owner probes it with each entry of its smaller window, keeping the matches
// that lie in its own window (p, p + W(p)].  Per candidate the work is its
// smaller window times the segments its window meets; the larger windows
// are read once per tile.

// Hub tiles: per graph, slices of kHubSlice positions of its S.  A slice
// holding a position with W >= hub_min goes on the work list (in no
// particular order: each tile writes its own row); the row of every other
// slice is zeroed here.  *count was zeroed by k_graph_tiles.
__global__ void k_hub_tiles(const uint64_t *planes, uint32_t hub_min, const uint32_t *eoff,
                            const uint32_t *htfirst, uint32_t G, uint32_t *count, uint32_t *list,
                            uint32_t levels, uint64_t lvl_stride, uint64_t *hpart) {
    const bool hub_first = hub_min <= kHubCap;
    const uint32_t n_tiles = htfirst[G];
    for (uint32_t ti = blockIdx.x * blockDim.x + threadIdx.x; ti < n_tiles;
         ti += gridDim.x * blockDim.x) {
        const uint32_t gi = last_le(htfirst, G + 1, ti);
        const uint32_t s0 = 2 * eoff[gi] + (ti - htfirst[gi]) * kHubSlice;
        const uint32_t s1 = min(2 * eoff[gi + 1], s0 + kHubSlice);
        bool any = false;
        for (uint32_t w = s0 / kWave; w <= (s1 - 1) / kWave && !any; w++) {
            uint64_t b = hub_word(planes, w, hub_first);
            const uint32_t wlo = w * kWave;
            if (s0 > wlo) b &= ~0ull << (s0 - wlo);
            if (s1 - wlo < kWave) b &= (1ull << (s1 - wlo)) - 1;
            any = b != 0;
        }
        if (any) {
            list[atomicAdd(count, 1u)] = ti;
        } else {
            for (uint32_t l = 0; l < levels; l++)
#pragma unroll
                for (int i = 0; i < 8; i++) hpart[l * lvl_stride + (uint64_t)ti * 8 + i] = 0;
        }
    }
}

// Exclusive prefix sum over the block (NT threads) of one value per thread;
// every thread also gets the block total.  Two block barriers.
template <uint32_t NT>
__device__ inline uint64_t block_scan_u64(uint64_t v, uint64_t *wtot, uint64_t &total) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wtot[wv] = x;
    __syncthreads();
    uint64_t off = 0, tot = 0;
#pragma unroll
    for (uint32_t i = 0; i < NT / kWave; i++) {
        const uint64_t sw = wtot[i];
        off += i < wv ? sw : 0;
        tot += sw;
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

constexpr uint64_t kLow48 = (1ull << 48) - 1;

struct HubArgs {
    SeqView S;
    const uint2 *epos2;
    const uint32_t *Wf;  // window sizes: window i of entry p at i * len + p
    uint64_t len;        // entries of S
    const uint64_t *planes;  // window bit planes (k_wlevels)
    const uint32_t *eoff, *htfirst, *count, *list;
    uint32_t G, hub_min;
    uint64_t lvl_stride;  // level l's rows go to hpart + l * lvl_stride
};

// K windows: owners, windows and segments are those of the largest one;
// each match is filed under its window level.
template <int K>
__global__ void __launch_bounds__(kHubBlock) __attribute__((amdgpu_waves_per_eu(6, 6)))
k_tri_hub(HubArgs a, uint64_t *hpart) {
    __shared__ uint32_t hk[kHubSlots];             // neighbour, or kEmptyKey
    __shared__ uint16_t ho[kHubSlots];             // entry's offset in the segment
    __shared__ uint32_t srd[kHubCap];              // rank << 1 | dir, by segment offset
    // owners: (p, W(p) | source side << 31, first position of the other
    // window, its size); W(p) < 2^31 as an S_u holds fewer than 2^31 entries
    __shared__ uint4 own_l[kHubSlice];
    __shared__ uint16_t sidx[kHubSlice];           // owners meeting the segment
    __shared__ uint64_t spre[kHubSlice + 1];       // their probe offsets
    __shared__ uint32_t wmark[kHubBlock / kWave][kWave];
    __shared__ uint64_t wtot[kHubBlock / kWave];
    __shared__ unsigned long long red[kHubBlock / kWave][8 * K];
    __shared__ uint32_t s_lo, s_hi;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave, nw = kHubBlock / kWave;
    const SeqView &S = a.S;
    const bool hub_first = a.hub_min <= kHubCap;
    const uint32_t n_list = *a.count;
    for (uint32_t li = blockIdx.x; li < n_list; li += gridDim.x) {
        const uint32_t ti = a.list[li];
        const uint32_t gi = last_le(a.htfirst, a.G + 1, ti);
        const uint32_t s0 = 2 * a.eoff[gi] + (ti - a.htfirst[gi]) * kHubSlice;
        const uint32_t s1 = min(2 * a.eoff[gi + 1], s0 + kHubSlice);
        if (threadIdx.x == 0) {
            s_lo = 0xffffffffu;
            s_hi = 0;
        }
        // A. owners among this thread's positions
        const uint32_t *Wtop = a.Wf + (K - 1) * a.len;  // the largest window
        uint32_t own = 0, rp[kHubPer], rw[kHubPer], rq[kHubPer], rwo[kHubPer];
#pragma unroll
        for (uint32_t k = 0; k < kHubPer; k++) {
            const uint32_t p = s0 + kHubPer * threadIdx.x + k;
            rp[k] = p;
            rw[k] = rq[k] = rwo[k] = 0;
            if (p < s1 && ((hub_word(a.planes, p / kWave, hub_first) >> (p % kWave)) & 1ull)) {
                const uint32_t W = Wtop[p];
                const uint2 e = a.epos2[S.rk[p]];
                const bool is_s = e.x == p;
                const uint32_t q = is_s ? e.y : e.x;
                const uint32_t Wo = Wtop[q];
                if (Wo != 0 && Wo < kHubCap && (is_s ? W >= Wo : W > Wo)) {
                    own |= 1u << k;
                    rw[k] = W | (is_s ? 0x80000000u : 0u);
                    rq[k] = q + 1;
                    rwo[k] = Wo;
                }
            }
        }
        uint64_t n_own64;
        uint32_t at = (uint32_t)block_scan_u64<kHubBlock>(__popc(own), wtot, n_own64);
        const uint32_t n_own = (uint32_t)n_own64;
#pragma unroll
        for (uint32_t k = 0; k < kHubPer; k++)
            if ((own >> k) & 1u) {
                own_l[at] = make_uint4(rp[k], rw[k], rq[k], rwo[k]);
                atomicMin(&s_lo, rp[k] + 1);
                atomicMax(&s_hi, rp[k] + (rw[k] & 0x7fffffffu));
                at++;
            }
        __syncthreads();
        // the previous tile's row was read before the barriers above
        if (threadIdx.x < nw * 8 * K) red[threadIdx.x / (8 * K)][threadIdx.x % (8 * K)] = 0;
        __syncthreads();
        const uint64_t lo = s_lo, hi = s_hi;
        for (uint64_t sl64 = lo; n_own != 0 && sl64 <= hi; sl64 += kHubCap) {
            const uint32_t sl = (uint32_t)sl64;
            const uint32_t sh = (uint32_t)min(hi, sl64 + kHubCap - 1);
            // B. owners whose window (p, p + W] meets [sl, sh], and where
            // their probes start in the flattened probe index; the scanned
            // value packs count << 48 | probes (< 2^42)
            uint32_t meet = 0;
            uint64_t mine = 0;
#pragma unroll
            for (uint32_t k = 0; k < kHubPer; k++) {
                const uint32_t i = threadIdx.x + k * kHubBlock;
                if (i < n_own) {
                    const uint4 o = own_l[i];
                    const uint32_t W = o.y & 0x7fffffffu;
                    if ((uint64_t)o.x + W >= sl && o.x + 1 <= sh) {
                        meet |= 1u << k;
                        mine += (1ull << 48) | o.w;
                    }
                }
            }
            uint64_t tot;
            const uint64_t pre = block_scan_u64<kHubBlock>(mine, wtot, tot);
            const uint32_t n_seg = (uint32_t)(tot >> 48);
            const uint64_t t_seg = tot & kLow48;
            {
                uint32_t idx = (uint32_t)(pre >> 48);
                uint64_t run = pre & kLow48;
#pragma unroll
                for (uint32_t k = 0; k < kHubPer; k++)
                    if ((meet >> k) & 1u) {
                        const uint32_t i = threadIdx.x + k * kHubBlock;
                        sidx[idx] = (uint16_t)i;
                        spre[idx] = run;
                        run += own_l[i].w;
                        idx++;
                    }
                if (threadIdx.x == 0) spre[n_seg] = t_seg;
            }
            // C. the segment's entries into the table
            for (uint32_t i = threadIdx.x; i < kHubSlots; i += kHubBlock) hk[i] = kEmptyKey;
            __syncthreads();
            for (uint32_t y = sl + threadIdx.x; y <= sh; y += kHubBlock) {
                const uint32_t nd = S.nd[y];
                const uint32_t key = nd >> 1;
                srd[y - sl] = (S.rk[y] << 1) | (nd & 1u);
                uint32_t h = (key * kHashMul) >> (32 - kHubBits);
                while (atomicCAS(&hk[h], kEmptyKey, key) != kEmptyKey) h = (h + 1) & (kHubSlots - 1);
                ho[h] = (uint16_t)(y - sl);
            }
            __syncthreads();
            // D. probes: each wave walks an equal share of the flattened index
            // space, lane j taking probe base + j.  Every owner has at least
            // one probe, so the probe ends spre[c + 1] are strictly
            // increasing and at most 64 of them fall in (base, base + 64]:
            // marking them in a 64-slot array gives each lane its owner by
            // a popcount.  Two 64-probe steps are mapped first and their
            // loads issued together, then both walk the table.
            // A match adds to its wave's LDS row of counters (u64) with an
            // LDS atomic: matches are rare next to the probes.
            const uint64_t jb = t_seg * wv / nw, je = t_seg * (wv + 1) / nw;
            if (jb < je) {
                uint32_t c0 = 0, chi = n_seg;  // last c with spre[c] <= jb
                while (chi - c0 > 1) {
                    const uint32_t mid = (c0 + chi) / 2;
                    if (spre[mid] <= jb) c0 = mid;
                    else chi = mid;
                }
                uint32_t *wm = wmark[wv];
                for (uint64_t base = jb; base < je; base += 2 * kWave) {
                    uint32_t cu[2];
#pragma unroll
                    for (int u = 0; u < 2; u++) {
                        const uint64_t bu = base + (uint64_t)u * kWave;
                        wm[lane] = 0;
                        wave_lds_sync();
                        const uint32_t k = c0 + (uint32_t)lane;
                        const uint64_t end = k < n_seg ? spre[k + 1] : ~0ull;  // > bu for k >= c0
                        if (end - bu < kWave) wm[end - bu] = 1;
                        wave_lds_sync();
                        const uint64_t M = __ballot(wm[lane] != 0);
                        const uint64_t done = __ballot(end <= bu + kWave);
                        const uint64_t below = lane == kWave - 1 ? M : (M & ((2ull << lane) - 1));
                        cu[u] = c0 + (uint32_t)__popcll(below);
                        c0 += (uint32_t)__popcll(done);
                        wave_lds_sync();
                    }
                    uint32_t nd[2], xs[2], pp[2], wpk[2], qq[2];
#pragma unroll
                    for (int u = 0; u < 2; u++) {
                        const uint64_t j = base + (uint64_t)u * kWave + (uint64_t)lane;
                        nd[u] = xs[u] = pp[u] = wpk[u] = qq[u] = 0;
                        if (j < je) {  // then cu[u] < n_seg
                            const uint4 o = own_l[sidx[cu[u]]];
                            const uint32_t x = o.z + (uint32_t)(j - spre[cu[u]]);
                            pp[u] = o.x;
                            wpk[u] = o.y;
                            qq[u] = o.z - 1;  // the other window's first edge entry
                            xs[u] = x;
                            nd[u] = S.nd[x];  // its rank is read on a (rare) match only
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 2; u++) {
                        if (base + (uint64_t)u * kWave + (uint64_t)lane >= je) continue;
                        const uint32_t key = nd[u] >> 1, p = pp[u], W = wpk[u] & 0x7fffffffu;
                        for (uint32_t h = (key * kHashMul) >> (32 - kHubBits);; h = (h + 1) & (kHubSlots - 1)) {
                            const uint32_t kk = hk[h];
                            if (kk == kEmptyKey) break;
                            if (kk == key) {
                                const uint32_t off = ho[h], y = sl + off;
                                if (y > p && y - p <= W) {
                                    const uint32_t v = srd[off], rx = S.rk[xs[u]], ox = xs[u] - qq[u];
                                    const bool own_s = (wpk[u] >> 31) != 0;
                                    const uint32_t cls = own_s ? tri_class(v >> 1, v & 1u, rx, nd[u] & 1u)
                                                               : tri_class(rx, nd[u] & 1u, v >> 1, v & 1u);
                                    const uint32_t l =
                                        own_s ? tri_level<K>(a.Wf, a.len, p, y - p, qq[u], ox)
                                              : tri_level<K>(a.Wf, a.len, qq[u], ox, p, y - p);
                                    tri_add(red[wv], l * 8 + cls);
                                }
                            }
                        }
                    }
                }
            }
            __syncthreads();  // the next segment rewrites the table and lists
        }
        // one row per tile and level (the segment loop ended on a barrier)
        if (threadIdx.x < 8 * K) {
            uint64_t v = 0;
#pragma unroll
            for (uint32_t q = 0; q < nw; q++) v += red[q][threadIdx.x];
            hpart[(uint64_t)(threadIdx.x / 8) * a.lvl_stride + (uint64_t)ti * 8 + threadIdx.x % 8] = v;
        }
    }
}

// Per graph: item tiles (star/pair), candidate tiles (triangles) and hub
// tiles (slices of its S, when the hub pass runs; the hub work-list counter
// is zeroed here).  A family that is not counted gets no tiles (its arrays
// are not read).
__global__ void k_graph_tiles(const uint32_t *mp_start, const uint32_t *mpb, const uint32_t *tidx,
                              const uint32_t *eoff, uint32_t G, int star_pair, int tri, int hub,
                              uint32_t elem_tile, uint32_t *n_item_tiles, uint32_t *n_cand_tiles,
                              uint32_t *n_hub_tiles, uint32_t *hub_count) {
    if (hub && blockIdx.x == 0 && threadIdx.x == 0) *hub_count = 0;
    for (uint32_t gi = blockIdx.x * blockDim.x + threadIdx.x; gi < G; gi += gridDim.x * blockDim.x) {
        const uint32_t elems = star_pair ? mp_start[mpb[gi + 1]] - mp_start[mpb[gi]] : 0u;
        const uint32_t cands = tri ? tidx[eoff[gi + 1]] - tidx[eoff[gi]] : 0u;
        const uint32_t ents = hub ? 2 * (eoff[gi + 1] - eoff[gi]) : 0u;
        n_item_tiles[gi] = (elems + elem_tile - 1) / elem_tile;
        n_cand_tiles[gi] = (cands + kCandTile - 1) / kCandTile;
        n_hub_tiles[gi] = (ents + kHubSlice - 1) / kHubSlice;
    }
}

// Per graph: sum its star/pair tile rows, its triangle tile rows and its hub
// tile rows.  Each graph's rows are split over `split` blocks (a single
// graph can have millions of rows); block (graph, part) writes one partial
// row of 40, and k_graph_sums_fin adds the parts.  Integer sums, no atomics.
constexpr uint32_t kSumSplitMin = 16, kSumSplitMax = 256;

// Blocks per graph: a few graphs get many each, large batches 16.
static uint32_t sum_split(uint32_t G) {
    return std::max(kSumSplitMin, std::min(kSumSplitMax, 4096u / std::max(G, 1u)));
}

__global__ void __launch_bounds__(kBlock) k_graph_sums(const uint64_t *spart, const uint32_t *tfirst,
                                                       const uint64_t *tpart,
                                                       const uint32_t *ctfirst,
                                                       const uint64_t *hpart,
                                                       const uint32_t *htfirst, uint32_t G,
                                                       uint32_t split, uint64_t *gpart) {
    __shared__ uint64_t lds[kBlock];
    for (uint64_t bi = blockIdx.x; bi < (uint64_t)G * split; bi += gridDim.x) {
        const uint32_t gi = (uint32_t)(bi / split), sp = (uint32_t)(bi % split);
        for (int pass = 0; pass < 3; pass++) {
            const uint32_t cols = pass == 0 ? 32u : 8u;
            const uint64_t *part = pass == 0 ? spart : pass == 1 ? tpart : hpart;
            const uint32_t *fr = pass == 0 ? tfirst : pass == 1 ? ctfirst : htfirst;
            const uint64_t rpt = pass == 1 ? kTriRowsPerTile : 1u;  // rows per tile
            const uint32_t c = threadIdx.x % cols, grp = threadIdx.x / cols, groups = kBlock / cols;
            uint64_t v = 0;
            for (uint64_t r = fr[gi] * rpt + sp * groups + grp; r < fr[gi + 1] * rpt;
                 r += groups * split)
                v += part[r * cols + c];
            lds[threadIdx.x] = v;
            __syncthreads();
            if (threadIdx.x < cols) {
                uint64_t sum = 0;
                for (uint32_t q = 0; q < groups; q++) sum += lds[q * cols + threadIdx.x];
                // the hub rows add to the triangle columns written by pass 1
                uint64_t *dst = &gpart[bi * 40 + (pass == 0 ? 0 : 32) + threadIdx.x];
                *dst = pass == 2 ? *dst + sum : sum;
            }
            __syncthreads();
        }
    }
}

// One block per graph: 6 groups of 40 threads take every 6th part row, then
// one thread per counter adds the groups.
__global__ void __launch_bounds__(kBlock) k_graph_sums_fin(const uint64_t *gpart, uint32_t G,
                                                           uint32_t split, uint64_t *out) {
    constexpr uint32_t kGroups = kBlock / 40;
    __shared__ uint64_t lds[kGroups * 40];
    const uint32_t c = threadIdx.x % 40, grp = threadIdx.x / 40;
    for (uint32_t gi = blockIdx.x; gi < G; gi += gridDim.x) {
        if (grp < kGroups) {
            uint64_t sum = 0;
            for (uint32_t sp = grp; sp < split; sp += kGroups)
                sum += gpart[((uint64_t)gi * split + sp) * 40 + c];
            lds[grp * 40 + c] = sum;
        }
        __syncthreads();
        if (threadIdx.x < 40) {
            uint64_t sum = 0;
            for (uint32_t q = 0; q < kGroups; q++) sum += lds[q * 40 + threadIdx.x];
            out[(uint64_t)gi * 40 + threadIdx.x] = sum;
        }
        __syncthreads();
    }
}

dim3 grid_for(uint64_t n, uint64_t cap) {
    uint64_t nb = (n + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    if (nb > cap) nb = cap;
    return dim3((unsigned)nb);
}

}  // namespace

constexpr uint32_t kDefaultRunChunk = 2;  // star/pair elements per thread
constexpr uint32_t kMaxRunChunk = 64;
constexpr uint32_t kDefaultTriLaneMax = 64;
constexpr uint32_t kDefaultHubMin = 32;

// ------------------------------------------------------------- host side
// Device workspace of one count: carved from one block, either per call or
// kept in the graph's plan for captured replays.
struct Workspace {
    uint32_t K = 1;  // windows counted in one pass (one graph when K > 1)
    int64_t *deltas;
    uint32_t *Wf;       // window i of entry p at i * len + p
    uint2 *recR, *recL; // window records: entry p's of window i at recR / recL[2 (i len + p)],
                        // the two side by side (one array, recL = recR + 1)
    uint64_t *planes;   // window bit planes, 3 words per 64 entries
    uint32_t *tflag, *tidx;
    uint4 *cand;
    uint32_t *n_itiles, *tfirst, *n_ctiles, *ctfirst, *tmp;
    uint32_t *n_htiles, *htfirst, *hcount, *hlist;
    uint64_t *spart, *tpart, *hpart, *gpart, *res;  // per window (res: K x G x 40)
    uint64_t max_itiles, max_ctiles, max_htiles;
};

static size_t workspace_bytes(const tm_graph *g, Workspace *w, uint32_t K = 1) {
    const uint32_t G = g->G;
    const uint64_t m = g->m, len = 2 * m, nm = g->n_multi, nme = g->n_me;
    w->K = K;
    w->max_itiles = nme / kBlock + G + 1;  // element tiles of at least kBlock elements
    w->max_ctiles = m / kCandTile + G + 1;
    w->max_htiles = len / kHubSlice + G + 1;
    const size_t n_tmp = scan_tmp_count(std::max<uint64_t>({m, nm, (uint64_t)G})) + 4;
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    return up((size_t)G * K * 8) + up(len * 4 * K) + up(len * 8 * K) * 2 + up((len / kWave + 1) * 24) +
           up((G + 1) * 4) * 2 + up(4) + up(w->max_htiles * 4) + up(w->max_htiles * 8 * 8 * K) +
           up((size_t)G * sum_split(G) * 40 * 8) +
           up(m * 4) + up((m + 1) * 4) + up(m * sizeof(uint4)) + up((G + 1) * 4) * 4 +
           up(n_tmp * 4) + up(w->max_itiles * 32 * 8 * K) +
           up(w->max_ctiles * kTriRowsPerTile * 8 * 8 * K) + up((size_t)G * 40 * 8 * K) + 4096;
}

static void workspace_carve(const tm_graph *g, Scratch &sc, Workspace *w) {
    const uint32_t G = g->G, K = w->K;
    const uint64_t m = g->m, len = 2 * m, nm = g->n_multi, nme = g->n_me;
    const size_t n_tmp = scan_tmp_count(std::max<uint64_t>({m, nm, (uint64_t)G})) + 4;
    w->deltas = sc.take<int64_t>((size_t)G * K);
    w->Wf = sc.take<uint32_t>(len * K);
    w->recR = sc.take<uint2>(2 * len * K);
    w->recL = w->recR + 1;
    w->planes = sc.take<uint64_t>(3 * (len / kWave + 1));
    w->n_htiles = sc.take<uint32_t>(G + 1);
    w->htfirst = sc.take<uint32_t>(G + 1);
    w->hcount = sc.take<uint32_t>(1);
    w->hlist = sc.take<uint32_t>(w->max_htiles);
    w->hpart = sc.take<uint64_t>(w->max_htiles * 8 * K);
    w->tflag = sc.take<uint32_t>(m);
    w->tidx = sc.take<uint32_t>(m + 1);
    w->cand = sc.take<uint4>(m);
    w->n_itiles = sc.take<uint32_t>(G + 1);
    w->tfirst = sc.take<uint32_t>(G + 1);
    w->n_ctiles = sc.take<uint32_t>(G + 1);
    w->ctfirst = sc.take<uint32_t>(G + 1);
    w->tmp = sc.take<uint32_t>(n_tmp);
    w->spart = sc.take<uint64_t>(w->max_itiles * 32 * K);
    w->tpart = sc.take<uint64_t>(w->max_ctiles * kTriRowsPerTile * 8 * K);
    w->gpart = sc.take<uint64_t>((size_t)G * sum_split(G) * 40);
    w->res = sc.take<uint64_t>((size_t)G * 40 * K);
}

// Launch a kernel template instantiated for K windows (1 .. kMaxLevels).
#define TM_LAUNCH_K(name, kern, K, grid, block, shm, stream, ...)                              \
    do {                                                                                       \
        switch (K) {                                                                           \
            case 1: TM_LAUNCH(name, kern<1>, grid, block, shm, stream, __VA_ARGS__); break;    \
            case 2: TM_LAUNCH(name, kern<2>, grid, block, shm, stream, __VA_ARGS__); break;    \
            case 3: TM_LAUNCH(name, kern<3>, grid, block, shm, stream, __VA_ARGS__); break;    \
            default: TM_LAUNCH(name, kern<4>, grid, block, shm, stream, __VA_ARGS__); break;   \
        }                                                                                      \
    } while (0)

// Every kernel of one count, deltas already in w.deltas (G x K, each graph's
// windows ascending), counters to w.res (K x G x 40; the triangle counters
// of window i hold the instances whose smallest window is i).  No host
// synchronisation, memset or allocation: capturable.
static int enqueue_count(tm_graph *g, const Workspace &w, const Params &pr, uint32_t families,
                         hipStream_t s) {
    // star/pair elements per thread (the run_chunk parameter)
    const uint32_t per = std::max(1u, std::min(pr.run_chunk, kMaxRunChunk));
    const uint32_t tri_lane_max = pr.tri_lane_max;
    const uint32_t G = g->G, K = w.K;
    if (K < 1 || K > (uint32_t)kMaxLevels || (K > 1 && G != 1)) {
        set_error("windows per pass out of range");
        return TM_EINTERNAL;
    }
    SeqView S{g->ent_t, g->ent_nd, g->ent_r, g->ent_c, g->X, g->off, g->epos};
    const uint64_t m = g->m, nme = g->n_me, len = 2 * m;
    const bool do_sp = (families & (TM_STARS | TM_PAIRS)) != 0;
    const bool do_tri = (families & TM_TRIANGLES) != 0;
    const bool do_hub = do_tri && pr.hub_min != TM_HUB_OFF;
    const uint64_t nm = do_sp ? g->n_multi : 0;
    const uint32_t *Wtop = w.Wf + (uint64_t)(K - 1) * len;  // entries' largest windows
    const uint64_t t_stride = w.max_ctiles * kTriRowsPerTile * 8, h_stride = w.max_htiles * 8;
    const uint64_t s_stride = w.max_itiles * 32;
    int rc;
    // one graph: the window kernel also writes the triangle bit planes
    const bool fused_levels = do_tri && G == 1;
    // trace rows: a4 star/pair (with the shared window kernel), a5 triangles,
    // a6 work items (chunks, tiles, hub slices), a7 reduction
    ProfRow row_a4("a4");
    TM_LAUNCH_K("windows", k_windows, K, dim3(std::min<uint32_t>(g->n_t_entries, 16384)), dim3(kBlock),
                0, s, S, g->t_entries, g->n_t_entries, len, w.deltas, w.Wf, pr.hub_min,
                fused_levels ? w.planes : nullptr,
                nm ? w.recR : nullptr, nm ? w.recL : nullptr);
    // ---- triangles: candidate first edges (of the largest window)
    if (do_tri) {
        ProfRow row_a5("a5");
        if (!fused_levels)  // batches: K == 1
            TM_LAUNCH("wlevels", k_wlevels, grid_for(2 * m, 16384), dim3(kBlock), 0, s, w.Wf, 2 * m,
                      pr.hub_min, w.planes);
        TM_LAUNCH("tri_flags", k_tri_flags, grid_for(m, 16384), dim3(kBlock), 0, s,
                  reinterpret_cast<const uint2 *>(g->epos), w.planes, pr.hub_min, m, w.tflag);
        rc = scan_u32_array(w.tflag, w.tidx, m, w.tmp, s);
        if (rc) return rc;
        TM_LAUNCH("tri_compact", k_tri_compact, grid_for(m, 16384), dim3(kBlock), 0, s,
                  reinterpret_cast<const uint2 *>(g->epos), Wtop, 1u, w.tflag, w.tidx, m, w.cand);
    }
    // ---- per-graph work tiles
    {
    ProfRow row_a6("a6");
    TM_LAUNCH("graph_tiles", k_graph_tiles, grid_for(G, 1024), dim3(kBlock), 0, s, g->mp_start,
              g->d_mpb, w.tidx, g->d_eoff, G, (int)(nm != 0), (int)do_tri, (int)do_hub,
              per * kBlock, w.n_itiles, w.n_ctiles, w.n_htiles, w.hcount);
    rc = scan_u32_array(w.n_itiles, w.tfirst, G, w.tmp, s);
    if (rc) return rc;
    rc = scan_u32_array(w.n_ctiles, w.ctfirst, G, w.tmp, s);
    if (rc) return rc;
    rc = scan_u32_array(w.n_htiles, w.htfirst, G, w.tmp, s);
    if (rc) return rc;
    if (do_hub)
        TM_LAUNCH("hub_tiles", k_hub_tiles, grid_for(w.max_htiles, 4096), dim3(kBlock), 0, s, w.planes,
                  pr.hub_min, g->d_eoff, w.htfirst, G, w.hcount, w.hlist, K, h_stride, w.hpart);
    }
    if (nm) {
        StarArgs sa{g->mp_start, g->me_t, g->me_o, g->me_a, g->me_p, w.recR, w.recL, len, K, s_stride,
                    g->d_mpb, w.tfirst, G, w.deltas, per, (families & TM_STARS) ? 1 : 0};
        TM_LAUNCH("star_pair", k_star_pair, dim3((unsigned)std::min<uint64_t>(w.max_itiles, 8192)),
                  dim3(kBlock), 0, s, sa, w.spart);
    }
    if (do_tri) {
        ProfRow row_a5("a5");
        TM_LAUNCH_K("triangles", k_triangles, K, dim3((unsigned)std::min<uint64_t>(w.max_ctiles, 8192)),
                    dim3(kBlock), 0, s, S, w.cand, w.tidx, g->d_eoff, w.ctfirst, G, tri_lane_max,
                    w.Wf, len, t_stride, w.tpart);
    }
    if (do_hub) {
        ProfRow row_a5("a5");
        HubArgs ha{S, reinterpret_cast<const uint2 *>(g->epos), w.Wf, len, w.planes, g->d_eoff,
                   w.htfirst, w.hcount, w.hlist, G, pr.hub_min, h_stride};
        TM_LAUNCH_K("tri_hub", k_tri_hub, K, dim3((unsigned)std::min<uint64_t>(w.max_htiles, 4096)),
                    dim3(kHubBlock), 0, s, ha, w.hpart);
    }
    const uint32_t split = sum_split(G);
    ProfRow row_a7("a7");
    for (uint32_t i = 0; i < K; i++) {
        TM_LAUNCH("graph_sums", k_graph_sums, dim3((unsigned)std::min<uint64_t>((uint64_t)G * split, 16384)),
                  dim3(kBlock), 0, s, w.spart + i * s_stride, w.tfirst, w.tpart + i * t_stride,
                  w.ctfirst, w.hpart + i * h_stride, w.htfirst, G, split, w.gpart);
        TM_LAUNCH("graph_sums_fin", k_graph_sums_fin, dim3(std::min<uint32_t>(G, 4096)), dim3(kBlock), 0,
                  s, w.gpart, G, split, w.res + (size_t)i * G * 40);
    }
    return TM_OK;
}

size_t count_workspace_bytes(const tm_graph *g) {
    Workspace w;
    return workspace_bytes(g, &w);
}

// Captured count sequence of one graph object, replayed on a private stream.
struct Plan {
    Scratch mem;
    Workspace w;
    Params pr;
    uint32_t families = 0;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev = nullptr;
};

void plan_release(tm_graph *g) {
    Plan *p = g->plan;
    if (!p) return;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->ev) (void)hipEventDestroy(p->ev);
    {
        // the workspace returns to the cache on the plan's stream
        Scratch tmp;
        std::swap(tmp.base, p->mem.base);
        tmp.stream = p->stream;
        tmp.cap = p->mem.cap;
    }
    if (p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
    g->plan = nullptr;
}

static int plan_prepare(tm_graph *g, const Params &pr, uint32_t families) {
    Plan *p = g->plan;
    if (p && p->exec && p->pr == pr && p->families == families) return TM_OK;
    plan_release(g);
    p = new (std::nothrow) Plan();
    if (!p) return TM_ENOMEM;
    g->plan = p;
    TM_HIP_TRY(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
    TM_HIP_TRY(hipEventCreateWithFlags(&p->ev, hipEventDisableTiming));
    const size_t bytes = workspace_bytes(g, &p->w);
    int rc = p->mem.reserve(bytes, p->stream);
    if (rc) return rc;
    workspace_carve(g, p->mem, &p->w);
    p->pr = pr;
    p->families = families;
    TM_HIP_TRY(hipStreamSynchronize(p->stream));
    TM_HIP_TRY(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    set_capturing(true);
    rc = enqueue_count(g, p->w, pr, families, p->stream);
    set_capturing(false);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(p->stream, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) {
        set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        return TM_EHIP;
    }
    p->graph = graph;
    TM_HIP_TRY(hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0));
    return TM_OK;
}

// Partition parameters used where a call passes 0: the graph's tuned values,
// else the autotuner table's entry for graphs of this shape, else defaults.
static void resolve_params(const tm_graph *g, Params *pr) {
    Params t = g->tuned;
    if (!t.run_chunk || !t.tri_lane_max || !t.hub_min) tune_table_lookup(g, &t);
    if (pr->run_chunk == 0) pr->run_chunk = t.run_chunk ? t.run_chunk : kDefaultRunChunk;
    if (pr->tri_lane_max == 0) pr->tri_lane_max = t.tri_lane_max ? t.tri_lane_max : kDefaultTriLaneMax;
    if (pr->hub_min == 0) pr->hub_min = t.hub_min ? t.hub_min : kDefaultHubMin;
}

// Raw counters (G x 56) from the kernels' per-graph counters (G x 40):
// Star | Pair as counted; the Tri views from the classes by the orbit
// Tri[I,a,b,c] = Tri[II,~c,~b,~a] = Tri[III,c,~a,~b].
void raw_from_counters(const uint64_t *res40, uint32_t G, uint64_t *raw) {
    for (uint32_t gi = 0; gi < G; gi++) {
        const uint64_t *h = res40 + (size_t)gi * 40;
        uint64_t *rw = raw + (size_t)gi * 56;
        for (int i = 0; i < 32; i++) rw[i] = h[i];
        const uint64_t *N = h + 32;
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                for (int c = 0; c < 2; c++) {
                    const uint64_t v = N[a * 4 + b * 2 + c];
                    rw[32 + 0 * 8 + a * 4 + b * 2 + c] = v;
                    rw[32 + 1 * 8 + (1 - c) * 4 + (1 - b) * 2 + (1 - a)] = v;
                    rw[32 + 2 * 8 + c * 4 + (1 - a) * 2 + (1 - b)] = v;
                }
    }
}

// Asynchronous count through the graph's captured plan: deltas are read from
// pinned host memory, the G x 40 counters land in pinned host memory, and
// `done` is recorded after the copy.  Returns without waiting.
// Capture the count plan count_graph_async will replay (for all motifs,
// with the graph's resolved partition parameters), so that the capture can
// run on a thread of the caller's choosing.
int count_plan_prepare(tm_graph *g) {
    if (g->m < 3) return TM_OK;
    Params pr;
    resolve_params(g, &pr);
    return plan_prepare(g, pr, TM_ALL_MOTIFS);
}

int count_graph_async(tm_graph *g, const int64_t *pinned_deltas, uint64_t *pinned_res,
                      hipEvent_t done) {
    const uint32_t G = g->G;
    if (g->m < 3) {
        for (size_t i = 0; i < (size_t)G * 40; i++) pinned_res[i] = 0;
        TM_HIP_TRY(hipEventRecord(done, g->stream));
        return TM_OK;
    }
    Params pr;
    resolve_params(g, &pr);
    int rc = plan_prepare(g, pr, TM_ALL_MOTIFS);
    if (rc) return rc;
    Plan *p = g->plan;
    TM_HIP_TRY(hipEventRecord(p->ev, g->stream));
    TM_HIP_TRY(hipStreamWaitEvent(p->stream, p->ev, 0));
    TM_HIP_TRY(hipMemcpyAsync(p->w.deltas, pinned_deltas, G * 8, hipMemcpyHostToDevice, p->stream));
    TM_HIP_TRY(hipGraphLaunch(p->exec, p->stream));
    TM_HIP_TRY(hipMemcpyAsync(pinned_res, p->w.res, (size_t)G * 40 * 8, hipMemcpyDeviceToHost,
                              p->stream));
    TM_HIP_TRY(hipEventRecord(done, p->stream));
    return TM_OK;
}

int count_graph(tm_graph *g, const int64_t *h_deltas, Params pr, uint64_t *raw, bool use_graph,
                uint32_t families) {
    resolve_params(g, &pr);
    const uint32_t G = g->G;
    std::vector<uint64_t> host((size_t)G * 40, 0);
    if (g->m >= 3) {
        if (use_graph) {
            int rc = plan_prepare(g, pr, families);
            if (rc) return rc;
            Plan *p = g->plan;
            // order after earlier work on the graph's stream, run, copy back
            TM_HIP_TRY(hipEventRecord(p->ev, g->stream));
            TM_HIP_TRY(hipStreamWaitEvent(p->stream, p->ev, 0));
            TM_HIP_TRY(hipMemcpyAsync(p->w.deltas, h_deltas, G * 8, hipMemcpyHostToDevice, p->stream));
            TM_HIP_TRY(hipGraphLaunch(p->exec, p->stream));
            TM_HIP_TRY(hipMemcpyAsync(host.data(), p->w.res, (size_t)G * 40 * 8,
                                      hipMemcpyDeviceToHost, p->stream));
            TM_HIP_TRY(hipStreamSynchronize(p->stream));
        } else {
            hipStream_t s = g->stream;
            Workspace w;
            const size_t bytes = workspace_bytes(g, &w);
            Scratch sc;
            int rc = sc.reserve(bytes, s);
            if (rc) return rc;
            workspace_carve(g, sc, &w);
            TM_HIP_TRY(hipMemcpyAsync(w.deltas, h_deltas, G * 8, hipMemcpyHostToDevice, s));
            rc = enqueue_count(g, w, pr, families, s);
            if (rc) return rc;
            TM_HIP_TRY(hipMemcpyAsync(host.data(), w.res, (size_t)G * 40 * 8, hipMemcpyDeviceToHost, s));
            TM_HIP_TRY(hipStreamSynchronize(s));
        }
    }
    raw_from_counters(host.data(), G, raw);
    // families not asked for are zero (their kernels did not run, or ran
    // only in part: the pair sweep also yields some star cells)
    for (uint32_t gi = 0; gi < G; gi++) {
        uint64_t *rw = raw + (size_t)gi * 56;
        if (!(families & TM_STARS))
            for (int i = 0; i < 24; i++) rw[i] = 0;
        if (!(families & TM_PAIRS))
            for (int i = 24; i < 32; i++) rw[i] = 0;
        if (!(families & TM_TRIANGLES))
            for (int i = 32; i < 56; i++) rw[i] = 0;
    }
    return TM_OK;
}

// ---------------------------------------------------- allocation-free count
// The workspace of tm_count_noalloc: one fixed device array per device,
// held from library load until the process ends.  Host code never passes
// `scratch` itself to a kernel (in host code the name is a host-side
// stand-in, not a device address); it uses the address hipGetSymbolAddress
// returns for the current device, looked up once per device.
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu[kMaxDevices];  // one call at a time per device (shared workspace)
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static int scratch_for_device(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index out of range for the allocation-free count");
        return TM_EINVAL;
    }
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return TM_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TM_OK;
}

int count_graph_noalloc(tm_graph *g, int64_t delta, uint64_t *raw) {
    uint64_t host[40] = {0};
    if (g->m >= 3) {
        Params pr;
        resolve_params(g, &pr);
        const int dev = g->device;
        if (dev < 0 || dev >= kMaxDevices) {
            set_error("device index out of range for the allocation-free count");
            return TM_EINVAL;
        }
        std::lock_guard<std::mutex> lk(g_noalloc_mu[dev]);
        void *base = nullptr;
        int rc = scratch_for_device(dev, &base);
        if (rc) return rc;
        Workspace w;
        const size_t bytes = workspace_bytes(g, &w);
        if (bytes > kNoAllocScratchBytes) {
            set_error("the allocation-free count needs " + std::to_string(bytes) +
                      " bytes of workspace for this graph; its fixed workspace holds " +
                      std::to_string(kNoAllocScratchBytes));
            return TM_ENOMEM;
        }
        hipStream_t s = g->stream;
        Scratch sc;
        sc.base = static_cast<char *>(base);
        sc.cap = kNoAllocScratchBytes;
        sc.stream = s;
        sc.owned = false;
        workspace_carve(g, sc, &w);
        TM_HIP_TRY(hipMemcpyAsync(w.deltas, &delta, 8, hipMemcpyHostToDevice, s));
        rc = enqueue_count(g, w, pr, TM_ALL_MOTIFS, s);
        if (rc) return rc;
        TM_HIP_TRY(hipMemcpyAsync(host, w.res, sizeof(host), hipMemcpyDeviceToHost, s));
        // the next call may reuse the workspace only after this one is done
        TM_HIP_TRY(hipStreamSynchronize(s));
    }
    raw_from_counters(host, 1, raw);
    return TM_OK;
}

// Several windows over one built graph (G == 1) in one call.  The windows
// are taken in ascending order, up to kMaxLevels per pass: a pass builds the
// window sizes of all its windows in one kernel, finds the triangle
// candidates and matches them once, for its largest window, and files each
// match under the smallest window holding it (so window i's triangles are
// the sum of levels 0 .. i); the star/pair sweeps run per window.  Each
// pass's counters go to their own device slot, then one download and one
// synchronisation return all of them.
int count_graph_multi(tm_graph *g, const int64_t *h_deltas, uint32_t k, Params pr, uint64_t *raw) {
    resolve_params(g, &pr);
    std::vector<uint32_t> ord(k);
    for (uint32_t i = 0; i < k; i++) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](uint32_t a, uint32_t b) { return h_deltas[a] < h_deltas[b]; });
    std::vector<int64_t> sorted(k);
    for (uint32_t i = 0; i < k; i++) sorted[i] = h_deltas[ord[i]];
    std::vector<uint64_t> host((size_t)k * 40, 0);  // ascending window order
    const uint32_t kmax = std::min<uint32_t>(k, (uint32_t)kMaxLevels);
    if (g->m >= 3 && k > 0) {
        hipStream_t s = g->stream;
        Workspace w;
        Scratch sc, sk;
        int rc = sc.reserve(workspace_bytes(g, &w, kmax), s);
        if (rc) return rc;
        workspace_carve(g, sc, &w);
        rc = sk.reserve((size_t)k * 8 + (size_t)k * 40 * 8 + 1024, s);
        if (rc) return rc;
        int64_t *dk = sk.take<int64_t>(k);
        uint64_t *resk = sk.take<uint64_t>((size_t)k * 40);
        TM_HIP_TRY(hipMemcpyAsync(dk, sorted.data(), (size_t)k * 8, hipMemcpyHostToDevice, s));
        for (uint32_t g0 = 0; g0 < k; g0 += kmax) {
            w.K = std::min(kmax, k - g0);
            TM_HIP_TRY(hipMemcpyAsync(w.deltas, dk + g0, (size_t)w.K * 8, hipMemcpyDeviceToDevice, s));
            rc = enqueue_count(g, w, pr, TM_ALL_MOTIFS, s);
            if (rc) return rc;
            TM_HIP_TRY(hipMemcpyAsync(resk + (size_t)g0 * 40, w.res, (size_t)w.K * 40 * 8,
                                      hipMemcpyDeviceToDevice, s));
        }
        TM_HIP_TRY(hipMemcpyAsync(host.data(), resk, (size_t)k * 40 * 8, hipMemcpyDeviceToHost, s));
        TM_HIP_TRY(hipStreamSynchronize(s));
        // a pass's window i holds the triangles of its levels 0 .. i
        for (uint32_t g0 = 0; g0 < k; g0 += kmax)
            for (uint32_t i = g0 + 1; i < std::min(k, g0 + kmax); i++)
                for (int c = 32; c < 40; c++) host[(size_t)i * 40 + c] += host[(size_t)(i - 1) * 40 + c];
    }
    for (uint32_t i = 0; i < k; i++)
        raw_from_counters(host.data() + (size_t)i * 40, 1, raw + (size_t)ord[i] * 56);
    return TM_OK;
}

// ------------------------------------------------------------- autotuner
// Times the eager count of this graph over partition parameters and keeps
// the fastest: first the work-item chunk of the star/pair sweeps with the
// lane/wave split of the triangle matching, then, with those fixed, the
// window size from which triangle candidates go to the hub kernel.  k == 1:
// the count of graph i at h_deltas[i]; k > 1 (one graph): one pass of the
// several-window count over the largest min(k, kMaxLevels) of the k windows.
// The result is stored on the graph and in a process-wide table keyed by the
// graph's shape (log2 of edges, of multi-pair edges, and of the graph
// count), which later graphs of that shape use by default.
int autotune(tm_graph *g, const int64_t *h_deltas, uint32_t k, Params *best, float *best_ms) {
    static const uint32_t chunks[] = {2, 4, 8};
    static const uint32_t lanes[] = {8, 32, 64, 256, 1024};
    static const uint32_t hubs[] = {16, 32, 64, 128, 256, 1024, TM_HUB_OFF};
    Params bp;
    bp.run_chunk = kDefaultRunChunk;
    bp.tri_lane_max = kDefaultTriLaneMax;
    bp.hub_min = kDefaultHubMin;
    float bt = 0;
    if (g->m >= 3) {
        hipStream_t s = g->stream;
        const uint32_t K = k > 1 ? std::min<uint32_t>(k, (uint32_t)kMaxLevels) : 1u;
        std::vector<int64_t> dl(h_deltas, h_deltas + (k > 1 ? k : g->G));
        if (k > 1) {
            std::sort(dl.begin(), dl.end());
            dl.erase(dl.begin(), dl.end() - K);
        }
        Workspace w;
        Scratch sc;
        int rc = sc.reserve(workspace_bytes(g, &w, K), s);
        if (rc) return rc;
        workspace_carve(g, sc, &w);
        TM_HIP_TRY(hipMemcpyAsync(w.deltas, dl.data(), dl.size() * 8, hipMemcpyHostToDevice, s));
        // the copy reads the host vector before it goes out of scope
        TM_HIP_TRY(hipStreamSynchronize(s));
        hipEvent_t e0, e1;
        TM_HIP_TRY(hipEventCreate(&e0));
        TM_HIP_TRY(hipEventCreate(&e1));
        bt = -1;
        // best of two runs of one setting; -1 on error
        auto time_one = [&](const Params &pr) -> float {
            float tbest = -1;
            for (int rep = 0; rep < 2 && rc == TM_OK; rep++) {
                (void)hipEventRecord(e0, s);
                rc = enqueue_count(g, w, pr, TM_ALL_MOTIFS, s);
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (tbest < 0 || ms < tbest) tbest = ms;
            }
            return rc == TM_OK ? tbest : -1.0f;
        };
        for (uint32_t c : chunks)
            for (uint32_t l : lanes) {
                Params pr = bp;
                pr.run_chunk = c;
                pr.tri_lane_max = l;
                const float t = time_one(pr);
                if (rc) break;
                if (bt < 0 || t < bt) {
                    bt = t;
                    bp = pr;
                }
            }
        for (uint32_t h : hubs) {
            if (rc) break;
            Params pr = bp;
            pr.hub_min = h;
            const float t = time_one(pr);
            if (rc) break;
            if (t < bt) {
                bt = t;
                bp = pr;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
    }
    g->tuned = bp;
    tune_table_store(g, bp);
    if (best) *best = bp;
    if (best_ms) *best_ms = bt;
    return TM_OK;
}

}  // namespace tmc
