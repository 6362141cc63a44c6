/*
 * Brute-force enumerator of the delta-temporal motif definition.
 *
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see tm_oracle.c).  It
 * shares no code with the paper's algorithms in tm_oracle.c, so that the two
 * can check each other.
 *
 * Definition 2 / Definition 3 / Problem 1 of the paper: an instance is a set
 * of three distinct edges, taken in chronological order E1 < E2 < E3, with
 * t(E3) - t(E1) <= delta and whose static graph is connected with at most
 * three nodes (without self-loops, "at most three endpoints" already implies
 * connected).  Ties in t are ordered by input index.  Every such triple is
 * enumerated directly (all triples inside delta, O(m * w^2)) and classified:
 *
 *   2 nodes            -> pair: seen from node p = src(E1), dirs (o, d2, d3)
 *   3 nodes, 2 pairs   -> star: center c on all three edges, d_k = o iff E_k
 *                         leaves c, type = position (1, 2, 3) of the edge whose
 *                         node pair is not shared (Section IV-A: Star-I/II/III)
 *   3 nodes, 3 pairs   -> triangle: r = the node not on E1, E2 = {r, v},
 *                         E3 = {r, w}; a = o iff E2 leaves r, b = o iff E3
 *                         leaves r, c = o iff E1 = v -> w
 *
 * Two outputs:
 *   canon[36]: class counts, [0,24) Star[type][d1][d2][d3] (o = 0, in = 1),
 *              [24,28) pair class [d2][d3], [28,36) triangle class [a][b][c].
 *   raw[56]:   the paper's per-center counters, built from the definition of
 *              each counter rather than from the algorithms: Star at the
 *              center; Pair[d1,d2,d3] once from each of the two nodes; and for
 *              triangles, from every vertex x: e_i, e_j = its two edges in time
 *              order, e_k the third; Type I/II/III = e_k before e_i / between /
 *              after e_j (Section IV-B); d_i, d_j relative to x; d_k = o iff
 *              e_k leaves v = the other node of e_i.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BR_OK 0
#define BR_EINVAL (-1)
#define BR_ENOMEM (-2)

typedef struct {
    const int32_t *s, *d;
    const int64_t *t;
} bref;
static bref g_b;

static int cmp_time(const void *pa, const void *pb) {
    uint32_t x = *(const uint32_t *)pa, y = *(const uint32_t *)pb;
    if (g_b.t[x] != g_b.t[y]) return g_b.t[x] < g_b.t[y] ? -1 : 1;
    return x < y ? -1 : (x > y);
}

static int same_pair(int32_t a1, int32_t b1, int32_t a2, int32_t b2) {
    return (a1 == a2 && b1 == b2) || (a1 == b2 && b1 == a2);
}

static int touches(int32_t a, int32_t b, int32_t x) { return a == x || b == x; }

static void classify(const int32_t *S, const int32_t *D, const uint32_t e[3], uint64_t *canon,
                     uint64_t *raw) {
    int32_t nodes[6];
    int nn = 0;
    for (int k = 0; k < 3; k++) {
        int32_t ends[2] = {S[e[k]], D[e[k]]};
        for (int q = 0; q < 2; q++) {
            int seen = 0;
            for (int z = 0; z < nn; z++) seen |= (nodes[z] == ends[q]);
            if (!seen) nodes[nn++] = ends[q];
        }
    }
    if (nn > 3) return;
    if (nn == 2) {
        /* pair */
        int32_t p = S[e[0]];
        int d2 = S[e[1]] == p ? 0 : 1, d3 = S[e[2]] == p ? 0 : 1;
        canon[24 + d2 * 2 + d3] += 1;
        for (int q = 0; q < 2; q++) {
            int32_t x = nodes[q];
            int d[3];
            for (int k = 0; k < 3; k++) d[k] = S[e[k]] == x ? 0 : 1;
            raw[24 + d[0] * 4 + d[1] * 2 + d[2]] += 1;
        }
        return;
    }
    /* three nodes: star (2 distinct pairs) or triangle (3 distinct pairs) */
    int p01 = same_pair(S[e[0]], D[e[0]], S[e[1]], D[e[1]]);
    int p02 = same_pair(S[e[0]], D[e[0]], S[e[2]], D[e[2]]);
    int p12 = same_pair(S[e[1]], D[e[1]], S[e[2]], D[e[2]]);
    if (p01 || p02 || p12) {
        int32_t c = -1;
        for (int z = 0; z < 3; z++) {
            int all = 1;
            for (int k = 0; k < 3; k++) all &= touches(S[e[k]], D[e[k]], nodes[z]);
            if (all) c = nodes[z];
        }
        int type = p12 ? 0 : (p02 ? 1 : 2); /* position of the unshared edge */
        int d[3];
        for (int k = 0; k < 3; k++) d[k] = S[e[k]] == c ? 0 : 1;
        int idx = type * 8 + d[0] * 4 + d[1] * 2 + d[2];
        canon[idx] += 1;
        raw[idx] += 1;
        return;
    }
    /* triangle: class at r = the node not on E1 */
    {
        int32_t r = -1;
        for (int z = 0; z < 3; z++)
            if (!touches(S[e[0]], D[e[0]], nodes[z])) r = nodes[z];
        int32_t v = S[e[1]] == r ? D[e[1]] : S[e[1]];
        int a = S[e[1]] == r ? 0 : 1;
        int b = S[e[2]] == r ? 0 : 1;
        int c = S[e[0]] == v ? 0 : 1;
        canon[28 + a * 4 + b * 2 + c] += 1;
    }
    /* per-vertex views (the paper's Tri counter) */
    for (int z = 0; z < 3; z++) {
        int32_t x = nodes[z];
        int at[2], na = 0, kk = -1;
        for (int k = 0; k < 3; k++) {
            if (touches(S[e[k]], D[e[k]], x)) at[na++] = k;
            else kk = k;
        }
        int ei = at[0], ej = at[1];            /* positions are already time order */
        int type = kk < ei ? 0 : (kk < ej ? 1 : 2);
        int di = S[e[ei]] == x ? 0 : 1;
        int dj = S[e[ej]] == x ? 0 : 1;
        int32_t v = S[e[ei]] == x ? D[e[ei]] : S[e[ei]];
        int dk = S[e[kk]] == v ? 0 : 1;
        raw[32 + type * 8 + di * 4 + dj * 2 + dk] += 1;
    }
}

int oracle_brute(const int32_t *src, const int32_t *dst, const int64_t *t, uint64_t m,
                 uint32_t n, int64_t delta, uint64_t raw[56], uint64_t canon[36]) {
    if (!raw || !canon || delta < 0) return BR_EINVAL;
    if (m && (!src || !dst || !t)) return BR_EINVAL;
    for (uint64_t k = 0; k < m; k++) {
        if (src[k] < 0 || dst[k] < 0 || (uint32_t)src[k] >= n || (uint32_t)dst[k] >= n ||
            src[k] == dst[k])
            return BR_EINVAL;
        if (t[k] >= ((int64_t)1 << 62) || t[k] <= -((int64_t)1 << 62)) return BR_EINVAL;
    }
    memset(raw, 0, 56 * sizeof(uint64_t));
    memset(canon, 0, 36 * sizeof(uint64_t));
    uint32_t *ord = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    if (!ord) return BR_ENOMEM;
    for (uint64_t k = 0; k < m; k++) ord[k] = (uint32_t)k;
    g_b.s = src;
    g_b.d = dst;
    g_b.t = t;
    qsort(ord, m, sizeof(uint32_t), cmp_time);
    for (uint64_t a = 0; a < m; a++) {
        for (uint64_t b = a + 1; b < m; b++) {
            if (t[ord[b]] - t[ord[a]] > delta) break;
            for (uint64_t c = b + 1; c < m; c++) {
                if (t[ord[c]] - t[ord[a]] > delta) break;
                uint32_t e[3] = {ord[a], ord[b], ord[c]};
                classify(src, dst, e, canon, raw);
            }
        }
    }
    free(ord);
    return BR_OK;
}
