/*
 * Four-node, three-edge delta-temporal motifs: the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle; see tm_oracle.c).  The
 * product path never links or calls it.
 *
 * The paper leaves higher-order motifs to future work (Section VI, counting
 * them with more centers and bigger counters).  Its Definitions 2 and 3 and
 * Problem 1 carry over unchanged to three edges on four nodes: three distinct
 * edges taken in chronological order E1 < E2 < E3 (ties in t ordered by input
 * index), t(E3) - t(E1) <= delta, and a static graph that is connected with
 * exactly four nodes.  Three edges on four nodes, every node on an edge, with
 * three distinct node pairs form a tree, so an instance is one of:
 *
 *   star   one node c on all three edges (three distinct leaves).  Class
 *          [d1][d2][d3] with d_k = 0 iff E_k leaves c (the paper's o), else 1.
 *   path   v0 - v1 - v2 - v3.  The middle edge {v1, v2} has an end edge on each
 *          side; the path is read from the end edge that comes first in the
 *          chronological order (it is {v0, v1}).  An edge {v_i, v_i+1} is
 *          forward (1) if it points from v_i to v_i+1.  Class
 *          [r][f1][f2][f3]: r = 0, 1, 2 the chronological position of the
 *          middle edge, f_k = forward bit of E_k.
 *
 * Output out[32]: [0, 8) star [d1][d2][d3]; [8, 32) path 8 + r * 8 + f1 * 4 +
 * f2 * 2 + f3.  (The 36 classes of three-edge motifs on at most three nodes
 * are counted by tm_oracle.c / tm_brute.c.)
 *
 * Two enumerations that share no code:
 *   oracle4_brute   every chronological edge triple inside delta, classified
 *                   from the triple's degrees alone (tiny inputs only);
 *   oracle4_local   per center node (stars: triples of its own edges) and per
 *                   middle edge (paths: one edge at each endpoint), each
 *                   classified by the role it was found in; OpenMP.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O4_OK 0
#define O4_EINVAL (-1)
#define O4_ENOMEM (-2)

static int validate(const int32_t *src, const int32_t *dst, const int64_t *t, uint64_t m,
                    uint32_t n, int64_t delta) {
    if (delta < 0) return O4_EINVAL;
    if (m && (!src || !dst || !t)) return O4_EINVAL;
    if (m >= 0xffffffffull) return O4_EINVAL;
    for (uint64_t k = 0; k < m; k++) {
        if (src[k] < 0 || dst[k] < 0 || (uint32_t)src[k] >= n || (uint32_t)dst[k] >= n ||
            src[k] == dst[k])
            return O4_EINVAL;
        if (t[k] >= ((int64_t)1 << 62) || t[k] <= -((int64_t)1 << 62)) return O4_EINVAL;
    }
    return O4_OK;
}

/* chronological order: t, then input index */
static const int64_t *g_sort_t;
static int cmp_chrono(const void *pa, const void *pb) {
    uint32_t x = *(const uint32_t *)pa, y = *(const uint32_t *)pb;
    if (g_sort_t[x] != g_sort_t[y]) return g_sort_t[x] < g_sort_t[y] ? -1 : 1;
    return x < y ? -1 : (x > y);
}

/* ------------------------------------------------------------- brute force */

/* E[0..2] in chronological order. */
static void classify_triple(const int32_t *S, const int32_t *D, const uint32_t E[3],
                            uint64_t out[32]) {
    int32_t node[6];
    int deg[6] = {0, 0, 0, 0, 0, 0};
    int nn = 0;
    for (int k = 0; k < 3; k++) {
        int32_t ends[2] = {S[E[k]], D[E[k]]};
        for (int q = 0; q < 2; q++) {
            int z = 0;
            while (z < nn && node[z] != ends[q]) z++;
            if (z == nn) node[nn++] = ends[q];
            deg[z]++;
        }
    }
    if (nn != 4) return;
    /* three distinct node pairs (with four nodes this makes a tree) */
    for (int a = 0; a < 3; a++)
        for (int b = a + 1; b < 3; b++) {
            int same = (S[E[a]] == S[E[b]] && D[E[a]] == D[E[b]]) ||
                       (S[E[a]] == D[E[b]] && D[E[a]] == S[E[b]]);
            if (same) return;
        }
    int32_t center = -1;
    for (int z = 0; z < 4; z++)
        if (deg[z] == 3) center = node[z];
    if (center >= 0) {
        int idx = 0;
        for (int k = 0; k < 3; k++) idx = idx * 2 + (S[E[k]] == center ? 0 : 1);
        out[idx] += 1;
        return;
    }
    /* path: the middle edge joins the two degree-2 nodes */
    int mid = -1;
    for (int k = 0; k < 3; k++) {
        int ds = 0, dd = 0;
        for (int z = 0; z < 4; z++) {
            if (node[z] == S[E[k]]) ds = deg[z];
            if (node[z] == D[E[k]]) dd = deg[z];
        }
        if (ds == 2 && dd == 2) mid = k;
    }
    int left = -1, right = -1; /* end edges; left = the earlier one */
    for (int k = 0; k < 3; k++) {
        if (k == mid) continue;
        if (left < 0) left = k;
        else right = k;
    }
    /* v1 = the left end edge's node on the middle edge */
    int32_t ms = S[E[mid]], md = D[E[mid]];
    int32_t ls = S[E[left]], ld = D[E[left]];
    int32_t v1 = (ls == ms || ls == md) ? ls : ld;
    int32_t v0 = (v1 == ls) ? ld : ls;
    int32_t v2 = (v1 == ms) ? md : ms;
    int32_t rs = S[E[right]];
    int f[3];
    f[left] = (S[E[left]] == v0);
    f[mid] = (S[E[mid]] == v1);
    f[right] = (rs == v2);
    (void)v0;
    out[8 + mid * 8 + f[0] * 4 + f[1] * 2 + f[2]] += 1;
}

int oracle4_brute(const int32_t *src, const int32_t *dst, const int64_t *t, uint64_t m,
                  uint32_t n, int64_t delta, uint64_t out[32]) {
    if (!out) return O4_EINVAL;
    int rc = validate(src, dst, t, m, n, delta);
    if (rc) return rc;
    memset(out, 0, 32 * sizeof(uint64_t));
    uint32_t *ord = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    if (!ord) return O4_ENOMEM;
    for (uint64_t k = 0; k < m; k++) ord[k] = (uint32_t)k;
    g_sort_t = t;
    qsort(ord, m, sizeof(uint32_t), cmp_chrono);
    for (uint64_t a = 0; a < m; a++)
        for (uint64_t b = a + 1; b < m && t[ord[b]] - t[ord[a]] <= delta; b++)
            for (uint64_t c = b + 1; c < m && t[ord[c]] - t[ord[a]] <= delta; c++) {
                uint32_t E[3] = {ord[a], ord[b], ord[c]};
                classify_triple(src, dst, E, out);
            }
    free(ord);
    return O4_OK;
}

/* ------------------------------------------------- per center / middle edge */

typedef struct {
    const int32_t *s, *d;
    const int64_t *t;
    uint64_t m;
    uint32_t n;
    uint32_t *rank;   /* edge -> chronological rank */
    uint32_t *byrank; /* rank -> edge */
    uint64_t *start;  /* n + 1: incidence list bounds */
    uint32_t *inc;    /* ranks of each node's edges, ascending */
} local_graph;

static void free_local(local_graph *g) {
    free(g->rank);
    free(g->byrank);
    free(g->start);
    free(g->inc);
}

static int make_local(local_graph *g, const int32_t *src, const int32_t *dst, const int64_t *t,
                      uint64_t m, uint32_t n) {
    memset(g, 0, sizeof(*g));
    g->s = src;
    g->d = dst;
    g->t = t;
    g->m = m;
    g->n = n;
    g->rank = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    g->byrank = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    g->start = (uint64_t *)calloc((size_t)n + 2, sizeof(uint64_t));
    g->inc = (uint32_t *)malloc(sizeof(uint32_t) * (2 * m + 1));
    if (!g->rank || !g->byrank || !g->start || !g->inc) {
        free_local(g);
        return O4_ENOMEM;
    }
    for (uint64_t k = 0; k < m; k++) g->byrank[k] = (uint32_t)k;
    g_sort_t = t;
    qsort(g->byrank, m, sizeof(uint32_t), cmp_chrono);
    for (uint64_t r = 0; r < m; r++) g->rank[g->byrank[r]] = (uint32_t)r;
    for (uint64_t k = 0; k < m; k++) {
        g->start[src[k] + 1]++;
        g->start[dst[k] + 1]++;
    }
    for (uint32_t u = 0; u < n; u++) g->start[u + 1] += g->start[u];
    uint64_t *fill = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)n + 1));
    if (!fill) {
        free_local(g);
        return O4_ENOMEM;
    }
    memcpy(fill, g->start, sizeof(uint64_t) * n);
    /* walking edges in rank order leaves every list ascending */
    for (uint64_t r = 0; r < m; r++) {
        uint32_t e = g->byrank[r];
        g->inc[fill[src[e]]++] = (uint32_t)r;
        g->inc[fill[dst[e]]++] = (uint32_t)r;
    }
    free(fill);
    return O4_OK;
}

static inline int32_t other_end(const local_graph *g, uint32_t e, int32_t u) {
    return g->s[e] == u ? g->d[e] : g->s[e];
}

/* first index i in [lo, hi) of node u's list with t >= x */
static uint64_t first_at_or_after(const local_graph *g, uint64_t lo, uint64_t hi, int64_t x) {
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (g->t[g->byrank[g->inc[mid]]] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/* stars centered at u: triples of u's edges, three distinct other ends */
static void stars_at(const local_graph *g, int32_t u, int64_t delta, uint64_t acc[32]) {
    uint64_t b = g->start[u], e = g->start[u + 1];
    for (uint64_t i = b; i < e; i++) {
        uint32_t ei = g->byrank[g->inc[i]];
        int32_t ni = other_end(g, ei, u);
        int di = g->s[ei] == u ? 0 : 1;
        for (uint64_t j = i + 1; j < e; j++) {
            uint32_t ej = g->byrank[g->inc[j]];
            if (g->t[ej] - g->t[ei] > delta) break;
            int32_t nj = other_end(g, ej, u);
            if (nj == ni) continue;
            int dj = g->s[ej] == u ? 0 : 1;
            for (uint64_t k = j + 1; k < e; k++) {
                uint32_t ek = g->byrank[g->inc[k]];
                if (g->t[ek] - g->t[ei] > delta) break;
                int32_t nk = other_end(g, ek, u);
                if (nk == ni || nk == nj) continue;
                int dk = g->s[ek] == u ? 0 : 1;
                acc[di * 4 + dj * 2 + dk] += 1;
            }
        }
    }
}

/* paths whose middle edge is the edge of rank re: one more edge x at its
   source s (other end a != d), one more edge y at its target d (other end
   w != s, w != a) */
static void paths_through(const local_graph *g, uint32_t re, int64_t delta, uint64_t acc[32]) {
    uint32_t e = g->byrank[re];
    int32_t s = g->s[e], d = g->d[e];
    int64_t te = g->t[e];
    uint64_t xs = first_at_or_after(g, g->start[s], g->start[s + 1], te - delta);
    uint64_t ys0 = first_at_or_after(g, g->start[d], g->start[d + 1], te - delta);
    for (uint64_t i = xs; i < g->start[s + 1]; i++) {
        uint32_t rx = g->inc[i];
        uint32_t x = g->byrank[rx];
        if (g->t[x] - te > delta) break;
        if (rx == re) continue;
        int32_t a = other_end(g, x, s);
        if (a == d) continue;
        for (uint64_t j = ys0; j < g->start[d + 1]; j++) {
            uint32_t ry = g->inc[j];
            uint32_t y = g->byrank[ry];
            if (g->t[y] - te > delta) break;
            if (ry == re) continue;
            int32_t w = other_end(g, y, d);
            if (w == s || w == a) continue;
            int64_t lo = te, hi = te;
            if (g->t[x] < lo) lo = g->t[x];
            if (g->t[y] < lo) lo = g->t[y];
            if (g->t[x] > hi) hi = g->t[x];
            if (g->t[y] > hi) hi = g->t[y];
            if (hi - lo > delta) continue;
            /* read the path from the earlier end edge */
            int fx, fe, fy;
            if (rx < ry) { /* a - s - d - w */
                fx = g->s[x] == a;
                fe = 1;
                fy = g->s[y] == d;
            } else { /* w - d - s - a */
                fy = g->s[y] == w;
                fe = 0;
                fx = g->s[x] == s;
            }
            /* chronological positions of e, x, y */
            uint32_t r3[3] = {re, rx, ry};
            int f3[3] = {fe, fx, fy};
            for (int p = 0; p < 3; p++)
                for (int q = p + 1; q < 3; q++)
                    if (r3[q] < r3[p]) {
                        uint32_t tr = r3[p];
                        r3[p] = r3[q];
                        r3[q] = tr;
                        int tf = f3[p];
                        f3[p] = f3[q];
                        f3[q] = tf;
                    }
            int mid = (r3[0] == re) ? 0 : (r3[1] == re ? 1 : 2);
            acc[8 + mid * 8 + f3[0] * 4 + f3[1] * 2 + f3[2]] += 1;
        }
    }
}

int oracle4_local(const int32_t *src, const int32_t *dst, const int64_t *t, uint64_t m,
                  uint32_t n, int64_t delta, int nthreads, uint64_t out[32]) {
    if (!out) return O4_EINVAL;
    int rc = validate(src, dst, t, m, n, delta);
    if (rc) return rc;
    memset(out, 0, 32 * sizeof(uint64_t));
    local_graph g;
    rc = make_local(&g, src, dst, t, m, n);
    if (rc) return rc;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        uint64_t acc[32];
        memset(acc, 0, sizeof(acc));
#pragma omp for schedule(dynamic, 64) nowait
        for (int64_t u = 0; u < (int64_t)n; u++) stars_at(&g, (int32_t)u, delta, acc);
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < (int64_t)m; r++) paths_through(&g, (uint32_t)r, delta, acc);
#pragma omp critical
        for (int k = 0; k < 32; k++) out[k] += acc[k];
    }
    free_local(&g);
    return O4_OK;
}
