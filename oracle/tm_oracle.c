/*
 * CPU oracle for exact delta-temporal motif counting (2- and 3-node, 3-edge).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * reference the HIP library is checked against.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg load it.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * This file holds "O-alg": the paper's two counting algorithms executed as the
 * paper states them, per center node:
 *   - FAST-Star (Section IV-A, Algorithm 1): for every first edge e1 of S_u,
 *     scan third edges e3 inside delta, keeping per-neighbour counts of the
 *     edges seen between them (the two HashMaps m_in / m_out and the totals
 *     #e_in / #e_out), and add to the quadruple counter Star[Type,d1,d2,d3]
 *     and the triple counter Pair[d1,d2,d3].
 *   - FAST-Tri (Section IV-B, Algorithm 2): for every pair (e_i, e_j) of S_u
 *     inside delta with different neighbours v, w, scan the node-pair edge set
 *     E_(v,w) and bin each e_k into Tri[Type,d_i,d_j,d_k] by its time position.
 *   - Merge (Sections IV-A and IV-B): isomorphic Pair cells and the three
 *     isomorphic Tri cells of each triangle motif are combined; each triangle
 *     instance is seen from its three vertices, so the Tri orbit sum is
 *     divided by three.
 *   - Parallelism (Section IV-C, inter-node mode): centers are independent;
 *     OpenMP dynamic scheduling over centers, private counters summed at the
 *     end (integer sums, so the result does not depend on the schedule).
 *
 * Readings taken where the paper is silent or garbled:
 *   - Ties: edges are totally ordered by (t, input index); every before/after
 *     test uses that order and every delta test uses t alone.
 *   - The delta bound is inclusive (t_last - t_first <= delta), as in
 *     Definition 2 and both algorithms.
 *   - Algorithm 1's direction test of e3 is read as "e3.dir == in".
 *   - Pair cells: each pair instance is seen from both of its nodes; the
 *     motif count is the Pair[o,.,.] slice (the view from the first edge's
 *     source), i.e. half of the isomorphic sum.
 *   - Triangle e_k direction is relative to v = e_i.v (o: v -> w).
 *   - Triangle types compare positions in the (t, id) order: Type I if
 *     e_k precedes e_i (and t_j - t_k <= delta), II if it lies between e_i
 *     and e_j, III if it follows e_j (and t_k - t_i <= delta).
 *   - E_(v,w) is scanned in (t, id) order starting at the first edge with
 *     t >= t_j - delta; edges before it fall in no branch of the scan.
 *   - Self-loops are rejected; |t| must be below 2^62 so differences cannot
 *     overflow.
 *
 * Raw counter layout (56 x u64): Star[3][2][2][2] | Pair[2][2][2] | Tri[3][2][2][2],
 * index order [type][d1][d2][d3] with o = 0, in = 1.
 * Motif layout (36 x u64): out[6*(row-1) + (col-1)] = M_{row,col}; see
 * oracle_layout_* below.  Only some cells of the paper's Figure 2 are fixed by
 * its text; the rest is a convention that honours all of them.  The class
 * counts themselves are pinned (brute force of the definition, closed forms,
 * the paper's worked examples); the grid positions of the cells the text does
 * not fix are parity unpinned against the paper.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_EINTERNAL (-6)

enum { DIR_O = 0, DIR_IN = 1 };

#define I_STAR(ty, a, b, c) ((ty) * 8 + (a) * 4 + (b) * 2 + (c))
#define I_PAIR(a, b, c) (24 + (a) * 4 + (b) * 2 + (c))
#define I_TRI(ty, a, b, c) (32 + (ty) * 8 + (a) * 4 + (b) * 2 + (c))

/* An edge seen from a center node u: e = (t, v, dir) (Table 1), plus the id
 * that breaks timestamp ties. */
typedef struct {
    int64_t t;
    uint32_t id;
    uint32_t v;
    int dir;
} inc_t;

static const int64_t T_LIMIT = (int64_t)1 << 62;

int oracle_validate(const int32_t *src, const int32_t *dst, const int64_t *t,
                    uint64_t m, uint32_t n) {
    if (!src || !dst || !t) return m == 0 ? OR_OK : OR_EINVAL;
    if (m >= ((uint64_t)1 << 31)) return OR_EINVAL;
    for (uint64_t e = 0; e < m; e++) {
        if (src[e] < 0 || dst[e] < 0) return OR_EINVAL;
        if ((uint32_t)src[e] >= n || (uint32_t)dst[e] >= n) return OR_EINVAL;
        if (src[e] == dst[e]) return OR_EINVAL;
        if (t[e] >= T_LIMIT || t[e] <= -T_LIMIT) return OR_EINVAL;
    }
    return OR_OK;
}

static int before(int64_t ta, uint32_t ia, int64_t tb, uint32_t ib) {
    return ta < tb || (ta == tb && ia < ib);
}

static int cmp_inc(const void *a, const void *b) {
    const inc_t *x = (const inc_t *)a, *y = (const inc_t *)b;
    if (before(x->t, x->id, y->t, y->id)) return -1;
    if (before(y->t, y->id, x->t, x->id)) return 1;
    return 0;
}

/* Per-node sequences S_u, each sorted by (t, id) (Section IV-A). */
typedef struct {
    uint64_t *off; /* n + 1 */
    inc_t *seq;    /* 2m */
} seqs_t;

static int build_sequences(const int32_t *src, const int32_t *dst, const int64_t *t,
                           uint64_t m, uint32_t n, seqs_t *S) {
    S->off = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    S->seq = (inc_t *)malloc(sizeof(inc_t) * (2 * m + 1));
    uint64_t *fill = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!S->off || !S->seq || !fill) {
        free(S->off); free(S->seq); free(fill);
        return OR_ENOMEM;
    }
    for (uint64_t e = 0; e < m; e++) {
        S->off[(uint32_t)src[e] + 1]++;
        S->off[(uint32_t)dst[e] + 1]++;
    }
    for (uint32_t u = 0; u < n; u++) S->off[u + 1] += S->off[u];
    for (uint64_t e = 0; e < m; e++) {
        uint32_t a = (uint32_t)src[e], b = (uint32_t)dst[e];
        inc_t x = {t[e], (uint32_t)e, b, DIR_O};   /* out of a */
        inc_t y = {t[e], (uint32_t)e, a, DIR_IN};  /* into b */
        S->seq[S->off[a] + fill[a]++] = x;
        S->seq[S->off[b] + fill[b]++] = y;
    }
    free(fill);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t u = 0; u < (int64_t)n; u++) {
        uint64_t lo = S->off[u], hi = S->off[u + 1];
        if (hi - lo > 1) qsort(S->seq + lo, hi - lo, sizeof(inc_t), cmp_inc);
    }
    return OR_OK;
}

/* Node-pair edge sets E_(v,w) (Algorithm 2): all edge ids sorted by
 * (min endpoint, max endpoint, t, id), so each pair's set is one contiguous,
 * time-ordered range; a per-node index of the distinct pairs finds it. */
typedef struct {
    const int32_t *src, *dst;
    const int64_t *t;
} edges_ref;
static edges_ref g_sort_ref;

static void pair_key(const edges_ref *r, uint32_t e, uint32_t *lo, uint32_t *hi) {
    uint32_t a = (uint32_t)r->src[e], b = (uint32_t)r->dst[e];
    *lo = a < b ? a : b;
    *hi = a < b ? b : a;
}

static int cmp_pair_edge(const void *pa, const void *pb) {
    uint32_t x = *(const uint32_t *)pa, y = *(const uint32_t *)pb;
    uint32_t xl, xh, yl, yh;
    pair_key(&g_sort_ref, x, &xl, &xh);
    pair_key(&g_sort_ref, y, &yl, &yh);
    if (xl != yl) return xl < yl ? -1 : 1;
    if (xh != yh) return xh < yh ? -1 : 1;
    if (before(g_sort_ref.t[x], x, g_sort_ref.t[y], y)) return -1;
    if (before(g_sort_ref.t[y], y, g_sort_ref.t[x], x)) return 1;
    return 0;
}

typedef struct {
    uint32_t *ids;    /* m edge ids, pair-sorted */
    uint64_t *plo;    /* n + 1: distinct pairs whose min endpoint is u */
    uint32_t *p_hi;   /* per distinct pair: max endpoint */
    uint64_t *p_beg;  /* per distinct pair: first index in ids (+ sentinel) */
} pair_sets;

static void free_pair_sets(pair_sets *P) {
    free(P->ids); free(P->plo); free(P->p_hi); free(P->p_beg);
}

static int build_pair_sets(const int32_t *src, const int32_t *dst, const int64_t *t,
                           uint64_t m, uint32_t n, pair_sets *P) {
    memset(P, 0, sizeof(*P));
    P->ids = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    P->plo = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    P->p_hi = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    P->p_beg = (uint64_t *)malloc(sizeof(uint64_t) * (m + 2));
    if (!P->ids || !P->plo || !P->p_hi || !P->p_beg) {
        free_pair_sets(P);
        return OR_ENOMEM;
    }
    for (uint64_t e = 0; e < m; e++) P->ids[e] = (uint32_t)e;
    g_sort_ref.src = src;
    g_sort_ref.dst = dst;
    g_sort_ref.t = t;
    qsort(P->ids, m, sizeof(uint32_t), cmp_pair_edge);
    uint64_t np = 0;
    uint32_t pl = 0, ph = 0;
    for (uint64_t k = 0; k < m; k++) {
        uint32_t l, h;
        pair_key(&g_sort_ref, P->ids[k], &l, &h);
        if (k == 0 || l != pl || h != ph) {
            P->p_hi[np] = h;
            P->p_beg[np] = k;
            P->plo[l + 1]++;
            np++;
            pl = l;
            ph = h;
        }
    }
    P->p_beg[np] = m;
    for (uint32_t u = 0; u < n; u++) P->plo[u + 1] += P->plo[u];
    return OR_OK;
}

/* Range [*b, *e) of E_(lo,hi) in the pair-sorted ids; empty if no such edge. */
static void pair_range(const pair_sets *P, uint32_t lo, uint32_t hi, uint64_t *b, uint64_t *e) {
    uint64_t x = P->plo[lo], y = P->plo[lo + 1];
    while (x < y) {
        uint64_t mid = x + (y - x) / 2;
        if (P->p_hi[mid] < hi) x = mid + 1;
        else y = mid;
    }
    if (x < P->plo[lo + 1] && P->p_hi[x] == hi) {
        *b = P->p_beg[x];
        *e = P->p_beg[x + 1];
    } else {
        *b = *e = 0;
    }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (FAST-Star) for one center.  m_in / m_out are the two maps of
 * the algorithm, stored as dense per-neighbour arrays (zero outside the
 * current e1) with a list of touched keys for the reset. */
typedef struct {
    uint64_t *m_cnt[2]; /* indexed by neighbour id, per direction */
    uint32_t *touched;
    uint64_t ntouched;
} star_maps;

static void fast_star_center(const inc_t *S, uint64_t s, int64_t delta, star_maps *mp,
                             uint64_t *raw) {
    for (uint64_t i = 0; i + 2 < s; i++) {          /* i = 1 .. s-2 */
        const inc_t e1 = S[i];
        uint64_t n_e[2] = {0, 0};                 /* #e_o, #e_in */
        for (uint64_t k = 0; k < mp->ntouched; k++) {  /* HashMap.Init() */
            mp->m_cnt[0][mp->touched[k]] = 0;
            mp->m_cnt[1][mp->touched[k]] = 0;
        }
        mp->ntouched = 0;
        for (uint64_t j = i + 1; j < s; j++) {
            const inc_t e3 = S[j];
            if (e3.t - e1.t > delta) break;
            if (e3.v == e1.v) {
                for (int d = 0; d < 2; d++) {
                    uint64_t mv = mp->m_cnt[d][e1.v];
                    raw[I_PAIR(e1.dir, d, e3.dir)] += mv;
                    raw[I_STAR(1, e1.dir, d, e3.dir)] += n_e[d] - mv;
                }
            } else {
                for (int d = 0; d < 2; d++) {
                    raw[I_STAR(0, e1.dir, d, e3.dir)] += mp->m_cnt[d][e3.v];
                    raw[I_STAR(2, e1.dir, d, e3.dir)] += mp->m_cnt[d][e1.v];
                }
            }
            if (mp->m_cnt[0][e3.v] == 0 && mp->m_cnt[1][e3.v] == 0)
                mp->touched[mp->ntouched++] = e3.v;
            mp->m_cnt[e3.dir][e3.v] += 1;
            n_e[e3.dir] += 1;
        }
    }
}

/* Algorithm 2 (FAST-Tri) for one center; every triangle instance is found
 * from each of its three vertices. */
static void fast_tri_center(const inc_t *S, uint64_t s, int64_t delta, const edges_ref *r,
                            const pair_sets *P, uint64_t *raw) {
    for (uint64_t i = 0; i + 1 < s; i++) {
        const inc_t ei = S[i];
        for (uint64_t j = i + 1; j < s; j++) {
            const inc_t ej = S[j];
            if (ej.t > ei.t + delta) break;
            if (ej.v == ei.v) continue;
            uint32_t v = ei.v, w = ej.v;
            uint32_t lo = v < w ? v : w, hi = v < w ? w : v;
            uint64_t a, e_end;
            pair_range(P, lo, hi, &a, &e_end);
            /* first edge of E_(v,w) with t >= t_j - delta */
            uint64_t x = a, y = e_end;
            while (x < y) {
                uint64_t mid = x + (y - x) / 2;
                if (r->t[P->ids[mid]] < ej.t - delta) x = mid + 1;
                else y = mid;
            }
            uint64_t b = x;
            for (uint64_t q = b; q < e_end; q++) {
                uint32_t ek = P->ids[q];
                int64_t tk = r->t[ek];
                if (tk > ei.t + delta) break;
                int dk = ((uint32_t)r->src[ek] == v) ? DIR_O : DIR_IN;
                int type;
                if (before(tk, ek, ei.t, ei.id)) {
                    if (ej.t - tk > delta) continue;
                    type = 0;
                } else if (before(tk, ek, ej.t, ej.id)) {
                    type = 1;
                } else {
                    if (tk - ei.t > delta) continue;
                    type = 2;
                }
                raw[I_TRI(type, ei.dir, ej.dir, dk)] += 1;
            }
        }
    }
}

typedef struct {
    seqs_t S;
    pair_sets P;
    uint32_t n;
    uint64_t m;
    uint64_t max_deg;
    edges_ref ref;
} oracle_graph;

static void free_graph(oracle_graph *g) {
    free(g->S.off);
    free(g->S.seq);
    free_pair_sets(&g->P);
}

static int prepare(const int32_t *src, const int32_t *dst, const int64_t *t, uint64_t m,
                   uint32_t n, oracle_graph *g) {
    memset(g, 0, sizeof(*g));
    int rc = oracle_validate(src, dst, t, m, n);
    if (rc) return rc;
    g->n = n;
    g->m = m;
    g->ref.src = src;
    g->ref.dst = dst;
    g->ref.t = t;
    rc = build_sequences(src, dst, t, m, n, &g->S);
    if (rc) return rc;
    rc = build_pair_sets(src, dst, t, m, n, &g->P);
    if (rc) {
        free(g->S.off);
        free(g->S.seq);
        return rc;
    }
    for (uint32_t u = 0; u < n; u++) {
        uint64_t d = g->S.off[u + 1] - g->S.off[u];
        if (d > g->max_deg) g->max_deg = d;
    }
    return OR_OK;
}

/* Count the raw counters contributed by the centers listed in `centers`
 * (all centers when centers == NULL). */
static int count_centers(oracle_graph *g, int64_t delta, const uint32_t *centers,
                         uint64_t ncent, int nthreads, uint64_t raw[56]) {
    memset(raw, 0, 56 * sizeof(uint64_t));
    uint64_t total = centers ? ncent : g->n;
    int ok = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        uint64_t loc[56];
        memset(loc, 0, sizeof(loc));
        star_maps mp;
        mp.m_cnt[0] = (uint64_t *)calloc((size_t)g->n + 1, sizeof(uint64_t));
        mp.m_cnt[1] = (uint64_t *)calloc((size_t)g->n + 1, sizeof(uint64_t));
        mp.touched = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)g->max_deg + 1));
        mp.ntouched = 0;
        if (!mp.m_cnt[0] || !mp.m_cnt[1] || !mp.touched) {
#pragma omp atomic write
            ok = 0;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t k = 0; k < (int64_t)total; k++) {
                uint32_t u = centers ? centers[k] : (uint32_t)k;
                if (u >= g->n) continue;
                const inc_t *S = g->S.seq + g->S.off[u];
                uint64_t s = g->S.off[u + 1] - g->S.off[u];
                fast_star_center(S, s, delta, &mp, loc);
                fast_tri_center(S, s, delta, &g->ref, &g->P, loc);
            }
        }
#pragma omp critical
        for (int c = 0; c < 56; c++) raw[c] += loc[c];
        free(mp.m_cnt[0]);
        free(mp.m_cnt[1]);
        free(mp.touched);
    }
    return ok ? OR_OK : OR_ENOMEM;
}

/* ------------------------------------------------------------------------ */
/* 36-cell layout (oracle's own copy).  Anchors fixed by the paper's text:
 * M24 = Star[I,in,o,in] (Section IV-A), M63 = Star[III,o,o,in] and the
 * instances named for M46 and M65 (Section III), M25 (Section IV-B's
 * three-view example), M26 = the time-respecting 3-cycle, M55/M56/M65 =
 * the pair cells (Section IV-A), M66 the remaining pair class. */
static int cell(int row, int col) { return 6 * (row - 1) + (col - 1); }

int oracle_layout_star(int type, int d1, int d2, int d3) {
    int row = 1 + 2 * type + (d3 == DIR_IN);
    int col = 1 + 2 * (d2 == DIR_O) + (d1 == DIR_IN);
    return cell(row, col);
}

int oracle_layout_tri(int a, int b, int c) {
    int col = 5 + (b == DIR_O);
    int ab = (a == b), cb = (c == b);
    int row = ab ? (cb ? 1 : 4) : (cb ? 3 : 2);
    return cell(row, col);
}

int oracle_layout_pair(int d2, int d3) { /* first edge leaves the pair's source */
    if (d2 == DIR_O && d3 == DIR_O) return cell(5, 5);
    if (d2 == DIR_IN && d3 == DIR_IN) return cell(5, 6);
    if (d2 == DIR_IN && d3 == DIR_O) return cell(6, 5);
    return cell(6, 6);
}

/* Merge the paper's counters into the 36 motif counts.  Returns
 * OR_EINTERNAL if the symmetries every exact count must satisfy fail. */
int oracle_merge(const uint64_t raw[56], uint64_t out[36]) {
    uint64_t res[36];
    memset(res, 0, sizeof(res));
    for (int ty = 0; ty < 3; ty++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                for (int c = 0; c < 2; c++)
                    res[oracle_layout_star(ty, a, b, c)] += raw[I_STAR(ty, a, b, c)];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int c = 0; c < 2; c++)
                if (raw[I_PAIR(a, b, c)] != raw[I_PAIR(1 - a, 1 - b, 1 - c)]) return OR_EINTERNAL;
    for (int b = 0; b < 2; b++)
        for (int c = 0; c < 2; c++) res[oracle_layout_pair(b, c)] += raw[I_PAIR(DIR_O, b, c)];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int c = 0; c < 2; c++) {
                uint64_t x = raw[I_TRI(0, a, b, c)];
                uint64_t y = raw[I_TRI(1, 1 - c, 1 - b, 1 - a)];
                uint64_t z = raw[I_TRI(2, c, 1 - a, 1 - b)];
                uint64_t sum = x + y + z;
                if (sum % 3 != 0 || x != y || y != z) return OR_EINTERNAL;
                res[oracle_layout_tri(a, b, c)] += sum / 3;
            }
    memcpy(out, res, sizeof(res));
    return OR_OK;
}

/* Whole-graph raw counters. */
int oracle_alg(const int32_t *src, const int32_t *dst, const int64_t *t, uint64_t m,
               uint32_t n, int64_t delta, int nthreads, uint64_t raw[56]) {
    if (delta < 0 || delta >= T_LIMIT || !raw) return OR_EINVAL;
    oracle_graph g;
    int rc = prepare(src, dst, t, m, n, &g);
    if (rc) return rc;
    rc = count_centers(&g, delta, NULL, 0, nthreads, raw);
    free_graph(&g);
    return rc;
}

/* Raw counters contributed by the listed centers only (per-center checks). */
int oracle_alg_centers(const int32_t *src, const int32_t *dst, const int64_t *t, uint64_t m,
                       uint32_t n, int64_t delta, const uint32_t *centers, uint64_t ncent,
                       int nthreads, uint64_t raw[56]) {
    if (delta < 0 || delta >= T_LIMIT || !raw || (!centers && ncent)) return OR_EINVAL;
    oracle_graph g;
    int rc = prepare(src, dst, t, m, n, &g);
    if (rc) return rc;
    rc = count_centers(&g, delta, centers, ncent, nthreads, raw);
    free_graph(&g);
    return rc;
}
