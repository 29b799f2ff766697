/*
 * fnn_oracle.c -- CPU oracle for exact fixed-radius (epsilon) near-neighbour
 * graphs in a general metric space.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg call it.  It shares no code, header, table
 * or helper with the GPU library; the two are built separately and neither
 * includes or links the other.
 *
 * Everything here is plain, slow and sequential per pair: FP64, IEEE
 * round-to-nearest, no FMA contraction (built with -ffp-contract=off), sums
 * taken k = 0..d-1 in order.  OpenMP is used only across rows / queries.
 *
 * What is computed (paper, Section III "Definitions" and Section IV-A/B):
 *   - the epsilon-graph E = {(p,q) : d(p,q) <= eps} (Definitions), read as
 *     ordered pairs with p != q, duplicates kept as separate vertices;
 *   - the batch cover-tree construction: vertex splitting (Algorithm 1) driven
 *     level by level (Algorithm 2), leaf vertex size zeta;
 *   - the single-point cover-tree range query (Algorithm 3);
 *   - a checker for the cover-tree invariants (nesting, covering 2^k, sibling
 *     separation; Definitions, "cover tree" and the relaxed separating
 *     property) plus the split invariants of Section IV-A.
 *
 * Pinned predicates (the definition of an edge that every result is compared
 * against; the paper does not fix a precision):
 *   L2          s = sum_k (x_k - y_k)*(x_k - y_k);   edge <=> s <= E2, E2 = eps*eps
 *   angular     g = sum x_k y_k, a = sum x_k^2, b = sum y_k^2, C = cos(eps)
 *               t = ((C*C)*a)*b
 *               C >= 0: edge <=> g >= 0 && g*g >= t
 *               C <  0: edge <=> g >= 0 || g*g <= t
 *               (theta = arccos of the cosine; eps >= pi => C = -1)
 *   Hamming     h = sum_w popcount(x_w ^ y_w);       edge <=> h <= floor(eps)
 *   Levenshtein unit-cost edit distance;             edge <=> lev <= floor(eps)
 * Reported distances: sqrt(s); 2*atan2(|xh-yh|, |xh+yh|) with xh = x/|x|
 * (Kahan's angle formula); h; lev.
 *
 * Comparisons against a power of two tau = 2^k inside the tree ("within
 * tau"): L2 compares s <= 4^k (exact); angular uses the angular predicate with
 * C = cos(tau); Hamming / Levenshtein compare the integer distance.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_L2 0
#define ORC_ANG 1
#define ORC_HAM 2
#define ORC_LEV 3

#define LEV_PAD 0xFF

/* ------------------------------------------------------------------------ */
/* Metric primitives (Definitions: metric space; distances named there)     */
/* ------------------------------------------------------------------------ */

double orc_l2_sq(const float *x, const float *y, int32_t d)
{
    double s = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double t = (double)x[k] - (double)y[k];
        s = s + t * t;
    }
    return s;
}

void orc_ang_terms(const float *x, const float *y, int32_t d,
                   double *g, double *a, double *b)
{
    double gg = 0.0, aa = 0.0, bb = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double xk = (double)x[k], yk = (double)y[k];
        gg = gg + xk * yk;
        aa = aa + xk * xk;
        bb = bb + yk * yk;
    }
    *g = gg;
    *a = aa;
    *b = bb;
}

int orc_ang_pred(double g, double a, double b, double C)
{
    double t = ((C * C) * a) * b;
    double g2 = g * g;
    if (C >= 0.0)
        return g >= 0.0 && g2 >= t;
    return g >= 0.0 || g2 <= t;
}

double orc_ang_dist(const float *x, const float *y, int32_t d)
{
    double a = 0.0, b = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        a = a + (double)x[k] * (double)x[k];
        b = b + (double)y[k] * (double)y[k];
    }
    double na = sqrt(a), nb = sqrt(b);
    double u = 0.0, v = 0.0;
    for (int32_t k = 0; k < d; ++k) {
        double xh = (double)x[k] / na, yh = (double)y[k] / nb;
        double m = xh - yh, p = xh + yh;
        u = u + m * m;
        v = v + p * p;
    }
    return 2.0 * atan2(sqrt(u), sqrt(v));
}

int32_t orc_ham(const uint64_t *x, const uint64_t *y, int32_t words)
{
    int32_t h = 0;
    for (int32_t w = 0; w < words; ++w)
        h += __builtin_popcountll(x[w] ^ y[w]);
    return h;
}

int32_t orc_str_len(const uint8_t *s, int32_t stride)
{
    int32_t l = 0;
    while (l < stride && s[l] != LEV_PAD)
        ++l;
    return l;
}

/* Wagner-Fischer dynamic programme, unit costs, two rows. */
int32_t orc_lev(const uint8_t *a, int32_t la, const uint8_t *b, int32_t lb)
{
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    for (int32_t j = 0; j <= lb; ++j)
        prev[j] = j;
    for (int32_t i = 1; i <= la; ++i) {
        cur[0] = i;
        for (int32_t j = 1; j <= lb; ++j) {
            int32_t sub = prev[j - 1] + (a[i - 1] != b[j - 1]);
            int32_t del = prev[j] + 1;
            int32_t ins = cur[j - 1] + 1;
            int32_t m = sub < del ? sub : del;
            cur[j] = m < ins ? m : ins;
        }
        int32_t *t = prev;
        prev = cur;
        cur = t;
    }
    int32_t r = prev[lb];
    free(prev);
    free(cur);
    return r;
}

/* Same recurrence restricted to the band |i-j| <= k (Ukkonen); cells outside
 * the band count as k+1.  Returns min(lev, k+1), which decides lev <= k
 * exactly and equals lev whenever lev <= k. */
int32_t orc_lev_banded(const uint8_t *a, int32_t la, const uint8_t *b,
                       int32_t lb, int32_t k)
{
    int32_t diff = la > lb ? la - lb : lb - la;
    if (diff > k)
        return k + 1;
    int32_t big = k + 1;
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lb + 1));
    for (int32_t j = 0; j <= lb; ++j)
        prev[j] = j <= k ? j : big;
    for (int32_t i = 1; i <= la; ++i) {
        int32_t lo = i - k < 1 ? 1 : i - k;
        int32_t hi = i + k > lb ? lb : i + k;
        cur[0] = i <= k ? i : big;
        if (lo > 1)
            cur[lo - 1] = big;
        for (int32_t j = lo; j <= hi; ++j) {
            int32_t sub = prev[j - 1] + (a[i - 1] != b[j - 1]);
            int32_t del = (j <= i - 1 + k) ? prev[j] + 1 : big;
            int32_t ins = cur[j - 1] + 1;
            int32_t m = sub < del ? sub : del;
            m = m < ins ? m : ins;
            cur[j] = m > big ? big : m;
        }
        if (hi < lb)
            cur[hi + 1] = big;
        int32_t *t = prev;
        prev = cur;
        cur = t;
    }
    int32_t r = prev[lb];
    free(prev);
    free(cur);
    return r > big ? big : r;
}

/* ------------------------------------------------------------------------ */
/* Point-set view                                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int metric;
    int64_t n;
    int32_t dim;       /* coordinates (L2/ang), bits (Hamming), stride (Lev) */
    const void *pts;
    int32_t *len;      /* Levenshtein lengths (owned) */
} pset;

static void pset_init(pset *P, int metric, const void *pts, int64_t n,
                      int32_t dim)
{
    P->metric = metric;
    P->n = n;
    P->dim = dim;
    P->pts = pts;
    P->len = NULL;
    if (metric == ORC_LEV) {
        P->len = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        const uint8_t *s = (const uint8_t *)pts;
        for (int64_t i = 0; i < n; ++i)
            P->len[i] = orc_str_len(s + i * (int64_t)dim, dim);
    }
}

static void pset_free(pset *P)
{
    free(P->len);
    P->len = NULL;
}

static const float *fpt(const pset *P, int64_t i)
{
    return (const float *)P->pts + i * (int64_t)P->dim;
}
static const uint64_t *hpt(const pset *P, int64_t i)
{
    return (const uint64_t *)P->pts + i * (int64_t)(P->dim / 64);
}
static const uint8_t *spt(const pset *P, int64_t i)
{
    return (const uint8_t *)P->pts + i * (int64_t)P->dim;
}

/* The metric's threshold parameter for a given eps. */
double orc_eps_param(int metric, double eps)
{
    switch (metric) {
    case ORC_L2:
        return eps * eps;
    case ORC_ANG:
        return eps >= M_PI ? -1.0 : cos(eps);
    default:
        return floor(eps);
    }
}

/* FP64 distance d(i, j). */
static double pdist(const pset *P, int64_t i, int64_t j)
{
    switch (P->metric) {
    case ORC_L2:
        return sqrt(orc_l2_sq(fpt(P, i), fpt(P, j), P->dim));
    case ORC_ANG:
        return orc_ang_dist(fpt(P, i), fpt(P, j), P->dim);
    case ORC_HAM:
        return (double)orc_ham(hpt(P, i), hpt(P, j), P->dim / 64);
    default:
        return (double)orc_lev(spt(P, i), P->len[i], spt(P, j), P->len[j]);
    }
}

/* Ordering key for "farthest point" searches; exactly monotone with the
 * within-tau comparisons for L2 (squared distance), Hamming and Levenshtein,
 * and the angle itself for the angular metric. */
static double pkey(const pset *P, int64_t i, int64_t j)
{
    if (P->metric == ORC_L2)
        return orc_l2_sq(fpt(P, i), fpt(P, j), P->dim);
    return pdist(P, i, j);
}

static double key_to_dist(const pset *P, double key)
{
    return P->metric == ORC_L2 ? sqrt(key) : key;
}

/* Pinned edge predicate for the pair (i, j); writes the FP64 distance. */
static int pedge(const pset *P, int64_t i, int64_t j, double param,
                 double *dist)
{
    switch (P->metric) {
    case ORC_L2: {
        double s = orc_l2_sq(fpt(P, i), fpt(P, j), P->dim);
        if (s <= param) {
            *dist = sqrt(s);
            return 1;
        }
        return 0;
    }
    case ORC_ANG: {
        double g, a, b;
        orc_ang_terms(fpt(P, i), fpt(P, j), P->dim, &g, &a, &b);
        if (orc_ang_pred(g, a, b, param)) {
            *dist = orc_ang_dist(fpt(P, i), fpt(P, j), P->dim);
            return 1;
        }
        return 0;
    }
    case ORC_HAM: {
        int32_t h = orc_ham(hpt(P, i), hpt(P, j), P->dim / 64);
        if ((double)h <= param) {
            *dist = (double)h;
            return 1;
        }
        return 0;
    }
    default: {
        int32_t k = (int32_t)param;
        int32_t l = orc_lev_banded(spt(P, i), P->len[i], spt(P, j), P->len[j],
                                   k);
        if (l <= k) {
            *dist = (double)l;
            return 1;
        }
        return 0;
    }
    }
}

/* "d(i,j) <= 2^lvl" under the pinned comparison for the metric. */
static int pwithin(const pset *P, int64_t i, int64_t j, int32_t lvl)
{
    switch (P->metric) {
    case ORC_L2:
        return orc_l2_sq(fpt(P, i), fpt(P, j), P->dim) <= ldexp(1.0, 2 * lvl);
    case ORC_ANG: {
        double g, a, b;
        double tau = ldexp(1.0, lvl);
        double C = tau >= M_PI ? -1.0 : cos(tau);
        orc_ang_terms(fpt(P, i), fpt(P, j), P->dim, &g, &a, &b);
        return orc_ang_pred(g, a, b, C);
    }
    default:
        return pdist(P, i, j) <= ldexp(1.0, lvl);
    }
}

/* Smallest integer l with d <= 2^l for the largest key of a set (level of a
 * vertex whose radius corresponds to key kmax > 0). */
static int32_t level_of_key(const pset *P, double kmax)
{
    int e;
    double d = key_to_dist(P, kmax);
    (void)frexp(d, &e);
    int32_t l = e;
    if (P->metric == ORC_L2) {
        while (ldexp(1.0, 2 * (l - 1)) >= kmax)
            --l;
        while (ldexp(1.0, 2 * l) < kmax)
            ++l;
    } else {
        while (ldexp(1.0, l - 1) >= d)
            --l;
        while (ldexp(1.0, l) < d)
            ++l;
    }
    return l;
}

/* ------------------------------------------------------------------------ */
/* Brute force: the definition of the epsilon-graph, all ordered pairs.     */
/* rows == NULL means every row 0..n-1; otherwise the listed rows, in order */
/* (used for sampled checks at full size).                                  */
/* ------------------------------------------------------------------------ */

int64_t orc_bf_count(int metric, const void *pts, int64_t n, int32_t dim,
                     double eps, const int64_t *rows, int64_t nrows,
                     int64_t *deg)
{
    pset P;
    pset_init(&P, metric, pts, n, dim);
    double param = orc_eps_param(metric, eps);
    int64_t R = rows ? nrows : n;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t r = 0; r < R; ++r) {
        int64_t i = rows ? rows[r] : r;
        int64_t c = 0;
        double dd;
        for (int64_t j = 0; j < n; ++j)
            if (j != i && pedge(&P, i, j, param, &dd))
                ++c;
        deg[r] = c;
        total += c;
    }
    pset_free(&P);
    return total;
}

void orc_bf_fill(int metric, const void *pts, int64_t n, int32_t dim,
                 double eps, const int64_t *rows, int64_t nrows,
                 const int64_t *row_ptr, int32_t *col, double *dist)
{
    pset P;
    pset_init(&P, metric, pts, n, dim);
    double param = orc_eps_param(metric, eps);
    int64_t R = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < R; ++r) {
        int64_t i = rows ? rows[r] : r;
        int64_t o = row_ptr[r];
        double dd;
        for (int64_t j = 0; j < n; ++j)
            if (j != i && pedge(&P, i, j, param, &dd)) {
                col[o] = (int32_t)j;
                dist[o] = dd;
                ++o;
            }
    }
    pset_free(&P);
}

/* Pairwise FP64 distances of listed rows against all points (calibration). */
void orc_rows_dist(int metric, const void *pts, int64_t n, int32_t dim,
                   const int64_t *rows, int64_t nrows, double *out)
{
    pset P;
    pset_init(&P, metric, pts, n, dim);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nrows; ++r)
        for (int64_t j = 0; j < n; ++j)
            out[r * n + j] = pdist(&P, rows[r], j);
    pset_free(&P);
}

/* ------------------------------------------------------------------------ */
/* Cover tree: batch construction (Algorithms 1 and 2)                      */
/*                                                                          */
/* Tree layout shared by the builder and the checker:                       */
/*   order[n]              original point ids in tree order                 */
/*   node arrays [nnodes]: center (original id), radius (FP64 distance),    */
/*     level, child_begin / child_count (children are consecutive nodes),   */
/*     pt_begin / pt_end (the node's points are order[pt_begin:pt_end]).    */
/*   A node with child_count == 0 is a leaf block: each of its points is a  */
/*   leaf vertex B(p, 0) (Algorithm 2); a block of one point is a single    */
/*   leaf.  Node 0 is the root.                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t node;    /* tree node this hub expands */
    int32_t level;   /* split level l; children sit at l-1 */
} hub_t;

/* Returns the number of nodes, or -1 on failure.  Arrays must hold 2n
 * nodes.  key[] is scratch of n doubles; label[] scratch of n int32. */
int64_t orc_tree_build(int metric, const void *pts, int64_t n, int32_t dim,
                       int32_t zeta, int32_t *order, int32_t *center,
                       double *radius, int32_t *level, int32_t *child_begin,
                       int32_t *child_count, int32_t *pt_begin,
                       int32_t *pt_end)
{
    if (n <= 0 || zeta < 1)
        return -1;
    pset P;
    pset_init(&P, metric, pts, n, dim);
    double *key = (double *)malloc(sizeof(double) * (size_t)n);
    int32_t *lab = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *ktmp = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t cap = 2 * n + 1;
    hub_t *hubs = (hub_t *)malloc(sizeof(hub_t) * (size_t)cap);
    hub_t *next = (hub_t *)malloc(sizeof(hub_t) * (size_t)cap);
    int32_t *cent = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);

    /* Root: the point with input index 0; D[p] = d(p, root). */
    for (int64_t i = 0; i < n; ++i) {
        order[i] = (int32_t)i;
        key[i] = pkey(&P, 0, i);
    }
    int64_t nn = 1;
    double kmax = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (key[i] > kmax)
            kmax = key[i];
    center[0] = 0;
    radius[0] = key_to_dist(&P, kmax);
    pt_begin[0] = 0;
    pt_end[0] = (int32_t)n;
    child_begin[0] = 0;
    child_count[0] = 0;
    int64_t nh = 0;
    if (n > zeta && kmax > 0.0) {
        level[0] = level_of_key(&P, kmax);
        hubs[nh].node = 0;
        hubs[nh].level = level[0];
        ++nh;
    } else {
        level[0] = kmax > 0.0 ? level_of_key(&P, kmax) : INT32_MIN / 2;
    }

    /* BuildLevel: split every hub of the current level, collect new hubs. */
    while (nh > 0) {
        int64_t nnext = 0;
        for (int64_t h = 0; h < nh; ++h) {
            int32_t v = hubs[h].node;
            int32_t l = hubs[h].level;
            int32_t b = pt_begin[v], e = pt_end[v];
            /* SplitVertex (Algorithm 1).  key[] holds D for this hub's
             * points (distance to pi_1); label 0 = pi_1. */
            int32_t m = 1;
            cent[0] = center[v];
            for (int32_t i = b; i < e; ++i)
                lab[i] = 0;
            for (;;) {
                /* farthest point pi_{m+1}: first maximum in tree order among
                 * points not certified to lie within 2^{l-1} of their
                 * centre.  For L2/Hamming/Levenshtein the key order agrees
                 * exactly with the within test; for the angle a narrow band
                 * around the threshold is resolved by the pinned test. */
                int32_t far = -1;
                double best = -1.0;
                double tau = ldexp(1.0, l - 1);
                for (int32_t i = b; i < e; ++i) {
                    double kk = key[i];
                    if (!(kk > best))
                        continue;
                    int covered;
                    if (P.metric == ORC_L2)
                        covered = kk <= ldexp(1.0, 2 * (l - 1));
                    else if (P.metric == ORC_ANG) {
                        if (kk < tau * (1.0 - 1e-9))
                            covered = 1;
                        else if (kk > tau * (1.0 + 1e-9))
                            covered = 0;
                        else
                            covered = pwithin(&P, order[i], cent[lab[i]],
                                              l - 1);
                    } else
                        covered = kk <= tau;
                    if (!covered) {
                        best = kk;
                        far = i;
                    }
                }
                if (far < 0)
                    break; /* every point is within 2^{l-1}: stop */
                int32_t pm = order[far];
                cent[m] = pm;
                for (int32_t i = b; i < e; ++i) {
                    double kk = pkey(&P, order[i], pm);
                    if (kk < key[i]) {
                        key[i] = kk;
                        lab[i] = m;
                    }
                }
                ++m;
            }
            /* Children H_i = {p : L[p] = pi_i}, stable in tree order. */
            int32_t *cnt = (int32_t *)calloc((size_t)m + 1, sizeof(int32_t));
            for (int32_t i = b; i < e; ++i)
                cnt[lab[i] + 1]++;
            for (int32_t c = 0; c < m; ++c)
                cnt[c + 1] += cnt[c];
            for (int32_t i = b; i < e; ++i) {
                int32_t pos = b + cnt[lab[i]]++;
                tmp[pos] = order[i];
                ktmp[pos] = key[i];
            }
            for (int32_t i = b; i < e; ++i) {
                order[i] = tmp[i];
                key[i] = ktmp[i];
            }
            /* cnt[c] now holds the end offset of child c (relative to b) */
            child_begin[v] = (int32_t)nn;
            child_count[v] = m;
            int32_t s = b;
            for (int32_t c = 0; c < m; ++c) {
                int32_t cb = s, ce = b + cnt[c];
                s = ce;
                int64_t u = nn++;
                double ck = 0.0;
                for (int32_t i = cb; i < ce; ++i)
                    if (key[i] > ck)
                        ck = key[i];
                center[u] = cent[c];
                radius[u] = key_to_dist(&P, ck);
                level[u] = l - 1;
                pt_begin[u] = cb;
                pt_end[u] = ce;
                child_begin[u] = 0;
                child_count[u] = 0;
                /* Algorithm 2: more than zeta points -> hub of the next
                 * round; otherwise a block of leaves B(p,0).  A child whose
                 * points all coincide with its centre (radius 0) holds
                 * duplicates and stays one leaf block of any size. */
                if (ce - cb > zeta && ck > 0.0) {
                    int32_t lc = level_of_key(&P, ck);
                    level[u] = lc;
                    next[nnext].node = (int32_t)u;
                    next[nnext].level = lc;
                    ++nnext;
                }
            }
            free(cnt);
        }
        hub_t *t = hubs;
        hubs = next;
        next = t;
        nh = nnext;
    }
    free(key);
    free(lab);
    free(tmp);
    free(ktmp);
    free(hubs);
    free(next);
    free(cent);
    pset_free(&P);
    return nn;
}

/* ------------------------------------------------------------------------ */
/* Cover tree query (Algorithm 3), one query point at a time, all points of */
/* the set as queries.  Pruning keeps v when d(q,v) <= radius(v) + eps; a   */
/* relative slack of 1e-9 (plus 1e-6 absolute for the angle, whose pinned   */
/* test works on the cosine) keeps FP64 rounding from dropping an edge.     */
/* Leaves are decided by the pinned predicate.  Two passes: count, fill.    */
/* ------------------------------------------------------------------------ */

static int64_t query_one(const pset *P, int64_t q, double eps, double param,
                         const int32_t *order, const int32_t *center,
                         const double *radius, const int32_t *child_begin,
                         const int32_t *child_count, const int32_t *pt_begin,
                         const int32_t *pt_end, int32_t *stack, int32_t *col,
                         double *dist)
{
    int64_t found = 0;
    int64_t sp = 0;
    double abs_slack = P->metric == ORC_ANG ? 1e-6 : 0.0;
    /* Stack entries: node id >= 0, or a leaf point encoded as -(id+1). */
    stack[sp++] = 0;
    while (sp > 0) {
        int32_t u = stack[--sp];
        if (u < 0) {
            int64_t p = -(int64_t)u - 1;
            double dd;
            if (p != q && pedge(P, q, p, param, &dd)) {
                if (col) {
                    col[found] = (int32_t)p;
                    dist[found] = dd;
                }
                ++found;
            }
            continue;
        }
        if (child_count[u] == 0) {
            /* leaf block: its leaves B(p,0) are the children */
            for (int32_t i = pt_begin[u]; i < pt_end[u]; ++i) {
                int64_t p = order[i];
                double d = pdist(P, q, p);
                if (d <= eps * (1.0 + 1e-9) + abs_slack)
                    stack[sp++] = -(int32_t)p - 1;
            }
            continue;
        }
        for (int32_t c = 0; c < child_count[u]; ++c) {
            int32_t v = child_begin[u] + c;
            double d = pdist(P, q, center[v]);
            if (d <= (radius[v] + eps) * (1.0 + 1e-9) + abs_slack)
                stack[sp++] = v;
        }
    }
    return found;
}

static int cmp_col(const void *a, const void *b)
{
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    return (x[0] > y[0]) - (x[0] < y[0]);
}

int64_t orc_tree_query(int metric, const void *pts, int64_t n, int32_t dim,
                       double eps, const int32_t *order,
                       const int32_t *center, const double *radius,
                       const int32_t *child_begin, const int32_t *child_count,
                       const int32_t *pt_begin, const int32_t *pt_end,
                       int64_t nnodes, int64_t *row_ptr, int32_t *col,
                       double *dist)
{
    pset P;
    pset_init(&P, metric, pts, n, dim);
    double param = orc_eps_param(metric, eps);
    int64_t stack_cap = nnodes + n + 16;
    if (!col) {
        int64_t total = 0;
#pragma omp parallel
        {
            int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)stack_cap);
#pragma omp for schedule(dynamic, 8) reduction(+ : total)
            for (int64_t q = 0; q < n; ++q) {
                int64_t c = query_one(&P, q, eps, param, order, center, radius,
                                      child_begin, child_count, pt_begin,
                                      pt_end, stack, NULL, NULL);
                row_ptr[q + 1] = c;
                total += c;
            }
            free(stack);
        }
        row_ptr[0] = 0;
        for (int64_t q = 0; q < n; ++q)
            row_ptr[q + 1] += row_ptr[q];
        pset_free(&P);
        return total;
    }
#pragma omp parallel
    {
        int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (size_t)stack_cap);
        int64_t *pairs = NULL;
        int64_t pcap = 0;
#pragma omp for schedule(dynamic, 8)
        for (int64_t q = 0; q < n; ++q) {
            int64_t o = row_ptr[q];
            int64_t c = query_one(&P, q, eps, param, order, center, radius,
                                  child_begin, child_count, pt_begin, pt_end,
                                  stack, col + o, dist + o);
            /* rows in ascending column order */
            if (c > pcap) {
                free(pairs);
                pcap = c;
                pairs = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)pcap);
            }
            for (int64_t k = 0; k < c; ++k) {
                pairs[2 * k] = col[o + k];
                double dv = dist[o + k];
                memcpy(&pairs[2 * k + 1], &dv, sizeof(double));
            }
            qsort(pairs, (size_t)c, 2 * sizeof(int64_t), cmp_col);
            for (int64_t k = 0; k < c; ++k) {
                col[o + k] = (int32_t)pairs[2 * k];
                memcpy(&dist[o + k], &pairs[2 * k + 1], sizeof(double));
            }
        }
        free(pairs);
        free(stack);
    }
    pset_free(&P);
    return row_ptr[n];
}

/* ------------------------------------------------------------------------ */
/* Invariant checker (FP64, pinned comparisons).  viol[] receives counts:   */
/*  0 I1  points not in exactly one leaf block / order not a permutation    */
/*  1 I2  nesting: first child's centre differs from the parent's centre,   */
/*        or a leaf block's centre is not one of its points                 */
/*  2 I3a covering: child centre farther than 2^{l_v} from the parent      */
/*  3 I3b radius: a subtree point farther than the stored radius           */
/*  4 I3c split covering: a child's point farther than 2^{l_v - 1}          */
/*  5 I4  sibling separation: siblings within 2^{l_v - 1}                   */
/*  6 I5  child hub level not below the parent's                            */
/*  7 structure: child ranges do not tile the parent's point range          */
/* Leaf-block members are leaves B(p,0) and exempt from separation.         */
/* radius_mode 0: radius compared to the FP64 distance (oracle tree);       */
/* 1: the stored radius must bound the FP64 distance (GPU tree, float).     */
/* ------------------------------------------------------------------------ */

void orc_check_tree(int metric, const void *pts, int64_t n, int32_t dim,
                    const int32_t *order, const int32_t *center,
                    const double *radius, const int32_t *level,
                    const int32_t *child_begin, const int32_t *child_count,
                    const int32_t *pt_begin, const int32_t *pt_end,
                    int64_t nnodes, int64_t *viol)
{
    pset P;
    pset_init(&P, metric, pts, n, dim);
    for (int k = 0; k < 8; ++k)
        viol[k] = 0;
    /* I1: order is a permutation and leaf blocks tile 0..n-1 */
    int32_t *seen = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) {
        if (order[i] < 0 || order[i] >= n || seen[order[i]]++)
            viol[0]++;
    }
    int32_t *cover = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    for (int64_t v = 0; v < nnodes; ++v)
        if (child_count[v] == 0)
            for (int32_t i = pt_begin[v]; i < pt_end[v]; ++i)
                cover[i]++;
    for (int64_t i = 0; i < n; ++i)
        if (cover[i] != 1)
            viol[0]++;
    free(seen);
    free(cover);
    if (pt_begin[0] != 0 || pt_end[0] != n)
        viol[7]++;

    int64_t v0[8] = {0};
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : v0[:8])
    for (int64_t v = 0; v < nnodes; ++v) {
        int32_t cv = center[v];
        /* radius bounds every point of the subtree */
        for (int32_t i = pt_begin[v]; i < pt_end[v]; ++i) {
            double d = pdist(&P, cv, order[i]);
            if (!(d <= radius[v]))
                v0[3]++;
        }
        if (child_count[v] == 0) {
            int ok = 0;
            for (int32_t i = pt_begin[v]; i < pt_end[v]; ++i)
                ok |= order[i] == cv;
            if (!ok)
                v0[1]++;
            continue;
        }
        int32_t lv = level[v];
        int32_t cb = child_begin[v], cc = child_count[v];
        if (center[cb] != cv)
            v0[1]++;
        int32_t expect = pt_begin[v];
        for (int32_t a = 0; a < cc; ++a) {
            int32_t u = cb + a;
            if (pt_begin[u] != expect || pt_end[u] <= pt_begin[u])
                v0[7]++;
            expect = pt_end[u];
            if (!pwithin(&P, cv, center[u], lv))
                v0[2]++;
            for (int32_t i = pt_begin[u]; i < pt_end[u]; ++i)
                if (!pwithin(&P, center[u], order[i], lv - 1))
                    v0[4]++;
            if (child_count[u] > 0 && level[u] > lv - 1)
                v0[6]++;
            for (int32_t b2 = a + 1; b2 < cc; ++b2)
                if (pwithin(&P, center[u], center[cb + b2], lv - 1))
                    v0[5]++;
        }
        if (expect != pt_end[v])
            v0[7]++;
    }
    for (int k = 0; k < 8; ++k)
        viol[k] += v0[k];
    pset_free(&P);
}
