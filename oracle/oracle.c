/*
 * oracle.c -- plain CPU reference for the exact nearest-neighbour
 * (single-linkage) clustering of N records with D features.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load it.  It shares no code, header, table or constant
 * with the GPU path.
 *
 * What it computes (all in IEEE FP64, compiled with -ffp-contract=off):
 *
 *  - The pair key.  Eq. (1) of the paper defines the Euclidean distance
 *    rho = sqrt(sum_j (x_j1 - x_j2)^2).  Because sqrt is monotone the order of
 *    pairs is carried by the squared distance s, computed here in a fixed
 *    way: each feature is widened exactly from FP32 to FP64, the difference
 *    is rounded once, its square is rounded once and the squares are added
 *    left to right over features 0..D-1 (no fused multiply-add).  Ties in s
 *    are broken by (min index, max index), which makes every key distinct.
 *
 *  - The merge tree.  Section "General description of the algorithm for
 *    constructing the set of minimum distances" unites clusters along the
 *    globally smallest pairs, skipping pairs already inside one cluster,
 *    until clustering ends.  Taken to the end this is the minimum spanning
 *    tree of the complete graph under the key order (the single-linkage
 *    dendrogram).  The oracle builds that tree with dense Prim: one pass of
 *    key updates and one arg-min per added vertex, so every unordered pair is
 *    evaluated exactly once.  The N-1 edges are returned sorted by key.
 *
 *  - The constrained cut.  Section "Problem settings" (KL1..KL4) and the
 *    distance threshold of the "Problem statement" are applied to the sorted
 *    tree edges, one edge at a time:
 *      1. stop once the number of clusters is <= KL1 (KL1 <= 0: off);
 *      2. with KL4 > 1, an edge whose smaller side has fewer than KL4 points
 *         has class 0, otherwise class 1; edges are taken in (class, key)
 *         order with the class evaluated when the edge is taken;
 *      3. an edge is discarded for good when sqrt(s) > dmax, when the larger
 *         side has more than KL2 points (KL2 < 0: off) or when the two sides
 *         hold more than KL3 points together (KL3 < 0: off);
 *      4. otherwise the two clusters are united.
 *    Labels are numbered 0..K-1 in order of first appearance over i = 0..N-1.
 *
 *  - The same settings applied to every pair of points (the process itself
 *    rather than a cut of its tree): oracle_cut_allpairs.  It equals the
 *    cut of the tree whenever KL2 and KL3 are off.
 *
 *  - Other metrics (L1, L-infinity; cosine as the Euclidean metric on rows
 *    scaled to unit length) for the tree and the neighbour lists.
 *
 *  - Exact k nearest neighbours and the exact nearest neighbour outside a
 *    given labelling, both by the same key, used to check samples of large
 *    runs one row at a time.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* Squared distance of eq. (1), FP64, fixed order, no contraction. */
static double sq_dist(const float *a, const float *b, int32_t d)
{
    double s = 0.0;
    for (int32_t f = 0; f < d; ++f) {
        double diff = (double)a[f] - (double)b[f];
        double sq = diff * diff;
        s = (f == 0) ? sq : s + sq;
    }
    return s;
}

double oracle_sqdist(const float *a, const float *b, int32_t d)
{
    return sq_dist(a, b, d);
}

/*
 * Other metrics ("Overall idea of the algorithm": after eq. (1) the paper
 * allows another metric to be chosen).  The key of a pair under
 *   metric 0  Euclidean: the squared distance above (distance = sqrt(key));
 *   metric 1  L1 (city block): sum over f of |x_f - y_f|, each term exact in
 *             FP64, added left to right (distance = key);
 *   metric 2  L-infinity (Chebyshev): max over f of |x_f - y_f|, exact
 *             (distance = key).
 * Cosine dissimilarity is the Euclidean metric on rows scaled to unit
 * length (oracle_normalize_rows), with distance sqrt(2 - 2 cos).
 */
static double pair_key(const float *a, const float *b, int32_t d, int metric)
{
    if (metric == 1) {
        double s = 0.0;
        for (int32_t f = 0; f < d; ++f) {
            double t = fabs((double)a[f] - (double)b[f]);
            s = (f == 0) ? t : s + t;
        }
        return s;
    }
    if (metric == 2) {
        double s = 0.0;
        for (int32_t f = 0; f < d; ++f) {
            double t = fabs((double)a[f] - (double)b[f]);
            if (t > s) s = t;
        }
        return s;
    }
    return sq_dist(a, b, d);
}

static double key_to_distance(double s, int metric)
{
    return (metric == 1 || metric == 2) ? s : sqrt(s);
}

double oracle_pair_key(const float *a, const float *b, int32_t d, int32_t metric)
{
    return pair_key(a, b, d, metric);
}

/*
 * Rows scaled to unit Euclidean length: the norm is the square root of the
 * FP64 sum of squares in feature order; every feature is divided by it in
 * FP64 and rounded once to FP32.  A zero row stays zero.
 */
int oracle_normalize_rows(const float *X, int64_t n, int32_t d, int64_t ld, float *out)
{
    if (!X || !out || n < 1 || d < 1 || ld < d) return ORACLE_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        const float *x = X + i * ld;
        double q = 0.0;
        for (int32_t f = 0; f < d; ++f) {
            double v = (double)x[f];
            double sq = v * v;
            q = (f == 0) ? sq : q + sq;
        }
        double nrm = sqrt(q);
        for (int32_t f = 0; f < d; ++f)
            out[i * d + f] = nrm > 0.0 ? (float)((double)x[f] / nrm) : 0.0f;
    }
    return ORACLE_OK;
}

/* Lexicographic (s, lo, hi) order. */
static int key_less(double s1, int32_t lo1, int32_t hi1,
                    double s2, int32_t lo2, int32_t hi2)
{
    if (s1 != s2) return s1 < s2;
    if (lo1 != lo2) return lo1 < lo2;
    return hi1 < hi2;
}

typedef struct { double s; int32_t lo, hi; } okey;

static int okey_cmp(const void *pa, const void *pb)
{
    const okey *a = (const okey *)pa, *b = (const okey *)pb;
    if (key_less(a->s, a->lo, a->hi, b->s, b->lo, b->hi)) return -1;
    if (key_less(b->s, b->lo, b->hi, a->s, a->lo, a->hi)) return 1;
    return 0;
}

static int n_threads(int want)
{
#ifdef _OPENMP
    if (want > 0) return want;
    return omp_get_max_threads();
#else
    (void)want;
    return 1;
#endif
}

/*
 * Dense Prim over the complete graph.  out_u/out_v/out_s/out_w hold n-1
 * edges on return, u < v, sorted by key; out_w = sqrt(out_s).
 */
int oracle_prim_mst_metric(const float *X, int64_t n, int32_t d, int64_t ld,
                           int32_t metric, int32_t *out_u, int32_t *out_v,
                           double *out_s, double *out_w, int nthreads);

int oracle_prim_mst(const float *X, int64_t n, int32_t d, int64_t ld,
                    int32_t *out_u, int32_t *out_v, double *out_s,
                    double *out_w, int nthreads)
{
    return oracle_prim_mst_metric(X, n, d, ld, 0, out_u, out_v, out_s, out_w, nthreads);
}

/* The same under metric 0, 1 or 2 (keys and distances as for pair_key). */
int oracle_prim_mst_metric(const float *X, int64_t n, int32_t d, int64_t ld,
                           int32_t metric, int32_t *out_u, int32_t *out_v,
                           double *out_s, double *out_w, int nthreads)
{
    if (metric < 0 || metric > 2) return ORACLE_EINVAL;
    if (!X || n < 1 || d < 1 || ld < d) return ORACLE_EINVAL;
    if (n == 1) return ORACLE_OK;
    if (!out_u || !out_v || !out_s || !out_w) return ORACLE_EINVAL;
    if (n > INT32_MAX) return ORACLE_EINVAL;

    int nt = n_threads(nthreads);
    int64_t m = n - 1;
    /* Vertices not yet in the tree, kept compact: id, coordinates, best key. */
    int32_t *rid = malloc(sizeof(int32_t) * (size_t)m);
    float *rx = malloc(sizeof(float) * (size_t)m * (size_t)d);
    double *bs = malloc(sizeof(double) * (size_t)m);
    int32_t *blo = malloc(sizeof(int32_t) * (size_t)m);
    int32_t *bhi = malloc(sizeof(int32_t) * (size_t)m);
    float *ax = malloc(sizeof(float) * (size_t)d);
    okey *tloc = malloc(sizeof(okey) * (size_t)nt);
    int64_t *tpos = malloc(sizeof(int64_t) * (size_t)nt);
    okey *edges = malloc(sizeof(okey) * (size_t)(n - 1));
    if (!rid || !rx || !bs || !blo || !bhi || !ax || !tloc || !tpos || !edges) {
        free(rid); free(rx); free(bs); free(blo); free(bhi); free(ax);
        free(tloc); free(tpos); free(edges);
        return ORACLE_ENOMEM;
    }
    for (int64_t r = 0; r < m; ++r) {
        rid[r] = (int32_t)(r + 1);
        memcpy(rx + r * d, X + (r + 1) * ld, sizeof(float) * (size_t)d);
        bs[r] = INFINITY;
        blo[r] = INT32_MAX;
        bhi[r] = INT32_MAX;
    }
    int32_t a = 0;
    memcpy(ax, X, sizeof(float) * (size_t)d);

    for (int64_t it = 0; it < n - 1; ++it) {
        int used = (m >= 16384) ? nt : 1;
#pragma omp parallel num_threads(used) if (used > 1)
        {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            okey best = {INFINITY, INT32_MAX, INT32_MAX};
            int64_t bpos = -1;
#pragma omp for schedule(static)
            for (int64_t r = 0; r < m; ++r) {
                double s = pair_key(ax, rx + r * d, d, metric);
                int32_t v = rid[r];
                int32_t lo = a < v ? a : v;
                int32_t hi = a < v ? v : a;
                if (key_less(s, lo, hi, bs[r], blo[r], bhi[r])) {
                    bs[r] = s;
                    blo[r] = lo;
                    bhi[r] = hi;
                }
                if (bpos < 0 || key_less(bs[r], blo[r], bhi[r], best.s, best.lo, best.hi)) {
                    best.s = bs[r];
                    best.lo = blo[r];
                    best.hi = bhi[r];
                    bpos = r;
                }
            }
            tloc[t] = best;
            tpos[t] = bpos;
        }
        /* The keys are distinct, so the winner does not depend on threads. */
        int64_t win = -1;
        okey wk = {INFINITY, INT32_MAX, INT32_MAX};
        for (int t = 0; t < used; ++t) {
            if (tpos[t] < 0) continue;
            if (win < 0 || key_less(tloc[t].s, tloc[t].lo, tloc[t].hi, wk.s, wk.lo, wk.hi)) {
                wk = tloc[t];
                win = tpos[t];
            }
        }
        edges[it] = wk;
        a = rid[win];
        memcpy(ax, rx + win * d, sizeof(float) * (size_t)d);
        --m;
        rid[win] = rid[m];
        memmove(rx + win * d, rx + m * d, sizeof(float) * (size_t)d);
        bs[win] = bs[m];
        blo[win] = blo[m];
        bhi[win] = bhi[m];
    }
    qsort(edges, (size_t)(n - 1), sizeof(okey), okey_cmp);
    for (int64_t e = 0; e < n - 1; ++e) {
        out_u[e] = edges[e].lo;
        out_v[e] = edges[e].hi;
        out_s[e] = edges[e].s;
        out_w[e] = key_to_distance(edges[e].s, metric);
    }
    free(rid); free(rx); free(bs); free(blo); free(bhi); free(ax);
    free(tloc); free(tpos); free(edges);
    return ORACLE_OK;
}

/* ---- constrained cut -------------------------------------------------- */

static int64_t uf_find(int64_t *par, int64_t x)
{
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

/* Binary min-heap of (class, edge index); edge index order is key order. */
typedef struct { int32_t cls; int64_t e; } hent;

static int hless(hent a, hent b)
{
    if (a.cls != b.cls) return a.cls < b.cls;
    return a.e < b.e;
}

static void hpush(hent *h, int64_t *hn, hent x)
{
    int64_t i = (*hn)++;
    h[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!hless(h[i], h[p])) break;
        hent t = h[i]; h[i] = h[p]; h[p] = t;
        i = p;
    }
}

static hent hpop(hent *h, int64_t *hn)
{
    hent top = h[0];
    int64_t n = --(*hn);
    h[0] = h[n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < n && hless(h[l], h[m])) m = l;
        if (r < n && hless(h[r], h[m])) m = r;
        if (m == i) break;
        hent t = h[i]; h[i] = h[m]; h[m] = t;
        i = m;
    }
    return top;
}

int oracle_cut(const int32_t *eu, const int32_t *ev, const double *es,
               const double *ew, int64_t n, int64_t kl1, int64_t kl2,
               int64_t kl3, int64_t kl4, double dmax, int32_t *labels,
               int64_t *n_clusters)
{
    if (n < 1 || !labels || !n_clusters) return ORACLE_EINVAL;
    int64_t ne = n - 1;
    if (ne > 0 && (!eu || !ev || !es || !ew)) return ORACLE_EINVAL;
    for (int64_t e = 0; e < ne; ++e) {
        if (eu[e] < 0 || ev[e] >= n || eu[e] >= ev[e]) return ORACLE_EINVAL;
        if (e > 0 && !key_less(es[e - 1], eu[e - 1], ev[e - 1], es[e], eu[e], ev[e]))
            return ORACLE_EINVAL; /* not sorted by key */
    }
    int64_t *par = malloc(sizeof(int64_t) * (size_t)n);
    int64_t *sz = malloc(sizeof(int64_t) * (size_t)n);
    hent *heap = malloc(sizeof(hent) * (size_t)(ne > 0 ? ne : 1));
    int64_t *map = malloc(sizeof(int64_t) * (size_t)n);
    if (!par || !sz || !heap || !map) {
        free(par); free(sz); free(heap); free(map);
        return ORACLE_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) { par[i] = i; sz[i] = 1; }
    int64_t clusters = n;
    int prio = kl4 > 1;
    int64_t hn = 0;
    for (int64_t e = 0; e < ne; ++e) {
        hent x = {prio ? 0 : 1, e};   /* all sizes are 1 < KL4 at start */
        hpush(heap, &hn, x);
    }
    while (hn > 0) {
        if (kl1 > 0 && clusters <= kl1) break;
        hent x = hpop(heap, &hn);
        int64_t ra = uf_find(par, eu[x.e]);
        int64_t rb = uf_find(par, ev[x.e]);
        int64_t sa = sz[ra], sb = sz[rb];
        if (prio) {
            int32_t cls = ((sa < sb ? sa : sb) < kl4) ? 0 : 1;
            if (cls != x.cls) {
                x.cls = cls;
                hpush(heap, &hn, x);
                continue;
            }
        }
        if (ew[x.e] > dmax) continue;
        if (kl2 >= 0 && (sa > sb ? sa : sb) > kl2) continue;
        if (kl3 >= 0 && sa + sb > kl3) continue;
        if (sa < sb) { par[ra] = rb; sz[rb] += sa; }
        else { par[rb] = ra; sz[ra] += sb; }
        --clusters;
    }
    for (int64_t i = 0; i < n; ++i) map[i] = -1;
    int64_t next = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t r = uf_find(par, i);
        if (map[r] < 0) map[r] = next++;
        labels[i] = (int32_t)map[r];
    }
    *n_clusters = next;
    free(par); free(sz); free(heap); free(map);
    return ORACLE_OK;
}

/* ---- the constrained process over all pairs ----------------------------- */

/*
 * The clustering process of the section "General description of the
 * algorithm for constructing the set of minimum distances" with the
 * settings of "Problem settings" applied to every pair of points, not only
 * to tree edges: at each step the admissible pair of points in two
 * different clusters with the smallest (class, key) is taken and its two
 * clusters are united, until the number of clusters is <= KL1 (KL1 <= 0:
 * off) or no admissible pair is left.  A pair of clusters A, B is
 * admissible when sqrt(s) <= dmax, max(|A|, |B|) <= KL2 (KL2 < 0: off) and
 * |A| + |B| <= KL3 (KL3 < 0: off); with KL4 > 1 its class is 0 when
 * min(|A|, |B|) < KL4, else 1.  Labels as for oracle_cut.
 *
 * All n(n-1)/2 pairs are sorted by key once.  Each step scans that list
 * for the first pair that qualifies; a pair skipped because its points are
 * in one cluster, or because it is not admissible, never qualifies again
 * (clusters only grow, so sizes only grow and the tests above only get
 * stricter), and a pair skipped by the class-0 search because its class is
 * 1 never has class 0 again.  So each search resumes where it stopped.
 * Memory: 16 bytes per pair (n up to a few thousand).
 */
int oracle_cut_allpairs(const float *X, int64_t n, int32_t d, int64_t ld,
                        int64_t kl1, int64_t kl2, int64_t kl3, int64_t kl4,
                        double dmax, int32_t *labels, int64_t *n_clusters)
{
    if (!X || n < 1 || d < 1 || ld < d || !labels || !n_clusters) return ORACLE_EINVAL;
    if (n > 200000) return ORACLE_EINVAL;
    int64_t np = n * (n - 1) / 2;
    okey *pairs = malloc(sizeof(okey) * (size_t)(np > 0 ? np : 1));
    int64_t *par = malloc(sizeof(int64_t) * (size_t)n);
    int64_t *sz = malloc(sizeof(int64_t) * (size_t)n);
    int64_t *map = malloc(sizeof(int64_t) * (size_t)n);
    if (!pairs || !par || !sz || !map) {
        free(pairs); free(par); free(sz); free(map);
        return ORACLE_ENOMEM;
    }
    int64_t q = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            pairs[q].s = sq_dist(X + i * ld, X + j * ld, d);
            pairs[q].lo = (int32_t)i;
            pairs[q].hi = (int32_t)j;
            ++q;
        }
    qsort(pairs, (size_t)np, sizeof(okey), okey_cmp);
    for (int64_t i = 0; i < n; ++i) { par[i] = i; sz[i] = 1; }
    int64_t clusters = n;
    int prio = kl4 > 1;
    int64_t p0 = 0, p1 = 0;          /* where the class-0 and the any-class searches resume */
    for (;;) {
        if (kl1 > 0 && clusters <= kl1) break;
        int64_t take = -1;
        for (int pass = prio ? 0 : 1; pass <= 1 && take < 0; ++pass) {
            int64_t *p = pass == 0 ? &p0 : &p1;
            for (; *p < np; ++*p) {
                const okey *e = &pairs[*p];
                int64_t ra = uf_find(par, e->lo), rb = uf_find(par, e->hi);
                if (ra == rb) continue;
                int64_t sa = sz[ra], sb = sz[rb];
                if (sqrt(e->s) > dmax) continue;
                if (kl2 >= 0 && (sa > sb ? sa : sb) > kl2) continue;
                if (kl3 >= 0 && sa + sb > kl3) continue;
                if (pass == 0 && (sa < sb ? sa : sb) >= kl4) continue;
                take = *p;
                break;
            }
        }
        if (take < 0) break;
        int64_t ra = uf_find(par, pairs[take].lo), rb = uf_find(par, pairs[take].hi);
        if (sz[ra] < sz[rb]) { par[ra] = rb; sz[rb] += sz[ra]; }
        else { par[rb] = ra; sz[ra] += sz[rb]; }
        --clusters;
    }
    for (int64_t i = 0; i < n; ++i) map[i] = -1;
    int64_t next = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t r = uf_find(par, i);
        if (map[r] < 0) map[r] = next++;
        labels[i] = (int32_t)map[r];
    }
    *n_clusters = next;
    free(pairs); free(par); free(sz); free(map);
    return ORACLE_OK;
}

/* ---- exact neighbour queries, one row at a time ----------------------- */

/*
 * For each query row i = rows[q]: the k smallest keys (s, j) over j != i,
 * ascending; out_idx/out_s are [nrows][k]; out_len[q] = min(k, n-1).
 */
int oracle_knn_metric(const float *X, int64_t n, int32_t d, int64_t ld,
                      int32_t metric, const int64_t *rows, int64_t nrows,
                      int32_t k, int32_t *out_idx, double *out_s,
                      int32_t *out_len, int nthreads);

int oracle_knn(const float *X, int64_t n, int32_t d, int64_t ld,
               const int64_t *rows, int64_t nrows, int32_t k,
               int32_t *out_idx, double *out_s, int32_t *out_len,
               int nthreads)
{
    return oracle_knn_metric(X, n, d, ld, 0, rows, nrows, k, out_idx, out_s, out_len, nthreads);
}

/* The same under metric 0, 1 or 2 (keys as for pair_key). */
int oracle_knn_metric(const float *X, int64_t n, int32_t d, int64_t ld,
                      int32_t metric, const int64_t *rows, int64_t nrows,
                      int32_t k, int32_t *out_idx, double *out_s,
                      int32_t *out_len, int nthreads)
{
    if (!X || n < 1 || d < 1 || ld < d || k < 1 || nrows < 0) return ORACLE_EINVAL;
    if (metric < 0 || metric > 2) return ORACLE_EINVAL;
    int nt = n_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t i = rows ? rows[q] : q;
        if (i < 0 || i >= n) { bad = 1; continue; }
        int32_t *bi = out_idx + q * k;
        double *bsv = out_s + q * k;
        int32_t len = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double s = pair_key(X + i * ld, X + j * ld, d, metric);
            /* insert (s, j) into the ascending list if it belongs there */
            if (len == k && !(s < bsv[k - 1] || (s == bsv[k - 1] && j < bi[k - 1])))
                continue;
            int32_t p = (len < k) ? len++ : k - 1;
            while (p > 0 && (s < bsv[p - 1] || (s == bsv[p - 1] && j < bi[p - 1]))) {
                bsv[p] = bsv[p - 1];
                bi[p] = bi[p - 1];
                --p;
            }
            bsv[p] = s;
            bi[p] = (int32_t)j;
        }
        for (int32_t p = len; p < k; ++p) { bsv[p] = INFINITY; bi[p] = -1; }
        out_len[q] = len;
    }
    return bad ? ORACLE_EINVAL : ORACLE_OK;
}

/*
 * For each query row i = rows[q]: the smallest key (s, j) over j with
 * label[j] != label[i] (label == NULL: over j != i).  out_j = -1 and
 * out_s = +inf when no such j exists.
 */
int oracle_nn_outside(const float *X, int64_t n, int32_t d, int64_t ld,
                      const int32_t *label, const int64_t *rows,
                      int64_t nrows, int32_t *out_j, double *out_s,
                      int nthreads)
{
    if (!X || n < 1 || d < 1 || ld < d || nrows < 0) return ORACLE_EINVAL;
    int nt = n_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
    for (int64_t q = 0; q < nrows; ++q) {
        int64_t i = rows ? rows[q] : q;
        if (i < 0 || i >= n) { bad = 1; continue; }
        double bs = INFINITY;
        int32_t bj = -1;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            if (label && label[j] == label[i]) continue;
            double s = sq_dist(X + i * ld, X + j * ld, d);
            if (s < bs || (s == bs && j < bj)) { bs = s; bj = (int32_t)j; }
        }
        out_j[q] = bj;
        out_s[q] = bs;
    }
    return bad ? ORACLE_EINVAL : ORACLE_OK;
}
