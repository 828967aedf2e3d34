/*
 * CPU oracle, part 1: DBSCAN computed from its definition.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the GPU path.
 *
 * What it computes (appendix "The DBSCAN Algorithm", Definitions 1-5):
 *   eps2      = floor(eps^2), exact (eps is a double in coordinate units).
 *   dist2     = sum_k (x_ik - x_jk)^2, exact int64.
 *   N(i)      = { j : dist2(i,j) <= eps2 }, i itself included (Definition 1,
 *               closed ball, q ranges over the whole data set).
 *   core(i)   = |N(i)| >= minPts (Definition 2, core-point condition).
 *   clusters  = connected components of the graph on core points whose edges
 *               join core pairs within eps (Definitions 3-5: a chain of
 *               directly density-reachable points passes only through core
 *               points; a cluster is maximal and connected).
 *   border    = non-core i with a core point in N(i).  The paper leaves the
 *               choice between several clusters open; this oracle fixes it:
 *               i joins the cluster of the core j minimising (dist2(i,j), j).
 *   noise     = every other point, label -1.
 *   labels    = clusters ranked by their smallest member index (core and
 *               assigned border points), so the first occurrence of each
 *               label while scanning i = 0..n-1 reads 0, 1, 2, ...
 *
 * The only shortcut taken: points are visited in order of coordinate 0, and a
 * pair with |dx_0| > floor(sqrt(eps2)) is skipped without computing dist2,
 * since dx_0^2 alone already exceeds eps2.  Nothing else is reordered, blocked
 * or fused.  Components use union-find: each thread unions the edges it finds
 * into its own forest, and the forests are then merged into one (the union of
 * edge sets has the union of their connectivity).
 *
 * Domain: 1 <= d <= 64, every per-dimension span (max - min) < 2^30, and the
 * sum over dimensions of span^2 below 2^63 (automatic for d <= 8), so that no
 * dist2 overflows int64.  The paper's data sets reach 54 dimensions (Table 1).
 * Violations return an error.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Planted mistakes, compiled in only with -DORACLE_MUTANT=k by the test that
 * checks that the pins catch each of them.  The default build has k = 0. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif
#define MUT(k) (ORACLE_MUTANT == (k))

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ERANGE 2
#define ORC_ENOMEM 3

/* floor(eps^2) computed exactly from the binary value of eps.  eps = m * 2^e
 * with an integer mantissa m < 2^53, so eps^2 = m^2 * 2^(2e) with m^2 < 2^106:
 * one unsigned 128-bit product and a shift.  Results above INT64_MAX saturate
 * (every int64 dist2 is then within eps). */
int oracle_exact_eps2(double eps, int64_t *out)
{
    if (!out || !(eps > 0.0) || !isfinite(eps))
        return ORC_EINVAL;
    int e2;
    double fr = frexp(eps, &e2);            /* eps = fr * 2^e2, fr in [0.5, 1) */
    uint64_t m = (uint64_t)ldexp(fr, 53);   /* exact: fr has 53 significant bits */
    int e = e2 - 53;                        /* eps = m * 2^e */
    unsigned __int128 sq = (unsigned __int128)m * m;
    if (MUT(9)) {                           /* mutant 9: floor(eps)^2 */
        int64_t f = (int64_t)floor(eps);
        *out = f * f;
        return ORC_OK;
    }
    int sh = 2 * e;
    unsigned __int128 lim = (unsigned __int128)INT64_MAX;
    if (sh >= 0) {
        if (sh >= 64 || sq > (lim >> sh)) { *out = INT64_MAX; return ORC_OK; }
        sq <<= sh;
    } else {
        int r = -sh;
        sq = (r >= 128) ? 0 : (sq >> r);
    }
    *out = (sq > lim) ? INT64_MAX : (int64_t)sq;
    return ORC_OK;
}

/* floor(sqrt(v)) for 0 <= v < 2^63, exact. */
static int64_t isqrt64(int64_t v)
{
    int64_t r = (int64_t)sqrt((double)v);
    while (r > 0 && (__int128)r * r > v) r--;
    while ((__int128)(r + 1) * (r + 1) <= v) r++;
    return r;
}

/* dist2, except that once the partial sum exceeds eps2 it stops early and
 * returns that partial sum: any value > eps2 means "not within eps". */
static int64_t dist2(const int32_t *a, const int32_t *b, int d, int64_t eps2)
{
    int64_t s = 0;
    for (int k = 0; k < d - MUT(6); k++) {          /* mutant 6: drops a dimension */
        int64_t t = (int64_t)a[k] - (int64_t)b[k];
        s += t * t;
        if (s > eps2) break;
    }
    return s;
}

/* mutant 1: strict "< eps" neighbourhood */
static int within(int64_t dd, int64_t eps2) { return MUT(1) ? dd < eps2 : dd <= eps2; }

/* ---- union-find (path halving, union by smaller index as root) ---- */
static int32_t uf_find(int32_t *p, int32_t x)
{
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}

static void uf_union(int32_t *p, int32_t a, int32_t b)
{
    a = uf_find(p, a);
    b = uf_find(p, b);
    if (a == b) return;
    if (a < b) p[b] = a; else p[a] = b;
}

/* ---- sort of point indices by (coordinate 0, index) ---- */
static const int32_t *g_sort_pts;
static int g_sort_d;
static int cmp_x0(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    int32_t xa = g_sort_pts[a * g_sort_d], xb = g_sort_pts[b * g_sort_d];
    if (xa != xb) return xa < xb ? -1 : 1;
    return a < b ? -1 : (a > b);
}

static int check_domain(const int32_t *pts, int64_t n, int d)
{
    unsigned __int128 reach = 0;          /* sum of span^2: the largest possible dist2 */
    for (int k = 0; k < d; k++) {
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        for (int64_t i = 0; i < n; i++) {
            int64_t v = pts[i * d + k];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        if (n > 0 && hi - lo >= ((int64_t)1 << 30)) return ORC_ERANGE;
        if (n > 0) reach += (unsigned __int128)(hi - lo) * (uint64_t)(hi - lo);
    }
    if (reach > (unsigned __int128)INT64_MAX) return ORC_ERANGE;
    return ORC_OK;
}

/*
 * labels[n]   out: canonical cluster label per input point, -1 for noise.
 * counts[n]   out (nullable): |N(i)|.
 * owner[n]    out (nullable): for a border point the original index of the
 *             core point it joined; -1 for core and noise points.
 * nthreads    OpenMP threads (<= 0: runtime default); ignored without OpenMP.
 */
int oracle_dbscan(const int32_t *pts, int64_t n, int32_t d, double eps, int32_t min_pts,
                  int32_t *labels, int32_t *counts, int32_t *owner, int32_t nthreads)
{
    if (n < 0 || n > INT32_MAX || d < 1 || d > 64 || min_pts < 1) return ORC_EINVAL;
    if (n > 0 && (!pts || !labels)) return ORC_EINVAL;
    int64_t eps2;
    int rc = oracle_exact_eps2(eps, &eps2);
    if (rc) return rc;
    if (n == 0) return ORC_OK;
    rc = check_domain(pts, n, d);
    if (rc) return rc;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    int nt = 1;
    (void)nthreads;
#endif
    const int64_t E = isqrt64(eps2) - MUT(10);  /* |dx_0| > E  =>  dist2 > eps2 (mutant 10: E-1) */

    int64_t *ord = malloc(sizeof(int64_t) * n);
    int64_t *x0 = malloc(sizeof(int64_t) * n);
    int32_t *sp = malloc(sizeof(int32_t) * n * d);   /* points in visit order */
    int64_t *lo = malloc(sizeof(int64_t) * n), *hi = malloc(sizeof(int64_t) * n);
    int32_t *cnt = malloc(sizeof(int32_t) * n);
    uint8_t *core = malloc(n);
    int32_t *own = malloc(sizeof(int32_t) * n);
    int32_t *forests = malloc(sizeof(int32_t) * n * nt);
    int32_t *parent = malloc(sizeof(int32_t) * n);
    int32_t *root_label = malloc(sizeof(int32_t) * n);
    if (!ord || !x0 || !sp || !lo || !hi || !cnt || !core || !own || !forests || !parent || !root_label) {
        rc = ORC_ENOMEM;
        goto out;
    }

    /* visit order: by coordinate 0, ties by index */
    for (int64_t i = 0; i < n; i++) ord[i] = i;
    g_sort_pts = pts;
    g_sort_d = d;
    qsort(ord, n, sizeof(int64_t), cmp_x0);
    for (int64_t a = 0; a < n; a++) {
        x0[a] = pts[ord[a] * d];
        memcpy(sp + a * d, pts + ord[a] * d, sizeof(int32_t) * d);
    }
    /* window [lo[a], hi[a]) = sorted positions with |x0 - x0[a]| <= E */
    for (int64_t a = 0; a < n; a++) {
        int64_t l = 0, h = a;               /* first b with x0[b] >= x0[a] - E */
        while (l < h) { int64_t m = (l + h) / 2; if (x0[m] < x0[a] - E) l = m + 1; else h = m; }
        lo[a] = l;
        l = a; h = n;                       /* first b with x0[b] > x0[a] + E */
        while (l < h) { int64_t m = (l + h) / 2; if (x0[m] <= x0[a] + E) l = m + 1; else h = m; }
        hi[a] = l;
    }

    /* Definition 1-2: |N(i)| and the core flag */
#pragma omp parallel for schedule(dynamic, 256) num_threads(nt)
    for (int64_t a = 0; a < n; a++) {
        const int32_t *p = sp + a * d;
        int32_t c = 0;
        for (int64_t b = lo[a]; b < hi[a]; b++)
            if ((!MUT(2) || b != a) && within(dist2(p, sp + b * d, d, eps2), eps2)) c++;
        cnt[ord[a]] = c;                    /* mutant 2: the point itself not counted */
    }
    for (int64_t i = 0; i < n; i++) core[i] = MUT(3) ? cnt[i] > min_pts : cnt[i] >= min_pts;

    /* Definitions 3-5: components of the core graph */
#pragma omp parallel num_threads(nt)
    {
#ifdef _OPENMP
        int t = omp_get_thread_num();
#else
        int t = 0;
#endif
        int32_t *f = forests + (int64_t)t * n;
        for (int64_t i = 0; i < n; i++) f[i] = (int32_t)i;
#pragma omp for schedule(dynamic, 256)
        for (int64_t a = 0; a < n; a++) {
            int64_t i = ord[a];
            if (!core[i] && !MUT(7)) continue;  /* mutant 7: non-core points link clusters */
            const int32_t *p = sp + a * d;
            for (int64_t b = a + 1; b < hi[a]; b++) {
                int64_t j = ord[b];
                if ((core[j] || MUT(7)) && within(dist2(p, sp + b * d, d, eps2), eps2))
                    uf_union(f, (int32_t)i, (int32_t)j);
            }
        }
    }
    for (int64_t i = 0; i < n; i++) parent[i] = (int32_t)i;
    for (int t = 0; t < nt; t++) {
        int32_t *f = forests + (int64_t)t * n;
        for (int64_t i = 0; i < n; i++) {
            int32_t r = uf_find(f, (int32_t)i);
            if (r != i) uf_union(parent, (int32_t)i, r);
        }
    }

    /* border points: nearest core point, ties to the smaller index */
#pragma omp parallel for schedule(dynamic, 256) num_threads(nt)
    for (int64_t a = 0; a < n; a++) {
        int64_t i = ord[a];
        own[i] = -1;
        if (core[i]) continue;
        const int32_t *p = sp + a * d;
        int64_t bd = INT64_MAX, bj = -1;
        for (int64_t b = lo[a]; b < hi[a]; b++) {
            int64_t j = ord[b];
            if (!core[j]) continue;
            int64_t dd = dist2(p, sp + b * d, d, eps2);
            int better = MUT(5) ? (bj < 0 || dd > bd || (dd == bd && j < bj))   /* mutant 5: farthest core */
                       : MUT(4) ? (dd < bd || (dd == bd && j > bj))              /* mutant 4: ties to larger index */
                                : (dd < bd || (dd == bd && j < bj));
            if (within(dd, eps2) && better) { bd = dd; bj = j; }
        }
        own[i] = (int32_t)bj;
    }

    /* canonical labels: scanning i upward, a cluster is numbered when its
     * first (= smallest-index) member appears */
    for (int64_t i = 0; i < n; i++) root_label[i] = -1;
    int32_t next = 0;
    for (int64_t ii = 0; ii < n; ii++) {
        int64_t i = MUT(8) ? n - 1 - ii : ii;  /* mutant 8: ranked by largest member */
        int32_t r;
        if (core[i]) r = uf_find(parent, (int32_t)i);
        else if (own[i] >= 0) r = uf_find(parent, own[i]);
        else { labels[i] = -1; continue; }
        if (root_label[r] < 0) root_label[r] = next++;
        labels[i] = root_label[r];
    }
    if (counts) memcpy(counts, cnt, sizeof(int32_t) * n);
    if (owner) memcpy(owner, own, sizeof(int32_t) * n);
    rc = ORC_OK;
out:
    free(ord); free(x0); free(sp); free(lo); free(hi); free(cnt); free(core); free(own);
    free(forests); free(parent); free(root_label);
    return rc;
}
