/*
 * CPU oracle, part 2: the paper's hypercube method, run sequentially.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code with the GPU path.
 *
 * It follows the methodology section and Algorithms 1-4 in their order, on
 * integer coordinates:
 *   1. Origin shift: coordinates are taken relative to the per-dimension
 *      minimum ("Choosing Representative Points", origin shift).
 *   2. Hypercubes whose space diagonal is at most eps ("Overlaying
 *      Hypercubes"; band width eps/sqrt(d) in Algorithm 1).  With integer
 *      points a cube c covers [c*s, c*s + s - 1] per axis and
 *      s = max(1, floor(sqrt(floor(eps2 / d)))), so d*s^2 <= eps2 and any two
 *      points of one cube are within eps of each other.
 *   3. Pre-processing sort on the leading dimension with ties broken by the
 *      following ones (methodology, first paragraph): points are sorted by
 *      their cube coordinates, dimension 0 most significant, then by index.
 *   4. The cube dictionary of Algorithm 1, holding only non-empty cubes.
 *   5. Neighbour cubes (Depth First Search and Layering paragraphs): every
 *      cube offset D != 0 whose closest integer points can still be within
 *      eps, i.e. sum over D_k != 0 of ((|D_k| - 1) * s + 1)^2 <= eps2.  This
 *      contains the paper's 20 neighbours in 2-D and its j and j+1 layers.
 *   6. Core points per the appendix (Definition 2): a cube holding at least
 *      minPts points makes all of them core; otherwise |N(p)| is counted over
 *      the own cube and the neighbour cubes.
 *   7. Representative points (Algorithm 2), over the core points of a cube,
 *      for each of the 3^d - 1 directions: the first point initialises every
 *      direction and a later point replaces a representative only when it is
 *      strictly closer to the ideal position on the cube's boundary.  Only
 *      for d <= 4 (80 directions); higher d skips them.
 *   8. Depth-first merge over core cubes (Algorithms 3 and 4, explicit stack
 *      in place of recursion): neighbour cube Y joins X's cluster when the
 *      representatives facing each other are within eps.  The paper stops
 *      there; that alone can split a cluster, so unless rep_mode == 1 a
 *      failed representative test falls back to testing every core pair of
 *      the two cubes, which makes the result exact DBSCAN.
 *   9. Border points join the cluster of their nearest core point (ties to
 *      the smaller index); labels are ranked by smallest member index.
 *
 * rep_mode: 0 = representatives then exact fallback (default),
 *           1 = representatives only (the paper's merging test, not exact),
 *           2 = no representatives, exact tests only.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Planted mistakes, compiled in only with -DORACLE_MUTANT=k by the test that
 * checks that the pins catch each of them (k = 11..14 live in this file).
 * The default build has k = 0. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif
#define MUT(k) (ORACLE_MUTANT == (k))

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ERANGE 2
#define ORC_ENOMEM 3

int oracle_exact_eps2(double eps, int64_t *out);

static int64_t g_isqrt(int64_t v)
{
    int64_t r = (int64_t)sqrt((double)v);
    while (r > 0 && (__int128)r * r > v) r--;
    while ((__int128)(r + 1) * (r + 1) <= v) r++;
    return r;
}

static int64_t g_dist2(const int32_t *a, const int32_t *b, int d)
{
    int64_t s = 0;
    for (int k = 0; k < d; k++) {
        int64_t t = (int64_t)a[k] - (int64_t)b[k];
        s += t * t;
    }
    return s;
}

typedef struct {
    const int32_t *pts;
    int d;
    int64_t eps2, s;
    int R;
    int64_t n, ncube;
    int64_t *ord;         /* sorted position -> original index */
    int64_t *cc;          /* cube coordinates per sorted position [n][d] */
    int64_t *cstart;      /* cube -> first sorted position, [ncube + 1] */
    int64_t *ccoord;      /* cube -> coordinates [ncube][d] */
    uint8_t *core;        /* per original index */
} grid_t;

static grid_t *g_sort_ctx;
static int cmp_cube(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    const grid_t *g = g_sort_ctx;
    for (int k = 0; k < g->d; k++) {
        int64_t ca = g->cc[a * g->d + k], cb = g->cc[b * g->d + k];
        if (ca != cb) return ca < cb ? -1 : 1;
    }
    return a < b ? -1 : (a > b);
}

/* Is cube B a neighbour of cube A (closest integer points within eps)? */
static int is_neighbour(const grid_t *g, int64_t A, int64_t B)
{
    if (A == B) return 0;
    __int128 acc = 0;
    for (int k = 0; k < g->d; k++) {
        int64_t dd = g->ccoord[A * g->d + k] - g->ccoord[B * g->d + k];
        if (dd < 0) dd = -dd;
        if (dd == 0) continue;
        if (dd > g->R) return 0;
        __int128 gap = (__int128)(dd - 1) * g->s + 1;
        acc += gap * gap;
        if (acc > g->eps2) return 0;
    }
    return 1;
}

/* Cubes whose dimension-0 coordinate lies within R of cube A: [*lo, *hi). */
static void column_window(const grid_t *g, int64_t A, int64_t *lo, int64_t *hi)
{
    int64_t c0 = g->ccoord[A * g->d];
    int64_t l = 0, h = g->ncube;
    while (l < h) { int64_t m = (l + h) / 2; if (g->ccoord[m * g->d] < c0 - g->R) l = m + 1; else h = m; }
    *lo = l;
    l = 0; h = g->ncube;
    while (l < h) { int64_t m = (l + h) / 2; if (g->ccoord[m * g->d] <= c0 + g->R) l = m + 1; else h = m; }
    *hi = l;
}

/* number of representative directions: 3^d - 1 */
static int n_dirs(int d)
{
    int v = 1;
    for (int k = 0; k < d; k++) v *= 3;
    return v - 1;
}

/* direction index t in [0, 3^d - 1) -> components in {-1, 0, 1}; the all-zero
 * combination is skipped. */
static void dir_of(int t, int d, int *delta)
{
    int zero = 0, m = 1;
    for (int k = 0; k < d; k++) { zero += m; m *= 3; }
    int v = t >= zero ? t + 1 : t;          /* skip base-3 code of (0,...,0) */
    for (int k = 0; k < d; k++) { delta[k] = v % 3 - 1; v /= 3; }
}

static int dir_index(const int *delta, int d)
{
    int v = 0, m = 1, zero = 0;
    for (int k = 0; k < d; k++) { v += (delta[k] + 1) * m; zero += m; m *= 3; }
    return v > zero ? v - 1 : v;
}

int oracle_hca_grid(const int32_t *pts, int64_t n, int32_t d, double eps, int32_t min_pts,
                    int32_t rep_mode, int32_t *labels, int32_t *core_out, int64_t *stats,
                    int32_t nthreads)
{
    if (n < 0 || n > INT32_MAX || d < 1 || d > 8 || min_pts < 1 || rep_mode < 0 || rep_mode > 2)
        return ORC_EINVAL;
    if (n > 0 && (!pts || !labels)) return ORC_EINVAL;
    grid_t g;
    memset(&g, 0, sizeof g);
    int rc = oracle_exact_eps2(eps, &g.eps2);
    if (rc) return rc;
    if (stats) memset(stats, 0, sizeof(int64_t) * 8);
    if (n == 0) return ORC_OK;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    int nt = 1;
    (void)nthreads;
#endif
    g.pts = pts; g.d = d; g.n = n;

    /* 1. origin shift */
    int64_t origin[8];
    for (int k = 0; k < d; k++) {
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        for (int64_t i = 0; i < n; i++) {
            int64_t v = pts[i * d + k];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        if (hi - lo >= ((int64_t)1 << 30)) return ORC_ERANGE;
        origin[k] = lo;
    }
    /* 2. cube side and neighbour radius */
    g.s = g_isqrt(g.eps2 / d);
    if (g.s < 1) g.s = 1;
    g.R = 0;
    while (g.R < (1 << 30)) {
        __int128 gap = (__int128)g.R * g.s + 1;   /* gap at offset R+1 */
        if (gap * gap > g.eps2) break;
        g.R++;
    }

    int64_t ndir = (d <= 4 && rep_mode != 2) ? n_dirs(d) : 0;
    g.ord = malloc(sizeof(int64_t) * n);
    g.cc = malloc(sizeof(int64_t) * n * d);
    g.cstart = malloc(sizeof(int64_t) * (n + 1));
    g.ccoord = malloc(sizeof(int64_t) * n * d);
    g.core = calloc(n, 1);
    int64_t *cube_of = malloc(sizeof(int64_t) * n);      /* per sorted position */
    int64_t *ncorept = calloc(n, sizeof(int64_t));       /* per cube */
    int64_t *cid = malloc(sizeof(int64_t) * n);          /* per cube */
    int64_t *stack = malloc(sizeof(int64_t) * n);
    int64_t *rep = ndir ? malloc(sizeof(int64_t) * n * ndir) : NULL;
    int64_t *lab_of = malloc(sizeof(int64_t) * n);
    if (!g.ord || !g.cc || !g.cstart || !g.ccoord || !g.core || !cube_of || !ncorept || !cid ||
        !stack || (ndir && !rep) || !lab_of) {
        rc = ORC_ENOMEM;
        goto out;
    }
    for (int64_t i = 0; i < n; i++)
        for (int k = 0; k < d; k++)
            g.cc[i * d + k] = ((int64_t)pts[i * d + k] - origin[k]) / g.s;

    /* 3. sort by cube coordinates (dimension 0 most significant), then index */
    for (int64_t i = 0; i < n; i++) g.ord[i] = i;
    g_sort_ctx = &g;
    qsort(g.ord, n, sizeof(int64_t), cmp_cube);

    /* 4. dictionary of non-empty cubes: runs of equal coordinates */
    g.ncube = 0;
    for (int64_t a = 0; a < n; a++) {
        int newcube = (a == 0);
        if (!newcube)
            for (int k = 0; k < d; k++)
                if (g.cc[g.ord[a] * d + k] != g.cc[g.ord[a - 1] * d + k]) { newcube = 1; break; }
        if (newcube) {
            g.cstart[g.ncube] = a;
            for (int k = 0; k < d; k++) g.ccoord[g.ncube * d + k] = g.cc[g.ord[a] * d + k];
            g.ncube++;
        }
        cube_of[a] = g.ncube - 1;
    }
    g.cstart[g.ncube] = n;

    /* 6. core points */
    int64_t ncube = g.ncube;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (int64_t A = 0; A < ncube; A++) {
        int64_t a0 = g.cstart[A], a1 = g.cstart[A + 1];
        if (a1 - a0 >= min_pts) {
            for (int64_t a = a0; a < a1; a++) g.core[g.ord[a]] = 1;
            continue;
        }
        int64_t wlo, whi;
        column_window(&g, A, &wlo, &whi);
        for (int64_t a = a0; a < a1; a++) {
            const int32_t *p = pts + g.ord[a] * d;
            int64_t count = a1 - a0;        /* the own cube lies wholly within eps */
            for (int64_t B = wlo; B < whi; B++) {
                if (!is_neighbour(&g, A, B)) continue;
                for (int64_t b = g.cstart[B]; b < g.cstart[B + 1]; b++)
                    if (g_dist2(p, pts + g.ord[b] * d, d) <= g.eps2) count++;
            }
            g.core[g.ord[a]] = count >= min_pts;
        }
    }
    int64_t n_core_pts = 0, n_core_cubes = 0, n_dense = 0;
    for (int64_t A = 0; A < ncube; A++) {
        for (int64_t a = g.cstart[A]; a < g.cstart[A + 1]; a++) ncorept[A] += g.core[g.ord[a]];
        n_core_pts += ncorept[A];
        n_core_cubes += ncorept[A] > 0;
        n_dense += (g.cstart[A + 1] - g.cstart[A]) >= min_pts;
    }

    /* 7. representative points over core points (Algorithm 2) */
    if (ndir) {
        int delta[8];
        for (int64_t A = 0; A < ncube; A++) {
            int64_t *rA = rep + A * ndir;
            int first = 1;
            for (int64_t a = g.cstart[A]; a < g.cstart[A + 1]; a++) {
                if (!g.core[g.ord[a]]) continue;
                if (first) {                 /* first point takes every position */
                    for (int t = 0; t < ndir; t++) rA[t] = a;
                    first = 0;
                    continue;
                }
                const int32_t *p = pts + g.ord[a] * d;
                for (int t = 0; t < ndir; t++) {
                    dir_of(t, d, delta);
                    const int32_t *r = pts + g.ord[rA[t]] * d;
                    int64_t sa = 0, sb = 0;
                    for (int k = 0; k < d; k++) {
                        if (!delta[k]) continue;
                        int64_t c = g.ccoord[A * d + k];
                        int64_t ideal = (delta[k] > 0 ? c + 1 : c) * g.s;
                        if (MUT(13) && delta[k] > 0) ideal = c * g.s;        /* +1 on the lower face */
                        if (MUT(14) && delta[k] < 0) ideal = (c + 1) * g.s;  /* -1 on the upper face */
                        int64_t ya = (int64_t)p[k] - origin[k] - ideal;
                        int64_t yb = (int64_t)r[k] - origin[k] - ideal;
                        sa += ya * ya;
                        sb += yb * yb;
                    }
                    if (sa < sb || (MUT(12) && sa == sb)) rA[t] = a;  /* replace only when strictly closer */
                }
            }
        }
    }

    /* 8. depth-first merge over core cubes (Algorithms 3-4) */
    int64_t rep_acc = 0, exact_acc = 0, exact_rej = 0, pair_tests = 0;
    for (int64_t A = 0; A < ncube; A++) cid[A] = -1;
    int64_t next_cluster = 0;
    for (int64_t A0 = 0; A0 < ncube; A0++) {
        if (!ncorept[A0] || cid[A0] >= 0) continue;
        cid[A0] = next_cluster;
        int64_t sp = 0;
        stack[sp++] = A0;
        while (sp) {
            int64_t X = stack[--sp];
            int64_t wlo, whi;
            column_window(&g, X, &wlo, &whi);
            for (int64_t Y = wlo; Y < whi; Y++) {
                if (!ncorept[Y] || cid[Y] >= 0 || !is_neighbour(&g, X, Y)) continue;
                int joined = 0;
                if (ndir) {                  /* facing representatives */
                    int dx[8], dy[8];
                    for (int k = 0; k < d; k++) {
                        int64_t dd = g.ccoord[Y * d + k] - g.ccoord[X * d + k];
                        dx[k] = (dd > 0) - (dd < 0);
                        dy[k] = MUT(11) ? dx[k] : -dx[k];   /* Y faces back towards X */
                    }
                    int64_t rx = rep[X * ndir + dir_index(dx, d)];
                    int64_t ry = rep[Y * ndir + dir_index(dy, d)];
                    pair_tests++;
                    if (g_dist2(pts + g.ord[rx] * d, pts + g.ord[ry] * d, d) <= g.eps2) {
                        joined = 1;
                        rep_acc++;
                    }
                }
                if (!joined && rep_mode != 1) {  /* exact fallback over core pairs */
                    for (int64_t a = g.cstart[X]; a < g.cstart[X + 1] && !joined; a++) {
                        if (!g.core[g.ord[a]]) continue;
                        const int32_t *p = pts + g.ord[a] * d;
                        for (int64_t b = g.cstart[Y]; b < g.cstart[Y + 1]; b++) {
                            if (!g.core[g.ord[b]]) continue;
                            pair_tests++;
                            if (g_dist2(p, pts + g.ord[b] * d, d) <= g.eps2) { joined = 1; break; }
                        }
                    }
                    if (joined) exact_acc++; else exact_rej++;
                }
                if (joined) {
                    cid[Y] = cid[X];
                    stack[sp++] = Y;
                }
            }
        }
        next_cluster++;
    }

    /* 9. border points and canonical labels */
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
    for (int64_t A = 0; A < ncube; A++) {
        int64_t wlo = 0, whi = 0, have_window = 0;
        for (int64_t a = g.cstart[A]; a < g.cstart[A + 1]; a++) {
            int64_t i = g.ord[a];
            if (g.core[i]) { lab_of[i] = cid[A]; continue; }
            if (!have_window) { column_window(&g, A, &wlo, &whi); have_window = 1; }
            const int32_t *p = pts + i * d;
            int64_t bd = INT64_MAX, bj = -1, bc = -1;
            for (int64_t B = wlo; B < whi; B++) {
                if (!ncorept[B] || (B != A && !is_neighbour(&g, A, B))) continue;
                for (int64_t b = g.cstart[B]; b < g.cstart[B + 1]; b++) {
                    int64_t j = g.ord[b];
                    if (!g.core[j]) continue;
                    int64_t dd = g_dist2(p, pts + j * d, d);
                    if (dd <= g.eps2 && (dd < bd || (dd == bd && j < bj))) { bd = dd; bj = j; bc = B; }
                }
            }
            lab_of[i] = bj >= 0 ? cid[bc] : -1;
        }
    }
    for (int64_t c = 0; c < n; c++) stack[c] = -1;   /* reuse as cluster -> label */
    int32_t next = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t c = lab_of[i];
        if (c < 0) { labels[i] = -1; continue; }
        if (stack[c] < 0) stack[c] = next++;
        labels[i] = (int32_t)stack[c];
    }
    if (core_out)
        for (int64_t i = 0; i < n; i++) core_out[i] = g.core[i];
    if (stats) {
        stats[0] = ncube;
        stats[1] = n_core_cubes;
        stats[2] = n_dense;
        stats[3] = n_core_pts;
        stats[4] = rep_acc;
        stats[5] = exact_acc;
        stats[6] = exact_rej;
        stats[7] = pair_tests;
    }
    rc = ORC_OK;
out:
    free(g.ord); free(g.cc); free(g.cstart); free(g.ccoord); free(g.core);
    free(cube_of); free(ncorept); free(cid); free(stack); free(rep); free(lab_of);
    return rc;
}

/* cube side s and neighbour radius R used above, for tests */
int oracle_grid_geometry(double eps, int32_t d, int64_t *s_out, int64_t *r_out)
{
    int64_t eps2;
    if (d < 1 || !s_out || !r_out) return ORC_EINVAL;
    int rc = oracle_exact_eps2(eps, &eps2);
    if (rc) return rc;
    int64_t s = g_isqrt(eps2 / d);
    if (s < 1) s = 1;
    int64_t R = 0;
    while (R < (1 << 30)) {
        __int128 gap = (__int128)R * s + 1;
        if (gap * gap > eps2) break;
        R++;
    }
    *s_out = s;
    *r_out = R;
    return ORC_OK;
}

/* Number of neighbour cube offsets (D != 0 passing the closest-point test)
 * for a given eps and dimension; -1 if the count would exceed max_count. */
int oracle_stencil_size(double eps, int32_t d, int64_t max_count, int64_t *out)
{
    int64_t s, R, eps2;
    if (d < 1 || d > 8 || !out) return ORC_EINVAL;
    int rc = oracle_grid_geometry(eps, d, &s, &R);
    if (rc) return rc;
    oracle_exact_eps2(eps, &eps2);
    int64_t w = 2 * R + 1, total = 1;
    for (int k = 0; k < d; k++) {
        if (total > max_count * 4 / w + 1) { *out = -1; return ORC_OK; }
        total *= w;
    }
    int64_t count = 0;
    for (int64_t code = 0; code < total; code++) {
        int64_t v = code, nz = 0;
        __int128 acc = 0;
        for (int k = 0; k < d; k++) {
            int64_t dd = v % w - R;
            v /= w;
            if (dd < 0) dd = -dd;
            if (!dd) continue;
            nz = 1;
            __int128 gap = (__int128)(dd - 1) * s + 1;
            acc += gap * gap;
        }
        if (nz && acc <= eps2) count++;
    }
    *out = count > max_count ? -1 : count;
    return ORC_OK;
}
