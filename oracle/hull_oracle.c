/*
 * CPU oracle for the interior-point-discarding preprocessor for 2D convex
 * hulls (G. Mei, "A Straightforward Preprocessing Approach for Accelerating
 * Convex Hull Computations on the GPU", arXiv:1405.3454).
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load this library.
 * It shares no code, header, table or helper with the GPU library: it is a
 * plain, slow, single-threaded restatement of the paper's steps, written so
 * that a reader can check each function against the paper by eye.
 *
 * Build (see oracle/__init__.py):
 *   gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -msse2 -mfpmath=sse
 *       -fPIC -shared hull_oracle.c -o liboracle.so
 * -ffp-contract=off matters: every expression below is meant as a sequence
 * of separately rounded IEEE binary64 operations (no fused multiply-add).
 *
 * Input domain: float32 coordinates that are multiples of 2^-24 in [0, 1).
 * On that grid every orientation predicate evaluated below in binary64 is
 * exact (coordinate differences need 25 bits, their products 49 bits, a
 * difference of two products 50 bits), so the discard test and the hull are
 * exact.  The directional projections are not exact; they are defined as the
 * rounded sequence written out in oracle_extremes().
 *
 * Readings of the paper taken here (the paper is silent or inconsistent):
 *  - angle set: the paper's text says 30/45/45 degrees (Sec. 2, Step 1) while
 *    Figure 1 and Sec. 5 say 30/45/60; the default table is {0,30,45,60}
 *    (its remaining-point fractions match Table 2).  A second table,
 *    {0,30,75,120}, reads the text's rotations as cumulative.
 *  - rotation is counter-clockwise: x' = x cos t - y sin t, y' = x sin t + y cos t.
 *  - extremes: lowest point index wins among equal binary64 values.
 *  - "inside" is strict: points on the polygon boundary survive.  A polygon
 *    with fewer than 3 vertices discards nothing.
 *  - duplicates and collinear points: the hull keeps the lowest index for a
 *    repeated coordinate pair and excludes collinear points; it is listed
 *    counter-clockwise starting from the lexicographically smallest (x, y).
 *  - survivors are listed in ascending index order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORACLE_NONE 0xFFFFFFFFu

/* ------------------------------------------------------------------------
 * Direction tables (Sec. 2, Step 1; Figure 1; Sec. 5).
 * Correctly rounded binary64 cosines and sines, written as hex literals so
 * that no run-time libm call (whose results are not correctly rounded)
 * enters the arithmetic.
 * ---------------------------------------------------------------------- */
#define COS30 0x1.bb67ae8584caap-1
#define COS45 0x1.6a09e667f3bcdp-1
#define COS75 0x1.0907dc1930690p-2
#define SIN75 0x1.ee8dd4748bf15p-1

/* preset 0: rotations by 0, 30, 45, 60 degrees (Figure 1, Sec. 5) */
static const double PRESET0_C[4] = {1.0, COS30, COS45, 0.5};
static const double PRESET0_S[4] = {0.0, 0.5, COS45, COS30};
/* preset 1: rotations 30, 45, 45 of Sec. 2 read cumulatively: 0, 30, 75, 120 */
static const double PRESET1_C[4] = {1.0, COS30, COS75, -0.5};
static const double PRESET1_S[4] = {0.0, 0.5, SIN75, COS30};

/* presets 2..7: direction families beyond the paper's table.  Preset 1 + G
 * has G rotation groups at 90 j / G degrees, j = 0..G-1, so its 4G extreme
 * directions are evenly spaced 90 / G degrees apart.  G = 1 is the plain
 * min/max x and y quadrilateral that the paper cites as the simplest
 * preprocessing filter (Sec. 1, ref. [3]).  Rows: cos(90 j / G) for
 * j = 0..5 (unused entries 0); the sines follow from
 * sin(90 j / G) = cos(90 (G - j) / G). */
static const double EVEN_COS[6][6] = {
    /* G = 1: 0 */
    {1.0, 0, 0, 0, 0, 0},
    /* G = 2: 0, 45 */
    {1.0, 0x1.6a09e667f3bcdp-1, 0, 0, 0, 0},
    /* G = 3: 0, 30, 60 */
    {1.0, 0x1.bb67ae8584caap-1, 0x1p-1, 0, 0, 0},
    /* G = 4: 0, 22.5, 45, 67.5 */
    {1.0, 0x1.d906bcf328d46p-1, 0x1.6a09e667f3bcdp-1, 0x1.87de2a6aea963p-2, 0, 0},
    /* G = 5: 0, 18, 36, 54, 72 */
    {1.0, 0x1.e6f0e134454ffp-1, 0x1.9e3779b97f4a8p-1, 0x1.2cf2304755a5ep-1,
     0x1.3c6ef372fe950p-2, 0},
    /* G = 6: 0, 15, 30, 45, 60, 75 */
    {1.0, 0x1.ee8dd4748bf15p-1, 0x1.bb67ae8584caap-1, 0x1.6a09e667f3bcdp-1, 0x1p-1,
     0x1.0907dc1930690p-2}};

/* Copy preset `preset` into c[], s[] (room for 6 groups); return the number
 * of groups or -1. */
int oracle_preset(int preset, double *c, double *s)
{
    const double *pc, *ps;
    if (preset == 0) { pc = PRESET0_C; ps = PRESET0_S; }
    else if (preset == 1) { pc = PRESET1_C; ps = PRESET1_S; }
    else if (preset >= 2 && preset <= 7) {
        int G = preset - 1;
        for (int j = 0; j < G; j++) {
            c[j] = EVEN_COS[G - 1][j];
            s[j] = j == 0 ? 0.0 : EVEN_COS[G - 1][G - j];
        }
        return G;
    }
    else return -1;
    for (int g = 0; g < 4; g++) { c[g] = pc[g]; s[g] = ps[g]; }
    return 4;
}

/* 64 candidate directions phi_d = 2 pi d / 64 for the learned proposal.
 * First-quadrant values d = 0..15 as correctly rounded literals; the other
 * quadrants follow from cos(phi + 90deg) = -sin(phi), sin(phi + 90deg) =
 * cos(phi), which is exact in binary64 (negation only). */
static const double Q1_C[16] = {
    1.0,                     0x1.fd88da3d12526p-1, 0x1.f6297cff75cb0p-1,
    0x1.e9f4156c62ddap-1,    0x1.d906bcf328d46p-1, 0x1.c38b2f180bdb1p-1,
    0x1.a9b66290ea1a3p-1,    0x1.8bc806b151741p-1, 0x1.6a09e667f3bcdp-1,
    0x1.44cf325091dd6p-1,    0x1.1c73b39ae68c8p-1, 0x1.e2b5d3806f63bp-2,
    0x1.87de2a6aea963p-2,    0x1.294062ed59f06p-2, 0x1.8f8b83c69a60bp-3,
    0x1.917a6bc29b42cp-4};
static const double Q1_S[16] = {
    0.0,                     0x1.917a6bc29b42cp-4, 0x1.8f8b83c69a60bp-3,
    0x1.294062ed59f06p-2,    0x1.87de2a6aea963p-2, 0x1.e2b5d3806f63bp-2,
    0x1.1c73b39ae68c8p-1,    0x1.44cf325091dd6p-1, 0x1.6a09e667f3bcdp-1,
    0x1.8bc806b151741p-1,    0x1.a9b66290ea1a3p-1, 0x1.c38b2f180bdb1p-1,
    0x1.d906bcf328d46p-1,    0x1.e9f4156c62ddap-1, 0x1.f6297cff75cb0p-1,
    0x1.fd88da3d12526p-1};

/* Fill c[64], s[64] with the candidate direction table. */
void oracle_direction_table(double *c, double *s)
{
    for (int d = 0; d < 64; d++) {
        int q = d / 16, r = d % 16;
        double cc = Q1_C[r], ss = Q1_S[r];
        for (int k = 0; k < q; k++) {      /* rotate by +90 degrees q times */
            double t = cc;
            cc = -ss;
            ss = t;
        }
        c[d] = cc + 0.0;                   /* -0.0 -> +0.0 */
        s[d] = ss + 0.0;
    }
}

/* ------------------------------------------------------------------------
 * Step 1 (Sec. 2): extreme points with min/max x and y of the original set
 * and of the rotated copies.  Rotating every point by the same angle does not
 * change which points are extreme, so the rotated copy is never stored: for
 * group g with constants (c, s) the rotated coordinates of point i are
 *     u = c*x - s*y,   v = s*x + c*y        (each product rounded, then the sum)
 * Slots per group: [4g+0] argmin u, [4g+1] argmax u, [4g+2] argmin v,
 * [4g+3] argmax v; the lowest index wins ties.  vals[] receives the extreme
 * values (may be NULL).  n == 0 fills the slots with ORACLE_NONE.
 * ---------------------------------------------------------------------- */
void oracle_extremes(const float *x, const float *y, int64_t n,
                     const double *c, const double *s, int G,
                     uint32_t *slots, double *vals)
{
    for (int g = 0; g < G; g++) {
        uint32_t best[4] = {ORACLE_NONE, ORACLE_NONE, ORACLE_NONE, ORACLE_NONE};
        double bv[4] = {NAN, NAN, NAN, NAN};
        for (int64_t i = 0; i < n; i++) {
            double xd = (double)x[i], yd = (double)y[i];
            double u = c[g] * xd - s[g] * yd;
            double v = s[g] * xd + c[g] * yd;
            if (i == 0) {
                for (int k = 0; k < 4; k++) best[k] = 0;
                bv[0] = u; bv[1] = u; bv[2] = v; bv[3] = v;
                continue;
            }
            if (u < bv[0]) { bv[0] = u; best[0] = (uint32_t)i; }
            if (u > bv[1]) { bv[1] = u; best[1] = (uint32_t)i; }
            if (v < bv[2]) { bv[2] = v; best[2] = (uint32_t)i; }
            if (v > bv[3]) { bv[3] = v; best[3] = (uint32_t)i; }
        }
        for (int k = 0; k < 4; k++) {
            slots[4 * g + k] = best[k];
            if (vals) vals[4 * g + k] = bv[k];
        }
    }
}

/* Extreme point along each direction (c[d], s[d]): argmax of c*x + s*y
 * (products rounded, then the sum), lowest index on ties.  Used for the
 * extra directions a learned proposal adds to the fixed ones. */
void oracle_extremes_dirs(const float *x, const float *y, int64_t n,
                          const double *c, const double *s, int D,
                          uint32_t *slots, double *vals)
{
    for (int d = 0; d < D; d++) {
        uint32_t best = ORACLE_NONE;
        double bv = NAN;
        for (int64_t i = 0; i < n; i++) {
            double w = c[d] * (double)x[i] + s[d] * (double)y[i];
            if (i == 0 || w > bv) { bv = w; best = (uint32_t)i; }
        }
        slots[d] = best;
        if (vals) vals[d] = bv;
    }
}

/* ------------------------------------------------------------------------
 * Andrew's monotone chain (Step 2 and the final hull; the paper's reference
 * [6] as corrected in its erratum).
 * ---------------------------------------------------------------------- */
typedef struct { double x, y; uint32_t i; } opt;

static int cmp_xyi(const void *pa, const void *pb)
{
    const opt *a = (const opt *)pa, *b = (const opt *)pb;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    if (a->y != b->y) return a->y < b->y ? -1 : 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    return 0;
}

/* z component of (a - o) x (b - o); exact on the input grid. */
static double cross3(const opt *o, const opt *a, const opt *b)
{
    return (a->x - o->x) * (b->y - o->y) - (a->y - o->y) * (b->x - o->x);
}

/* Convex hull of the points listed in idx[0..k) (or of points 0..k-1 when idx
 * is NULL).  Writes vertex indices counter-clockwise from the
 * lexicographically smallest point to out[], their count to *h.  Collinear
 * points are excluded; a repeated coordinate pair is represented by its
 * lowest index.  Returns 0, or -1 when memory runs out. */
int oracle_hull_subset(const float *x, const float *y, const uint32_t *idx,
                       int64_t k, uint32_t *out, int64_t *h)
{
    *h = 0;
    if (k <= 0) return 0;
    opt *p = (opt *)malloc((size_t)k * sizeof(opt));
    opt **st = (opt **)malloc((size_t)(2 * k + 2) * sizeof(opt *));
    if (!p || !st) { free(p); free(st); return -1; }
    for (int64_t j = 0; j < k; j++) {
        uint32_t i = idx ? idx[j] : (uint32_t)j;
        p[j].x = (double)x[i];
        p[j].y = (double)y[i];
        p[j].i = i;
    }
    qsort(p, (size_t)k, sizeof(opt), cmp_xyi);
    /* drop repeated coordinates, keeping the first (= lowest index) */
    int64_t u = 0;
    for (int64_t j = 0; j < k; j++)
        if (u == 0 || p[j].x != p[u - 1].x || p[j].y != p[u - 1].y) p[u++] = p[j];
    if (u == 1) {
        out[0] = p[0].i;
        *h = 1;
        free(p); free(st);
        return 0;
    }
    int64_t t = 0;
    for (int64_t j = 0; j < u; j++) {                 /* lower chain */
        while (t >= 2 && cross3(st[t - 2], st[t - 1], &p[j]) <= 0) t--;
        st[t++] = &p[j];
    }
    int64_t lo = t + 1;
    for (int64_t j = u - 2; j >= 0; j--) {            /* upper chain */
        while (t >= lo && cross3(st[t - 2], st[t - 1], &p[j]) <= 0) t--;
        st[t++] = &p[j];
    }
    t--;                                              /* last == first */
    for (int64_t j = 0; j < t; j++) out[j] = st[j]->i;
    *h = t;
    free(p); free(st);
    return 0;
}

/* Step 2 (Sec. 2): the convex polygon formed by the extreme points.  slots
 * may repeat indices and may hold ORACLE_NONE (ignored).  Writes the polygon
 * vertices counter-clockwise to verts[] (capacity nslots) and their count to
 * *m. */
int oracle_polygon(const float *x, const float *y, const uint32_t *slots,
                   int nslots, uint32_t *verts, int *m)
{
    uint32_t tmp[256];
    int k = 0;
    *m = 0;
    if (nslots > 256) return -1;
    for (int j = 0; j < nslots; j++)
        if (slots[j] != ORACLE_NONE) tmp[k++] = slots[j];
    int64_t h = 0;
    int rc = oracle_hull_subset(x, y, tmp, k, verts, &h);
    *m = (int)h;
    return rc;
}

/* Step 3 (Sec. 2): discard every point strictly inside the counter-clockwise
 * polygon verts[0..m).  Point p is strictly inside iff for every edge (a, b)
 * the cross product (b - a) x (p - a) is > 0.  With m < 3 nothing is
 * discarded.  Survivor indices go to surv[] in ascending order, their count
 * to *cnt. */
void oracle_discard(const float *x, const float *y, int64_t n,
                    const uint32_t *verts, int m, uint32_t *surv, int64_t *cnt)
{
    int64_t c = 0;
    for (int64_t i = 0; i < n; i++) {
        int inside = (m >= 3);
        double px = (double)x[i], py = (double)y[i];
        for (int e = 0; e < m && inside; e++) {
            uint32_t a = verts[e], b = verts[(e + 1) % m];
            double ax = x[a], ay = y[a], bx = x[b], by = y[b];
            double cr = (bx - ax) * (py - ay) - (by - ay) * (px - ax);
            if (!(cr > 0)) inside = 0;
        }
        if (!inside) surv[c++] = (uint32_t)i;
    }
    *cnt = c;
}

/* The whole method: extremes -> polygon -> discard -> hull of the survivors
 * (Sec. 2, Steps 1-3, then the hull of the remaining points as in Sec. 3).
 * With nofilter != 0 the hull of all points is computed instead (the paper's
 * case (1)).  surv (capacity n) and n_surv may be NULL. */
int oracle_compute(const float *x, const float *y, int64_t n,
                   const double *c, const double *s, int G, int nofilter,
                   uint32_t *hull, int64_t *h, uint32_t *surv, int64_t *n_surv)
{
    *h = 0;
    if (n_surv) *n_surv = 0;
    if (G < 0 || G > 16) return -1;
    if (n <= 0) return 0;
    if (nofilter) return oracle_hull_subset(x, y, NULL, n, hull, h);
    uint32_t slots[64], verts[64];
    int m = 0;
    oracle_extremes(x, y, n, c, s, G, slots, NULL);
    if (oracle_polygon(x, y, slots, 4 * G, verts, &m)) return -1;
    uint32_t *sv = surv ? surv : (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    if (!sv) return -1;
    int64_t cnt = 0;
    oracle_discard(x, y, n, verts, m, sv, &cnt);
    int rc = oracle_hull_subset(x, y, sv, cnt, hull, h);
    if (n_surv) *n_surv = cnt;
    if (!surv) free(sv);
    return rc;
}

/* ------------------------------------------------------------------------
 * Learned direction proposal (an extension of this project, not the paper's).
 * ---------------------------------------------------------------------- */

/* 32 x 32 occupancy histogram of a point set, the network's input.
 * Sample: every stride-th point, stride = ceil(n / 16384), starting at 0.
 * Grid coordinates kx = x * 2^24 (integers on the input grid).  The bins
 * span a square window around the sample's bounding box, so the set keeps its
 * aspect ratio: with box widths wx = max kx - min kx + 1, wy likewise, and
 * w = max(wx, wy), the window starts at (min kx - (w - wx) / 2,
 * min ky - (w - wy) / 2) and bx = (kx - start x) * 32 / w in integer
 * arithmetic, likewise by.  hist[by * 32 + bx] = count * 1024 / ns (binary64
 * product and quotient, rounded to float), ns the sample size. */
/* Index of sample j (j < oracle_hist_samples(n)) of a set of n points: all
 * points when n <= 16384, else 256 runs of 64 consecutive points, run r
 * starting at floor(r (n - 64) / 255) (the first at 0, the last ending at
 * n - 1; the runs are disjoint since (n - 64) / 255 >= 64). */
static int64_t oracle_hist_samples(int64_t n) { return n <= 16384 ? n : 16384; }
static int64_t oracle_hist_index(int64_t n, int64_t j)
{
    if (n <= 16384) return j;
    return (j / 64) * (n - 64) / 255 + j % 64;
}

void oracle_histogram(const float *x, const float *y, int64_t n, float *hist)
{
    int64_t cnt[1024];
    memset(cnt, 0, sizeof(cnt));
    for (int b = 0; b < 1024; b++) hist[b] = 0.0f;
    if (n <= 0) return;
    const int64_t ns = oracle_hist_samples(n);
    int64_t x0 = INT64_MAX, x1 = INT64_MIN, y0 = INT64_MAX, y1 = INT64_MIN;
    for (int64_t j = 0; j < ns; j++) {
        const int64_t i = oracle_hist_index(n, j);
        int64_t kx = (int64_t)((double)x[i] * 16777216.0);
        int64_t ky = (int64_t)((double)y[i] * 16777216.0);
        if (kx < x0) x0 = kx;
        if (kx > x1) x1 = kx;
        if (ky < y0) y0 = ky;
        if (ky > y1) y1 = ky;
    }
    int64_t wx = x1 - x0 + 1, wy = y1 - y0 + 1, w = wx > wy ? wx : wy;
    int64_t sx = x0 - (w - wx) / 2, sy = y0 - (w - wy) / 2;
    for (int64_t j = 0; j < ns; j++) {
        const int64_t i = oracle_hist_index(n, j);
        int64_t kx = (int64_t)((double)x[i] * 16777216.0);
        int64_t ky = (int64_t)((double)y[i] * 16777216.0);
        int64_t bx = (kx - sx) * 32 / w;
        int64_t by = (ky - sy) * 32 / w;
        cnt[by * 32 + bx]++;
    }
    for (int b = 0; b < 1024; b++)
        hist[b] = (float)((double)cnt[b] * 1024.0 / (double)ns);
}

/* Training labels: for each of the D candidate directions, the fraction of
 * all n points that the plain filter keeps but the polygon of the fixed
 * extremes plus that direction's extreme point discards.
 * gain[d] = #{base survivors strictly inside hull(fixed extremes + e_d)} / n. */
int oracle_labels(const float *x, const float *y, int64_t n,
                  const double *c, const double *s, int G,
                  const double *cd, const double *sd, int D, double *gain)
{
    for (int d = 0; d < D; d++) gain[d] = 0.0;
    if (G < 0 || G > 16 || D < 0 || D > 256) return -1;
    if (n <= 0) return 0;
    uint32_t slots[64], verts[64], ed[256];
    int m = 0;
    oracle_extremes(x, y, n, c, s, G, slots, NULL);
    oracle_polygon(x, y, slots, 4 * G, verts, &m);
    uint32_t *sv = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    if (!sv) return -1;
    int64_t cnt = 0;
    oracle_discard(x, y, n, verts, m, sv, &cnt);
    oracle_extremes_dirs(x, y, n, cd, sd, D, ed, NULL);
    for (int d = 0; d < D; d++) {
        uint32_t sl2[65];
        for (int j = 0; j < 4 * G; j++) sl2[j] = slots[j];
        sl2[4 * G] = ed[d];
        int m2 = 0;
        uint32_t v2[65];
        oracle_polygon(x, y, sl2, 4 * G + 1, v2, &m2);
        int64_t inside = 0;
        for (int64_t j = 0; j < cnt; j++) {
            uint32_t i = sv[j];
            int in = (m2 >= 3);
            double px = (double)x[i], py = (double)y[i];
            for (int e = 0; e < m2 && in; e++) {
                uint32_t a = v2[e], b = v2[(e + 1) % m2];
                double ax = x[a], ay = y[a], bx = x[b], by = y[b];
                if (!((bx - ax) * (py - ay) - (by - ay) * (px - ax) > 0)) in = 0;
            }
            inside += in;
        }
        gain[d] = (double)inside / (double)n;
    }
    free(sv);
    return 0;
}

/* ------------------------------------------------------------------------
 * Greedy joint training targets for the learned proposal (an extension of
 * this project; the paper has no learned part).  The fixed filter's extreme
 * points start the set E.  Round r = 0, 1, ... tries every candidate
 * direction d: g_d(r) = number of the fixed filter's survivors strictly
 * inside polygon(E + {e_d}) but not strictly inside polygon(E).  The
 * direction with the largest g_d(r) (lowest d on ties) joins E; a round
 * whose largest gain is 0 ends the sequence.  Targets: the direction chosen
 * in round r gets 1 - r / (2R); any other direction d gets 0.5 g_d(0) / max
 * g(0), or 0 when that maximum is 0.  order[r] is the chosen direction or -1.
 * ---------------------------------------------------------------------- */
static int strictly_inside(const float *x, const float *y, const uint32_t *v, int m, uint32_t i)
{
    if (m < 3) return 0;
    double px = (double)x[i], py = (double)y[i];
    for (int e = 0; e < m; e++) {
        uint32_t a = v[e], b = v[(e + 1) % m];
        double ax = x[a], ay = y[a], bx = x[b], by = y[b];
        if (!((bx - ax) * (py - ay) - (by - ay) * (px - ax) > 0)) return 0;
    }
    return 1;
}

int oracle_label_targets(const float *x, const float *y, int64_t n,
                         const double *c, const double *s, int G,
                         const double *cd, const double *sd, int D, int R,
                         float *target, int32_t *order)
{
    if (G < 0 || G > 16 || D < 1 || D > 256 || R < 1 || R > 16) return -1;
    for (int d = 0; d < D; d++) target[d] = 0.0f;
    for (int r = 0; r < R; r++) order[r] = -1;
    if (n <= 0) return 0;
    uint32_t base[64], ed[256], pts[96], cur[96], trial[96];
    int64_t *g0 = (int64_t *)calloc((size_t)D, sizeof(int64_t));
    uint32_t *sv = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    if (!g0 || !sv) { free(g0); free(sv); return -1; }
    int m = 0;
    oracle_extremes(x, y, n, c, s, G, base, NULL);
    oracle_polygon(x, y, base, 4 * G, cur, &m);
    int64_t cnt = 0;
    oracle_discard(x, y, n, cur, m, sv, &cnt);
    oracle_extremes_dirs(x, y, n, cd, sd, D, ed, NULL);
    int np = 4 * G;
    for (int j = 0; j < np; j++) pts[j] = base[j];
    for (int r = 0; r < R; r++) {
        int mc = 0;
        oracle_polygon(x, y, pts, np, cur, &mc);
        int best = -1;
        int64_t bestg = 0;
        for (int d = 0; d < D; d++) {
            pts[np] = ed[d];
            int mt = 0;
            oracle_polygon(x, y, pts, np + 1, trial, &mt);
            int64_t g = 0;
            for (int64_t j = 0; j < cnt; j++)
                if (!strictly_inside(x, y, cur, mc, sv[j]) && strictly_inside(x, y, trial, mt, sv[j])) g++;
            if (r == 0) g0[d] = g;
            if (g > bestg) { bestg = g; best = d; }
        }
        if (best < 0) break;
        order[r] = best;
        pts[np++] = ed[best];
    }
    int64_t gmax = 0;
    for (int d = 0; d < D; d++) if (g0[d] > gmax) gmax = g0[d];
    for (int d = 0; d < D; d++)
        target[d] = gmax > 0 ? (float)(0.5 * ((double)g0[d] / (double)gmax)) : 0.0f;
    for (int r = 0; r < R; r++)
        if (order[r] >= 0) target[order[r]] = (float)(1.0 - (double)r / (2.0 * R));
    free(g0);
    free(sv);
    return 0;
}
