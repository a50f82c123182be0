/*
 * CPU oracle for the 3D form of the interior-point-discarding preprocessor
 * (G. Mei, arXiv:1405.3454; the conclusion, Sec. 5, names the extension to
 * three dimensions as the next step).
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load this library.
 * It shares no code with the GPU library: a plain, slow, single-threaded
 * statement of the 3D steps.
 *
 * Build (oracle/hull3d.py): gcc -O2 -std=gnu11 -ffp-contract=off
 *   -fno-fast-math -msse2 -mfpmath=sse -fPIC -shared hull3d_oracle.c
 *
 * Input domain: float32 x, y, z that are multiples of 2^-24 in [0, 1).  In
 * grid units (coordinate * 2^24) every coordinate is an integer below 2^24,
 * so every orientation predicate below is evaluated EXACTLY in integer
 * arithmetic: differences need 25 bits, a cross product 50 bits (int64),
 * and a 3x3 determinant 75 bits (__int128).
 *
 * The 3D method (the readings taken here):
 *  Step 1  extremes along the directions of "rotations about an axis": for a
 *          rotation by angle t (constants c = cos t, s = sin t of a 2D
 *          direction preset) about axis z, x or y, the rotated coordinates of
 *          the plane perpendicular to the axis, (a, b) = (x, y), (y, z) or
 *          (z, x), are u = c*a - s*b and v = s*a + c*b (each product rounded
 *          to binary64, then the sum), and the axis coordinate itself stays.
 *          Each rotation gives six extremes (min/max of u, v and the axis
 *          coordinate); the distinct ones are min/max of x, y, z and min/max
 *          of u and v for every plane and every non-zero angle.  Slot order:
 *          [0..5] = argmin x, argmax x, argmin y, argmax y, argmin z, argmax z;
 *          then for plane k = 0 (about z), 1 (about x), 2 (about y) and group
 *          g = 1..G-1: 6 + 4 ((G - 1) k + g - 1) + {argmin u, argmax u,
 *          argmin v, argmax v}.  Ties: lowest index.
 *  Step 2  the convex polyhedron of the slot points: every plane through
 *          three of them that has all of them on one side and at least one
 *          strictly; fewer than four affinely independent points: no
 *          interior.
 *  Step 3  discard every point strictly inside the polyhedron (strictly on
 *          the inner side of every such plane); points on its boundary
 *          survive.
 *  Step 4  the hull of the survivors: its extreme points (vertices of the
 *          convex hull, points on a face or an edge but not corners
 *          excluded), a repeated coordinate triple named by its lowest index,
 *          listed in ascending index order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NONE3 0xFFFFFFFFu
typedef __int128 i128;

static int64_t gx(float v) { return (int64_t)((double)v * 16777216.0); }

/* ------------------------------------------------------------------------
 * Step 1.
 * ---------------------------------------------------------------------- */
int oracle3_slot_count(int G) { return G < 1 ? -1 : 6 + 12 * (G - 1); }

void oracle3_extremes(const float *x, const float *y, const float *z, int64_t n,
                      const double *c, const double *s, int G, uint32_t *slots, double *vals)
{
    const int ns = 6 + 12 * (G - 1);
    double best[6 + 12 * 15];
    for (int k = 0; k < ns; k++) {
        slots[k] = NONE3;
        best[k] = 0.0;
    }
    for (int64_t i = 0; i < n; i++) {
        const double X = x[i], Y = y[i], Z = z[i];
        double key[6 + 12 * 15];
        key[0] = X; key[1] = X; key[2] = Y; key[3] = Y; key[4] = Z; key[5] = Z;
        for (int k = 0; k < 3; k++) {
            const double a = k == 0 ? X : k == 1 ? Y : Z;
            const double b = k == 0 ? Y : k == 1 ? Z : X;
            for (int g = 1; g < G; g++) {
                const double pa = c[g] * a, pb = s[g] * b, qa = s[g] * a, qb = c[g] * b;
                const double u = pa - pb, v = qa + qb;
                const int base = 6 + 4 * ((G - 1) * k + g - 1);
                key[base + 0] = u; key[base + 1] = u;
                key[base + 2] = v; key[base + 3] = v;
            }
        }
        for (int k = 0; k < ns; k++) {
            const int is_min = (k & 1) == 0;
            if (slots[k] == NONE3 || (is_min ? key[k] < best[k] : key[k] > best[k])) {
                slots[k] = (uint32_t)i;
                best[k] = key[k];
            }
        }
    }
    if (vals)
        for (int k = 0; k < ns; k++) vals[k] = best[k];
}

/* ------------------------------------------------------------------------
 * Exact predicates on grid coordinates.
 * ---------------------------------------------------------------------- */
typedef struct { int64_t x, y, z; } P3;

static P3 pt(const float *x, const float *y, const float *z, uint32_t i)
{
    P3 p = {gx(x[i]), gx(y[i]), gx(z[i])};
    return p;
}

static P3 sub3(P3 a, P3 b) { P3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }

static P3 cross3(P3 a, P3 b)
{
    P3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}

static i128 dot3(P3 n, P3 d)
{
    return (i128)n.x * d.x + (i128)n.y * d.y + (i128)n.z * d.z;
}

/* det[b - a, c - a, d - a]: > 0 when d lies on the side of plane (a, b, c)
 * that its normal (b - a) x (c - a) points to. */
static i128 orient3(P3 a, P3 b, P3 c, P3 d)
{
    return dot3(cross3(sub3(b, a), sub3(c, a)), sub3(d, a));
}

static int is_zero3(P3 v) { return v.x == 0 && v.y == 0 && v.z == 0; }

/* ------------------------------------------------------------------------
 * Step 2: the polyhedron of the slot points.  planes[f] = (nx, ny, nz) and a
 * point (px, py, pz) on the plane, in grid units, with the normal pointing
 * into the polyhedron.  Returns the number of planes (0: no interior).
 * ---------------------------------------------------------------------- */
int oracle3_polyhedron(const float *x, const float *y, const float *z, const uint32_t *slots,
                       int ns, int64_t *planes, int cap)
{
    /* distinct points: unique indices, then unique coordinates */
    P3 q[256];
    int m = 0;
    for (int k = 0; k < ns && m < 256; k++) {
        if (slots[k] == NONE3) continue;
        P3 p = pt(x, y, z, slots[k]);
        int dup = 0;
        for (int j = 0; j < m; j++)
            if (q[j].x == p.x && q[j].y == p.y && q[j].z == p.z) dup = 1;
        if (!dup) q[m++] = p;
    }
    int nf = 0;
    for (int i = 0; i < m; i++)
        for (int j = i + 1; j < m; j++)
            for (int k = j + 1; k < m; k++) {
                P3 nrm = cross3(sub3(q[j], q[i]), sub3(q[k], q[i]));
                if (is_zero3(nrm)) continue;          /* collinear */
                int pos = 0, neg = 0;
                for (int t = 0; t < m; t++) {
                    i128 d = dot3(nrm, sub3(q[t], q[i]));
                    pos += d > 0;
                    neg += d < 0;
                }
                if (pos && neg) continue;             /* not a supporting plane */
                if (!pos && !neg) continue;           /* every point on it: no interior */
                if (pos == 0) { nrm.x = -nrm.x; nrm.y = -nrm.y; nrm.z = -nrm.z; }
                if (nf < cap) {
                    int64_t *r = planes + 6 * nf;
                    r[0] = nrm.x; r[1] = nrm.y; r[2] = nrm.z;
                    r[3] = q[i].x; r[4] = q[i].y; r[5] = q[i].z;
                }
                nf++;
            }
    return nf;
}

/* Step 3: survivors (ascending) of the strict-inside test. */
void oracle3_discard(const float *x, const float *y, const float *z, int64_t n,
                     const int64_t *planes, int nf, uint32_t *surv, int64_t *cnt)
{
    int64_t c = 0;
    for (int64_t i = 0; i < n; i++) {
        P3 p = pt(x, y, z, (uint32_t)i);
        int inside = nf > 0;
        for (int f = 0; f < nf && inside; f++) {
            const int64_t *r = planes + 6 * f;
            P3 nrm = {r[0], r[1], r[2]}, a = {r[3], r[4], r[5]};
            if (!(dot3(nrm, sub3(p, a)) > 0)) inside = 0;
        }
        if (!inside) surv[c++] = (uint32_t)i;
    }
    *cnt = c;
}

/* ------------------------------------------------------------------------
 * Step 4: the extreme points of a subset.
 *
 * Repeated coordinates are reduced to their lowest index.  Then an
 * incremental hull: start from four affinely independent points, add the
 * others one by one; the faces a new point sees strictly are removed and
 * the horizon is joined to it.  Points that see no face are inside or on
 * the boundary and are skipped.  Coplanar neighbouring faces are not
 * merged, so at the end a hull vertex is a corner (an extreme point) iff
 * its incident faces span at least three distinct planes.  Inputs without
 * four affinely independent points are flat: their extreme points are those
 * of the 2D hull in their plane (collinear points excluded).
 * ---------------------------------------------------------------------- */
typedef struct { int v[3]; int nb[3]; int alive; } Face;   /* nb[e]: across edge v[e] -> v[e+1] */

typedef struct { P3 p; uint32_t idx; } IP;

static int cmp_ip(const void *pa, const void *pb)
{
    const IP *a = (const IP *)pa, *b = (const IP *)pb;
    if (a->p.x != b->p.x) return a->p.x < b->p.x ? -1 : 1;
    if (a->p.y != b->p.y) return a->p.y < b->p.y ? -1 : 1;
    if (a->p.z != b->p.z) return a->p.z < b->p.z ? -1 : 1;
    return a->idx < b->idx ? -1 : a->idx > b->idx;
}

static int cmp_u32(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    return a < b ? -1 : a > b;
}

/* 2D extreme points of points lying in one plane: drop the coordinate of
 * the normal's largest component, then Andrew's chain (pop on turns <= 0). */
static int flat_hull(IP *u, int m, P3 nrm, uint32_t *out)
{
    int drop = 0;
    int64_t ax = nrm.x < 0 ? -nrm.x : nrm.x, ay = nrm.y < 0 ? -nrm.y : nrm.y, az = nrm.z < 0 ? -nrm.z : nrm.z;
    if (ay > ax && ay >= az) drop = 1;
    else if (az > ax && az > ay) drop = 2;
    int64_t (*q)[2] = malloc(sizeof(int64_t[2]) * (size_t)m);
    int *ord = malloc(sizeof(int) * (size_t)m), *st = malloc(sizeof(int) * (size_t)(2 * m + 2));
    for (int i = 0; i < m; i++) {
        int64_t c3[3] = {u[i].p.x, u[i].p.y, u[i].p.z};
        q[i][0] = c3[drop == 0 ? 1 : 0];
        q[i][1] = c3[drop == 2 ? 1 : 2];
        ord[i] = i;
    }
    /* sort by projected (a, b); projection is one-to-one on the plane */
    for (int i = 1; i < m; i++) {
        int t = ord[i], j = i - 1;
        while (j >= 0 && (q[ord[j]][0] > q[t][0] || (q[ord[j]][0] == q[t][0] && q[ord[j]][1] > q[t][1]))) {
            ord[j + 1] = ord[j];
            j--;
        }
        ord[j + 1] = t;
    }
    int k = 0;
    for (int pass = 0; pass < 2; pass++) {
        int start = k;
        for (int ii = 0; ii < m; ii++) {
            int i = pass == 0 ? ord[ii] : ord[m - 1 - ii];
            while (k >= start + 2) {
                int a = st[k - 2], b = st[k - 1];
                i128 cr = (i128)(q[b][0] - q[a][0]) * (q[i][1] - q[a][1]) -
                          (i128)(q[b][1] - q[a][1]) * (q[i][0] - q[a][0]);
                if (cr > 0) break;
                k--;
            }
            st[k++] = i;
        }
        k--;   /* the last point starts the other chain */
    }
    int h = m == 1 ? 1 : k;
    for (int i = 0; i < h; i++) out[i] = u[st[i]].idx;
    if (m == 1) out[0] = u[0].idx;
    free(q);
    free(ord);
    free(st);
    return h;
}

int oracle3_hull_subset(const float *x, const float *y, const float *z, const uint32_t *idx,
                        int64_t k, uint32_t *out, int64_t *h)
{
    *h = 0;
    if (k == 0) return 0;
    IP *u = malloc(sizeof(IP) * (size_t)k);
    for (int64_t i = 0; i < k; i++) {
        u[i].idx = idx ? idx[i] : (uint32_t)i;
        u[i].p = pt(x, y, z, u[i].idx);
    }
    qsort(u, (size_t)k, sizeof(IP), cmp_ip);
    int64_t m = 0;
    for (int64_t i = 0; i < k; i++)
        if (m == 0 || u[i].p.x != u[m - 1].p.x || u[i].p.y != u[m - 1].p.y || u[i].p.z != u[m - 1].p.z)
            u[m++] = u[i];
    /* four affinely independent points */
    int64_t i1 = -1, i2 = -1, i3 = -1;
    for (int64_t i = 1; i < m && i1 < 0; i++) i1 = i;
    P3 nrm = {0, 0, 0};
    for (int64_t i = 1; i1 >= 0 && i < m && i2 < 0; i++) {
        P3 c = cross3(sub3(u[i1].p, u[0].p), sub3(u[i].p, u[0].p));
        if (!is_zero3(c)) { i2 = i; nrm = c; }
    }
    for (int64_t i = 1; i2 >= 0 && i < m && i3 < 0; i++)
        if (orient3(u[0].p, u[i1].p, u[i2].p, u[i].p) != 0) i3 = i;
    if (i3 < 0) {                       /* flat: one point, a segment or a polygon */
        if (m == 1) {
            out[0] = u[0].idx;
            *h = 1;
        } else if (i2 < 0) {            /* collinear: the two ends (sorted order) */
            out[0] = u[0].idx;
            out[1] = u[m - 1].idx;
            *h = 2;
        } else {
            *h = flat_hull(u, (int)m, nrm, out);
        }
        free(u);
        qsort(out, (size_t)*h, sizeof(uint32_t), cmp_u32);
        return 0;
    }
    /* insertion order: the tetrahedron, then the rest in a fixed shuffle */
    int64_t *ord = malloc(sizeof(int64_t) * (size_t)m);
    int64_t no = 0;
    ord[no++] = 0; ord[no++] = i1; ord[no++] = i2; ord[no++] = i3;
    for (int64_t i = 1; i < m; i++)
        if (i != i1 && i != i2 && i != i3) ord[no++] = i;
    uint64_t rs = 0x9E3779B97F4A7C15ull;
    for (int64_t i = m - 1; i > 4; i--) {
        rs = rs * 6364136223846793005ull + 1442695040888963407ull;
        int64_t j = 4 + (int64_t)((rs >> 33) % (uint64_t)(i - 3));
        int64_t t = ord[i]; ord[i] = ord[j]; ord[j] = t;
    }
    size_t fcap = 1024;
    Face *F = malloc(sizeof(Face) * fcap);
    int nfc = 0;
    /* tetrahedron faces, oriented so that the fourth point is behind each */
    {
        int64_t t[4] = {ord[0], ord[1], ord[2], ord[3]};
        int fv[4][3] = {{0, 1, 2}, {0, 3, 1}, {1, 3, 2}, {0, 2, 3}};
        if (orient3(u[t[0]].p, u[t[1]].p, u[t[2]].p, u[t[3]].p) > 0) {
            /* flip every face */
            for (int f = 0; f < 4; f++) { int s = fv[f][1]; fv[f][1] = fv[f][2]; fv[f][2] = s; }
        }
        for (int f = 0; f < 4; f++) {
            for (int e = 0; e < 3; e++) F[f].v[e] = (int)t[fv[f][e]];
            F[f].alive = 1;
        }
        nfc = 4;
        /* neighbours: the face sharing the reversed edge */
        for (int f = 0; f < 4; f++)
            for (int e = 0; e < 3; e++) {
                int a = F[f].v[e], b = F[f].v[(e + 1) % 3];
                for (int g = 0; g < 4; g++)
                    for (int e2 = 0; e2 < 3; e2++)
                        if (F[g].v[e2] == b && F[g].v[(e2 + 1) % 3] == a) F[f].nb[e] = g;
            }
    }
    int *vis = malloc(sizeof(int) * fcap);
    int *hz_face = NULL, *hz_edge = NULL;
    size_t hzcap = 0;
    int *start_of = malloc(sizeof(int) * (size_t)m), *end_of = malloc(sizeof(int) * (size_t)m);
    for (int64_t oi = 4; oi < m; oi++) {
        const int64_t pi = ord[oi];
        const P3 p = u[pi].p;
        int any = 0;
        if ((size_t)nfc > fcap) abort();
        for (int f = 0; f < nfc; f++) {
            vis[f] = 0;
            if (!F[f].alive) continue;
            if (orient3(u[F[f].v[0]].p, u[F[f].v[1]].p, u[F[f].v[2]].p, p) > 0) { vis[f] = 1; any = 1; }
        }
        if (!any) continue;
        /* horizon: edges of visible faces whose neighbour is not visible */
        size_t nh = 0;
        for (int f = 0; f < nfc; f++) {
            if (!vis[f]) continue;
            for (int e = 0; e < 3; e++)
                if (!vis[F[f].nb[e]]) {
                    if (nh == hzcap) {
                        hzcap = hzcap ? 2 * hzcap : 64;
                        hz_face = realloc(hz_face, sizeof(int) * hzcap);
                        hz_edge = realloc(hz_edge, sizeof(int) * hzcap);
                    }
                    hz_face[nh] = f;
                    hz_edge[nh] = e;
                    nh++;
                }
        }
        /* new faces (a, b, p) on every horizon edge a -> b */
        if ((size_t)nfc + nh + 8 > fcap) {
            while ((size_t)nfc + nh + 8 > fcap) fcap *= 2;
            F = realloc(F, sizeof(Face) * fcap);
            vis = realloc(vis, sizeof(int) * fcap);
        }
        const int first = nfc;
        for (size_t j = 0; j < nh; j++) {
            const int f = hz_face[j], e = hz_edge[j];
            const int a = F[f].v[e], b = F[f].v[(e + 1) % 3];
            const int g = F[f].nb[e];
            Face *nf = &F[nfc];
            nf->v[0] = a; nf->v[1] = b; nf->v[2] = (int)pi;
            nf->alive = 1;
            nf->nb[0] = g;
            /* the outside neighbour now borders the new face */
            for (int e2 = 0; e2 < 3; e2++)
                if (F[g].v[e2] == b && F[g].v[(e2 + 1) % 3] == a) F[g].nb[e2] = nfc;
            start_of[a] = nfc;
            end_of[b] = nfc;
            vis[nfc] = 0;
            nfc++;
        }
        for (int f = first; f < nfc; f++) {
            /* edge b -> p borders the new face starting at b; p -> a the one ending at a */
            F[f].nb[1] = start_of[F[f].v[1]];
            F[f].nb[2] = end_of[F[f].v[0]];
        }
        for (int f = 0; f < first; f++)
            if (vis[f]) F[f].alive = 0;
    }
    /* corners: vertices whose faces span at least three distinct planes */
    int64_t nh = 0;
    char *seen = calloc((size_t)m, 1);
    for (int f = 0; f < nfc; f++) {
        if (!F[f].alive) continue;
        for (int e = 0; e < 3; e++) {
            const int v = F[f].v[e];
            if (seen[v]) continue;
            seen[v] = 1;
            P3 pl[3];
            int np = 0;
            for (int g = 0; g < nfc && np < 3; g++) {
                if (!F[g].alive) continue;
                if (F[g].v[0] != v && F[g].v[1] != v && F[g].v[2] != v) continue;
                P3 nn = cross3(sub3(u[F[g].v[1]].p, u[F[g].v[0]].p), sub3(u[F[g].v[2]].p, u[F[g].v[0]].p));
                int same = 0;
                for (int t = 0; t < np; t++) {
                    /* parallel normals of faces through v: the same plane */
                    i128 cx = (i128)pl[t].y * nn.z - (i128)pl[t].z * nn.y;
                    i128 cy = (i128)pl[t].z * nn.x - (i128)pl[t].x * nn.z;
                    i128 cz = (i128)pl[t].x * nn.y - (i128)pl[t].y * nn.x;
                    if (cx == 0 && cy == 0 && cz == 0) same = 1;
                }
                if (!same) pl[np++] = nn;
            }
            if (np >= 3) out[nh++] = u[v].idx;
        }
    }
    free(seen);
    free(F);
    free(vis);
    free(hz_face);
    free(hz_edge);
    free(start_of);
    free(end_of);
    free(ord);
    free(u);
    qsort(out, (size_t)nh, sizeof(uint32_t), cmp_u32);
    *h = nh;
    return 0;
}

/* The whole 3D method (nofilter: the hull of all points). */
int oracle3_compute(const float *x, const float *y, const float *z, int64_t n, const double *c,
                    const double *s, int G, int nofilter, uint32_t *hull, int64_t *h,
                    uint32_t *surv_out, int64_t *n_surv)
{
    if (G < 1 || G > 16) return -1;
    uint32_t *sv = malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    int64_t cnt = 0;
    if (nofilter) {
        for (int64_t i = 0; i < n; i++) sv[i] = (uint32_t)i;
        cnt = n;
    } else {
        const int ns = 6 + 12 * (G - 1);
        uint32_t slots[6 + 12 * 15];
        double vals[6 + 12 * 15];
        oracle3_extremes(x, y, z, n, c, s, G, slots, vals);
        int64_t planes[6 * 4096];
        int nf = oracle3_polyhedron(x, y, z, slots, ns, planes, 4096);
        if (nf > 4096) { free(sv); return -1; }
        oracle3_discard(x, y, z, n, planes, nf, sv, &cnt);
    }
    if (surv_out) memcpy(surv_out, sv, sizeof(uint32_t) * (size_t)cnt);
    if (n_surv) *n_surv = cnt;
    int rc = oracle3_hull_subset(x, y, z, sv, cnt, hull, h);
    free(sv);
    return rc;
}
