// The method in three dimensions (the paper's Sec. 5 names the 3D extension
// as its next step): extremes along the directions of rotations about each
// axis, the convex polyhedron of those extremes, the strict-inside discard,
// and the hull of the survivors.
//
// Points are three float32 arrays on the 2^-24 grid, 16-byte aligned; in
// grid units every coordinate is an integer below 2^24, so every predicate
// is decided exactly: plane normals (cross products of 25-bit differences)
// fit in int64 and are exact in binary64, and a plane evaluated at a point
// (up to 2^75) is first estimated in binary64 with an error bound and, only
// when that bound cannot decide the sign, recomputed in 128-bit integers.
//
// Slots (Step 1): [0..5] = argmin x, argmax x, argmin y, argmax y,
// argmin z, argmax z; then for the rotations about z, x and y (planes
// (x, y), (y, z), (z, x)) and each non-zero angle g = 1..3 of the preset:
// 6 + 4 (3 k + g - 1) + {argmin u, argmax u, argmin v, argmax v}, with
// u = c a - s b, v = s a + c b for the plane's coordinates (a, b), each
// product rounded to binary64 and then the sum.  Lowest index on ties.
#include "hg_device.h"

namespace hg {

constexpr int S3 = 42;                  // slots for the paper's four-group presets
constexpr int S3_PART0 = 18;            // pass 0: axes and plane (x, y); pass 1: the rest
constexpr int F3_CAP = 256;             // polyhedron planes kept
constexpr int TRIPLES3 = S3 * (S3 - 1) * (S3 - 2) / 6;

// Exact integer point and plane helpers (grid units).
struct I3 {
    int64_t x, y, z;
};
__device__ __forceinline__ I3 i3_sub(I3 a, I3 b) { return I3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ I3 i3_cross(I3 a, I3 b) {
    return I3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ __int128 i3_dot(I3 n, I3 d) {
    return (__int128)n.x * d.x + (__int128)n.y * d.y + (__int128)n.z * d.z;
}
__device__ __forceinline__ I3 grid3(const float *x, const float *y, const float *z, uint32_t i) {
    return I3{(int64_t)(x[i] * GRIDF), (int64_t)(y[i] * GRIDF), (int64_t)(z[i] * GRIDF)};
}

// A plane: normal (exact integers held in binary64, |n_i| < 2^51), an
// anchor point on it (grid units) and the bound of the binary64 evaluation's
// rounding error.  Polyhedron planes point inwards, hull faces outwards.
struct Plane3 {
    double nx, ny, nz;
    double ax, ay, az;
    double bound;
};

__device__ __forceinline__ Plane3 make_plane(I3 n, I3 a) {
    Plane3 P;
    P.nx = (double)n.x; P.ny = (double)n.y; P.nz = (double)n.z;
    P.ax = (double)a.x; P.ay = (double)a.y; P.az = (double)a.z;
    // three products of |n_i| < 2^51 by |d_i| < 2^25 and two sums: the
    // rounding error stays far below 2^-49 |n|_1 2^25
    P.bound = (fabs(P.nx) + fabs(P.ny) + fabs(P.nz)) * 0x1p-24;
    return P;
}

// Sign of the plane at grid point (px, py, pz): binary64 estimate, exact
// 128-bit fallback when it is within the error bound.
__device__ __forceinline__ int plane_sign(const Plane3 &P, double px, double py, double pz) {
    const double e = fma(P.nz, pz - P.az, fma(P.ny, py - P.ay, P.nx * (px - P.ax)));
    if (e > P.bound) return 1;
    if (e < -P.bound) return -1;
    const __int128 v = (__int128)(int64_t)P.nx * (int64_t)(px - P.ax) +
                       (__int128)(int64_t)P.ny * (int64_t)(py - P.ay) +
                       (__int128)(int64_t)P.nz * (int64_t)(pz - P.az);
    return v > 0 ? 1 : v < 0 ? -1 : 0;
}
// Distance estimate of a point beyond a plane (for choosing far points).
__device__ __forceinline__ double plane_dist(const Plane3 &P, double px, double py, double pz) {
    const double e = fma(P.nz, pz - P.az, fma(P.ny, py - P.ay, P.nx * (px - P.ax)));
    return e * rsqrt(P.nx * P.nx + P.ny * P.ny + P.nz * P.nz);
}

// ---------------------------------------------------------------------------
// Step 1: directional extremes, two passes over the points (the slots
// [0, 18) and [18, 42)); each wave walks a contiguous run of tiles and keeps
// per lane the best key of every slot and the tile where it first reached
// it, resolved to the lowest index once at the end of its run.
template <int PART>
struct Keys3 {
    static constexpr int K0 = PART == 0 ? 0 : S3_PART0;
    static constexpr int NK = PART == 0 ? S3_PART0 : S3 - S3_PART0;
    __device__ __forceinline__ static void eval(const Dirs &d, double X, double Y, double Z, double *key) {
#pragma clang fp contract(off)
        double full[S3];
        full[0] = X; full[1] = X; full[2] = Y; full[3] = Y; full[4] = Z; full[5] = Z;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            if (PART == 0 && k > 0) continue;
            if (PART == 1 && k == 0) continue;
            const double a = k == 0 ? X : k == 1 ? Y : Z;
            const double b = k == 0 ? Y : k == 1 ? Z : X;
#pragma unroll
            for (int g = 1; g < 4; g++) {
                const double c = d.gc[g], s = d.gs[g];
                const double u = c * a - s * b, v = s * a + c * b;
                const int base = 6 + 4 * (3 * k + g - 1);
                full[base + 0] = u; full[base + 1] = u; full[base + 2] = v; full[base + 3] = v;
            }
        }
#pragma unroll
        for (int j = 0; j < NK; j++) key[j] = full[K0 + j];
    }
};

template <int PART>
__global__ __launch_bounds__(256) void k3_extremes(const float *__restrict__ x, const float *__restrict__ y,
                                                  const float *__restrict__ z, int64_t n, Dirs dirs,
                                                  double *__restrict__ pval, uint32_t *__restrict__ pidx) {
    using K = Keys3<PART>;
    constexpr int NK = K::NK;
    const int lane = lane_id();
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t W = (int64_t(gridDim.x) * blockDim.x) >> 6;
    const int64_t T = (n + TILE - 1) / TILE;
    const int64_t q = (T + W - 1) / W;
    const int64_t t0 = min(wave * q, T), t1 = min(t0 + q, T);
    double lb[NK];
    uint32_t rt[NK];
#pragma unroll
    for (int k = 0; k < NK; k++) {
        lb[k] = ((K::K0 + k) & 1) ? -INFINITY : INFINITY;
        rt[k] = NONE;
    }
    for (int64_t t = t0; t < t1; t++) {
        const int64_t tb = t * TILE;
        float xv[TILE_CHUNKS][4], yv[TILE_CHUNKS][4], zv[TILE_CHUNKS][4];
        if (tb + TILE <= n) {
            typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int c = 0; c < TILE_CHUNKS; c++) {
                const int64_t a = tb + c * CHUNK + 4 * lane;
                const f4 fx = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(x + a));
                const f4 fy = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(y + a));
                const f4 fz = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(z + a));
                xv[c][0] = fx.x; xv[c][1] = fx.y; xv[c][2] = fx.z; xv[c][3] = fx.w;
                yv[c][0] = fy.x; yv[c][1] = fy.y; yv[c][2] = fy.z; yv[c][3] = fy.w;
                zv[c][0] = fz.x; zv[c][1] = fz.y; zv[c][2] = fz.z; zv[c][3] = fz.w;
            }
        } else {
#pragma unroll
            for (int c = 0; c < TILE_CHUNKS; c++)
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int64_t p = tb + c * CHUNK + 4 * lane + j;
                    const int64_t pc = p < n ? p : tb;      // the tile's first point stands in
                    xv[c][j] = x[pc];
                    yv[c][j] = y[pc];
                    zv[c][j] = z[pc];
                }
        }
        double acc[NK];
#pragma unroll
        for (int c = 0; c < TILE_CHUNKS; c++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                double key[NK];
                K::eval(dirs, (double)xv[c][j], (double)yv[c][j], (double)zv[c][j], key);
#pragma unroll
                for (int k = 0; k < NK; k++)
                    acc[k] = (c == 0 && j == 0) ? key[k]
                             : ((K::K0 + k) & 1) ? fmax(acc[k], key[k]) : fmin(acc[k], key[k]);
            }
        const uint32_t rel = (uint32_t)(t - t0);
#pragma unroll
        for (int k = 0; k < NK; k++) {
            const bool upd = ((K::K0 + k) & 1) ? acc[k] > lb[k] : acc[k] < lb[k];
            lb[k] = upd ? acc[k] : lb[k];
            rt[k] = upd ? rel : rt[k];
        }
    }
    // resolve: the run's extreme of each slot, then the lowest index that
    // reaches it (each lane holding it rescans its 16 points of that tile);
    // unrolled so that every array index is a constant (registers, no
    // scratch)
#pragma unroll
    for (int k = 0; k < NK; k++) {
        const bool mx = (K::K0 + k) & 1;
        double m = lb[k];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double v = __shfl_xor(m, o);
            m = mx ? fmax(m, v) : fmin(m, v);
        }
        uint32_t found = NONE;
        if (rt[k] != NONE && lb[k] == m) {
            const int64_t tb = (t0 + rt[k]) * TILE;
            for (int c = 0; c < TILE_CHUNKS && found == NONE; c++)
                for (int j = 0; j < 4; j++) {
                    const int64_t p = tb + c * CHUNK + 4 * lane + j;
                    if (p >= n) continue;
                    double key[NK];
                    K::eval(dirs, (double)x[p], (double)y[p], (double)z[p], key);
                    if (key[k] == m) {
                        found = (uint32_t)p;
                        break;
                    }
                }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) found = min(found, (uint32_t)__shfl_xor((int)found, o));
        if (lane == 0) {
            pval[wave * S3 + K::K0 + k] = m;
            pidx[wave * S3 + K::K0 + k] = t0 < t1 ? found : NONE;
        }
    }
}

// ---------------------------------------------------------------------------
// Step 2, one block: reduce the waves' partials to the slots, then the
// polyhedron of the distinct slot points: every plane through three of them
// with all of them on one side and at least one strictly, deduplicated and
// oriented inwards.  Also the inscribed ball used as a quick accept (centre:
// the mean of the distinct points, strictly inside when there is an
// interior; radius: the least binary64 distance to a plane, reduced by a
// safety margin), and the distinct points for the hull stage.
struct Poly3 {
    int nf;                 // planes; 0: no interior, nothing is discarded
    int m;                  // distinct slot points
    double cx, cy, cz;      // quick-accept ball: (p - c)^2 < r2 is strictly inside
    double r2;
    uint32_t pts[S3];       // the distinct slot points (indices)
    Plane3 f[F3_CAP];
};

// Triple number t -> (i < j < k) over S3 points.
__device__ __forceinline__ void triple_of(int t, int &i, int &j, int &k) {
    int rem = t, cnt;
    i = 0;
    while (rem >= (cnt = (S3 - 1 - i) * (S3 - 2 - i) / 2)) { rem -= cnt; i++; }
    j = i + 1;
    while (rem >= (cnt = S3 - 1 - j)) { rem -= cnt; j++; }
    k = j + 1 + rem;
}

__device__ __forceinline__ bool i3_zero(I3 a) { return a.x == 0 && a.y == 0 && a.z == 0; }

constexpr int TWORDS3 = (TRIPLES3 + 63) / 64;

__global__ __launch_bounds__(1024) void k3_poly(const float *__restrict__ x, const float *__restrict__ y,
                                                const float *__restrict__ z, int64_t W,
                                                const double *__restrict__ pval,
                                                const uint32_t *__restrict__ pidx,
                                                uint32_t *__restrict__ slots_out, Poly3 *__restrict__ out) {
    __shared__ uint32_t bi[S3];
    __shared__ I3 qs[S3];
    __shared__ I3 q[S3];
    __shared__ uint32_t qi[S3];
    __shared__ int m, nf;
    __shared__ unsigned long long keep[TWORDS3], flipb[TWORDS3];
    __shared__ int wpre[TWORDS3];
    __shared__ I3 fn[F3_CAP];
    __shared__ I3 fa[F3_CAP];
    __shared__ double rmin[1024 / WAVE];
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6, NW = blockDim.x >> 6;
    // 1. slots: wave w reduces slots w, w + NW, ... over the partials
    for (int k = w; k < S3; k += NW) {
        const bool mx = k & 1;
        double v = mx ? -INFINITY : INFINITY;
        uint32_t i = NONE;
        for (int64_t r = lane; r < W; r += WAVE) {
            const uint32_t ii = pidx[r * S3 + k];
            const double vv = pval[r * S3 + k];
            if (ii == NONE) continue;
            if (i == NONE || (mx ? vv > v : vv < v) || (vv == v && ii < i)) { v = vv; i = ii; }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double ov = __shfl_xor(v, o);
            const uint32_t oi = (uint32_t)__shfl_xor((int)i, o);
            if (oi != NONE && (i == NONE || (mx ? ov > v : ov < v) || (ov == v && oi < i))) { v = ov; i = oi; }
        }
        if (lane == 0) bi[k] = i;
    }
    for (int i = tid; i < TWORDS3; i += blockDim.x) { keep[i] = 0; flipb[i] = 0; }
    __syncthreads();
    if (tid < S3 && slots_out) slots_out[tid] = bi[tid];
    // 2. distinct points: the first slot of each coordinate triple, in slot order
    if (w == 0) {
        const bool valid = lane < S3 && bi[lane] != NONE;
        I3 p{0, 0, 0};
        if (valid) p = grid3(x, y, z, bi[lane]);
        if (lane < S3) qs[lane] = p;
        wave_sync();
        bool first = valid;
        for (int j = 0; j < lane && first; j++)
            if (bi[j] != NONE && qs[j].x == p.x && qs[j].y == p.y && qs[j].z == p.z) first = false;
        const uint64_t bm = __ballot(first);
        if (first) {
            const int pos = __popcll(bm & lanemask_lt());
            q[pos] = p;
            qi[pos] = bi[lane];
        }
        if (lane == 0) m = __popcll(bm);
    }
    __syncthreads();
    // 3. supporting planes through three distinct points; of the triples on
    // one plane only the canonical one is kept: the plane's two lowest
    // points and the lowest point after them off their line
    const int mm = m;
    for (int t = tid; t < TRIPLES3; t += blockDim.x) {
        int i, j, k;
        triple_of(t, i, j, k);
        if (k >= mm) continue;
        const I3 nrm = i3_cross(i3_sub(q[j], q[i]), i3_sub(q[k], q[i]));
        if (i3_zero(nrm)) continue;
        const Plane3 P = make_plane(nrm, q[i]);
        int pos = 0, neg = 0;
        unsigned long long on = 0;
        for (int r = 0; r < mm; r++) {
            const int sg = plane_sign(P, (double)q[r].x, (double)q[r].y, (double)q[r].z);
            pos += sg > 0;
            neg += sg < 0;
            on |= (unsigned long long)(sg == 0) << r;
        }
        if ((pos && neg) || (!pos && !neg)) continue;
        const int i0 = __ffsll(on) - 1;
        const unsigned long long on1 = on & (on - 1);
        const int j0 = __ffsll(on1) - 1;
        if (i != i0 || j != j0) continue;
        int k0 = -1;
        for (unsigned long long rest = on1 & (on1 - 1); rest; rest &= rest - 1) {
            const int r = __ffsll(rest) - 1;
            if (!i3_zero(i3_cross(i3_sub(q[j0], q[i0]), i3_sub(q[r], q[i0])))) { k0 = r; break; }
        }
        if (k != k0) continue;
        atomicOr(&keep[t >> 6], 1ull << (t & 63));
        if (neg) atomicOr(&flipb[t >> 6], 1ull << (t & 63));   // inwards: towards the points off it
    }
    __syncthreads();
    // 4. the kept planes in triple order
    if (tid == 0) {
        int sum = 0;
        for (int wd = 0; wd < TWORDS3; wd++) { wpre[wd] = sum; sum += __popcll(keep[wd]); }
        nf = min(sum, F3_CAP);      // at most 2 * 42 - 4 faces
    }
    __syncthreads();
    for (int t = tid; t < TRIPLES3; t += blockDim.x) {
        const unsigned long long kw = keep[t >> 6], bit = 1ull << (t & 63);
        if (!(kw & bit)) continue;
        const int pos = wpre[t >> 6] + __popcll(kw & (bit - 1));
        if (pos >= F3_CAP) continue;
        int i, j, k;
        triple_of(t, i, j, k);
        I3 nrm = i3_cross(i3_sub(q[j], q[i]), i3_sub(q[k], q[i]));
        if (flipb[t >> 6] & bit) nrm = I3{-nrm.x, -nrm.y, -nrm.z};
        fn[pos] = nrm;
        fa[pos] = q[i];
    }
    __syncthreads();
    // 5. output and the quick-accept ball
    const int nff = nf;
    for (int g = tid; g < nff; g += blockDim.x) out->f[g] = make_plane(fn[g], fa[g]);
    if (tid < mm) out->pts[tid] = qi[tid];
    double cx = 0, cy = 0, cz = 0;
    for (int r = 0; r < mm; r++) { cx += (double)q[r].x; cy += (double)q[r].y; cz += (double)q[r].z; }
    cx /= mm > 0 ? mm : 1; cy /= mm > 0 ? mm : 1; cz /= mm > 0 ? mm : 1;
    double r = INFINITY;
    for (int g = tid; g < nff; g += blockDim.x) {
        const I3 nn = fn[g], a = fa[g];
        const double e = (double)nn.x * (cx - (double)a.x) + (double)nn.y * (cy - (double)a.y) +
                         (double)nn.z * (cz - (double)a.z);
        const double len = sqrt((double)nn.x * nn.x + (double)nn.y * nn.y + (double)nn.z * nn.z);
        r = fmin(r, e / len);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) r = fmin(r, __shfl_xor(r, o));
    if (lane == 0) rmin[w] = r;
    __syncthreads();
    if (tid == 0) {
        for (int ww = 1; ww < NW; ww++) r = fmin(r, rmin[ww]);
        out->nf = nff;
        out->m = mm;
        // relative and absolute margins far above the rounding of these sums
        const double rs = nff > 0 ? r * (1.0 - 0x1p-20) - 4.0 : -1.0;
        out->cx = cx; out->cy = cy; out->cz = cz;
        out->r2 = rs > 0 ? rs * rs * (1.0 - 0x1p-20) : -1.0;
    }
}

// ---------------------------------------------------------------------------
// Step 3: strict-inside test, survivor masks and counts per tile in the
// layout of the 2D passes (bit l of word 4 c + j: point c*256 + 4 l + j).
// Each lane takes its four points of a chunk together through the planes.
// A plane is evaluated as n.p - n.a with n.a rounded once per block: both
// dot products stay below |n|_1 2^24, so the three roundings of each, and
// the final subtraction, err by less than |n|_1 2^-26, inside the plane's
// bound |n|_1 2^-24; within the bound the sign is taken exactly.
struct PlaneK {
    double nx, ny, nz, na, bound;
};

__global__ __launch_bounds__(256) void k3_discard(const float *__restrict__ x, const float *__restrict__ y,
                                                  const float *__restrict__ z, int64_t n,
                                                  const Poly3 *__restrict__ P, uint64_t *__restrict__ masks,
                                                  uint32_t *__restrict__ tile_cnt) {
    __shared__ Plane3 fl[F3_CAP];
    __shared__ PlaneK fk[F3_CAP];
    __shared__ int nfs;
    __shared__ double ball[4];
    const int tid = threadIdx.x, lane = lane_id();
    if (tid == 0) {
        nfs = P->nf;
        ball[0] = P->cx; ball[1] = P->cy; ball[2] = P->cz; ball[3] = P->r2;
    }
    __syncthreads();
    const int nf = nfs;
    for (int g = tid; g < nf; g += blockDim.x) {
        const Plane3 Q = P->f[g];
        fl[g] = Q;
        PlaneK K;
        K.nx = Q.nx; K.ny = Q.ny; K.nz = Q.nz;
        K.na = fma(Q.nz, Q.az, fma(Q.ny, Q.ay, Q.nx * Q.ax));
        K.bound = Q.bound;
        fk[g] = K;
    }
    __syncthreads();
    const double cx = ball[0], cy = ball[1], cz = ball[2], r2 = ball[3];
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + tid) >> 6;
    const int64_t W = (int64_t(gridDim.x) * blockDim.x) >> 6;
    const int64_t T = (n + TILE - 1) / TILE;
    for (int64_t t = wave; t < T; t += W) {
        const int64_t tb = t * TILE;
        const bool full = tb + TILE <= n;
        uint32_t cnt = 0;
#pragma unroll 1
        for (int c = 0; c < TILE_CHUNKS; c++) {
            const int64_t p0 = tb + c * CHUNK + 4 * lane;
            float xs[4], ys[4], zs[4];
            bool valid[4];
            if (full) {
                const float4 X = *reinterpret_cast<const float4 *>(x + p0);
                const float4 Y = *reinterpret_cast<const float4 *>(y + p0);
                const float4 Z = *reinterpret_cast<const float4 *>(z + p0);
                xs[0] = X.x; xs[1] = X.y; xs[2] = X.z; xs[3] = X.w;
                ys[0] = Y.x; ys[1] = Y.y; ys[2] = Y.z; ys[3] = Y.w;
                zs[0] = Z.x; zs[1] = Z.y; zs[2] = Z.z; zs[3] = Z.w;
#pragma unroll
                for (int j = 0; j < 4; j++) valid[j] = true;
            } else {
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    valid[j] = p0 + j < n;
                    xs[j] = valid[j] ? x[p0 + j] : 0.f;
                    ys[j] = valid[j] ? y[p0 + j] : 0.f;
                    zs[j] = valid[j] ? z[p0 + j] : 0.f;
                }
            }
            double px[4], py[4], pz[4];
            bool live[4], out[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                px[j] = (double)(int64_t)(xs[j] * GRIDF);
                py[j] = (double)(int64_t)(ys[j] * GRIDF);
                pz[j] = (double)(int64_t)(zs[j] * GRIDF);
                const double dx = px[j] - cx, dy = py[j] - cy, dz = pz[j] - cz;
                const bool in_ball = dx * dx + dy * dy + dz * dz < r2;
                live[j] = valid[j] && nf > 0 && !in_ball;     // still to be tested
                out[j] = false;
            }
            for (int g = 0; g < nf; g++) {
                if (!__ballot(live[0] || live[1] || live[2] || live[3])) break;
                const PlaneK K = fk[g];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    if (!live[j]) continue;
                    const double e = fma(K.nz, pz[j], fma(K.ny, py[j], K.nx * px[j])) - K.na;
                    if (e > K.bound) continue;
                    if (e < -K.bound || plane_sign(fl[g], px[j], py[j], pz[j]) <= 0) {
                        live[j] = false;
                        out[j] = true;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const bool surv = valid[j] && (nf == 0 || out[j]);
                const uint64_t bm = __ballot(surv);
                cnt += (uint32_t)__popcll(bm);
                if (lane == 0) masks[t * TILE_WORDS + c * 4 + j] = bm;
            }
        }
        if (lane == 0) tile_cnt[t] = cnt;
    }
}

// ---------------------------------------------------------------------------
// Step 4: the extreme points of the survivors, QuickHull by rounds.
//
// Start: a tetrahedron of survivors (the first survivor, the one farthest
// from it, the one farthest from their line, the one farthest from their
// plane).  A round assigns every candidate to one face of the current hull
// that it lies strictly beyond (its face of the last round while that face
// lives, else one of the faces the last round created: a point beyond a
// face that an insertion removes is either inside the new hull or beyond one
// of the faces that insertion creates) and drops the others, which lie
// inside or on the hull of points already taken; then each face's farthest
// candidate (lowest index among equal distances) is inserted: the faces it
// sees strictly are removed and the horizon is joined to it.  The hull is
// final when no candidate is beyond any face.  Neighbouring coplanar faces
// are not merged, so the extreme points are the vertices whose incident
// faces span at least three distinct planes.  Copies of a point (equal
// coordinates) make every decision together, so the one inserted is the
// lowest index among them.
struct Face3 {
    int v[3];       // point indices, counter-clockwise seen from outside
    int nb[3];      // face across edge v[e] -> v[(e + 1) % 3]
    int alive;
    int pad;
};

struct Hull3Ctl {
    unsigned long long seed[3];   // farthest-point keys of the start
    int64_t lo_dot;               // collinear sets: smallest projection
    int64_t hi_dot;               // and largest
    int state;                    // 0 solid, 1 flat, 2 collinear, 3 one point, 4 empty
    int nfaces, fcap, born_lo;
    int ncand, nout, inserted, overflow;
    int ncorner, lo_idx, hi_idx, npair;
    uint32_t p[4];                // start simplex
    int64_t nrm[3];               // flat sets: their plane's normal
};

__device__ __forceinline__ double pdx(const float *v, uint32_t i) { return (double)(int64_t)(v[i] * GRIDF); }

// far key: distance estimate (non-negative float bits) above, ~index below
__device__ __forceinline__ unsigned long long key_of(double d, uint32_t i) {
    const float f = d > 0 ? (float)d : 0.0f;
    return ((unsigned long long)__float_as_uint(f) << 32) | (unsigned long long)(~i);
}

// Start, phase 1..3: candidate farthest from p0 / from line p0 p1 / from the
// plane p0 p1 p2, by atomic maximum of (distance estimate, ~index); a
// distance that is exactly zero gives key 0.
__global__ __launch_bounds__(256) void k3_seed(const float *__restrict__ x, const float *__restrict__ y,
                                               const float *__restrict__ z, const uint32_t *__restrict__ cand,
                                               int64_t nc, int phase, Hull3Ctl *__restrict__ C) {
    if (nc <= 0) return;
    // a phase runs only when the one before found a point
    if (phase >= 2 && C->seed[0] == 0) return;
    if (phase >= 3 && C->seed[1] == 0) return;
    const uint32_t i0 = cand[0];
    const I3 a = grid3(x, y, z, i0);
    I3 b{0, 0, 0}, c{0, 0, 0};
    if (phase >= 2) b = grid3(x, y, z, (uint32_t)~(uint32_t)C->seed[0]);
    if (phase >= 3) c = grid3(x, y, z, (uint32_t)~(uint32_t)C->seed[1]);
    unsigned long long best = 0;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < nc; t += int64_t(gridDim.x) * blockDim.x) {
        const uint32_t i = cand[t];
        const I3 p = grid3(x, y, z, i);
        const I3 d = i3_sub(p, a);
        double est = 0;
        bool nz = false;
        if (phase == 1) {
            nz = d.x != 0 || d.y != 0 || d.z != 0;
            est = (double)d.x * d.x + (double)d.y * d.y + (double)d.z * d.z;
        } else if (phase == 2) {
            const I3 cr = i3_cross(i3_sub(b, a), d);
            nz = cr.x != 0 || cr.y != 0 || cr.z != 0;
            est = (double)cr.x * cr.x + (double)cr.y * cr.y + (double)cr.z * cr.z;
        } else {
            const __int128 o = i3_dot(i3_cross(i3_sub(b, a), i3_sub(c, a)), d);
            nz = o != 0;
            const I3 nn = i3_cross(i3_sub(b, a), i3_sub(c, a));
            est = fabs((double)nn.x * d.x + (double)nn.y * d.y + (double)nn.z * d.z);
        }
        if (nz) {
            unsigned long long k = key_of(fmax(est, 1.0), i);
            best = k > best ? k : best;
        }
    }
    if (best) atomicMax(&C->seed[phase - 1], best);
}

// Collinear sets: smallest and largest projection on the line, then the
// lowest index reaching each.
__global__ __launch_bounds__(256) void k3_line(const float *__restrict__ x, const float *__restrict__ y,
                                               const float *__restrict__ z, const uint32_t *__restrict__ cand,
                                               int64_t nc, int phase, Hull3Ctl *__restrict__ C) {
    const I3 a = grid3(x, y, z, C->p[0]), b = grid3(x, y, z, C->p[1]);
    const I3 d = i3_sub(b, a);
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < nc; t += int64_t(gridDim.x) * blockDim.x) {
        const uint32_t i = cand[t];
        const I3 p = grid3(x, y, z, i);
        const I3 e = i3_sub(p, a);
        const long long dot = (long long)(d.x * e.x + d.y * e.y + d.z * e.z);   // |.| < 2^52
        if (phase == 0) {
            atomicMin((long long *)&C->lo_dot, dot);
            atomicMax((long long *)&C->hi_dot, dot);
        } else {
            if (dot == C->lo_dot) atomicMin((unsigned *)&C->lo_idx, i);
            if (dot == C->hi_dot) atomicMin((unsigned *)&C->hi_idx, i);
        }
    }
}

__device__ __forceinline__ void face_plane(const float *x, const float *y, const float *z, const Face3 &F,
                                           Plane3 *P) {
    const I3 a = grid3(x, y, z, (uint32_t)F.v[0]), b = grid3(x, y, z, (uint32_t)F.v[1]),
             c = grid3(x, y, z, (uint32_t)F.v[2]);
    *P = make_plane(i3_cross(i3_sub(b, a), i3_sub(c, a)), a);
}

// The start simplex (or the kind of degenerate set), one thread.
__global__ void k3_start(const float *__restrict__ x, const float *__restrict__ y, const float *__restrict__ z,
                         const uint32_t *__restrict__ cand, int64_t nc, Hull3Ctl *__restrict__ C,
                         Face3 *__restrict__ faces, Plane3 *__restrict__ planes,
                         unsigned long long *__restrict__ far) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    C->nfaces = 0;
    C->born_lo = 0;
    C->inserted = 0;
    C->overflow = 0;
    C->ncorner = 0;
    C->ncand = (int)nc;
    if (nc <= 0) { C->state = 4; return; }
    C->p[0] = cand[0];
    if (!C->seed[0]) { C->state = 3; return; }
    C->p[1] = ~(uint32_t)C->seed[0];
    if (!C->seed[1]) {
        C->state = 2;
        C->lo_dot = INT64_MAX;
        C->hi_dot = INT64_MIN;
        C->lo_idx = -1;
        C->hi_idx = -1;
        return;
    }
    C->p[2] = ~(uint32_t)C->seed[1];
    if (!C->seed[2]) {
        const I3 a = grid3(x, y, z, C->p[0]), b = grid3(x, y, z, C->p[1]), c = grid3(x, y, z, C->p[2]);
        const I3 nn = i3_cross(i3_sub(b, a), i3_sub(c, a));
        C->nrm[0] = nn.x; C->nrm[1] = nn.y; C->nrm[2] = nn.z;
        C->state = 1;
        return;
    }
    C->p[3] = ~(uint32_t)C->seed[2];
    C->state = 0;
    int t[4] = {(int)C->p[0], (int)C->p[1], (int)C->p[2], (int)C->p[3]};
    const I3 P0 = grid3(x, y, z, t[0]), P1 = grid3(x, y, z, t[1]), P2 = grid3(x, y, z, t[2]),
             P3 = grid3(x, y, z, t[3]);
    // faces (0 1 2), (0 3 1), (1 3 2), (0 2 3) face outwards when point 3 is
    // behind (0 1 2); otherwise every face is reversed
    int fv[4][3] = {{0, 1, 2}, {0, 3, 1}, {1, 3, 2}, {0, 2, 3}};
    const bool flip = i3_dot(i3_cross(i3_sub(P1, P0), i3_sub(P2, P0)), i3_sub(P3, P0)) > 0;
    for (int f = 0; f < 4; f++) {
        if (flip) { const int s = fv[f][1]; fv[f][1] = fv[f][2]; fv[f][2] = s; }
        for (int e = 0; e < 3; e++) faces[f].v[e] = t[fv[f][e]];
        faces[f].alive = 1;
        far[f] = 0;
    }
    for (int f = 0; f < 4; f++)
        for (int e = 0; e < 3; e++) {
            const int a = faces[f].v[e], b = faces[f].v[(e + 1) % 3];
            for (int g = 0; g < 4; g++)
                for (int e2 = 0; e2 < 3; e2++)
                    if (faces[g].v[e2] == b && faces[g].v[(e2 + 1) % 3] == a) faces[f].nb[e] = g;
        }
    for (int f = 0; f < 4; f++) face_plane(x, y, z, faces[f], &planes[f]);
    C->nfaces = 4;
}

// Candidates of the hull stage carry their coordinates: (x, y, z, index
// bits), so the rounds stream them instead of gathering from the inputs.
__global__ __launch_bounds__(256) void k3_gather(const float *__restrict__ x, const float *__restrict__ y,
                                                 const float *__restrict__ z, const uint32_t *__restrict__ idx,
                                                 int64_t n, float4 *__restrict__ out) {
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
        const uint32_t i = idx[t];
        out[t] = make_float4(x[i], y[i], z[i], __uint_as_float(i));
    }
}

// A round's assignment (see above).  first: every candidate tests the start
// faces.  A candidate whose face was removed follows the removals: the
// insertion that removed a face created faces repl[f] = (first, count); the
// candidate is beyond one of them (then it moves there, and on if that one
// was removed too) or inside the hull that insertion made (then it drops).
// A block takes AS_ITEMS * 256 candidates per step and appends the kept ones
// with one counter update; each wave merges the farthest keys of lanes that
// share a face before updating far[].
constexpr int CHAIN_MAX = 256;      // chain steps before a full scan
constexpr int AS_ITEMS = 4;
constexpr int AS_MERGE = 4;         // faces merged per wave and item; the rest update directly

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

__device__ __forceinline__ void far_raise(unsigned long long *slot, unsigned long long k) {
    if (__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) atomicMax(slot, k);
}

__global__ __launch_bounds__(256) void k3_assign(const float4 *__restrict__ cin, const int *__restrict__ fin,
                                                 float4 *__restrict__ cout, int *__restrict__ fout,
                                                 Hull3Ctl *__restrict__ C, const Face3 *__restrict__ faces,
                                                 const Plane3 *__restrict__ planes, const int2 *__restrict__ repl,
                                                 unsigned long long *__restrict__ far, int first) {
    __shared__ int bcnt, bbase;
    const int64_t nc = C->ncand;
    const int nfaces = C->nfaces;
    const int lane = lane_id();
    constexpr int STEP = 256 * AS_ITEMS;
    if (threadIdx.x == 0) bcnt = 0;
    __syncthreads();
    for (int64_t c0 = int64_t(blockIdx.x) * STEP; c0 < nc; c0 += int64_t(gridDim.x) * STEP) {
        float4 c[AS_ITEMS];
        int f[AS_ITEMS];
        unsigned long long key[AS_ITEMS];
#pragma unroll
        for (int it = 0; it < AS_ITEMS; it++) {
            const int64_t t = c0 + it * 256 + threadIdx.x;
            f[it] = -1;
            key[it] = 0;
            c[it] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (t >= nc) continue;
            c[it] = cin[t];
            const double px = (double)(int64_t)(c[it].x * GRIDF), py = (double)(int64_t)(c[it].y * GRIDF),
                         pz = (double)(int64_t)(c[it].z * GRIDF);
            auto best_of = [&](int lo, int hi, bool alive_only) {
                int bf = -1;
                double bd = 0;
                for (int g = lo; g < hi; g++) {
                    if (alive_only && !faces[g].alive) continue;
                    if (plane_sign(planes[g], px, py, pz) > 0) {
                        const double dg = plane_dist(planes[g], px, py, pz);
                        if (bf < 0 || dg > bd) { bf = g; bd = dg; }
                    }
                }
                return bf;
            };
            int g;
            if (first) {
                g = best_of(0, nfaces, true);
            } else {
                g = fin[t];
                int steps = 0;
                while (g >= 0 && !faces[g].alive && steps < CHAIN_MAX) {
                    const int2 r = repl[g];
                    g = best_of(r.x, r.x + r.y, false);
                    steps++;
                }
                if (g >= 0 && !faces[g].alive) g = best_of(0, nfaces, true);   // chain too long
            }
            f[it] = g;
            if (g >= 0) key[it] = key_of(plane_dist(planes[g], px, py, pz), __float_as_uint(c[it].w));
        }
        // appends: wave counts, a block offset, the wave's place in it
        uint64_t bal[AS_ITEMS];
        int wc = 0;
#pragma unroll
        for (int it = 0; it < AS_ITEMS; it++) {
            bal[it] = __ballot(f[it] >= 0);
            wc += __popcll(bal[it]);
        }
        int wo = 0;
        if (lane == 0 && wc) wo = atomicAdd(&bcnt, wc);
        wo = __shfl(wo, 0);
        __syncthreads();
        if (threadIdx.x == 0) {
            bbase = bcnt ? atomicAdd(&C->nout, bcnt) : 0;
            bcnt = 0;
        }
        __syncthreads();
        int o = bbase + wo;
#pragma unroll
        for (int it = 0; it < AS_ITEMS; it++) {
            if (f[it] >= 0) {
                const int at = o + __popcll(bal[it] & lanemask_lt());
                cout[at] = c[it];
                fout[at] = f[it];
            }
            o += __popcll(bal[it]);
        }
        // farthest keys: lanes on the same face merged first
#pragma unroll
        for (int it = 0; it < AS_ITEMS; it++) {
            bool pend = f[it] >= 0;
            uint64_t pm = bal[it];
            for (int r = 0; r < AS_MERGE && pm; r++) {
                const int lead = __ffsll((unsigned long long)pm) - 1;
                const int f0 = __shfl(f[it], lead);
                const bool mine = pend && f[it] == f0;
                const unsigned long long v = wave_max_u64(mine ? key[it] : 0ull);
                if (lane == lead) far_raise(&far[f0], v);
                pend = pend && !mine;
                pm = __ballot(pend);
            }
            if (pend) far_raise(&far[f[it]], key[it]);
        }
    }
}

// ---------------------------------------------------------------------------
// Parallel insertion.  Every face with candidates proposes its farthest one
// q.  Each proposal finds the faces q sees (breadth-first from its face) and
// the horizon, and claims those faces and the outside faces across the
// horizon with its priority (round, coarse distance, ~index; maximum wins).
// A proposal that holds every claim is inserted.  Two winners touch disjoint
// faces, so no face one of them creates is seen by the other and the
// insertions give the hull of inserting them one after another; the
// proposal of highest priority always wins, so every round inserts.
struct Pair3 {
    uint32_t q;
    int f;
    unsigned long long key;     // the far key of q on f
};
constexpr int PAIR_CAP = 16384;     // proposals per round at most
constexpr int PV_CAP = 512;         // faces seen, and horizon edges, per proposal
constexpr int INS_PASSES = 4;       // claim-and-insert passes per assignment

// Round start: the proposals.  Clears far[] for the next assignment.
__global__ __launch_bounds__(256) void k3_pick(Hull3Ctl *__restrict__ C, unsigned long long *__restrict__ far,
                                               Pair3 *__restrict__ pairs) {
    if (blockIdx.x == 0 && threadIdx.x == 0) C->inserted = 0;
    const int F = C->nfaces;
    const int64_t Fw = (F + WAVE - 1) / WAVE * WAVE;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < Fw; t += int64_t(gridDim.x) * blockDim.x) {
        const unsigned long long k = t < F ? far[t] : 0ull;
        if (k) far[t] = 0;
        const uint64_t m = __ballot(k != 0);
        if (m == 0) continue;
        const int lead = __ffsll((unsigned long long)m) - 1;
        int base = 0;
        if (lane_id() == lead) base = atomicAdd(&C->npair, __popcll(m));
        base = __shfl(base, lead);
        const int s = base + __popcll(m & lanemask_lt());
        if (k && s < PAIR_CAP) {
            Pair3 P;
            P.q = ~(uint32_t)k;
            P.f = (int)t;
            P.key = k;
            pairs[s] = P;
        }
    }
}

// Priority of a proposal in claim pass `stamp` (increasing over the whole
// hull stage, so claims left from earlier passes always lose).
__device__ __forceinline__ unsigned long long claim_prio(unsigned long long key, int stamp) {
    return ((unsigned long long)stamp << 44) | ((key >> 52) << 32) | (key & 0xffffffffull);
}

// One wave per proposal: the faces seen and the horizon, then the claims.
// pn[p] = (faces seen, horizon edges), or (-1, -1) when either list would
// exceed PV_CAP or the proposal's face is gone (inserted, or removed by
// another insertion: the proposal waits for the next round).  A proposal
// that lost a pass and whose face lives is still valid (its point is still
// strictly beyond a face of the hull) and tries again in the next pass.
__global__ __launch_bounds__(64) void k3_visible(const float *__restrict__ x, const float *__restrict__ y,
                                                 const float *__restrict__ z, Hull3Ctl *__restrict__ C,
                                                 const Face3 *__restrict__ faces, const Plane3 *__restrict__ planes,
                                                 const Pair3 *__restrict__ pairs, int *__restrict__ pv,
                                                 int *__restrict__ ph, int2 *__restrict__ pn,
                                                 unsigned long long *__restrict__ claim, int stamp) {
    __shared__ int vl[PV_CAP];
    __shared__ int hl[PV_CAP];
    __shared__ int tmp[WAVE];
    const int lane = threadIdx.x;
    const int np = min(C->npair, PAIR_CAP);
    for (int p = blockIdx.x; p < np; p += gridDim.x) {
        const Pair3 P = pairs[p];
        if (!faces[P.f].alive) {
            if (lane == 0) pn[p] = make_int2(-1, -1);
            continue;
        }
        const unsigned long long prio = claim_prio(P.key, stamp);
        const double qx = pdx(x, P.q), qy = pdx(y, P.q), qz = pdx(z, P.q);
        if (lane == 0) vl[0] = P.f;
        __syncthreads();
        int nv = 1, nh = 0, head = 0;
        bool ok = true;
        while (head < nv && ok) {
            const int nb = min(nv - head, WAVE / 3);
            int g = -1, code = 0;
            bool seen = false, hz = false;
            if (lane < 3 * nb) {
                const int fi = vl[head + lane / 3], e = lane % 3;
                code = (fi << 2) | e;
                g = faces[fi].nb[e];
                if (g < 0) {            // an open mesh: reported, never followed
                    atomicMax(&C->overflow, 2);
                } else {
                    seen = plane_sign(planes[g], qx, qy, qz) > 0;
                    hz = !seen;
                }
                for (int i = 0; i < nv && seen; i++)
                    if (vl[i] == g) seen = false;       // listed already
            }
            tmp[lane] = seen ? g : -1;
            __syncthreads();
            for (int j = 0; j < lane && seen; j++)
                if (tmp[j] == g) seen = false;          // a lower lane lists it
            const uint64_t mv = __ballot(seen), mh = __ballot(hz);
            const int cv = __popcll(mv), ch = __popcll(mh);
            if (nv + cv > PV_CAP || nh + ch > PV_CAP) {
                ok = false;
            } else {
                if (seen) vl[nv + __popcll(mv & lanemask_lt())] = g;
                if (hz) hl[nh + __popcll(mh & lanemask_lt())] = code;
            }
            __syncthreads();
            nv += cv;
            nh += ch;
            head += nb;
        }
        if (ok) {
            for (int i = lane; i < nv; i += WAVE) {
                pv[(int64_t)p * PV_CAP + i] = vl[i];
                atomicMax(&claim[vl[i]], prio);
            }
            for (int h = lane; h < nh; h += WAVE) {
                ph[(int64_t)p * PV_CAP + h] = hl[h];
                atomicMax(&claim[faces[hl[h] >> 2].nb[hl[h] & 3]], prio);
            }
        }
        if (lane == 0) pn[p] = ok ? make_int2(nv, nh) : make_int2(-1, -1);
        __syncthreads();
    }
}

// One wave per proposal: the winners insert.  New face F + h on horizon edge
// a -> b is (a, b, q); across a -> b it borders the outside face, across
// b -> q the new face starting at b, across q -> a the new face ending at a.
__global__ __launch_bounds__(64) void k3_apply(const float *__restrict__ x, const float *__restrict__ y,
                                               const float *__restrict__ z, Hull3Ctl *__restrict__ C,
                                               Face3 *__restrict__ faces, Plane3 *__restrict__ planes,
                                               unsigned long long *__restrict__ far, int *__restrict__ vis,
                                               int2 *__restrict__ repl, const Pair3 *__restrict__ pairs,
                                               const int *__restrict__ pv, const int *__restrict__ ph,
                                               const int2 *__restrict__ pn,
                                               const unsigned long long *__restrict__ claim, int stamp) {
    __shared__ int ha[PV_CAP], hb[PV_CAP], ho[PV_CAP];
    __shared__ int base;
    const int lane = threadIdx.x;
    const int np = min(C->npair, PAIR_CAP);
    const int fcap = C->fcap;
    for (int p = blockIdx.x; p < np; p += gridDim.x) {
        const int2 cnt = pn[p];
        if (cnt.x < 0) continue;
        const Pair3 P = pairs[p];
        const unsigned long long prio = claim_prio(P.key, stamp);
        const int *V = pv + (int64_t)p * PV_CAP;
        const int *Hz = ph + (int64_t)p * PV_CAP;
        const int NV = cnt.x, NH = cnt.y;
        bool won = true;
        for (int i = lane; i < NV; i += WAVE) won = won && claim[V[i]] == prio;
        for (int h = lane; h < NH; h += WAVE) {
            const int fi = Hz[h] >> 2, e = Hz[h] & 3;
            const int O = faces[fi].nb[e];
            won = won && claim[O] == prio;
            ha[h] = faces[fi].v[e];
            hb[h] = faces[fi].v[e == 2 ? 0 : e + 1];
            ho[h] = O;
        }
        if (__ballot(!won) != 0) {
            __syncthreads();
            continue;
        }
        if (lane == 0) base = atomicAdd(&C->nfaces, NH);
        __syncthreads();
        const int F = base;
        if (F + NH > fcap) {
            if (lane == 0) atomicOr(&C->overflow, 1);
            __syncthreads();
            continue;
        }
        bool bad = false;
        for (int h = lane; h < NH; h += WAVE) {
            const int a = ha[h], b = hb[h];
            Face3 nf;
            nf.v[0] = a; nf.v[1] = b; nf.v[2] = (int)P.q;
            nf.nb[0] = ho[h];
            nf.nb[1] = -1;
            nf.nb[2] = -1;
            for (int k = 0; k < NH; k++) {
                if (ha[k] == b) nf.nb[1] = F + k;
                if (hb[k] == a) nf.nb[2] = F + k;
            }
            bad = bad || nf.nb[1] < 0 || nf.nb[2] < 0;
            nf.alive = 1;
            nf.pad = 0;
            faces[F + h] = nf;
            face_plane(x, y, z, nf, &planes[F + h]);
            far[F + h] = 0;
            vis[F + h] = -1;
            // the outside face now borders the new one
            const int O = ho[h];
            for (int e2 = 0; e2 < 3; e2++)
                if (faces[O].v[e2] == b && faces[O].v[e2 == 2 ? 0 : e2 + 1] == a) faces[O].nb[e2] = F + h;
        }
        for (int i = lane; i < NV; i += WAVE) {
            faces[V[i]].alive = 0;
            repl[V[i]] = make_int2(F, NH);
        }
        if (__ballot(bad) != 0 && lane == 0) atomicMax(&C->overflow, 2);   // not a closed horizon
        if (lane == 0) atomicAdd(&C->inserted, 1);
        __syncthreads();
    }
}

// Round end: the assignment's output is the next round's input.
__global__ void k3_round_end(Hull3Ctl *__restrict__ C) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    C->ncand = C->nout;
    C->nout = 0;
    C->npair = 0;
}

constexpr int INS_THREADS = 1024;
constexpr int INS_LIST = 2048;      // points inserted per round at most
constexpr int HZ_CAP = 2048;        // horizon edges of one insertion
constexpr int VIS_CAP = 2048;       // faces one insertion removes

// A round's insertions, one block: each face's farthest candidate q, in turn.
// The faces q sees are found from the face it was assigned to, which it
// sees while that face lives (else q waits for the next round), by a
// breadth-first walk over neighbours: the faces a point sees form one
// connected patch whose border is the horizon.
__global__ __launch_bounds__(INS_THREADS) void k3_insert(const float *__restrict__ x, const float *__restrict__ y,
                                                         const float *__restrict__ z, Hull3Ctl *__restrict__ C,
                                                         Face3 *__restrict__ faces, Plane3 *__restrict__ planes,
                                                         unsigned long long *__restrict__ far,
                                                         int *__restrict__ vis, int2 *__restrict__ repl) {
    __shared__ uint32_t list[INS_LIST];
    __shared__ int lface[INS_LIST];
    __shared__ int nl, nh, nv, nf0, bad, over;
    __shared__ int fr_n[2];
    __shared__ int hz_f[HZ_CAP], hz_e[HZ_CAP];
    __shared__ int vlist[VIS_CAP];
    __shared__ int front[2][VIS_CAP];
    const int tid = threadIdx.x;
    if (tid == 0) {
        nl = 0;
        bad = 0;
        over = 0;
        nf0 = C->nfaces;
        C->inserted = 0;
        C->ncand = C->nout;     // the assignment's output is the next input
        C->nout = 0;
    }
    __syncthreads();
    const int F0 = nf0;
    for (int f = tid; f < F0; f += blockDim.x) {
        const unsigned long long k = far[f];
        if (k && faces[f].alive) {
            const int s = atomicAdd(&nl, 1);
            if (s < INS_LIST) { list[s] = ~(uint32_t)k; lface[s] = f; }
        }
        far[f] = 0;
    }
    __syncthreads();
    const int L = min(nl, INS_LIST);
    int inserted = 0;
    for (int li = 0; li < L; li++) {
        const uint32_t q = list[li];
        const int fq = lface[li];
        if (!faces[fq].alive) continue;      // removed by an earlier insertion: next round
        const double qx = pdx(x, q), qy = pdx(y, q), qz = pdx(z, q);
        const int tag = (int)q;              // faces seen by q carry its index
        const int F = C->nfaces;
        if (tid == 0) {
            nh = 0;
            nv = 1;
            vlist[0] = fq;
            vis[fq] = tag;
            front[0][0] = fq;
            fr_n[0] = 1;
            fr_n[1] = 0;
        }
        __syncthreads();
        int cur = 0;
        for (;;) {
            const int nfr = fr_n[cur];
            __syncthreads();
            if (nfr == 0 || over) break;
            if (tid == 0) fr_n[1 - cur] = 0;
            __syncthreads();
            for (int w = tid; w < 3 * nfr; w += blockDim.x) {
                const int f = front[cur][w / 3], e = w % 3;
                const int g = faces[f].nb[e];
                const int old = vis[g];
                if (old == tag) continue;
                if (plane_sign(planes[g], qx, qy, qz) > 0) {
                    if (atomicCAS(&vis[g], old, tag) == old) {
                        const int sv = atomicAdd(&nv, 1), sf = atomicAdd(&fr_n[1 - cur], 1);
                        if (sv < VIS_CAP && sf < VIS_CAP) {
                            vlist[sv] = g;
                            front[1 - cur][sf] = g;
                        } else {
                            over = 1;
                        }
                    }
                } else {
                    const int h = atomicAdd(&nh, 1);
                    if (h < HZ_CAP) { hz_f[h] = f; hz_e[h] = e; } else over = 1;
                }
            }
            __syncthreads();
            cur = 1 - cur;
        }
        const int H = nh, NV = nv;
        if (over || F + H > C->fcap) {
            if (tid == 0) C->overflow = 1;
            __syncthreads();
            break;
        }
        // new face F + h on horizon edge a -> b: (a, b, q); its neighbours:
        // across a -> b the outside face, across b -> q the new face starting
        // at b, across q -> a the new face ending at a
        for (int h = tid; h < H; h += blockDim.x) {
            const int f = hz_f[h], e = hz_e[h];
            const int a = faces[f].v[e], b = faces[f].v[(e + 1) % 3];
            Face3 nf;
            nf.v[0] = a; nf.v[1] = b; nf.v[2] = (int)q;
            nf.nb[0] = faces[f].nb[e];
            nf.nb[1] = -1;
            nf.nb[2] = -1;
            for (int k = 0; k < H; k++) {
                const int fk = hz_f[k], ek = hz_e[k];
                const int ak = faces[fk].v[ek], bk = faces[fk].v[(ek + 1) % 3];
                if (ak == b) nf.nb[1] = F + k;
                if (bk == a) nf.nb[2] = F + k;
            }
            if (nf.nb[1] < 0 || nf.nb[2] < 0) bad = 1;   // not a closed horizon
            nf.alive = 1;
            nf.pad = 0;
            faces[F + h] = nf;
            face_plane(x, y, z, nf, &planes[F + h]);
            far[F + h] = 0;
            vis[F + h] = -1;
        }
        __syncthreads();
        if (bad) {     // leave the hull as it was; the caller reports the failure
            if (tid == 0) C->overflow = 2;
            break;
        }
        // the outside faces now border the new ones; the seen faces go
        for (int h = tid; h < H; h += blockDim.x) {
            const int f = hz_f[h], e = hz_e[h];
            const int g = faces[f].nb[e];
            const int a = faces[f].v[e], b = faces[f].v[(e + 1) % 3];
            for (int e2 = 0; e2 < 3; e2++)
                if (faces[g].v[e2] == b && faces[g].v[(e2 + 1) % 3] == a) faces[g].nb[e2] = F + h;
        }
        __syncthreads();
        for (int k = tid; k < NV; k += blockDim.x) {
            const int f = vlist[k];
            faces[f].alive = 0;
            repl[f] = make_int2(F, H);
        }
        if (tid == 0) C->nfaces = F + H;
        inserted++;
        __syncthreads();
    }
    if (tid == 0) {
        C->born_lo = nf0;
        C->inserted = inserted;
    }
}

// Extreme points: for every alive face and each of its vertices, walk the
// faces around the vertex; the face of lowest index reports the vertex when
// those faces span at least three distinct planes.
__global__ __launch_bounds__(256) void k3_corners(const Hull3Ctl *__restrict__ Cc, const Face3 *__restrict__ faces,
                                                  const Plane3 *__restrict__ planes,
                                                  uint64_t *__restrict__ out, int *__restrict__ nout) {
    const int F = Cc->nfaces;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < 3 * (int64_t)F;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int f0 = (int)(t / 3), e0 = (int)(t % 3);
        if (!faces[f0].alive) continue;
        const int v = faces[f0].v[e0];
        double n[3][3];
        int np = 0;
        bool owner = true;
        int f = f0, e = e0;
        for (int step = 0; step < 1 << 16; step++) {
            if (f < f0) { owner = false; break; }
            const Plane3 &P = planes[f];
            bool same = false;
            for (int k = 0; k < np && !same; k++) {
                const __int128 cx = (__int128)(int64_t)n[k][1] * (int64_t)P.nz - (__int128)(int64_t)n[k][2] * (int64_t)P.ny;
                const __int128 cy = (__int128)(int64_t)n[k][2] * (int64_t)P.nx - (__int128)(int64_t)n[k][0] * (int64_t)P.nz;
                const __int128 cz = (__int128)(int64_t)n[k][0] * (int64_t)P.ny - (__int128)(int64_t)n[k][1] * (int64_t)P.nx;
                same = cx == 0 && cy == 0 && cz == 0;
            }
            if (!same && np < 3) { n[np][0] = P.nx; n[np][1] = P.ny; n[np][2] = P.nz; np++; }
            // next face around v: across the edge that ends at v
            const int g = faces[f].nb[(e + 2) % 3];
            int eg = -1;
            for (int k = 0; k < 3; k++)
                if (faces[g].v[k] == v) eg = k;
            f = g;
            e = eg;
            if (f == f0 || eg < 0) break;
        }
        if (owner && np >= 3) {
            const int o = atomicAdd(nout, 1);
            out[o] = (uint64_t)(uint32_t)v;
        }
    }
}

// Keys of a flat set for the 2D hull stage: the two coordinates kept after
// dropping the one of the plane normal's largest component.
__global__ __launch_bounds__(256) void k3_flat_keys(const float *__restrict__ x, const float *__restrict__ y,
                                                    const float *__restrict__ z, const uint32_t *__restrict__ cand,
                                                    int64_t nc, const Hull3Ctl *__restrict__ C,
                                                    uint64_t *__restrict__ keys) {
    const int64_t ax = C->nrm[0] < 0 ? -C->nrm[0] : C->nrm[0], ay = C->nrm[1] < 0 ? -C->nrm[1] : C->nrm[1],
                  az = C->nrm[2] < 0 ? -C->nrm[2] : C->nrm[2];
    const int drop = (ay > ax && ay >= az) ? 1 : (az > ax && az > ay) ? 2 : 0;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < nc; t += int64_t(gridDim.x) * blockDim.x) {
        const uint32_t i = cand[t];
        const uint64_t c[3] = {(uint64_t)(x[i] * GRIDF), (uint64_t)(y[i] * GRIDF), (uint64_t)(z[i] * GRIDF)};
        const uint64_t a = c[drop == 0 ? 1 : 0], b = c[drop == 2 ? 1 : 2];
        keys[t] = (a << 24) | b;
    }
}

// Small outputs of the degenerate cases and the final copy.
__global__ void k3_small_out(const Hull3Ctl *__restrict__ C, uint32_t *__restrict__ hull, int64_t *__restrict__ h) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (C->state == 4) { *h = 0; return; }
    if (C->state == 3) { hull[0] = C->p[0]; *h = 1; return; }
    // collinear: the two ends, ascending
    const uint32_t a = (uint32_t)C->lo_idx, b = (uint32_t)C->hi_idx;
    hull[0] = min(a, b);
    hull[1] = max(a, b);
    *h = 2;
}

__global__ void k3_copy_sorted(const uint64_t *__restrict__ keys, const int64_t *__restrict__ n,
                               uint32_t *__restrict__ hull, int64_t *__restrict__ h) {
    const int64_t m = *n;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += int64_t(gridDim.x) * blockDim.x)
        hull[i] = (uint32_t)keys[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) *h = m;
}

__global__ void k3_count_i64(const int *__restrict__ n, int64_t *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = *n;
}

__global__ __launch_bounds__(256) void k3_iota(uint32_t *__restrict__ p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k3_u64_of(const uint32_t *__restrict__ v, const int64_t *__restrict__ n,
                                                 uint64_t *__restrict__ out) {
    const int64_t m = *n;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += int64_t(gridDim.x) * blockDim.x)
        out[i] = v[i];
}

__global__ void k3_ctl_init(Hull3Ctl *__restrict__ C, int fcap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    Hull3Ctl c = {};
    c.fcap = fcap;
    *C = c;
}

__global__ __launch_bounds__(256) void k3_fill_i32(int *__restrict__ p, int64_t n, int v) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

}  // namespace hg
