// Filter passes: tile map, Step 1 (directional extremes, one fused pass),
// Step 2 (filter polygon + quick-accept rows), Step 3 (strict-inside test with
// survivor masks), survivor scatter, and the shared scan kernels.
//
// Work decomposition.  Set s covers points [o_s, o_{s+1}).  Its tiles start
// at A_s = o_s rounded down to the nearest position whose address is 16-byte
// aligned (so every float4 load is aligned) and cover TILE = 1024 point
// slots each; slots outside
// [o_s, o_{s+1}) are masked.  The persistent filter kernels give wave w the
// contiguous tile range [w q, (w+1) q), q = ceil(T / W), so a wave walks
// ascending point indices and meets each set as one contiguous "run".
#include <type_traits>

#include "hg_device.h"

namespace hg {

// First tile position of a set starting at o: o rounded down so that the
// point's address is 16-byte aligned, given the block position (phase) of
// x[0].  May be up to 3 below 0; those positions lie in x[0]'s own block.
__device__ __forceinline__ int64_t tile_base(int64_t o, int phase) {
    return o - ((o + phase) & 3);
}

// ---------------------------------------------------------------------------
// Tile map: tile_off[s] = first tile of set s (exclusive scan of tile
// counts), tile_off[S] = T.  One block of 1024 threads.
__global__ __launch_bounds__(1024) void k_tile_offsets(const int64_t *__restrict__ off,
                                                       int64_t n1, int64_t S, int64_t unit,
                                                       int phase, int64_t *__restrict__ tile_off,
                                                       uint32_t *__restrict__ zero) {
    __shared__ int64_t sh[17];
    if (zero)     // per-set tickets of the polygon kernel
        for (int64_t s = threadIdx.x; s < S; s += blockDim.x) zero[s] = 0;
    int64_t carry = 0;
    for (int64_t base = 0; base < S; base += blockDim.x) {
        int64_t s = base + threadIdx.x;
        int64_t cnt = 0;
        if (s < S) {
            int64_t b = set_begin(off, s), e = set_end(off, n1, s);
            if (e > b) {
                int64_t a = phase >= 0 ? tile_base(b, phase) : b;
                cnt = (e - a + unit - 1) / unit;
            }
        }
        int64_t tot;
        int64_t ex = block_excl_scan_i64(cnt, sh, &tot);
        if (s < S) tile_off[s] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) tile_off[S] = carry;
}

// tile_set[t] = s for every tile of set s: grid-stride over the tiles, the
// set found by binary search in tile_off (last s with tile_off[s] <= t).
__global__ __launch_bounds__(256) void k_tile_sets(const int64_t *__restrict__ tile_off, int64_t S,
                                                   int32_t *__restrict__ tile_set) {
    const int64_t T = tile_off[S];
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < T;
         t += int64_t(gridDim.x) * blockDim.x) {
        int64_t lo = 0, hi = S - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (tile_off[mid] <= t) lo = mid; else hi = mid - 1;
        }
        tile_set[t] = (int32_t)lo;
    }
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of uint32 counts into int64 offsets, with the
// element count read from device memory (*cnt_ptr).  out has count+1 entries;
// out[count] = total.  Two launches with a fixed grid of SCAN_BLOCKS.
constexpr int SCAN_BLOCKS = 256;
constexpr int SCAN_THREADS = 1024;

__device__ __forceinline__ void scan_segment(int64_t count, int64_t b, int64_t *lo, int64_t *hi) {
    int64_t seg = (count + SCAN_BLOCKS - 1) / SCAN_BLOCKS;
    seg = (seg + SCAN_THREADS - 1) / SCAN_THREADS * SCAN_THREADS;
    *lo = b * seg;
    *hi = min(count, *lo + seg);
}

// Blocks whose segment is not empty: 0 .. scan_busy(count) - 1.
__device__ __forceinline__ int scan_busy(int64_t count) {
    int64_t seg = (count + SCAN_BLOCKS - 1) / SCAN_BLOCKS;
    seg = (seg + SCAN_THREADS - 1) / SCAN_THREADS * SCAN_THREADS;
    return seg ? (int)((count + seg - 1) / seg) : 0;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const uint32_t *__restrict__ in,
                                                              const int64_t *__restrict__ cnt_ptr,
                                                              int64_t *__restrict__ block_sums,
                                                              int64_t *__restrict__ out,
                                                              uint32_t *__restrict__ ticket) {
    __shared__ int64_t sh[17];
    __shared__ bool last;
    int64_t count = *cnt_ptr, lo, hi;
    const int nbusy = scan_busy(count);
    if ((int)blockIdx.x >= nbusy) {    // empty segment: only the empty scan writes
        if (nbusy == 0 && blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
        return;
    }
    scan_segment(count, blockIdx.x, &lo, &hi);
    int64_t acc = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) acc += in[i];
    int64_t tot;
    block_excl_scan_i64(acc, sh, &tot);
    // the last block to finish (ticket, self-resetting) scans the block sums
    if (threadIdx.x == 0) {
        block_sums[blockIdx.x] = tot;
        __threadfence();
        last = atomicAdd(ticket, 1u) == (uint32_t)nbusy - 1;
        if (last) __threadfence();
    }
    __syncthreads();
    if (!last) return;
    int64_t v = (int)threadIdx.x < nbusy ? block_sums[threadIdx.x] : 0;
    int64_t ex = block_excl_scan_i64(v, sh, &tot);
    if (threadIdx.x < SCAN_BLOCKS) block_sums[threadIdx.x] = ex;
    if (threadIdx.x == 0) {
        out[count] = tot;
        *ticket = 0;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_down(const uint32_t *__restrict__ in,
                                                            const int64_t *__restrict__ cnt_ptr,
                                                            const int64_t *__restrict__ block_sums,
                                                            int64_t *__restrict__ out) {
    __shared__ int64_t sh[17];
    int64_t count = *cnt_ptr, lo, hi;
    scan_segment(count, blockIdx.x, &lo, &hi);
    int64_t carry = block_sums[blockIdx.x];
    for (int64_t base = lo; base < hi; base += blockDim.x) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < hi ? in[i] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan_i64(v, sh, &tot);
        if (i < hi) out[i] = carry + ex;
        carry += tot;
    }
}

// ---------------------------------------------------------------------------
// Point loads: float4 of x and y for 4 consecutive points starting at the
// 4-aligned global index a; slots at or beyond n_total read as 0.
__device__ __forceinline__ void load4(const float *__restrict__ x, const float *__restrict__ y,
                                      int64_t a, int64_t n_total, float xv[4], float yv[4]) {
    if (a + 4 <= n_total) {
        // streaming reads: marked non-temporal so they do not displace
        // reusable lines from the caches
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 fx = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(x + a));
        const f4 fy = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(y + a));
        xv[0] = fx.x; xv[1] = fx.y; xv[2] = fx.z; xv[3] = fx.w;
        yv[0] = fy.x; yv[1] = fy.y; yv[2] = fy.z; yv[3] = fy.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            bool in = a + j < n_total;
            xv[j] = in ? x[a + j] : 0.0f;
            yv[j] = in ? y[a + j] : 0.0f;
        }
    }
}

// The same for positions known to lie in [0, n_total): no guard.
__device__ __forceinline__ void load4_full(const float *__restrict__ x, const float *__restrict__ y,
                                           int64_t a, float xv[4], float yv[4]) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 fx = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(x + a));
    const f4 fy = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(y + a));
    xv[0] = fx.x; xv[1] = fx.y; xv[2] = fx.z; xv[3] = fx.w;
    yv[0] = fy.x; yv[1] = fy.y; yv[2] = fy.z; yv[3] = fy.w;
}

// ---------------------------------------------------------------------------
// Step 1 keys.  Fixed slot 4g+0 / 4g+1 is the argmin / argmax of
// u_g = cos_g x - sin_g y and 4g+2 / 4g+3 that of v_g = sin_g x + cos_g y,
// each product rounded to binary64 and then the sum (no contraction).
//
// PRESET 0 (0/30/45/60 degrees) and PRESET 1 (0/30/75/120) compare 2 u_g and
// 2 v_g for the 30- and 60-degree groups: there sin30 = cos60 = 1/2 and
// sin60 = cos30, so 2 u_30 = fl(fl(2 cos30 x) - y) and so on, which is
// exactly twice the rounded u_30 (scaling by 2 commutes with rounding here)
// and orders the points identically with two fewer products.  Only the
// comparisons see these keys; the reported values are recomputed from the
// winning points.  Under PRESET 1 u_120 = -v_30 and v_120 = u_30 bit for bit,
// so slots 12..15 are copies of 7, 6, 4, 5 made when the polygon is built.
//
// PRESET 1 + G (G = 1..6) has G groups at 90 j / G degrees.  Since
// sin(90 j / G) = cos(90 (G - j) / G), the groups j and G - j use the same
// two products c x and c y, so the pass needs 2 (G - 1) products and as
// many sums; group 0 is x and y themselves.
constexpr double C30 = 0x1.bb67ae8584caap-1;
constexpr double C30X2 = 0x1.bb67ae8584caap+0;   // 2 cos30, exact
constexpr double C45 = 0x1.6a09e667f3bcdp-1;
constexpr double C75 = 0x1.0907dc1930690p-2;
constexpr double S75 = 0x1.ee8dd4748bf15p-1;

// EVEN_COS[G][j] = cos(90 j / G degrees), correctly rounded, j = 0..G
// (the last entry of each row, cos 90, is exactly 0).
constexpr double EVEN_COS[MAX_GROUPS + 1][MAX_GROUPS + 1] = {
    {1.0, 0, 0, 0, 0, 0, 0},
    {1.0, 0.0, 0, 0, 0, 0, 0},
    {1.0, 0x1.6a09e667f3bcdp-1, 0.0, 0, 0, 0, 0},
    {1.0, 0x1.bb67ae8584caap-1, 0x1p-1, 0.0, 0, 0, 0},
    {1.0, 0x1.d906bcf328d46p-1, 0x1.6a09e667f3bcdp-1, 0x1.87de2a6aea963p-2, 0.0, 0, 0},
    {1.0, 0x1.e6f0e134454ffp-1, 0x1.9e3779b97f4a8p-1, 0x1.2cf2304755a5ep-1,
     0x1.3c6ef372fe950p-2, 0.0, 0},
    {1.0, 0x1.ee8dd4748bf15p-1, 0x1.bb67ae8584caap-1, 0x1.6a09e667f3bcdp-1, 0x1p-1,
     0x1.0907dc1930690p-2, 0.0}};

template <int PRESET>
struct Proj {
    static constexpr int NG = preset_eval_groups(PRESET);   // groups actually evaluated
    __device__ __forceinline__ static void uv(const Dirs &d, double xd, double yd,
                                              double u[MAX_GROUPS], double v[MAX_GROUPS]) {
#pragma clang fp contract(off)
        (void)d;
        if constexpr (PRESET == 0) {
            const double p = C30X2 * xd, q = C30X2 * yd, r = C45 * xd, t = C45 * yd;
            u[0] = xd;
            v[0] = yd;
            u[1] = p - yd;       // 2 u_30
            v[1] = xd + q;       // 2 v_30
            u[2] = r - t;
            v[2] = r + t;
            u[3] = xd - q;       // 2 u_60
            v[3] = p + yd;       // 2 v_60
        } else if constexpr (PRESET == 1) {
            const double p = C30X2 * xd, q = C30X2 * yd;
            u[0] = xd;
            v[0] = yd;
            u[1] = p - yd;
            v[1] = xd + q;
            u[2] = C75 * xd - S75 * yd;
            v[2] = S75 * xd + C75 * yd;
        } else {
            constexpr int G = PRESET - 1;
            u[0] = xd;
            v[0] = yd;
#pragma unroll
            for (int j = 1; j < G; j++) {
                // the same constants give the same rounded products, which
                // the compiler computes once for groups j and G - j
                const double c = EVEN_COS[G][j], s = EVEN_COS[G][G - j];
                u[j] = c * xd - s * yd;
                v[j] = s * xd + c * yd;
            }
        }
    }
};

// Directional projection for a learned direction: c*x + s*y.
__device__ __forceinline__ double proj_dir(double c, double s, double xd, double yd) {
#pragma clang fp contract(off)
    return c * xd + s * yd;
}

// Fixed slots with even index are minima; all others (learned ones too) maxima.
__device__ __forceinline__ constexpr bool slot_is_min(int k, int nfixed) {
    return k < nfixed && (k & 1) == 0;
}

// Key of tracked slot k (fixed slots first, then the learned directions).
template <int PRESET, int NDIR>
__device__ __forceinline__ void slot_keys(const Dirs &d, const double *dc, const double *ds,
                                          double xd, double yd, double *key) {
    constexpr int NF = 4 * Proj<PRESET>::NG;
    double u[MAX_GROUPS], v[MAX_GROUPS];
    Proj<PRESET>::uv(d, xd, yd, u, v);
#pragma unroll
    for (int k = 0; k < NF; k++) key[k] = (k & 2) ? v[k >> 2] : u[k >> 2];
#pragma unroll
    for (int e = 0; e < NDIR; e++) key[NF + e] = proj_dir(dc[e], ds[e], xd, yd);
}

// Cross-lane moves within rows of 16 lanes (DPP) and whole-wave extremes.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = dpp_u32<CTRL>((uint32_t)b), hi = dpp_u32<CTRL>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)((hi << 32) | lo));
}
template <bool MN>
__device__ __forceinline__ double pick(double a, double b) { return MN ? fmin(a, b) : fmax(a, b); }

// Minimum (MN) or maximum of v over the 64 lanes, in every lane.  Steps:
// swap neighbours, swap pairs, mirror half rows, mirror rows (each lane then
// holds its row's extreme), then combine the four rows.
template <bool MN>
__device__ __forceinline__ double wave_extreme(double v) {
    v = pick<MN>(v, dpp_f64<0xB1>(v));
    v = pick<MN>(v, dpp_f64<0x4E>(v));
    v = pick<MN>(v, dpp_f64<0x141>(v));
    v = pick<MN>(v, dpp_f64<0x140>(v));
    return pick<MN>(pick<MN>(readlane_f64(v, 0), readlane_f64(v, 16)),
                    pick<MN>(readlane_f64(v, 32), readlane_f64(v, 48)));
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    v = min(v, dpp_u32<0xB1>(v));
    v = min(v, dpp_u32<0x4E>(v));
    v = min(v, dpp_u32<0x141>(v));
    v = min(v, dpp_u32<0x140>(v));
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
    const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return min(min(a, b), min(c, e));
}

// Step 1: directional extremes of every slot over the wave's tiles, with the
// lowest index on ties; one partial per (wave, set) run, stored at the run's
// first tile.  Learned directions (NDIR > 0) come per set from
// set_dirs[s][d] = (c, s).
//
// Per lane and slot the kernel keeps the best key seen so far (lb) and the
// tile of the run in which the lane first reached it (rt); a tile costs one
// min/max per point and slot plus one compare per slot.  At the end of a run
// the wave takes the extreme m of lb and, for the lanes holding m, reloads
// their 16 points of tile rt to find the lowest index whose key is m.  In
// tiles that straddle a set boundary, positions outside the set hold a copy of
// the set's first point o0: a copy never beats a genuine extreme, and if the
// run's extreme is only met by copies, the run reports (key(o0), o0), a
// genuine pair of the set.
template <int PRESET, int NDIR, int BS = 256>
__global__ __launch_bounds__(BS) void k_extremes(
    const float *__restrict__ x, const float *__restrict__ y, int64_t n_total, int phase,
    const int64_t *__restrict__ off, int64_t n1, int64_t S,
    const int64_t *__restrict__ tile_off, const int32_t *__restrict__ tile_set, Dirs dirs,
    const double *__restrict__ set_dirs, double *__restrict__ pval, uint32_t *__restrict__ pidx) {
    constexpr int NF = 4 * Proj<PRESET>::NG;   // fixed slots evaluated
    constexpr int NS = NF + NDIR;               // slots tracked
    const int lane = lane_id();
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t W = (int64_t(gridDim.x) * blockDim.x) >> 6;
    const int64_t T = tile_off[S];
    const int64_t q = (T + W - 1) / W;
    const int64_t t0 = wave * q, t1 = min(t0 + q, T);
    if (t0 >= t1) return;

    double dc[NDIR > 0 ? NDIR : 1], ds[NDIR > 0 ? NDIR : 1];
    double lb[NS];
    uint32_t rt[NS];
    int64_t run = t0, o0 = 0, o1 = 0, tile0 = 0, abase = 0, cur_end = -1;
    float x0f = 0.0f, y0f = 0.0f;

    auto reset = [&]() {
#pragma unroll
        for (int k = 0; k < NS; k++) {
            lb[k] = slot_is_min(k, NF) ? INFINITY : -INFINITY;
            rt[k] = NONE;
        }
    };
    // Resolve the run's extremes and store its partial.
    auto flush = [&]() {
#pragma unroll
        for (int k = 0; k < NS; k++) {
            const bool mn = slot_is_min(k, NF);
            const double m = mn ? wave_extreme<true>(lb[k]) : wave_extreme<false>(lb[k]);
            uint64_t cand = __ballot(rt[k] != NONE && lb[k] == m);
            uint32_t found = NONE;
            // lane l examines point (chunk l/16, element l%4) of candidate (l/4)%4
            const int cq = (lane >> 2) & 3;
            while (cand) {     // up to four candidate lanes per round
                int cl[4];
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    cl[e] = cand ? __ffsll((unsigned long long)cand) - 1 : -1;
                    if (cand) cand &= cand - 1;
                }
                const int L = cq == 0 ? cl[0] : cq == 1 ? cl[1] : cq == 2 ? cl[2] : cl[3];
                // tile of candidate L (whole wave active for the permute)
                const uint32_t rl = (uint32_t)__builtin_amdgcn_ds_bpermute((L < 0 ? 0 : L) << 2, (int)rt[k]);
                uint32_t my = NONE;
                if (L >= 0) {
                    const int64_t tb = abase + (run + (int64_t)rl - tile0) * TILE;
                    const int64_t p = tb + (lane >> 4) * CHUNK + 4 * L + (lane & 3);
                    if (p >= o0 && p < o1) {
                        double key[NS];
                        slot_keys<PRESET, NDIR>(dirs, dc, ds, (double)x[p], (double)y[p], key);
                        if (key[k] == m) my = (uint32_t)p;
                    }
                }
                found = min(found, wave_min_u32(my));
            }
            if (found == NONE) found = (uint32_t)o0;
            if (lane == 0) {
                pval[run * MAX_SLOTS + k] = m;
                pidx[run * MAX_SLOTS + k] = found;
            }
        }
    };

    for (int64_t t = t0; t < t1; ++t) {
        if (t >= cur_end) {     // a new set starts (looked up once per set)
            if (cur_end >= 0) flush();
            const int64_t s = tile_set[t];
            cur_end = tile_off[s + 1];
            run = t;
            o0 = set_begin(off, s);
            o1 = set_end(off, n1, s);
            tile0 = tile_off[s];
            abase = tile_base(o0, phase);
            x0f = x[o0];
            y0f = y[o0];
#pragma unroll
            for (int e = 0; e < NDIR; e++) {
                dc[e] = set_dirs[(s * MAX_DIRS + e) * 2 + 0];
                ds[e] = set_dirs[(s * MAX_DIRS + e) * 2 + 1];
            }
            reset();
        }
        const int64_t tb = abase + (t - tile0) * TILE;
        double acc[NS];
        // FULL: every position of the tile lies in the set (loads unguarded)
        auto accumulate = [&](auto full_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
            // issue the whole tile's loads first: 8 KB in flight per wave
            float xv[TILE_CHUNKS][4], yv[TILE_CHUNKS][4];
#pragma unroll
            for (int c = 0; c < TILE_CHUNKS; c++) {
                if (FULL) load4_full(x, y, tb + c * CHUNK + 4 * lane, xv[c], yv[c]);
                else load4(x, y, tb + c * CHUNK + 4 * lane, n_total, xv[c], yv[c]);
            }
#pragma unroll
            for (int c = 0; c < TILE_CHUNKS; c++) {
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    float xf = xv[c][j], yf = yv[c][j];
                    if (!FULL) {
                        const int64_t p = tb + c * CHUNK + 4 * lane + j;
                        const bool valid = p >= o0 && p < o1;
                        xf = valid ? xf : x0f;
                        yf = valid ? yf : y0f;
                    }
                    double key[NS];
                    slot_keys<PRESET, NDIR>(dirs, dc, ds, (double)xf, (double)yf, key);
#pragma unroll
                    for (int k = 0; k < NS; k++)
                        acc[k] = (c == 0 && j == 0) ? key[k]
                                 : slot_is_min(k, NF) ? fmin(acc[k], key[k]) : fmax(acc[k], key[k]);
                }
            }
        };
        if (tb >= o0 && tb + TILE <= o1)
            accumulate(std::integral_constant<bool, true>());
        else
            accumulate(std::integral_constant<bool, false>());
        const uint32_t rel = (uint32_t)(t - run);
#pragma unroll
        for (int k = 0; k < NS; k++) {
            const bool upd = slot_is_min(k, NF) ? acc[k] < lb[k] : acc[k] > lb[k];
            lb[k] = upd ? acc[k] : lb[k];
            rt[k] = upd ? rel : rt[k];
        }
    }
    flush();
}
// ---------------------------------------------------------------------------
// Step 2: one block per set.  Reduce the runs' partials (or take the
// caller's slots), build the convex polygon of the slot points with Andrew's
// monotone chain (collinear points dropped, repeated coordinates by lowest
// index), and derive the edge functions and quick-accept rows.

struct SlotBest {
    double v;
    uint32_t i;
};

// (v, i) beats (bv, bi) for a minimum (mn) or maximum slot; lower index on ties
__device__ __forceinline__ bool better(bool mn, double v, uint32_t i, double bv, uint32_t bi) {
    return (mn ? v < bv : v > bv) || (v == bv && i < bi);
}

__device__ __forceinline__ double grid_of(float f) { return (double)f * GRIDD; }

// Exact edge function of (ex, ey, c) at grid point (px, py).
__device__ __forceinline__ double edge_eval(double ex, double ey, double c, double px, double py) {
    return fma(ex, py, fma(-ey, px, c));
}

constexpr int POLY_THREADS = 512;
constexpr int POLY_SPLIT = 16;     // blocks per set sharing the extremes pass's partials

template <int PRESET, int NDIR>
__global__ __launch_bounds__(POLY_THREADS) void k_polygon(
    const float *__restrict__ x, const float *__restrict__ y, int64_t n_total, int64_t S,
    const int64_t *__restrict__ tile_off, int64_t W1, const double *__restrict__ pval,
    const uint32_t *__restrict__ pidx, const uint32_t *__restrict__ slots_in, int n_in, Dirs dirs,
    const double *__restrict__ set_dirs, uint32_t *__restrict__ slots_out,
    double *__restrict__ vals_out, Poly *__restrict__ polys, Span *__restrict__ spans,
    uint32_t *__restrict__ redges, REdge *__restrict__ rtab, unsigned long long *__restrict__ rfar,
    SlotBest *__restrict__ bpart, uint32_t *__restrict__ ticket) {
    // NEV: fixed slots the extremes pass evaluated (12 for preset 1, whose
    // 120-degree group is a copy of the 30-degree one); NFIX: fixed slot
    // positions (at least 16; learned slots follow, NDIR of them).
    // Grid (S, POLY_SPLIT): block (s, y) reduces its share of set s's
    // partials; the last of the set's blocks to finish (per-set ticket,
    // zeroed by k_tile_offsets, reset here) combines the shares in bpart and
    // builds the polygon.  With slots_in the grid is (S, 1).
    constexpr int NEV = 4 * Proj<PRESET>::NG;
    constexpr int NFIX = preset_fixed_slots(PRESET);
    constexpr int NS = NFIX + NDIR;
    constexpr int NE = NEV + NDIR;
    static_assert(NS <= MAX_SLOTS, "learned slots need a fixed table of at most 16 slots");
    __shared__ SlotBest wbest[POLY_THREADS / WAVE][MAX_SLOTS];
    __shared__ SlotBest spart[POLY_SPLIT][MAX_SLOTS];  // the set's shares (last block)
    __shared__ uint32_t sl[MAX_SLOTS];
    __shared__ double gx[MAX_SLOTS], gy[MAX_SLOTS];   // slot points (grid units)
    __shared__ double sx[MAX_SLOTS], sy[MAX_SLOTS];   // sorted by (x, y, index, slot)
    __shared__ uint32_t si[MAX_SLOTS];
    __shared__ int st[2 * MAX_SLOTS + 2];
    __shared__ int lc[MAX_SLOTS], uc[MAX_SLOTS], hcount;   // lower / upper chain positions
    __shared__ double vx[MAX_SLOTS], vy[MAX_SLOTS];   // polygon vertices
    __shared__ int nvalid;
    __shared__ bool last;
    __shared__ Poly P;
    const int64_t s = blockIdx.x;
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;

    if (slots_in) {
        if (tid < MAX_SLOTS) {
            uint32_t i = tid < n_in ? slots_in[s * n_in + tid] : NONE;
            sl[tid] = (int64_t)i < n_total ? i : NONE;    // out-of-range slots are ignored
        }
    } else {
        const int64_t T = tile_off[S];
        const int64_t q = (T + W1 - 1) / W1;
        const int64_t ta = tile_off[s], tb = tile_off[s + 1];
        int64_t nruns = 0, m0 = 0;
        if (tb > ta) {
            m0 = (ta / q + 1) * q;
            nruns = 1 + (m0 < tb ? (tb - 1 - m0) / q + 1 : 0);
        }
        // a wave reads LPR consecutive slots of RPW runs per load, so a load
        // covers whole partial records; lane (sub, k) keeps the best (value,
        // then lowest index) of slot k over the runs it reads
        constexpr int LPR = NE <= 16 ? 16 : 32;
        constexpr int RPW = WAVE / LPR;
        const int k = lane & (LPR - 1), sub = lane / LPR;
        const bool mn = k < NE && slot_is_min(k, NEV);
        double bv = mn ? INFINITY : -INFINITY;
        uint32_t bi = NONE;
        const int64_t nw = (int64_t)gridDim.y * (blockDim.x >> 6);      // waves sharing the set
        const int64_t wg = (int64_t)blockIdx.y * (blockDim.x >> 6) + w;
        for (int64_t r0 = wg * RPW; r0 < nruns; r0 += 2 * nw * RPW) {  // two records in flight
            const int64_t ra = r0 + sub, rb = r0 + nw * RPW + sub;
            const bool ina = k < NE && ra < nruns, inb = k < NE && rb < nruns;
            const int64_t qa = ra == 0 ? ta : m0 + (ra - 1) * q;
            const int64_t qb = rb == 0 ? ta : m0 + (rb - 1) * q;
            const double va = ina ? pval[qa * MAX_SLOTS + k] : 0.0;
            const uint32_t ia = ina ? pidx[qa * MAX_SLOTS + k] : NONE;
            const double vb = inb ? pval[qb * MAX_SLOTS + k] : 0.0;
            const uint32_t ib = inb ? pidx[qb * MAX_SLOTS + k] : NONE;
            if (ia != NONE && better(mn, va, ia, bv, bi)) {
                bv = va;
                bi = ia;
            }
            if (ib != NONE && better(mn, vb, ib, bv, bi)) {
                bv = vb;
                bi = ib;
            }
        }
        // combine the RPW lanes of each slot (whole wave active)
#pragma unroll
        for (int off = LPR; off < WAVE; off <<= 1) {
            const double ov = __shfl_xor(bv, off);
            const uint32_t oi = (uint32_t)__shfl_xor((int)bi, off);
            if (oi != NONE && (bi == NONE || better(mn, ov, oi, bv, bi))) {
                bv = ov;
                bi = oi;
            }
        }
        if (sub == 0 && k < NE) wbest[w][k] = SlotBest{bv, bi};
        __syncthreads();
        if (tid < NE) {
            const bool mn = slot_is_min(tid, NEV);
            double v = wbest[0][tid].v;
            uint32_t i = wbest[0][tid].i;
            for (int ww = 1; ww < (int)(blockDim.x >> 6); ww++) {
                SlotBest b = wbest[ww][tid];
                if (b.i != NONE && (i == NONE || better(mn, b.v, b.i, v, i))) {
                    v = b.v;
                    i = b.i;
                }
            }
            wbest[0][tid] = SlotBest{v, i};
        }
        if (gridDim.y > 1) {     // publish this block's share; the set's last block goes on
            // (the share is written by the first wave, whose fence publishes it)
            if (tid < NE) bpart[(s * gridDim.y + blockIdx.y) * MAX_SLOTS + tid] = wbest[0][tid];
            __syncthreads();
            if (tid == 0) {
                __threadfence();
                last = atomicAdd(&ticket[s], 1u) == gridDim.y - 1;
                if (last) {
                    __threadfence();
                    ticket[s] = 0;
                }
            }
            __syncthreads();
            if (!last) return;
            // every share in one step of loads, then reduced in LDS
            for (int j = tid; j < (int)gridDim.y * MAX_SLOTS; j += blockDim.x)
                spart[j / MAX_SLOTS][j % MAX_SLOTS] = bpart[(s * gridDim.y) * MAX_SLOTS + j];
            __syncthreads();
            if (tid < NE) {
                const bool mn = slot_is_min(tid, NEV);
                SlotBest b0 = spart[0][tid];
                for (int yy = 1; yy < (int)gridDim.y; yy++) {
                    const SlotBest b = spart[yy][tid];
                    if (b.i != NONE && (b0.i == NONE || better(mn, b.v, b.i, b0.v, b0.i))) b0 = b;
                }
                wbest[0][tid] = b0;
            }
            __syncthreads();
        }
        if (tid < NE) {
            // partial slot k < NEV holds fixed slot k; learned slots follow
            int dst = tid < NEV ? tid : NFIX + (tid - NEV);
            sl[dst] = wbest[0][tid].i;
        }
        // positions no slot fills (preset 1's fourth group is filled below)
        if (tid < MAX_SLOTS && (tid >= NS || (tid >= NEV && tid < NFIX))) sl[tid] = NONE;
        __syncthreads();
        if (PRESET == 1 && tid == 0) {   // 120-degree group repeats the 30-degree one
            sl[12] = sl[7];
            sl[13] = sl[6];
            sl[14] = sl[4];
            sl[15] = sl[5];
        }
    }
    __syncthreads();

    // slots and their values (recomputed from the winning index)
    if (slots_out && tid < NS && !slots_in) slots_out[s * NS + tid] = sl[tid];
    if (vals_out && tid < NS && !slots_in) {
        uint32_t i = sl[tid];
        double val = NAN;
        if (i != NONE) {
            double xd = x[i], yd = y[i];
            if (tid < NFIX) {
                int g = tid >> 2, t = tid & 3;
                double c = dirs.gc[g], sn = dirs.gs[g];
                val = t < 2 ? c * xd - sn * yd : sn * xd + c * yd;
            } else {
                int d = tid - NFIX;
                val = proj_dir(set_dirs[(s * MAX_DIRS + d) * 2], set_dirs[(s * MAX_DIRS + d) * 2 + 1],
                               xd, yd);
            }
        }
        vals_out[s * NS + tid] = val;
    }

    // sort the slot points by (x, y, index, slot) with a rank per thread
    if (tid < MAX_SLOTS) {
        uint32_t i = sl[tid];
        gx[tid] = i != NONE ? grid_of(x[i]) : 0.0;
        gy[tid] = i != NONE ? grid_of(y[i]) : 0.0;
    }
    if (w == 0) {
        uint64_t vm = __ballot(tid < MAX_SLOTS && sl[tid < MAX_SLOTS ? tid : 0] != NONE);
        if (tid == 0) nvalid = __popcll(vm);
    }
    __syncthreads();
    if (tid < MAX_SLOTS && sl[tid] != NONE) {
        double ax = gx[tid], ay = gy[tid];
        uint32_t ai = sl[tid];
        int rank = 0;
        for (int j = 0; j < MAX_SLOTS; j++) {
            uint32_t bj = sl[j];
            if (bj == NONE || j == tid) continue;
            double bx = gx[j], by = gy[j];
            bool less = bx < ax || (bx == ax && (by < ay || (by == ay && (bj < ai ||
                                                     (bj == ai && j < tid)))));
            rank += less;
        }
        sx[rank] = ax;
        sy[rank] = ay;
        si[rank] = ai;
    }
    __syncthreads();

    // Andrew's chains on the sorted slot points, by the first wave: repeated
    // coordinates dropped (the lowest index stays first), then the lower and
    // the upper chain pruned in parallel: a point on or beyond the segment of
    // its two neighbours is no strict vertex, and once a pass drops nothing
    // each list turns strictly one way at every point (at most MAX_SLOTS
    // passes: each earlier pass drops a point)
    if (w == 0) {
        const uint64_t lt = lanemask_lt();
        const int k = nvalid;
        bool keep = false;
        double ax = 0.0, ay = 0.0;
        uint32_t ai = 0;
        if (lane < k) {
            ax = sx[lane];
            ay = sy[lane];
            ai = si[lane];
            keep = lane == 0 || ax != sx[lane - 1] || ay != sy[lane - 1];
        }
        const uint64_t bk = __ballot(keep);
        const int u = __popcll(bk);
        wave_sync();
        if (keep) {
            const int p = __popcll(bk & lt);
            sx[p] = ax;
            sy[p] = ay;
            si[p] = ai;
            lc[p] = p;
            uc[p] = p;
        }
        wave_sync();
        int nl = u, nu = u;
        for (int pass = 0; pass < MAX_SLOTS; pass++) {
            bool kl = lane < nl, ku = lane < nu;
            const int ml = kl ? lc[lane] : 0, mu = ku ? uc[lane] : 0;
            if (lane > 0 && lane + 1 < nl) {
                const int pa = lc[lane - 1], pc = lc[lane + 1];
                if (orient(sx[pa], sy[pa], sx[ml], sy[ml], sx[pc], sy[pc]) <= 0) kl = false;
            }
            if (lane > 0 && lane + 1 < nu) {
                const int pa = uc[lane - 1], pc = uc[lane + 1];
                if (orient(sx[pa], sy[pa], sx[mu], sy[mu], sx[pc], sy[pc]) >= 0) ku = false;
            }
            const uint64_t bl = __ballot(kl), bu = __ballot(ku);
            wave_sync();
            if (kl) lc[__popcll(bl & lt)] = ml;
            if (ku) uc[__popcll(bu & lt)] = mu;
            wave_sync();
            const int nl2 = __popcll(bl), nu2 = __popcll(bu);
            if (nl2 == nl && nu2 == nu) break;
            nl = nl2;
            nu = nu2;
        }
        // counter-clockwise from the lowest point: the lower chain, then the
        // upper chain's interior backwards
        const int h = u == 0 ? 0 : (u == 1 ? 1 : nl + nu - 2);
        if (lane < h) st[lane] = lane < nl ? lc[lane] : uc[nu - 2 - (lane - nl)];
        if (lane == 0) hcount = h;
    }
    __syncthreads();
    if (w == 0) {     // lane e: vertex e and the edge from it to vertex e + 1
        const int h = hcount;
        const int e = lane;
        const bool ev = e < h && h >= 3;
        int ya = 0;
        if (e < MAX_SLOTS) {
            double ax = 0.0, ay = 0.0;
            if (e < h) {
                ax = sx[st[e]];
                ay = sy[st[e]];
                vx[e] = ax;
                vy[e] = ay;
            }
            P.verts[e] = e < h ? si[st[e]] : NONE;
            P.vx[e] = e < h ? (int32_t)ax : 0;
            P.vy[e] = e < h ? (int32_t)ay : 0;
            if (ev) {
                const int bb = st[(e + 1) % h];
                const double ex = sx[bb] - ax, ey = sy[bb] - ay;
                P.ex[e] = ex;
                P.ey[e] = ey;
                P.c[e] = fma(ey, ax, -(ex * ay));
                ya = (int)ay;
            } else {
                P.ex[e] = 0.0;
                P.ey[e] = 0.0;
                P.c[e] = 1.0;
            }
        }
        // the vertices' y-range (grid units, below 2^24)
        const int ylo = (int)wave_min_u32(ev ? (uint32_t)ya : 0xFFFFFFFFu);
        const int yhi = 0x7FFFFFFF - (int)wave_min_u32(ev ? (uint32_t)(0x7FFFFFFF - ya) : 0xFFFFFFFFu);
        if (lane == 0) {
            P.m = h;
            if (h < 3) {
                P.c[0] = -1.0;    // nothing strictly inside
                P.yspan = -1;
                P.ky_lo = 0;
                P.shift = 0;
                P.ymin = 1;
                P.ymax = 0;
            } else {
                // the rows stop a thin sliver (1/1024 of the height) short of
                // the top and bottom vertices, where the polygon narrows to a
                // point or an edge and a row could hold no quick-accept span;
                // points in the slivers take the exact test
                const int d = (yhi - ylo) >> 10;
                P.ymin = ylo;
                P.ymax = yhi;
                P.ky_lo = ylo + d;
                P.yspan = (yhi - d) - (ylo + d);
                // rows for the set's size: 8 per tile of points, 16 to
                // SPAN_ROWS (a small set gains nothing from a fine table it
                // would spend longer building and loading than using; one row
                // per two tiles made the 4096-set batch's discard pass 10 %
                // slower for 40 us less building)
                const int64_t ts = tile_off[s + 1] - tile_off[s];
                int rows = 16;
                while (rows < SPAN_ROWS && rows < 8 * ts) rows <<= 1;
                int sh = 0;
                while ((P.yspan >> sh) >= rows) sh++;
                P.shift = sh;
            }
        }
    }
    __syncthreads();
    {   // the record, a word per thread
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&P);
        uint32_t *dst = reinterpret_cast<uint32_t *>(polys + s);
        static_assert(sizeof(Poly) % 4 == 0, "Poly is copied in words");
        for (int i = tid; i < (int)(sizeof(Poly) / 4); i += (int)blockDim.x) dst[i] = src[i];
    }
    if (rtab) {    // the refinement's round-0 edges (the polygon's) and cleared farthest keys
        const int m = P.m >= 3 ? P.m : 0;
        for (int e = tid; e < RE_CAP; e += blockDim.x) {
            REdge r = redge_empty();
            if (e < m) {
                const int b = (e + 1) % m;
                r = REdge{(int32_t)vx[e], (int32_t)vy[e], (int32_t)vx[b], (int32_t)vy[b]};
            }
            rtab[s * RE_CAP + e] = r;
            rfar[s * RE_CAP + e] = 0;
        }
    }
}

// Rows of each set's polygon (after k_polygon): quick-accept span from the
// edges at the row's ends, shrunk to integers and kept only if its four
// corners are strictly inside; the polygon's x-extent over the row (vertices
// in the row and the edges' crossings of its two boundary lines); the edges
// whose y-range meets it.  Block (s, b) does rows 16b .. 16b + 15 of set s,
// 16 lanes per row, lane l taking edges l and l + 16; the lanes' results meet
// by shuffles within the row's 16 lanes.
constexpr int ROWS_PER_BLOCK = 16;

__device__ __forceinline__ double row_min(double v) {
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double row_max(double v) {
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ uint32_t row_or(uint32_t v) {
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

// Grid (S, ny): block (s, b) builds the row groups b, b + ny, ... (16 rows
// each, 16 lanes per row) of set s up to the set's last row; ny shrinks as
// S grows, so that thousands of sets do not each pay a block's latency per
// group.
__global__ __launch_bounds__(256) void k_rows(const Poly *__restrict__ polys,
                                              Span *__restrict__ spans,
                                              uint32_t *__restrict__ redges) {
    static_assert(MAX_SLOTS <= 32, "two edges per lane");
    const int64_t s = blockIdx.x;
    const int tid = threadIdx.x, el = tid & 15;
    const Poly &P = polys[s];
    // rows past the set's last one are never read
    const int last = P.yspan >= 0 ? (P.yspan >> P.shift) : 0;
    const int m = P.m;
    // the lane's two edges, loaded once for all its rows; a crossing is
    // ax + (ex (y - ay)) / ey with the product exact and the quotient taken
    // as a product with 1 / ey (an ulp more than the division, well inside
    // the extent's grid unit of margin; the spans are verified exactly)
    bool ev[2];
    double gex[2], gey[2], gax[2], gay[2], ginv[2], gc[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const int e = el + 16 * h;
        ev[h] = e < m;
        gex[h] = ev[h] ? P.ex[e] : 0.0;
        gey[h] = ev[h] ? P.ey[e] : 0.0;
        gc[h] = ev[h] ? P.c[e] : 1.0;
        gax[h] = ev[h] ? (double)P.vx[e] : 0.0;
        gay[h] = ev[h] ? (double)P.vy[e] : 0.0;
        ginv[h] = gey[h] != 0 ? 1.0 / gey[h] : 0.0;
    }
    const int32_t ky_lo = P.ky_lo, yspan = P.yspan, shift = P.shift;
    for (int rg = blockIdx.y; rg * ROWS_PER_BLOCK <= last && rg < SPAN_ROWS / ROWS_PER_BLOCK;
         rg += gridDim.y) {
    const int r = rg * ROWS_PER_BLOCK + (tid >> 4);
    Span sp{SPAN_FAR, 0, SPAN_FAR, 0};     // no span; nothing strictly inside the extent
    uint32_t re = ROW_EDGES_ALL;
    const int64_t ytop = (int64_t)ky_lo + yspan;
    const int64_t y0 = (int64_t)ky_lo + ((int64_t)r << shift);
    // (uniform per row: all 16 lanes of a row take the same branches)
    if (yspan >= 0 && y0 <= ytop) {
        const int64_t y1 = min(y0 + (int64_t(1) << shift) - 1, ytop);
        const double fy0 = (double)y0, fy1 = (double)y1;
        double xl = -1e300, xr = 1e300, mnx = 1e300, mxx = -1e300;
        uint32_t bad = 0, meets = 0;
#pragma unroll
        for (int h = 0; h < 2; h++) {
            if (!ev[h]) continue;
            const int e = el + 16 * h;
            const double ex = gex[h], ey = gey[h], ax = gax[h], ay = gay[h];
            const double by = ay + ey;
            const double x0 = ax + (ex * (fy0 - ay)) * ginv[h], x1 = ax + (ex * (fy1 - ay)) * ginv[h];
            if (ey > 0) {
                xr = fmin(xr, fmin(x0, x1));
            } else if (ey < 0) {
                xl = fmax(xl, fmax(x0, x1));
            } else if (ex > 0) {
                if (fy0 <= ay) bad = 1;      // bottom edge
            } else if (ex < 0) {
                if (fy1 >= ay) bad = 1;      // top edge
            }
            if (ay >= fy0 && ay <= fy1) {
                mnx = fmin(mnx, ax);
                mxx = fmax(mxx, ax);
            }
            const double elo = fmin(ay, by), ehi = fmax(ay, by);
            if (ey != 0) {
                if (elo <= fy0 && fy0 <= ehi) {
                    mnx = fmin(mnx, x0);
                    mxx = fmax(mxx, x0);
                }
                if (elo <= fy1 && fy1 <= ehi) {
                    mnx = fmin(mnx, x1);
                    mxx = fmax(mxx, x1);
                }
            }
            if (elo <= fy1 && ehi >= fy0) meets |= 1u << e;
        }
        xl = row_max(xl);
        xr = row_min(xr);
        mnx = row_min(mnx);
        mxx = row_max(mxx);
        bad = row_or(bad);
        meets = row_or(meets);
        // the lowest four edges meeting the row, in order
        const int ne = __popc(meets);
        if (ne > 4) {
            re = ROW_EDGES_ALL;
        } else {
            re = 0;
            uint32_t mm = meets;
            for (int k = 0; k < 4; k++) {
                const uint32_t e = mm ? (uint32_t)__ffs(mm) - 1 : ROW_EDGE_NONE;
                re |= e << (8 * k);
                mm &= mm - 1;
            }
        }
        // the crossings carry at most a few ulps of rounding; one grid unit of
        // margin keeps the outer test conservative
        if (mnx <= mxx) {
            // strictly between ol = floor(mnx) - 1 and orr = ceil(mxx) + 1
            const int32_t ol = (int32_t)floor(mnx) - 1, orr = (int32_t)ceil(mxx) + 1;
            sp.ob = ol + 1;
            sp.ow = orr - ol - 2;      // >= 1: orr - ol >= 3
        } else {
            // unreachable: every point of the row in the extent, so that it
            // gets the exact test
            sp.ob = -SPAN_FAR;
            sp.ow = INT32_MIN;         // as uint32: 2^31
            re = ROW_EDGES_ALL;
        }
        if (!bad && xl > -1e299 && xr < 1e299) {
            double fl = floor(xl) + 1.0, fr = ceil(xr) - 1.0;
            for (int attempt = 0; attempt < 3 && fl <= fr; attempt++) {
                uint32_t fail = 0;
                const double cx[2] = {fl, fr}, cy[2] = {fy0, fy1};
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    if (!ev[h]) continue;
                    for (int a2 = 0; a2 < 2; a2++)
                        for (int b2 = 0; b2 < 2; b2++)
                            if (!(edge_eval(gex[h], gey[h], gc[h], cx[a2], cy[b2]) > 0)) fail = 1;
                }
                if (!row_or(fail)) {
                    sp.xl = (int32_t)fl;
                    sp.xw = (int32_t)(fr - fl);
                    break;
                }
                fl += 2.0;
                fr -= 2.0;
            }
        }
    }
    if (el == 0 && r < SPAN_ROWS) {
        spans[s * SPAN_ROWS + r] = sp;
        redges[s * SPAN_ROWS + r] = re;
    }
    }
}

// ---------------------------------------------------------------------------
// Step 3: strict-inside test.  Each point is first classified with its row
// of the polygon's y-range (wave-private LDS copy): quick accept (strictly
// inside), quick reject (outside the row's x-extent or the polygon's y-range:
// a survivor), or undecided.  Undecided points go to a per-wave queue and are
// tested exactly, in full 64-lane batches, against the edges that meet their
// row.  Output (MODE):
//  - DISCARD_MASKS: per tile, survivor mask words (word 4c + j, bit l = point
//    c*256 + 4l + j of the tile) and the survivor count, for the ordered
//    scatter;
//  - DISCARD_APPEND: the quick rejects join the queue too, flagged, and the
//    64-lane batches write every survivor (index, key) to the wave's own
//    region of the survivor list, [wave * q * TILE, ...) for q tiles per
//    wave, with no atomics; seg_cnt[wave] gets the region's count and
//    seg_meta[0] the region size q * TILE (the hull stage does not need
//    index order: it sorts by key, and maps keys back to the lowest index);
//  - DISCARD_ASSIGN: as APPEND, and each survivor also gets the first
//    polygon edge it is strictly outside of (RE_NONE: on the boundary), from
//    the same edge evaluations, with the farthest-point key of every edge
//    raised: the refinement's round-0 state.
constexpr int QCAP = 320;
constexpr int DISCARD_MASKS = 0, DISCARD_APPEND = 1, DISCARD_ASSIGN = 2;
constexpr int EDGE_SLOTS = 32;        // edge arrays in LDS; slots >= m hold (0, 0, 1)

struct DiscardLds {
    Span rows[SPAN_ROWS];
    uint32_t redge[SPAN_ROWS];
    double ex[EDGE_SLOTS], ey[EDGE_SLOTS], c[EDGE_SLOTS];
    uint64_t q[QCAP];                 // kx | ky << 24 | pos << 48
    unsigned long long mask[TILE_WORDS];
    unsigned long long far[MAX_SLOTS];  // DISCARD_ASSIGN: farthest-point keys of the set's edges
};

// Raise the global farthest-point keys of set s's edges from the wave's
// copies, and clear those.
__device__ __forceinline__ void far_flush(DiscardLds &L, unsigned long long *gfar, int64_t s) {
    const int lane = lane_id();
    wave_sync();
    if (lane < MAX_SLOTS) {
        const unsigned long long v = L.far[lane];
        if (v) far_update(&gfar[s * RE_CAP + lane], v);
        L.far[lane] = 0;
    }
    wave_sync();
}

// Where an appending discard pass writes its survivors (see k_discard).
struct AppendOut {
    uint32_t *surv;
    uint64_t *keys;
    uint16_t *edges;       // DISCARD_ASSIGN only
    int64_t at;            // next free entry of the wave's region (uniform)
    int64_t tb;            // global index of the tile's first point
    uint64_t setkey;       // set << 48
    int pm;                // polygon vertices
};

constexpr uint64_t Q_OUTSIDE = 1ull << 63;   // queue entry already known to be a survivor
// Appending modes keep queue entries across tiles: an entry's position is
// (tile - base tile) * TILE + position in the tile, below 2^15, so a queue
// spans at most Q_TILES tiles before it is drained whatever its length.
constexpr int Q_TILES = 32;

// Exact test of queue entries [from, from + count), one per lane, against the
// edges meeting the point's row (all edges outside the rows).  MASKS: a
// point not strictly inside sets its mask bit.  APPEND/ASSIGN: every
// survivor (tested, or queued as known) is written to o's region, with
// (ASSIGN) the first edge it is strictly outside of and that edge's
// farthest-point key raised.
template <int NEDGE, int MODE>
__device__ __forceinline__ void drain(DiscardLds &L, int from, int count, int32_t ky_lo, int shift,
                                      uint32_t ylim, AppendOut &o) {
    const int lane = lane_id();
    bool out = false;
    uint64_t e = 0;
    uint16_t e_out = RE_NONE;
    double dist = 0.0;
    if (lane < count) {
        e = L.q[from + lane];
        const int32_t kx = (int32_t)(e & 0xFFFFFF), ky = (int32_t)((e >> 24) & 0xFFFFFF);
        const double px = (double)kx, py = (double)ky;
        const uint32_t dy = (uint32_t)(ky - ky_lo);   // outside the rows: every edge
        const uint32_t re = dy <= ylim ? L.redge[dy >> shift] : ROW_EDGES_ALL;
        bool inside = true;
        if (re != ROW_EDGES_ALL) {
            // all four evaluated (no short circuit): unused entries name an
            // always-satisfied edge
#pragma unroll
            for (int q4 = 0; q4 < 4; q4++) {
                const int k = (re >> (8 * q4)) & 0xFF;
                const double E = edge_eval(L.ex[k], L.ey[k], L.c[k], px, py);
                inside = inside && E > 0;
                if (MODE == DISCARD_ASSIGN && E < 0 && e_out == RE_NONE) { e_out = (uint16_t)k; dist = -E; }
            }
        } else {
            // points outside the rows (rare): stop at the first edge that
            // decides (not strictly inside; with ASSIGN, strictly outside)
#pragma unroll 1
            for (int k = 0; k < NEDGE; k++) {
                const double E = edge_eval(L.ex[k], L.ey[k], L.c[k], px, py);
                inside = inside && E > 0;
                if (E < 0) {
                    if (MODE == DISCARD_ASSIGN) { e_out = (uint16_t)k; dist = -E; }
                    break;
                }
                if (MODE != DISCARD_ASSIGN && !inside) break;
            }
        }
        out = (e & Q_OUTSIDE) || !inside;
        if (MODE == DISCARD_ASSIGN && o.pm < 3) e_out = RE_NONE;   // no refinement edges
    }
    if constexpr (MODE == DISCARD_MASKS) {
        if (out) {
            const int pos = (int)((e >> 48) & 0x3FF);
            const int c = pos >> 8, l = (pos >> 2) & 63, j = pos & 3;
            atomicOr(&L.mask[c * 4 + j], 1ull << l);
        }
    } else {
        const uint64_t m = __ballot(out);
        if (out) {
            const int64_t gi = o.tb + (int64_t)((e >> 48) & 0x7FFF);
            const int64_t pp = o.at + __popcll(m & lanemask_lt());
            o.surv[pp] = (uint32_t)gi;
            o.keys[pp] = o.setkey | ((e & 0xFFFFFF) << 24) | ((e >> 24) & 0xFFFFFF);
            if constexpr (MODE == DISCARD_ASSIGN) {
                o.edges[pp] = e_out;
                if (e_out != RE_NONE) {
                    const uint64_t fk = far_key(dist, (uint32_t)gi);
                    if (L.far[e_out] < fk) atomicMax(&L.far[e_out], (unsigned long long)fk);
                }
            }
        }
        o.at += __popcll(m);
    }
}

// Sum over lanes 0..15 (other lanes' values are ignored), in every lane.
__device__ __forceinline__ uint32_t row0_sum_u32(uint32_t v) {
    v += dpp_u32<0xB1>(v);
    v += dpp_u32<0x4E>(v);
    v += dpp_u32<0x141>(v);
    v += dpp_u32<0x140>(v);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
}

template <int NEDGE, int MODE, int BS = 256>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_discard(
    const float *__restrict__ x, const float *__restrict__ y, int64_t n_total, int phase,
    const int64_t *__restrict__ off, int64_t n1, int64_t S, const int64_t *__restrict__ tile_off,
    const int32_t *__restrict__ tile_set, const Poly *__restrict__ polys,
    const Span *__restrict__ spans, const uint32_t *__restrict__ redges,
    uint64_t *__restrict__ masks, uint32_t *__restrict__ tile_cnt, uint32_t *__restrict__ surv,
    uint64_t *__restrict__ keys, uint16_t *__restrict__ edges, int64_t *__restrict__ seg_cnt,
    int64_t *__restrict__ seg_meta, unsigned long long *__restrict__ gfar, int64_t nreg,
    int *__restrict__ regctr) {
    __shared__ DiscardLds lds[BS / WAVE];
    DiscardLds &L = lds[threadIdx.x >> 6];
    const int lane = lane_id();
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t W = (int64_t(gridDim.x) * blockDim.x) >> 6;
    const int64_t T = tile_off[S];
    // Regions: q consecutive tiles each.  Without regctr region w is wave
    // w's; with it (appending modes, several sets) there are nreg regions and
    // each wave takes the next one from *regctr until none is left, so the
    // waves that meet cheap tiles take more (sets differ in cost per tile).
    // A region's survivors go to its own part of the list, [r q TILE, ...).
    const int64_t R = regctr ? nreg : W;
    const int64_t q = (T + R - 1) / R;
    if (MODE != DISCARD_MASKS && wave == 0 && lane == 0) seg_meta[0] = q * TILE;
    auto next_region = [&](int64_t cur) -> int64_t {
        if (!regctr) return cur < 0 ? wave : R;
        int v = 0;
        if (lane == 0) v = atomicAdd(regctr, 1);
        return (int64_t)__shfl(v, 0);
    };
    AppendOut ao{surv, keys, edges, 0, 0, 0, 0};

    int64_t o0 = 0, o1 = 0, tile0 = 0, abase = 0, cur_end = -1, cur_s = -1;
    int qn = 0;                 // queued points (wave-uniform)
    int64_t qt = 0;             // appending modes: tile the queue's positions count from
    int32_t ky_lo = 0, shift = 0, ymin = 0, pm = 0;
    uint32_t ylim = 0;          // in the rows: (ky - ky_lo) <= ylim (unsigned)
    uint32_t yext = 0;          // in the polygon's y-range: (ky - ymin) <= yext
    bool has_rows = false;

    for (int64_t r = next_region(-1); r < R; r = next_region(r)) {
    const int64_t t0 = r * q, t1 = min(t0 + q, T);
    if (t0 >= t1) {
        if (MODE != DISCARD_MASKS && lane == 0) seg_cnt[r] = 0;
        continue;
    }
    ao.at = t0 * TILE;
    for (int64_t t = t0; t < t1; ++t) {
        if (t >= cur_end) {     // a new set starts (looked up once per set)
            // the queue holds the previous set's points: test them against
            // its polygon first
            if (MODE != DISCARD_MASKS && qn > 0) {
                wave_sync();
                drain<NEDGE, MODE>(L, 0, qn, ky_lo, shift, ylim, ao);
                qn = 0;
                wave_sync();
            }
            const int64_t s = __builtin_amdgcn_readfirstlane(tile_set[t]);
            if (MODE == DISCARD_ASSIGN) {
                if (cur_s >= 0) far_flush(L, gfar, cur_s);
                else if (lane < MAX_SLOTS) L.far[lane] = 0;
            }
            cur_s = s;
            ao.setkey = (uint64_t)s << 48;
            cur_end = tile_off[s + 1];
            o0 = set_begin(off, s);
            o1 = set_end(off, n1, s);
            tile0 = tile_off[s];
            abase = tile_base(o0, phase);
            const Poly *P = polys + s;
            ky_lo = P->ky_lo;
            has_rows = P->yspan >= 0;
            ylim = (uint32_t)max(P->yspan, 0);
            shift = P->shift;
            pm = P->m;
            ao.pm = pm;
            ymin = P->ymin;
            yext = (uint32_t)(P->ymax - P->ymin);
            if (!has_rows) {     // nothing strictly inside: every point is outside
                ky_lo = INT32_MAX;
                ylim = 0;
                ymin = INT32_MAX;
                yext = 0;
            }
            wave_sync();
            // the set's rows (a point outside them never reads its row's entry)
            const int nrows = has_rows ? (int)(ylim >> shift) + 1 : 0;
            for (int r = lane; r < nrows; r += WAVE) {
                L.rows[r] = spans[s * SPAN_ROWS + r];
                L.redge[r] = redges[s * SPAN_ROWS + r];
            }
            if (lane < EDGE_SLOTS) {
                const bool used = lane < MAX_SLOTS;
                L.ex[lane] = used ? P->ex[lane] : 0.0;
                L.ey[lane] = used ? P->ey[lane] : 0.0;
                L.c[lane] = used ? P->c[lane] : 1.0;
            }
            wave_sync();
        }
        const int64_t tb = abase + (t - tile0) * TILE;
        if (MODE != DISCARD_MASKS) {
            // positions count from tile qt; past Q_TILES tiles the queue is
            // drained whatever its length
            if (qn > 0 && t - qt >= Q_TILES) {
                wave_sync();
                drain<NEDGE, MODE>(L, 0, qn, ky_lo, shift, ylim, ao);
                qn = 0;
                wave_sync();
            }
            if (qn == 0) qt = t;
        } else {
            qt = t;
        }
        ao.tb = abase + (qt - tile0) * TILE;
        const int tpos = (int)(t - qt) * TILE;   // position of the tile's first point in the queue
        // one tile (FULL: every position lies in the set, so the loads need
        // no guard): per chunk, classify its 4 points per lane, queue the
        // undecided ones (one ballot per chunk when there are none), drain
        // full batches
        auto tile = [&](auto full_tag) {
            constexpr bool FULL = decltype(full_tag)::value;
            float xv[TILE_CHUNKS][4], yv[TILE_CHUNKS][4];
#pragma unroll
            for (int c = 0; c < TILE_CHUNKS; c++) {
                if (FULL) load4_full(x, y, tb + c * CHUNK + 4 * lane, xv[c], yv[c]);
                else load4(x, y, tb + c * CHUNK + 4 * lane, n_total, xv[c], yv[c]);
            }
#pragma unroll
            for (int c = 0; c < TILE_CHUNKS; c++) {
                const int64_t a = tb + c * CHUNK + 4 * lane;
                int32_t kx[4], ky[4];
                uint32_t dy[4];
                Span sp[4];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    kx[j] = (int32_t)(xv[c][j] * GRIDF);
                    ky[j] = (int32_t)(yv[c][j] * GRIDF);
                    dy[j] = (uint32_t)(ky[j] - ky_lo);
                    sp[j] = L.rows[min(dy[j] >> shift, (uint32_t)(SPAN_ROWS - 1))];
                }
                // classification as wave masks (one bit per lane), combined
                // with scalar logic: outside = not in the polygon's y-range,
                // or in the rows and outside the row's extent; inside = in
                // the rows and in the row's quick-accept span
                uint64_t sw[4], slow[4];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const uint64_t m_valid = FULL ? __ballot(true)
                                                  : __ballot(a + j >= o0) & __ballot(a + j < o1);
                    const uint64_t m_rows = __ballot(dy[j] <= ylim);
                    const uint64_t m_ext = __ballot((uint32_t)(ky[j] - ymin) <= yext);
                    // one unsigned range comparison per ballot: xl <= kx <= xr
                    // (quick-accept span), ol < kx < orr (inside the row's
                    // extent); the rows store the ranges as (start, width)
                    const uint64_t m_span = __ballot((uint32_t)(kx[j] - sp[j].xl) <= (uint32_t)sp[j].xw);
                    const uint64_t m_in = __ballot((uint32_t)(kx[j] - sp[j].ob) <= (uint32_t)sp[j].ow);
                    const uint64_t outside = ~m_ext | (m_rows & ~m_in);
                    const uint64_t inside = m_rows & m_span;
                    sw[j] = outside & m_valid;
                    slow[j] = ~(outside | inside) & m_valid;
                }
                // queued: the undecided points, and in the appending modes the
                // survivors already known (flagged), so that the 64-lane
                // drain writes every survivor
                uint64_t push[4];
#pragma unroll
                for (int j = 0; j < 4; j++) push[j] = MODE == DISCARD_MASKS ? slow[j] : (slow[j] | sw[j]);
                // The queued lanes append in lane order at qn; a lane's own
                // bit of a wave mask is read back with inverse ballot (the
                // mask itself as the lane condition).
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    if (push[j]) {
                        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(push[j] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)push[j], 0u));
                        if (__builtin_amdgcn_inverse_ballot_w64(push[j]))
                            L.q[qn + (int)below] = (uint64_t)((uint32_t)kx[j] & 0xFFFFFFu) |
                                                   ((uint64_t)((uint32_t)ky[j] & 0xFFFFFFu) << 24) |
                                                   ((uint64_t)(tpos + c * CHUNK + 4 * lane + j) << 48) |
                                                   (__builtin_amdgcn_inverse_ballot_w64(sw[j]) ? Q_OUTSIDE : 0);
                        qn += __popcll(push[j]);
                    }
                }
                if (MODE == DISCARD_MASKS && lane < 4)
                    L.mask[c * 4 + lane] = lane == 0 ? sw[0] : lane == 1 ? sw[1] : lane == 2 ? sw[2] : sw[3];
                wave_sync();
                while (qn >= WAVE) {
                    qn -= WAVE;
                    drain<NEDGE, MODE>(L, qn, WAVE, ky_lo, shift, ylim, ao);
                }
                wave_sync();
            }
            if (MODE == DISCARD_MASKS && qn > 0) {
                drain<NEDGE, MODE>(L, 0, qn, ky_lo, shift, ylim, ao);
                qn = 0;
            }
            wave_sync();
        };
        if (tb >= o0 && tb + TILE <= o1)
            tile(std::integral_constant<bool, true>());
        else
            tile(std::integral_constant<bool, false>());
        if constexpr (MODE == DISCARD_MASKS) {
            const uint64_t mw = lane < TILE_WORDS ? L.mask[lane] : 0;
            const uint32_t cnt = row0_sum_u32((uint32_t)__popcll(mw));
            if (cnt > 0 && lane < TILE_WORDS) masks[t * TILE_WORDS + lane] = mw;
            if (lane == 0) tile_cnt[t] = cnt;
        }
        wave_sync();
    }
    // the region's queued points, then its count
    if (MODE != DISCARD_MASKS && qn > 0) {
        wave_sync();
        drain<NEDGE, MODE>(L, 0, qn, ky_lo, shift, ylim, ao);
        qn = 0;
        wave_sync();
    }
    if (MODE != DISCARD_MASKS && lane == 0) seg_cnt[r] = ao.at - t0 * TILE;
    }
    if (MODE == DISCARD_ASSIGN && cur_s >= 0) far_flush(L, gfar, cur_s);
}

// ---------------------------------------------------------------------------
// Survivor scatter: tile t's survivors go to positions tile_pos[t]... in
// ascending index order.  keys (optional): set << 48 | kx << 24 | ky.
__global__ __launch_bounds__(256) void k_scatter(
    const float *__restrict__ x, const float *__restrict__ y, int64_t n_total, int phase,
    const int64_t *__restrict__ off,
    int64_t S, const int64_t *__restrict__ tile_off, const int32_t *__restrict__ tile_set,
    const uint64_t *__restrict__ masks, const uint32_t *__restrict__ tile_cnt,
    const int64_t *__restrict__ tile_pos, uint32_t *__restrict__ surv, uint64_t *__restrict__ keys,
    const int64_t *__restrict__ out_base, int64_t cap) {
    // out_base (optional): device count of entries already in surv/keys, to
    // append after them; entries at or past cap are not written
    const int lane = lane_id();
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t W = (int64_t(gridDim.x) * blockDim.x) >> 6;
    const int64_t T = tile_off[S];
    const uint64_t lt = lanemask_lt();
    const int64_t ob = out_base ? *out_base : 0;
    for (int64_t t = wave; t < T; t += W) {
        const uint32_t tc = tile_cnt[t];
        if (tc == 0) continue;
        const int64_t s = tile_set[t];
        const int64_t o0 = set_begin(off, s);
        const int64_t tb = tile_base(o0, phase) + (t - tile_off[s]) * TILE;
        int64_t base = ob + tile_pos[t];
        // all loads of the tile are issued together: the 16 mask words, then
        // either the whole tile as float4 rows (many survivors) or one
        // gather per survivor
        const bool dense = keys && tc >= WAVE;
        uint64_t M[TILE_WORDS];
#pragma unroll
        for (int w = 0; w < TILE_WORDS; w++) M[w] = masks[t * TILE_WORDS + w];
        float xv[TILE_CHUNKS][4], yv[TILE_CHUNKS][4];
        if (dense) {
#pragma unroll
            for (int c = 0; c < TILE_CHUNKS; c++)
                load4(x, y, tb + c * CHUNK + 4 * lane, n_total, xv[c], yv[c]);
        } else if (keys) {
#pragma unroll
            for (int c = 0; c < TILE_CHUNKS; c++)
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int64_t gi = tb + c * CHUNK + 4 * lane + j;
                    xv[c][j] = 0.0f;
                    yv[c][j] = 0.0f;
                    if ((M[c * 4 + j] >> lane) & 1) {   // survivors only: in range
                        xv[c][j] = x[gi];
                        yv[c][j] = y[gi];
                    }
                }
        }
#pragma unroll
        for (int c = 0; c < TILE_CHUNKS; c++) {
            int pre = 0, tot = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                pre += __popcll(M[c * 4 + j] & lt);
                tot += __popcll(M[c * 4 + j]);
            }
            int k = 0;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                if ((M[c * 4 + j] >> lane) & 1) {
                    const int64_t gi = tb + c * CHUNK + 4 * lane + j;
                    const int64_t p = base + pre + k;
                    if (p < cap) surv[p] = (uint32_t)gi;
                    if (keys && p < cap) {
                        const uint64_t kx = (uint64_t)(uint32_t)(xv[c][j] * GRIDF);
                        const uint64_t ky = (uint64_t)(uint32_t)(yv[c][j] * GRIDF);
                        keys[p] = ((uint64_t)s << 48) | (kx << 24) | ky;
                    }
                    k++;
                }
            }
            base += tot;
        }
    }
}

// Per-set offsets from the tile scan: out[s] = tile_pos[tile_off[s]].
__global__ void k_set_offsets(const int64_t *__restrict__ tile_off,
                              const int64_t *__restrict__ tile_pos, int64_t S,
                              int64_t *__restrict__ out) {
    int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s <= S) out[s] = tile_pos[tile_off[s]];
}

// Unfiltered arm: every point survives (survivor list = identity).
__global__ __launch_bounds__(256) void k_all_keys(const float *__restrict__ x,
                                                  const float *__restrict__ y,
                                                  const int64_t *__restrict__ off, int64_t n1,
                                                  int64_t S, int64_t n_total,
                                                  uint32_t *__restrict__ surv,
                                                  uint64_t *__restrict__ keys,
                                                  int64_t *__restrict__ surv_off) {
    // sets are found by a scan of the offsets; each thread walks its points
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_total; i += stride) {
        int64_t s = 0;
        if (off) {   // binary search: largest s with off[s] <= i
            int64_t lo = 0, hi = S - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) >> 1;
                if (off[mid] <= i) lo = mid; else hi = mid - 1;
            }
            s = lo;
        }
        uint64_t kx = (uint64_t)(uint32_t)(x[i] * GRIDF);
        uint64_t ky = (uint64_t)(uint32_t)(y[i] * GRIDF);
        surv[i] = (uint32_t)i;
        keys[i] = ((uint64_t)s << 48) | (kx << 24) | ky;
    }
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g <= S) surv_off[g] = off ? off[g] : (g == 0 ? 0 : n1);
}

// Copy a polygon's vertex list and count to caller memory.
__global__ void k_poly_out(const Poly *__restrict__ P, int cap, uint32_t *__restrict__ verts,
                           int32_t *__restrict__ m) {
    int t = threadIdx.x;
    if (t < cap) verts[t] = t < P->m ? P->verts[t] : NONE;
    if (t == 0) *m = P->m;
}

// Input domain check: coordinates finite, in [0, 1), multiples of 2^-24;
// offsets non-decreasing from 0 to n_total.  Sets *err on a violation.
__global__ __launch_bounds__(256) void k_validate(const float *__restrict__ x,
                                                  const float *__restrict__ y, int64_t n,
                                                  const int64_t *__restrict__ off, int64_t S,
                                                  int *__restrict__ err) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    bool bad = false;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        float a = x[i], b = y[i];
        float ga = a * GRIDF, gb = b * GRIDF;
        bad |= !(a >= 0.0f && a < 1.0f && b >= 0.0f && b < 1.0f);
        bad |= (ga != truncf(ga)) || (gb != truncf(gb));
    }
    if (off) {
        for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s <= S; s += stride) {
            if (s == 0 && off[0] != 0) bad = true;
            if (s == S && off[S] != n) bad = true;
            if (s < S && off[s + 1] < off[s]) bad = true;
        }
    }
    if (bad) atomicOr(err, 1);
}

}  // namespace hg
