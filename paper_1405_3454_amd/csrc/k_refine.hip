// Hull of the survivors, first stage: QuickHull-style refinement rounds that
// shrink the survivor list before the sort and the monotone chain.
//
// Every survivor of Step 3 lies outside the filter polygon or on its
// boundary.  The discard pass assigns each survivor to an edge of the polygon
// that it lies strictly outside of (points on the boundary are kept and never
// looked at again).  Each round then, for every edge a->b, takes an outside point f
// of (close to) the largest distance from the edge's line, and replaces the
// edge by a->f and f->b; a point of the edge strictly inside the triangle
// (a, f, b) is dropped (the triangle's corners are points of the set, so such
// a point is strictly inside the hull), a point outside a->f or f->b moves to
// that edge.  Nothing depends on f being the exact farthest point: only the
// drops change the work, never the hull.  Repeated coordinates share every
// test, so all copies of a point stay or go together, and the hull stage picks
// the lowest index among them whatever order the kept survivors are in: each
// round appends them with one atomic allocation per chunk.
//
// Distances are exact edge functions in grid units (binary64, |E| < 2^52 on
// the grid); the farthest point per edge is the maximum of the packed key
// (float(distance) bits << 32 | ~index): close to the farthest, lowest index
// among equal keys, independent of the order of the atomics.
#include "hg_device.h"

namespace hg {

constexpr int REF_CH = 2048;                      // survivors per block step
constexpr int REF_THREADS = 256;
constexpr int REF_PER_THREAD = REF_CH / REF_THREADS;

struct REdge {
    int32_t ax, ay, bx, by;                       // grid units; ax == INT32_MIN: empty slot
};

__device__ __forceinline__ REdge redge_empty() { return REdge{INT32_MIN, 0, 0, 0}; }

// Exact edge function of a->b at p: > 0 strictly left (inside), < 0 outside.
__device__ __forceinline__ double redge_eval(const REdge &e, double px, double py) {
    const double ax = (double)e.ax, ay = (double)e.ay;
    const double ex = (double)e.bx - ax, ey = (double)e.by - ay;
    const double c = fma(ey, ax, -(ex * ay));
    return fma(ex, py, fma(-ey, px, c));
}

__device__ __forceinline__ void key_point(uint64_t k, int64_t *s, double *px, double *py) {
    *s = (int64_t)(k >> 48);
    *px = (double)((k >> 24) & 0xFFFFFF);
    *py = (double)(k & 0xFFFFFF);
}

// Round-0 edge table from the filter polygons; clears the farthest-point keys.
__global__ __launch_bounds__(64) void k_ref_init(const float *__restrict__ x,
                                                 const float *__restrict__ y,
                                                 const Poly *__restrict__ polys,
                                                 REdge *__restrict__ tab,
                                                 unsigned long long *__restrict__ far) {
    const int64_t s = blockIdx.x;
    const Poly &P = polys[s];
    const int m = P.m >= 3 ? P.m : 0;
    for (int e = threadIdx.x; e < RE_CAP; e += blockDim.x) {
        REdge r = redge_empty();
        if (e < m) {
            const uint32_t a = P.verts[e], b = P.verts[(e + 1) % m];
            r = REdge{(int32_t)(x[a] * GRIDF), (int32_t)(y[a] * GRIDF), (int32_t)(x[b] * GRIDF),
                      (int32_t)(y[b] * GRIDF)};
        }
        tab[s * RE_CAP + e] = r;
        far[s * RE_CAP + e] = 0;
    }
}

// Split every edge of round r at its farthest outside point: children 2e
// (a->f) and 2e+1 (f->b); an edge without outside points keeps itself as
// child 2e.  Clears the next round's farthest-point keys and the segment
// counts the round's pass appends to, and records the round's input total.
__global__ __launch_bounds__(256) void k_ref_split(const float *__restrict__ x,
                                                   const float *__restrict__ y, int64_t S, int er,
                                                   const REdge *__restrict__ tab,
                                                   const unsigned long long *__restrict__ far,
                                                   REdge *__restrict__ tab_nxt,
                                                   unsigned long long *__restrict__ far_nxt,
                                                   const int64_t *__restrict__ cnt_in,
                                                   int64_t *__restrict__ cnt_nxt,
                                                   int64_t *__restrict__ total_in) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < NSEG) {
        cnt_nxt[t] = 0;
        const int64_t v = wave_sum_i64(cnt_in[t]);
        if (t == 0) *total_in = v;
    }
    if (t >= S * er) return;
    const int64_t s = t / er;
    const int e = (int)(t % er);
    const REdge cur = tab[s * RE_CAP + e];
    REdge c0 = redge_empty(), c1 = redge_empty();
    if (cur.ax != INT32_MIN) {
        const uint64_t k = far[s * RE_CAP + e];
        if (k == 0) {
            c0 = cur;
        } else {
            const uint32_t f = ~(uint32_t)k;
            const int32_t fx = (int32_t)(x[f] * GRIDF), fy = (int32_t)(y[f] * GRIDF);
            c0 = REdge{cur.ax, cur.ay, fx, fy};
            c1 = REdge{fx, fy, cur.bx, cur.by};
        }
    }
    tab_nxt[s * RE_CAP + 2 * e] = c0;
    tab_nxt[s * RE_CAP + 2 * e + 1] = c1;
    far_nxt[s * RE_CAP + 2 * e] = 0;
    far_nxt[s * RE_CAP + 2 * e + 1] = 0;
}

// Farthest-point keys of a chunk: when the whole chunk belongs to one set,
// the block keeps them in LDS (ds_max_u64) and raises the global slots once
// per edge at the end; otherwise every point goes to the global slot.
struct RefFar {
    unsigned long long v[RE_CAP];
};

__device__ __forceinline__ void far_put(bool local, RefFar &L, unsigned long long *far, int64_t s,
                                        int e, uint64_t key) {
    if (local) {
        if (L.v[e] < key) atomicMax(&L.v[e], (unsigned long long)key);
    } else {
        far_update(&far[s * RE_CAP + e], key);
    }
}

// Chunks of REF_CH entries of a segmented list: prefix of the per-segment
// chunk counts (NSEG + 1 entries, computed by the block's first wave).
__device__ __forceinline__ void seg_chunks(const int64_t *__restrict__ cnt, int64_t *pre) {
    if (threadIdx.x < WAVE) {
        const int64_t nc = (cnt[threadIdx.x] + REF_CH - 1) / REF_CH;
        const int64_t inc = wave_incl_scan_i64(nc);
        pre[threadIdx.x] = inc - nc;
        if (threadIdx.x == WAVE - 1) pre[NSEG] = inc;
    }
    __syncthreads();
}

// Exclusive prefix of the segment counts themselves (NSEG + 1 entries).
__device__ __forceinline__ void seg_prefix(const int64_t *__restrict__ cnt, int64_t *pre) {
    if (threadIdx.x < WAVE) {
        const int64_t v = cnt[threadIdx.x];
        const int64_t inc = wave_incl_scan_i64(v);
        pre[threadIdx.x] = inc - v;
        if (threadIdx.x == WAVE - 1) pre[NSEG] = inc;
    }
    __syncthreads();
}

// Segment of chunk c: the last i with pre[i] <= c (one ballot per wave).
__device__ __forceinline__ int seg_of(const int64_t *pre, int64_t c) {
    const uint64_t m = __ballot(pre[lane_id()] <= c);
    return 63 - __clzll((long long)m);
}

// One round over the survivors, a chunk of REF_CH entries of one segment per
// block step (thread t holds entries t * REF_PER_THREAD ...).  Each survivor
// is classified against the two children of its edge (RE_DROP, RE_NONE or the
// new edge id); the kept ones are appended to segment (chunk mod NSEG) of the
// next list, the block's kept count reserving their range with one atomic.
// The farthest-point key of each new edge is raised.  (Round 0's edge states
// come from the discard pass.)
__global__ __launch_bounds__(REF_THREADS) void k_ref_pass(
    const uint32_t *__restrict__ idx, const uint64_t *__restrict__ keys,
    const uint16_t *__restrict__ edge, const int64_t *__restrict__ cnt_in, int64_t segcap,
    const REdge *__restrict__ tab_nxt, unsigned long long *__restrict__ far,
    uint32_t *__restrict__ idx_out, uint64_t *__restrict__ keys_out,
    uint16_t *__restrict__ edge_out, unsigned long long *__restrict__ cnt_out) {
    static_assert(NSEG == WAVE, "segment lookups use one lane per segment");
    __shared__ RefFar L;
    __shared__ int64_t scan_sh[17];
    __shared__ int64_t pre[NSEG + 1];
    __shared__ unsigned long long out_base;
    const int tid = threadIdx.x;
    seg_chunks(cnt_in, pre);
    const int64_t nch = pre[NSEG];
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const int sg = seg_of(pre, c);
        const int64_t jb = sg * segcap + (c - pre[sg]) * REF_CH;
        const int64_t je = min(sg * segcap + cnt_in[sg], jb + REF_CH);
        const int64_t j0 = jb + (int64_t)tid * REF_PER_THREAD;
        uint64_t k[REF_PER_THREAD];
        uint16_t st[REF_PER_THREAD];
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            const bool in = j0 + i < je;
            k[i] = in ? keys[j0 + i] : 0;
            st[i] = in ? edge[j0 + i] : RE_DROP;
        }
        // one set in the whole chunk?  (survivors of different sets can
        // interleave, so both ends alone do not tell)
        const int64_t s0 = (int64_t)(keys[jb] >> 48);
        bool same = true;
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++)
            same = same && (j0 + i >= je || (int64_t)(k[i] >> 48) == s0);
        const bool local = __syncthreads_and(same) != 0;
        if (local)
            for (int e = tid; e < RE_CAP; e += REF_THREADS) L.v[e] = 0;
        __syncthreads();
        int kept = 0;
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            if (st[i] == RE_DROP) continue;
            int64_t s;
            double px, py;
            key_point(k[i], &s, &px, &py);
            uint16_t out = RE_NONE;
            double dist = 0.0;
            if (st[i] != RE_NONE) {
                const REdge c0 = tab_nxt[s * RE_CAP + 2 * st[i]];
                const REdge c1 = tab_nxt[s * RE_CAP + 2 * st[i] + 1];
                if (c1.ax == INT32_MIN) {            // edge without a split point
                    const double E0 = redge_eval(c0, px, py);
                    if (E0 < 0) { out = (uint16_t)(2 * st[i]); dist = -E0; }
                } else {
                    const double E1 = redge_eval(c0, px, py), E2 = redge_eval(c1, px, py);
                    if (E1 > 0 && E2 > 0) out = RE_DROP;
                    else if (E1 < 0) { out = (uint16_t)(2 * st[i]); dist = -E1; }
                    else if (E2 < 0) { out = (uint16_t)(2 * st[i] + 1); dist = -E2; }
                }
            }
            if (out != RE_NONE && out != RE_DROP) far_put(local, L, far, s, out, far_key(dist, idx[j0 + i]));
            st[i] = out;
            kept += out != RE_DROP;
        }
        const int og = (int)(c & (NSEG - 1));
        int64_t tot;
        int64_t pos = block_excl_scan_i64(kept, scan_sh, &tot);
        if (tid == 0) out_base = tot ? atomicAdd(&cnt_out[og], (unsigned long long)tot) : 0;
        __syncthreads();
        pos += og * segcap + (int64_t)out_base;
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            if (st[i] == RE_DROP) continue;
            idx_out[pos] = idx[j0 + i];
            keys_out[pos] = k[i];
            edge_out[pos] = st[i];
            pos++;
        }
        __syncthreads();
        if (local)
            for (int e = tid; e < RE_CAP; e += REF_THREADS) {
                const unsigned long long v = L.v[e];
                if (v) far_update(&far[s0 * RE_CAP + e], v);
            }
        __syncthreads();
    }
}

// Segmented list (idx, keys) -> contiguous arrays; *total_out = entries.
// Block b copies segment b mod NSEG, entries (b / NSEG) * 256 + t, stepping
// by the blocks per segment.
__global__ __launch_bounds__(256) void k_seg_gather(const uint32_t *__restrict__ idx,
                                                    const uint64_t *__restrict__ keys,
                                                    const int64_t *__restrict__ cnt, int64_t segcap,
                                                    uint32_t *__restrict__ idx_out,
                                                    uint64_t *__restrict__ keys_out,
                                                    int64_t *__restrict__ total_out) {
    __shared__ int64_t pre[NSEG + 1];
    seg_prefix(cnt, pre);
    const int sg = (int)(blockIdx.x % NSEG);
    const int64_t per = gridDim.x / NSEG;
    const int64_t n = cnt[sg], dst = pre[sg], src = sg * segcap;
    for (int64_t i = (int64_t)(blockIdx.x / NSEG) * blockDim.x + threadIdx.x; i < n;
         i += per * blockDim.x) {
        idx_out[dst + i] = idx[src + i];
        keys_out[dst + i] = keys[src + i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *total_out = pre[NSEG];
}

}  // namespace hg
