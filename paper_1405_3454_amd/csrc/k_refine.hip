// Hull of the survivors, first stage: QuickHull-style refinement rounds that
// shrink the survivor list before the sort and the monotone chain.
//
// Every survivor of Step 3 lies outside the filter polygon or on its
// boundary.  Round 0 assigns each survivor to an edge of the polygon that it
// lies strictly outside of (points on the boundary are kept and never looked
// at again).  Each round then, for every edge a->b, takes an outside point f
// of (close to) the largest distance from the edge's line, and replaces the
// edge by a->f and f->b; a point of the edge strictly inside the triangle
// (a, f, b) is dropped (the triangle's corners are points of the set, so such
// a point is strictly inside the hull), a point outside a->f or f->b moves to
// that edge.  Nothing depends on f being the exact farthest point: only the
// drops change the work, never the hull.  The survivors stay in ascending
// index order within each set, so the hull's lowest-index representatives of
// repeated coordinates are the ones the chain finds.
//
// Distances are exact edge functions in grid units (binary64, |E| < 2^52 on
// the grid); the farthest point per edge is the maximum of the packed key
// (float(distance) bits << 32 | ~index): close to the farthest, lowest index
// among equal keys, independent of the order of the atomics.
#include "hg_device.h"

namespace hg {

constexpr int REF_ROUNDS = 4;
constexpr int RE_CAP = MAX_SLOTS << REF_ROUNDS;   // edge slots per set and round
constexpr int REF_CH = 2048;                      // survivors per compaction chunk
constexpr int REF_THREADS = 256;
constexpr int REF_PER_THREAD = REF_CH / REF_THREADS;
constexpr uint16_t RE_NONE = 0xFFFF;              // kept, not assigned to an edge
constexpr uint16_t RE_DROP = 0xFFFE;              // strictly inside the hull

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

__device__ __forceinline__ uint64_t far_key(double dist, uint32_t idx) {
    return ((uint64_t)__float_as_uint((float)dist) << 32) | (uint64_t)(~idx);
}

// Raise *slot to key unless it already holds at least as much.
__device__ __forceinline__ void far_update(unsigned long long *slot, uint64_t key) {
    if (*reinterpret_cast<volatile unsigned long long *>(slot) < key) atomicMax(slot, key);
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
// child 2e.  Clears the next round's farthest-point keys.
__global__ __launch_bounds__(256) void k_ref_split(const float *__restrict__ x,
                                                   const float *__restrict__ y, int64_t S, int er,
                                                   const REdge *__restrict__ tab,
                                                   const unsigned long long *__restrict__ far,
                                                   REdge *__restrict__ tab_nxt,
                                                   unsigned long long *__restrict__ far_nxt) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
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

// Number of compaction chunks for the current survivor count.
__global__ void k_ref_nchunks(const int64_t *__restrict__ cnt_ptr, int64_t *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = (*cnt_ptr + REF_CH - 1) / REF_CH;
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

// One pass over the survivors in chunks of REF_CH (thread t holds elements
// t * REF_PER_THREAD ...).  ASSIGN (round 0): each survivor goes to the first
// filter-polygon edge it is strictly outside of (RE_NONE: on the boundary).
// Otherwise: each survivor is classified against the two children of its
// edge (state written in place: RE_DROP, RE_NONE or the new edge id) and the
// kept ones are counted per chunk.  Either way the farthest-point key of each
// (new) edge is raised.
template <bool ASSIGN>
__global__ __launch_bounds__(REF_THREADS) void k_ref_pass(
    const uint32_t *__restrict__ idx, const uint64_t *__restrict__ keys,
    const int64_t *__restrict__ cnt_ptr, uint16_t *__restrict__ edge,
    const Poly *__restrict__ polys, const uint32_t *__restrict__ redges,
    const REdge *__restrict__ tab_nxt, unsigned long long *__restrict__ far,
    uint32_t *__restrict__ chunk_cnt) {
    __shared__ RefFar L;
    __shared__ double pex[ROW_EDGE_NONE + 1], pey[ROW_EDGE_NONE + 1], pc[ROW_EDGE_NONE + 1];
    __shared__ uint32_t lre[SPAN_ROWS];     // the set's row edge lists (Step 3's rows)
    __shared__ int pm, pky, pyl, psh;
    __shared__ uint32_t wsum[REF_THREADS / WAVE];
    const int64_t cnt = *cnt_ptr;
    const int64_t nch = (cnt + REF_CH - 1) / REF_CH;
    const int tid = threadIdx.x;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const int64_t jb = c * REF_CH, je = min(cnt, jb + REF_CH);
        const int64_t s0 = (int64_t)(keys[jb] >> 48), s1 = (int64_t)(keys[je - 1] >> 48);
        const bool local = s0 == s1;
        if (local) {
            for (int e = tid; e < RE_CAP; e += REF_THREADS) L.v[e] = 0;
            if (ASSIGN) {
                const Poly &P = polys[s0];
                if (tid <= ROW_EDGE_NONE) {    // unused slots: an always-satisfied edge
                    pex[tid] = tid < MAX_SLOTS ? P.ex[tid] : 0.0;
                    pey[tid] = tid < MAX_SLOTS ? P.ey[tid] : 0.0;
                    pc[tid] = tid < MAX_SLOTS ? P.c[tid] : 1.0;
                }
                for (int r = tid; r < SPAN_ROWS; r += REF_THREADS) lre[r] = redges[s0 * SPAN_ROWS + r];
                if (tid == 0) {
                    pm = P.m >= 3 ? P.m : 0;
                    pky = P.ky_lo;
                    pyl = P.yspan;
                    psh = P.shift;
                }
            }
        }
        __syncthreads();
        const int64_t j0 = jb + (int64_t)tid * REF_PER_THREAD;
        uint64_t k[REF_PER_THREAD];
        uint16_t st[REF_PER_THREAD];
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            const bool in = j0 + i < je;
            k[i] = in ? keys[j0 + i] : 0;
            st[i] = in ? (ASSIGN ? (uint16_t)0 : edge[j0 + i]) : RE_DROP;
        }
        uint32_t kept = 0;
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            if (st[i] == RE_DROP) continue;
            int64_t s;
            double px, py;
            key_point(k[i], &s, &px, &py);
            uint16_t out = RE_NONE;
            double dist = 0.0;
            if (ASSIGN) {
                if (local) {
                    // a point of a row is strictly outside the polygon iff it is
                    // strictly outside one of the (at most four) edges meeting
                    // the row; points outside the rows try every edge
                    const uint32_t dy = (uint32_t)((int32_t)py - pky);
                    const uint32_t re = (pm > 0 && pyl >= 0 && dy <= (uint32_t)pyl) ? lre[dy >> psh]
                                                                                 : ROW_EDGES_ALL;
                    if (re != ROW_EDGES_ALL) {
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            const int e = (re >> (8 * q)) & 0xFF;
                            const double E = edge_eval(pex[e], pey[e], pc[e], px, py);
                            if (E < 0 && out == RE_NONE) { out = (uint16_t)e; dist = -E; }
                        }
                    } else {
                        for (int e = 0; e < pm; e++) {
                            const double E = edge_eval(pex[e], pey[e], pc[e], px, py);
                            if (E < 0) { out = (uint16_t)e; dist = -E; break; }
                        }
                    }
                } else {
                    const Poly &P = polys[s];
                    const int m = P.m >= 3 ? P.m : 0;
                    for (int e = 0; e < m; e++) {
                        const double E = edge_eval(P.ex[e], P.ey[e], P.c[e], px, py);
                        if (E < 0) { out = (uint16_t)e; dist = -E; break; }
                    }
                }
            } else if (st[i] != RE_NONE) {
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
            if (ASSIGN || st[i] != RE_NONE) edge[j0 + i] = out;
            kept += out != RE_DROP;
        }
        if (!ASSIGN) {
            uint32_t v = kept;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
            if (lane_id() == 0) wsum[tid >> 6] = v;
        }
        __syncthreads();
        if (local)
            for (int e = tid; e < RE_CAP; e += REF_THREADS) {
                const unsigned long long v = L.v[e];
                if (v) far_update(&far[s0 * RE_CAP + e], v);
            }
        if (!ASSIGN && tid == 0) {
            uint32_t t = 0;
            for (int w = 0; w < REF_THREADS / WAVE; w++) t += wsum[w];
            chunk_cnt[c] = t;
        }
        __syncthreads();
    }
}

// Order-preserving compaction of the kept survivors into the next arrays.
__global__ __launch_bounds__(REF_THREADS) void k_ref_compact(
    const uint32_t *__restrict__ idx, const uint64_t *__restrict__ keys,
    const uint16_t *__restrict__ edge, const int64_t *__restrict__ cnt_ptr,
    const int64_t *__restrict__ chunk_pos, uint32_t *__restrict__ idx_nxt,
    uint64_t *__restrict__ keys_nxt, uint16_t *__restrict__ edge_nxt) {
    __shared__ int64_t sh[REF_THREADS / WAVE + 1];
    const int64_t cnt = *cnt_ptr;
    const int64_t nch = (cnt + REF_CH - 1) / REF_CH;
    const int tid = threadIdx.x;
    for (int64_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const int64_t j0 = c * REF_CH + (int64_t)tid * REF_PER_THREAD;
        uint16_t st[REF_PER_THREAD];
        uint64_t k[REF_PER_THREAD];
        uint32_t ix[REF_PER_THREAD];
        int kept = 0;
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            st[i] = (j0 + i < cnt) ? edge[j0 + i] : RE_DROP;
            const bool keep = st[i] != RE_DROP;
            k[i] = keep ? keys[j0 + i] : 0;
            ix[i] = keep ? idx[j0 + i] : 0;
            kept += keep;
        }
        int64_t tot;
        int64_t pos = chunk_pos[c] + block_excl_scan_i64(kept, sh, &tot);
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            if (st[i] == RE_DROP) continue;
            idx_nxt[pos] = ix[i];
            keys_nxt[pos] = k[i];
            edge_nxt[pos] = st[i];
            pos++;
        }
    }
}

// Survivor count after a round: the chunk scan's total.
__global__ void k_ref_total(const int64_t *__restrict__ chunk_pos,
                            const int64_t *__restrict__ nch_ptr, int64_t *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = chunk_pos[*nch_ptr];
}

}  // namespace hg
