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
                                                   const int64_t *__restrict__ cnt_in, int nseg_in,
                                                   int64_t *__restrict__ cnt_nxt,
                                                   int64_t *__restrict__ total_in) {
    __shared__ int64_t sh[17];
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0) {     // the whole block: record the input total
        int64_t acc = 0;
        for (int j = threadIdx.x; j < nseg_in; j += blockDim.x) acc += cnt_in[j];
        int64_t tot;
        block_excl_scan_i64(acc, sh, &tot);
        if (threadIdx.x == 0) *total_in = tot;
        if (threadIdx.x < NSEG) cnt_nxt[threadIdx.x] = 0;
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

// Blocks of a grid over the segments of a list: bps blocks per segment,
// `lanes` segments at a time (every segment, when there are more of them than
// blocks, goes to one block).
struct SegWalk {
    int64_t bps, lanes;
    __device__ SegWalk(int64_t nseg) {
        bps = max((int64_t)1, (int64_t)gridDim.x / max(nseg, (int64_t)1));
        lanes = (int64_t)gridDim.x / bps;
    }
    __device__ bool idle() const { return (int64_t)blockIdx.x >= bps * lanes; }
    __device__ int64_t first_seg() const { return (int64_t)blockIdx.x / bps; }
    __device__ int64_t first_part() const { return (int64_t)blockIdx.x % bps; }
};

// One round over the survivors: input segment sg (region sg * segcap_in,
// cnt_in[sg] entries) in chunks of REF_CH, thread t holding entries
// t * REF_PER_THREAD ... of a chunk.  Each survivor is classified against the
// two children of its edge (RE_DROP, RE_NONE or the new edge id); the kept
// ones are appended to output segment sg mod NSEG, the block's kept count
// reserving their range with one atomic.  The farthest-point key of each new
// edge is raised.  (Round 0's input is the discard pass's per-wave regions,
// with their edge states.)
__global__ __launch_bounds__(REF_THREADS) void k_ref_pass(
    const uint32_t *__restrict__ idx, const uint64_t *__restrict__ keys,
    const uint16_t *__restrict__ edge, const int64_t *__restrict__ cnt_in, int nseg_in,
    const int64_t *__restrict__ segcap_in, const REdge *__restrict__ tab_nxt, int er2,
    unsigned long long *__restrict__ far, uint32_t *__restrict__ idx_out,
    uint64_t *__restrict__ keys_out, uint16_t *__restrict__ edge_out,
    unsigned long long *__restrict__ cnt_out, int64_t segcap_out) {
    __shared__ RefFar L;
    __shared__ REdge ltab[RE_CAP];          // the chunk's set's child edges (er2 of them)
    __shared__ int64_t scan_sh[17];
    __shared__ unsigned long long out_base;
    const int tid = threadIdx.x;
    const SegWalk wk(nseg_in);
    if (wk.idle()) return;
    const int64_t segcap = *segcap_in;
    for (int64_t sg = wk.first_seg(); sg < nseg_in; sg += wk.lanes) {
    const int64_t n_sg = cnt_in[sg];
    for (int64_t ch = wk.first_part(); ch * REF_CH < n_sg; ch += wk.bps) {
        const int64_t jb = sg * segcap + ch * REF_CH;
        const int64_t je = sg * segcap + min(n_sg, (ch + 1) * REF_CH);
        const int64_t j0 = jb + (int64_t)tid * REF_PER_THREAD;
        uint64_t k[REF_PER_THREAD];
        uint16_t st[REF_PER_THREAD];
        uint32_t ix[REF_PER_THREAD];
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            const bool in = j0 + i < je;
            k[i] = in ? keys[j0 + i] : 0;
            st[i] = in ? edge[j0 + i] : RE_DROP;
            ix[i] = in ? idx[j0 + i] : 0;
        }
        // one set in the whole chunk?  (survivors of different sets can
        // interleave, so both ends alone do not tell)
        const int64_t s0 = (int64_t)(keys[jb] >> 48);
        bool same = true;
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++)
            same = same && (j0 + i >= je || (int64_t)(k[i] >> 48) == s0);
        const bool local = __syncthreads_and(same) != 0;
        if (local) {
            for (int e = tid; e < RE_CAP; e += REF_THREADS) L.v[e] = 0;
            for (int e = tid; e < er2; e += REF_THREADS) ltab[e] = tab_nxt[s0 * RE_CAP + e];
        }
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
                const int e0 = 2 * st[i];
                const REdge c0 = local ? ltab[e0] : tab_nxt[s * RE_CAP + e0];
                const REdge c1 = local ? ltab[e0 + 1] : tab_nxt[s * RE_CAP + e0 + 1];
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
            if (out != RE_NONE && out != RE_DROP) far_put(local, L, far, s, out, far_key(dist, ix[i]));
            st[i] = out;
            kept += out != RE_DROP;
        }
        const int og = (int)(sg & (NSEG - 1));
        int64_t tot;
        int64_t pos = block_excl_scan_i64(kept, scan_sh, &tot);
        if (tid == 0) out_base = tot ? atomicAdd(&cnt_out[og], (unsigned long long)tot) : 0;
        __syncthreads();
        pos += og * segcap_out + (int64_t)out_base;
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            if (st[i] == RE_DROP) continue;
            idx_out[pos] = ix[i];
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
}

// Segmented list (idx, keys) -> contiguous arrays in segment order;
// *total_out = entries.  Each block carries the output offset of its
// segments forward (its own segments come `lanes` apart).
__global__ __launch_bounds__(256) void k_seg_gather(const uint32_t *__restrict__ idx,
                                                    const uint64_t *__restrict__ keys,
                                                    const int64_t *__restrict__ cnt, int nseg,
                                                    const int64_t *__restrict__ segcap_in,
                                                    uint32_t *__restrict__ idx_out,
                                                    uint64_t *__restrict__ keys_out,
                                                    int64_t *__restrict__ total_out) {
    __shared__ int64_t sh[17];
    const SegWalk wk(nseg);
    const int tid = threadIdx.x;
    if (blockIdx.x == 0) {
        int64_t acc = 0;
        for (int j = tid; j < nseg; j += blockDim.x) acc += cnt[j];
        int64_t tot;
        block_excl_scan_i64(acc, sh, &tot);
        if (tid == 0) *total_out = tot;
    }
    if (wk.idle()) return;
    const int64_t segcap = *segcap_in;
    int64_t dst = 0, done = 0;          // dst = sum of cnt[0 .. done)
    for (int64_t sg = wk.first_seg(); sg < nseg; sg += wk.lanes) {
        int64_t acc = 0;
        for (int64_t j = done + tid; j < sg; j += blockDim.x) acc += cnt[j];
        int64_t add;
        block_excl_scan_i64(acc, sh, &add);
        dst += add;
        done = sg;
        const int64_t n = cnt[sg], src = sg * segcap;
        for (int64_t i = wk.first_part() * blockDim.x + tid; i < n; i += wk.bps * blockDim.x) {
            idx_out[dst + i] = idx[src + i];
            keys_out[dst + i] = keys[src + i];
        }
    }
}

}  // namespace hg
