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
// round packs them into its blocks' own output regions.
//
// Distances are exact edge functions in grid units (binary64, |E| < 2^52 on
// the grid); the farthest point per edge is the maximum of the packed key
// (float(distance) bits << 32 | ~index): close to the farthest, lowest index
// among equal keys, independent of the order of the atomics.
#include "hg_device.h"

namespace hg {

constexpr int REF_PER_THREAD = 8;                 // survivors per thread and block step
constexpr int REF_THREADS = 256;                  // pass block size
constexpr int REF_THREADS_LATE = 512;             // one set, rounds after 0 (fewer blocks)


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

// Children of edge cur at its farthest outside point (key k): 2e = a->f and
// 2e+1 = f->b; an edge without outside points keeps itself as child 2e.
__device__ __forceinline__ void split_pair(const float *__restrict__ x, const float *__restrict__ y,
                                           const REdge &cur, uint64_t k, REdge *c0, REdge *c1) {
    *c0 = redge_empty();
    *c1 = redge_empty();
    if (cur.ax == INT32_MIN) return;
    if (k == 0) {
        *c0 = cur;
        return;
    }
    const uint32_t f = ~(uint32_t)k;
    const int32_t fx = (int32_t)(x[f] * GRIDF), fy = (int32_t)(y[f] * GRIDF);
    *c0 = REdge{cur.ax, cur.ay, fx, fy};
    *c1 = REdge{fx, fy, cur.bx, cur.by};
}

// Split every edge of round r (er per set) at its farthest outside point and
// clear the children's farthest-point keys.
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
    REdge c0, c1;
    split_pair(x, y, tab[s * RE_CAP + e], far[s * RE_CAP + e], &c0, &c1);
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

constexpr int REF_GROUP = 4;                      // most input regions one block reads
// input regions per block in round r.  One set: fuller chunks early, enough
// blocks late.  Several sets: one region per block (their survivor counts
// differ with the sets' shapes, and a block walks its chunks in turn, so
// the fullest block sets the pass's time).
__host__ __device__ inline int ref_group(int r, bool batched) { return batched ? 1 : r == 0 ? 4 : 2; }

// One round over the survivors.  A list is a row of regions (region r at
// r * segcap, cnt[r] entries; round 0 reads the discard pass's, one per
// wave).  Block g reads regions [g * kg, (g + 1) * kg) as one list, in
// chunks of RT * REF_PER_THREAD (thread t holds list entries t, t + RT, ...).
// Each survivor is classified against the two children of its edge
// (RE_DROP, RE_NONE or the new edge id); the kept ones are packed into region
// g (size kg * segcap) of the next list, whose count the block writes at the
// end: no atomics.  The farthest-point key of each new edge is raised.  (Round 0's
// input is the discard pass's regions, with their edge states.)  With one set
// (one_set), the set's child edges are staged once per block, before the
// first chunk's loads return, and the farthest keys are raised once per block.
template <int RT>
__global__ __launch_bounds__(RT) void k_ref_pass(
    const uint32_t *__restrict__ idx, const uint64_t *__restrict__ keys,
    const uint16_t *__restrict__ edge, const int64_t *__restrict__ cnt_in, int nreg_in, int kg,
    const int64_t *__restrict__ region_size, int64_t mult, const REdge *__restrict__ tab_nxt, int er2,
    unsigned long long *__restrict__ far, uint32_t *__restrict__ idx_out,
    uint64_t *__restrict__ keys_out, uint16_t *__restrict__ edge_out,
    int64_t *__restrict__ cnt_out, int one_set, const float *__restrict__ x,
    const float *__restrict__ y, const REdge *__restrict__ tab_par,
    const unsigned long long *__restrict__ far_par, REdge *__restrict__ tab_out,
    unsigned long long *__restrict__ far_clr) {
    constexpr int NW = RT / WAVE;
    __shared__ RefFar L;
    __shared__ REdge ltab[RE_CAP];          // the chunk's set's child edges (er2 of them)
    __shared__ uint32_t kc[REF_PER_THREAD][NW];   // kept per (element row, wave) -> offsets
    __shared__ uint32_t ktot;
    __shared__ int64_t pre[REF_GROUP + 1];  // list offsets of the group's regions
    const int tid = threadIdx.x, w = tid / WAVE;
    const int64_t g = blockIdx.x;
    const int64_t segcap = *region_size * mult;      // input region size
    const int64_t r0 = g * kg, nr = max((int64_t)0, min((int64_t)kg, (int64_t)nreg_in - r0));
    if (tid == 0) {
        int64_t run = 0;
        for (int j = 0; j < nr; j++) {
            pre[j] = run;
            run += cnt_in[r0 + j];
        }
        pre[nr] = run;
    }
    __syncthreads();
    const int64_t n_sg = pre[nr];
    // One set with tab_par: the block splits the er2 / 2 parent edges itself
    // (children into LDS); block 0 also publishes them for the next round and
    // clears the farthest keys the round after this one raises.
    auto split_here = [&](bool to_lds) {
        for (int e = tid; e < er2 / 2; e += RT) {
            REdge c0, c1;
            split_pair(x, y, tab_par[e], far_par[e], &c0, &c1);
            if (to_lds) {
                ltab[2 * e] = c0;
                ltab[2 * e + 1] = c1;
            }
            if (g == 0) {
                tab_out[2 * e] = c0;
                tab_out[2 * e + 1] = c1;
            }
        }
        if (g == 0)
            for (int e = tid; e < RE_CAP; e += RT) far_clr[e] = 0;
    };
    if (n_sg == 0) {                        // nothing to read: an empty region, no far keys
        if (tid == 0) cnt_out[g] = 0;
        if (tab_par && g == 0) split_here(false);
        return;
    }
    const int64_t region = r0 * segcap;     // output region g: [region, region + kg * segcap)
    // list entry v -> its address (regions of the group in order)
    auto addr = [&](int64_t v) {
        int j = 0;
        while (j + 1 < nr && pre[j + 1] <= v) j++;
        return (r0 + j) * segcap + (v - pre[j]);
    };
    int64_t outn = 0;                       // entries packed into the region so far
    int64_t held = -1;                      // several sets: the set held in LDS (ltab, L.v)
    __shared__ int64_t sfirst;
    if (one_set) {
        for (int e = tid; e < RE_CAP; e += RT) L.v[e] = 0;
        if (tab_par)
            split_here(true);
        else
            for (int e = tid; e < er2; e += RT) ltab[e] = tab_nxt[e];
    }
    for (int64_t jb = 0; jb < n_sg; jb += (RT * REF_PER_THREAD)) {
        const int64_t je = min(n_sg, jb + (RT * REF_PER_THREAD));
        const int64_t j0 = jb + tid;        // element i: j0 + i * RT (coalesced)
        uint64_t k[REF_PER_THREAD];
        uint16_t st[REF_PER_THREAD];
        uint32_t ix[REF_PER_THREAD];
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            const int64_t j = j0 + (int64_t)i * RT;
            const bool in = j < je;
            const int64_t a = in ? addr(j) : 0;
            k[i] = in ? keys[a] : 0;
            st[i] = in ? edge[a] : RE_DROP;
            ix[i] = in ? idx[a] : 0;
        }
        // one set in the whole chunk?  (a region can span sets)  The set
        // whose child edges and farthest keys the block holds in LDS stays
        // there over consecutive chunks of that set; its keys are raised in
        // global memory when another set's chunk comes, and at the end.
        int64_t s0 = 0;
        bool local = true;
        if (!one_set) {
            if (tid == 0) sfirst = (int64_t)(k[0] >> 48);   // entry jb is thread 0's first
            __syncthreads();
            s0 = sfirst;
            bool same = true;
#pragma unroll
            for (int i = 0; i < REF_PER_THREAD; i++)
                same = same && (j0 + (int64_t)i * RT >= je || (int64_t)(k[i] >> 48) == s0);
            local = __syncthreads_and(same) != 0;
            if (held >= 0 && (!local || s0 != held)) {   // the held set's keys go out
                for (int e = tid; e < er2; e += RT) {
                    const unsigned long long v = L.v[e];
                    if (v) far_update(&far[held * RE_CAP + e], v);
                }
                held = -1;
                __syncthreads();
            }
            if (local && held < 0) {
                for (int e = tid; e < er2; e += RT) {
                    L.v[e] = 0;
                    ltab[e] = tab_nxt[s0 * RE_CAP + e];
                }
                held = s0;
            }
        }
        __syncthreads();
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
                    if (E0 < 0) { out = (uint16_t)e0; dist = -E0; }
                } else {
                    const double E1 = redge_eval(c0, px, py), E2 = redge_eval(c1, px, py);
                    if (E1 > 0 && E2 > 0) out = RE_DROP;
                    else if (E1 < 0) { out = (uint16_t)e0; dist = -E1; }
                    else if (E2 < 0) { out = (uint16_t)(e0 + 1); dist = -E2; }
                }
            }
            if (out != RE_NONE && out != RE_DROP) far_put(local, L, far, s, out, far_key(dist, ix[i]));
            st[i] = out;
        }
        // kept entries packed in (element row, wave, lane) order: every row's
        // stores from a wave go to consecutive slots
        uint64_t bm[REF_PER_THREAD];
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            bm[i] = __ballot(st[i] != RE_DROP);
            if (lane_id() == 0) kc[i][w] = (uint32_t)__popcll(bm[i]);
        }
        __syncthreads();
        if (tid < WAVE) {     // exclusive prefix over (row, wave) in one wave
            static_assert(REF_PER_THREAD * NW <= WAVE, "one lane per (row, wave)");
            uint32_t *flat = &kc[0][0];
            const uint32_t c = tid < REF_PER_THREAD * NW ? flat[tid] : 0;
            const uint32_t inc = (uint32_t)wave_incl_scan_i64(c);
            if (tid < REF_PER_THREAD * NW) flat[tid] = inc - c;
            if (tid == WAVE - 1) ktot = inc;
        }
        __syncthreads();
        const uint64_t lt = lanemask_lt();
        const int64_t base = region + outn;
#pragma unroll
        for (int i = 0; i < REF_PER_THREAD; i++) {
            if (st[i] == RE_DROP) continue;
            const int64_t pos = base + kc[i][w] + __popcll(bm[i] & lt);
            idx_out[pos] = ix[i];
            keys_out[pos] = k[i];
            edge_out[pos] = st[i];
        }
        outn += ktot;
        __syncthreads();
    }
    if (one_set || held >= 0) {
        __syncthreads();
        const int64_t fs = one_set ? 0 : held;
        for (int e = tid; e < er2; e += RT) {
            const unsigned long long v = L.v[e];
            if (v) far_update(&far[fs * RE_CAP + e], v);
        }
    }
    if (tid == 0) cnt_out[g] = outn;
}

// Regions of list stage r (0: the discard pass's, one per wave; round r
// reads them and writes stage r + 1, one region per group of ref_group(r)).
__host__ __device__ inline int64_t stage_regions(int64_t nwave, int r, bool batched) {
    int64_t n = nwave;
    for (int i = 0; i < r; i++) n = (n + ref_group(i, batched) - 1) / ref_group(i, batched);
    return n;
}

// Region list (idx, keys) of list stage nstage - 1 (region counts of stage r
// at cnt_all + r * nwave) -> contiguous arrays in region order.  Block b
// copies the consecutive regions [b * per, (b + 1) * per), starting at the
// sum of the counts before them; totals[r] gets the entries of stage r for
// every r < nstage.
__global__ __launch_bounds__(256) void k_seg_gather(const uint32_t *__restrict__ idx,
                                                    const uint64_t *__restrict__ keys,
                                                    const int64_t *__restrict__ cnt_all, int nwave,
                                                    int nstage, int batched,
                                                    const int64_t *__restrict__ region_size,
                                                    int64_t mult,
                                                    uint32_t *__restrict__ idx_out,
                                                    uint64_t *__restrict__ keys_out,
                                                    int64_t *__restrict__ totals) {
    __shared__ int64_t sh[17];
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < nstage) {
        const int64_t *c = cnt_all + (int64_t)blockIdx.x * nwave;
        const int64_t nr = stage_regions(nwave, (int)blockIdx.x, batched);
        int64_t a = 0;
        for (int64_t j = tid; j < nr; j += blockDim.x) a += c[j];
        int64_t t;
        block_excl_scan_i64(a, sh, &t);
        if (tid == 0) totals[blockIdx.x] = t;
    }
    // stage nstage - 1: its regions, of size region_size * mult
    const int64_t *cnt = cnt_all + (int64_t)(nstage - 1) * nwave;
    const int64_t nseg = stage_regions(nwave, nstage - 1, batched);
    const int64_t per = (nseg + gridDim.x - 1) / gridDim.x;
    const int64_t g0 = min((int64_t)nseg, (int64_t)blockIdx.x * per);
    const int64_t g1 = min((int64_t)nseg, g0 + per);
    int64_t acc = 0;
    for (int64_t j = tid; j < g0; j += blockDim.x) acc += cnt[j];
    int64_t dst;
    block_excl_scan_i64(acc, sh, &dst);
    const int64_t segcap = *region_size * mult;
    for (int64_t sg = g0; sg < g1; sg++) {
        const int64_t n = cnt[sg], src = sg * segcap;
        for (int64_t i = tid; i < n; i += blockDim.x) {
            idx_out[dst + i] = idx[src + i];
            keys_out[dst + i] = keys[src + i];
        }
        dst += n;
    }
}

}  // namespace hg
