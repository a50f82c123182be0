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

// A child edge a->b as the coefficients of its edge function at p,
// E(p) = ex py - ey px + c with (ex, ey) = b - a and c = ey ax - ex ay:
// > 0 strictly left of a->b (inside), < 0 outside.  On the grid (integers
// below 2^24) every product and fused sum here is exact in binary64 (|E| <
// 2^52), so a survivor's test costs two fused multiply-adds per edge.  An
// empty slot has c = NaN: E is NaN, and no comparison with it holds.
struct EdgeF {
    double ex, ey, c;
};
__device__ __forceinline__ EdgeF edge_f(const REdge &e) {
    if (e.ax == INT32_MIN) return EdgeF{0.0, 0.0, __longlong_as_double(0x7ff8000000000000ll)};
    const double ax = (double)e.ax, ay = (double)e.ay;
    const double ex = (double)e.bx - ax, ey = (double)e.by - ay;
    return EdgeF{ex, ey, fma(ey, ax, -(ex * ay))};
}
__device__ __forceinline__ double edge_eval(const EdgeF &f, double px, double py) {
    return fma(f.ex, py, fma(-f.ey, px, f.c));
}

// A wave-uniform int64 moved into scalar registers.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
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

constexpr int REF_GROUP = 4;                      // most input regions one wave reads
// input regions per wave in round r.  One region per wave in round 0 (the
// discard pass's regions hold the most survivors, and a wave walks its
// chunks in turn); later rounds hold about four times fewer per round, and
// several sets leave many regions nearly empty, so their waves read two.
__host__ __device__ inline int ref_group(int r, bool batched) { return r == 0 ? 1 : 2; }

// Waves per block of a pass.  Each wave works alone; the block shares the
// farthest keys (one table with one set, and waves holding the same set
// merge theirs at the end), so each block raises the global slots once
// instead of each wave: thousands of waves raising the same few dozen slots
// serialise on them.
constexpr int REF_WAVES = 4;

// LDS of a pass: the farthest keys, then the child edges (as EdgeF), er2 of
// each: one table per block with one set, one per wave with several.
__host__ __device__ inline size_t ref_lds_bytes(int er2, bool one_set) {
    return (size_t)(one_set ? 1 : REF_WAVES) * er2 * (sizeof(unsigned long long) + 3 * sizeof(double));
}

// One round over the survivors.  A list is a row of regions (region r at
// r * segcap, cnt[r] entries; round 0 reads the discard pass's).  Wave g of
// the grid reads regions [g * kg, (g + 1) * kg) as one list, in chunks of
// REF_CHUNK (lane l holds chunk entries l, l + 64, ...), with no block
// barriers in its walk.  Each survivor is classified against the two
// children of its edge (RE_DROP, RE_NONE or the new edge id); the kept ones
// are packed into region g (size kg * segcap) of the next list in (chunk,
// row, lane) order, and the wave writes their count at the end: no atomics.
// The farthest-point key of each new edge is raised in LDS and, at the end,
// in the global slots.  One set (one_set): the block stages the set's child
// edges once (with tab_par it splits the parent edges itself, and block 0
// also publishes the children for the next round and clears the farthest
// keys the round after this one raises) and shares one key table.  Several
// sets: each wave holds the set of a chunk that lies in one set, in its own
// tables, over consecutive chunks of that set, and raises its keys in global
// memory when another set comes; a chunk that spans sets reads the tables
// and raises the keys in global memory.  At the end the waves of a block that
// hold the same set merge their keys and raise them once.
constexpr int REF_PER_LANE = 8;
constexpr int REF_CHUNK = WAVE * REF_PER_LANE;    // 512 entries

__global__ __launch_bounds__(REF_WAVES * WAVE) void k_ref_pass(
    const uint32_t *__restrict__ idx, const uint64_t *__restrict__ keys,
    const uint16_t *__restrict__ edge, const int64_t *__restrict__ cnt_in, int nreg_in, int kg,
    const int64_t *__restrict__ region_size, int64_t mult, const REdge *__restrict__ tab_nxt, int er2,
    unsigned long long *__restrict__ far, uint32_t *__restrict__ idx_out,
    uint64_t *__restrict__ keys_out, uint16_t *__restrict__ edge_out,
    int64_t *__restrict__ cnt_out, int one_set, const float *__restrict__ x,
    const float *__restrict__ y, const REdge *__restrict__ tab_par,
    const unsigned long long *__restrict__ far_par, REdge *__restrict__ tab_out,
    unsigned long long *__restrict__ far_clr) {
    extern __shared__ unsigned long long ref_lds[];
    __shared__ int64_t hsh[REF_WAVES];            // several sets: the set each wave holds at the end
    const int lane = lane_id(), w = threadIdx.x >> 6, tid = threadIdx.x;
    const int tw = one_set ? 0 : w;               // this wave's tables
    unsigned long long *Lv = ref_lds + (size_t)tw * er2 * 4;               // er2 farthest keys
    EdgeF *ltab = reinterpret_cast<EdgeF *>(ref_lds + (size_t)tw * er2 * 4 + er2);  // er2 child edges
    const int64_t g = (int64_t)blockIdx.x * REF_WAVES + w;
    const int64_t ngroups = ((int64_t)nreg_in + kg - 1) / kg;
    const int64_t segcap = *region_size * mult;      // input region size
    const int64_t r0 = g * kg;
    const int nr = (int)max((int64_t)0, min((int64_t)kg, (int64_t)nreg_in - r0));
    // list offsets of the group's regions (pre[j]: entries before region j)
    const int64_t c = lane < nr ? cnt_in[r0 + lane] : 0;
    const int64_t incl = wave_incl_scan_i64(c);
    const int64_t n_sg = uniform_i64(__shfl(incl, WAVE - 1));
    int64_t pre[REF_GROUP];
    pre[0] = 0;
#pragma unroll
    for (int j = 1; j < REF_GROUP; j++) pre[j] = uniform_i64(__shfl(incl, j - 1));
    auto addr = [&](int64_t v) {     // list entry v -> its address
        int64_t a = r0 * segcap + v;
#pragma unroll
        for (int j = 1; j < REF_GROUP; j++)
            if (j < nr && pre[j] <= v) a += segcap - (pre[j] - pre[j - 1]);
        return a;
    };
    uint64_t k[REF_PER_LANE];
    uint16_t st[REF_PER_LANE];
    uint32_t ix[REF_PER_LANE];
    // the chunk at jb: a chunk with no other region start in it is read from
    // one base address (scalar) plus the lane's offset
    auto load_chunk = [&](int64_t jb) {
        int jr = 0;
#pragma unroll
        for (int t = 1; t < REF_GROUP; t++) jr += (t < nr && pre[t] <= jb);
        int64_t pre_jr = 0, pre_nx = n_sg;
#pragma unroll
        for (int t = 0; t < REF_GROUP; t++) {
            if (t == jr) pre_jr = pre[t];
            if (t == jr + 1 && t < nr) pre_nx = pre[t];
        }
        if (pre_nx >= min(n_sg, jb + REF_CHUNK)) {
            const int64_t base = (r0 + jr) * segcap + (jb - pre_jr);
            const int lim = (int)min((int64_t)REF_CHUNK, n_sg - jb);
            const uint64_t *kp = keys + base;
            const uint16_t *ep = edge + base;
            const uint32_t *ip = idx + base;
            if (lim == REF_CHUNK) {
#pragma unroll
                for (int i = 0; i < REF_PER_LANE; i++) {
                    const int j = lane + i * WAVE;
                    k[i] = kp[j];
                    st[i] = ep[j];
                    ix[i] = ip[j];
                }
            } else {
#pragma unroll
                for (int i = 0; i < REF_PER_LANE; i++) {
                    const int j = lane + i * WAVE;
                    const bool in = j < lim;
                    k[i] = in ? kp[j] : 0;
                    st[i] = in ? ep[j] : RE_DROP;
                    ix[i] = in ? ip[j] : 0;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < REF_PER_LANE; i++) {
                const int64_t j = jb + lane + (int64_t)i * WAVE;
                const bool in = j < n_sg;
                const int64_t a = in ? addr(j) : 0;
                k[i] = in ? keys[a] : 0;
                st[i] = in ? edge[a] : RE_DROP;
                ix[i] = in ? idx[a] : 0;
            }
        }
    };
    if (n_sg > 0) load_chunk(0);              // in flight while the tables are staged
    if (!__syncthreads_or(n_sg > 0 ? 1 : 0)) {  // the whole block is empty
        if (lane == 0 && g < ngroups) cnt_out[g] = 0;
        if (!(one_set && tab_par && blockIdx.x == 0)) return;
    }
    if (one_set) {
        for (int e = tid; e < er2; e += REF_WAVES * WAVE) Lv[e] = 0;
        if (tab_par) {
            for (int e = tid; e < er2 / 2; e += REF_WAVES * WAVE) {
                REdge c0, c1;
                split_pair(x, y, tab_par[e], far_par[e], &c0, &c1);
                ltab[2 * e] = edge_f(c0);
                ltab[2 * e + 1] = edge_f(c1);
                if (blockIdx.x == 0) {
                    tab_out[2 * e] = c0;
                    tab_out[2 * e + 1] = c1;
                }
            }
            if (blockIdx.x == 0)
                for (int e = tid; e < RE_CAP; e += REF_WAVES * WAVE) far_clr[e] = 0;
        } else {
            for (int e = tid; e < er2; e += REF_WAVES * WAVE) ltab[e] = edge_f(tab_nxt[e]);
        }
        __syncthreads();
    }
    const int64_t region = r0 * segcap;     // output region g: [region, region + kg * segcap)
    const uint64_t lt = lanemask_lt();
    int64_t outn = 0;                       // entries packed into the region so far
    int64_t held = -1;                      // several sets: the set held in LDS
    auto flush_wave = [&](int64_t fs) {     // the wave's held keys -> global slots
        for (int e = lane; e < er2; e += WAVE) {
            const unsigned long long v = Lv[e];
            if (v) far_update(&far[fs * RE_CAP + e], v);
        }
    };
    for (int64_t jb = 0; jb < n_sg; jb += REF_CHUNK) {
        if (jb > 0) load_chunk(jb);
        bool local = true;
        if (!one_set) {
            // one set in the whole chunk?  (a region can span sets)  Entry jb
            // is lane 0's first.
            const int64_t s0 = (int64_t)(__shfl(k[0], 0) >> 48);
            bool same = true;
#pragma unroll
            for (int i = 0; i < REF_PER_LANE; i++)
                same = same && (jb + lane + (int64_t)i * WAVE >= n_sg || (int64_t)(k[i] >> 48) == s0);
            local = __ballot(!same) == 0;
            if (held >= 0 && (!local || s0 != held)) {
                flush_wave(held);
                held = -1;
                wave_sync();
            }
            if (local && held < 0) {
                for (int e = lane; e < er2; e += WAVE) {
                    Lv[e] = 0;
                    ltab[e] = edge_f(tab_nxt[s0 * RE_CAP + e]);
                }
                held = s0;
                wave_sync();
            }
        }
        // each entry against the two children of its edge, without branches
        // but the farthest-key update: E1 < 0 -> child 2e, else E2 < 0 ->
        // child 2e + 1, else both > 0 -> dropped, else kept unassigned
        auto classify = [&](int i, const EdgeF &f0, const EdgeF &f1, int e0, uint16_t *out_, double *dist_) {
            const double px = (double)(uint32_t)((k[i] >> 24) & 0xFFFFFF);
            const double py = (double)(uint32_t)(k[i] & 0xFFFFFF);
            const double E1 = edge_eval(f0, px, py), E2 = edge_eval(f1, px, py);
            uint16_t out = (E1 > 0 && E2 > 0) ? RE_DROP : RE_NONE;
            double dist = 0.0;
            if (E2 < 0) { out = (uint16_t)(e0 + 1); dist = -E2; }
            if (E1 < 0) { out = (uint16_t)e0; dist = -E1; }
            *out_ = out;
            *dist_ = dist;
        };
        if (__builtin_amdgcn_readfirstlane((int)local)) {
#pragma unroll
            for (int i = 0; i < REF_PER_LANE; i++) {
                const uint16_t s_in = st[i];
                const bool act = s_in < RE_DROP;           // assigned to an edge
                const int e0 = act ? 2 * (int)s_in : 0;
                uint16_t out;
                double dist;
                classify(i, ltab[e0], ltab[e0 + 1], e0, &out, &dist);
                st[i] = act ? out : s_in;
                if (act && out < RE_DROP) atomicMax(&Lv[out], (unsigned long long)far_key(dist, ix[i]));
            }
        } else {
#pragma unroll
            for (int i = 0; i < REF_PER_LANE; i++) {
                const uint16_t s_in = st[i];
                const bool act = s_in < RE_DROP;
                const int e0 = act ? 2 * (int)s_in : 0;
                const int64_t s = (int64_t)(k[i] >> 48);
                uint16_t out;
                double dist;
                classify(i, edge_f(tab_nxt[s * RE_CAP + e0]), edge_f(tab_nxt[s * RE_CAP + e0 + 1]), e0,
                         &out, &dist);
                st[i] = act ? out : s_in;
                if (act && out < RE_DROP) far_update(&far[s * RE_CAP + out], far_key(dist, ix[i]));
            }
        }
        // kept entries packed row by row: every row's stores go to
        // consecutive slots
#pragma unroll
        for (int i = 0; i < REF_PER_LANE; i++) {
            const uint64_t bm = __ballot(st[i] != RE_DROP);
            if (st[i] != RE_DROP) {
                const int pos = __popcll(bm & lt);
                idx_out[region + outn + pos] = ix[i];
                keys_out[region + outn + pos] = k[i];
                edge_out[region + outn + pos] = st[i];
            }
            outn += __popcll(bm);
        }
    }
    if (lane == 0 && g < ngroups) cnt_out[g] = outn;
    // the block's farthest keys -> global slots, once per set
    if (!one_set && lane == 0) hsh[w] = held;
    __syncthreads();
    if (one_set) {
        for (int e = tid; e < er2; e += REF_WAVES * WAVE) {
            const unsigned long long v = Lv[e];
            if (v) far_update(&far[e], v);
        }
        return;
    }
    int first = w;                          // the first wave holding the same set
    if (held >= 0) {
        for (int v = w - 1; v >= 0; v--)
            if (hsh[v] == held) first = v;
        if (first != w) {
            unsigned long long *dst = ref_lds + (size_t)first * er2 * 4;
            for (int e = lane; e < er2; e += WAVE)
                if (Lv[e]) atomicMax(&dst[e], Lv[e]);
        }
    }
    __syncthreads();
    if (held >= 0 && first == w) flush_wave(held);
}

// Regions of list stage r (0: the discard pass's, one per wave; round r
// reads them and writes stage r + 1, one region per group of ref_group(r)).
__host__ __device__ inline int64_t stage_regions(int64_t nwave, int r, bool batched) {
    int64_t n = nwave;
    for (int i = 0; i < r; i++) n = (n + ref_group(i, batched) - 1) / ref_group(i, batched);
    return n;
}

// This thread's share of c[0, n) (thread t: entries t, t + 256, ...), eight
// loads in flight.
__device__ __forceinline__ int64_t sum_counts(const int64_t *__restrict__ c, int64_t n) {
    constexpr int GT = 256, K = 8;
    int64_t a = 0;
    for (int64_t j0 = threadIdx.x; j0 < n; j0 += (int64_t)GT * K) {
        int64_t v[K];
#pragma unroll
        for (int u = 0; u < K; u++) {
            const int64_t j = j0 + (int64_t)u * GT;
            v[u] = j < n ? c[j] : 0;
        }
#pragma unroll
        for (int u = 0; u < K; u++) a += v[u];
    }
    return a;
}

// Region list (idx, keys) of list stage nstage - 1 (region counts of stage r
// at cnt_all + r * nwave) -> contiguous arrays in region order.  Block b
// copies the consecutive regions [b * per, (b + 1) * per), starting at the
// sum of the counts before them, up to 256 regions at a time: their counts
// are scanned into LDS and every thread copies entries of any of them (its
// region by binary search), four in flight.  totals[r] gets the entries of
// stage r for every r < nstage.
__global__ __launch_bounds__(256) void k_seg_gather(const uint32_t *__restrict__ idx,
                                                    const uint64_t *__restrict__ keys,
                                                    const int64_t *__restrict__ cnt_all, int nwave,
                                                    int nstage, int batched,
                                                    const int64_t *__restrict__ region_size,
                                                    int64_t mult,
                                                    uint32_t *__restrict__ idx_out,
                                                    uint64_t *__restrict__ keys_out,
                                                    int64_t *__restrict__ totals) {
    constexpr int GT = 256, GK = 4;
    __shared__ int64_t sh[17];
    __shared__ int64_t roff[GT];
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < nstage) {
        const int64_t *c = cnt_all + (int64_t)blockIdx.x * nwave;
        const int64_t nr = stage_regions(nwave, (int)blockIdx.x, batched);
        const int64_t a = sum_counts(c, nr);
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
    const int64_t acc = sum_counts(cnt, g0);
    int64_t dst;
    block_excl_scan_i64(acc, sh, &dst);
    const int64_t segcap = *region_size * mult;
    for (int64_t b0 = g0; b0 < g1; b0 += GT) {
        const int nb = (int)min((int64_t)GT, g1 - b0);
        const int64_t n = tid < nb ? cnt[b0 + tid] : 0;
        int64_t tot;
        roff[tid] = block_excl_scan_i64(n, sh, &tot);   // ends with a barrier
        __syncthreads();
        for (int64_t i0 = 0; i0 < tot; i0 += (int64_t)GT * GK) {
            uint32_t vi[GK];
            uint64_t vk[GK];
#pragma unroll
            for (int u = 0; u < GK; u++) {
                const int64_t i = i0 + (int64_t)u * GT + tid;
                vi[u] = 0;
                vk[u] = 0;
                if (i < tot) {
                    int lo = 0, hi = nb - 1;       // the last region starting at or before i
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (roff[mid] <= i) lo = mid; else hi = mid - 1;
                    }
                    const int64_t src = (b0 + lo) * segcap + (i - roff[lo]);
                    vi[u] = idx[src];
                    vk[u] = keys[src];
                }
            }
#pragma unroll
            for (int u = 0; u < GK; u++) {
                const int64_t i = i0 + (int64_t)u * GT + tid;
                if (i < tot) {
                    idx_out[dst + i] = vi[u];
                    keys_out[dst + i] = vk[u];
                }
            }
        }
        dst += tot;
        __syncthreads();      // roff is rewritten by the next batch
    }
}

}  // namespace hg
