// Hull of the sorted survivors: Andrew's monotone chain (the paper's
// reference [6], corrected in its erratum), run in parallel.
//
// Keys are set << 48 | kx << 24 | ky, sorted ascending, so each set is a
// contiguous run ordered by (x, y).  Every chain below is segmented by the
// set field: it never joins points of different sets.
//  1. k_chain_chunks: one wave per CHAIN_C consecutive keys computes the
//     lower and the upper chain of its chunk (duplicates dropped; a point
//     goes while it does not make a strict turn, so collinear points go).
//  2. k_chain_merge: one wave per group of CHAIN_G neighbouring chains joins
//     them: at the first level the chains side by side are pruned like a
//     chunk (below); above it they are joined left to right, the tail of the
//     chain built so far and the head of the next one walked to their common
//     tangent (the bridge) at each junction.  Repeated until one chain per
//     kind is left.
//  3. Per set: the lower chain followed by the upper chain's interior in
//     reverse gives the counter-clockwise hull from the lexicographic
//     minimum; each hull key is mapped back to the lowest point index with
//     that key among the candidates.
#include "hg_device.h"

namespace hg {

constexpr int CHAIN_C = 256;
constexpr int CHAIN_G = 32;

__device__ __forceinline__ uint32_t key_set(uint64_t k) { return (uint32_t)(k >> 48); }
__device__ __forceinline__ double key_x(uint64_t k) { return (double)((k >> 24) & 0xFFFFFF); }
__device__ __forceinline__ double key_y(uint64_t k) { return (double)(k & 0xFFFFFF); }

__device__ __forceinline__ double korient(uint64_t o, uint64_t a, uint64_t b) {
    return orient(key_x(o), key_y(o), key_x(a), key_y(a), key_x(b), key_y(b));
}

// Should b be removed when the chain ... a, b is followed by c?
template <bool UPPER>
__device__ __forceinline__ bool drop_mid(uint64_t a, uint64_t b, uint64_t c) {
    double o = korient(a, b, c);
    return UPPER ? (o >= 0) : (o <= 0);
}

// ---------------------------------------------------------------------------
// Level 0: one wave per CHAIN_C consecutive sorted keys (four per lane).
// Along x-sorted points of one set, a vertex of the lower chain on its
// falling part has a smaller y than every earlier point, and on its rising
// part a smaller y than every later point (the first and last points count
// as such).  Mirrored with maxima for the upper chain.  So only strict
// prefix/suffix minima of y can be lower-chain vertices and only strict
// prefix/suffix maxima upper-chain ones; wave-wide scans find both kinds and
// each goes to a list of its own.  A chunk that spans two sets keeps every
// point in both lists.
//
// The lists are then pruned in parallel: a point whose neighbours in its list
// (same set) make it lie on or above (lower chain; below for the upper) the
// segment joining them is no strict vertex of the chain, and removing such
// points, all at once, leaves the chain unchanged; a repeated key goes too.
// A pass that removes nothing leaves an x-monotone list that turns strictly
// the same way at every point, which is a convex chain: the answer.  When the
// passes run out first, lanes 0 and 1 finish with the serial monotone chain.
constexpr uint32_t YMIN_ID = 0x7fffffffu;   // identity of min over y < 2^24
constexpr int32_t YMAX_ID = -1;
constexpr int PRUNE_PASSES = 24;

struct Chain0Lds {
    uint64_t list[2][2][CHAIN_C];   // [lower, upper][ping-pong]
};

__device__ __forceinline__ uint32_t scan_min_up(uint32_t v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t t = __shfl_up(v, o);
        if (l >= o) v = min(v, t);
    }
    return v;
}
__device__ __forceinline__ int32_t scan_max_up(int32_t v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int32_t t = __shfl_up(v, o);
        if (l >= o) v = max(v, t);
    }
    return v;
}
__device__ __forceinline__ uint32_t scan_min_down(uint32_t v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t t = __shfl_down(v, o);
        if (l + o < WAVE) v = min(v, t);
    }
    return v;
}
__device__ __forceinline__ int32_t scan_max_down(int32_t v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int32_t t = __shfl_down(v, o);
        if (l + o < WAVE) v = max(v, t);
    }
    return v;
}

// One pruning pass over src[0..n) into dst; returns the kept count (uniform).
// dst may be src: a round reads its 64 entries and their neighbours before
// it writes, and a kept entry never moves up, so no later read is clobbered.
template <bool UPPER>
__device__ __forceinline__ int prune_pass(const uint64_t *src, uint64_t *dst, int n,
                                          uint64_t lt) {
    const int lane = lane_id();
    int out = 0;
    for (int r = 0; r < n; r += WAVE) {
        const int i = r + lane;
        bool keep = false;
        uint64_t me = 0;
        if (i < n) {
            me = src[i];
            keep = true;
            if (i > 0) {
                const uint64_t pv = src[i - 1];
                if (pv == me) {
                    keep = false;                  // a repeated key
                } else if (i + 1 < n) {
                    const uint64_t nx = src[i + 1];
                    const uint32_t sm = key_set(me);
                    if (nx != me && key_set(pv) == sm && key_set(nx) == sm &&
                        drop_mid<UPPER>(pv, me, nx))
                        keep = false;
                }
            }
        }
        const uint64_t b = __ballot(keep);
        if (keep) dst[out + __popcll(b & lt)] = me;
        out += __popcll(b);
    }
    return out;
}

// Serial monotone chain over st[0..n) in place (the stack never passes the
// read position); resets at set boundaries.
template <bool UPPER>
__device__ int serial_chain(uint64_t *st, int n) {
    int h = 0, seg = 0;
    uint64_t prev = ~uint64_t(0);
    for (int i = 0; i < n; i++) {
        const uint64_t kk = st[i];
        if (kk == prev) continue;
        prev = kk;
        if (h > seg && key_set(st[h - 1]) != key_set(kk)) seg = h;
        while (h - seg >= 2 && drop_mid<UPPER>(st[h - 2], st[h - 1], kk)) h--;
        st[h++] = kk;
    }
    return h;
}

__global__ __launch_bounds__(256) void k_chain_chunks(const uint64_t *__restrict__ keys,
                                                      const int64_t *__restrict__ cnt_ptr,
                                                      uint64_t *__restrict__ lo,
                                                      uint64_t *__restrict__ up,
                                                      uint32_t *__restrict__ lo_cnt,
                                                      uint32_t *__restrict__ up_cnt,
                                                      int *__restrict__ big) {
    __shared__ Chain0Lds lds[4];
    Chain0Lds &L = lds[threadIdx.x >> 6];
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int64_t cnt = *cnt_ptr;
    if (big && blockIdx.x == 0 && threadIdx.x == 0) *big = 0;   // raised by k_chain_sets
    const int64_t U = (cnt + CHAIN_C - 1) / CHAIN_C;
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = (int64_t(gridDim.x) * blockDim.x) >> 6;
    if (U == 0 && wave == 0 && lane == 0) {   // no candidates: the chains are empty
        lo_cnt[0] = 0;
        up_cnt[0] = 0;
    }
    // a fixed grid walks the chunks the count actually has
    for (int64_t j = wave; j < U; j += nw) {
    const int64_t a = j * CHAIN_C, e = min(a + CHAIN_C, cnt);
    uint64_t k[4];
    bool valid[4];
    const int64_t p = a + 4 * lane;
    if (p + 4 <= e) {
        const ulonglong2 *q = reinterpret_cast<const ulonglong2 *>(keys + p);
        ulonglong2 v0 = q[0], v1 = q[1];
        k[0] = v0.x; k[1] = v0.y; k[2] = v1.x; k[3] = v1.y;
#pragma unroll
        for (int i = 0; i < 4; i++) valid[i] = true;
    } else {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            valid[i] = p + i < e;
            k[i] = valid[i] ? keys[p + i] : 0;
        }
    }
    const bool multi = key_set(keys[a]) != key_set(keys[e - 1]);
    uint32_t ymin[4];
    int32_t ymax[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t yy = (uint32_t)(k[i] & 0xFFFFFF);
        ymin[i] = valid[i] ? yy : YMIN_ID;
        ymax[i] = valid[i] ? (int32_t)yy : YMAX_ID;
    }
    const uint32_t lmin = min(min(ymin[0], ymin[1]), min(ymin[2], ymin[3]));
    const int32_t lmax = max(max(ymax[0], ymax[1]), max(ymax[2], ymax[3]));
    uint32_t pmin = __shfl_up(scan_min_up(lmin), 1);
    int32_t pmax = __shfl_up(scan_max_up(lmax), 1);
    uint32_t smin = __shfl_down(scan_min_down(lmin), 1);
    int32_t smax = __shfl_down(scan_max_down(lmax), 1);
    if (lane == 0) { pmin = YMIN_ID; pmax = YMAX_ID; }
    if (lane == WAVE - 1) { smin = YMIN_ID; smax = YMAX_ID; }
    bool cl[4], cu[4];
    {
        uint32_t rmin = pmin;
        int32_t rmax = pmax;
#pragma unroll
        for (int i = 0; i < 4; i++) {            // strict prefix records
            cl[i] = valid[i] && (multi || ymin[i] < rmin);
            cu[i] = valid[i] && (multi || ymax[i] > rmax);
            rmin = min(rmin, ymin[i]);
            rmax = max(rmax, ymax[i]);
        }
        rmin = smin;
        rmax = smax;
#pragma unroll
        for (int i = 3; i >= 0; i--) {           // strict suffix records
            cl[i] = cl[i] || (valid[i] && ymin[i] < rmin);
            cu[i] = cu[i] || (valid[i] && ymax[i] > rmax);
            rmin = min(rmin, ymin[i]);
            rmax = max(rmax, ymax[i]);
        }
    }
    // compact both lists in key order: (lane, item)
    int pl = 0, pu = 0, nl = 0, nu = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const uint64_t bl = __ballot(cl[i]), bu = __ballot(cu[i]);
        pl += __popcll(bl & lt);
        nl += __popcll(bl);
        pu += __popcll(bu & lt);
        nu += __popcll(bu);
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if (cl[i]) L.list[0][0][pl++] = k[i];
        if (cu[i]) L.list[1][0][pu++] = k[i];
    }
    wave_sync();
    int cur = 0, pass = 0;
    bool moved = true;
    for (; moved && pass < PRUNE_PASSES; pass++) {
        const int ml = prune_pass<false>(L.list[0][cur], L.list[0][1 - cur], nl, lt);
        const int mu = prune_pass<true>(L.list[1][cur], L.list[1][1 - cur], nu, lt);
        moved = ml != nl || mu != nu;
        nl = ml;
        nu = mu;
        cur = 1 - cur;
        wave_sync();
    }
    if (moved) {      // passes ran out: finish serially (lane 0 lower, lane 1 upper)
        int h = 0;
        if (lane == 0) h = serial_chain<false>(L.list[0][cur], nl);
        if (lane == 1) h = serial_chain<true>(L.list[1][cur], nu);
        wave_sync();
        nl = __builtin_amdgcn_readlane(h, 0);
        nu = __builtin_amdgcn_readlane(h, 1);
    }
    for (int i = lane; i < nl; i += WAVE) lo[a + i] = L.list[0][cur][i];
    for (int i = lane; i < nu; i += WAVE) up[a + i] = L.list[1][cur][i];
    if (lane == 0) {
        lo_cnt[j] = (uint32_t)nl;
        up_cnt[j] = (uint32_t)nu;
    }
    wave_sync();       // the next chunk reuses the wave's LDS
    }
}

// Index of the first element of src[lo..hi) whose set equals set(src[hi-1]).
template <typename P>
__device__ __forceinline__ int64_t last_seg_start(P src, int64_t lo, int64_t hi) {
    uint32_t s = key_set(src[hi - 1]);
    while (lo < hi - 1) {
        int64_t mid = (lo + hi - 1) >> 1;
        if (key_set(src[mid]) == s) hi = mid + 1; else lo = mid + 1;
    }
    return lo;
}

// Walk the junction of the chain built so far (o[0..len), its last set
// segment starting at tailseg) with the next chain c[0..m) to their common
// tangent.  Returns the new length of o and sets *bstart to the first
// element of c to append.
template <bool UPPER, typename PO, typename PC>
__device__ __forceinline__ int64_t bridge(PO o, int64_t len, int64_t tailseg, PC c, int64_t m,
                                          int64_t *bstart) {
    int64_t b = 0;
    if (len > 0) {
        uint64_t last = o[len - 1];
        if (c[0] == last) b = 1;
        if (b < m && key_set(last) == key_set(c[b])) {
            int64_t a = len - 1;
            bool changed = true;
            while (changed) {
                changed = false;
                while (a > tailseg && drop_mid<UPPER>(o[a - 1], o[a], c[b])) {
                    a--;
                    changed = true;
                }
                while (b + 1 < m && key_set(c[b + 1]) == key_set(c[b]) &&
                       drop_mid<UPPER>(o[a], c[b], c[b + 1])) {
                    b++;
                    changed = true;
                }
            }
            len = a + 1;
        }
    }
    *bstart = b;
    return len;
}

// Merge of CHAIN_G neighbouring chains by one wave.  Groups that fit are
// staged in LDS: at level 0 (many short chains) pruned in parallel (serial
// chain only when the passes run out), above it (few long chains) joined by
// serial bridge walks; larger groups walk the bridges in global memory.
constexpr int MERGE_CAP = 4096;           // keys staged per wave (32 KB)

// The group's ng chains side by side in buf (chain g of length m_g from
// in + (u0 + g) R to buf[off_g, off_g + m_g), off_g the sum of the lengths
// before it; lane g < ng holds incl = off_g + m_g, M the total).  Every lane
// loads entries of any chain (its chain by binary search over the offsets in
// goff), eight in flight, so the loads of all the chains overlap.
__device__ __forceinline__ void stage_group(const uint64_t *__restrict__ in, int64_t R, int64_t u0,
                                            int ng, int64_t incl, int64_t M, int64_t *goff,
                                            uint64_t *buf) {
    constexpr int K = 8;
    const int lane = lane_id();
    if (lane < ng) goff[lane + 1] = incl;
    if (lane == 0) goff[0] = 0;
    wave_sync();
    for (int64_t i0 = 0; i0 < M; i0 += (int64_t)K * WAVE) {
        uint64_t v[K];
#pragma unroll
        for (int u = 0; u < K; u++) {
            const int64_t i = i0 + (int64_t)u * WAVE + lane;
            v[u] = 0;
            if (i < M) {
                int lo = 0, hi = ng - 1;       // the last chain starting at or before i
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (goff[mid] <= i) lo = mid; else hi = mid - 1;
                }
                v[u] = in[(u0 + lo) * R + (i - goff[lo])];
            }
        }
#pragma unroll
        for (int u = 0; u < K; u++) {
            const int64_t i = i0 + (int64_t)u * WAVE + lane;
            if (i < M) buf[i] = v[u];
        }
    }
    wave_sync();
}

// The junctions of the staged chains walked at once, one lane per junction
// (chain A, then the next non-empty chain B): the same retreat along A's
// tail and advance along B's head as the left-to-right join, except that
// the retreat stops at the start of A's last set segment within A.  Chain i
// keeps [lo_i, hi_i] (lo from its left junction, hi from its right one).
// When every walk stays inside its own two chains, which holds when no chain
// whose both junctions were walked is left with fewer than two points and
// none is consumed, the joined chain is these pieces in order, the same as
// the left-to-right join's, and it is written to o; otherwise returns false
// (nothing written) and the caller joins left to right.
template <bool UPPER>
__device__ bool parallel_join(const uint64_t *__restrict__ buf, const int64_t *__restrict__ goff,
                              int ng, int64_t mine, uint64_t *__restrict__ o, int64_t *len_out,
                              int *__restrict__ ne, int64_t *__restrict__ pref,
                              int64_t *__restrict__ src) {
    const int lane = lane_id();
    wave_sync();
    const uint64_t nz = __ballot(lane < ng && mine > 0);
    const int nn = __popcll(nz);
    if (lane < ng && mine > 0) ne[__popcll(nz & lanemask_lt())] = lane;
    wave_sync();
    int64_t aj = 0, bj = 0;
    int walked = 0;
    if (lane < nn - 1) {
        const int ga = ne[lane], gb = ne[lane + 1];
        const uint64_t *A = buf + goff[ga], *B = buf + goff[gb];
        const int64_t ma = goff[ga + 1] - goff[ga], mb = goff[gb + 1] - goff[gb];
        const uint64_t last = A[ma - 1];
        int64_t a = ma - 1, b = B[0] == last ? 1 : 0;
        if (b < mb && key_set(last) == key_set(B[b])) {
            const int64_t ls = last_seg_start(A, 0, ma);
            bool changed = true;
            while (changed) {
                changed = false;
                while (a > ls && drop_mid<UPPER>(A[a - 1], A[a], B[b])) {
                    a--;
                    changed = true;
                }
                while (b + 1 < mb && key_set(B[b + 1]) == key_set(B[b]) &&
                       drop_mid<UPPER>(A[a], B[b], B[b + 1])) {
                    b++;
                    changed = true;
                }
            }
            walked = 1;
        }
        aj = a;
        bj = b;
    }
    const int64_t bl = __shfl_up(bj, 1);
    const int wl_ = __shfl_up(walked, 1);
    const bool wl = lane >= 1 && wl_;
    const int gi = lane < nn ? ne[lane] : 0;
    const int64_t mi = lane < nn ? goff[gi + 1] - goff[gi] : 0;
    const int64_t lo = lane >= 1 && lane < nn ? bl : 0;
    const int64_t hi = lane < nn - 1 ? aj : mi - 1;
    const bool wr = lane < nn - 1 && walked;
    const bool bad = lane < nn && (lo > hi || (wl && wr && lo == hi));
    if (__ballot(bad)) return false;
    const int64_t cnt = lane < nn ? hi - lo + 1 : 0;
    const int64_t inc = wave_incl_scan_i64(cnt);
    const int64_t total = __shfl(inc, WAVE - 1);
    if (lane < nn) {
        pref[lane] = inc - cnt;
        src[lane] = goff[gi] + lo - (inc - cnt);
    }
    wave_sync();
    for (int64_t i = lane; i < total; i += WAVE) {
        int l = 0, h = nn - 1;          // the last piece starting at or before i
        while (l < h) {
            const int mid = (l + h + 1) >> 1;
            if (pref[mid] <= i) l = mid; else h = mid - 1;
        }
        o[i] = buf[src[l] + i];
    }
    *len_out = total;
    return true;
}

template <bool UPPER>
__device__ void merge_group(const uint64_t *__restrict__ in, const uint32_t *__restrict__ cin,
                            int64_t U, int64_t R, int64_t v, int lev, uint64_t *__restrict__ out,
                            uint32_t *__restrict__ cout, uint64_t *__restrict__ buf,
                            int64_t *__restrict__ goff, int *__restrict__ ne,
                            int64_t *__restrict__ pref, int64_t *__restrict__ psrc) {
    const int lane = lane_id();
    const int64_t base = v * R * CHAIN_G;
    uint64_t *o = out + base;
    // chain sizes of the group and their offsets
    const int64_t u0 = v * CHAIN_G;
    int64_t mine = (lane < CHAIN_G && u0 + lane < U) ? (int64_t)cin[u0 + lane] : 0;
    int64_t incl = wave_incl_scan_i64(mine);
    const int64_t M = __shfl(incl, WAVE - 1);
    int64_t len = 0, tailseg = 0;
    const int nonempty = __popcll(__ballot(mine > 0));
    if (nonempty <= 1) {     // one chain: copied as it is
        for (int g = 0; g < CHAIN_G && u0 + g < U; g++) {
            const int64_t m = __shfl(mine, g);
            const uint64_t *src = in + (u0 + g) * R;
            for (int64_t i = lane; i < m; i += WAVE) o[i] = src[i];
        }
        len = M;
    } else if (M <= MERGE_CAP && lev > 0) {
        // a few long chains (the upper levels): joined left to right in LDS,
        // walking each junction to its bridge
        stage_group(in, R, u0, (int)min((int64_t)CHAIN_G, U - u0), incl, M, goff, buf);
        if (!parallel_join<UPPER>(buf, goff, (int)min((int64_t)CHAIN_G, U - u0), mine, o, &len, ne, pref,
                                  psrc)) {
            for (int g = 0; g < CHAIN_G && u0 + g < U; g++) {
                const int64_t m = __shfl(mine, g), og = __shfl(incl, g) - m;
                if (m == 0) continue;
                const uint64_t *c = buf + og;
                int64_t b;
                len = bridge<UPPER>(buf, len, tailseg, c, m, &b);
                if (b < m) {
                    int64_t ls = last_seg_start(c, b, m);
                    int64_t newtail;
                    if (ls > b) newtail = len + (ls - b);
                    else newtail = (len > 0 && key_set(buf[len - 1]) == key_set(c[b])) ? tailseg : len;
                    // move c[b..m) down to buf[len..): len <= og + b, copy forward
                    for (int64_t i0 = 0; i0 < m - b; i0 += WAVE) {
                        int64_t i = i0 + lane;
                        uint64_t val = i < m - b ? c[b + i] : 0;
                        wave_sync();
                        if (i < m - b) buf[len + i] = val;
                        wave_sync();
                    }
                    len += m - b;
                    tailseg = newtail;
                }
            }
            for (int64_t i = lane; i < len; i += WAVE) o[i] = buf[i];
        }
    } else if (M <= MERGE_CAP) {
        // level 0: many short chains side by side form one x-sorted list
        // holding every vertex of the merged chain: prune it in place like a
        // level-0 chunk
        stage_group(in, R, u0, (int)min((int64_t)CHAIN_G, U - u0), incl, M, goff, buf);
        const uint64_t lt = lanemask_lt();
        int n = (int)M;
        bool moved = true;
        for (int pass = 0; moved && pass < PRUNE_PASSES; pass++) {
            const int m2 = prune_pass<UPPER>(buf, buf, n, lt);
            moved = m2 != n;
            n = m2;
            wave_sync();
        }
        if (moved) {      // passes ran out: finish serially
            int h = 0;
            if (lane == 0) h = serial_chain<UPPER>(buf, n);
            wave_sync();
            n = __builtin_amdgcn_readlane(h, 0);
        }
        len = n;
        for (int64_t i = lane; i < len; i += WAVE) o[i] = buf[i];
    } else {
        for (int g = 0; g < CHAIN_G && u0 + g < U; g++) {
            const int64_t m = __shfl(mine, g);
            if (m == 0) continue;
            const uint64_t *src = in + (u0 + g) * R;
            int64_t b;
            len = bridge<UPPER>(o, len, tailseg, src, m, &b);
            if (b < m) {
                int64_t ls = last_seg_start(src, b, m);
                int64_t newtail;
                if (ls > b) newtail = len + (ls - b);
                else newtail = (len > 0 && key_set(o[len - 1]) == key_set(src[b])) ? tailseg : len;
                wave_sync();
                for (int64_t i = b + lane; i < m; i += WAVE) o[len + (i - b)] = src[i];
                __threadfence_block();
                wave_sync();
                len += m - b;
                tailseg = newtail;
            }
        }
    }
    if (lane == 0) cout[v] = (uint32_t)len;
}

// Copy n keys src -> dst (disjoint) with the whole block, four loads in
// flight per thread.
__device__ __forceinline__ void block_copy(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst,
                                           int64_t n) {
    constexpr int K = 4;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int64_t i0 = 0; i0 < n; i0 += (int64_t)nt * K) {
        uint64_t v[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int64_t i = i0 + (int64_t)k * nt + tid;
            v[k] = i < n ? src[i] : 0;
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int64_t i = i0 + (int64_t)k * nt + tid;
            if (i < n) dst[i] = v[k];
        }
    }
}

// A group too large for one wave's LDS stage (or a single long chain), by
// the whole block: thread 0 walks each junction to its bridge in global
// memory, then every thread copies the next chain's remainder.
// sh: 3 + 2 * CHAIN_G int64 of LDS.
template <bool UPPER>
__device__ void merge_group_block(const uint64_t *__restrict__ in, const uint32_t *__restrict__ cin,
                                  int64_t U, int64_t R, int64_t v, uint64_t *__restrict__ out,
                                  uint32_t *__restrict__ cout, int64_t *sh) {
    const int64_t base = v * R * CHAIN_G;
    uint64_t *o = out + base;
    const int64_t u0 = v * CHAIN_G;
    int64_t *gm = sh + 3, *gls = sh + 3 + CHAIN_G;
    // each chain's length and the start of its last set segment, in parallel
    // (the start within [b, m) is max(b, that)); the barrier keeps these
    // from being overwritten while the previous group still reads them
    __syncthreads();
    if (threadIdx.x < CHAIN_G) {
        const int g = threadIdx.x;
        const int64_t m = u0 + g < U ? (int64_t)cin[u0 + g] : 0;
        gm[g] = m;
        gls[g] = m > 0 ? last_seg_start(in + (u0 + g) * R, 0, m) : 0;
    }
    __syncthreads();
    int64_t len = 0, tailseg = 0;
    for (int g = 0; g < CHAIN_G && u0 + g < U; g++) {
        const int64_t m = gm[g];
        if (m == 0) continue;
        const uint64_t *src = in + (u0 + g) * R;
        if (threadIdx.x == 0) {
            int64_t b;
            const int64_t nl = bridge<UPPER>(o, len, tailseg, src, m, &b);
            int64_t nt = tailseg;
            if (b < m) {
                const int64_t ls = max(b, gls[g]);
                if (ls > b) nt = nl + (ls - b);
                else nt = (nl > 0 && key_set(o[nl - 1]) == key_set(src[b])) ? tailseg : nl;
            }
            sh[0] = nl;
            sh[1] = b;
            sh[2] = nt;
        }
        __syncthreads();
        const int64_t nl = sh[0], b = sh[1], nt = sh[2];
        if (b < m) {
            block_copy(src + b, o + nl, m - b);
            len = nl + (m - b);
            tailseg = nt;
        } else {
            len = nl;
        }
        __threadfence_block();
        __syncthreads();     // sh and the copied keys are read by the next junction
    }
    if (threadIdx.x == 0) cout[v] = (uint32_t)len;
}

// Groups that go to the block form: more keys than a wave stages, or one
// long chain to move.
constexpr int64_t BLOCK_COPY_MIN = 2048;

__device__ __forceinline__ bool block_group(const uint32_t *__restrict__ cin, int64_t U, int64_t v) {
    const int lane = lane_id();
    const int64_t u0 = v * CHAIN_G;
    const int64_t mine = (lane < CHAIN_G && u0 + lane < U) ? (int64_t)cin[u0 + lane] : 0;
    int64_t tot = mine;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) tot += __shfl_xor(tot, o);
    const int nonempty = __popcll(__ballot(mine > 0));
    return tot > MERGE_CAP || (nonempty <= 1 && tot > BLOCK_COPY_MIN);
}

__global__ __launch_bounds__(256) void k_chain_merge(const uint64_t *__restrict__ lo_in,
                                                     const uint64_t *__restrict__ up_in,
                                                     const uint32_t *__restrict__ lo_cin,
                                                     const uint32_t *__restrict__ up_cin,
                                                     const int64_t *__restrict__ cnt_ptr, int lev,
                                                     int nlev,
                                                     uint64_t *__restrict__ lo_out,
                                                     uint64_t *__restrict__ up_out,
                                                     uint32_t *__restrict__ lo_cout,
                                                     uint32_t *__restrict__ up_cout,
                                                     const int *__restrict__ big) {
    __shared__ uint64_t mbuf[4][MERGE_CAP];
    if (big && *big == 0) return;      // several sets, all merged per set already
    const int64_t cnt = *cnt_ptr;
    int64_t R = CHAIN_C;
    int first1 = -1;                                      // first level with at most one chain
    for (int l = 0; l < lev; l++) {
        if (first1 < 0 && (cnt + R - 1) / R <= 1) first1 = l;
        R *= CHAIN_G;
    }
    const int64_t U = (cnt + R - 1) / R;                  // chains at this level
    if (first1 < 0 && U <= 1) first1 = lev;
    // Levels that merge (U > 1) are 0 .. first1 - 1 and alternate the two
    // buffers from the first.  After them the single chain stays where the
    // last one left it, in the buffer of parity first1; only the last level
    // moves it into this level's output buffer, and only if it is not there
    // yet (and records an empty chain when there are no candidates).
    if (U <= 1 && (lev != nlev - 1 || (U == 1 && (first1 & 1) != (lev & 1)))) return;
    const int64_t V = (U + CHAIN_G - 1) / CHAIN_G;        // groups
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = (int64_t(gridDim.x) * blockDim.x) >> 6;
    if (V == 0 && wave == 0 && threadIdx.x == 0)   // no candidates: empty top chain
        (blockIdx.y == 0 ? lo_cout : up_cout)[0] = 0;
    __shared__ int64_t moff[4][CHAIN_G + 1], mpre[4][CHAIN_G], msrc[4][CHAIN_G];
    __shared__ int mne[4][CHAIN_G];
    uint64_t *buf = mbuf[threadIdx.x >> 6];
    int64_t *goff = moff[threadIdx.x >> 6];
    const uint32_t *cin = blockIdx.y == 0 ? lo_cin : up_cin;
    for (int64_t v = wave; v < V; v += nw) {        // groups the count actually has
        if (block_group(cin, U, v)) continue;
        const int wv = threadIdx.x >> 6;
        if (blockIdx.y == 0)
            merge_group<false>(lo_in, lo_cin, U, R, v, lev, lo_out, lo_cout, buf, goff, mne[wv], mpre[wv], msrc[wv]);
        else
            merge_group<true>(up_in, up_cin, U, R, v, lev, up_out, up_cout, buf, goff, mne[wv], mpre[wv], msrc[wv]);
        wave_sync();
    }
    __shared__ int64_t sh[3 + 2 * CHAIN_G];
    __syncthreads();
    for (int64_t v = blockIdx.x; v < V; v += gridDim.x) {
        if (!block_group(cin, U, v)) continue;     // uniform over the block
        if (blockIdx.y == 0) merge_group_block<false>(lo_in, lo_cin, U, R, v, lo_out, lo_cout, sh);
        else merge_group_block<true>(up_in, up_cin, U, R, v, up_out, up_cout, sh);
    }
}

// Several sets: after the chunk chains, each set's keys are one range
// [start, end) of the sorted keys and its chain is merged from the pieces
// the chunks covering that range hold, by one wave, independently of the
// other sets.  The set's chain goes to out[start, start + len) and the rest
// of its range is filled with SET_GAP keys (set field beyond every set), so
// that out[0, cnt) lists every set's chain in set order.  Pieces are joined
// left to right at their bridges (staged in LDS when the range fits).
constexpr uint64_t SET_GAP = ~0ull;

// First index i in sorted[0, n) with set(sorted[i]) >= s.
__device__ __forceinline__ int64_t set_lower_bound(const uint64_t *__restrict__ sorted, int64_t n, uint32_t s) {
    int64_t a = 0, b = n;
    while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (key_set(sorted[m]) < s) a = m + 1; else b = m;
    }
    return a;
}

// [p0, p1) of set s in a chunk list (sorted by key, so by set).
__device__ __forceinline__ void piece_of(const uint64_t *list, int64_t m, uint32_t s, int64_t *p0, int64_t *p1) {
    int64_t a = 0, b = m;
    while (a < b) {
        const int64_t h = (a + b) >> 1;
        if (key_set(list[h]) < s) a = h + 1; else b = h;
    }
    int64_t c = a, d = m;
    while (c < d) {
        const int64_t h = (c + d) >> 1;
        if (key_set(list[h]) <= s) c = h + 1; else d = h;
    }
    *p0 = a;
    *p1 = c;
}

// A set spanning more chunks is not merged here: it raises *big, and the
// hierarchical merge of all chains (k_chain_merge) then runs and replaces
// this output.
constexpr int64_t SET_CHUNKS_MAX = 32;

template <bool UPPER>
__device__ void set_chain(const uint64_t *__restrict__ sorted, int64_t n, uint32_t s,
                          const int64_t *__restrict__ starts,
                          const uint64_t *__restrict__ lists, const uint32_t *__restrict__ lcnt,
                          uint64_t *__restrict__ out, uint64_t *__restrict__ buf,
                          int64_t *__restrict__ goff, int64_t *__restrict__ gsrc, int *__restrict__ big) {
    const int lane = lane_id();
    const int64_t start = starts ? starts[s] : set_lower_bound(sorted, n, s);
    const int64_t end = starts ? starts[s + 1] : set_lower_bound(sorted, n, s + 1);
    if (start >= end) return;
    const int64_t c0 = start / CHAIN_C, c1 = (end - 1) / CHAIN_C;
    if (c1 - c0 + 1 > SET_CHUNKS_MAX) {     // too many pieces for one wave
        if (lane == 0) atomicOr(big, 1);
        return;
    }
    uint64_t *dst = out + start;
    int64_t len = 0;
    if (end - start <= MERGE_CAP) {
        // staged: lane j finds the set's piece of chunk c0 + j, the pieces
        // are loaded side by side into LDS together, then joined left to
        // right at their bridges in place
        const int nc = (int)(c1 - c0 + 1);
        int64_t p0 = 0, p1 = 0;
        if (lane < nc) piece_of(lists + (c0 + lane) * CHAIN_C, (int64_t)lcnt[c0 + lane], s, &p0, &p1);
        const int64_t m = p1 - p0;
        const int64_t incl = wave_incl_scan_i64(m);
        const int64_t M = __shfl(incl, WAVE - 1);
        if (lane < nc) gsrc[lane] = (c0 + lane) * CHAIN_C + p0 - (incl - m);   // list address - buffer offset
        if (lane < nc) goff[lane + 1] = incl;
        if (lane == 0) goff[0] = 0;
        wave_sync();
        for (int64_t i = lane; i < M; i += WAVE) {
            int lo = 0, hi = nc - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (goff[mid] <= i) lo = mid; else hi = mid - 1;
            }
            buf[i] = lists[gsrc[lo] + i];
        }
        wave_sync();
        for (int j = 0; j < nc; j++) {
            const int64_t mj = __shfl(m, j), oj = __shfl(incl, j) - mj;
            if (mj <= 0) continue;
            const uint64_t *c = buf + oj;
            int64_t b;
            len = bridge<UPPER>(buf, len, 0, c, mj, &b);
            // move c[b..mj) down to buf[len..): len <= oj + b, copy forward
            for (int64_t i0 = 0; i0 < mj - b; i0 += WAVE) {
                const int64_t i = i0 + lane;
                const uint64_t val = i < mj - b ? c[b + i] : 0;
                wave_sync();
                if (i < mj - b) buf[len + i] = val;
                wave_sync();
            }
            len += mj - b;
        }
        for (int64_t i = lane; i < len; i += WAVE) dst[i] = buf[i];
    } else {
        for (int64_t c = c0; c <= c1; c++) {
            const uint64_t *list = lists + c * CHAIN_C;
            int64_t p0, p1;
            piece_of(list, (int64_t)lcnt[c], s, &p0, &p1);
            const int64_t m = p1 - p0;
            if (m <= 0) continue;
            const uint64_t *src = list + p0;
            int64_t b;
            len = bridge<UPPER>(dst, len, 0, src, m, &b);
            wave_sync();
            for (int64_t i = b + lane; i < m; i += WAVE) dst[len + (i - b)] = src[i];
            __threadfence_block();
            wave_sync();
            len += m - b;
        }
    }
    for (int64_t i = len + lane; i < end - start; i += WAVE) dst[i] = SET_GAP;
    wave_sync();
}

__global__ __launch_bounds__(256) void k_chain_sets(const uint64_t *__restrict__ sorted,
                                                    const int64_t *__restrict__ cnt_ptr, int64_t S,
                                                    const uint64_t *__restrict__ lo_in,
                                                    const uint64_t *__restrict__ up_in,
                                                    const uint32_t *__restrict__ lo_cin,
                                                    const uint32_t *__restrict__ up_cin,
                                                    uint64_t *__restrict__ lo_out, uint64_t *__restrict__ up_out,
                                                    uint32_t *__restrict__ lo_len, uint32_t *__restrict__ up_len,
                                                    int *__restrict__ big,
                                                    const int64_t *__restrict__ set_starts,
                                                    const int *__restrict__ seg_flag) {
    __shared__ uint64_t mbuf[4][MERGE_CAP];
    __shared__ int64_t moff[4][SET_CHUNKS_MAX + 1], msrc[4][SET_CHUNKS_MAX];
    const int64_t n = *cnt_ptr;
    if (blockIdx.x == 0 && threadIdx.x == 0) (blockIdx.y == 0 ? lo_len : up_len)[0] = (uint32_t)n;
    uint64_t *buf = mbuf[threadIdx.x >> 6];
    int64_t *goff = moff[threadIdx.x >> 6], *gsrc = msrc[threadIdx.x >> 6];
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = (int64_t(gridDim.x) * blockDim.x) >> 6;
    // the sets' ranges from the sort's set starts when the keys came in set
    // order, else by binary search in the sorted keys
    const int64_t *starts = set_starts && (*seg_flag & SEG_UNORDERED) == 0 ? set_starts : nullptr;
    for (int64_t s = wave; s < S; s += nw) {
        if (blockIdx.y == 0)
            set_chain<false>(sorted, n, (uint32_t)s, starts, lo_in, lo_cin, lo_out, buf, goff, gsrc, big);
        else
            set_chain<true>(sorted, n, (uint32_t)s, starts, up_in, up_cin, up_out, buf, goff, gsrc, big);
    }
}

// Fill helpers (kernels, so that graph capture records no memset node).
__global__ void k_fill_i64(int64_t *__restrict__ p, int64_t n, int64_t v) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// Per-set [start, end) of the final lower (kind 0) and upper (kind 1) chains.
__global__ __launch_bounds__(256) void k_seg_bounds(const uint64_t *__restrict__ lo,
                                                    const uint64_t *__restrict__ up,
                                                    const uint32_t *__restrict__ lo_len,
                                                    const uint32_t *__restrict__ up_len,
                                                    int64_t *__restrict__ bounds /*[4][S]*/,
                                                    int64_t S) {
    const uint64_t *c = blockIdx.y == 0 ? lo : up;
    const int64_t n = blockIdx.y == 0 ? lo_len[0] : up_len[0];
    int64_t *st = bounds + (blockIdx.y * 2) * S, *en = bounds + (blockIdx.y * 2 + 1) * S;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        uint32_t s = key_set(c[i]);
        if (s >= S) continue;
        if (i == 0 || key_set(c[i - 1]) != s) st[s] = i;
        if (i == n - 1 || key_set(c[i + 1]) != s) en[s] = i + 1;
    }
}


// Number of keys in sorted c[lo..hi) that are < k.
__device__ __forceinline__ int64_t count_less(const uint64_t *__restrict__ c, int64_t lo, int64_t hi,
                                              uint64_t k) {
    int64_t a = lo, b = hi;
    while (a < b) {
        int64_t m = (a + b) >> 1;
        if (c[m] < k) a = m + 1; else b = m;
    }
    return a - lo;
}

// Lay out one chain entry k = c[i] of its set's hull (lower chain [ls, le),
// upper [us, ue), output [o, o + h)): its CCW position, a key-sorted copy
// (hkeys, hpos) for the index lookup, and its output slot preset to
// HULL_NONE.
__device__ __forceinline__ void emit_entry(bool upper, int64_t i, uint64_t k, int64_t ls,
                                           int64_t le, int64_t us, int64_t ue, int64_t o,
                                           int64_t h, const uint64_t *__restrict__ lo,
                                           const uint64_t *__restrict__ up,
                                           uint64_t *__restrict__ hkeys,
                                           uint32_t *__restrict__ hpos,
                                           uint32_t *__restrict__ hull) {
    const int64_t hl = le - ls, hu = ue - us;
    int64_t pos, rank;
    if (!upper) {
        int64_t r = i - ls;
        if (hl == 1) {
            pos = 0;
            rank = 0;
        } else {
            pos = r;
            rank = r + (hu > 2 ? count_less(up, us + 1, ue - 1, k) : 0);
        }
    } else {
        int64_t r = i - us;
        if (hl <= 1 || r == 0 || r == hu - 1) return;   // shared ends
        pos = hl + (hu - 2 - r);
        rank = (r - 1) + count_less(lo, ls, le, k);
    }
    if (pos >= h || rank >= h) return;   // inconsistent chains: never write outside
    hkeys[o + rank] = k;
    hpos[o + rank] = (uint32_t)pos;
    hull[o + pos] = NONE;
}

// Hull size from the chain lengths: lower + upper - 2 shared ends; one
// point -> 1.
__device__ __forceinline__ int64_t hull_size(int64_t hl, int64_t hu) {
    return hl == 0 ? 0 : (hl == 1 ? 1 : hl + hu - 2);
}

// Hull size per set.
__global__ void k_hull_counts(const int64_t *__restrict__ bounds, int64_t S,
                              uint32_t *__restrict__ hcnt) {
    int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= S) return;
    hcnt[s] = (uint32_t)hull_size(bounds[S + s] - bounds[s], bounds[3 * S + s] - bounds[2 * S + s]);
}

__global__ __launch_bounds__(256) void k_hull_emit(const uint64_t *__restrict__ lo,
                                                   const uint64_t *__restrict__ up,
                                                   const uint32_t *__restrict__ lo_len,
                                                   const uint32_t *__restrict__ up_len,
                                                   const int64_t *__restrict__ bounds, int64_t S,
                                                   const int64_t *__restrict__ hoff,
                                                   uint64_t *__restrict__ hkeys,
                                                   uint32_t *__restrict__ hpos,
                                                   uint32_t *__restrict__ hull) {
    const bool upper = blockIdx.y == 1;
    const uint64_t *c = upper ? up : lo;
    const int64_t n = upper ? up_len[0] : lo_len[0];
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        uint64_t k = c[i];
        uint32_t s = key_set(k);
        if (s >= S) continue;
        const int64_t o = hoff[s];
        emit_entry(upper, i, k, bounds[s], bounds[S + s], bounds[2 * S + s], bounds[3 * S + s],
                   o, hoff[s + 1] - o, lo, up, hkeys, hpos, hull);
    }
}

// One set: offsets, hull size (also to *h_out when given) and layout in one
// block (the chains hold set 0 only).
__global__ __launch_bounds__(1024) void k_hull_final1(const uint64_t *__restrict__ lo,
                                                      const uint64_t *__restrict__ up,
                                                      const uint32_t *__restrict__ lo_len,
                                                      const uint32_t *__restrict__ up_len,
                                                      int64_t *__restrict__ hoff,
                                                      uint64_t *__restrict__ hkeys,
                                                      uint32_t *__restrict__ hpos,
                                                      uint32_t *__restrict__ hull,
                                                      int64_t *__restrict__ h_out) {
    const int64_t le = lo_len[0], ue = up_len[0];
    const int64_t h = hull_size(le, ue);
    if (threadIdx.x == 0) {
        hoff[0] = 0;
        hoff[1] = h;
        if (h_out) *h_out = h;
    }
    for (int64_t i = threadIdx.x; i < le + ue; i += blockDim.x) {
        const bool upper = i >= le;
        const int64_t j = upper ? i - le : i;
        emit_entry(upper, j, upper ? up[j] : lo[j], 0, le, 0, ue, 0, h, lo, up, hkeys, hpos, hull);
    }
}

// Map hull keys back to point indices: every candidate (index, key) whose key
// is a hull vertex of its set lowers that vertex's slot to its index.
__global__ __launch_bounds__(256) void k_hull_lookup(const uint32_t *__restrict__ idx,
                                                     const uint64_t *__restrict__ keys,
                                                     const int64_t *__restrict__ cnt_ptr,
                                                     int64_t S,
                                                     const int64_t *__restrict__ hoff,
                                                     const uint64_t *__restrict__ hkeys,
                                                     const uint32_t *__restrict__ hpos,
                                                     uint32_t *__restrict__ hull) {
    const int64_t n = *cnt_ptr;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        uint64_t k = keys[i];
        uint32_t s = key_set(k);
        if (s >= S) continue;
        int64_t a = hoff[s], b = hoff[s + 1];
        if (a == b) continue;
        int64_t r = a + count_less(hkeys, a, b, k);
        if (r < b && hkeys[r] == k) {
            uint32_t p = hpos[r];
            if (p < (uint64_t)(b - a)) atomicMin(&hull[a + p], idx[i]);
        }
    }
}

// Gather keys for an explicit index list (hull of a subset).
__global__ __launch_bounds__(256) void k_gather_keys(const float *__restrict__ x,
                                                     const float *__restrict__ y, int64_t n_pts,
                                                     const uint32_t *__restrict__ idx,
                                                     const int64_t *__restrict__ cnt_ptr,
                                                     uint64_t *__restrict__ keys) {
    const int64_t n = *cnt_ptr;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        uint32_t j = idx[i];
        if ((int64_t)j >= n_pts) j = 0;     // out-of-range index: read point 0 instead
        uint64_t kx = (uint64_t)(uint32_t)(x[j] * GRIDF);
        uint64_t ky = (uint64_t)(uint32_t)(y[j] * GRIDF);
        keys[i] = (kx << 24) | ky;
    }
}

// Before a computation: the recorded stage counts to -1 (stages that do not
// run keep it).
// Counts of a computation set to -1; clr[0, nclr) (optional) cleared.
__global__ void k_counts_init(int64_t *__restrict__ c, int n, unsigned long long *__restrict__ clr,
                              int nclr) {
    if (blockIdx.x == 0 && (int)threadIdx.x < n) c[threadIdx.x] = -1;
    if (clr)
        for (int i = threadIdx.x; i < nclr; i += blockDim.x) clr[i] = 0;
}

__global__ void k_copy_count(const int64_t *__restrict__ src, int64_t *__restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

}  // namespace hg
