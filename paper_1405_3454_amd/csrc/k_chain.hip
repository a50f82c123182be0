// Hull of the sorted survivors: Andrew's monotone chain (the paper's
// reference [6], corrected in its erratum), run in parallel.
//
// Keys are set << 48 | kx << 24 | ky, sorted ascending, so each set is a
// contiguous run ordered by (x, y).  Every chain below is segmented by the
// set field: it never joins points of different sets.
//  1. k_chain_chunks: one thread per CHAIN_C consecutive keys computes the
//     lower and the upper chain of its chunk (duplicates dropped; a point is
//     popped while it does not make a strict turn, so collinear points go).
//  2. k_chain_merge: one wave per group of CHAIN_G neighbouring chains joins
//     them left to right: at each junction the tail of the chain built so far
//     and the head of the next one are walked to their common tangent (the
//     bridge), then the rest of the next chain is appended.  Repeated until
//     one chain per kind is left.
//  3. Per set: the lower chain followed by the upper chain's interior in
//     reverse gives the counter-clockwise hull from the lexicographic
//     minimum; each hull key is mapped back to the lowest point index with
//     that key among the candidates.
#include "hg_device.h"

namespace hg {

constexpr int CHAIN_C = 256;
constexpr int CHAIN_G = 8;

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

// Sequential chain state: stack st[0..h) in memory with its top four
// entries mirrored in registers (t1 = st[h-1] ... t4 = st[h-4]), so a pop
// only issues a load for an entry that is needed two pops later.  seg is
// where the current set's part of the stack starts.
struct ChainState {
    uint64_t t1, t2, t3, t4;
    int h, seg;
};

template <bool UPPER>
__device__ __forceinline__ void chain_push(ChainState &c, uint64_t k, uint64_t *__restrict__ st) {
    if (c.h > c.seg && key_set(c.t1) != key_set(k)) c.seg = c.h;
    while (c.h - c.seg >= 2 && drop_mid<UPPER>(c.t2, c.t1, k)) {
        c.h--;
        c.t1 = c.t2;
        c.t2 = c.t3;
        c.t3 = c.t4;
        if (c.h - c.seg >= 4) c.t4 = st[c.h - 4];
    }
    st[c.h++] = k;
    c.t4 = c.t3;
    c.t3 = c.t2;
    c.t2 = c.t1;
    c.t1 = k;
}

__device__ __forceinline__ void load_keys8(const uint64_t *__restrict__ keys, int64_t base, int64_t b,
                                           uint64_t kb[8]) {
    if (base + 8 <= b) {
        const ulonglong2 *p = reinterpret_cast<const ulonglong2 *>(keys + base);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            ulonglong2 v = p[q];
            kb[2 * q] = v.x;
            kb[2 * q + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; q++) kb[q] = base + q < b ? keys[base + q] : ~uint64_t(0);
    }
}

// One thread per chunk: lower and upper chains of keys[a..b) in one walk;
// keys are read eight at a time, the next eight in flight while the current
// ones are consumed.
__global__ __launch_bounds__(256) void k_chain_chunks(const uint64_t *__restrict__ keys,
                                                      const int64_t *__restrict__ cnt_ptr,
                                                      uint64_t *__restrict__ lo,
                                                      uint64_t *__restrict__ up,
                                                      uint32_t *__restrict__ lo_cnt,
                                                      uint32_t *__restrict__ up_cnt) {
    const int64_t cnt = *cnt_ptr;
    const int64_t U = (cnt + CHAIN_C - 1) / CHAIN_C;
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (U == 0 && j == 0) {   // no candidates: the chains are empty
        lo_cnt[0] = 0;
        up_cnt[0] = 0;
    }
    if (j >= U) return;
    const int64_t a = j * CHAIN_C, b = min(a + CHAIN_C, cnt);
    ChainState L{0, 0, 0, 0, 0, 0}, Up{0, 0, 0, 0, 0, 0};
    uint64_t *lst = lo + a, *ust = up + a;
    uint64_t prev = ~uint64_t(0);
    uint64_t kb[8], kn[8];
    load_keys8(keys, a, b, kb);
    for (int64_t base = a; base < b; base += 8) {
        if (base + 8 < b) load_keys8(keys, base + 8, b, kn);
#pragma unroll
        for (int q = 0; q < 8; q++) {
            uint64_t k = kb[q];
            if (base + q >= b || k == prev) continue;
            prev = k;
            chain_push<false>(L, k, lst);
            chain_push<true>(Up, k, ust);
        }
#pragma unroll
        for (int q = 0; q < 8; q++) kb[q] = kn[q];
    }
    lo_cnt[j] = (uint32_t)L.h;
    up_cnt[j] = (uint32_t)Up.h;
}

// Index of the first element of src[lo..hi) whose set equals set(src[hi-1]).
__device__ __forceinline__ int64_t last_seg_start(const uint64_t *__restrict__ src, int64_t lo,
                                                  int64_t hi) {
    uint32_t s = key_set(src[hi - 1]);
    while (lo < hi - 1) {
        int64_t mid = (lo + hi - 1) >> 1;
        if (key_set(src[mid]) == s) hi = mid + 1; else lo = mid + 1;
    }
    return lo;
}

// One wave per group of CHAIN_G chains of level `lev` (unit span R keys).
// blockIdx.y: 0 = lower chains, 1 = upper chains.
template <bool UPPER>
__device__ void merge_group(const uint64_t *__restrict__ in, const uint32_t *__restrict__ cin,
                            int64_t U, int64_t R, int64_t v, uint64_t *__restrict__ out,
                            uint32_t *__restrict__ cout) {
    const int lane = lane_id();
    const int64_t base = v * R * CHAIN_G;
    uint64_t *o = out + base;
    int64_t len = 0, tailseg = 0;
    for (int g = 0; g < CHAIN_G; g++) {
        const int64_t u = v * CHAIN_G + g;
        if (u >= U) break;
        const uint64_t *src = in + u * R;
        const int64_t m = cin[u];
        if (m == 0) continue;
        int64_t b = 0;
        if (len > 0) {
            uint64_t last = o[len - 1];
            if (src[0] == last) b = 1;
            if (b < m && key_set(last) == key_set(src[b])) {
                int64_t a = len - 1;
                bool changed = true;
                while (changed) {
                    changed = false;
                    while (a > tailseg && drop_mid<UPPER>(o[a - 1], o[a], src[b])) {
                        a--;
                        changed = true;
                    }
                    while (b + 1 < m && key_set(src[b + 1]) == key_set(src[b]) &&
                           drop_mid<UPPER>(o[a], src[b], src[b + 1])) {
                        b++;
                        changed = true;
                    }
                }
                len = a + 1;
            }
        }
        if (b < m) {
            // the appended part's last set segment decides where the tail starts
            int64_t ls = last_seg_start(src, b, m);
            int64_t newtail;
            if (ls > b) newtail = len + (ls - b);
            else newtail = (len > 0 && key_set(o[len - 1]) == key_set(src[b])) ? tailseg : len;
            // all lanes must have read o[] before it is overwritten
            wave_sync();
            for (int64_t i = b + lane; i < m; i += WAVE) o[len + (i - b)] = src[i];
            wave_sync();
            __threadfence_block();
            len += m - b;
            tailseg = newtail;
        }
    }
    if (lane == 0) cout[v] = (uint32_t)len;
}

__global__ __launch_bounds__(256) void k_chain_merge(const uint64_t *__restrict__ lo_in,
                                                     const uint64_t *__restrict__ up_in,
                                                     const uint32_t *__restrict__ lo_cin,
                                                     const uint32_t *__restrict__ up_cin,
                                                     const int64_t *__restrict__ cnt_ptr, int lev,
                                                     uint64_t *__restrict__ lo_out,
                                                     uint64_t *__restrict__ up_out,
                                                     uint32_t *__restrict__ lo_cout,
                                                     uint32_t *__restrict__ up_cout) {
    const int64_t cnt = *cnt_ptr;
    int64_t R = CHAIN_C;
    for (int l = 0; l < lev; l++) R *= CHAIN_G;
    const int64_t U = (cnt + R - 1) / R;                  // chains at this level
    const int64_t V = (U + CHAIN_G - 1) / CHAIN_G;        // groups
    const int64_t v = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (V == 0 && v == 0 && threadIdx.x == 0)   // no candidates: empty top chain
        (blockIdx.y == 0 ? lo_cout : up_cout)[0] = 0;
    if (v >= V) return;
    if (blockIdx.y == 0) merge_group<false>(lo_in, lo_cin, U, R, v, lo_out, lo_cout);
    else merge_group<true>(up_in, up_cin, U, R, v, up_out, up_cout);
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

// Hull size per set: lower + upper - 2 shared ends; one point -> 1.
__global__ void k_hull_counts(const int64_t *__restrict__ bounds, int64_t S,
                              uint32_t *__restrict__ hcnt) {
    int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= S) return;
    int64_t hl = bounds[S + s] - bounds[s], hu = bounds[3 * S + s] - bounds[2 * S + s];
    hcnt[s] = (uint32_t)(hl == 0 ? 0 : (hl == 1 ? 1 : hl + hu - 2));
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

// Lay out each set's hull: CCW position of every chain entry, a key-sorted
// copy (hkeys, hpos) for the index lookup, and the output slots preset to
// HULL_NONE.
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
        int64_t ls = bounds[s], le = bounds[S + s], us = bounds[2 * S + s], ue = bounds[3 * S + s];
        int64_t hl = le - ls, hu = ue - us;
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
            if (hl <= 1 || r == 0 || r == hu - 1) continue;   // shared ends
            pos = hl + (hu - 2 - r);
            rank = (r - 1) + count_less(lo, ls, le, k);
        }
        int64_t o = hoff[s], h = hoff[s + 1] - o;
        if (pos >= h || rank >= h) continue;   // inconsistent chains: never write outside
        hkeys[o + rank] = k;
        hpos[o + rank] = (uint32_t)pos;
        hull[o + pos] = NONE;
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

__global__ void k_copy_count(const int64_t *__restrict__ src, int64_t *__restrict__ dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

}  // namespace hg
