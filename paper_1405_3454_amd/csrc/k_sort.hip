// Key-only LSD radix sort of uint64 point keys (8-bit digits, stable per
// pass).  The key count is read from device memory so the whole sort can run
// behind earlier kernels without a host round trip.
//
// Decomposition: the keys are cut into at most SORT_BLOCKS contiguous ranges
// of qq tiles of SORT_TILE keys.  One kernel counts every pass's digits over
// all keys (global digit totals, hence each digit's start in the output).
// Then one kernel per pass: a block claims the next range (a counter, so
// ranges are taken in order), counts its digits, publishes the counts and
// sums those of the ranges before it by decoupled look-back (a range's entry
// holds its own counts or, once known, the counts of all ranges up to it),
// and scatters its keys: each tile ranked stably with wave ballots (peers =
// lanes with the same digit) plus per-wave digit counts in LDS, so equal
// digits keep their input order across lanes, waves, tiles and ranges.
#include "hg_device.h"

namespace hg {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ROUNDS = 8;
constexpr int SORT_TILE = SORT_THREADS * SORT_ROUNDS;   // 2048 keys
constexpr int SORT_BLOCKS = 512;
constexpr int RADIX = 256;
constexpr int SORT_SMALL = 4096;      // up to this many keys one block sorts them (k_sort_small)
constexpr int SMALL_THREADS = 1024;
constexpr int SMALL_CLEAR_BLOCKS = 32;  // k_sort_small's blocks after the first: clear the passes' state

// Tiles per range: enough for SORT_BLOCKS ranges, and up to 8 when that
// keeps the ranges at 64 or fewer (a shorter look-back per pass).
__device__ __forceinline__ int64_t sort_qq(int64_t count) {
    const int64_t tiles = (count + SORT_TILE - 1) / SORT_TILE;
    return max((tiles + SORT_BLOCKS - 1) / SORT_BLOCKS, min((int64_t)8, (tiles + 63) / 64));
}

__device__ __forceinline__ void sort_range(int64_t count, int64_t b, int64_t *lo, int64_t *hi) {
    const int64_t qq = sort_qq(count);
    *lo = min(count, b * qq * SORT_TILE);
    *hi = min(count, (b + 1) * qq * SORT_TILE);
}

// Ranges of sort_range that hold keys: 0 .. sort_busy(count) - 1.
__device__ __forceinline__ int64_t sort_busy(int64_t count) {
    const int64_t tiles = (count + SORT_TILE - 1) / SORT_TILE;
    const int64_t qq = sort_qq(count);
    return qq ? (tiles + qq - 1) / qq : 0;
}

// Range look-back entries: pass tag (pass + 1) << 56 | state << 54 | value,
// 0 = not yet written this call.
constexpr uint64_t LB_AGG = 1ull << 54, LB_INC = 2ull << 54;
constexpr uint64_t LB_VAL = (1ull << 54) - 1, LB_TAG = ~((1ull << 56) - 1);
constexpr int SORT_MAX_PASSES = 8;

// At most SORT_SMALL keys: block 0 sorts them in LDS (bitonic network over
// the next power of two, padded with the largest key) and writes them where
// the radix passes would have left them; the passes then return at once.
// Above SORT_SMALL the other blocks clear the passes' state (the digit
// totals, the range counters and the look-back entries of the busy ranges).
// The sort is by key only, so equal keys are interchangeable and the result
// is the radix sort's.
__global__ __launch_bounds__(SMALL_THREADS) void k_sort_small(const uint64_t *__restrict__ keys,
                                                              const int64_t *__restrict__ cnt_ptr,
                                                              uint64_t *__restrict__ out,
                                                              unsigned long long *__restrict__ status,
                                                              uint32_t *__restrict__ gstate,
                                                              int *__restrict__ seg_fallback) {
    __shared__ uint64_t b[SORT_SMALL];
    const int64_t count = *cnt_ptr;
    const int tid = threadIdx.x;
    if (seg_fallback && blockIdx.x == 0 && tid == 0) *seg_fallback = 0;
    if (count > SORT_SMALL) {
        if (blockIdx.x == 0) return;
        const int64_t nst = sort_busy(count) * RADIX;
        const int64_t nt = (int64_t)(gridDim.x - 1) * SMALL_THREADS;
        for (int64_t i = (int64_t)(blockIdx.x - 1) * SMALL_THREADS + tid; i < nst; i += nt) status[i] = 0;
        if (blockIdx.x == 1)
            for (int i = tid; i < SORT_MAX_PASSES * (RADIX + 1); i += SMALL_THREADS) gstate[i] = 0;
        return;
    }
    if (blockIdx.x != 0 || count <= 0) return;
    const int n = (int)count;
    int m = 2;
    while (m < n) m <<= 1;
    for (int i = tid; i < m; i += SMALL_THREADS) b[i] = i < n ? keys[i] : ~0ull;
    __syncthreads();
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = tid; t < (m >> 1); t += SMALL_THREADS) {
                const int i = 2 * j * (t / j) + (t % j), l = i + j;    // pair (i, l), i < l
                const bool up = (i & k) == 0;                         // ascending run
                const uint64_t a = b[i], c = b[l];
                if ((a > c) == up) {
                    b[i] = c;
                    b[l] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < n; i += SMALL_THREADS) out[i] = b[i];
}

// Several sets.  The candidates of the hull stage arrive grouped by set in
// ascending set order (the filter's regions follow the tiles, and the tiles
// follow the sets), so each set can be sorted alone: start[s] = the first
// candidate of set s for s = 0..S (start[S] = n), from the keys' set field;
// a key whose set is below its predecessor's raises SEG_UNORDERED in
// *fallback, and the radix passes then sort everything.  Without it the
// starts are also the sets' ranges in the sorted keys (the sort keeps each
// set's range), which the chain stage reads.
constexpr int SEG_TOO_BIG = 1, SEG_UNORDERED = 2;

__global__ __launch_bounds__(256) void k_set_starts(const uint64_t *__restrict__ keys,
                                                    const int64_t *__restrict__ cnt_ptr, int64_t S,
                                                    int64_t *__restrict__ start, int *__restrict__ fallback) {
    const int64_t n = *cnt_ptr;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i <= n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t prev = i == 0 ? -1 : (int64_t)(keys[i - 1] >> 48);
        const int64_t cur = i == n ? S : (int64_t)(keys[i] >> 48);
        if (cur < prev) atomicOr(fallback, SEG_UNORDERED);
        for (int64_t t = prev + 1; t <= cur && t <= S; t++) start[t] = i;
    }
}

constexpr int SEG_THREADS = 1024;
constexpr int SEG_MAX = 8192;         // keys of one set a block sorts in LDS (64 KB)

// Each set's range [start[s], start[s + 1]) sorted in LDS by one block
// (bitonic network over the next power of two, padded with the largest key)
// into out, where the radix passes would have left it; block b takes the
// sets b, b + gridDim.x, ...  A set of more than SEG_MAX keys, or a key in a
// range that is not its set's, raises *fallback.
__global__ __launch_bounds__(SEG_THREADS) void k_sort_sets(const uint64_t *__restrict__ keys,
                                                           const int64_t *__restrict__ cnt_ptr, int64_t S,
                                                           const int64_t *__restrict__ start,
                                                           uint64_t *__restrict__ out,
                                                           int *__restrict__ fallback) {
    __shared__ uint64_t b[SEG_MAX];
    __shared__ int bad;
    const int64_t n = *cnt_ptr;
    if (n <= SORT_SMALL) return;
    const int tid = threadIdx.x;
    for (int64_t s = blockIdx.x; s < S; s += gridDim.x) {
        const int64_t a = start[s], e = start[s + 1];
        if (e <= a) continue;
        if (e - a > SEG_MAX) {
            if (tid == 0) atomicOr(fallback, SEG_TOO_BIG);
            continue;
        }
        const int m = (int)(e - a);
        int P = 1;
        while (P < m) P <<= 1;
        if (tid == 0) bad = 0;
        __syncthreads();
        for (int i = tid; i < P; i += SEG_THREADS) {
            const uint64_t k = i < m ? keys[a + i] : ~0ull;
            if (i < m && (int64_t)(k >> 48) != s) bad = 1;
            b[i] = k;
        }
        __syncthreads();
        if (bad) {
            if (tid == 0) atomicOr(fallback, SEG_UNORDERED);
            __syncthreads();
            continue;
        }
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int t = tid; t < (P >> 1); t += SEG_THREADS) {
                    const int i = 2 * j * (t / j) + (t % j), l = i + j;    // pair (i, l), i < l
                    const bool up = (i & k) == 0;                         // ascending run
                    const uint64_t x = b[i], y = b[l];
                    if ((x > y) == up) {
                        b[i] = y;
                        b[l] = x;
                    }
                }
                __syncthreads();
            }
        }
        for (int i = tid; i < m; i += SEG_THREADS) out[a + i] = b[i];
        __syncthreads();      // b is refilled for the next set
    }
}

// Digit totals of every pass over all keys: block b counts the digits of
// range b in LDS and adds them to gcount[pass][digit] (cleared by
// k_sort_small).
__global__ __launch_bounds__(SORT_THREADS) void k_sort_prep(const uint64_t *__restrict__ keys,
                                                            const int64_t *__restrict__ cnt_ptr,
                                                            int passes, uint32_t *__restrict__ gcount,
                                                            const int *__restrict__ seg_fallback) {
    __shared__ uint32_t h[SORT_MAX_PASSES][RADIX];
    const int tid = threadIdx.x;
    const int64_t count = *cnt_ptr;
    if (count <= SORT_SMALL) return;
    if (seg_fallback && *seg_fallback == 0) return;    // k_sort_sets has sorted every set
    if ((int64_t)blockIdx.x >= sort_busy(count)) return;
    for (int ps = 0; ps < SORT_MAX_PASSES; ps++) h[ps][tid] = 0;
    __syncthreads();
    int64_t lo, hi;
    sort_range(count, blockIdx.x, &lo, &hi);
    for (int64_t base = lo; base < hi; base += SORT_TILE) {
        uint64_t k[SORT_ROUNDS];
#pragma unroll
        for (int r = 0; r < SORT_ROUNDS; r++) {
            const int64_t i = base + r * SORT_THREADS + tid;
            k[r] = i < hi ? keys[i] : 0;
        }
#pragma unroll
        for (int r = 0; r < SORT_ROUNDS; r++) {
            if (base + r * SORT_THREADS + tid >= hi) continue;
            for (int ps = 0; ps < passes; ps++) atomicAdd(&h[ps][(uint32_t)(k[r] >> (8 * ps)) & (RADIX - 1)], 1u);
        }
    }
    __syncthreads();
    for (int ps = 0; ps < passes; ps++)
        if (h[ps][tid]) atomicAdd(&gcount[ps * RADIX + tid], h[ps][tid]);
}

// Sum of the digit-d counts of the ranges before range r (thread d), from
// their look-back entries: an entry with the range's own counts (LB_AGG) is
// added and the walk goes on, one with the counts up to and including that
// range (LB_INC) ends it; an entry not yet written this pass is read again.
// Ranges are claimed in order by running blocks, and each publishes its own
// counts before it looks back, so every wait ends.
__device__ __forceinline__ int64_t look_back(const unsigned long long *__restrict__ status, int64_t r,
                                             int d, uint64_t tag) {
    constexpr int LB = 16;
    int64_t excl = 0;
    int64_t k = r - 1;
    while (k >= 0) {
        uint64_t v[LB];
#pragma unroll
        for (int i = 0; i < LB; i++)
            v[i] = k - i >= 0 ? __hip_atomic_load(&status[(k - i) * RADIX + d], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT)
                              : 0;
        int used = 0;
        bool done = false;
#pragma unroll
        for (int i = 0; i < LB; i++) {
            if (done || used < i || k - i < 0) continue;
            if ((v[i] & LB_TAG) != tag) continue;     // not written yet: read it again
            excl += (int64_t)(v[i] & LB_VAL);
            used = i + 1;
            if (v[i] & LB_INC) done = true;
        }
        if (done) break;
        k -= used;
        if (used == 0) __builtin_amdgcn_s_sleep(1);
    }
    return excl;
}

// One pass: claim a range, count its digits, publish them, look back, and
// scatter the range tile by tile.  Per tile (round r, wave w, lane l holds
// key r*256 + w*64 + l): stable ranks from wave ballots and per (round,
// wave, digit) counts; the tile is reordered by digit in LDS and then
// written out run by run, so consecutive lanes write consecutive addresses.
__global__ __launch_bounds__(SORT_THREADS) void k_sort_pass(const uint64_t *__restrict__ in,
                                                            const int64_t *__restrict__ cnt_ptr,
                                                            int pass, const uint32_t *__restrict__ gcount,
                                                            unsigned long long *__restrict__ status,
                                                            uint32_t *__restrict__ claim,
                                                            uint64_t *__restrict__ out,
                                                            const int *__restrict__ seg_fallback) {
    constexpr int NW = SORT_THREADS / WAVE;
    __shared__ int64_t run[RADIX];                       // next output position per digit
    __shared__ __attribute__((aligned(16))) uint16_t wcnt[SORT_ROUNDS][NW][RADIX];
    __shared__ uint32_t dstart[RADIX + 1], dtot[RADIX], rh[RADIX];
    __shared__ int64_t scan_sh[17];
    __shared__ uint64_t buf[SORT_TILE];
    __shared__ int64_t rsh;
    const int tid = threadIdx.x, w = tid >> 6;
    const int shift = 8 * pass;
    const int64_t count = *cnt_ptr;
    if (count <= SORT_SMALL) return;     // k_sort_small has sorted them
    if (seg_fallback && *seg_fallback == 0) return;    // k_sort_sets has sorted every set
    if (tid == 0) rsh = (int64_t)atomicAdd(claim, 1u);
    const uint32_t gd = gcount[pass * RADIX + tid];      // this digit's total (in flight with the claim)
    rh[tid] = 0;
    __syncthreads();
    const int64_t rr = rsh;
    if (rr >= sort_busy(count)) return;
    int64_t lo, hi;
    sort_range(count, rr, &lo, &hi);
    // the range's digit counts (a single tile keeps its keys in registers)
    const bool one_tile = hi - lo <= SORT_TILE;
    uint64_t k[SORT_ROUNDS];
    for (int64_t base = lo; base < hi; base += SORT_TILE) {
#pragma unroll
        for (int r = 0; r < SORT_ROUNDS; r++) {
            const int64_t i = base + r * SORT_THREADS + tid;
            k[r] = i < hi ? in[i] : 0;
        }
#pragma unroll
        for (int r = 0; r < SORT_ROUNDS; r++)
            if (base + r * SORT_THREADS + tid < hi) atomicAdd(&rh[(uint32_t)(k[r] >> shift) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    {   // publish, look back, and the digit's first output position
        const uint64_t tag = (uint64_t)(pass + 1) << 56;
        const uint32_t mine = rh[tid];
        int64_t tot;
        const int64_t gs = block_excl_scan_i64((int64_t)gd, scan_sh, &tot);
        unsigned long long *e = &status[rr * RADIX + tid];
        int64_t excl = 0;
        if (rr == 0) {
            __hip_atomic_store(e, tag | LB_INC | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(e, tag | LB_AGG | mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            excl = look_back(status, rr, tid, tag);
            __hip_atomic_store(e, tag | LB_INC | (uint64_t)(excl + mine), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        run[tid] = gs + excl;
    }
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    for (int64_t base = lo; base < hi; base += SORT_TILE) {
        const int ntile = (int)min((int64_t)SORT_TILE, hi - base);
        {   // clear the per-(round, wave, digit) counts: 16 KB, 64 B per thread
            uint4 *z = reinterpret_cast<uint4 *>(&wcnt[0][0][0]);
            for (int i = tid; i < (int)(sizeof(wcnt) / sizeof(uint4)); i += SORT_THREADS)
                z[i] = make_uint4(0, 0, 0, 0);
        }
        uint32_t d[SORT_ROUNDS];
        int rank[SORT_ROUNDS], cnt[SORT_ROUNDS];
#pragma unroll
        for (int r = 0; r < SORT_ROUNDS; r++) {
            const int i = r * SORT_THREADS + tid;
            const bool valid = i < ntile;
            if (!one_tile) k[r] = valid ? in[base + i] : 0;
            d[r] = (uint32_t)(k[r] >> shift) & (RADIX - 1);
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; b++) {
                bool bit = (d[r] >> b) & 1;
                uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            rank[r] = valid ? __popcll(peers & lt) : -1;
            cnt[r] = __popcll(peers);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SORT_ROUNDS; r++)
            if (rank[r] == 0) wcnt[r][w][d[r]] = (uint16_t)cnt[r];
        __syncthreads();
        {   // digit tid: exclusive prefix over (round, wave) in key order
            uint32_t acc = 0;
            for (int r = 0; r < SORT_ROUNDS; r++)
                for (int ww = 0; ww < NW; ww++) {
                    uint32_t c = wcnt[r][ww][tid];
                    wcnt[r][ww][tid] = (uint16_t)acc;
                    acc += c;
                }
            dtot[tid] = acc;
        }
        __syncthreads();
        {
            int64_t tot;
            int64_t ex = block_excl_scan_i64(dtot[tid], scan_sh, &tot);
            dstart[tid] = (uint32_t)ex;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SORT_ROUNDS; r++)
            if (rank[r] >= 0) buf[dstart[d[r]] + wcnt[r][w][d[r]] + rank[r]] = k[r];
        __syncthreads();
        for (int i = tid; i < ntile; i += SORT_THREADS) {
            uint64_t kk = buf[i];
            uint32_t dd = (uint32_t)(kk >> shift) & (RADIX - 1);
            out[run[dd] + (i - (int)dstart[dd])] = kk;
        }
        __syncthreads();
        run[tid] += dtot[tid];
        __syncthreads();
    }
}

}  // namespace hg
