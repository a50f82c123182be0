// Key-only LSD radix sort of uint64 point keys (8-bit digits, stable per
// pass).  The key count is read from device memory so the whole sort can run
// behind earlier kernels without a host round trip.
//
// Decomposition: SORT_BLOCKS persistent blocks; block b owns the contiguous
// key tiles [b qq, (b+1) qq) of SORT_TILE keys.  Per pass: (1) per-block digit
// histograms, after which the last block to finish scans the table
// hist[b][d] digit-major (only the blocks that hold keys), (2) scatter: each block
// walks its tiles in order and ranks keys stably with wave ballots (peers =
// lanes with the same digit) plus per-wave digit counts in LDS, so equal
// digits keep their input order across lanes, waves, rounds and blocks.
#include "hg_device.h"

namespace hg {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ROUNDS = 8;
constexpr int SORT_TILE = SORT_THREADS * SORT_ROUNDS;   // 2048 keys
constexpr int SORT_BLOCKS = 512;
constexpr int RADIX = 256;
constexpr int SORT_SMALL = 4096;      // up to this many keys one block sorts them (k_sort_small)
constexpr int SMALL_THREADS = 1024;

// Tiles per block: enough for SORT_BLOCKS blocks, and up to 8 when that
// keeps the busy blocks at 64 or fewer (the last block's digit scan then
// holds every block's count in registers in one batch of loads).
__device__ __forceinline__ int64_t sort_qq(int64_t count) {
    const int64_t tiles = (count + SORT_TILE - 1) / SORT_TILE;
    return max((tiles + SORT_BLOCKS - 1) / SORT_BLOCKS, min((int64_t)8, (tiles + 63) / 64));
}

__device__ __forceinline__ void sort_range(int64_t count, int64_t b, int64_t *lo, int64_t *hi) {
    const int64_t qq = sort_qq(count);
    *lo = min(count, b * qq * SORT_TILE);
    *hi = min(count, (b + 1) * qq * SORT_TILE);
}

// Blocks of sort_range that hold keys: 0 .. sort_busy(count) - 1.
__device__ __forceinline__ int64_t sort_busy(int64_t count) {
    const int64_t tiles = (count + SORT_TILE - 1) / SORT_TILE;
    const int64_t qq = sort_qq(count);
    return qq ? (tiles + qq - 1) / qq : 0;
}

// At most SORT_SMALL keys: one block sorts them in LDS (bitonic network over
// the next power of two, padded with the largest key) and writes them where
// the radix passes would have left them; the passes then return at once.
// Above SORT_SMALL it returns at once.  The sort is by key only, so equal
// keys are interchangeable and the result is the radix sort's.
__global__ __launch_bounds__(SMALL_THREADS) void k_sort_small(const uint64_t *__restrict__ keys,
                                                              const int64_t *__restrict__ cnt_ptr,
                                                              uint64_t *__restrict__ out) {
    __shared__ uint64_t b[SORT_SMALL];
    const int64_t count = *cnt_ptr;
    if (count > SORT_SMALL || count <= 0) return;
    const int n = (int)count, tid = threadIdx.x;
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

// Per-block digit histograms of the blocks that hold keys; the last of them
// to finish (ticket, self-resetting) turns them into the exclusive offsets
// hoff[b][d] of the stable scatter.  Both tables are block-major, so a block
// writes its column, and the last block reads each block's, with consecutive
// lanes on consecutive words.  Blocks without keys leave at once (the scatter
// does not read their offsets).
__global__ __launch_bounds__(SORT_THREADS) void k_sort_hist(const uint64_t *__restrict__ keys,
                                                            const int64_t *__restrict__ cnt_ptr,
                                                            int shift, uint32_t *__restrict__ hist,
                                                            int64_t *__restrict__ hoff,
                                                            uint32_t *__restrict__ ticket) {
    __shared__ uint32_t h[RADIX];
    __shared__ int64_t scan_sh[17];
    __shared__ bool last;
    const int tid = threadIdx.x;
    const int64_t count = *cnt_ptr;
    if (count <= SORT_SMALL) return;     // k_sort_small has sorted them
    const int nb = (int)sort_busy(count);
    if ((int)blockIdx.x >= nb) return;   // no keys: nothing to count or scan
    h[tid] = 0;
    __syncthreads();
    int64_t lo, hi;
    sort_range(count, blockIdx.x, &lo, &hi);
    for (int64_t base = lo; base < hi; base += SORT_TILE) {     // a tile's loads, then its counts
        uint32_t d[SORT_ROUNDS];
#pragma unroll
        for (int r = 0; r < SORT_ROUNDS; r++) {
            const int64_t i = base + r * SORT_THREADS + tid;
            d[r] = i < hi ? (uint32_t)(keys[i] >> shift) & (RADIX - 1) : (uint32_t)RADIX;
        }
#pragma unroll
        for (int r = 0; r < SORT_ROUNDS; r++)
            if (d[r] < RADIX) atomicAdd(&h[d[r]], 1u);
    }
    __syncthreads();
    hist[(int64_t)blockIdx.x * RADIX + tid] = h[tid];
    __threadfence();   // every wave publishes its part of the block's column
    __syncthreads();
    if (tid == 0) {
        last = atomicAdd(ticket, 1u) == (uint32_t)nb - 1;
        if (last) __threadfence();
    }
    __syncthreads();
    if (!last) return;
    // thread d: digit d over the busy blocks, up to HB independent loads per
    // step (in groups of HG, skipped past the last busy block); with at most
    // HB busy blocks the values stay in registers for the second walk
    constexpr int HB = 64, HG = 8;
    uint32_t v[HB];
    auto load = [&](int b0) {
#pragma unroll
        for (int gi = 0; gi < HB / HG; gi++) {
            const bool any = b0 + gi * HG < nb;
#pragma unroll
            for (int i = 0; i < HG; i++) {
                const int bb = b0 + gi * HG + i;
                v[gi * HG + i] = any && bb < nb ? hist[(int64_t)bb * RADIX + tid] : 0u;
            }
        }
    };
    uint32_t tot = 0;
    for (int b0 = 0; b0 < nb; b0 += HB) {
        load(b0);
#pragma unroll
        for (int i = 0; i < HB; i++) tot += v[i];
    }
    int64_t all;
    int64_t run = block_excl_scan_i64(tot, scan_sh, &all);
    for (int b0 = 0; b0 < nb; b0 += HB) {
        if (nb > HB) load(b0);
#pragma unroll
        for (int gi = 0; gi < HB / HG; gi++) {
            if (b0 + gi * HG < nb) {
#pragma unroll
                for (int i = 0; i < HG; i++) {
                    const int bb = b0 + gi * HG + i;
                    if (bb < nb) hoff[(int64_t)bb * RADIX + tid] = run;
                    run += v[gi * HG + i];
                }
            }
        }
    }
    if (tid == 0) *ticket = 0;
}

// Scatter of one pass.  Per tile of SORT_TILE keys (round r, wave w, lane l
// holds key r*256 + w*64 + l): stable ranks from wave ballots and per
// (round, wave, digit) counts; the tile is reordered by digit in LDS and then
// written out run by run, so consecutive lanes write consecutive addresses.
__global__ __launch_bounds__(SORT_THREADS) void k_sort_scatter(const uint64_t *__restrict__ in,
                                                               const int64_t *__restrict__ cnt_ptr,
                                                               int shift,
                                                               const int64_t *__restrict__ hoff,
                                                               uint64_t *__restrict__ out) {
    constexpr int NW = SORT_THREADS / WAVE;
    __shared__ int64_t run[RADIX];                       // next output position per digit
    __shared__ __attribute__((aligned(16))) uint16_t wcnt[SORT_ROUNDS][NW][RADIX];
    __shared__ uint32_t dstart[RADIX + 1], dtot[RADIX];
    __shared__ int64_t scan_sh[17];
    __shared__ uint64_t buf[SORT_TILE];
    const int tid = threadIdx.x, w = tid >> 6;
    if (*cnt_ptr <= SORT_SMALL) return;  // k_sort_small has sorted them
    run[tid] = hoff[(int64_t)blockIdx.x * RADIX + tid];
    int64_t lo, hi;
    sort_range(*cnt_ptr, blockIdx.x, &lo, &hi);
    const uint64_t lt = lanemask_lt();
    for (int64_t base = lo; base < hi; base += SORT_TILE) {
        const int ntile = (int)min((int64_t)SORT_TILE, hi - base);
        {   // clear the per-(round, wave, digit) counts: 16 KB, 64 B per thread
            uint4 *z = reinterpret_cast<uint4 *>(&wcnt[0][0][0]);
            for (int i = tid; i < (int)(sizeof(wcnt) / sizeof(uint4)); i += SORT_THREADS)
                z[i] = make_uint4(0, 0, 0, 0);
        }
        uint64_t k[SORT_ROUNDS];
        uint32_t d[SORT_ROUNDS];
        int rank[SORT_ROUNDS], cnt[SORT_ROUNDS];
#pragma unroll
        for (int r = 0; r < SORT_ROUNDS; r++) {
            const int i = r * SORT_THREADS + tid;
            const bool valid = i < ntile;
            k[r] = valid ? in[base + i] : 0;
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
