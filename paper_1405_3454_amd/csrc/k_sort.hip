// Key-only LSD radix sort of uint64 point keys (8-bit digits, stable per
// pass).  The key count is read from device memory so the whole sort can run
// behind earlier kernels without a host round trip.
//
// Decomposition: SORT_BLOCKS persistent blocks; block b owns the contiguous
// key tiles [b qq, (b+1) qq) of SORT_TILE keys.  Per pass: (1) per-block digit
// histograms, (2) exclusive scan of the digit-major table hist[d][b],
// (3) scatter: each block walks its tiles in order and ranks keys stably with
// wave ballots (peers = lanes with the same digit) plus per-wave digit counts
// in LDS, so equal digits keep their input order across lanes, waves, rounds
// and blocks.
#include "hg_device.h"

namespace hg {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ROUNDS = 8;
constexpr int SORT_TILE = SORT_THREADS * SORT_ROUNDS;   // 2048 keys
constexpr int SORT_BLOCKS = 512;
constexpr int RADIX = 256;

__device__ __forceinline__ void sort_range(int64_t count, int64_t b, int64_t *lo, int64_t *hi) {
    int64_t tiles = (count + SORT_TILE - 1) / SORT_TILE;
    int64_t qq = (tiles + SORT_BLOCKS - 1) / SORT_BLOCKS;
    *lo = min(count, b * qq * SORT_TILE);
    *hi = min(count, (b + 1) * qq * SORT_TILE);
}

__global__ __launch_bounds__(SORT_THREADS) void k_sort_hist(const uint64_t *__restrict__ keys,
                                                            const int64_t *__restrict__ cnt_ptr,
                                                            int shift, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[RADIX];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t lo, hi;
    sort_range(*cnt_ptr, blockIdx.x, &lo, &hi);
    for (int64_t i = lo + threadIdx.x; i < hi; i += SORT_THREADS)
        atomicAdd(&h[(keys[i] >> shift) & (RADIX - 1)], 1u);
    __syncthreads();
    hist[threadIdx.x * SORT_BLOCKS + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(SORT_THREADS) void k_sort_scatter(const uint64_t *__restrict__ in,
                                                               const int64_t *__restrict__ cnt_ptr,
                                                               int shift,
                                                               const int64_t *__restrict__ hoff,
                                                               uint64_t *__restrict__ out) {
    constexpr int NW = SORT_THREADS / WAVE;
    __shared__ int64_t run[RADIX];
    __shared__ uint32_t wcnt[NW][RADIX];
    const int tid = threadIdx.x, w = tid >> 6;
    run[tid] = hoff[tid * SORT_BLOCKS + blockIdx.x];
    for (int ww = 0; ww < NW; ww++) wcnt[ww][tid] = 0;
    __syncthreads();
    int64_t lo, hi;
    sort_range(*cnt_ptr, blockIdx.x, &lo, &hi);
    const uint64_t lt = lanemask_lt();
    for (int64_t base = lo; base < hi; base += SORT_THREADS) {
        const int64_t i = base + tid;
        const bool valid = i < hi;
        uint64_t k = valid ? in[i] : 0;
        uint32_t d = (uint32_t)(k >> shift) & (RADIX - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            bool bit = (d >> b) & 1;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        int rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            int64_t p = run[d] + rank;
            for (int ww = 0; ww < w; ww++) p += wcnt[ww][d];
            out[p] = k;
        }
        __syncthreads();
        uint32_t t = 0;
        for (int ww = 0; ww < NW; ww++) {
            t += wcnt[ww][tid];
            wcnt[ww][tid] = 0;
        }
        run[tid] += t;
        __syncthreads();
    }
}

}  // namespace hg
