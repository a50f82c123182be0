// Device-side helpers used by several kernel files of the library.
#pragma once
#include "hg_common.h"

namespace hg {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// Make the wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Farthest-point key of a refinement edge: float(distance) bits << 32 |
// ~index, so the maximum is (close to) the farthest point, lowest index among
// equal keys, whatever the order of the updates.
__device__ __forceinline__ uint64_t far_key(double dist, uint32_t idx) {
    return ((uint64_t)__float_as_uint((float)dist) << 32) | (uint64_t)(~idx);
}

// Raise *slot to key unless it already holds at least as much.
__device__ __forceinline__ void far_update(unsigned long long *slot, uint64_t key) {
    if (*reinterpret_cast<volatile unsigned long long *>(slot) < key) atomicMax(slot, key);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << lane_id()) - 1;
}

// A wave-uniform double moved into scalar registers.
__device__ __forceinline__ double uniform_f64(double v) {
    uint64_t b = __double_as_longlong(v);
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Inclusive scan across the wave.
__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int64_t t = __shfl_up(v, o);
        if (l >= o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over a block of `nwaves` waves.
// `sh` must hold at least nwaves + 1 entries.  Returns the exclusive prefix;
// *total gets the block sum.  Every thread of the block must call it.
__device__ __forceinline__ int64_t block_excl_scan_i64(int64_t v, int64_t *sh, int64_t *total) {
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6, l = lane_id();
    int64_t inc = wave_incl_scan_i64(v);
    if (l == WAVE - 1) sh[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int i = 0; i < nw; i++) {
            int64_t t = sh[i];
            sh[i] = run;
            run += t;
        }
        sh[nw] = run;
    }
    __syncthreads();
    int64_t r = sh[w] + inc - v;
    *total = sh[nw];
    __syncthreads();
    return r;
}

// Point range of set s: [begin, end).  off == nullptr means one set [0, n1).
__device__ __forceinline__ int64_t set_begin(const int64_t *off, int64_t s) {
    return off ? off[s] : 0;
}
__device__ __forceinline__ int64_t set_end(const int64_t *off, int64_t n1, int64_t s) {
    return off ? off[s + 1] : n1;
}

// Exact orientation in grid units: z of (a - o) x (b - o).  Coordinates are
// integers below 2^24 held in doubles; each product is exact and the fused
// difference is exact (|result| < 2^50).
__device__ __forceinline__ double orient(double ox, double oy, double ax, double ay,
                                         double bx, double by) {
    double dx1 = ax - ox, dy1 = ay - oy, dx2 = bx - ox, dy2 = by - oy;
    return fma(dx1, dy2, -(dy1 * dx2));
}

}  // namespace hg
