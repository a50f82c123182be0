// Learned direction proposal (this project's extension, not the paper's):
// a 32 x 32 occupancy histogram of each set feeds a small MLP that scores 64
// candidate directions; the eight best are added to the fixed extremes.
// Extra extremes can only enlarge the filter polygon inside the hull, so the
// hull never depends on the network.
#include "hg_device.h"

namespace hg {

constexpr int NCAND = 64;

// Candidate directions phi_d = 2 pi d / 64 as correctly rounded binary64
// (cos, sin); multiples of 90 degrees are exact.
static const double kCandCos[NCAND] = {
    0x1.0000000000000p+0, 0x1.fd88da3d12526p-1, 0x1.f6297cff75cb0p-1, 0x1.e9f4156c62ddap-1,
    0x1.d906bcf328d46p-1, 0x1.c38b2f180bdb1p-1, 0x1.a9b66290ea1a3p-1, 0x1.8bc806b151741p-1,
    0x1.6a09e667f3bcdp-1, 0x1.44cf325091dd6p-1, 0x1.1c73b39ae68c8p-1, 0x1.e2b5d3806f63bp-2,
    0x1.87de2a6aea963p-2, 0x1.294062ed59f06p-2, 0x1.8f8b83c69a60bp-3, 0x1.917a6bc29b42cp-4,
    0.0, -0x1.917a6bc29b42cp-4, -0x1.8f8b83c69a60bp-3, -0x1.294062ed59f06p-2,
    -0x1.87de2a6aea963p-2, -0x1.e2b5d3806f63bp-2, -0x1.1c73b39ae68c8p-1, -0x1.44cf325091dd6p-1,
    -0x1.6a09e667f3bcdp-1, -0x1.8bc806b151741p-1, -0x1.a9b66290ea1a3p-1, -0x1.c38b2f180bdb1p-1,
    -0x1.d906bcf328d46p-1, -0x1.e9f4156c62ddap-1, -0x1.f6297cff75cb0p-1, -0x1.fd88da3d12526p-1,
    -0x1.0000000000000p+0, -0x1.fd88da3d12526p-1, -0x1.f6297cff75cb0p-1, -0x1.e9f4156c62ddap-1,
    -0x1.d906bcf328d46p-1, -0x1.c38b2f180bdb1p-1, -0x1.a9b66290ea1a3p-1, -0x1.8bc806b151741p-1,
    -0x1.6a09e667f3bcdp-1, -0x1.44cf325091dd6p-1, -0x1.1c73b39ae68c8p-1, -0x1.e2b5d3806f63bp-2,
    -0x1.87de2a6aea963p-2, -0x1.294062ed59f06p-2, -0x1.8f8b83c69a60bp-3, -0x1.917a6bc29b42cp-4,
    0.0, 0x1.917a6bc29b42cp-4, 0x1.8f8b83c69a60bp-3, 0x1.294062ed59f06p-2,
    0x1.87de2a6aea963p-2, 0x1.e2b5d3806f63bp-2, 0x1.1c73b39ae68c8p-1, 0x1.44cf325091dd6p-1,
    0x1.6a09e667f3bcdp-1, 0x1.8bc806b151741p-1, 0x1.a9b66290ea1a3p-1, 0x1.c38b2f180bdb1p-1,
    0x1.d906bcf328d46p-1, 0x1.e9f4156c62ddap-1, 0x1.f6297cff75cb0p-1, 0x1.fd88da3d12526p-1,
};
static const double kCandSin[NCAND] = {
    0.0, 0x1.917a6bc29b42cp-4, 0x1.8f8b83c69a60bp-3, 0x1.294062ed59f06p-2,
    0x1.87de2a6aea963p-2, 0x1.e2b5d3806f63bp-2, 0x1.1c73b39ae68c8p-1, 0x1.44cf325091dd6p-1,
    0x1.6a09e667f3bcdp-1, 0x1.8bc806b151741p-1, 0x1.a9b66290ea1a3p-1, 0x1.c38b2f180bdb1p-1,
    0x1.d906bcf328d46p-1, 0x1.e9f4156c62ddap-1, 0x1.f6297cff75cb0p-1, 0x1.fd88da3d12526p-1,
    0x1.0000000000000p+0, 0x1.fd88da3d12526p-1, 0x1.f6297cff75cb0p-1, 0x1.e9f4156c62ddap-1,
    0x1.d906bcf328d46p-1, 0x1.c38b2f180bdb1p-1, 0x1.a9b66290ea1a3p-1, 0x1.8bc806b151741p-1,
    0x1.6a09e667f3bcdp-1, 0x1.44cf325091dd6p-1, 0x1.1c73b39ae68c8p-1, 0x1.e2b5d3806f63bp-2,
    0x1.87de2a6aea963p-2, 0x1.294062ed59f06p-2, 0x1.8f8b83c69a60bp-3, 0x1.917a6bc29b42cp-4,
    0.0, -0x1.917a6bc29b42cp-4, -0x1.8f8b83c69a60bp-3, -0x1.294062ed59f06p-2,
    -0x1.87de2a6aea963p-2, -0x1.e2b5d3806f63bp-2, -0x1.1c73b39ae68c8p-1, -0x1.44cf325091dd6p-1,
    -0x1.6a09e667f3bcdp-1, -0x1.8bc806b151741p-1, -0x1.a9b66290ea1a3p-1, -0x1.c38b2f180bdb1p-1,
    -0x1.d906bcf328d46p-1, -0x1.e9f4156c62ddap-1, -0x1.f6297cff75cb0p-1, -0x1.fd88da3d12526p-1,
    -0x1.0000000000000p+0, -0x1.fd88da3d12526p-1, -0x1.f6297cff75cb0p-1, -0x1.e9f4156c62ddap-1,
    -0x1.d906bcf328d46p-1, -0x1.c38b2f180bdb1p-1, -0x1.a9b66290ea1a3p-1, -0x1.8bc806b151741p-1,
    -0x1.6a09e667f3bcdp-1, -0x1.44cf325091dd6p-1, -0x1.1c73b39ae68c8p-1, -0x1.e2b5d3806f63bp-2,
    -0x1.87de2a6aea963p-2, -0x1.294062ed59f06p-2, -0x1.8f8b83c69a60bp-3, -0x1.917a6bc29b42cp-4,
};

__constant__ double dCandCos[NCAND];
__constant__ double dCandSin[NCAND];

constexpr int HBINS = 1024;                   // 32 x 32 histogram
constexpr int HSAMPLE = 16384;                // at most this many sampled points
constexpr int HRUNS = HSAMPLE / WAVE;          // in runs of WAVE consecutive points
constexpr int L1 = 512, L2 = 512, NOUT = NCAND;
// parameter layout (float32): W1[512][1024] b1[512] W2[512][512] b2[512] W3[64][512] b3[64]
constexpr int64_t P_W1 = 0, P_B1 = P_W1 + (int64_t)L1 * HBINS, P_W2 = P_B1 + L1,
                  P_B2 = P_W2 + (int64_t)L2 * L1, P_W3 = P_B2 + L2, P_B3 = P_W3 + (int64_t)NOUT * L2,
                  P_TOTAL = P_B3 + NOUT;
// bf16 copies of the weight matrices: W1b | W2b | W3b
constexpr int64_t Q_W1 = 0, Q_W2 = Q_W1 + (int64_t)L1 * HBINS, Q_W3 = Q_W2 + (int64_t)L2 * L1,
                  Q_TOTAL = Q_W3 + (int64_t)NOUT * L2;

typedef uint16_t bf16_t;   // storage of bfloat16 values
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest even (inputs here are finite)
__device__ __forceinline__ bf16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// 32 x 32 occupancy histogram of each set (one block per set).  Sample: every
// stride-th point of the set, stride = ceil(n / 16384).  Bins cover a square
// window of side w = max(width, height) of the sample's bounding box (grid
// units), centred on the box, so that the set's aspect ratio and the angles
// of its features are kept: origin (x0 - (w - wx) / 2, y0 - (w - wy) / 2),
// bin = (k - origin) * 32 / w in integer arithmetic; value = count * 1024 / ns
// (binary64 product and quotient, then float, then bf16).
constexpr int HIST_THREADS = 1024;
constexpr int HPER = HSAMPLE / HIST_THREADS;    // samples per thread, held in registers
static_assert(HSAMPLE % HIST_THREADS == 0, "the samples split evenly over the threads");

__global__ __launch_bounds__(HIST_THREADS) void k_hist32(const float *__restrict__ x,
                                                         const float *__restrict__ y,
                                                         const int64_t *__restrict__ off, int64_t n1,
                                                         int64_t S, bf16_t *__restrict__ hist,
                                                         float *__restrict__ hist_f) {
    constexpr int NW = HIST_THREADS / WAVE;
    __shared__ uint32_t cnt[HBINS];
    __shared__ int32_t bb[NW][4];
    const int64_t s = blockIdx.x;
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    const int64_t a = set_begin(off, s), n = set_end(off, n1, s) - a;
    for (int b = tid; b < HBINS; b += blockDim.x) cnt[b] = 0;
    if (n <= 0) {
        __syncthreads();
        for (int b = tid; b < HBINS; b += blockDim.x) {
            hist[s * HBINS + b] = 0;
            if (hist_f) hist_f[s * HBINS + b] = 0.0f;
        }
        return;
    }
    // the sample: every point when n <= HSAMPLE, else HRUNS runs of WAVE
    // consecutive points, run r from floor(r (n - WAVE) / (HRUNS - 1)); each
    // sample loaded once, all of a thread's loads issued together (a wave
    // reads one run: whole cache lines)
    const int64_t ns = n <= HSAMPLE ? n : HSAMPLE;
    int32_t kx[HPER], ky[HPER];
#pragma unroll
    for (int i = 0; i < HPER; i++) {
        const int64_t j = tid + (int64_t)i * HIST_THREADS;
        const int64_t p = n <= HSAMPLE ? j : (j / WAVE) * (n - WAVE) / (HRUNS - 1) + j % WAVE;
        kx[i] = j < ns ? (int32_t)(x[a + p] * GRIDF) : 0;
        ky[i] = j < ns ? (int32_t)(y[a + p] * GRIDF) : 0;
    }
    int32_t x0 = 0x7fffffff, x1 = -1, y0 = 0x7fffffff, y1 = -1;
#pragma unroll
    for (int i = 0; i < HPER; i++) {
        if (tid + (int64_t)i * HIST_THREADS < ns) {
            x0 = min(x0, kx[i]); x1 = max(x1, kx[i]); y0 = min(y0, ky[i]); y1 = max(y1, ky[i]);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        x0 = min(x0, __shfl_xor(x0, o)); x1 = max(x1, __shfl_xor(x1, o));
        y0 = min(y0, __shfl_xor(y0, o)); y1 = max(y1, __shfl_xor(y1, o));
    }
    if (lane == 0) { bb[w][0] = x0; bb[w][1] = x1; bb[w][2] = y0; bb[w][3] = y1; }
    __syncthreads();
    x0 = bb[0][0]; x1 = bb[0][1]; y0 = bb[0][2]; y1 = bb[0][3];
    for (int ww = 1; ww < NW; ww++) {
        x0 = min(x0, bb[ww][0]); x1 = max(x1, bb[ww][1]);
        y0 = min(y0, bb[ww][2]); y1 = max(y1, bb[ww][3]);
    }
    const int64_t wx = (int64_t)x1 - x0 + 1, wy = (int64_t)y1 - y0 + 1, wd = max(wx, wy);
    const int64_t cx0 = x0 - (wd - wx) / 2, cy0 = y0 - (wd - wy) / 2;
    // bin = floor((k - c0) * 32 / wd): 0 <= k - c0 < wd <= 2^24, so the
    // product stays below 2^29 and a 32-bit division is exact
    const uint32_t uwd = (uint32_t)wd;
#pragma unroll
    for (int i = 0; i < HPER; i++) {
        if (tid + (int64_t)i * HIST_THREADS < ns) {
            const uint32_t bx = (uint32_t)((int64_t)kx[i] - cx0) * 32u / uwd;
            const uint32_t by = (uint32_t)((int64_t)ky[i] - cy0) * 32u / uwd;
            atomicAdd(&cnt[by * 32 + bx], 1u);
        }
    }
    __syncthreads();
    for (int b = tid; b < HBINS; b += blockDim.x) {
        float v = (float)((double)cnt[b] * 1024.0 / (double)ns);
        hist[s * HBINS + b] = f2bf(v);
        if (hist_f) hist_f[s * HBINS + b] = v;
    }
}

// ---------------------------------------------------------------------------
// C[M x N] = A[M x K] * B[K x N] in bf16 on MFMA (16x16x32), fp32 accumulate,
// with element (m, k) of A at A[m*sam + k*sak] and (k, n) of B at
// B[k*sbk + n*sbn].  M and N multiples of 64, K of 32.  Block: 64 x 64 tile,
// four waves of 32 x 32 (2 x 2 MFMA tiles each).  Epilogue by MODE.
enum GemmMode { G_RELU_BF16 = 0, G_BIAS_F32 = 1, G_MASK_BF16 = 2, G_F32 = 3 };
constexpr int GBM = 64, GBN = 64, GBK = 32, GPAD = 8;

template <int MODE>
__global__ __launch_bounds__(256) void k_gemm(const bf16_t *__restrict__ A, int64_t sam, int64_t sak,
                                              const bf16_t *__restrict__ B, int64_t sbk, int64_t sbn,
                                              int M, int N, int K, const float *__restrict__ bias,
                                              const bf16_t *__restrict__ mask,
                                              bf16_t *__restrict__ Cb, float *__restrict__ Cf,
                                              int ldc) {
    __shared__ __attribute__((aligned(16))) bf16_t As[GBM][GBK + GPAD];
    __shared__ __attribute__((aligned(16))) bf16_t Bs[GBN][GBK + GPAD];   // n-major
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
    const int wm = w >> 1, wn = w & 1;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lr = tid >> 2, lk = (tid & 3) * 8;     // loader: row / column and 8 k's
    for (int k0 = 0; k0 < K; k0 += GBK) {
        {
            const bf16_t *pa = A + (int64_t)(m0 + lr) * sam + (int64_t)(k0 + lk) * sak;
            if (sak == 1) {
                *reinterpret_cast<uint4 *>(&As[lr][lk]) = *reinterpret_cast<const uint4 *>(pa);
            } else {
#pragma unroll
                for (int t = 0; t < 8; t++) As[lr][lk + t] = pa[t * sak];
            }
            const bf16_t *pb = B + (int64_t)(k0 + lk) * sbk + (int64_t)(n0 + lr) * sbn;
            if (sbk == 1) {
                *reinterpret_cast<uint4 *>(&Bs[lr][lk]) = *reinterpret_cast<const uint4 *>(pb);
            } else {
#pragma unroll
                for (int t = 0; t < 8; t++) Bs[lr][lk + t] = pb[t * sbk];
            }
        }
        __syncthreads();
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; i++) {
            af[i] = *reinterpret_cast<const bf16x8 *>(&As[wm * 32 + i * 16 + (lane & 15)][(lane >> 4) * 8]);
            bfr[i] = *reinterpret_cast<const bf16x8 *>(&Bs[wn * 32 + i * 16 + (lane & 15)][(lane >> 4) * 8]);
        }
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int j = 0; j < 2; j++)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + r;
                const int n = n0 + wn * 32 + j * 16 + (lane & 15);
                float v = acc[i][j][r];
                const int64_t o = (int64_t)m * ldc + n;
                if (MODE == G_RELU_BF16) Cb[o] = f2bf(fmaxf(v + bias[n], 0.0f));
                else if (MODE == G_BIAS_F32) Cf[o] = v + bias[n];
                else if (MODE == G_MASK_BF16) Cb[o] = bf2f(mask[o]) > 0.0f ? f2bf(v) : (bf16_t)0;
                else Cf[o] = v;
            }
}

// Column sums of a bf16 matrix X[rows][cols] (bias gradients), fp32.
__global__ void k_colsum(const bf16_t *__restrict__ X, int rows, int cols, float *__restrict__ out) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float acc = 0.0f;
    for (int r = 0; r < rows; r++) acc += bf2f(X[(int64_t)r * cols + c]);
    out[c] = acc;
}

// float32 -> bf16 copy (weights after an update, or inputs)
__global__ void k_to_bf16(const float *__restrict__ src, int64_t n, bf16_t *__restrict__ dst) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = f2bf(src[i]);
}

// Copy (and zero-pad) histogram rows into the network's input matrix.
__global__ void k_pad_rows(const bf16_t *__restrict__ src, int64_t rows, int64_t rows_pad, int cols,
                           bf16_t *__restrict__ dst) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < rows_pad * cols;
         i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = (i / cols) < rows ? src[i] : (bf16_t)0;
}

// float32 rows -> zero-padded bf16 rows
__global__ void k_pad_f32_bf16(const float *__restrict__ src, int64_t rows, int64_t rows_pad,
                               int cols, bf16_t *__restrict__ dst) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < rows_pad * cols;
         i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = (i / cols) < rows ? f2bf(src[i]) : (bf16_t)0;
}

// Loss: targets t = gain / max(gain) per set (0 when no direction gains),
// L = mean over sets and directions of (score - t)^2.  dS = dL/dscore (bf16
// for the backward products); per-set partial losses for a fixed-order sum.
__global__ void k_loss(const float *__restrict__ scores, const float *__restrict__ gain, int64_t B,
                       int64_t Bp, bf16_t *__restrict__ dS, float *__restrict__ part) {
    const int64_t b = blockIdx.x;
    const int d = threadIdx.x;   // 64 threads
    float s = 0.0f, t = 0.0f;
    if (b < B) {
        float g = gain[b * NOUT + d];
        float mx = g;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
        t = mx > 0.0f ? g / mx : 0.0f;
        s = scores[b * NOUT + d];
    }
    float diff = b < B ? s - t : 0.0f;
    dS[b * NOUT + d] = f2bf(2.0f * diff / (float)(B * NOUT));
    float sq = diff * diff;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) sq += __shfl_xor(sq, o);
    if (d == 0) part[b] = sq;
    (void)Bp;
}

__global__ void k_loss_sum(const float *__restrict__ part, int64_t B, float *__restrict__ loss) {
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int64_t b = 0; b < B; b++) acc += part[b];
        *loss = (float)(acc / (double)(B * NOUT));
    }
}

// Adam on the float32 master parameters; refreshes the bf16 weight copies.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, bf16_t *__restrict__ wb) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        float gi = g[i];
        float mi = b1 * m[i] + (1.0f - b1) * gi;
        float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        int64_t q = -1;   // position of weight-matrix entries in the bf16 copy
        if (i < P_B1) q = Q_W1 + (i - P_W1);
        else if (i >= P_W2 && i < P_B2) q = Q_W2 + (i - P_W2);
        else if (i >= P_W3 && i < P_B3) q = Q_W3 + (i - P_W3);
        if (q >= 0) wb[q] = f2bf(wi);
    }
}

// Top eight of the 64 scores of each set (higher first, lower index on
// ties; NaN counts as -inf); their (cos, sin) go to set_dirs.  One wave per
// set, lane d holds direction d.  Scores are compared through an
// order-preserving integer image; a direction already taken ranks below all.
__device__ __forceinline__ int32_t score_rank(float v) {
    if (!(v == v)) v = -INFINITY;
    v = v + 0.0f;   // -0 ranks with +0
    uint32_t u = __float_as_uint(v);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return (int32_t)(u - 0x80000000u);
}

// Eight directions per set (one wave per set): repeatedly the highest score
// (lowest index on ties, NaN as -inf) among the directions still available;
// each pick removes itself and, for gap > 0, the directions within gap steps
// of it on the circle of 64, so that picks are at least gap + 1 steps apart.
// gap <= 3 always leaves eight picks.
__global__ void k_top8(const float *__restrict__ scores, int64_t S, int gap,
                       int32_t *__restrict__ dirs, double *__restrict__ set_dirs) {
    const int64_t s = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int d = lane_id();
    if (s >= S) return;
    int32_t key = score_rank(scores[s * NOUT + d]);
    for (int r = 0; r < MAX_DIRS; r++) {
        int32_t bk = key;
        int bi = d;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            int32_t k2 = __shfl_xor(bk, o);
            int i2 = __shfl_xor(bi, o);
            if (k2 > bk || (k2 == bk && i2 < bi)) { bk = k2; bi = i2; }
        }
        if (d == 0) {
            if (dirs) dirs[s * MAX_DIRS + r] = bi;
            set_dirs[(s * MAX_DIRS + r) * 2 + 0] = dCandCos[bi];
            set_dirs[(s * MAX_DIRS + r) * 2 + 1] = dCandSin[bi];
        }
        const int dist = min((d - bi) & (NOUT - 1), (bi - d) & (NOUT - 1));
        if (dist <= gap) key = INT32_MIN;
    }
}

// ---------------------------------------------------------------------------
// Training labels.
// (1) Extreme point of every set along each of the 64 candidate directions
//     (argmax of c*x + s*y, lowest index on ties); one block per set, eight
//     directions per pass.
__global__ __launch_bounds__(256) void k_cand_extremes(const float *__restrict__ x,
                                                       const float *__restrict__ y,
                                                       const int64_t *__restrict__ off,
                                                       int64_t n1, int64_t S,
                                                       uint32_t *__restrict__ cand) {
    __shared__ double rv[4][8];
    __shared__ uint32_t ri[4][8];
    const int64_t s = blockIdx.x;
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    const int64_t a = set_begin(off, s), e = set_end(off, n1, s);
    for (int d0 = 0; d0 < NCAND; d0 += 8) {
        double bv[8];
        uint32_t bi[8];
        double cc[8], ss[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
            bv[q] = -INFINITY;
            bi[q] = NONE;
            cc[q] = dCandCos[d0 + q];
            ss[q] = dCandSin[d0 + q];
        }
        for (int64_t i = a + tid; i < e; i += blockDim.x) {
            double xd = x[i], yd = y[i];
#pragma unroll
            for (int q = 0; q < 8; q++) {
                double v = proj_dir(cc[q], ss[q], xd, yd);
                if (v > bv[q]) { bv[q] = v; bi[q] = (uint32_t)i; }
            }
        }
#pragma unroll
        for (int q = 0; q < 8; q++) {
            double v = bv[q];
            uint32_t i = bi[q];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                double v2 = __shfl_xor(v, o);
                uint32_t i2 = __shfl_xor(i, o);
                if (i2 != NONE && (i == NONE || v2 > v || (v2 == v && i2 < i))) { v = v2; i = i2; }
            }
            if (lane == 0) { rv[w][q] = v; ri[w][q] = i; }
        }
        __syncthreads();
        if (tid < 8) {
            double v = rv[0][tid];
            uint32_t i = ri[0][tid];
            for (int ww = 1; ww < (int)(blockDim.x >> 6); ww++) {
                double v2 = rv[ww][tid];
                uint32_t i2 = ri[ww][tid];
                if (i2 != NONE && (i == NONE || v2 > v || (v2 == v && i2 < i))) { v = v2; i = i2; }
            }
            cand[s * NCAND + d0 + tid] = i;
        }
        __syncthreads();
    }
}

// (2) gain[s][d] = #{base survivors strictly inside hull(base polygon + e_d)}
//     / n.  One block per set; thread d < 64 builds the enlarged polygon of
//     direction d (Andrew's chain over the base vertices plus e_d), then all
//     threads count survivors against each polygon.
constexpr int LPV = FIXED_SLOTS + 1;   // vertices of an enlarged polygon

__global__ __launch_bounds__(256) void k_labels(const float *__restrict__ x,
                                                const float *__restrict__ y,
                                                const int64_t *__restrict__ off, int64_t n1,
                                                int64_t S, const Poly *__restrict__ polys,
                                                const uint32_t *__restrict__ cand,
                                                const uint32_t *__restrict__ surv,
                                                const int64_t *__restrict__ surv_off,
                                                float *__restrict__ gain) {
    __shared__ double bx[FIXED_SLOTS], by[FIXED_SLOTS];      // base vertices sorted by (x, y)
    __shared__ uint32_t bid[FIXED_SLOTS];
    __shared__ int nb;
    __shared__ double ex[NCAND][LPV], ey[NCAND][LPV], ec[NCAND][LPV];
    __shared__ int ne[NCAND];
    __shared__ uint32_t pcnt[4][NCAND];
    const int64_t s = blockIdx.x;
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    const int64_t a = set_begin(off, s), n = set_end(off, n1, s) - a;
    const Poly &P = polys[s];
    if (tid == 0) {
        int m = P.m;
        for (int i = 0; i < m; i++) {
            uint32_t id = P.verts[i];
            double gx = (double)x[id] * GRIDD, gy = (double)y[id] * GRIDD;
            int p = i;
            while (p > 0 && (bx[p - 1] > gx || (bx[p - 1] == gx && by[p - 1] > gy))) {
                bx[p] = bx[p - 1]; by[p] = by[p - 1]; bid[p] = bid[p - 1];
                p--;
            }
            bx[p] = gx; by[p] = gy; bid[p] = id;
        }
        nb = m;
    }
    __syncthreads();
    if (tid < NCAND) {
        const int d = tid;
        double px[LPV], py[LPV];
        int k = 0;
        uint32_t e = n > 0 ? cand[s * NCAND + d] : NONE;
        double gx = 0, gy = 0;
        bool ins = e != NONE;
        if (ins) { gx = (double)x[e] * GRIDD; gy = (double)y[e] * GRIDD; }
        for (int i = 0; i < nb; i++) {   // merge e_d into the sorted base vertices, no repeats
            if (ins && (gx < bx[i] || (gx == bx[i] && gy <= by[i]))) {
                if (!(gx == bx[i] && gy == by[i])) { px[k] = gx; py[k] = gy; k++; }
                ins = false;
            }
            px[k] = bx[i]; py[k] = by[i]; k++;
        }
        if (ins) { px[k] = gx; py[k] = gy; k++; }
        int st[2 * LPV + 2];
        int h = 0;
        if (k >= 3) {
            for (int j = 0; j < k; j++) {
                while (h >= 2 && orient(px[st[h - 2]], py[st[h - 2]], px[st[h - 1]], py[st[h - 1]],
                                        px[j], py[j]) <= 0)
                    h--;
                st[h++] = j;
            }
            int lo = h + 1;
            for (int j = k - 2; j >= 0; j--) {
                while (h >= lo && orient(px[st[h - 2]], py[st[h - 2]], px[st[h - 1]], py[st[h - 1]],
                                         px[j], py[j]) <= 0)
                    h--;
                st[h++] = j;
            }
            h--;
        }
        if (h < 3) h = 0;
        for (int i = 0; i < h; i++) {
            int p0 = st[i], p1 = st[(i + 1) % h];
            double ddx = px[p1] - px[p0], ddy = py[p1] - py[p0];
            ex[d][i] = ddx;
            ey[d][i] = ddy;
            ec[d][i] = fma(ddy, px[p0], -(ddx * py[p0]));
        }
        ne[d] = h;
    }
    __syncthreads();
    const int64_t sa = surv_off[s], sb = surv_off[s + 1];
    for (int d = 0; d < NCAND; d++) {
        const int m = ne[d];
        uint32_t c = 0;
        if (m >= 3) {
            for (int64_t j = sa + tid; j < sb; j += blockDim.x) {
                uint32_t id = surv[j];
                double qx = (double)x[id] * GRIDD, qy = (double)y[id] * GRIDD;
                bool in = true;
                for (int i = 0; i < m && in; i++) in = edge_eval(ex[d][i], ey[d][i], ec[d][i], qx, qy) > 0;
                c += in;
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
        if (lane == 0) pcnt[w][d] = c;
    }
    __syncthreads();
    if (tid < NCAND) {
        uint32_t c = 0;
        for (int ww = 0; ww < (int)(blockDim.x >> 6); ww++) c += pcnt[ww][tid];
        gain[s * NCAND + tid] = n > 0 ? (float)((double)c / (double)n) : 0.0f;
    }
}

// Greedy joint training targets (this project's extension).  One block per
// set.  V starts as the fixed filter's polygon vertices; each of R rounds
// adds the candidate extreme whose polygon hull(V + {e_d}) newly contains,
// strictly inside, the most of the fixed filter's survivors (ties: lowest
// d); a round whose best gain is zero ends the sequence.  Targets: the
// direction chosen in round r gets 1 - r / (2R); every other direction gets
// 0.5 g_d / g_max with g_d its round-0 gain (0 if g_max = 0).
constexpr int LT_MAXR = MAX_DIRS;
constexpr int LT_V = FIXED_SLOTS + LT_MAXR + 1;       // vertices of hull(V + {e_d})

// Edges of the convex hull of k points sorted by (x, y) without repeats
// (Andrew's monotone chain, collinear points dropped); returns the vertex
// count, or 0 when fewer than 3 vertices remain.
__device__ int hull_edges_sorted(const double *px, const double *py, int k, double *ex, double *ey,
                                 double *ec) {
    int st[2 * LT_V + 2];
    int h = 0;
    if (k >= 3) {
        for (int j = 0; j < k; j++) {
            while (h >= 2 && orient(px[st[h - 2]], py[st[h - 2]], px[st[h - 1]], py[st[h - 1]],
                                    px[j], py[j]) <= 0)
                h--;
            st[h++] = j;
        }
        const int lo = h + 1;
        for (int j = k - 2; j >= 0; j--) {
            while (h >= lo && orient(px[st[h - 2]], py[st[h - 2]], px[st[h - 1]], py[st[h - 1]],
                                     px[j], py[j]) <= 0)
                h--;
            st[h++] = j;
        }
        h--;
    }
    if (h < 3) return 0;
    for (int i = 0; i < h; i++) {
        const int p0 = st[i], p1 = st[(i + 1) % h];
        const double ddx = px[p1] - px[p0], ddy = py[p1] - py[p0];
        ex[i] = ddx;
        ey[i] = ddy;
        ec[i] = fma(ddy, px[p0], -(ddx * py[p0]));
    }
    return h;
}

// Insert (gx, gy) into the (x, y)-sorted list of k points unless it is
// already there; writes k' points to (ox, oy) and returns k'.
__device__ int merge_point(const double *vx, const double *vy, int k, double gx, double gy,
                           double *ox, double *oy) {
    int o = 0;
    bool ins = true;
    for (int i = 0; i < k; i++) {
        if (ins && (gx < vx[i] || (gx == vx[i] && gy <= vy[i]))) {
            if (!(gx == vx[i] && gy == vy[i])) { ox[o] = gx; oy[o] = gy; o++; }
            ins = false;
        }
        ox[o] = vx[i]; oy[o] = vy[i]; o++;
    }
    if (ins) { ox[o] = gx; oy[o] = gy; o++; }
    return o;
}

__global__ __launch_bounds__(256) void k_label_targets(
    const float *__restrict__ x, const float *__restrict__ y, const int64_t *__restrict__ off,
    int64_t n1, int64_t S, const Poly *__restrict__ polys, const uint32_t *__restrict__ cand,
    const uint32_t *__restrict__ surv, const int64_t *__restrict__ surv_off, int R,
    float *__restrict__ target, int32_t *__restrict__ order) {
    __shared__ double vx[LT_V], vy[LT_V];                  // current vertex set, sorted
    __shared__ int nv;
    __shared__ double ex[NCAND][LT_V], ey[NCAND][LT_V], ec[NCAND][LT_V];
    __shared__ int ne[NCAND];
    __shared__ double cex[LT_V], cey[LT_V], cec[LT_V];     // hull(V)
    __shared__ int cm;
    __shared__ uint32_t pcnt[4][NCAND];
    __shared__ uint32_t g0[NCAND];
    __shared__ int chosen[LT_MAXR];
    __shared__ int stop;
    const int64_t s = blockIdx.x;
    const int tid = threadIdx.x, lane = lane_id(), w = tid >> 6;
    const int64_t a = set_begin(off, s), n = set_end(off, n1, s) - a;
    const Poly &P = polys[s];
    if (tid == 0) {
        int k = 0;
        for (int i = 0; i < P.m; i++) {       // insertion sort by (x, y)
            const uint32_t id = P.verts[i];
            const double gx = (double)x[id] * GRIDD, gy = (double)y[id] * GRIDD;
            int p = k++;
            while (p > 0 && (vx[p - 1] > gx || (vx[p - 1] == gx && vy[p - 1] > gy))) {
                vx[p] = vx[p - 1]; vy[p] = vy[p - 1];
                p--;
            }
            vx[p] = gx; vy[p] = gy;
        }
        nv = k;
        stop = n <= 0;
    }
    if (tid < LT_MAXR) chosen[tid] = -1;
    __syncthreads();
    const int64_t sa = surv_off[s], sb = surv_off[s + 1];
    for (int r = 0; r < R && !stop; r++) {
        if (tid < NCAND) {
            const uint32_t e = cand[s * NCAND + tid];
            double px[LT_V], py[LT_V];
            int k = nv;
            if (e != NONE) {
                k = merge_point(vx, vy, nv, (double)x[e] * GRIDD, (double)y[e] * GRIDD, px, py);
            } else {
                for (int i = 0; i < nv; i++) { px[i] = vx[i]; py[i] = vy[i]; }
            }
            ne[tid] = hull_edges_sorted(px, py, k, ex[tid], ey[tid], ec[tid]);
        } else if (tid == NCAND) {
            cm = hull_edges_sorted(vx, vy, nv, cex, cey, cec);
        }
        __syncthreads();
        uint32_t cnt[NCAND];
#pragma unroll
        for (int d = 0; d < NCAND; d++) cnt[d] = 0;
        for (int64_t j = sa + tid; j < sb; j += blockDim.x) {
            const uint32_t id = surv[j];
            const double qx = (double)x[id] * GRIDD, qy = (double)y[id] * GRIDD;
            bool in = cm >= 3;
            for (int i = 0; i < cm && in; i++) in = edge_eval(cex[i], cey[i], cec[i], qx, qy) > 0;
            if (in) continue;                 // already inside hull(V): no candidate gains it
#pragma unroll
            for (int d = 0; d < NCAND; d++) {
                const int m = ne[d];
                bool ind = m >= 3;
                for (int i = 0; i < m && ind; i++) ind = edge_eval(ex[d][i], ey[d][i], ec[d][i], qx, qy) > 0;
                cnt[d] += ind;
            }
        }
#pragma unroll
        for (int d = 0; d < NCAND; d++) {
            uint32_t c = cnt[d];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
            if (lane == 0) pcnt[w][d] = c;
        }
        __syncthreads();
        if (tid == 0) {
            int best = -1;
            uint32_t bc = 0;
            for (int d = 0; d < NCAND; d++) {
                uint32_t c = 0;
                for (int ww = 0; ww < (int)(blockDim.x >> 6); ww++) c += pcnt[ww][d];
                if (r == 0) g0[d] = c;
                if (c > bc) { bc = c; best = d; }
            }
            if (best < 0) {
                stop = 1;
            } else {
                chosen[r] = best;
                const uint32_t e = cand[s * NCAND + best];
                double tx[LT_V], ty[LT_V];
                const int k = merge_point(vx, vy, nv, (double)x[e] * GRIDD, (double)y[e] * GRIDD, tx, ty);
                for (int i = 0; i < k; i++) { vx[i] = tx[i]; vy[i] = ty[i]; }
                nv = k;
            }
        }
        __syncthreads();
    }
    if (tid < NCAND) {
        uint32_t gmax = 0;
        bool g0_set = !(n <= 0);
        for (int d = 0; d < NCAND && g0_set; d++) gmax = max(gmax, g0[d]);
        float t = (g0_set && gmax > 0) ? (float)(0.5 * ((double)g0[tid] / (double)gmax)) : 0.0f;
        for (int r = 0; r < R; r++)
            if (chosen[r] == tid) t = (float)(1.0 - (double)r / (2.0 * R));
        target[s * NCAND + tid] = t;
    }
    if (tid < R) order[s * R + tid] = chosen[tid];
}

struct LearnedState {
    bool loaded = false;
    int64_t bcap = 0;          // rows the activation buffers hold
    int64_t step = 0;          // Adam step counter
    float *params = nullptr, *grads = nullptr, *m1 = nullptr, *m2 = nullptr;
    bf16_t *wb = nullptr;      // bf16 weight matrices
    bf16_t *X = nullptr, *H1 = nullptr, *H2 = nullptr, *dS = nullptr, *dZ2 = nullptr,
           *dZ1 = nullptr;
    float *scores = nullptr, *part = nullptr;
};

static size_t learned_ws_bytes(int64_t S) {
    return (size_t)S * HBINS * sizeof(bf16_t) + (size_t)S * NCAND * sizeof(float) + 256;
}

static void learned_free(LearnedState &L) {
    void *ps[] = {L.params, L.grads, L.m1, L.m2, L.wb, L.X, L.H1, L.H2, L.dS, L.dZ2, L.dZ1,
                  L.scores, L.part};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    L = LearnedState();
}

}  // namespace hg
