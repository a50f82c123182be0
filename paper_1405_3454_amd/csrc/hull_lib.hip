// C ABI of the library (include/hull.h): context, workspace planning and the
// launch sequences of every entry point.  The kernels are compiled into this
// translation unit so that the host code can launch every template directly.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/hull.h"
#include "hg_common.h"
#include "k_filter.hip"
#include "k_sort.hip"
#include "k_chain.hip"
#include "k_learned.hip"
#include "k_refine.hip"
#include "k_hull3d.hip"

using namespace hg;

// ---------------------------------------------------------------------------
// direction tables (host copies)
static const double H_C30 = 0x1.bb67ae8584caap-1;
static const double H_C45 = 0x1.6a09e667f3bcdp-1;
static const double H_C75 = 0x1.0907dc1930690p-2;
static const double H_S75 = 0x1.ee8dd4748bf15p-1;

static bool preset_valid(int preset) { return preset >= 0 && preset < NUM_PRESETS; }

static Dirs preset_dirs(int preset) {
    Dirs d = {};
    if (preset == HULL_DIRS_PAPER) {
        const double c[4] = {1.0, H_C30, H_C45, 0.5}, s[4] = {0.0, 0.5, H_C45, H_C30};
        for (int g = 0; g < 4; g++) { d.gc[g] = c[g]; d.gs[g] = s[g]; }
    } else if (preset == HULL_DIRS_CUMULATIVE) {
        const double c[4] = {1.0, H_C30, H_C75, -0.5}, s[4] = {0.0, 0.5, H_S75, H_C30};
        for (int g = 0; g < 4; g++) { d.gc[g] = c[g]; d.gs[g] = s[g]; }
    } else {
        // G evenly spaced groups: cos(90 j / G), sin(90 j / G) = cos(90 (G - j) / G)
        const int G = preset_groups(preset);
        for (int j = 0; j < G; j++) {
            d.gc[j] = EVEN_COS[G][j];
            d.gs[j] = EVEN_COS[G][G - j];
        }
    }
    return d;
}

// ---------------------------------------------------------------------------
// Launch shape of a persistent filter kernel: threads per block, blocks per
// CU (capped at what stays resident) and the fewest tiles (1024 points, 16
// per lane) a wave walks, which shrinks the grid for small inputs.
struct Shape {
    int bs, bpc, tpw;
};
constexpr int SHAPE_BS[3] = {128, 256, 512};
// Size buckets of the tuning table: points below 2^14, 2^17, 2^20, 2^23,
// 2^26 and above, each for one set and for batches.
constexpr int NSIZE = 6, NBUCKETS = 2 * NSIZE;
static int bucket_of(int64_t n, int64_t S) {
    int b = 0;
    while (b < NSIZE - 1 && n >= (int64_t(1) << (14 + 3 * b))) b++;
    return b + (S > 1 ? NSIZE : 0);
}

struct StreamBufs;                  // host-resident input path (hull_stream.hip)
static void stream_free(StreamBufs *b);
struct Hull3Bufs;                   // the 3D path (hull3d_host.hip)
static void hull3_free(Hull3Bufs *h);

struct hull_ctx {
    int device = 0;
    int preset = HULL_DIRS_PAPER;
    Dirs dirs;
    int dir_gap = 2;           // learned picks: minimum spacing - 1 on the circle of 64
    int cus = 256;
    hipError_t last = hipSuccess;
    char *ws = nullptr;
    size_t ws_cap = 0;
    char *scratch = nullptr;            // this device's copy of the fixed scratch array
    int64_t *counts = nullptr;          // candidates per stage of the last computation
    uint32_t *tickets = nullptr;        // last-block tickets (zero between launches)
    std::vector<char *> retired;        // old workspaces a graph may still use
    // launch shapes of the persistent filter kernels (extremes pass, discard
    // pass): defaults, and the autotuner's choices per size bucket
    Shape def[2] = {{256, 3, 1}, {256, 4, 1}};
    Shape tuned[2][NBUCKETS];
    bool has_tuned[2][NBUCKETS] = {};
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_pending;   // kind, index of start event
    double ms[K_NKINDS] = {};
    int64_t launches[K_NKINDS] = {};
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // learned proposal
    LearnedState learned;
    // host-resident input: chunk buffers, staging, copy stream
    StreamBufs *sb = nullptr;
    // the 3D path's buffers
    Hull3Bufs *h3 = nullptr;
};

// Slots of one set's extremes: the preset's fixed positions, then the
// learned directions.  Learned slots need a fixed table of at most 16.
static int slot_count(const hull_ctx *ctx, bool learned) {
    return preset_fixed_slots(ctx->preset) + (learned ? MAX_DIRS : 0);
}
static bool learned_ok(const hull_ctx *ctx) { return preset_fixed_slots(ctx->preset) == FIXED_SLOTS; }

static const char *kKindNames[K_NKINDS] = {
    "tile_map", "extremes", "polygon", "discard", "scan", "scatter", "keys",
    "sort_hist", "sort_scan", "sort_scatter", "chain", "chain_merge", "hull_final",
    "hull_lookup", "validate", "misc", "histogram32", "mlp", "labels", "refine_pass", "refine_split"};

#define HIPCHECK(expr)                                   \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) {                          \
            ctx->last = e_;                              \
            return HULL_EHIP;                            \
        }                                                \
    } while (0)

// Launch helper: records events around the launch when timing is on.
template <typename F>
static int launch(hull_ctx *ctx, int kind, hipStream_t st, F &&f) {
    size_t e0 = 0;
    if (ctx->timing && ctx->ev_used + 2 > ctx->ev_pool.size()) {
        size_t old = ctx->ev_pool.size();
        ctx->ev_pool.resize(old + 4096);
        for (size_t i = old; i < ctx->ev_pool.size(); i++)
            HIPCHECK(hipEventCreate(&ctx->ev_pool[i]));
    }
    if (ctx->timing && ctx->ev_used + 2 <= ctx->ev_pool.size()) {
        e0 = ctx->ev_used;
        ctx->ev_used += 2;
        HIPCHECK(hipEventRecord(ctx->ev_pool[e0], st));
    } else {
        e0 = SIZE_MAX;
    }
    f();
    HIPCHECK(hipGetLastError());
    if (e0 != SIZE_MAX) {
        HIPCHECK(hipEventRecord(ctx->ev_pool[e0 + 1], st));
        ctx->ev_pending.push_back({kind, e0});
    }
    return HULL_OK;
}

#define LAUNCH(kind, ...)                                                    \
    do {                                                                     \
        int rc_ = launch(ctx, kind, st, [&]() { __VA_ARGS__; });             \
        if (rc_) return rc_;                                                 \
    } while (0)

// ---------------------------------------------------------------------------
// Workspace plan.  All sizes are upper bounds derived from (n_total, S).
struct Plan {
    char *base = nullptr;   // device workspace the offsets below point into
    size_t tile_off, tile_set, pval, pidx, slots, vals, polys, spans, redges, masks, tile_cnt, tile_pos,
        scan_bs, surv_off, surv, keys0, keysA, keysB, lo0, up0, lo1, up1, ccnt, bounds, hcnt,
        hoff, hkeys, hpos, sstat, sgst, consts, err, setdirs, learn, cand, rtab0, rtab1, rfar0,
        rfar1, rfar2, segcnt, segmeta, cidx, ckeys, bpart, pticket, total;
    int64_t tcap, u0cap;
    int64_t nwave;      // discard waves = regions of the full method's survivor lists
};

static constexpr size_t al(size_t v) { return (v + 255) & ~size_t(255); }

static Plan make_plan(int64_t n, int64_t S, int64_t W) {
    Plan p;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += al(bytes);
        return r;
    };
    p.tcap = n / TILE + 2 * S + 2;
    p.u0cap = n / CHAIN_C + 2;
    p.nwave = W;
    // list entries: the discard pass's regions (q = ceil(T / W) tiles of
    // points per wave) end by T * TILE
    const size_t lcap = (size_t)std::max(n, p.tcap * TILE);
    p.tile_off = take((S + 1) * 8);
    p.tile_set = take(p.tcap * 4);
    p.pval = take(p.tcap * MAX_SLOTS * 8);
    p.pidx = take(p.tcap * MAX_SLOTS * 4);
    p.slots = take(S * MAX_SLOTS * 4);
    p.vals = take(S * MAX_SLOTS * 8);
    p.polys = take(S * sizeof(Poly));
    p.spans = take(S * SPAN_ROWS * sizeof(Span));
    p.redges = take(S * SPAN_ROWS * 4);
    p.masks = take(p.tcap * TILE_WORDS * 8);
    p.tile_cnt = take(p.tcap * 4);
    p.tile_pos = take((p.tcap + 1) * 8);
    p.scan_bs = take(SCAN_BLOCKS * 8);
    p.surv_off = take((S + 1) * 8);
    p.surv = take(lcap * 4 + 16);
    p.keys0 = take(lcap * 8 + 16);
    p.keysA = take(n * 8 + 16);
    p.keysB = take(n * 8 + 16);
    p.lo0 = take(lcap * 8 + 16);
    p.up0 = take(lcap * 8 + 16);
    p.lo1 = take(lcap * 8 + 16);
    p.up1 = take(lcap * 8 + 16);
    p.ccnt = take(4 * p.u0cap * 4);
    p.bounds = take(4 * S * 8);
    p.hcnt = take(S * 4);
    p.hoff = take((S + 1) * 8);
    p.hkeys = take(n * 8 + 16);
    p.hpos = take(n * 4 + 16);
    p.sstat = take(SORT_BLOCKS * RADIX * 8);                    // look-back entries of the ranges
    p.sgst = take(SORT_MAX_PASSES * (RADIX + 1) * 4);          // digit totals, range counters
    p.consts = take(8 * 8);
    p.err = take(8);
    p.setdirs = take(S * MAX_DIRS * 2 * 8);
    p.learn = take(learned_ws_bytes(S));
    p.cand = take(S * NCAND * 4);
    p.rtab0 = take(S * RE_CAP * sizeof(REdge));
    p.rtab1 = take(S * RE_CAP * sizeof(REdge));
    p.rfar0 = take(S * RE_CAP * 8);
    p.rfar1 = take(S * RE_CAP * 8);
    p.rfar2 = take(RE_CAP * 8);          // one set: third farthest-key buffer of the rounds
    p.bpart = take(S * POLY_SPLIT * MAX_SLOTS * sizeof(SlotBest));
    p.pticket = take(S * 4);
    p.cidx = take(n * 4 + 16);
    p.ckeys = take(n * 8 + 16);
    // last: the only entries whose size depends on the discard pass's waves
    p.segmeta = take(8);                             // region size (q * TILE)
    p.segcnt = take((REF_ROUNDS + 1) * W * 8);      // region counts per list stage
    p.total = o;
    return p;
}

// ---------------------------------------------------------------------------
// Allocation-free Step 1 (hull_extremes_noalloc).  Its buffers live in one
// fixed device array: each device that loads the library holds its own copy
// until the process ends, and no call allocates or frees device memory.
// Host code never uses the array's name as an address: hull_create looks up
// the device's copy with hipGetSymbolAddress (once per device) and every
// kernel gets that pointer.
constexpr int64_t NOALLOC_MAX_POINTS = HULL_NOALLOC_MAX_POINTS;
constexpr size_t NOALLOC_SCRATCH_BYTES = HULL_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

// Layout of Step 1 for one set of n points (tile map, run partials, the
// polygon kernel's shares and ticket, its polygon and rows); the other plan
// entries are unused by that path and stay 0.
static constexpr Plan make_plan_extremes(int64_t n) {
    Plan p{};
    size_t o = 0;
    p.tcap = n / TILE + 4;
    p.nwave = 0;
    p.tile_off = o; o += al(2 * 8);
    p.tile_set = o; o += al(p.tcap * 4);
    p.pval = o; o += al(p.tcap * MAX_SLOTS * 8);
    p.pidx = o; o += al(p.tcap * MAX_SLOTS * 4);
    p.polys = o; o += al(sizeof(Poly));
    p.spans = o; o += al(SPAN_ROWS * sizeof(Span));
    p.redges = o; o += al(SPAN_ROWS * 4);
    p.setdirs = o; o += al(MAX_DIRS * 2 * 8);
    p.bpart = o; o += al(POLY_SPLIT * MAX_SLOTS * sizeof(SlotBest));
    p.pticket = o; o += al(4);
    p.total = o;
    return p;
}
static_assert(make_plan_extremes(NOALLOC_MAX_POINTS).total <= NOALLOC_SCRATCH_BYTES,
              "the scratch array must hold Step 1 at the largest accepted size");

// Per-device address of `scratch`, looked up once per device.
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[256];

static int scratch_setup(int device, char **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= 256) return HULL_EINVAL;
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        // the caller has made `device` current
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return HULL_EHIP;
        }
        g_scratch_ptr[device] = static_cast<char *>(ptr);
    }
    *out = g_scratch_ptr[device];
    return HULL_OK;
}

static int ensure_ws(hull_ctx *ctx, size_t bytes, hipStream_t st) {
    if (bytes <= ctx->ws_cap) return HULL_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHECK(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) return HULL_ECAPTURE;
    HIPCHECK(hipDeviceSynchronize());
    // a captured graph holds pointers into the old workspace: keep it alive
    // until the graph is replaced or the context destroyed
    if (ctx->ws && ctx->gexec) ctx->retired.push_back(ctx->ws);
    else if (ctx->ws) HIPCHECK(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_cap = 0;
    size_t want = bytes + bytes / 8;
    if (hipMalloc(&ctx->ws, want) != hipSuccess) {
        ctx->ws = nullptr;
        (void)hipGetLastError();
        return HULL_ENOMEM;
    }
    ctx->ws_cap = want;
    return HULL_OK;
}

// Buffer at offset `off` of the plan's workspace.
template <typename T>
static T *W(const Plan &p, size_t off) {
    return reinterpret_cast<T *>(p.base + off);
}

static int check_points(const float *x, const float *y, int64_t n) {
    if (n < 0) return HULL_EINVAL;
    if (n >= (int64_t(1) << 32) - 1) return HULL_ETOOBIG;
    if (n > 0 && (!x || !y)) return HULL_EINVAL;
    if (((uintptr_t)x & 3) || ((uintptr_t)y & 3) || (((uintptr_t)x ^ (uintptr_t)y) & 15))
        return HULL_EINVAL;
    return HULL_OK;
}

// Position of x[0] within its 16-byte block, in floats: the filter passes
// align their tiles to absolute 16-byte boundaries.
static int phase_of(const float *x) { return (int)(((uintptr_t)x >> 2) & 3); }

// The extremes pass instantiated for a preset (learned: with eight learned
// directions) and block size, as a host handle for occupancy queries.
template <int PR, int ND>
static const void *k1_fn(int bs) {
    switch (bs) {
    case 128: return (const void *)k_extremes<PR, ND, 128>;
    case 512: return (const void *)k_extremes<PR, ND, 512>;
    default: return (const void *)k_extremes<PR, ND, 256>;
    }
}
static const void *k1_kernel(int preset, bool learned, int bs) {
    switch (preset) {
    case 0: return learned ? k1_fn<0, MAX_DIRS>(bs) : k1_fn<0, 0>(bs);
    case 1: return learned ? k1_fn<1, MAX_DIRS>(bs) : k1_fn<1, 0>(bs);
    case 2: return learned ? k1_fn<2, MAX_DIRS>(bs) : k1_fn<2, 0>(bs);
    case 3: return learned ? k1_fn<3, MAX_DIRS>(bs) : k1_fn<3, 0>(bs);
    case 4: return learned ? k1_fn<4, MAX_DIRS>(bs) : k1_fn<4, 0>(bs);
    case 5: return learned ? k1_fn<5, MAX_DIRS>(bs) : k1_fn<5, 0>(bs);
    case 6: return k1_fn<6, 0>(bs);
    case 7: return k1_fn<7, 0>(bs);
    default: return nullptr;
    }
}
// The full method's discard pass at a block size (all its modes share the
// register cap of 4 waves per SIMD).
static const void *k3_kernel(int bs) {
    switch (bs) {
    case 128: return (const void *)k_discard<FIXED_SLOTS, DISCARD_ASSIGN, 128>;
    case 512: return (const void *)k_discard<FIXED_SLOTS, DISCARD_ASSIGN, 512>;
    default: return (const void *)k_discard<FIXED_SLOTS, DISCARD_ASSIGN, 256>;
    }
}

// Blocks of bs threads per CU that stay resident for a kernel (its register
// and LDS use), cached per (kernel, block size) in a fixed table that
// hull_create fills for every filter variant, so later calls neither query
// nor allocate; 1 if the query fails.
static int resident_blocks(const void *fn, int bs) {
    static std::mutex mu;
    constexpr int CAP = 128;
    static const void *keys[CAP];
    static int kbs[CAP], vals[CAP];
    static int used = 0;
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < used; i++)
        if (keys[i] == fn && kbs[i] == bs) return vals[i];
    int b = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, bs, 0) != hipSuccess || b < 1) {
        (void)hipGetLastError();
        b = 1;
    }
    if (used < CAP) {
        keys[used] = fn;
        kbs[used] = bs;
        vals[used] = b;
        used++;
    }
    return b;
}

// Grid of a persistent filter kernel for n points in S sets: the bucket's
// shape, blocks per CU capped at what stays resident (the extremes variants
// hold 100 to 254 VGPRs: 2 to 4 waves per SIMD), and no more waves than
// give each its tpw tiles.
struct Launch {
    int bs;
    unsigned blocks;
    int64_t waves;
};
static Shape shape_of(const hull_ctx *ctx, int kind, int64_t n, int64_t S) {
    const int b = bucket_of(n, S);
    return ctx->has_tuned[kind][b] ? ctx->tuned[kind][b] : ctx->def[kind];
}
static Launch make_launch(const hull_ctx *ctx, const Shape &sh, const void *fn, int64_t n, int64_t S) {
    const int wpb = sh.bs / WAVE;
    const int bpc = std::min(sh.bpc, resident_blocks(fn, sh.bs));
    int64_t blocks = (int64_t)ctx->cus * bpc;
    const int64_t tiles = n / TILE + 2 * S + 2;           // upper bound of the tile count
    const int64_t want = (tiles + sh.tpw - 1) / sh.tpw;   // waves with tpw tiles each
    blocks = std::max<int64_t>(1, std::min(blocks, (want + wpb - 1) / wpb));
    return Launch{sh.bs, (unsigned)blocks, blocks * wpb};
}
static Launch k1_launch(const hull_ctx *ctx, int64_t n, int64_t S, bool learned) {
    const Shape sh = shape_of(ctx, 0, n, S);
    return make_launch(ctx, sh, k1_kernel(ctx->preset, learned && learned_ok(ctx), sh.bs), n, S);
}
static Launch k3_launch(const hull_ctx *ctx, int64_t n, int64_t S) {
    const Shape sh = shape_of(ctx, 1, n, S);
    return make_launch(ctx, sh, k3_kernel(sh.bs), n, S);
}
// Regions of the full method's survivor lists: one per discard wave for one
// set; for several sets DYN_REGIONS per wave, which the waves take in turn
// (the sets' tiles differ in cost, so equal shares would leave waves idle).
constexpr int DYN_REGIONS = 4;
static int64_t regions_for(int64_t waves, int64_t S) { return waves * (S > 1 ? DYN_REGIONS : 1); }
static int64_t region_count(const hull_ctx *ctx, int64_t n, int64_t S) {
    return regions_for(k3_launch(ctx, n, S).waves, S);
}

// ---------------------------------------------------------------------------
// Launch sequences

// Exclusive scan of u32 counts (count at *cnt) into out[0..count] (int64).
static int run_scan(hull_ctx *ctx, const Plan &p, hipStream_t st, const uint32_t *in,
                    const int64_t *cnt, int64_t *out) {
    int64_t *bs = W<int64_t>(p, p.scan_bs);
    LAUNCH(K_SCAN, k_scan_reduce<<<SCAN_BLOCKS, SCAN_THREADS, 0, st>>>(in, cnt, bs, out,
                                                                       ctx->tickets + 0));
    LAUNCH(K_SCAN, k_scan_down<<<SCAN_BLOCKS, SCAN_THREADS, 0, st>>>(in, cnt, bs, out));
    return HULL_OK;
}

static int run_validate(hull_ctx *ctx, const Plan &p, hipStream_t st, const float *x,
                        const float *y, int64_t n, const int64_t *off, int64_t S) {
    int *err = W<int>(p, p.err);
    LAUNCH(K_VALIDATE, k_fill_i64<<<1, 64, 0, st>>>(reinterpret_cast<int64_t *>(err), 1, 0));
    LAUNCH(K_VALIDATE, k_validate<<<1024, 256, 0, st>>>(x, y, n, off, S, err));
    int h = 0;
    HIPCHECK(hipMemcpyAsync(&h, err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    return h ? HULL_EDOMAIN : HULL_OK;
}

static int run_tilemap(hull_ctx *ctx, const Plan &p, hipStream_t st, const float *x,
                       const int64_t *off, int64_t n1, int64_t S) {
    int64_t *tile_off = W<int64_t>(p, p.tile_off);
    LAUNCH(K_TILEMAP, k_tile_offsets<<<1, 1024, 0, st>>>(off, n1, S, TILE, phase_of(x), tile_off,
                                                         W<uint32_t>(p, p.pticket)));
    LAUNCH(K_TILEMAP, k_tile_sets<<<(unsigned)std::min<int64_t>(ctx->cus * 4, (p.tcap + 255) / 256), 256,
                                     0, st>>>(tile_off, S, W<int32_t>(p, p.tile_set)));
    return HULL_OK;
}

// Launch the extremes pass / discard pass at a block size.
template <int PR, int ND, typename... A>
static void launch_k1(const Launch &L, hipStream_t st, A... a) {
    switch (L.bs) {
    case 128: k_extremes<PR, ND, 128><<<L.blocks, 128, 0, st>>>(a...); break;
    case 512: k_extremes<PR, ND, 512><<<L.blocks, 512, 0, st>>>(a...); break;
    default: k_extremes<PR, ND, 256><<<L.blocks, 256, 0, st>>>(a...); break;
    }
}
template <int NE, int MODE, typename... A>
static void launch_k3(const Launch &L, hipStream_t st, A... a) {
    switch (L.bs) {
    case 128: k_discard<NE, MODE, 128><<<L.blocks, 128, 0, st>>>(a...); break;
    case 512: k_discard<NE, MODE, 512><<<L.blocks, 512, 0, st>>>(a...); break;
    default: k_discard<NE, MODE, 256><<<L.blocks, 256, 0, st>>>(a...); break;
    }
}

// Step 1 (+ partial reduction and polygon in k_polygon).
static int run_extremes(hull_ctx *ctx, const Plan &p, hipStream_t st, const float *x,
                        const float *y, int64_t n_total, const int64_t *off, int64_t n1,
                        int64_t S, bool learned) {
    const int64_t *tile_off = W<int64_t>(p, p.tile_off);
    const int32_t *tile_set = W<int32_t>(p, p.tile_set);
    double *pval = W<double>(p, p.pval);
    uint32_t *pidx = W<uint32_t>(p, p.pidx);
    const double *sd = W<double>(p, p.setdirs);
    const Launch L = k1_launch(ctx, n_total, S, learned);
    const Dirs d = ctx->dirs;
#define K1(PR, ND)                                                                           \
    LAUNCH(K_EXTREMES, (launch_k1<PR, ND>(L, st, x, y, n_total, phase_of(x), off, n1, S,      \
                                          tile_off, tile_set, d, sd, pval, pidx)))
    if (learned && !learned_ok(ctx)) return HULL_EINVAL;
    switch (ctx->preset) {
    case 0: if (learned) K1(0, MAX_DIRS); else K1(0, 0); break;
    case 1: if (learned) K1(1, MAX_DIRS); else K1(1, 0); break;
    case 2: if (learned) K1(2, MAX_DIRS); else K1(2, 0); break;
    case 3: if (learned) K1(3, MAX_DIRS); else K1(3, 0); break;
    case 4: if (learned) K1(4, MAX_DIRS); else K1(4, 0); break;
    case 5: if (learned) K1(5, MAX_DIRS); else K1(5, 0); break;
    case 6: K1(6, 0); break;
    case 7: K1(7, 0); break;
    default: return HULL_EINVAL;
    }
#undef K1
    return HULL_OK;
}

static int run_polygon(hull_ctx *ctx, const Plan &p, hipStream_t st, const float *x,
                       const float *y, int64_t n_total, int64_t S, bool learned, const uint32_t *slots_in,
                       int n_in, uint32_t *slots_out, double *vals_out, bool ref_init = false) {
    REdge *rtab = ref_init ? W<REdge>(p, p.rtab0) : nullptr;
    unsigned long long *rfar = ref_init ? W<unsigned long long>(p, p.rfar0) : nullptr;
    const int64_t W1 = k1_launch(ctx, n_total, S, learned).waves;   // the extremes pass's waves
    auto *polys = W<Poly>(p, p.polys);
    auto *spans = W<Span>(p, p.spans);
    const double *sd = W<double>(p, p.setdirs);
    // blocks per set sharing the reduction of the extremes partials: about one
    // per POLY_THREADS of the set's runs (W1 / S on average)
    const unsigned split = slots_in ? 1u
        : (unsigned)std::max<int64_t>(1, std::min<int64_t>(POLY_SPLIT, W1 / (S * POLY_THREADS / 16)));
#define K2(PR, ND)                                                                            \
    LAUNCH(K_POLYGON, k_polygon<PR, ND><<<dim3((unsigned)S, split), POLY_THREADS, 0, st>>>(      \
        x, y, n_total, S, W<int64_t>(p, p.tile_off), W1, W<double>(p, p.pval),             \
        W<uint32_t>(p, p.pidx), slots_in, n_in, ctx->dirs, sd, slots_out, vals_out, polys,  \
        spans, W<uint32_t>(p, p.redges), rtab, rfar, W<SlotBest>(p, p.bpart),             \
        W<uint32_t>(p, p.pticket)))
    if (learned && !learned_ok(ctx)) return HULL_EINVAL;
    switch (ctx->preset) {
    case 0: if (learned) K2(0, MAX_DIRS); else K2(0, 0); break;
    case 1: if (learned) K2(1, MAX_DIRS); else K2(1, 0); break;
    case 2: if (learned) K2(2, MAX_DIRS); else K2(2, 0); break;
    case 3: if (learned) K2(3, MAX_DIRS); else K2(3, 0); break;
    case 4: if (learned) K2(4, MAX_DIRS); else K2(4, 0); break;
    case 5: if (learned) K2(5, MAX_DIRS); else K2(5, 0); break;
    case 6: K2(6, 0); break;
    case 7: K2(7, 0); break;
    default: return HULL_EINVAL;
    }
#undef K2
    // row-group blocks per set: all 16 for a few sets, one for thousands
    const unsigned ny = (unsigned)std::max<int64_t>(1, std::min<int64_t>(SPAN_ROWS / ROWS_PER_BLOCK,
                                                                         (2 * ctx->cus + S - 1) / S));
    LAUNCH(K_POLYGON, k_rows<<<dim3((unsigned)S, ny), 256, 0, st>>>(polys, spans, W<uint32_t>(p, p.redges)));
    return HULL_OK;
}

// Step 3 + compaction.  surv_off gets the per-set survivor offsets (S+1);
// keys (optional) the sort keys of the survivors.
// out_base (optional, device): append after that many entries of surv/keys,
// writing no entry at or past cap.
static int run_discard(hull_ctx *ctx, const Plan &p, hipStream_t st, const float *x,
                       const float *y, int64_t n_total, const int64_t *off, int64_t n1,
                       int64_t S, int nedge, uint32_t *surv, int64_t *surv_off, uint64_t *keys,
                       const int64_t *out_base = nullptr, int64_t cap = INT64_MAX) {
    const int64_t *tile_off = W<int64_t>(p, p.tile_off);
    const int32_t *tile_set = W<int32_t>(p, p.tile_set);
    auto *polys = W<Poly>(p, p.polys);
    auto *spans = W<Span>(p, p.spans);
    const uint32_t *redges = W<uint32_t>(p, p.redges);
    uint64_t *masks = W<uint64_t>(p, p.masks);
    uint32_t *tcnt = W<uint32_t>(p, p.tile_cnt);
    int64_t *tpos = W<int64_t>(p, p.tile_pos);
    const Launch L = k3_launch(ctx, n_total, S);
    const unsigned g = (unsigned)std::max<int64_t>(1, (L.waves + 3) / 4);   // scatter blocks: as many waves
    uint32_t *nu = nullptr;
    uint64_t *nk = nullptr;
    uint16_t *ne = nullptr;
    int64_t *nc = nullptr, *nm = nullptr;
    unsigned long long *nf = nullptr;
    if (nedge <= FIXED_SLOTS)
        LAUNCH(K_DISCARD, (launch_k3<FIXED_SLOTS, DISCARD_MASKS>(
            L, st, x, y, n_total, phase_of(x), off, n1, S, tile_off, tile_set, polys, spans, redges,
            masks, tcnt, nu, nk, ne, nc, nm, nf, L.waves, nullptr)));
    else
        LAUNCH(K_DISCARD, (launch_k3<MAX_SLOTS, DISCARD_MASKS>(
            L, st, x, y, n_total, phase_of(x), off, n1, S, tile_off, tile_set, polys, spans, redges,
            masks, tcnt, nu, nk, ne, nc, nm, nf, L.waves, nullptr)));
    int rc = run_scan(ctx, p, st, tcnt, tile_off + S, tpos);
    if (rc) return rc;
    LAUNCH(K_SCATTER, k_set_offsets<<<(unsigned)((S + 256) / 256), 256, 0, st>>>(tile_off, tpos, S,
                                                                                  surv_off));
    LAUNCH(K_SCATTER, k_scatter<<<g, 256, 0, st>>>(x, y, n_total, phase_of(x), off, S, tile_off, tile_set, masks, tcnt,
                                                   tpos, surv, keys, out_base, cap));
    return HULL_OK;
}

// Step 3 for the full method: survivors written to the regions of
// (surv, keys[, edges]) -- one per discard wave for one set, DYN_REGIONS per
// wave for several sets, taken by the waves in turn from a counter --,
// region counts to seg_cnt[p.nwave] and the region size to segmeta[0]; with
// gfar, also the refinement's round-0 edge states and farthest points.
static int run_discard_append(hull_ctx *ctx, const Plan &p, hipStream_t st, const float *x,
                              const float *y, int64_t n_total, const int64_t *off, int64_t n1,
                              int64_t S, int nedge, uint32_t *surv, uint64_t *keys,
                              uint16_t *edges, int64_t *seg_cnt, unsigned long long *gfar) {
    const int64_t *tile_off = W<int64_t>(p, p.tile_off);
    const int32_t *tile_set = W<int32_t>(p, p.tile_set);
    auto *polys = W<Poly>(p, p.polys);
    auto *spans = W<Span>(p, p.spans);
    const uint32_t *redges = W<uint32_t>(p, p.redges);
    int64_t *meta = W<int64_t>(p, p.segmeta);
    const Launch L = k3_launch(ctx, n_total, S);
    if (region_count(ctx, n_total, S) != p.nwave) return HULL_EINVAL;   // the plan's regions
    const int ph = phase_of(x);
    uint64_t *nmask = nullptr;
    uint32_t *ncnt = nullptr;
    int *ctr = nullptr;
    if (S > 1) {       // regions handed out by a counter, cleared by a kernel (graph-safe)
        ctr = reinterpret_cast<int *>(W<int64_t>(p, p.consts) + 3);
        LAUNCH(K_MISC, k_fill_i64<<<1, 64, 0, st>>>(W<int64_t>(p, p.consts) + 3, 1, 0));
    }
#define K3A(NE, MODE)                                                                             \
    LAUNCH(K_DISCARD, (launch_k3<NE, MODE>(L, st, x, y, n_total, ph, off, n1, S, tile_off,       \
                                           tile_set, polys, spans, redges, nmask, ncnt, surv,    \
                                           keys, edges, seg_cnt, meta, gfar, p.nwave, ctr)))
    if (gfar) {
        if (nedge <= FIXED_SLOTS) K3A(FIXED_SLOTS, DISCARD_ASSIGN);
        else K3A(MAX_SLOTS, DISCARD_ASSIGN);
    } else {
        if (nedge <= FIXED_SLOTS) K3A(FIXED_SLOTS, DISCARD_APPEND);
        else K3A(MAX_SLOTS, DISCARD_APPEND);
    }
#undef K3A
    return HULL_OK;
}

static int sort_passes(int64_t S) {
    int setbits = 0;
    while (setbits < 16 && (int64_t(1) << setbits) < S) setbits++;
    return (48 + setbits + 7) / 8;
}

// Sort keys (count at *cnt) ascending; returns the buffer holding the result.
// Several sets (S > 1): the keys arrive grouped by set in set order, and each
// set is sorted alone in LDS; the radix passes run only when that is not so
// or a set is too large for it.
static int run_sort(hull_ctx *ctx, const Plan &p, hipStream_t st, const uint64_t *keys,
                    const int64_t *cnt, int passes, int64_t S, const uint64_t **sorted) {
    if (passes > SORT_MAX_PASSES) return HULL_EINVAL;
    uint64_t *A = W<uint64_t>(p, p.keysA), *B = W<uint64_t>(p, p.keysB);
    unsigned long long *status = W<unsigned long long>(p, p.sstat);
    uint32_t *gst = W<uint32_t>(p, p.sgst);
    int *seg = S > 1 ? reinterpret_cast<int *>(W<int64_t>(p, p.consts) + 4) : nullptr;
    const uint64_t *in = keys;
    uint64_t *out = A;
    uint64_t *fin = passes % 2 ? A : B;        // where the last pass leaves the keys
    // small counts: sorted at once into that buffer; otherwise the passes'
    // state is cleared (and the sets' fallback flag)
    LAUNCH(K_SORT_HIST, k_sort_small<<<1 + SMALL_CLEAR_BLOCKS, SMALL_THREADS, 0, st>>>(
        keys, cnt, fin, status, gst, seg));
    if (seg) {
        int64_t *starts = W<int64_t>(p, p.bounds);    // S + 1 entries (the final stage rewrites it)
        LAUNCH(K_SORT_HIST, k_set_starts<<<(unsigned)ctx->cus * 4, 256, 0, st>>>(keys, cnt, S, starts, seg));
        LAUNCH(K_SORT_HIST, k_sort_sets<<<(unsigned)std::min<int64_t>(S, (int64_t)ctx->cus * 2), SEG_THREADS, 0,
                                          st>>>(keys, cnt, S, starts, fin, seg));
    }
    LAUNCH(K_SORT_HIST, k_sort_prep<<<SORT_BLOCKS, SORT_THREADS, 0, st>>>(keys, cnt, passes, gst, seg));
    for (int ps = 0; ps < passes; ps++) {
        LAUNCH(K_SORT_SCATTER, k_sort_pass<<<SORT_BLOCKS, SORT_THREADS, 0, st>>>(
            in, cnt, ps, gst, status, gst + SORT_MAX_PASSES * RADIX + ps, out, seg));
        in = out;
        out = (out == A) ? B : A;
    }
    *sorted = in;
    return HULL_OK;
}

static int chain_levels(int64_t ncap) {
    int64_t u = (ncap + CHAIN_C - 1) / CHAIN_C;
    int L = 0;
    int64_t span = 1;
    while (span < u) {
        span *= CHAIN_G;
        L++;
    }
    return L;
}

// Hull of the candidates (idx[i], keys[i]) i < *cnt, grouped into S sets by
// the key's set field.  hoff (S+1) receives the per-set hull offsets, hull
// the vertex indices, *h_out (optional) the total hull size.
static int run_hull(hull_ctx *ctx, const Plan &p, hipStream_t st, const uint32_t *idx,
                    const uint64_t *keys, const int64_t *cnt, int64_t ncap, int64_t S,
                    int64_t *hoff, uint32_t *hull, int64_t *h_out = nullptr) {
    const uint64_t *sorted = nullptr;
    int rc = run_sort(ctx, p, st, keys, cnt, sort_passes(S), S, &sorted);
    if (rc) return rc;
    uint64_t *lo[2] = {W<uint64_t>(p, p.lo0), W<uint64_t>(p, p.lo1)};
    uint64_t *up[2] = {W<uint64_t>(p, p.up0), W<uint64_t>(p, p.up1)};
    uint32_t *cc = W<uint32_t>(p, p.ccnt);
    uint32_t *locnt[2] = {cc, cc + p.u0cap};
    uint32_t *upcnt[2] = {cc + 2 * p.u0cap, cc + 3 * p.u0cap};
    const int64_t u0 = (ncap + CHAIN_C - 1) / CHAIN_C;
    const int64_t gmax = (int64_t)ctx->cus * 4;       // blocks of 4 waves; kernels loop
    int *big = S > 1 ? reinterpret_cast<int *>(W<int64_t>(p, p.consts) + 2) : nullptr;
    LAUNCH(K_CHAIN, k_chain_chunks<<<(unsigned)std::min(gmax, std::max<int64_t>(1, (u0 + 3) / 4)), 256, 0, st>>>(
        sorted, cnt, lo[0], up[0], locnt[0], upcnt[0], big));
    int L = chain_levels(ncap);
    if (S > 1) {
        // several sets: each set's chain from its own chunk pieces into
        // buffer 1; a set of too many pieces raises *big, and the levels
        // below (which return at once otherwise) merge every chain into
        // buffer 1 instead (an odd number of levels ends there)
        const int64_t gs = std::min<int64_t>(gmax, (S + 3) / 4);
        LAUNCH(K_CHAIN_COMPACT, k_chain_sets<<<dim3((unsigned)gs, 2), 256, 0, st>>>(
            sorted, cnt, S, lo[0], up[0], locnt[0], upcnt[0], lo[1], up[1], locnt[1], upcnt[1], big,
            W<int64_t>(p, p.bounds), reinterpret_cast<const int *>(W<int64_t>(p, p.consts) + 4)));
        if (L % 2 == 0) L++;
    }
    int cur = 0;
    int64_t R = CHAIN_C;
    for (int lev = 0; lev < L; lev++) {
        int64_t ucap = (ncap + R - 1) / R;
        int64_t vcap = (ucap + CHAIN_G - 1) / CHAIN_G;
        // one block per CU at most (each stages 4 x 32 KB in LDS, so no
        // second one fits); the waves loop over the groups the count has
        const int64_t mcap = std::max<int64_t>(1, (int64_t)ctx->cus / 2);
        dim3 grid((unsigned)std::min(mcap, std::max<int64_t>(1, (vcap + 3) / 4)), 2);
        LAUNCH(K_CHAIN_COMPACT, k_chain_merge<<<grid, 256, 0, st>>>(
            lo[cur], up[cur], locnt[cur], upcnt[cur], cnt, lev, L, lo[1 - cur], up[1 - cur],
            locnt[1 - cur], upcnt[1 - cur], big));
        cur = 1 - cur;
        R *= CHAIN_G;
    }
    int64_t *bounds = W<int64_t>(p, p.bounds);
    uint32_t *hcnt = W<uint32_t>(p, p.hcnt);
    uint64_t *hkeys = W<uint64_t>(p, p.hkeys);
    uint32_t *hpos = W<uint32_t>(p, p.hpos);
    if (S == 1) {
        LAUNCH(K_FINAL, k_hull_final1<<<1, 1024, 0, st>>>(lo[cur], up[cur], locnt[cur], upcnt[cur],
                                                          hoff, hkeys, hpos, hull, h_out));
        LAUNCH(K_LOOKUP, k_hull_lookup<<<2048, 256, 0, st>>>(idx, keys, cnt, S, hoff, hkeys, hpos, hull));
        return HULL_OK;
    }
    int64_t *scount = W<int64_t>(p, p.consts) + 1;   // = S
    LAUNCH(K_FINAL, k_fill_i64<<<64, 256, 0, st>>>(bounds, 4 * S, 0));
    LAUNCH(K_FINAL, k_fill_i64<<<1, 64, 0, st>>>(scount, 1, S));
    LAUNCH(K_FINAL, k_seg_bounds<<<dim3(256, 2), 256, 0, st>>>(lo[cur], up[cur], locnt[cur],
                                                               upcnt[cur], bounds, S));
    LAUNCH(K_FINAL, k_hull_counts<<<(unsigned)((S + 255) / 256), 256, 0, st>>>(bounds, S, hcnt));
    rc = run_scan(ctx, p, st, hcnt, scount, hoff);
    if (rc) return rc;
    LAUNCH(K_FINAL, k_hull_emit<<<dim3(256, 2), 256, 0, st>>>(lo[cur], up[cur], locnt[cur],
                                                              upcnt[cur], bounds, S, hoff, hkeys,
                                                              hpos, hull));
    LAUNCH(K_LOOKUP, k_hull_lookup<<<2048, 256, 0, st>>>(idx, keys, cnt, S, hoff, hkeys, hpos, hull));
    if (h_out) LAUNCH(K_MISC, k_copy_count<<<1, 64, 0, st>>>(hoff + S, h_out));
    return HULL_OK;
}

// Refinement rounds on the segmented survivor list (surv, keys0, round-0
// edge states in up0 and farthest points in rfar0 from the discard pass,
// segment counts at stage 0 of segcnt): QuickHull splits of the filter
// polygon's edges.  Round r appends to stage r + 1; an even number of rounds
// ends back in surv/keys0 (ping-pong through lo0/lo1/up1, which the hull stage
// only uses afterwards).
// Region counts of list stage r (0: the discard pass's output).
static int64_t *seg_stage(const Plan &p, int64_t *segcnt, int r) {
    return segcnt + r * p.nwave;
}

// Region size of list stage r in discard regions (q * TILE entries).
static int64_t region_mult(int r, bool batched) {
    int64_t m = 1;
    for (int i = 0; i < r; i++) m *= ref_group(i, batched);
    return m;
}

static_assert(HULL_NCOUNTS == 1 + REF_ROUNDS, "one count per refinement round");
static_assert(REF_ROUNDS % 2 == 0, "refinement must end in the first buffer set");
static int run_refine(hull_ctx *ctx, const Plan &p, hipStream_t st, const float *x,
                      const float *y, int64_t S) {
    uint32_t *idxs[2] = {W<uint32_t>(p, p.surv), W<uint32_t>(p, p.lo0)};
    uint64_t *keys[2] = {W<uint64_t>(p, p.keys0), W<uint64_t>(p, p.lo1)};
    uint16_t *eds[2] = {W<uint16_t>(p, p.up0), W<uint16_t>(p, p.up1)};
    REdge *tab[2] = {W<REdge>(p, p.rtab0), W<REdge>(p, p.rtab1)};
    unsigned long long *far[2] = {W<unsigned long long>(p, p.rfar0),
                                  W<unsigned long long>(p, p.rfar1)};
    int64_t *segcnt = W<int64_t>(p, p.segcnt);
    const int64_t *meta = W<int64_t>(p, p.segmeta);
    // one set: pass r splits the parents (tab[r % 2], F[r % 3]) itself, raises
    // F[(r + 1) % 3] (cleared before: k_counts_init, then the pass before)
    // and clears F[(r + 2) % 3], which no pass reads until two rounds later
    unsigned long long *F[3] = {far[0], far[1], W<unsigned long long>(p, p.rfar2)};
    for (int r = 0; r < REF_ROUNDS; r++) {
        const int a = r & 1, b = 1 - a;
        const int er = MAX_SLOTS << r;
        int64_t *cin = seg_stage(p, segcnt, r), *cout = seg_stage(p, segcnt, r + 1);
        const bool batched = S > 1;
        const int64_t nin = stage_regions(p.nwave, r, batched), nout = stage_regions(p.nwave, r + 1, batched);
        const int kg = ref_group(r, batched);
        const size_t lds = ref_lds_bytes(2 * er, S == 1);
        const unsigned nb = (unsigned)((nout + REF_WAVES - 1) / REF_WAVES);
        if (S == 1) {
            LAUNCH(K_REFINE, k_ref_pass<<<nb, REF_WAVES * WAVE, lds, st>>>(
                idxs[a], keys[a], eds[a], cin, (int)nin, kg, meta, region_mult(r, batched), tab[b], 2 * er,
                F[(r + 1) % 3], idxs[b], keys[b], eds[b], cout, 1, x, y, tab[a], F[r % 3], tab[b],
                F[(r + 2) % 3]));
            continue;
        }
        LAUNCH(K_REFINE_SPLIT, k_ref_split<<<(unsigned)((S * er + 255) / 256), 256, 0, st>>>(
            x, y, S, er, tab[a], far[a], tab[b], far[b]));
        LAUNCH(K_REFINE, k_ref_pass<<<nb, REF_WAVES * WAVE, lds, st>>>(
            idxs[a], keys[a], eds[a], cin, (int)nin, kg, meta, region_mult(r, batched), tab[b], 2 * er,
            far[b], idxs[b], keys[b], eds[b], cout, 0, x, y, nullptr, nullptr, nullptr, nullptr));
    }
    return HULL_OK;
}

// Region list (surv, keys0) of list stage `stage` -> contiguous (cidx,
// ckeys); ctx->counts[r] gets the total of stage r <= stage.
static int run_gather(hull_ctx *ctx, const Plan &p, hipStream_t st, int stage, int64_t S) {
    const int64_t gb = std::max<int64_t>(stage + 1, std::min<int64_t>(256, p.nwave));
    LAUNCH(K_SCATTER, k_seg_gather<<<(unsigned)gb, 256, 0, st>>>(
        W<uint32_t>(p, p.surv), W<uint64_t>(p, p.keys0), W<int64_t>(p, p.segcnt),
        (int)p.nwave, stage + 1, (int)(S > 1), W<int64_t>(p, p.segmeta), region_mult(stage, S > 1),
        W<uint32_t>(p, p.cidx), W<uint64_t>(p, p.ckeys), ctx->counts));
    return HULL_OK;
}

// Learned proposal: per-set histogram -> network -> eight directions written
// to the workspace's set_dirs table (defined with the network code below).
static int run_learned_dirs(hull_ctx *ctx, const Plan &p, hipStream_t st, const float *x,
                            const float *y, int64_t n_total, const int64_t *off, int64_t n1,
                            int64_t S);
static int learned_ensure(hull_ctx *ctx, int64_t B, hipStream_t st);
static int init_cand_table();

static int prepare(hull_ctx *ctx, int64_t n, int64_t S, hipStream_t st, Plan *p) {
    HIPCHECK(hipSetDevice(ctx->device));
    *p = make_plan(n, S, region_count(ctx, n, S));
    int rc = ensure_ws(ctx, p->total, st);
    p->base = ctx->ws;
    return rc;
}

// Full method for S sets (off == nullptr: one set of n1 points).
static int run_compute(hull_ctx *ctx, hipStream_t st, const float *x, const float *y,
                       int64_t n_total, const int64_t *off, int64_t n1, int64_t S, int flags,
                       uint32_t *hull, int64_t *hoff_out, int64_t *h_out) {
    Plan p;
    int rc = prepare(ctx, n_total, S, st, &p);
    if (rc) return rc;
    if (flags & HULL_VALIDATE) {
        rc = run_validate(ctx, p, st, x, y, n_total, off, S);
        if (rc) return rc;
    }
    const bool learned = (flags & HULL_LEARNED) && !(flags & HULL_NOFILTER);
    if (learned && !learned_ok(ctx)) return HULL_EINVAL;
    if (learned && !ctx->learned.loaded) return HULL_ENOMODEL;
    uint32_t *surv = W<uint32_t>(p, p.surv);
    uint64_t *keys = W<uint64_t>(p, p.keys0);
    int64_t *surv_off = W<int64_t>(p, p.surv_off);
    int64_t *hoff = hoff_out ? hoff_out : W<int64_t>(p, p.hoff);
    const bool refine = !(flags & (HULL_NOREFINE | HULL_NOFILTER));
    const int64_t *cnt = ctx->counts;
    int64_t *segcnt = W<int64_t>(p, p.segcnt);
    // one set: the farthest keys of refinement round 0's children start cleared
    const bool one_ref = S == 1 && refine;
    LAUNCH(K_MISC, k_counts_init<<<1, 64, 0, st>>>(
        ctx->counts, HULL_NCOUNTS, one_ref ? W<unsigned long long>(p, p.rfar1) : nullptr, RE_CAP));
    if (flags & HULL_NOFILTER) {
        LAUNCH(K_KEYS, k_all_keys<<<2048, 256, 0, st>>>(x, y, off, n1, S, n_total, surv, keys,
                                                         surv_off));
        LAUNCH(K_MISC, k_copy_count<<<1, 64, 0, st>>>(surv_off + S, ctx->counts));
    } else {
        if ((rc = run_tilemap(ctx, p, st, x, off, n1, S))) return rc;
        if (learned) {
            rc = run_learned_dirs(ctx, p, st, x, y, n_total, off, n1, S);
            if (rc) return rc;
        }
        if ((rc = run_extremes(ctx, p, st, x, y, n_total, off, n1, S, learned))) return rc;
        if ((rc = run_polygon(ctx, p, st, x, y, n_total, S, learned, nullptr, 0, nullptr, nullptr,
                              refine)))
            return rc;
        unsigned long long *far0 = nullptr;
        uint16_t *edges = nullptr;
        if (refine) {    // round-0 edge table from k_polygon; the discard pass fills its states
            far0 = W<unsigned long long>(p, p.rfar0);
            edges = W<uint16_t>(p, p.up0);
        }
        if ((rc = run_discard_append(ctx, p, st, x, y, n_total, off, n1, S,
                                     slot_count(ctx, learned), surv, keys, edges,
                                     segcnt, far0)))
            return rc;
        const int stage = refine ? REF_ROUNDS : 0;
        if (refine && (rc = run_refine(ctx, p, st, x, y, S))) return rc;
        if ((rc = run_gather(ctx, p, st, stage, S))) return rc;
        surv = W<uint32_t>(p, p.cidx);
        keys = W<uint64_t>(p, p.ckeys);
        cnt = ctx->counts + stage;
    }
    return run_hull(ctx, p, st, surv, keys, cnt, n_total, S, hoff, hull, h_out);
}

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char *hull_strerror(int code) {
    switch (code) {
    case HULL_OK: return "ok";
    case HULL_EINVAL: return "invalid argument (null pointer, size, preset or alignment)";
    case HULL_ETOOBIG: return "too many points (indices are uint32)";
    case HULL_ENOMEM: return "device workspace allocation failed";
    case HULL_EHIP: return "HIP runtime error";
    case HULL_EDOMAIN: return "coordinate outside the 2^-24 grid of [0,1) or bad offsets";
    case HULL_ECAPTURE: return "workspace must grow but the stream is being captured";
    case HULL_ENOMODEL: return "learned proposal requested without network weights";
    case HULL_ESCRATCH: return "input larger than the fixed scratch of the allocation-free call";
    case HULL_EOVERFLOW: return "more survivors than the output capacity";
    default: return "unknown error";
    }
}

int hull_last_hip_error(hull_ctx *ctx) { return ctx ? (int)ctx->last : 0; }

int hull_create(hull_ctx **out, int device) {
    if (!out) return HULL_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return HULL_EINVAL;
    }
    hull_ctx *ctx = new hull_ctx();
    ctx->device = device;
    ctx->dirs = preset_dirs(HULL_DIRS_PAPER);
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return HULL_EHIP;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        cus > 0)
        ctx->cus = cus;
    // this device's scratch array (allocation-free entry point) and the
    // occupancy of every extremes variant, so that later calls query nothing
    if (scratch_setup(device, &ctx->scratch) != HULL_OK) {
        delete ctx;
        return HULL_EHIP;
    }
    for (int bs : SHAPE_BS) {
        for (int pr = 0; pr < NUM_PRESETS; pr++) {
            (void)resident_blocks(k1_kernel(pr, false, bs), bs);
            if (preset_fixed_slots(pr) == FIXED_SLOTS) (void)resident_blocks(k1_kernel(pr, true, bs), bs);
        }
        (void)resident_blocks(k3_kernel(bs), bs);
    }
    if (hipMalloc(&ctx->counts, HULL_NCOUNTS * sizeof(int64_t)) != hipSuccess ||
        hipMemset(ctx->counts, 0xff, HULL_NCOUNTS * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&ctx->tickets, 8 * sizeof(uint32_t)) != hipSuccess ||
        hipMemset(ctx->tickets, 0, 8 * sizeof(uint32_t)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->counts) (void)hipFree(ctx->counts);
        if (ctx->tickets) (void)hipFree(ctx->tickets);
        delete ctx;
        return HULL_ENOMEM;
    }
    *out = ctx;
    return HULL_OK;
}

int hull_destroy(hull_ctx *ctx) {
    if (!ctx) return HULL_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    learned_free(ctx->learned);
    stream_free(ctx->sb);
    hull3_free(ctx->h3);
    for (char *r : ctx->retired) (void)hipFree(r);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->counts) (void)hipFree(ctx->counts);
    if (ctx->tickets) (void)hipFree(ctx->tickets);
    delete ctx;
    return HULL_OK;
}

int hull_set_directions(hull_ctx *ctx, int preset) {
    if (!ctx || !preset_valid(preset)) return HULL_EINVAL;
    ctx->preset = preset;
    ctx->dirs = preset_dirs(preset);
    return HULL_OK;
}

int hull_slot_count(hull_ctx *ctx, int flags) {
    if (!ctx) return HULL_EINVAL;
    const bool learned = flags & HULL_LEARNED;
    if (learned && !learned_ok(ctx)) return HULL_EINVAL;
    return slot_count(ctx, learned);
}

int hull_direction_table(hull_ctx *ctx, int which, double *c, double *s, int cap) {
    if (!c || !s) return HULL_EINVAL;
    if (which == 0 || (which >= 16 && which < 16 + NUM_PRESETS)) {
        const int preset = which ? which - 16 : ctx ? ctx->preset : HULL_DIRS_PAPER;
        const Dirs d = preset_dirs(preset);
        const int G = preset_groups(preset);
        if (cap < G) return HULL_EINVAL;
        for (int g = 0; g < G; g++) { c[g] = d.gc[g]; s[g] = d.gs[g]; }
        return G;
    }
    if (which == 1) {
        if (cap < NCAND) return HULL_EINVAL;
        for (int k = 0; k < NCAND; k++) { c[k] = kCandCos[k]; s[k] = kCandSin[k]; }
        return NCAND;
    }
    return HULL_EINVAL;
}

int hull_extremes(hull_ctx *ctx, const float *x, const float *y, int64_t n, uint32_t *slots,
                  double *vals, int flags, void *stream) {
    if (!ctx || !slots) return HULL_EINVAL;
    int rc = check_points(x, y, n);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Plan p;
    if ((rc = prepare(ctx, n, 1, st, &p))) return rc;
    if (flags & HULL_VALIDATE && (rc = run_validate(ctx, p, st, x, y, n, nullptr, 1))) return rc;
    const bool learned = flags & HULL_LEARNED;
    if (learned && !learned_ok(ctx)) return HULL_EINVAL;
    if (learned && !ctx->learned.loaded) return HULL_ENOMODEL;
    if ((rc = run_tilemap(ctx, p, st, x, nullptr, n, 1))) return rc;
    if (learned && (rc = run_learned_dirs(ctx, p, st, x, y, n, nullptr, n, 1))) return rc;
    if ((rc = run_extremes(ctx, p, st, x, y, n, nullptr, n, 1, learned))) return rc;
    return run_polygon(ctx, p, st, x, y, n, 1, learned, nullptr, 0, slots, vals);
}

int hull_extremes_noalloc(hull_ctx *ctx, const float *x, const float *y, int64_t n,
                          uint32_t *slots, double *vals, int flags, void *stream) {
    if (!ctx || !slots || flags != 0) return HULL_EINVAL;
    int rc = check_points(x, y, n);
    if (rc) return rc;
    if (n > NOALLOC_MAX_POINTS) return HULL_ESCRATCH;
    if (!ctx->scratch) return HULL_EHIP;
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(hipSetDevice(ctx->device));
    Plan p = make_plan_extremes(n);
    p.base = ctx->scratch;
    // no timing events here: the event pool may have to grow
    const bool was_timing = ctx->timing;
    ctx->timing = false;
    // the tile map zeroes the polygon kernel's ticket; every other buffer is
    // written before it is read
    if (!(rc = run_tilemap(ctx, p, st, x, nullptr, n, 1)) &&
        !(rc = run_extremes(ctx, p, st, x, y, n, nullptr, n, 1, false)))
        rc = run_polygon(ctx, p, st, x, y, n, 1, false, nullptr, 0, slots, vals);
    ctx->timing = was_timing;
    return rc;
}

int hull_polygon(hull_ctx *ctx, const float *x, const float *y, int64_t n, const uint32_t *slots,
                 int n_slots, uint32_t *verts, int32_t *m, void *stream) {
    if (!ctx || !slots || !verts || !m || n_slots < 0 || n_slots > MAX_SLOTS) return HULL_EINVAL;
    int rc = check_points(x, y, n);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Plan p;
    if ((rc = prepare(ctx, n, 1, st, &p))) return rc;
    if ((rc = run_tilemap(ctx, p, st, x, nullptr, n, 1))) return rc;    // the set's size sets its rows
    if ((rc = run_polygon(ctx, p, st, x, y, n, 1, false, slots, n_slots, nullptr, nullptr))) return rc;
    LAUNCH(K_MISC, k_poly_out<<<1, 64, 0, st>>>(W<Poly>(p, p.polys), n_slots, verts, m));
    return HULL_OK;
}

int hull_discard(hull_ctx *ctx, const float *x, const float *y, int64_t n, const uint32_t *slots,
                 int n_slots, uint32_t *surv, int64_t *n_surv, void *stream) {
    if (!ctx || !slots || !surv || !n_surv || n_slots < 0 || n_slots > MAX_SLOTS)
        return HULL_EINVAL;
    int rc = check_points(x, y, n);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Plan p;
    if ((rc = prepare(ctx, n, 1, st, &p))) return rc;
    if ((rc = run_tilemap(ctx, p, st, x, nullptr, n, 1))) return rc;
    if ((rc = run_polygon(ctx, p, st, x, y, n, 1, false, slots, n_slots, nullptr, nullptr))) return rc;
    int64_t *so = W<int64_t>(p, p.surv_off);
    if ((rc = run_discard(ctx, p, st, x, y, n, nullptr, n, 1, n_slots, surv, so, nullptr)))
        return rc;
    LAUNCH(K_MISC, k_copy_count<<<1, 64, 0, st>>>(so + 1, n_surv));
    return HULL_OK;
}

int hull_of_subset(hull_ctx *ctx, const float *x, const float *y, int64_t n, const uint32_t *idx,
                   const int64_t *k_dev, int64_t k_cap, uint32_t *hull, int64_t *h, void *stream) {
    if (!ctx || !idx || !k_dev || !hull || !h || k_cap < 0) return HULL_EINVAL;
    int rc = check_points(x, y, n);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Plan p;
    if ((rc = prepare(ctx, k_cap, 1, st, &p))) return rc;
    uint64_t *keys = W<uint64_t>(p, p.keys0);
    LAUNCH(K_KEYS, k_gather_keys<<<1024, 256, 0, st>>>(x, y, n, idx, k_dev, keys));
    int64_t *hoff = W<int64_t>(p, p.hoff);
    if ((rc = run_hull(ctx, p, st, idx, keys, k_dev, k_cap, 1, hoff, hull))) return rc;
    LAUNCH(K_MISC, k_copy_count<<<1, 64, 0, st>>>(hoff + 1, h));
    return HULL_OK;
}

int hull_compute(hull_ctx *ctx, const float *x, const float *y, int64_t n, uint32_t *hull,
                 int64_t *h, int flags, void *stream) {
    if (!ctx || !hull || !h) return HULL_EINVAL;
    int rc = check_points(x, y, n);
    if (rc) return rc;
    return run_compute(ctx, (hipStream_t)stream, x, y, n, nullptr, n, 1, flags, hull, nullptr, h);
}

static int check_batch(const float *x, const float *y, const int64_t *off, int64_t S,
                       int64_t n_total) {
    // set ids fill a key's 16-bit set field; 0xFFFF marks gaps in the hull stage
    if (!off || S <= 0 || S > 65535) return HULL_EINVAL;
    return check_points(x, y, n_total);
}

int hull_extremes_batched(hull_ctx *ctx, const float *x, const float *y, const int64_t *offsets,
                          int64_t S, int64_t n_total, uint32_t *slots, int flags, void *stream) {
    if (!ctx || !slots) return HULL_EINVAL;
    int rc = check_batch(x, y, offsets, S, n_total);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Plan p;
    if ((rc = prepare(ctx, n_total, S, st, &p))) return rc;
    if (flags & HULL_VALIDATE && (rc = run_validate(ctx, p, st, x, y, n_total, offsets, S)))
        return rc;
    const bool learned = flags & HULL_LEARNED;
    if (learned && !learned_ok(ctx)) return HULL_EINVAL;
    if (learned && !ctx->learned.loaded) return HULL_ENOMODEL;
    if ((rc = run_tilemap(ctx, p, st, x, offsets, 0, S))) return rc;
    if (learned && (rc = run_learned_dirs(ctx, p, st, x, y, n_total, offsets, 0, S))) return rc;
    if ((rc = run_extremes(ctx, p, st, x, y, n_total, offsets, 0, S, learned))) return rc;
    return run_polygon(ctx, p, st, x, y, n_total, S, learned, nullptr, 0, slots, nullptr);
}

int hull_discard_batched(hull_ctx *ctx, const float *x, const float *y, const int64_t *offsets,
                         int64_t S, int64_t n_total, const uint32_t *slots, int n_slots,
                         uint32_t *surv, int64_t *surv_offsets, void *stream) {
    if (!ctx || !slots || !surv || !surv_offsets || n_slots < 0 || n_slots > MAX_SLOTS)
        return HULL_EINVAL;
    int rc = check_batch(x, y, offsets, S, n_total);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    Plan p;
    if ((rc = prepare(ctx, n_total, S, st, &p))) return rc;
    if ((rc = run_tilemap(ctx, p, st, x, offsets, 0, S))) return rc;
    if ((rc = run_polygon(ctx, p, st, x, y, n_total, S, false, slots, n_slots, nullptr, nullptr))) return rc;
    return run_discard(ctx, p, st, x, y, n_total, offsets, 0, S, n_slots, surv, surv_offsets,
                       nullptr);
}

int hull_compute_batched(hull_ctx *ctx, const float *x, const float *y, const int64_t *offsets,
                         int64_t S, int64_t n_total, uint32_t *hull, int64_t *hull_offsets,
                         int flags, void *stream) {
    if (!ctx || !hull || !hull_offsets) return HULL_EINVAL;
    int rc = check_batch(x, y, offsets, S, n_total);
    if (rc) return rc;
    return run_compute(ctx, (hipStream_t)stream, x, y, n_total, offsets, 0, S, flags, hull,
                       hull_offsets, nullptr);
}

int hull_graph_capture(hull_ctx *ctx, const float *x, const float *y, const int64_t *offsets,
                       int64_t S, int64_t n_total, uint32_t *hull, int64_t *hull_offsets,
                       int flags, void *stream) {
    if (!ctx || !hull || !hull_offsets) return HULL_EINVAL;
    if (flags & HULL_VALIDATE) return HULL_EINVAL;   // validation synchronises
    int rc = check_batch(x, y, offsets, S, n_total);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(hipSetDevice(ctx->device));
    Plan p = make_plan(n_total, S, region_count(ctx, n_total, S));
    if ((rc = ensure_ws(ctx, p.total, st))) return rc;
    p.base = ctx->ws;
    if ((flags & HULL_LEARNED) && !(flags & HULL_NOFILTER)) {
        // the network's buffers are sized before capture: nothing allocates inside
        if (!learned_ok(ctx)) return HULL_EINVAL;
        if (!ctx->learned.loaded) return HULL_ENOMODEL;
        if ((rc = init_cand_table())) return rc;
        if ((rc = learned_ensure(ctx, S, st))) return rc;
    }
    hipStream_t cs;
    HIPCHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const bool was_timing = ctx->timing;
    ctx->timing = false;
    if (ctx->gexec) {
        (void)hipDeviceSynchronize();
        (void)hipGraphExecDestroy(ctx->gexec);
        ctx->gexec = nullptr;
    }
    if (ctx->graph) { (void)hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
    for (char *r : ctx->retired) (void)hipFree(r);
    ctx->retired.clear();
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        ctx->timing = was_timing;
        (void)hipStreamDestroy(cs);
        ctx->last = e;
        return HULL_EHIP;
    }
    rc = run_compute(ctx, cs, x, y, n_total, offsets, 0, S, flags, hull, hull_offsets, nullptr);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    ctx->timing = was_timing;
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) { ctx->last = e; return HULL_EHIP; }
    ctx->graph = g;
    HIPCHECK(hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0));
    return HULL_OK;
}

int hull_graph_launch(hull_ctx *ctx, void *stream) {
    if (!ctx || !ctx->gexec) return HULL_EINVAL;
    HIPCHECK(hipSetDevice(ctx->device));
    HIPCHECK(hipGraphLaunch(ctx->gexec, (hipStream_t)stream));
    return HULL_OK;
}

int hull_tuning(hull_ctx *ctx, int get, int *k1, int *k3) {
    if (!ctx || !k1 || !k3) return HULL_EINVAL;
    if (get) {
        *k1 = ctx->def[0].bpc;
        *k3 = ctx->def[1].bpc;
        return HULL_OK;
    }
    if (*k1 < 1 || *k1 > 64 || *k3 < 1 || *k3 > 64) return HULL_EINVAL;
    ctx->def[0].bpc = *k1;
    ctx->def[1].bpc = *k3;
    // an explicit choice replaces every tuned bucket
    for (int k = 0; k < 2; k++)
        for (int b = 0; b < NBUCKETS; b++) ctx->has_tuned[k][b] = false;
    return HULL_OK;
}

static bool shape_valid(int bs, int bpc, int tpw) {
    return (bs == 128 || bs == 256 || bs == 512) && bpc >= 1 && bpc <= 16 && tpw >= 1 && tpw <= 1024;
}

int hull_shape(hull_ctx *ctx, int get, int kernel, int64_t n, int64_t S, int *bs, int *bpc, int *tpw) {
    if (!ctx || !bs || !bpc || !tpw || kernel < 0 || kernel > 1 || n < 0 || S < 1) return HULL_EINVAL;
    const int b = bucket_of(n, S);
    if (get) {
        const Shape sh = shape_of(ctx, kernel, n, S);
        *bs = sh.bs;
        *bpc = sh.bpc;
        *tpw = sh.tpw;
        return ctx->has_tuned[kernel][b] ? 1 : 0;
    }
    if (!shape_valid(*bs, *bpc, *tpw)) return HULL_EINVAL;
    ctx->tuned[kernel][b] = Shape{*bs, *bpc, *tpw};
    ctx->has_tuned[kernel][b] = true;
    return HULL_OK;
}

int hull_tuning_table(hull_ctx *ctx, int32_t *rows, int cap) {
    if (!ctx || (!rows && cap > 0) || cap < 0) return HULL_EINVAL;
    int k = 0;
    for (int kernel = 0; kernel < 2; kernel++)
        for (int b = 0; b < NBUCKETS; b++) {
            if (!ctx->has_tuned[kernel][b]) continue;
            if (k < cap) {
                int32_t *r = rows + 6 * k;
                r[0] = kernel;
                r[1] = b % NSIZE;
                r[2] = b >= NSIZE;
                r[3] = ctx->tuned[kernel][b].bs;
                r[4] = ctx->tuned[kernel][b].bpc;
                r[5] = ctx->tuned[kernel][b].tpw;
            }
            k++;
        }
    return k;
}

// Candidate shapes of the tuner: each block size at 1..8 blocks per CU (the
// same waves per CU counted once per block size) and 1, 4 or 16 tiles per
// wave, the latter only where they shrink the grid.
// Candidate shapes of a kernel for n points: every (block size, blocks per
// CU, tiles per wave) that launches a distinct number of waves.  On large
// inputs (2^26 points and more) only the shapes that keep the kernel's most
// waves resident per CU: timed alone, a shape of lower occupancy has come out
// ahead several times and then run 8-17 % slower in the step, where each
// pass follows the other kernels instead of itself.
static std::vector<Shape> shape_candidates(const hull_ctx *ctx, int kind, int64_t n, int64_t S,
                                           bool learned) {
    std::vector<Shape> out;
    std::vector<std::pair<int, int64_t>> seen;     // (block size, waves)
    auto per_cu = [&](const Shape &sh, const void *fn) {
        return (int64_t)std::min(sh.bpc, resident_blocks(fn, sh.bs)) * (sh.bs / WAVE);
    };
    int64_t full = 0;
    for (int bs : SHAPE_BS)
        for (int bpc : {1, 2, 3, 4, 6, 8}) {
            const void *fn = kind == 0 ? k1_kernel(ctx->preset, learned, bs) : k3_kernel(bs);
            full = std::max(full, per_cu(Shape{bs, bpc, 1}, fn));
        }
    const bool full_only = n >= (int64_t(1) << 26);
    for (int bs : SHAPE_BS)
        for (int bpc : {1, 2, 3, 4, 6, 8})
            for (int tpw : {1, 4, 16}) {
                const Shape sh{bs, bpc, tpw};
                const void *fn = kind == 0 ? k1_kernel(ctx->preset, learned, bs) : k3_kernel(bs);
                if (full_only && per_cu(sh, fn) < full) continue;
                const Launch L = make_launch(ctx, sh, fn, n, S);
                bool dup = false;
                for (auto &q : seen) dup = dup || (q.first == bs && q.second == L.waves);
                if (dup) continue;
                seen.push_back({bs, L.waves});
                out.push_back(sh);
            }
    return out;
}

int hull_autotune(hull_ctx *ctx, const float *x, const float *y, const int64_t *offsets,
                  int64_t S, int64_t n_total, void *stream) {
    if (!ctx) return HULL_EINVAL;
    const bool batched = offsets != nullptr;
    if (batched) {
        int rc = check_batch(x, y, offsets, S, n_total);
        if (rc) return rc;
    } else {
        int rc = check_points(x, y, n_total);
        if (rc) return rc;
        S = 1;
    }
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(hipSetDevice(ctx->device));
    const int b = bucket_of(n_total, S);
    const int64_t n1 = batched ? 0 : n_total;
    const auto c1 = shape_candidates(ctx, 0, n_total, S, false);
    const auto c3 = shape_candidates(ctx, 1, n_total, S, false);
    // one workspace for every candidate: only the region counts at the
    // plan's end depend on the discard pass's waves
    int64_t wmax = 1;
    for (const Shape &sh : c3)
        wmax = std::max(wmax, regions_for(make_launch(ctx, sh, k3_kernel(sh.bs), n_total, S).waves, S));
    Plan big = make_plan(n_total, S, wmax);
    int rc = ensure_ws(ctx, big.total, st);
    if (rc) return rc;
    big.base = ctx->ws;
    const bool was_timing = ctx->timing;
    ctx->timing = false;
    hipEvent_t ea, eb;
    HIPCHECK(hipEventCreate(&ea));
    HIPCHECK(hipEventCreate(&eb));
    // a candidate's time: the best of its timed runs, taken in three rounds
    // over all the candidates (two runs each, after a warm-up one in the
    // first), so that a drift of the clocks during the sweep does not favour
    // the candidates timed at one end of it
    auto timed = [&](auto &&fn, bool warm, float *best_ms) -> int {
        for (int rep = warm ? 0 : 1; rep < 3; rep++) {
            HIPCHECK(hipEventRecord(ea, st));
            int r = fn();
            if (r) return r;
            HIPCHECK(hipEventRecord(eb, st));
            HIPCHECK(hipEventSynchronize(eb));
            float ms = 0;
            HIPCHECK(hipEventElapsedTime(&ms, ea, eb));
            if (rep) *best_ms = std::min(*best_ms, ms);
        }
        return HULL_OK;
    };
    constexpr int ROUNDS = 3;
    const bool had1 = ctx->has_tuned[0][b], had3 = ctx->has_tuned[1][b];
    const Shape old1 = ctx->tuned[0][b], old3 = ctx->tuned[1][b];
    Shape best1 = shape_of(ctx, 0, n_total, S), best3 = shape_of(ctx, 1, n_total, S);
    std::vector<float> t1(c1.size(), 1e30f), t3(c3.size(), 1e30f);
    rc = run_tilemap(ctx, big, st, x, offsets, n1, S);
    for (int round = 0; !rc && round < ROUNDS; round++)
        for (size_t i = 0; !rc && i < c1.size(); i++) {
            ctx->tuned[0][b] = c1[i];
            ctx->has_tuned[0][b] = true;
            rc = timed([&]() { return run_extremes(ctx, big, st, x, y, n_total, offsets, n1, S, false); },
                       round == 0, &t1[i]);
        }
    {
        size_t k = 0;
        for (size_t i = 1; i < c1.size(); i++)
            if (t1[i] < t1[k]) k = i;
        if (!c1.empty()) best1 = c1[k];
    }
    ctx->tuned[0][b] = best1;
    ctx->has_tuned[0][b] = true;
    // the full method's discard pass (refinement round 0 included) on the
    // polygon of the best extremes shape
    if (!rc) rc = run_extremes(ctx, big, st, x, y, n_total, offsets, n1, S, false);
    if (!rc) rc = run_polygon(ctx, big, st, x, y, n_total, S, false, nullptr, 0, nullptr, nullptr, true);
    for (int round = 0; !rc && round < ROUNDS; round++)
        for (size_t i = 0; !rc && i < c3.size(); i++) {
            ctx->tuned[1][b] = c3[i];
            ctx->has_tuned[1][b] = true;
            Plan pc = make_plan(n_total, S, region_count(ctx, n_total, S));
            pc.base = ctx->ws;
            rc = timed([&]() {
                return run_discard_append(ctx, pc, st, x, y, n_total, offsets, n1, S, slot_count(ctx, false),
                                          W<uint32_t>(pc, pc.surv), W<uint64_t>(pc, pc.keys0),
                                          W<uint16_t>(pc, pc.up0), W<int64_t>(pc, pc.segcnt),
                                          W<unsigned long long>(pc, pc.rfar0));
            }, round == 0, &t3[i]);
        }
    {
        size_t k = 0;
        for (size_t i = 1; i < c3.size(); i++)
            if (t3[i] < t3[k]) k = i;
        if (!c3.empty()) best3 = c3[k];
    }
    ctx->tuned[1][b] = best3;
    ctx->has_tuned[1][b] = true;
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    ctx->timing = was_timing;
    if (rc) {   // keep the table as it was
        ctx->tuned[0][b] = old1;
        ctx->has_tuned[0][b] = had1;
        ctx->tuned[1][b] = old3;
        ctx->has_tuned[1][b] = had3;
    }
    return rc;
}

int hull_timing_enable(hull_ctx *ctx, int on) {
    if (!ctx) return HULL_EINVAL;
    HIPCHECK(hipSetDevice(ctx->device));
    if (on && ctx->ev_pool.empty()) {
        ctx->ev_pool.resize(8192);
        for (auto &e : ctx->ev_pool) HIPCHECK(hipEventCreate(&e));
    }
    ctx->timing = on != 0;
    return HULL_OK;
}

static int drain_events(hull_ctx *ctx) {
    for (auto &pe : ctx->ev_pending) {
        HIPCHECK(hipEventSynchronize(ctx->ev_pool[pe.second + 1]));
        float ms = 0;
        HIPCHECK(hipEventElapsedTime(&ms, ctx->ev_pool[pe.second], ctx->ev_pool[pe.second + 1]));
        ctx->ms[pe.first] += ms;
        ctx->launches[pe.first] += 1;
    }
    ctx->ev_pending.clear();
    ctx->ev_used = 0;
    return HULL_OK;
}

int hull_timing_read(hull_ctx *ctx, double *ms, int64_t *launches, int cap) {
    if (!ctx || !ms || !launches) return HULL_EINVAL;
    int rc = drain_events(ctx);
    if (rc) return rc;
    int n = std::min(cap, (int)K_NKINDS);
    for (int k = 0; k < n; k++) {
        ms[k] = ctx->ms[k];
        launches[k] = ctx->launches[k];
    }
    return n;
}

const char *hull_timing_name(int kind) {
    return (kind >= 0 && kind < K_NKINDS) ? kKindNames[kind] : "";
}

int hull_candidate_counts(hull_ctx *ctx, int64_t *counts, int cap) {
    if (!ctx || !counts || cap < 0) return HULL_EINVAL;
    HIPCHECK(hipSetDevice(ctx->device));
    HIPCHECK(hipDeviceSynchronize());
    const int k = std::min(cap, HULL_NCOUNTS);
    if (k > 0) HIPCHECK(hipMemcpy(counts, ctx->counts, k * sizeof(int64_t), hipMemcpyDeviceToHost));
    return k;
}

int hull_timing_reset(hull_ctx *ctx) {
    if (!ctx) return HULL_EINVAL;
    int rc = drain_events(ctx);
    for (int k = 0; k < K_NKINDS; k++) {
        ctx->ms[k] = 0;
        ctx->launches[k] = 0;
    }
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned proposal: network buffers, forward, backward, training step,
// labels.  Weight matrices in bf16, activations in bf16, accumulation and
// the master copy of the parameters in float32.

static int learned_ensure(hull_ctx *ctx, int64_t B, hipStream_t st) {
    LearnedState &L = ctx->learned;
    const int64_t Bp = std::max<int64_t>(64, (B + 63) / 64 * 64);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (!L.params || Bp > L.bcap) {
        HIPCHECK(hipStreamIsCapturing(st, &cs));
        if (cs != hipStreamCaptureStatusNone) return HULL_ECAPTURE;
        HIPCHECK(hipDeviceSynchronize());
    }
    if (!L.params) {
        HIPCHECK(hipMalloc(&L.params, P_TOTAL * sizeof(float)));
        HIPCHECK(hipMalloc(&L.grads, P_TOTAL * sizeof(float)));
        HIPCHECK(hipMalloc(&L.m1, P_TOTAL * sizeof(float)));
        HIPCHECK(hipMalloc(&L.m2, P_TOTAL * sizeof(float)));
        HIPCHECK(hipMalloc(&L.wb, Q_TOTAL * sizeof(bf16_t)));
    }
    if (Bp > L.bcap) {
        void *old[] = {L.X, L.H1, L.H2, L.dS, L.dZ2, L.dZ1, L.scores, L.part};
        for (void *q : old)
            if (q) HIPCHECK(hipFree(q));
        HIPCHECK(hipMalloc(&L.X, Bp * HBINS * sizeof(bf16_t)));
        HIPCHECK(hipMalloc(&L.H1, Bp * L1 * sizeof(bf16_t)));
        HIPCHECK(hipMalloc(&L.H2, Bp * L2 * sizeof(bf16_t)));
        HIPCHECK(hipMalloc(&L.dS, Bp * NOUT * sizeof(bf16_t)));
        HIPCHECK(hipMalloc(&L.dZ2, Bp * L2 * sizeof(bf16_t)));
        HIPCHECK(hipMalloc(&L.dZ1, Bp * L1 * sizeof(bf16_t)));
        HIPCHECK(hipMalloc(&L.scores, Bp * NOUT * sizeof(float)));
        HIPCHECK(hipMalloc(&L.part, Bp * sizeof(float)));
        L.bcap = Bp;
    }
    return HULL_OK;
}

template <int MODE>
static int gemm(hull_ctx *ctx, hipStream_t st, const bf16_t *A, int64_t sam, int64_t sak,
                const bf16_t *B, int64_t sbk, int64_t sbn, int M, int N, int K, const float *bias,
                const bf16_t *mask, bf16_t *Cb, float *Cf, int ldc) {
    if (M % GBM || N % GBN || K % GBK) return HULL_EINVAL;
    dim3 grid(N / GBN, M / GBM);
    LAUNCH(K_MLP, k_gemm<MODE><<<grid, 256, 0, st>>>(A, sam, sak, B, sbk, sbn, M, N, K, bias, mask,
                                                     Cb, Cf, ldc));
    return HULL_OK;
}

#define RC(expr)                 \
    do {                         \
        int rc_ = (expr);        \
        if (rc_) return rc_;     \
    } while (0)

// scores (float32 [Bp][64]) of histogram rows hist[B][1024] into L.scores
static int mlp_forward(hull_ctx *ctx, hipStream_t st, const bf16_t *hist, int64_t B) {
    LearnedState &L = ctx->learned;
    RC(learned_ensure(ctx, B, st));
    const int Bp = (int)std::max<int64_t>(64, (B + 63) / 64 * 64);
    LAUNCH(K_MLP, k_pad_rows<<<256, 256, 0, st>>>(hist, B, Bp, HBINS, L.X));
    RC(gemm<G_RELU_BF16>(ctx, st, L.X, HBINS, 1, L.wb + Q_W1, 1, HBINS, Bp, L1, HBINS,
                         L.params + P_B1, nullptr, L.H1, nullptr, L1));
    RC(gemm<G_RELU_BF16>(ctx, st, L.H1, L1, 1, L.wb + Q_W2, 1, L1, Bp, L2, L1, L.params + P_B2,
                         nullptr, L.H2, nullptr, L2));
    RC(gemm<G_BIAS_F32>(ctx, st, L.H2, L2, 1, L.wb + Q_W3, 1, L2, Bp, NOUT, L2, L.params + P_B3,
                        nullptr, nullptr, L.scores, NOUT));
    return HULL_OK;
}

// gradients of every parameter into L.grads, from L.dS (bf16 [Bp][64]) and
// the activations of the last forward pass
static int mlp_backward(hull_ctx *ctx, hipStream_t st, int64_t B) {
    LearnedState &L = ctx->learned;
    const int Bp = (int)std::max<int64_t>(64, (B + 63) / 64 * 64);
    RC(gemm<G_F32>(ctx, st, L.dS, 1, NOUT, L.H2, L2, 1, NOUT, L2, Bp, nullptr, nullptr, nullptr,
                   L.grads + P_W3, L2));
    LAUNCH(K_MLP, k_colsum<<<1, 64, 0, st>>>(L.dS, Bp, NOUT, L.grads + P_B3));
    RC(gemm<G_MASK_BF16>(ctx, st, L.dS, NOUT, 1, L.wb + Q_W3, L2, 1, Bp, L2, NOUT, nullptr, L.H2,
                         L.dZ2, nullptr, L2));
    RC(gemm<G_F32>(ctx, st, L.dZ2, 1, L2, L.H1, L1, 1, L2, L1, Bp, nullptr, nullptr, nullptr,
                   L.grads + P_W2, L1));
    LAUNCH(K_MLP, k_colsum<<<(L2 + 255) / 256, 256, 0, st>>>(L.dZ2, Bp, L2, L.grads + P_B2));
    RC(gemm<G_MASK_BF16>(ctx, st, L.dZ2, L2, 1, L.wb + Q_W2, L1, 1, Bp, L1, L2, nullptr, L.H1,
                         L.dZ1, nullptr, L1));
    RC(gemm<G_F32>(ctx, st, L.dZ1, 1, L1, L.X, HBINS, 1, L1, HBINS, Bp, nullptr, nullptr, nullptr,
                   L.grads + P_W1, HBINS));
    LAUNCH(K_MLP, k_colsum<<<(L1 + 255) / 256, 256, 0, st>>>(L.dZ1, Bp, L1, L.grads + P_B1));
    return HULL_OK;
}

static int run_learned_dirs(hull_ctx *ctx, const Plan &p, hipStream_t st, const float *x,
                            const float *y, int64_t n_total, const int64_t *off, int64_t n1,
                            int64_t S) {
    (void)n_total;
    if (!ctx->learned.loaded) return HULL_ENOMODEL;
    bf16_t *hist = W<bf16_t>(p, p.learn);
    LAUNCH(K_HIST32, k_hist32<<<(unsigned)S, HIST_THREADS, 0, st>>>(x, y, off, n1, S, hist, nullptr));
    RC(mlp_forward(ctx, st, hist, S));
    LAUNCH(K_MLP, k_top8<<<(unsigned)((S + 3) / 4), 256, 0, st>>>(ctx->learned.scores, S, ctx->dir_gap, nullptr,
                                                                 W<double>(p, p.setdirs)));
    return HULL_OK;
}

static int init_cand_table() {
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    std::call_once(once, [] {
        err = hipMemcpyToSymbol(HIP_SYMBOL(dCandCos), kCandCos, sizeof(kCandCos));
        if (err == hipSuccess) err = hipMemcpyToSymbol(HIP_SYMBOL(dCandSin), kCandSin, sizeof(kCandSin));
    });
    return err == hipSuccess ? HULL_OK : HULL_EHIP;
}

extern "C" {

int64_t hull_mlp_param_count(void) { return P_TOTAL; }

int hull_mlp_set_params(hull_ctx *ctx, const float *params, int64_t count) {
    if (!ctx || !params || count != P_TOTAL) return HULL_EINVAL;
    HIPCHECK(hipSetDevice(ctx->device));
    RC(init_cand_table());
    hipStream_t st = nullptr;
    RC(learned_ensure(ctx, 64, st));
    LearnedState &L = ctx->learned;
    HIPCHECK(hipMemcpy(L.params, params, P_TOTAL * sizeof(float), hipMemcpyHostToDevice));
    HIPCHECK(hipMemset(L.m1, 0, P_TOTAL * sizeof(float)));
    HIPCHECK(hipMemset(L.m2, 0, P_TOTAL * sizeof(float)));
    LAUNCH(K_MLP, k_to_bf16<<<1024, 256, 0, st>>>(L.params + P_W1, (int64_t)L1 * HBINS, L.wb + Q_W1));
    LAUNCH(K_MLP, k_to_bf16<<<1024, 256, 0, st>>>(L.params + P_W2, (int64_t)L2 * L1, L.wb + Q_W2));
    LAUNCH(K_MLP, k_to_bf16<<<256, 256, 0, st>>>(L.params + P_W3, (int64_t)NOUT * L2, L.wb + Q_W3));
    HIPCHECK(hipDeviceSynchronize());
    L.step = 0;
    L.loaded = true;
    return HULL_OK;
}

int hull_mlp_get_params(hull_ctx *ctx, float *params, int64_t count) {
    if (!ctx || !params || count != P_TOTAL || !ctx->learned.loaded) return HULL_EINVAL;
    HIPCHECK(hipSetDevice(ctx->device));
    HIPCHECK(hipDeviceSynchronize());
    HIPCHECK(hipMemcpy(params, ctx->learned.params, P_TOTAL * sizeof(float), hipMemcpyDeviceToHost));
    return HULL_OK;
}

int hull_mlp_get_state(hull_ctx *ctx, float *state, int64_t count, int64_t *step) {
    if (!ctx || !state || !step || count != 3 * P_TOTAL || !ctx->learned.loaded) return HULL_EINVAL;
    HIPCHECK(hipSetDevice(ctx->device));
    HIPCHECK(hipDeviceSynchronize());
    const LearnedState &L = ctx->learned;
    HIPCHECK(hipMemcpy(state, L.params, P_TOTAL * sizeof(float), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(state + P_TOTAL, L.m1, P_TOTAL * sizeof(float), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(state + 2 * P_TOTAL, L.m2, P_TOTAL * sizeof(float), hipMemcpyDeviceToHost));
    *step = L.step;
    return HULL_OK;
}

int hull_mlp_set_state(hull_ctx *ctx, const float *state, int64_t count, int64_t step) {
    if (!ctx || !state || count != 3 * P_TOTAL || step < 0) return HULL_EINVAL;
    RC(hull_mlp_set_params(ctx, state, P_TOTAL));      // parameters and their bf16 copies
    LearnedState &L = ctx->learned;
    HIPCHECK(hipMemcpy(L.m1, state + P_TOTAL, P_TOTAL * sizeof(float), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(L.m2, state + 2 * P_TOTAL, P_TOTAL * sizeof(float), hipMemcpyHostToDevice));
    L.step = step;
    return HULL_OK;
}

int hull_histogram_batched(hull_ctx *ctx, const float *x, const float *y, const int64_t *offsets,
                           int64_t S, int64_t n_total, uint16_t *hist, float *hist_f32,
                           void *stream) {
    if (!ctx || !hist || S <= 0) return HULL_EINVAL;
    int rc = check_points(x, y, n_total);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(hipSetDevice(ctx->device));
    const int64_t n1 = offsets ? 0 : n_total;
    if (!offsets && S != 1) return HULL_EINVAL;
    LAUNCH(K_HIST32, k_hist32<<<(unsigned)S, HIST_THREADS, 0, st>>>(x, y, offsets, n1, S, hist, hist_f32));
    return HULL_OK;
}

int hull_mlp_forward(hull_ctx *ctx, const uint16_t *hist, int64_t B, float *scores, void *stream) {
    if (!ctx || !hist || !scores || B <= 0) return HULL_EINVAL;
    if (!ctx->learned.loaded) return HULL_ENOMODEL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(hipSetDevice(ctx->device));
    RC(mlp_forward(ctx, st, hist, B));
    HIPCHECK(hipMemcpyAsync(scores, ctx->learned.scores, B * NOUT * sizeof(float),
                            hipMemcpyDeviceToDevice, st));
    return HULL_OK;
}

int hull_mlp_backward(hull_ctx *ctx, const uint16_t *hist, const float *dscores, int64_t B,
                      float *grads, void *stream) {
    if (!ctx || !hist || !dscores || !grads || B <= 0) return HULL_EINVAL;
    if (!ctx->learned.loaded) return HULL_ENOMODEL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(hipSetDevice(ctx->device));
    RC(mlp_forward(ctx, st, hist, B));
    LearnedState &L = ctx->learned;
    const int Bp = (int)std::max<int64_t>(64, (B + 63) / 64 * 64);
    LAUNCH(K_MLP, k_pad_f32_bf16<<<256, 256, 0, st>>>(dscores, B, Bp, NOUT, L.dS));
    RC(mlp_backward(ctx, st, B));
    HIPCHECK(hipMemcpyAsync(grads, L.grads, P_TOTAL * sizeof(float), hipMemcpyDeviceToDevice, st));
    return HULL_OK;
}

int hull_mlp_train_step(hull_ctx *ctx, const uint16_t *hist, const float *gain, int64_t B, float lr,
                        float *loss, void *stream) {
    if (!ctx || !hist || !gain || !loss || B <= 0 || !(lr > 0)) return HULL_EINVAL;
    if (!ctx->learned.loaded) return HULL_ENOMODEL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(hipSetDevice(ctx->device));
    RC(mlp_forward(ctx, st, hist, B));
    LearnedState &L = ctx->learned;
    const int Bp = (int)std::max<int64_t>(64, (B + 63) / 64 * 64);
    LAUNCH(K_MLP, k_loss<<<(unsigned)Bp, 64, 0, st>>>(L.scores, gain, B, Bp, L.dS, L.part));
    LAUNCH(K_MLP, k_loss_sum<<<1, 64, 0, st>>>(L.part, B, loss));
    RC(mlp_backward(ctx, st, B));
    L.step++;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - std::pow(b1, (float)L.step), c2 = 1.0f - std::pow(b2, (float)L.step);
    LAUNCH(K_MLP, k_adam<<<1024, 256, 0, st>>>(L.params, L.grads, L.m1, L.m2, P_TOTAL, lr, b1, b2,
                                               eps, c1, c2, L.wb));
    return HULL_OK;
}

int hull_set_direction_gap(hull_ctx *ctx, int gap) {
    if (!ctx || gap < 0 || gap > 3) return HULL_EINVAL;
    ctx->dir_gap = gap;
    return HULL_OK;
}

int hull_top_directions(hull_ctx *ctx, const float *scores, int64_t S, int32_t *dirs, void *stream) {
    if (!ctx || !scores || !dirs || S <= 0) return HULL_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(hipSetDevice(ctx->device));
    RC(init_cand_table());
    Plan p;
    RC(prepare(ctx, 0, S, st, &p));
    LAUNCH(K_MLP, k_top8<<<(unsigned)((S + 3) / 4), 256, 0, st>>>(scores, S, ctx->dir_gap, dirs,
                                                                 W<double>(p, p.setdirs)));
    return HULL_OK;
}

int hull_labels_batched(hull_ctx *ctx, const float *x, const float *y, const int64_t *offsets,
                        int64_t S, int64_t n_total, float *gain, void *stream) {
    if (!ctx || !gain || !learned_ok(ctx)) return HULL_EINVAL;
    int rc = check_batch(x, y, offsets, S, n_total);
    if (rc) return rc;
    RC(init_cand_table());
    hipStream_t st = (hipStream_t)stream;
    Plan p;
    RC(prepare(ctx, n_total, S, st, &p));
    RC(run_tilemap(ctx, p, st, x, offsets, 0, S));
    RC(run_extremes(ctx, p, st, x, y, n_total, offsets, 0, S, false));
    RC(run_polygon(ctx, p, st, x, y, n_total, S, false, nullptr, 0, nullptr, nullptr));
    uint32_t *surv = W<uint32_t>(p, p.surv);
    int64_t *so = W<int64_t>(p, p.surv_off);
    RC(run_discard(ctx, p, st, x, y, n_total, offsets, 0, S, slot_count(ctx, false), surv, so, nullptr));
    uint32_t *cand = W<uint32_t>(p, p.cand);
    LAUNCH(K_LABELS, k_cand_extremes<<<(unsigned)S, 256, 0, st>>>(x, y, offsets, 0, S, cand));
    LAUNCH(K_LABELS, k_labels<<<(unsigned)S, 256, 0, st>>>(x, y, offsets, 0, S, W<Poly>(p, p.polys),
                                                          cand, surv, so, gain));
    return HULL_OK;
}

int hull_label_targets_batched(hull_ctx *ctx, const float *x, const float *y,
                               const int64_t *offsets, int64_t S, int64_t n_total, int rounds,
                               float *target, int32_t *order, void *stream) {
    if (!ctx || !target || !order || rounds < 1 || rounds > LT_MAXR || !learned_ok(ctx))
        return HULL_EINVAL;
    int rc = check_batch(x, y, offsets, S, n_total);
    if (rc) return rc;
    RC(init_cand_table());
    hipStream_t st = (hipStream_t)stream;
    Plan p;
    RC(prepare(ctx, n_total, S, st, &p));
    RC(run_tilemap(ctx, p, st, x, offsets, 0, S));
    RC(run_extremes(ctx, p, st, x, y, n_total, offsets, 0, S, false));
    RC(run_polygon(ctx, p, st, x, y, n_total, S, false, nullptr, 0, nullptr, nullptr));
    uint32_t *surv = W<uint32_t>(p, p.surv);
    int64_t *so = W<int64_t>(p, p.surv_off);
    RC(run_discard(ctx, p, st, x, y, n_total, offsets, 0, S, slot_count(ctx, false), surv, so, nullptr));
    uint32_t *cand = W<uint32_t>(p, p.cand);
    LAUNCH(K_LABELS, k_cand_extremes<<<(unsigned)S, 256, 0, st>>>(x, y, offsets, 0, S, cand));
    LAUNCH(K_LABELS, k_label_targets<<<(unsigned)S, 256, 0, st>>>(
        x, y, offsets, 0, S, W<Poly>(p, p.polys), cand, surv, so, rounds, target, order));
    return HULL_OK;
}

}  // extern "C"

#include "hull_stream.hip"
#include "hull3d_host.hip"
