// Host-resident input: the whole method for a set that lives in host memory
// (the paper's setting, Sec. 3: its card held at most ~20M points, so the
// points were moved to the device first).  Included by hull_lib.hip after its
// launch sequences.
//
// The points cross PCIe in chunks through device buffers: two streaming
// buffers used in turn, plus as many resident chunk buffers as the caller's
// device budget allows.  Pass 1 runs Step 1 on every chunk and folds the
// chunk's extremes into a running best per slot (better value, then lower
// index, exactly the single-set rule), keeping the winners' coordinates.
// The filter polygon is then built from those coordinates alone.  Pass 2
// copies the non-resident chunks again and runs Step 3 on each, appending
// its survivors (global indices, ascending) and their keys.  The hull of the
// survivors follows on the device from the keys (sort + monotone chain).
//
// A chunk c covering global points [a, b) sits in a device buffer d; the
// kernels get x = d - a, so that global index i addresses d[i - a], with
// offsets {a, b} as a one-set CSR: every index the kernels form lies in
// [a, b), and a is a multiple of the tile size, so the buffer's alignment
// carries over.  Copies run on a second stream, ordered against the kernels
// by events, so chunk c + 1 crosses PCIe while chunk c is processed.

namespace hg {

__global__ void k_chunk_offsets(int64_t *__restrict__ off, int64_t nch, int64_t chunk, int64_t n) {
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c <= nch;
         c += int64_t(gridDim.x) * blockDim.x)
        off[c] = min(c * chunk, n);
}

__global__ void k_slot_init(uint32_t *__restrict__ bi, int ns) {
    if ((int)threadIdx.x < ns) bi[threadIdx.x] = NONE;
}

// Fold one chunk's slots (global indices cs, values cv) into the running best
// (bi, bv) and record the winners' coordinates (bx, by).  xs, ys address the
// chunk's points by global index.
__global__ void k_slot_merge(const uint32_t *__restrict__ cs, const double *__restrict__ cv, int ns,
                             int nfix, const float *__restrict__ xs, const float *__restrict__ ys,
                             uint32_t *__restrict__ bi, double *__restrict__ bv,
                             float *__restrict__ bx, float *__restrict__ by) {
    const int k = threadIdx.x;
    if (k >= ns) return;
    const uint32_t i = cs[k];
    if (i == NONE) return;
    const double v = cv[k];
    if (bi[k] == NONE || better(slot_is_min(k, nfix), v, i, bv[k], bi[k])) {
        bi[k] = i;
        bv[k] = v;
        bx[k] = xs[i];
        by[k] = ys[i];
    }
}

// Polygon input from the winners: slot k names point k of (bx, by), empty
// slots stay empty; the global slots go to slots_out (optional).
__global__ void k_slot_compact(const uint32_t *__restrict__ bi, int ns, uint32_t *__restrict__ cidx,
                               uint32_t *__restrict__ slots_out) {
    const int k = threadIdx.x;
    if (k >= ns) return;
    cidx[k] = bi[k] == NONE ? NONE : (uint32_t)k;
    if (slots_out) slots_out[k] = bi[k];
}

__global__ void k_count_add(int64_t *__restrict__ acc, const int64_t *__restrict__ add) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *acc += *add;
}

}  // namespace hg

// Buffers of the host-resident path, owned by the context and grown on
// demand.
struct StreamBufs {
    int64_t chunk = 0;            // points per chunk buffer
    int nbuf = 0;                 // device chunk buffers: 2 streaming + resident
    float *dev = nullptr;         // [nbuf][x | y][chunk]
    float *pin = nullptr;         // pinned staging [2][x | y][chunk]
    uint64_t *keys = nullptr;     // survivor keys
    int64_t keys_cap = 0;
    char *small = nullptr;        // slot records, chunk offsets, counter
    int64_t small_nch = -1;       // chunk offsets room
    hipStream_t cs = nullptr;     // copy stream
    hipEvent_t copied[2] = {};    // staging slot s free again
    hipEvent_t done[2] = {};      // streaming buffer r free again
    bool events = false;
};

static void stream_free(StreamBufs *b) {
    if (!b) return;
    if (b->dev) (void)hipFree(b->dev);
    if (b->pin) (void)hipHostFree(b->pin);
    if (b->keys) (void)hipFree(b->keys);
    if (b->small) (void)hipFree(b->small);
    if (b->events) {
        for (int i = 0; i < 2; i++) {
            (void)hipEventDestroy(b->copied[i]);
            (void)hipEventDestroy(b->done[i]);
        }
    }
    if (b->cs) (void)hipStreamDestroy(b->cs);
    delete b;
}

// Layout of the small device arrays: chunk slots and values, running best
// (index, value, x, y), compacted polygon input, survivor counter, chunk
// offsets.
struct SmallPlan {
    size_t cslots, cvals, bi, bv, bx, by, cidx, counter, offs, total;
};
static SmallPlan small_plan(int64_t nch) {
    SmallPlan s;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += al(bytes);
        return r;
    };
    s.cslots = take(MAX_SLOTS * 4);
    s.cvals = take(MAX_SLOTS * 8);
    s.bi = take(MAX_SLOTS * 4);
    s.bv = take(MAX_SLOTS * 8);
    s.bx = take(MAX_SLOTS * 4);
    s.by = take(MAX_SLOTS * 4);
    s.cidx = take(MAX_SLOTS * 4);
    s.counter = take(8);
    s.offs = take((nch + 1) * 8);
    s.total = o;
    return s;
}

static bool host_pinned(const void *p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeHost || a.type == hipMemoryTypeManaged;
}

static int stream_ensure(hull_ctx *ctx, int64_t chunk, int nbuf, int64_t keys_cap, int64_t nch,
                         bool staging) {
    if (!ctx->sb) ctx->sb = new StreamBufs();
    StreamBufs *b = ctx->sb;
    HIPCHECK(hipDeviceSynchronize());
    if (!b->cs) HIPCHECK(hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking));
    if (!b->events) {
        for (int i = 0; i < 2; i++) {
            HIPCHECK(hipEventCreateWithFlags(&b->copied[i], hipEventDisableTiming));
            HIPCHECK(hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming));
        }
        b->events = true;
    }
    if (b->chunk != chunk || b->nbuf < nbuf) {
        if (b->dev) HIPCHECK(hipFree(b->dev));
        b->dev = nullptr;
        b->nbuf = 0;
        if (b->pin) HIPCHECK(hipHostFree(b->pin));
        b->pin = nullptr;
        if (hipMalloc(&b->dev, (size_t)nbuf * 2 * chunk * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            b->dev = nullptr;
            return HULL_ENOMEM;
        }
        b->nbuf = nbuf;
        b->chunk = chunk;
    }
    if (staging && !b->pin) {
        if (hipHostMalloc(&b->pin, (size_t)2 * 2 * chunk * sizeof(float), hipHostMallocDefault) !=
            hipSuccess) {
            (void)hipGetLastError();
            b->pin = nullptr;
            return HULL_ENOMEM;
        }
    }
    if (b->keys_cap < keys_cap) {
        if (b->keys) HIPCHECK(hipFree(b->keys));
        b->keys = nullptr;
        b->keys_cap = 0;
        if (hipMalloc(&b->keys, (size_t)keys_cap * 8 + 16) != hipSuccess) {
            (void)hipGetLastError();
            b->keys = nullptr;
            return HULL_ENOMEM;
        }
        b->keys_cap = keys_cap;
    }
    if (b->small_nch < nch) {
        if (b->small) HIPCHECK(hipFree(b->small));
        b->small = nullptr;
        b->small_nch = -1;
        if (hipMalloc(&b->small, small_plan(nch).total) != hipSuccess) {
            (void)hipGetLastError();
            b->small = nullptr;
            return HULL_ENOMEM;
        }
        b->small_nch = nch;
    }
    return HULL_OK;
}

extern "C" int hull_compute_host(hull_ctx *ctx, const float *x, const float *y, int64_t n,
                                 int64_t chunk_points, int64_t device_budget, uint32_t *slots,
                                 uint32_t *surv, int64_t *n_surv, int64_t cap, uint32_t *hull,
                                 int64_t *h, int flags, void *stream) {
    if (!ctx || !surv || !n_surv || !hull || !h || cap < 0 || device_budget < 0 || flags != 0 ||
        chunk_points < 0)
        return HULL_EINVAL;
    if (n < 0) return HULL_EINVAL;
    if (n >= (int64_t(1) << 32) - 1) return HULL_ETOOBIG;
    if (n > 0 && (!x || !y)) return HULL_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(hipSetDevice(ctx->device));
    int64_t chunk = chunk_points ? chunk_points : (int64_t(1) << 24);
    chunk = (chunk + TILE - 1) / TILE * TILE;
    chunk = std::min<int64_t>(chunk, std::max<int64_t>(TILE, (n + TILE - 1) / TILE * TILE));
    const int64_t nch = (n + chunk - 1) / chunk;
    // chunks that stay on the device after pass 1 (all of them: one crossing)
    const int64_t per = chunk * 2 * (int64_t)sizeof(float);
    const int64_t nres = nch <= 2 ? nch : std::min<int64_t>(nch, device_budget / per);
    const int nstream = nres == nch ? 0 : 2;
    const bool pinned = n == 0 || (host_pinned(x) && host_pinned(y));
    int rc = stream_ensure(ctx, chunk, (int)std::max<int64_t>(1, nres + nstream), std::max<int64_t>(cap, 1),
                           nch, !pinned);
    if (rc) return rc;
    StreamBufs *B = ctx->sb;
    Plan p;
    if ((rc = prepare(ctx, chunk, 1, st, &p))) return rc;
    const SmallPlan sp = small_plan(nch);
    auto S8 = [&](size_t off) { return B->small + off; };
    uint32_t *cslots = reinterpret_cast<uint32_t *>(S8(sp.cslots));
    double *cvals = reinterpret_cast<double *>(S8(sp.cvals));
    uint32_t *bi = reinterpret_cast<uint32_t *>(S8(sp.bi));
    double *bv = reinterpret_cast<double *>(S8(sp.bv));
    float *bx = reinterpret_cast<float *>(S8(sp.bx));
    float *by = reinterpret_cast<float *>(S8(sp.by));
    uint32_t *cidx = reinterpret_cast<uint32_t *>(S8(sp.cidx));
    int64_t *counter = reinterpret_cast<int64_t *>(S8(sp.counter));
    int64_t *offs = reinterpret_cast<int64_t *>(S8(sp.offs));
    const int ns = slot_count(ctx, false);
    const int nfix = preset_fixed_slots(ctx->preset);

    // every event starts recorded, so the first waits pass at once
    for (int i = 0; i < 2; i++) {
        HIPCHECK(hipEventRecord(B->copied[i], B->cs));
        HIPCHECK(hipEventRecord(B->done[i], st));
    }
    LAUNCH(K_MISC, k_chunk_offsets<<<1, 256, 0, st>>>(offs, nch, chunk, n));
    LAUNCH(K_MISC, k_slot_init<<<1, 64, 0, st>>>(bi, ns));
    LAUNCH(K_MISC, k_fill_i64<<<1, 64, 0, st>>>(counter, 1, 0));
    int64_t copies = 0;     // staging slots used so far

    // Device buffer of chunk c (x part; y follows chunk floats later), and
    // the copy that brings it there when `copy`.
    auto chunk_ptr = [&](int64_t c) -> float * {
        const int64_t slot = c < nres ? c : nres + (c - nres) % 2;
        return B->dev + slot * 2 * chunk;
    };
    auto bring = [&](int64_t c) -> int {
        const int64_t a = c * chunk, m = std::min(n, a + chunk) - a;
        float *d = chunk_ptr(c);
        const int ring = c < nres ? -1 : (int)((c - nres) % 2);
        const float *sx = x + a, *sy = y + a;
        const int sl = (int)(copies++ % 2);
        if (!pinned) {
            // staging slot sl is free once its last copy has finished
            HIPCHECK(hipEventSynchronize(B->copied[sl]));
            float *px = B->pin + (size_t)sl * 2 * chunk;
            std::memcpy(px, sx, (size_t)m * sizeof(float));
            std::memcpy(px + chunk, sy, (size_t)m * sizeof(float));
            sx = px;
            sy = px + chunk;
        }
        // a streaming buffer is free once the kernels of its last chunk ran
        if (ring >= 0) HIPCHECK(hipStreamWaitEvent(B->cs, B->done[ring], 0));
        HIPCHECK(hipMemcpyAsync(d, sx, (size_t)m * sizeof(float), hipMemcpyHostToDevice, B->cs));
        HIPCHECK(hipMemcpyAsync(d + chunk, sy, (size_t)m * sizeof(float), hipMemcpyHostToDevice, B->cs));
        HIPCHECK(hipEventRecord(B->copied[sl], B->cs));
        HIPCHECK(hipStreamWaitEvent(st, B->copied[sl], 0));
        return HULL_OK;
    };
    auto release = [&](int64_t c) -> int {
        if (c >= nres) HIPCHECK(hipEventRecord(B->done[(c - nres) % 2], st));
        return HULL_OK;
    };

    // pass 1: extremes of every chunk folded into the running best
    for (int64_t c = 0; c < nch; c++) {
        if ((rc = bring(c))) return rc;
        const int64_t a = c * chunk, b = std::min(n, a + chunk);
        const float *xs = chunk_ptr(c) - a, *ys = chunk_ptr(c) + chunk - a;
        if ((rc = run_tilemap(ctx, p, st, xs, offs + c, 0, 1))) return rc;
        if ((rc = run_extremes(ctx, p, st, xs, ys, b, offs + c, 0, 1, false))) return rc;
        if ((rc = run_polygon(ctx, p, st, xs, ys, b, 1, false, nullptr, 0, cslots, cvals))) return rc;
        LAUNCH(K_MISC, k_slot_merge<<<1, 64, 0, st>>>(cslots, cvals, ns, nfix, xs, ys, bi, bv, bx, by));
        if ((rc = release(c))) return rc;
    }
    // the filter polygon from the winners' coordinates
    LAUNCH(K_MISC, k_slot_compact<<<1, 64, 0, st>>>(bi, ns, cidx, slots));
    if ((rc = run_polygon(ctx, p, st, bx, by, ns, 1, false, cidx, ns, nullptr, nullptr))) return rc;
    // pass 2: Step 3 per chunk, survivors appended in ascending index order
    int64_t *so = W<int64_t>(p, p.surv_off);
    for (int64_t c = 0; c < nch; c++) {
        if (c >= nres && (rc = bring(c))) return rc;
        const int64_t a = c * chunk, b = std::min(n, a + chunk);
        const float *xs = chunk_ptr(c) - a, *ys = chunk_ptr(c) + chunk - a;
        if ((rc = run_tilemap(ctx, p, st, xs, offs + c, 0, 1))) return rc;
        if ((rc = run_discard(ctx, p, st, xs, ys, b, offs + c, 0, 1, ns, surv, so, B->keys, counter,
                              cap)))
            return rc;
        LAUNCH(K_MISC, k_count_add<<<1, 64, 0, st>>>(counter, so + 1));
        if ((rc = release(c))) return rc;
    }
    LAUNCH(K_MISC, k_copy_count<<<1, 64, 0, st>>>(counter, n_surv));
    int64_t total = 0;
    HIPCHECK(hipMemcpyAsync(&total, counter, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (total > cap) return HULL_EOVERFLOW;
    // hull of the survivors (the hull stage reads keys only)
    Plan ph;
    if ((rc = prepare(ctx, std::max<int64_t>(total, 1), 1, st, &ph))) return rc;
    int64_t *hoff = W<int64_t>(ph, ph.hoff);
    return run_hull(ctx, ph, st, surv, B->keys, counter, std::max<int64_t>(total, 1), 1, hoff, hull, h);
}
