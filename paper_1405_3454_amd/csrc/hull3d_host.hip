// The 3D form of the method (hull3_compute); included by hull_lib.hip after
// its launch sequences.  The kernels are in k_hull3d.hip; the tile map,
// survivor scan and scatter, the radix sort and the 2D hull stage (for flat
// sets) are the 2D path's.

// Device buffers of the 3D path, owned by the context and grown on demand:
// A holds what the filter passes need, B the hull stage (sized once the
// survivor count is known).
struct Hull3Bufs {
    char *a = nullptr, *b = nullptr;
    size_t acap = 0, bcap = 0;
};

static void hull3_free(Hull3Bufs *h) {
    if (!h) return;
    if (h->a) (void)hipFree(h->a);
    if (h->b) (void)hipFree(h->b);
    delete h;
}

static int grow(char **p, size_t *cap, size_t want) {
    if (want <= *cap) return HULL_OK;
    if (*p && hipFree(*p) != hipSuccess) { (void)hipGetLastError(); }
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(p, want) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return HULL_ENOMEM;
    }
    *cap = want;
    return HULL_OK;
}

extern "C" int hull3_compute(hull_ctx *ctx, const float *x, const float *y, const float *z, int64_t n,
                             uint32_t *slots, uint32_t *surv, int64_t *n_surv, uint32_t *hull,
                             int64_t *h, int flags, void *stream) {
    if (!ctx || !hull || !h || n < 0 || (flags & ~(HULL_NOFILTER | HULL3_SERIAL))) return HULL_EINVAL;
    if (n >= (int64_t(1) << 32) - 1) return HULL_ETOOBIG;
    if (n > 0 && (!x || !y || !z)) return HULL_EINVAL;
    if (((uintptr_t)x | (uintptr_t)y | (uintptr_t)z) & 15) return HULL_EINVAL;
    if (preset_groups(ctx->preset) != 4) return HULL_EINVAL;     // the paper's two tables
    hipStream_t st = (hipStream_t)stream;
    HIPCHECK(hipSetDevice(ctx->device));
    if (!ctx->h3) ctx->h3 = new Hull3Bufs();
    Hull3Bufs *B = ctx->h3;
    const bool nofilter = flags & HULL_NOFILTER;
    int rc;
    Plan p;
    if ((rc = prepare(ctx, std::max<int64_t>(n, 1), 1, st, &p))) return rc;
    // A: wave partials of the extremes, the polyhedron, the hull control
    const int bpc3 = std::max(1, resident_blocks((const void *)k3_extremes<0>, 256));
    const unsigned g3 = (unsigned)(ctx->cus * std::min(bpc3, 2));
    const int64_t W3 = (int64_t)g3 * 4;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += al(bytes); return r; };
    const size_t a_pval = take(W3 * S3 * 8), a_pidx = take(W3 * S3 * 4), a_poly = take(sizeof(Poly3)),
                 a_ctl = take(sizeof(Hull3Ctl)), a_cnt = take(8);
    if ((rc = grow(&B->a, &B->acap, o))) return rc;
    double *pval = reinterpret_cast<double *>(B->a + a_pval);
    uint32_t *pidx = reinterpret_cast<uint32_t *>(B->a + a_pidx);
    Poly3 *poly = reinterpret_cast<Poly3 *>(B->a + a_poly);
    Hull3Ctl *C = reinterpret_cast<Hull3Ctl *>(B->a + a_ctl);
    int64_t *scount = reinterpret_cast<int64_t *>(B->a + a_cnt);
    uint32_t *sv = surv ? surv : W<uint32_t>(p, p.surv);
    int64_t *so = W<int64_t>(p, p.surv_off);
    if (!nofilter) {
        // Steps 1-3
        if ((rc = run_tilemap(ctx, p, st, x, nullptr, n, 1))) return rc;
        const Dirs d = ctx->dirs;
        LAUNCH(K_EXTREMES, (k3_extremes<0><<<g3, 256, 0, st>>>(x, y, z, n, d, pval, pidx)));
        LAUNCH(K_EXTREMES, (k3_extremes<1><<<g3, 256, 0, st>>>(x, y, z, n, d, pval, pidx)));
        LAUNCH(K_POLYGON, k3_poly<<<1, 1024, 0, st>>>(x, y, z, W3, pval, pidx, slots, poly));
        const unsigned gd = (unsigned)(ctx->cus * 4);
        LAUNCH(K_DISCARD, k3_discard<<<gd, 256, 0, st>>>(x, y, z, n, poly, W<uint64_t>(p, p.masks),
                                                        W<uint32_t>(p, p.tile_cnt)));
        const int64_t *tile_off = W<int64_t>(p, p.tile_off);
        if ((rc = run_scan(ctx, p, st, W<uint32_t>(p, p.tile_cnt), tile_off + 1, W<int64_t>(p, p.tile_pos))))
            return rc;
        LAUNCH(K_SCATTER, k_set_offsets<<<1, 256, 0, st>>>(tile_off, W<int64_t>(p, p.tile_pos), 1, so));
        uint64_t *nokeys = nullptr;
        const int64_t *nobase = nullptr;
        LAUNCH(K_SCATTER, k_scatter<<<gd, 256, 0, st>>>(x, y, n, phase_of(x), nullptr, 1, tile_off,
                                                        W<int32_t>(p, p.tile_set), W<uint64_t>(p, p.masks),
                                                        W<uint32_t>(p, p.tile_cnt), W<int64_t>(p, p.tile_pos),
                                                        sv, nokeys, nobase, INT64_MAX));
        LAUNCH(K_MISC, k_copy_count<<<1, 64, 0, st>>>(so + 1, scount));
    } else {
        LAUNCH(K_MISC, k3_iota<<<1024, 256, 0, st>>>(sv, n));
        LAUNCH(K_MISC, k_fill_i64<<<1, 64, 0, st>>>(scount, 1, n));
    }
    if (n_surv) LAUNCH(K_MISC, k_copy_count<<<1, 64, 0, st>>>(scount, n_surv));
    int64_t nc = 0;
    HIPCHECK(hipMemcpyAsync(&nc, scount, 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));

    // Step 4, with face room grown and the hull restarted if it runs out
    for (int64_t fcap = std::min<int64_t>(8 * nc + 1024, int64_t(1) << 24);; fcap *= 2) {
        size_t ob = 0;
        auto tb = [&](size_t bytes) { size_t r = ob; ob += al(bytes); return r; };
        const size_t b_idx = tb(nc * 4 + 16), b_ca = tb(nc * 16 + 16), b_cb = tb(nc * 16 + 16),
                     b_fa = tb(nc * 4 + 16), b_fb = tb(nc * 4 + 16), b_faces = tb(fcap * sizeof(Face3)),
                     b_planes = tb(fcap * sizeof(Plane3)), b_far = tb(fcap * 8), b_vis = tb(fcap * 4),
                     b_repl = tb(fcap * sizeof(int2)), b_claim = tb(fcap * 8),
                     b_pairs = tb(PAIR_CAP * sizeof(Pair3)), b_pn = tb(PAIR_CAP * sizeof(int2)),
                     b_pv = tb((size_t)PAIR_CAP * PV_CAP * 4), b_ph = tb((size_t)PAIR_CAP * PV_CAP * 4),
                     b_corner = tb(nc * 8 + 16), b_ncorner = tb(16);
        if ((rc = grow(&B->b, &B->bcap, ob))) return rc;
        char *hb = B->b;
        uint32_t *cidx = reinterpret_cast<uint32_t *>(hb + b_idx);
        float4 *cand[2] = {reinterpret_cast<float4 *>(hb + b_ca), reinterpret_cast<float4 *>(hb + b_cb)};
        int *cf[2] = {reinterpret_cast<int *>(hb + b_fa), reinterpret_cast<int *>(hb + b_fb)};
        unsigned long long *claim = reinterpret_cast<unsigned long long *>(hb + b_claim);
        Pair3 *pairs = reinterpret_cast<Pair3 *>(hb + b_pairs);
        int2 *pn = reinterpret_cast<int2 *>(hb + b_pn);
        int *pvis = reinterpret_cast<int *>(hb + b_pv);
        int *phz = reinterpret_cast<int *>(hb + b_ph);
        Face3 *faces = reinterpret_cast<Face3 *>(hb + b_faces);
        Plane3 *planes = reinterpret_cast<Plane3 *>(hb + b_planes);
        unsigned long long *far = reinterpret_cast<unsigned long long *>(hb + b_far);
        int *vis = reinterpret_cast<int *>(hb + b_vis);
        int2 *repl = reinterpret_cast<int2 *>(hb + b_repl);
        uint64_t *corner = reinterpret_cast<uint64_t *>(hb + b_corner);
        int *ncorner = reinterpret_cast<int *>(hb + b_ncorner);
        if (nc > 0)
            HIPCHECK(hipMemcpyAsync(cidx, sv, nc * 4, hipMemcpyDeviceToDevice, st));
        LAUNCH(K_MISC, k3_ctl_init<<<1, 64, 0, st>>>(C, (int)fcap));
        const unsigned gs = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ctx->cus * 4, (nc + 255) / 256));
        for (int phase = 1; phase <= 3; phase++)
            LAUNCH(K_MISC, k3_seed<<<gs, 256, 0, st>>>(x, y, z, cidx, nc, phase, C));
        LAUNCH(K_MISC, k3_start<<<1, 64, 0, st>>>(x, y, z, cidx, nc, C, faces, planes, far));
        Hull3Ctl hc;
        HIPCHECK(hipMemcpyAsync(&hc, C, sizeof(hc), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        if (hc.state == 2) {
            LAUNCH(K_MISC, k3_line<<<gs, 256, 0, st>>>(x, y, z, cidx, nc, 0, C));
            LAUNCH(K_MISC, k3_line<<<gs, 256, 0, st>>>(x, y, z, cidx, nc, 1, C));
        }
        if (hc.state >= 2) {
            LAUNCH(K_MISC, k3_small_out<<<1, 64, 0, st>>>(C, hull, h));
            return HULL_OK;
        }
        Plan ph;
        if ((rc = prepare(ctx, std::max<int64_t>(nc, 1), 1, st, &ph))) return rc;
        int64_t *hcount = W<int64_t>(ph, ph.hoff) + 1;      // count slot for the sort
        const uint64_t *sorted = nullptr;
        if (hc.state == 1) {
            // flat: the 2D hull of the coordinates kept in the plane
            uint64_t *keys = W<uint64_t>(ph, ph.keys0);
            LAUNCH(K_KEYS, k3_flat_keys<<<gs, 256, 0, st>>>(x, y, z, cidx, nc, C, keys));
            LAUNCH(K_MISC, k_fill_i64<<<1, 64, 0, st>>>(scount, 1, nc));
            uint32_t *h2 = W<uint32_t>(ph, ph.cidx);
            int64_t *hoff = W<int64_t>(ph, ph.hoff);
            if ((rc = run_hull(ctx, ph, st, cidx, keys, scount, std::max<int64_t>(nc, 1), 1, hoff, h2,
                               hcount)))
                return rc;
            LAUNCH(K_MISC, k3_u64_of<<<256, 256, 0, st>>>(h2, hcount, corner));
        } else {
            LAUNCH(K_MISC, k3_fill_i32<<<256, 256, 0, st>>>(vis, fcap, -1));
            LAUNCH(K_MISC, k_fill_i64<<<256, 256, 0, st>>>(reinterpret_cast<int64_t *>(claim), fcap, 0));
            LAUNCH(K_MISC, k3_gather<<<gs, 256, 0, st>>>(x, y, z, cidx, nc, cand[0]));
            const unsigned gp = (unsigned)(ctx->cus * 4), gv = (unsigned)(ctx->cus * 16);
            const unsigned ga = (unsigned)std::max<int64_t>(
                1, std::min<int64_t>(ctx->cus * 4, (nc + 256 * AS_ITEMS - 1) / (256 * AS_ITEMS)));
            int cur = 0;
            const bool all_serial = flags & HULL3_SERIAL;
            bool overflow = false, serial = all_serial;
            for (int round = 0;; round++) {
                LAUNCH(K_REFINE, k3_assign<<<ga, 256, 0, st>>>(cand[cur], cf[cur], cand[1 - cur], cf[1 - cur], C,
                                                               faces, planes, repl, far, round == 0));
                if (serial) {
                    // one block inserts every face's farthest candidate in turn
                    LAUNCH(K_REFINE_SPLIT, k3_insert<<<1, INS_THREADS, 0, st>>>(x, y, z, C, faces, planes, far,
                                                                                 vis, repl));
                } else {
                    LAUNCH(K_REFINE_SPLIT, k3_pick<<<gp, 256, 0, st>>>(C, far, pairs));
                    for (int sub = 0; sub < INS_PASSES; sub++) {
                        const int stamp = round * INS_PASSES + sub + 1;
                        LAUNCH(K_REFINE_SPLIT, k3_visible<<<gv, 64, 0, st>>>(x, y, z, C, faces, planes, pairs, pvis,
                                                                              phz, pn, claim, stamp));
                        LAUNCH(K_REFINE_SPLIT, k3_apply<<<gv, 64, 0, st>>>(x, y, z, C, faces, planes, far, vis,
                                                                            repl, pairs, pvis, phz, pn, claim,
                                                                            stamp));
                    }
                    LAUNCH(K_MISC, k3_round_end<<<1, 64, 0, st>>>(C));
                }
                HIPCHECK(hipMemcpyAsync(&hc, C, sizeof(hc), hipMemcpyDeviceToHost, st));
                HIPCHECK(hipStreamSynchronize(st));
                cur = 1 - cur;
                if (hc.overflow == 2) return HULL_EHIP;      // internal: the mesh lost its shape
                if (hc.overflow) { overflow = true; break; }
                if (hc.ncand == 0) break;
                if ((round + 2) * INS_PASSES >= (1 << 20)) return HULL_EHIP;
                // a round whose proposals all exceeded the per-proposal room
                // is followed by one serial round
                serial = all_serial || (!serial && hc.inserted == 0);
            }
            if (overflow) {
                if (fcap >= (int64_t(1) << 28)) return HULL_ENOMEM;
                continue;
            }
            LAUNCH(K_MISC, k3_fill_i32<<<1, 64, 0, st>>>(ncorner, 1, 0));
            LAUNCH(K_FINAL, k3_corners<<<(unsigned)std::max(1, std::min(ctx->cus * 4, (3 * hc.nfaces + 255) / 256)),
                                         256, 0, st>>>(C, faces, planes, corner, ncorner));
            LAUNCH(K_MISC, k3_count_i64<<<1, 64, 0, st>>>(ncorner, hcount));
        }
        // ascending indices
        if ((rc = run_sort(ctx, ph, st, corner, hcount, 4, 1, &sorted))) return rc;
        LAUNCH(K_MISC, k3_copy_sorted<<<256, 256, 0, st>>>(sorted, hcount, hull, h));
        return HULL_OK;
    }
}
