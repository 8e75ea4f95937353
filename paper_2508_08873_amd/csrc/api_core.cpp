// Host side of the C ABI: contexts, factors, batched fine/adjoint sweeps.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "lrpr_internal.h"

using namespace lrpr;

namespace lrpr {

lrpr_status fail(lrpr_ctx ctx, lrpr_status st, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return st;
}

static lrpr_status hipfail(lrpr_ctx ctx, hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? LRPR_ERR_NOMEM : LRPR_ERR_HIP, m);
}

}  // namespace lrpr

#define HIPCHK(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return lrpr::hipfail(ctx, e_, what); \
    } while (0)

extern "C" {

lrpr_status lrpr_ctx_create(int device, void *hip_stream, lrpr_ctx *out) {
    if (!out) return LRPR_ERR_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LRPR_ERR_ARG;
    lrpr_ctx ctx = new (std::nothrow) lrpr_ctx_s();
    if (!ctx) return LRPR_ERR_NOMEM;
    ctx->dev = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return LRPR_ERR_HIP;
    }
    *out = ctx;
    return LRPR_OK;
}

void lrpr_ctx_destroy(lrpr_ctx ctx) {
    if (!ctx) return;
    hipSetDevice(ctx->dev);
    hipStreamSynchronize(ctx->stream);
    if (ctx->d_items) hipFree(ctx->d_items);
    for (auto &kv : ctx->ws)
        if (kv.second.first) hipFree(kv.second.first);
    delete ctx;
}

lrpr_status lrpr_ctx_set_stream(lrpr_ctx ctx, void *hip_stream) {
    if (!ctx) return LRPR_ERR_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return LRPR_OK;
}

const char *lrpr_last_error(lrpr_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// ---------------------------------------------------------------------------
static void free_tiles(TileSet &t) {
    for (void *p : t.alloc)
        if (p) hipFree(p);
    if (t.zt) hipFree(t.zt);
    if (t.sink) hipFree(t.sink);
    t = TileSet();
}

// Tile arrays with guard_rows(nb) zero tile rows on both sides; the TileSet
// pointers address tile row 0.  The mirrored band arrays only with `mirror`.
static hipError_t alloc_tiles(TileSet &t, int NT, int nb, size_t esz, bool mirror) {
    const size_t G = (size_t)guard_rows(nb);
    const size_t rows = (size_t)NT + 2 * G;
    hipError_t e;
    for (int a = 0; a < TS_COUNT; ++a) {
        const bool band = a == TS_LB || a == TS_UB || a == TS_UTB || a == TS_LTB;
        if (!mirror && (a == TS_UTB || a == TS_LTB)) continue;
        const size_t per_row = band ? (size_t)nb : 1;
        const size_t bytes = rows * per_row * TILE_ELEMS * esz;
        if ((e = hipMalloc(&t.alloc[a], bytes)) != hipSuccess) return e;
        if ((e = hipMemset(t.alloc[a], 0, bytes)) != hipSuccess) return e;
        t.a[a] = (char *)t.alloc[a] + G * per_row * TILE_ELEMS * esz;
    }
    if ((e = hipMalloc(&t.zt, TILE_ELEMS * esz)) != hipSuccess) return e;
    if ((e = hipMemset(t.zt, 0, TILE_ELEMS * esz)) != hipSuccess) return e;
    if ((e = hipMalloc(&t.sink, TILE_ELEMS * esz)) != hipSuccess) return e;
    return hipSuccess;
}

void lrpr_factor_destroy(lrpr_fac f) {
    if (!f) return;
    hipSetDevice(f->dev);
    hipDeviceSynchronize();
    if (f->lu) hipFree(f->lu);
    free_tiles(f->t64);
    free_tiles(f->t32);
    delete f;
}

lrpr_status lrpr_factor(lrpr_ctx ctx, const lrpr_op_desc *op, int store_mask, lrpr_fac *out) {
    if (!ctx || !op || !out) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor: null argument");
    if ((op->dim != 1 && op->dim != 2) || op->nx < 1 || !(op->nu > 0) || !(op->dt > 0) ||
        !(op->c >= 0) || !std::isfinite(op->beta1) || !std::isfinite(op->beta2))
        return fail(ctx, LRPR_ERR_ARG, "lrpr_factor: invalid operator descriptor");
    if (store_mask == 0) store_mask = LRPR_STORE_F64;
    if ((store_mask & ~(LRPR_STORE_F64 | LRPR_STORE_F32 | LRPR_STORE_MIRROR)) ||
        !(store_mask & (LRPR_STORE_F64 | LRPR_STORE_F32)))
        return fail(ctx, LRPR_ERR_ARG, "lrpr_factor: store_mask must hold F64 and/or F32 (and optionally MIRROR)");
    const bool mirror = (store_mask & LRPR_STORE_MIRROR) != 0;
    const int64_t n = op->dim == 1 ? op->nx : (int64_t)op->nx * op->nx;
    const int bw = op->dim == 1 ? 1 : op->nx;
    if (n >= (int64_t)1 << 31) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor: n too large");
    if (bw > 1023) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor: half-bandwidth above 1023");
    HIPCHK(hipSetDevice(ctx->dev), "hipSetDevice");
    lrpr_fac f = new (std::nothrow) lrpr_factor_s();
    if (!f) return fail(ctx, LRPR_ERR_NOMEM, "lrpr_factor: host allocation");
    f->dev = ctx->dev;
    f->op = *op;
    f->n = n;
    f->bw = bw;
    f->NT = (int)((n + TILE - 1) / TILE);
    f->nb = (bw + TILE - 1) / TILE;
    f->mask = store_mask;
    double *band = nullptr;
    void *scratch = nullptr;
    hipError_t e;
    auto cleanup = [&](lrpr_status st, const std::string &msg) {
        if (band && band != f->lu) hipFree(band);
        if (scratch) hipFree(scratch);
        lrpr_factor_destroy(f);
        return fail(ctx, st, msg);
    };
    // scratch: tile-LU panels and flags, later the diagonal-tile inverses
    size_t sbytes = tile_lu_scratch_bytes(f->NT, f->nb);
    const size_t inv_bytes = sizeof(double) * 2 * (size_t)f->NT * TILE_ELEMS;
    if (inv_bytes > sbytes) sbytes = inv_bytes;
    if ((e = hipMalloc(&band, sizeof(double) * (size_t)n * (2 * bw + 1))) != hipSuccess)
        return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: band allocation");
    if ((e = hipMalloc(&scratch, sbytes)) != hipSuccess)
        return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: scratch allocation");
    if ((e = launch_assemble(*op, n, bw, band, ctx->stream)) != hipSuccess)
        return cleanup(LRPR_ERR_HIP, std::string("assemble: ") + hipGetErrorString(e));
    int *d_info = nullptr, *d_err = nullptr;
    if ((e = launch_tile_lu(n, bw, f->NT, f->nb, band, scratch, &d_info, &d_err, ctx->stream)) != hipSuccess)
        return cleanup(LRPR_ERR_HIP, std::string("band LU: ") + hipGetErrorString(e));
    int flags[2] = {0, 0};
    if ((e = hipMemcpyAsync(&flags[0], d_info, sizeof(int), hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(&flags[1], d_err, sizeof(int), hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(ctx->stream)) != hipSuccess)
        return cleanup(LRPR_ERR_HIP, std::string("band LU: ") + hipGetErrorString(e));
    if (flags[1] != 0) return cleanup(LRPR_ERR_HIP, "band LU: a panel wait timed out");
    if (flags[0] != 0x7f7f7f7f) {
        char msg[128];
        snprintf(msg, sizeof msg, "lrpr_factor: zero or non-finite pivot at row %d", flags[0] - 1);
        return cleanup(LRPR_ERR_ZERO_PIVOT, msg);
    }
    if (store_mask & LRPR_STORE_F64) {
        if (alloc_tiles(f->t64, f->NT, f->nb, sizeof(double), mirror) != hipSuccess)
            return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: FP64 tile allocation");
    }
    if (store_mask & LRPR_STORE_F32) {
        if (alloc_tiles(f->t32, f->NT, f->nb, sizeof(float), mirror) != hipSuccess)
            return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: FP32 tile allocation");
    }
    if ((e = launch_pack_tiles(n, bw, f->NT, f->nb, band, (store_mask & LRPR_STORE_F64) ? &f->t64 : nullptr,
                               (store_mask & LRPR_STORE_F32) ? &f->t32 : nullptr, (double *)scratch,
                               ctx->stream)) != hipSuccess)
        return cleanup(LRPR_ERR_HIP, std::string("pack: ") + hipGetErrorString(e));
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess)
        return cleanup(LRPR_ERR_HIP, std::string("factor: ") + hipGetErrorString(e));
    hipFree(scratch);
    scratch = nullptr;
    if (store_mask & LRPR_STORE_F64) {
        f->lu = band;
    } else {
        hipFree(band);
    }
    band = nullptr;
    *out = f;
    return LRPR_OK;
}

lrpr_status lrpr_factor_info(lrpr_fac f, int64_t *n, int *bw, double *dt) {
    if (!f) return LRPR_ERR_ARG;
    if (n) *n = f->n;
    if (bw) *bw = f->bw;
    if (dt) *dt = f->op.dt;
    return LRPR_OK;
}

lrpr_status lrpr_factor_copy_lu(lrpr_ctx ctx, lrpr_fac f, double *lu_host) {
    if (!ctx || !f || !lu_host) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor_copy_lu: null argument");
    if (!f->lu) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor_copy_lu: factor kept without FP64 band LU");
    HIPCHK(hipSetDevice(ctx->dev), "hipSetDevice");
    HIPCHK(hipMemcpyAsync(lu_host, f->lu, sizeof(double) * (size_t)f->n * (2 * f->bw + 1),
                          hipMemcpyDeviceToHost, ctx->stream),
           "copy LU");
    HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
    return LRPR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched sweeps
// ---------------------------------------------------------------------------
namespace lrpr {

FacView fac_view(lrpr_fac f, bool f32) {
    const TileSet &t = f32 ? f->t32 : f->t64;
    FacView v;
    for (int a = 0; a < TS_COUNT; ++a) v.a[a] = t.a[a];
    v.zt = t.zt;
    v.sink = t.sink;
    v.n = (int)f->n;
    v.NT = f->NT;
    v.nb = f->nb;
    v.dt = f->op.dt;
    return v;
}

lrpr_status ensure_items(lrpr_ctx ctx, size_t count) {
    if (count <= ctx->items_cap) return LRPR_OK;
    if (ctx->d_items) {
        hipStreamSynchronize(ctx->stream);
        hipFree(ctx->d_items);
        ctx->d_items = nullptr;
        ctx->items_cap = 0;
    }
    size_t cap = 1024;
    while (cap < count) cap *= 2;
    hipError_t e = hipMalloc(&ctx->d_items, cap * sizeof(SweepItem));
    if (e != hipSuccess) return hipfail(ctx, e, "sweep item buffer");
    ctx->items_cap = cap;
    return LRPR_OK;
}

// Validate panels and turn them into 16-column work items; launch one sweep.
lrpr_status run_sweep(lrpr_ctx ctx, int npanels, const lrpr_panel *panels, int nsteps, lrpr_prec prec,
                      bool adjoint) {
    if (!ctx) return LRPR_ERR_ARG;
    if (npanels < 0 || (npanels > 0 && !panels) || nsteps < 0 || (prec != LRPR_F64 && prec != LRPR_F32))
        return fail(ctx, LRPR_ERR_ARG, "sweep: invalid arguments");
    const bool f32 = prec == LRPR_F32;
    std::vector<SweepItem> items;
    int max_nb = 1;
    bool strided = false;   // adjoint: some factor has no mirrored set
    for (int p = 0; p < npanels; ++p) {
        const lrpr_panel &P = panels[p];
        if (!P.F || (P.w > 0 && !P.X) || P.w < 0 || P.ldx < P.F->n)
            return fail(ctx, LRPR_ERR_ARG, "sweep: panel with null factor/X or ldx < n");
        if (P.F->dev != ctx->dev) return fail(ctx, LRPR_ERR_ARG, "sweep: factor on another device");
        if ((f32 && !(P.F->mask & LRPR_STORE_F32)) || (!f32 && !(P.F->mask & LRPR_STORE_F64)))
            return fail(ctx, LRPR_ERR_ARG, "sweep: factor has no copy in the requested precision");
        if (!adjoint && P.f && P.ldf < P.F->n) return fail(ctx, LRPR_ERR_ARG, "sweep: ldf < n");
        if (P.F->nb > max_nb) max_nb = P.F->nb;
        if (P.w > 0 && !(P.F->mask & LRPR_STORE_MIRROR)) strided = true;
        const size_t esz = f32 ? sizeof(float) : sizeof(double);
        for (int c0 = 0; c0 < P.w; c0 += TILE) {
            SweepItem it;
            it.fac = fac_view(P.F, f32);
            it.X = (char *)P.X + (size_t)c0 * P.ldx * esz;
            it.ldx = P.ldx;
            it.ncols = P.w - c0 < TILE ? P.w - c0 : TILE;
            it.pad_ = 0;
            it.f = adjoint ? nullptr : P.f;
            it.ldf = P.ldf;
            it.fcol = (!adjoint && P.f && P.fcol) ? P.fcol + c0 : nullptr;
            it.fscale = (!adjoint && P.f && P.fscale) ? P.fscale + (size_t)c0 * nsteps : nullptr;
            items.push_back(it);
        }
    }
    if (items.empty() || nsteps == 0) return LRPR_OK;
    if (max_nb > 64) return fail(ctx, LRPR_ERR_ARG, "sweep: half-bandwidth above 1023");
    hipError_t e = hipSetDevice(ctx->dev);
    if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
    lrpr_status st = ensure_items(ctx, items.size());
    if (st != LRPR_OK) return st;
    e = hipMemcpyAsync(ctx->d_items, items.data(), items.size() * sizeof(SweepItem),
                       hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return hipfail(ctx, e, "sweep item upload");
    lrpr_ctx_s::ProfRec rec{};
    if (ctx->prof) {
        // algorithmic work: 4 n b flops and 2 n s bytes per RHS step, plus one
        // read of each distinct factor per step
        const double s = f32 ? 4.0 : 8.0;
        std::vector<lrpr_fac> seen;
        for (int p = 0; p < npanels; ++p) {
            const lrpr_panel &P = panels[p];
            const double n = (double)P.F->n, b = (double)P.F->bw;
            rec.flops += 4.0 * n * b * P.w * nsteps;
            rec.bytes += 2.0 * n * s * P.w * nsteps;
            rec.rhs_steps += (double)P.w * nsteps;
            bool dup = false;
            for (lrpr_fac q : seen) dup = dup || q == P.F;
            if (!dup) {
                seen.push_back(P.F);
                rec.bytes += n * (2.0 * b + 1.0) * s * nsteps;
            }
        }
        if ((e = hipEventCreate(&rec.a)) != hipSuccess || (e = hipEventCreate(&rec.b)) != hipSuccess ||
            (e = hipEventRecord(rec.a, ctx->stream)) != hipSuccess)
            return hipfail(ctx, e, "profile event");
    }
    e = launch_sweep(adjoint, strided, f32, (int)items.size(), ctx->d_items, nsteps, max_nb, ctx->stream);
    if (e != hipSuccess) return hipfail(ctx, e, "sweep launch");
    if (ctx->prof) {
        if ((e = hipEventRecord(rec.b, ctx->stream)) != hipSuccess) return hipfail(ctx, e, "profile event");
        ctx->prof_recs.push_back(rec);
    }
    return LRPR_OK;
}

}  // namespace lrpr

extern "C" {

lrpr_status lrpr_fine_step_batched(lrpr_ctx ctx, int npanels, const lrpr_panel *panels, int nsteps,
                                   lrpr_prec prec) {
    return run_sweep(ctx, npanels, panels, nsteps, prec, false);
}

lrpr_status lrpr_profile_enable(lrpr_ctx ctx, int enable) {
    if (!ctx) return LRPR_ERR_ARG;
    ctx->prof = enable != 0;
    return LRPR_OK;
}

lrpr_status lrpr_profile_read(lrpr_ctx ctx, double *ms, int64_t *launches, double *flops, double *bytes,
                              double *rhs_steps) {
    if (!ctx) return LRPR_ERR_ARG;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hipfail(ctx, e, "profile sync");
    double tms = 0, fl = 0, by = 0, rs = 0;
    for (auto &r : ctx->prof_recs) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) tms += t;
        fl += r.flops;
        by += r.bytes;
        rs += r.rhs_steps;
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    if (ms) *ms = tms;
    if (launches) *launches = (int64_t)ctx->prof_recs.size();
    if (flops) *flops = fl;
    if (bytes) *bytes = by;
    if (rhs_steps) *rhs_steps = rs;
    ctx->prof_recs.clear();
    return LRPR_OK;
}

lrpr_status lrpr_adjoint_step_batched(lrpr_ctx ctx, int npanels, const lrpr_panel *panels, int nsteps,
                                      lrpr_prec prec) {
    return run_sweep(ctx, npanels, panels, nsteps, prec, true);
}

}  // extern "C"
