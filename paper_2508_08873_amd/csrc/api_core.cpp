// Host side of the C ABI: contexts, factors, batched fine/adjoint sweeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <type_traits>

#include "dense.h"
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

namespace lrpr {

// Blocks of handle memory freed by destroy calls, kept per device and size
// for the next allocation of the same size (handles of one shape are
// destroyed and made again step after step), until lrpr_device_trim.
namespace {
std::mutex g_mem_mu;
std::multimap<std::pair<int, size_t>, void *> g_free;   // (device, bytes) -> block
std::map<void *, std::pair<int, size_t>> g_live;        // block -> (device, bytes)
}  // namespace

hipError_t dmalloc(void **p, size_t bytes, hipStream_t) {
    if (!bytes) bytes = 16;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> lock(g_mem_mu);
        auto it = g_free.find({dev, bytes});
        if (it != g_free.end()) {
            *p = it->second;
            g_free.erase(it);
            g_live[*p] = {dev, bytes};
            return hipSuccess;
        }
    }
    e = hipMalloc(p, bytes);
    if (e == hipErrorOutOfMemory) {   // give the kept blocks back and try once more
        lrpr_device_trim(dev);
        hipSetDevice(dev);
        e = hipMalloc(p, bytes);
    }
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_mem_mu);
    g_live[*p] = {dev, bytes};
    return hipSuccess;
}

// p must not be in use by queued work (callers synchronise first)
void dfree(void *p, hipStream_t) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_mem_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) {
        hipFree(p);
        return;
    }
    g_free.insert({it->second, p});
    g_live.erase(it);
}

}  // namespace lrpr

extern "C" {

lrpr_status lrpr_ctx_create(int device, void *hip_stream, lrpr_ctx *out) {
    if (!out) return LRPR_ERR_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LRPR_ERR_ARG;
    lrpr_ctx ctx = new (std::nothrow) lrpr_ctx_s();
    if (!ctx) return LRPR_ERR_NOMEM;
    ctx->dev = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess || lrpr::noalloc_scratch_init(device, nullptr) != hipSuccess ||
        hipDeviceGetAttribute(&ctx->ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
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
    lrpr_device_trim(ctx->dev);
    delete ctx;
}

lrpr_status lrpr_device_trim(int device) {
    if (hipSetDevice(device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return LRPR_ERR_HIP;
    std::vector<void *> blocks;
    {
        std::lock_guard<std::mutex> lock(lrpr::g_mem_mu);
        for (auto it = lrpr::g_free.begin(); it != lrpr::g_free.end();) {
            if (it->first.first == device) {
                blocks.push_back(it->second);
                it = lrpr::g_free.erase(it);
            } else {
                ++it;
            }
        }
    }
    for (void *p : blocks) hipFree(p);
    return LRPR_OK;
}

lrpr_status lrpr_ctx_set_stream(lrpr_ctx ctx, void *hip_stream) {
    if (!ctx) return LRPR_ERR_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return LRPR_OK;
}

const char *lrpr_last_error(lrpr_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

// ---------------------------------------------------------------------------
static void free_tiles(TileSet &t) {
    dfree(t.block, nullptr);
    t = TileSet();
}

// Tile arrays with guard_rows(nb) zero tile rows on both sides; the TileSet
// pointers address tile row 0.  The mirrored band arrays only with `mirror`.
// One allocation (and one clearing fill) holds every array of the set, the
// zero tile and the sink tile.
static hipError_t alloc_tiles(TileSet &t, int NT, int nb, size_t esz, bool mirror, hipStream_t s) {
    const size_t G = (size_t)guard_rows(nb);
    const size_t rows = (size_t)NT + 2 * G;
    const size_t tile = TILE_ELEMS * esz;
    size_t off[TS_COUNT] = {}, total = 0;
    for (int a = 0; a < TS_COUNT; ++a) {
        const bool band = a == TS_LB || a == TS_UB || a == TS_UTB || a == TS_LTB;
        if (!mirror && (a == TS_UTB || a == TS_LTB)) continue;
        off[a] = total;
        total += rows * (band ? (size_t)nb : 1) * tile;
    }
    const size_t zoff = total, soff = total + tile;
    total += 2 * tile;
    hipError_t e;
    if ((e = dmalloc(&t.block, total, s)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(t.block, 0, total, s)) != hipSuccess) return e;
    char *b = (char *)t.block;
    for (int a = 0; a < TS_COUNT; ++a) {
        const bool band = a == TS_LB || a == TS_UB || a == TS_UTB || a == TS_LTB;
        if (!mirror && (a == TS_UTB || a == TS_LTB)) continue;
        t.alloc[a] = b + off[a];
        t.a[a] = b + off[a] + G * (band ? (size_t)nb : 1) * tile;
    }
    t.zt = b + zoff;
    t.sink = b + soff;
    return hipSuccess;
}

void lrpr_factor_destroy(lrpr_fac f) {
    if (!f) return;
    for (lrpr_fac g : f->seq) lrpr_factor_destroy(g);
    f->seq.clear();
    hipSetDevice(f->dev);
    hipDeviceSynchronize();
    dfree(f->lu, nullptr);
    free_tiles(f->t64);
    free_tiles(f->t32);
    free_tiles(f->t64r);
    free_tiles(f->t32r);
    for (void *p : {f->s64.S, f->s64.T, f->s32.S, f->s32.T}) dfree(p, nullptr);
    if (f->d_blk) hipFree(f->d_blk);
    delete f;
}

}  // extern "C"

namespace lrpr {
FacView fac_view(lrpr_fac f, bool f32);
lrpr_status ensure_items(lrpr_ctx ctx, size_t count);
// workspace cached per context and purpose; grows on demand
void *ws_get(lrpr_ctx ctx, const char *key, size_t bytes, hipError_t *err);

// Block starts of the partitioned solve: P ~ 24 blocks (balances the local
// solves, NT/P tile rows, against the sequential chain, P steps of nb^2 tile
// products), each at least 2 nb tile rows.
static std::vector<int> split_blocks(int NT, int nb) {
    int P = 24 < SPLIT_MAX_P ? 24 : SPLIT_MAX_P;
    if (P > NT / (2 * nb)) P = NT / (2 * nb);
    std::vector<int> blk;
    if (P < 2) return blk;
    for (int p = 0; p <= P; ++p) blk.push_back((int)((int64_t)NT * p / P));
    return blk;
}

// Spikes S_p = L_pp^{-1} L_{p,p-1}[:, tail], T_p = U_pp^{-1} U_{p,p+1}[:, head]
// of every stored precision: local sweeps of the coupling columns, packed
// into tiles.
static lrpr_status build_split(lrpr_ctx ctx, lrpr_fac f, const double *band) {
    f->blk = split_blocks(f->NT, f->nb);
    if (f->blk.empty()) return LRPR_OK;   // too few rows to partition
    const int P = (int)f->blk.size() - 1, NT = f->NT, nb = f->nb;
    hipStream_t st = ctx->stream;
    hipError_t e;
    const int64_t ld = (int64_t)NT * TILE;
    const size_t dense = (size_t)ld * nb * TILE;
    // the dense spike staging arrays come from the context's workspaces
    double *RL = nullptr, *RU = nullptr;
    float *RL32 = nullptr, *RU32 = nullptr;
    auto bail = [&](hipError_t err, const char *what) {
        return fail(ctx, err == hipErrorOutOfMemory ? LRPR_ERR_NOMEM : LRPR_ERR_HIP,
                    std::string(what) + ": " + hipGetErrorString(err));
    };
    auto wsa = [&](auto **p, const char *key, size_t bytes) -> hipError_t {
        hipError_t er = hipSuccess;
        *p = (std::remove_pointer_t<decltype(p)>)ws_get(ctx, key, bytes, &er);
        return *p ? hipSuccess : (er == hipSuccess ? hipErrorOutOfMemory : er);
    };
    if ((e = hipMalloc(&f->d_blk, sizeof(int) * (P + 1))) != hipSuccess) return bail(e, "block table");
    if ((e = hipMemcpyAsync(f->d_blk, f->blk.data(), sizeof(int) * (P + 1), hipMemcpyHostToDevice, st)) != hipSuccess)
        return bail(e, "block table");
    if ((e = wsa(&RL, "spike_rl", sizeof(double) * dense)) != hipSuccess ||
        (e = wsa(&RU, "spike_ru", sizeof(double) * dense)) != hipSuccess)
        return bail(e, "spike scratch");
    if ((e = launch_spike_rhs(f->n, f->bw, NT, nb, P, f->d_blk, band, RL, RU, st)) != hipSuccess)
        return bail(e, "spike right-hand sides");
    // solve once, in FP64 when the factor keeps FP64 tiles (else FP32), then
    // pack into every stored precision
    const bool solve32 = !(f->mask & LRPR_STORE_F64);
    void *L = RL, *U = RU;
    if (solve32 || (f->mask & LRPR_STORE_F32)) {
        if ((e = wsa(&RL32, "spike_rl32", sizeof(float) * dense)) != hipSuccess ||
            (e = wsa(&RU32, "spike_ru32", sizeof(float) * dense)) != hipSuccess)
            return bail(e, "spike scratch");
    }
    if (solve32) {
        if ((e = launch_convert(0, 1, RL, RL32, (int64_t)dense, st)) != hipSuccess ||
            (e = launch_convert(0, 1, RU, RU32, (int64_t)dense, st)) != hipSuccess)
            return bail(e, "spike convert");
        L = RL32;
        U = RU32;
    }
    {
        // local sweeps: L pass on the coupling columns of blocks 1..P-1, U pass
        // on those of blocks 0..P-2 (nb column groups each)
        const size_t esz = solve32 ? 4 : 8;
        std::vector<SweepItem> items;
        for (int pass = 0; pass < 2; ++pass)
            for (int p = (pass == 0 ? 1 : 0); p < (pass == 0 ? P : P - 1); ++p)
                for (int cg = 0; cg < nb; ++cg) {
                    SweepItem it{};
                    it.fac = fac_view(f, solve32);
                    it.X = (char *)(pass == 0 ? L : U) + (size_t)cg * TILE * ld * esz;
                    it.ldx = ld;
                    it.ncols = TILE;
                    it.passes = pass == 0 ? 1 : 2;
                    it.r0 = f->blk[p];
                    it.r1 = f->blk[p + 1];
                    it.fsteps = 1;
                    items.push_back(it);
                }
        lrpr_status ls = ensure_items(ctx, items.size());
        if (ls != LRPR_OK) return ls;
        if ((e = hipMemcpyAsync(ctx->d_items, items.data(), items.size() * sizeof(SweepItem), hipMemcpyHostToDevice,
                                st)) != hipSuccess)
            return bail(e, "spike items");
        if ((e = launch_sweep(false, false, solve32, (int)items.size(), ctx->d_items, 1, nb, st, 0, true)) != hipSuccess)
            return bail(e, "spike solves");
    }
    if (!solve32 && (f->mask & LRPR_STORE_F32)) {
        if ((e = launch_convert(0, 1, RL, RL32, (int64_t)dense, st)) != hipSuccess ||
            (e = launch_convert(0, 1, RU, RU32, (int64_t)dense, st)) != hipSuccess)
            return bail(e, "spike convert");
    }
    for (int prec = 0; prec < 2; ++prec) {
        const bool f32 = prec == 1;
        if (!(f->mask & (f32 ? LRPR_STORE_F32 : LRPR_STORE_F64))) continue;
        SplitSet &ss = f32 ? f->s32 : f->s64;
        const size_t tiles = (size_t)NT * nb * TILE_ELEMS * (f32 ? 4 : 8);
        if ((e = dmalloc(&ss.S, tiles, ctx->stream)) != hipSuccess || (e = dmalloc(&ss.T, tiles, ctx->stream)) != hipSuccess)
            return bail(e, "spike tiles");
        if ((e = launch_spike_pack(f32, NT, nb, f32 ? (void *)RL32 : (void *)RL, ld, ss.S, st)) != hipSuccess ||
            (e = launch_spike_pack(f32, NT, nb, f32 ? (void *)RU32 : (void *)RU, ld, ss.T, st)) != hipSuccess)
            return bail(e, "spike pack");
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e, "spike build");
    f->P = P;
    return LRPR_OK;
}
}  // namespace lrpr

namespace lrpr {
void *ws_get(lrpr_ctx ctx, const char *key, size_t bytes, hipError_t *err);
}

// Factor m operators of one grid together: assembly, then the band LUs in
// batched launches (the matrices' workgroups run side by side), one check of
// the pivots, tile packing and, with LRPR_STORE_SPLIT, the spikes.
static lrpr_status factor_batch(lrpr_ctx ctx, const lrpr_op_desc *ops, int m, int store_mask, lrpr_fac *outs) {
    for (int j = 0; j < m; ++j) {
        const lrpr_op_desc *op = &ops[j];
        if ((op->dim != 1 && op->dim != 2) || op->nx < 1 || !(op->nu > 0) || !(op->dt > 0) || !(op->c >= 0) ||
            !std::isfinite(op->beta1) || !std::isfinite(op->beta2) || op->dim != ops[0].dim || op->nx != ops[0].nx ||
            (op->bc != LRPR_BC_DIRICHLET && op->bc != LRPR_BC_NEUMANN) || (op->bc == LRPR_BC_NEUMANN && op->nx < 2))
            return fail(ctx, LRPR_ERR_ARG, "lrpr_factor: invalid operator descriptor");
    }
    if (store_mask == 0) store_mask = LRPR_STORE_F64;
    if ((store_mask & ~(LRPR_STORE_F64 | LRPR_STORE_F32 | LRPR_STORE_MIRROR | LRPR_STORE_SPLIT | LRPR_STORE_UL)) ||
        !(store_mask & (LRPR_STORE_F64 | LRPR_STORE_F32)))
        return fail(ctx, LRPR_ERR_ARG, "lrpr_factor: store_mask must hold F64 and/or F32 (and optionally MIRROR)");
    const bool mirror = (store_mask & LRPR_STORE_MIRROR) != 0;
    const bool ul = (store_mask & LRPR_STORE_UL) != 0;
    const int64_t n = ops[0].dim == 1 ? ops[0].nx : (int64_t)ops[0].nx * ops[0].nx;
    const int bw = ops[0].dim == 1 ? 1 : ops[0].nx;
    if (n >= (int64_t)1 << 31) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor: n too large");
    if (bw > 1023) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor: half-bandwidth above 1023");
    HIPCHK(hipSetDevice(ctx->dev), "hipSetDevice");
    const int NT = (int)((n + TILE - 1) / TILE), nb = (bw + TILE - 1) / TILE;
    hipStream_t st = ctx->stream;
    // matrices j < m: M_j (n rows); with LRPR_STORE_UL also j >= m: the
    // reversed J diag(M_j, I) J (NT * 16 rows), whose LU is M_j's UL
    const int mm = ul ? 2 * m : m;
    const int64_t nrev = (int64_t)NT * TILE;
    std::vector<lrpr_fac> fs(m, nullptr);
    std::vector<double *> bands(mm, nullptr);
    std::vector<void *> scr(mm, nullptr);
    std::vector<int64_t> rows(mm, n);
    for (int j = m; j < mm; ++j) rows[j] = nrev;
    // Band arrays and scratch come from the context's cached workspaces,
    // except the FP64 LU that a factor keeps (LRPR_STORE_F64): after the
    // first factorisation of a shape, factoring frees no device memory.
    const bool keep_lu = (store_mask & LRPR_STORE_F64) != 0;
    std::vector<char> owned(mm, 0);   // bands[j] allocated here (kept by the factor)
    auto cleanup = [&](lrpr_status stt, const std::string &msg) {
        hipStreamSynchronize(st);
        for (int j = 0; j < mm; ++j) {
            if (bands[j] && owned[j] && (!fs[j] || bands[j] != fs[j]->lu)) dfree(bands[j], st);
            if (j < m && fs[j]) lrpr_factor_destroy(fs[j]);
        }
        return fail(ctx, stt, msg);
    };
    hipError_t e;
    // scratch: tile-LU panels and flags, later the diagonal-tile inverses
    size_t sbytes = tile_lu_scratch_bytes(NT, nb);
    const size_t inv_bytes = sizeof(double) * 2 * (size_t)NT * TILE_ELEMS;
    if (inv_bytes > sbytes) sbytes = inv_bytes;
    for (int j = 0; j < m; ++j) {
        lrpr_fac f = new (std::nothrow) lrpr_factor_s();
        if (!f) return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: host allocation");
        fs[j] = f;
        f->dev = ctx->dev;
        f->op = ops[j];
        f->n = n;
        f->bw = bw;
        f->NT = NT;
        f->nb = nb;
        f->mask = store_mask;
        f->dt_step = ops[j].dt;
    }
    // temporaries (bands not kept, LU scratch) carved from the context's
    // arena, the workspace that the rSVD build's panels reuse afterwards
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t arena_bytes = 0;
    for (int j = 0; j < mm; ++j) {
        if (!(j < m && keep_lu)) arena_bytes += al(sizeof(double) * (size_t)rows[j] * (2 * bw + 1));
        arena_bytes += al(sbytes);
    }
    char *arena = (char *)ws_get(ctx, "arena", arena_bytes, &e);
    if (!arena) return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: band and scratch workspace");
    size_t at = 0;
    for (int j = 0; j < mm; ++j) {
        const size_t bbytes = sizeof(double) * (size_t)rows[j] * (2 * bw + 1);
        if (j < m && keep_lu) {
            if ((e = dmalloc((void **)&bands[j], bbytes, st)) != hipSuccess)
                return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: band allocation");
            owned[j] = 1;
        } else {
            bands[j] = (double *)(arena + at);
            at += al(bbytes);
        }
        scr[j] = arena + at;
        at += al(sbytes);
        if ((e = launch_assemble(ops[j % m], n, rows[j], bw, j >= m, bands[j], st)) != hipSuccess)
            return cleanup(LRPR_ERR_HIP, std::string("assemble: ") + hipGetErrorString(e));
    }
    void *d_args = ws_get(ctx, "lu_args", tile_lu_args_bytes(mm), &e);
    if (!d_args) return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: LU argument buffer");
    std::vector<int *> d_info(mm), d_err(mm);
    if ((e = launch_tile_lu_batch(mm, rows.data(), bw, NT, nb, bands.data(), scr.data(), d_info.data(),
                                  d_err.data(), d_args, st, ctx->tune_lu_wgs)) != hipSuccess)
        return cleanup(LRPR_ERR_HIP, std::string("band LU: ") + hipGetErrorString(e));
    std::vector<int> flags(2 * (size_t)mm, 0);
    for (int j = 0; j < mm; ++j)
        if ((e = hipMemcpyAsync(&flags[2 * j], d_info[j], sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipMemcpyAsync(&flags[2 * j + 1], d_err[j], sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
            return cleanup(LRPR_ERR_HIP, std::string("band LU: ") + hipGetErrorString(e));
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return cleanup(LRPR_ERR_HIP, std::string("band LU: ") + hipGetErrorString(e));
    for (int j = 0; j < mm; ++j) {
        if (flags[2 * j + 1] != 0) return cleanup(LRPR_ERR_HIP, "band LU: a panel wait timed out");
        if (flags[2 * j] != 0x7f7f7f7f) {
            char msg[128];
            if (j < m)
                snprintf(msg, sizeof msg, "lrpr_factor: zero or non-finite pivot at row %d", flags[2 * j] - 1);
            else   // row r of the reversed matrix is row nrev - 1 - r of the operator
                snprintf(msg, sizeof msg, "lrpr_factor: zero or non-finite pivot of the UL factorisation at row %lld",
                         (long long)(nrev - flags[2 * j]));
            return cleanup(LRPR_ERR_ZERO_PIVOT, msg);
        }
    }
    for (int j = 0; j < m; ++j) {
        lrpr_fac f = fs[j];
        if ((store_mask & LRPR_STORE_F64) && alloc_tiles(f->t64, NT, nb, sizeof(double), mirror, st) != hipSuccess)
            return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: FP64 tile allocation");
        if ((store_mask & LRPR_STORE_F32) && alloc_tiles(f->t32, NT, nb, sizeof(float), mirror, st) != hipSuccess)
            return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: FP32 tile allocation");
        if ((e = launch_pack_tiles(n, bw, NT, nb, bands[j], false, (store_mask & LRPR_STORE_F64) ? &f->t64 : nullptr,
                                   (store_mask & LRPR_STORE_F32) ? &f->t32 : nullptr, (double *)scr[j], st)) !=
            hipSuccess)
            return cleanup(LRPR_ERR_HIP, std::string("pack: ") + hipGetErrorString(e));
        if (!ul) continue;
        if ((store_mask & LRPR_STORE_F64) && alloc_tiles(f->t64r, NT, nb, sizeof(double), mirror, st) != hipSuccess)
            return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: FP64 UL tile allocation");
        if ((store_mask & LRPR_STORE_F32) && alloc_tiles(f->t32r, NT, nb, sizeof(float), mirror, st) != hipSuccess)
            return cleanup(LRPR_ERR_NOMEM, "lrpr_factor: FP32 UL tile allocation");
        if ((e = launch_pack_tiles(n, bw, NT, nb, bands[m + j], true,
                                   (store_mask & LRPR_STORE_F64) ? &f->t64r : nullptr,
                                   (store_mask & LRPR_STORE_F32) ? &f->t32r : nullptr, (double *)scr[m + j], st)) !=
            hipSuccess)
            return cleanup(LRPR_ERR_HIP, std::string("pack: ") + hipGetErrorString(e));
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess)
        return cleanup(LRPR_ERR_HIP, std::string("factor: ") + hipGetErrorString(e));
    for (int j = m; j < mm; ++j) bands[j] = nullptr;   // workspace
    for (int j = 0; j < m; ++j) {
        if (store_mask & LRPR_STORE_SPLIT) {
            const lrpr_status stt = build_split(ctx, fs[j], bands[j]);
            if (stt != LRPR_OK) return cleanup(stt, std::string("lrpr_factor: partitioned solve: ") + ctx->err);
        }
        if (keep_lu) fs[j]->lu = bands[j];
        bands[j] = nullptr;
    }
    for (int j = 0; j < m; ++j) outs[j] = fs[j];
    return LRPR_OK;
}

extern "C" {

lrpr_status lrpr_mass_weights(const lrpr_op_desc *op, double *w_host) {
    if (!op || !w_host || (op->dim != 1 && op->dim != 2) || op->nx < 1 ||
        (op->bc != LRPR_BC_DIRICHLET && op->bc != LRPR_BC_NEUMANN) || (op->bc == LRPR_BC_NEUMANN && op->nx < 2))
        return LRPR_ERR_ARG;
    const int nx = op->nx;
    const bool neu = op->bc == LRPR_BC_NEUMANN;
    const double h = neu ? 1.0 / (nx - 1) : 1.0 / (nx + 1);
    std::vector<double> w1(nx, h);
    if (neu) w1[0] = w1[nx - 1] = 0.5 * h;
    if (op->dim == 1) {
        for (int i = 0; i < nx; ++i) w_host[i] = w1[i];
    } else {
        for (int j = 0; j < nx; ++j)
            for (int i = 0; i < nx; ++i) w_host[i + (size_t)nx * j] = w1[i] * w1[j];
    }
    return LRPR_OK;
}

lrpr_status lrpr_factor(lrpr_ctx ctx, const lrpr_op_desc *op, int store_mask, lrpr_fac *out) {
    if (!ctx || !op || !out) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor: null argument");
    return factor_batch(ctx, op, 1, store_mask, out);
}

}  // extern "C"

// Matrices lrpr_factor_many factors together: as many as the workspace
// budget holds (FP64 band and LU scratch per matrix; 110 GB by default,
// which takes 32 matrices of 511^2 at once: one launch of 8 workgroups
// each), at most 64, in equal chunks; each chunk's band LUs run in as few
// launches as its size allows.
static int many_chunk(lrpr_ctx ctx, const lrpr_op_desc &op, int count, int store_mask) {
    const int64_t n = op.dim == 1 ? op.nx : (int64_t)op.nx * op.nx;
    const int bw = op.dim == 1 ? 1 : op.nx;
    const int NT = (int)((n + TILE - 1) / TILE), nb = (bw + TILE - 1) / TILE;
    const double per_matrix = 8.0 * (double)n * (2 * bw + 1) + (double)tile_lu_scratch_bytes(NT, nb);
    const double budget = ctx->tune_lu_budget ? (double)ctx->tune_lu_budget : 110e9;
    int chunk = (int)std::max(1.0, std::min(64.0, budget / std::max(per_matrix, 1.0)));
    if (store_mask & LRPR_STORE_UL) chunk = std::max(1, chunk / 2);
    const int nchunk = (count + chunk - 1) / chunk;
    return (count + nchunk - 1) / nchunk;
}

extern "C" {

lrpr_status lrpr_factor_many(lrpr_ctx ctx, const lrpr_op_desc *ops, int count, int store_mask, lrpr_fac *outs) {
    if (!ctx || !ops || !outs || count < 1) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor_many: invalid arguments");
    for (int j = 1; j < count; ++j)
        if (ops[j].dim != ops[0].dim || ops[j].nx != ops[0].nx)
            return fail(ctx, LRPR_ERR_ARG, "lrpr_factor_many: the operators must share dim and nx");
    for (int j = 0; j < count; ++j) outs[j] = nullptr;
    const int chunk = many_chunk(ctx, ops[0], count, store_mask);
    for (int j0 = 0; j0 < count; j0 += chunk) {
        const int c = std::min(chunk, count - j0);
        lrpr_status r = factor_batch(ctx, ops + j0, c, store_mask, outs + j0);
        if (r != LRPR_OK) {
            for (int j = 0; j < j0; ++j) {
                lrpr_factor_destroy(outs[j]);
                outs[j] = nullptr;
            }
            return r;
        }
    }
    return LRPR_OK;
}

lrpr_status lrpr_tune_set(lrpr_ctx ctx, int param, int64_t value) {
    if (!ctx) return LRPR_ERR_ARG;
    switch (param) {
        case LRPR_TUNE_LU_WGS:
            if (value < 0 || value > 256) return fail(ctx, LRPR_ERR_ARG, "lrpr_tune_set: LU workgroups in [0, 256]");
            ctx->tune_lu_wgs = (int)value;
            return LRPR_OK;
        case LRPR_TUNE_LU_BUDGET:
            if (value < 0) return fail(ctx, LRPR_ERR_ARG, "lrpr_tune_set: negative budget");
            ctx->tune_lu_budget = (size_t)value;
            return LRPR_OK;
        case LRPR_TUNE_PARAREAL_GRAPH:
            if (value != 0 && value != 1) return fail(ctx, LRPR_ERR_ARG, "lrpr_tune_set: graph switch is 0 or 1");
            ctx->tune_pr_graph = (int)value;
            return LRPR_OK;
        case LRPR_TUNE_SWEEP_GROUPS:
            if (value < 0 || value > 3) return fail(ctx, LRPR_ERR_ARG, "lrpr_tune_set: sweep groups in [0, 3]");
            ctx->tune_sweep_groups = (int)value;
            return LRPR_OK;
        case LRPR_TUNE_RSVD_BUDGET:
            if (value < 0) return fail(ctx, LRPR_ERR_ARG, "lrpr_tune_set: negative budget");
            ctx->tune_rsvd_budget = (size_t)value;
            return LRPR_OK;
        default:
            return fail(ctx, LRPR_ERR_ARG, "lrpr_tune_set: unknown parameter");
    }
}

lrpr_status lrpr_tune_get(lrpr_ctx ctx, int param, int64_t *value) {
    if (!ctx || !value) return LRPR_ERR_ARG;
    switch (param) {
        case LRPR_TUNE_LU_WGS: *value = ctx->tune_lu_wgs; return LRPR_OK;
        case LRPR_TUNE_LU_BUDGET: *value = (int64_t)ctx->tune_lu_budget; return LRPR_OK;
        case LRPR_TUNE_PARAREAL_GRAPH: *value = ctx->tune_pr_graph; return LRPR_OK;
        case LRPR_TUNE_SWEEP_GROUPS: *value = ctx->tune_sweep_groups; return LRPR_OK;
        case LRPR_TUNE_RSVD_BUDGET: *value = (int64_t)ctx->tune_rsvd_budget; return LRPR_OK;
        default: return fail(ctx, LRPR_ERR_ARG, "lrpr_tune_get: unknown parameter");
    }
}

lrpr_status lrpr_autotune_factor(lrpr_ctx ctx, const lrpr_op_desc *op, int count, int store_mask, int *best_wgs,
                                 double *best_ms) {
    if (!ctx || !op || count < 1) return fail(ctx, LRPR_ERR_ARG, "lrpr_autotune_factor: invalid arguments");
    const int64_t n = op->dim == 1 ? op->nx : (int64_t)op->nx * op->nx;
    const int bw = op->dim == 1 ? 1 : op->nx;
    const int NT = (int)((n + TILE - 1) / TILE), nb = (bw + TILE - 1) / TILE;
    const int full = std::min(nb + 9, NT);
    HIPCHK(hipSetDevice(ctx->dev), "hipSetDevice");
    // one chunk of a factor_many of `count` operators
    const int cnt = many_chunk(ctx, *op, count, store_mask);
    // candidates: the default choice for the chunk, the full width and
    // narrower ones that fit more matrices into a launch; each times one
    // factor_many of the chunk's `cnt` copies of op
    std::vector<int> cand;
    for (int c : {tile_lu_wgs(cnt, NT, nb, 0, tile_lu_resident(nb)), full, 24, 16, 12, 8, 6, 4})
        if (c <= full && c >= 1 && std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
    std::vector<lrpr_op_desc> ops(cnt, *op);
    std::vector<lrpr_fac> outs(cnt, nullptr);
    const int saved = ctx->tune_lu_wgs;
    int best = 0;
    double best_t = 1e300;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0), "event");
    HIPCHK(hipEventCreate(&e1), "event");
    lrpr_status r = LRPR_OK;
    // one untimed run first (first-use allocations), then one timed run per candidate
    for (int i = -1; i < (int)cand.size() && r == LRPR_OK; ++i) {
        const int c = cand[i < 0 ? 0 : i];
        ctx->tune_lu_wgs = c;
        hipEventRecord(e0, ctx->stream);
        r = lrpr_factor_many(ctx, ops.data(), cnt, store_mask, outs.data());
        hipEventRecord(e1, ctx->stream);
        hipEventSynchronize(e1);
        for (lrpr_fac f : outs)
            if (f) lrpr_factor_destroy(f);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (i >= 0 && r == LRPR_OK && ms < best_t) {
            best_t = ms;
            best = c;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    ctx->tune_lu_wgs = r == LRPR_OK ? best : saved;
    if (r != LRPR_OK) return r;
    if (best_wgs) *best_wgs = best;
    if (best_ms) *best_ms = best_t;
    return LRPR_OK;
}

lrpr_status lrpr_ctx_release_workspaces(lrpr_ctx ctx) {
    if (!ctx) return LRPR_ERR_ARG;
    HIPCHK(hipSetDevice(ctx->dev), "hipSetDevice");
    HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
    for (auto &kv : ctx->ws)
        if (kv.second.first) hipFree(kv.second.first);
    ctx->ws.clear();
    return LRPR_OK;
}

lrpr_status lrpr_factor_info(lrpr_fac f, int64_t *n, int *bw, double *dt) {
    if (!f) return LRPR_ERR_ARG;
    if (n) *n = f->n;
    if (bw) *bw = f->bw;
    if (dt) *dt = f->dt_step;
    return LRPR_OK;
}

lrpr_status lrpr_factor_sequence(lrpr_ctx ctx, const lrpr_op_desc *ops, int m, int store_mask, lrpr_fac *out) {
    if (!ctx || !ops || !out || m < 1) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor_sequence: invalid arguments");
    for (int j = 1; j < m; ++j)
        if (ops[j].dim != ops[0].dim || ops[j].nx != ops[0].nx)
            return fail(ctx, LRPR_ERR_ARG, "lrpr_factor_sequence: the steps' operators must share dim and nx");
    lrpr_fac h = new (std::nothrow) lrpr_factor_s();
    if (!h) return fail(ctx, LRPR_ERR_NOMEM, "lrpr_factor_sequence: host allocation");
    constexpr int CHUNK = 64;   // factors assembled and factored together (device memory in flight)
    for (int j0 = 0; j0 < m; j0 += CHUNK) {
        const int c = m - j0 < CHUNK ? m - j0 : CHUNK;
        std::vector<lrpr_fac> gs(c, nullptr);
        lrpr_status r = factor_batch(ctx, ops + j0, c, store_mask, gs.data());
        if (r != LRPR_OK) {
            lrpr_factor_destroy(h);
            return r;
        }
        for (lrpr_fac g : gs) h->seq.push_back(g);
    }
    // the handle carries the common shape; it holds no tiles of its own
    const lrpr_fac g0 = h->seq[0];
    h->dev = g0->dev;
    h->op = g0->op;
    h->n = g0->n;
    h->bw = g0->bw;
    h->NT = g0->NT;
    h->nb = g0->nb;
    h->mask = g0->mask;
    h->P = g0->P;
    h->stepper = LRPR_STEP_SEQUENCE;
    h->dt_step = g0->dt_step;
    *out = h;
    return LRPR_OK;
}

lrpr_status lrpr_factor_stepper(lrpr_ctx ctx, const lrpr_op_desc *op, int store_mask, int stepper,
                                lrpr_fac *out) {
    if (!ctx || !op || !out) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor_stepper: null argument");
    if (stepper != LRPR_STEP_EULER && stepper != LRPR_STEP_SDIRK2 && stepper != LRPR_STEP_SDIRK2L)
        return fail(ctx, LRPR_ERR_ARG, "lrpr_factor_stepper: unknown stepper");
    lrpr_op_desc o = *op;
    if (stepper == LRPR_STEP_SDIRK2L) o.dt = op->dt * SDIRK2L_GAMMA;   // I + g dt A
    lrpr_status r = lrpr_factor(ctx, &o, store_mask, out);
    if (r != LRPR_OK) return r;
    (*out)->stepper = stepper;
    (*out)->dt_step = op->dt;
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

lrpr_status lrpr_factor_copy_tiles(lrpr_ctx ctx, lrpr_fac f, int set, lrpr_prec prec, void *host) {
    if (!ctx || !f || !host || (set != 0 && set != 1) || (prec != LRPR_F64 && prec != LRPR_F32))
        return fail(ctx, LRPR_ERR_ARG, "lrpr_factor_copy_tiles: invalid arguments");
    const bool f32 = prec == LRPR_F32;
    const void *src = (f32 ? f->t32 : f->t64).a[set == 0 ? TS_LB : TS_UB];
    if (!src) return fail(ctx, LRPR_ERR_ARG, "lrpr_factor_copy_tiles: factor kept without tiles of that precision");
    const size_t bytes = (f32 ? 4 : 8) * (size_t)f->NT * f->nb * TILE_ELEMS;
    HIPCHK(hipSetDevice(ctx->dev), "hipSetDevice");
    HIPCHK(hipMemcpyAsync(host, src, bytes, hipMemcpyDeviceToHost, ctx->stream), "copy tiles");
    HIPCHK(hipStreamSynchronize(ctx->stream), "sync");
    return LRPR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched sweeps
// ---------------------------------------------------------------------------
namespace lrpr {

// narrow sweeps (at most this many 16-column groups) take the partitioned path
constexpr int SPLIT_MAX_GROUPS = 32;
// most consecutive groups on one factor whose update shares a spike read
constexpr int SPLIT_RUN_GROUPS = 8;

FacView fac_view(lrpr_fac f, bool f32) {
    const TileSet &t = f32 ? f->t32 : f->t64;
    const TileSet &tr = f32 ? f->t32r : f->t64r;
    FacView v;
    for (int a = 0; a < TS_COUNT; ++a) {
        v.a[a] = t.a[a];
        v.ar[a] = tr.a[a];
    }
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

// Profiling record of one sweep: algorithmic work of 4 n b flops and 2 n s
// bytes per RHS step, plus one read of each distinct factor per step; event
// recorded before the launch.
static hipError_t prof_begin(lrpr_ctx ctx, int npanels, const lrpr_panel *panels, int nsteps, bool f32,
                             lrpr_ctx_s::ProfRec &rec) {
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
    hipError_t e;
    if ((e = hipEventCreate(&rec.a)) != hipSuccess || (e = hipEventCreate(&rec.b)) != hipSuccess) return e;
    return hipEventRecord(rec.a, ctx->stream);
}

void *ws_get(lrpr_ctx ctx, const char *key, size_t bytes, hipError_t *err);

// Partitioned fine sweep (few column groups): per step, the L pass as local
// solves of all blocks, chain, update; then the U pass the same way.
static lrpr_status run_split(lrpr_ctx ctx, int npanels, const lrpr_panel *panels,
                             const std::vector<SweepItem> &groups, int nsteps, bool f32, int max_nb, int step0,
                             bool record, SweepPlan *plan, const std::string &pre) {
    hipStream_t st = ctx->stream;
    const size_t esz = f32 ? 4 : 8;
    // factor of every group (items were built panel by panel)
    std::vector<lrpr_fac> gf;
    for (int p = 0; p < npanels; ++p)
        for (int c0 = 0; c0 < panels[p].w; c0 += TILE) gf.push_back(panels[p].F);
    std::vector<SweepItem> loc;
    std::vector<SplitGroup> sg(groups.size());
    size_t bnd_elems = 0;
    int max_P = 0, max_rows = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
        const lrpr_fac F = gf[g];
        max_P = std::max(max_P, F->P);
        for (int p = 0; p < F->P; ++p) max_rows = std::max(max_rows, F->blk[p + 1] - F->blk[p]);
        bnd_elems += (size_t)F->P * F->nb * TILE_ELEMS;
    }
    hipError_t e = hipSuccess;
    char *bnd = (char *)ws_get(ctx, (pre + "split_bnd").c_str(), bnd_elems * esz, &e);
    // runs of consecutive groups on one factor (the update reads their spikes once)
    // (at most SPLIT_RUN_GROUPS groups per run, so wide launches still spread
    // the update over many workgroups; a group's arithmetic is the same in any run)
    std::vector<int2> runs;
    for (size_t g = 0; g < groups.size(); ++g) {
        if (g > 0 && gf[g] == gf[g - 1] && runs.back().y < SPLIT_RUN_GROUPS) ++runs.back().y;
        else runs.push_back(make_int2((int)g, 1));
    }
    SplitGroup *d_groups =
        (SplitGroup *)ws_get(ctx, (pre + "split_groups").c_str(), sizeof(SplitGroup) * sg.size(), &e);
    int2 *d_runs =
        d_groups ? (int2 *)ws_get(ctx, (pre + "split_runs").c_str(), sizeof(int2) * runs.size(), &e) : nullptr;
    if (!bnd || !d_groups || !d_runs)
        return hipfail(ctx, e == hipSuccess ? hipErrorOutOfMemory : e, "split workspace");
    size_t off = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (size_t g = 0; g < groups.size(); ++g) {
            const lrpr_fac F = gf[g];
            for (int p = 0; p < F->P; ++p) {
                SweepItem it = groups[g];
                it.r0 = F->blk[p];
                it.r1 = F->blk[p + 1];
                it.passes = pass == 0 ? 1 : 2;
                if (pass == 1) {
                    it.f = nullptr;
                    it.fcol = nullptr;
                    it.fscale = nullptr;
                }
                loc.push_back(it);
            }
        }
    for (size_t g = 0; g < groups.size(); ++g) {
        const lrpr_fac F = gf[g];
        const SplitSet &ss = f32 ? F->s32 : F->s64;
        SplitGroup &G = sg[g];
        G.X = groups[g].X;
        G.ldx = groups[g].ldx;
        G.ncols = groups[g].ncols;
        G.n = (int)F->n;
        G.NT = F->NT;
        G.nb = F->nb;
        G.P = F->P;
        G.blk = F->d_blk;
        G.S = ss.S;
        G.T = ss.T;
        G.bnd = bnd + off * esz;
        off += (size_t)F->P * F->nb * TILE_ELEMS;
    }
    const int nL = (int)(loc.size() / 2);
    SweepItem *d_items = nullptr;
    if (plan) {
        d_items = (SweepItem *)ws_get(ctx, (pre + "items").c_str(), sizeof(SweepItem) * loc.size(), &e);
        if (!d_items) return hipfail(ctx, e == hipSuccess ? hipErrorOutOfMemory : e, "split items");
    } else {
        lrpr_status ls = ensure_items(ctx, loc.size());
        if (ls != LRPR_OK) return ls;
        d_items = ctx->d_items;
    }
    if ((e = hipMemcpyAsync(d_items, loc.data(), loc.size() * sizeof(SweepItem), hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(d_groups, sg.data(), sg.size() * sizeof(SplitGroup), hipMemcpyHostToDevice, st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(d_runs, runs.data(), runs.size() * sizeof(int2), hipMemcpyHostToDevice, st)) !=
            hipSuccess)
        return hipfail(ctx, e, "split upload");
    lrpr_ctx_s::ProfRec rec{};
    record = record && !plan;
    if (record && ctx->prof && (e = prof_begin(ctx, npanels, panels, nsteps, f32, rec)) != hipSuccess)
        return hipfail(ctx, e, "profile event");
    const int ng = (int)sg.size();
    bool uni = max_nb == 8 || max_nb == 16 || max_nb == 32;
    for (const SplitGroup &G : sg) uni = uni && G.nb == max_nb;
    const int nr = uni ? (int)runs.size() : 0;
    const int2 *dr = uni ? d_runs : nullptr;
    for (int step = 0; step < nsteps; ++step) {
        const int sj = step0 + step;
        auto one = [=](hipStream_t s) -> hipError_t {
            hipError_t ee;
            if ((ee = launch_sweep(false, false, f32, nL, d_items, 1, max_nb, s, sj, true)) != hipSuccess ||
                (ee = launch_split_chain(f32, false, ng, d_groups, max_nb, s, uni)) != hipSuccess ||
                (ee = launch_split_update(f32, false, ng, d_groups, max_P, max_rows, s, max_nb, nr, dr)) !=
                    hipSuccess ||
                (ee = launch_sweep(false, false, f32, nL, d_items + nL, 1, max_nb, s, sj, true)) != hipSuccess ||
                (ee = launch_split_chain(f32, true, ng, d_groups, max_nb, s, uni)) != hipSuccess ||
                (ee = launch_split_update(f32, true, ng, d_groups, max_P, max_rows, s, max_nb, nr, dr)) !=
                    hipSuccess)
                return ee;
            return hipSuccess;
        };
        if (plan) plan->launches.push_back(one);
        else if ((e = one(st)) != hipSuccess) return hipfail(ctx, e, "split sweep");
    }
    if (record && ctx->prof) {
        if ((e = hipEventRecord(rec.b, st)) != hipSuccess) return hipfail(ctx, e, "profile event");
        ctx->prof_recs.push_back(rec);
    }
    return LRPR_OK;
}

// XCD-aware order of a launch's work items.  Workgroups are dispatched to
// the chip's 8 XCDs round-robin (workgroup i on XCD i % 8), and each XCD has
// its own L2.  Runs of consecutive items on one factor (the column groups of
// one panel) are dealt whole to the XCD queue with the fewest items (split
// only to keep the queues equal), and item l of queue x goes to position
// 8 l + x: the groups that read the same factor tiles start together on one
// XCD and share its L2 instead of each fetching the factor from HBM.  The
// items are independent, so the order changes no result.
static void xcd_order(std::vector<SweepItem> &items) {
    constexpr int NX = 8;
    const size_t ni = items.size();
    if (ni < 2 * NX) return;
    std::vector<std::pair<size_t, size_t>> runs;   // first item, count
    for (size_t i = 0; i < ni; ++i) {
        if (i > 0 && items[i].fac.a[TS_LB] == items[i - 1].fac.a[TS_LB] &&
            items[i].fac.a[TS_UB] == items[i - 1].fac.a[TS_UB])
            ++runs.back().second;
        else
            runs.push_back({i, 1});
    }
    if (runs.size() < 2) return;
    const size_t target = (ni + NX - 1) / NX;
    std::vector<std::vector<size_t>> q(NX);
    for (auto r : runs) {
        size_t at = r.first, left = r.second;
        while (left > 0) {
            int x = 0;
            for (int y = 1; y < NX; ++y)
                if (q[y].size() < q[x].size()) x = y;
            const size_t room = target > q[x].size() ? target - q[x].size() : 1;
            const size_t take = std::min(left, room);
            for (size_t k = 0; k < take; ++k) q[x].push_back(at + k);
            at += take;
            left -= take;
        }
    }
    std::vector<SweepItem> out;
    out.reserve(ni);
    size_t maxlen = 0;
    for (auto &v : q) maxlen = std::max(maxlen, v.size());
    for (size_t l = 0; l < maxlen; ++l)
        for (int x = 0; x < NX; ++x)
            if (l < q[x].size()) out.push_back(items[q[x][l]]);
    items.swap(out);
}

// Merge runs of consecutive 16-column items of one panel (same factor and
// sources, columns 16 apart, all but the last full) into items of up to ng
// groups.
static std::vector<SweepItem> group_items(const std::vector<SweepItem> &items, int ng, size_t esz) {
    std::vector<SweepItem> out;
    for (size_t i = 0; i < items.size();) {
        SweepItem m = items[i];
        size_t j = i + 1;
        int groups = 1;
        while (j < items.size() && groups < ng) {
            const SweepItem &b = items[j];
            const bool next = b.fac.a[TS_LB] == m.fac.a[TS_LB] && b.fac.a[TS_UB] == m.fac.a[TS_UB] &&
                              b.ldx == m.ldx && m.ncols == 16 * groups &&
                              (const char *)b.X == (const char *)m.X + (size_t)16 * groups * m.ldx * esz &&
                              b.f == m.f && b.ldf == m.ldf && b.passes == m.passes && b.r0 == m.r0 && b.r1 == m.r1 &&
                              b.fsteps == m.fsteps && (b.fcol == nullptr) == (m.fcol == nullptr) &&
                              (!m.fcol || b.fcol == m.fcol + 16 * groups) &&
                              (b.fscale == nullptr) == (m.fscale == nullptr) &&
                              (!m.fscale || b.fscale == m.fscale + (size_t)16 * groups * m.fsteps);
            if (!next) break;
            m.ncols += b.ncols;
            ++groups;
            ++j;
        }
        out.push_back(m);
        i = j;
    }
    return out;
}

// Validate panels and turn them into 16-column work items; launch one sweep
// of nsteps solve steps.  A column's source factors are fscale[c * fstride +
// step0 + j], j < nsteps.  record: add a profile record for the launch.
static lrpr_status run_sweep_core(lrpr_ctx ctx, int npanels, const lrpr_panel *panels, int nsteps, lrpr_prec prec,
                                  bool adjoint, int fstride, int step0, bool record, bool split_any_width,
                                  SweepPlan *plan = nullptr, const std::string &pre = std::string()) {
    const bool f32 = prec == LRPR_F32;
    std::vector<SweepItem> items;
    std::vector<int> item_w;   // width of the item's panel
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
            it.passes = 3;
            it.r0 = 0;
            it.r1 = P.F->NT;
            it.fsteps = fstride;
            it.pad_ = 0;
            it.f = adjoint ? nullptr : P.f;
            it.ldf = P.ldf;
            it.fcol = (!adjoint && P.f && P.fcol) ? P.fcol + c0 : nullptr;
            it.fscale = (!adjoint && P.f && P.fscale) ? P.fscale + (size_t)c0 * fstride : nullptr;
            items.push_back(it);
            item_w.push_back(P.w);
        }
    }
    if (items.empty() || nsteps == 0) return LRPR_OK;
    if (max_nb > 64) return fail(ctx, LRPR_ERR_ARG, "sweep: half-bandwidth above 1023");
    hipError_t e = hipSetDevice(ctx->dev);
    if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
    // Few column groups on factors with spikes: partitioned passes, so that
    // every group spreads over P compute units.  With split_any_width the
    // choice does not depend on the launch's width.
    bool split = !adjoint && ((int)items.size() <= SPLIT_MAX_GROUPS || split_any_width) &&
                 max_nb <= (f32 ? 64 : 32);
    for (int p = 0; p < npanels && split; ++p)
        split = panels[p].w == 0 || (panels[p].F->P >= 2 && (f32 ? panels[p].F->s32.S : panels[p].F->s64.S));
    if (split) return run_split(ctx, npanels, panels, items, nsteps, f32, max_nb, step0, record, plan, pre);
    // Pass pairs when every factor carries the UL set (and, for the
    // adjoint, its mirrored tiles) and all have the same band-tile count
    // (tile arrays addressed with 32-bit byte offsets).  Not with
    // split_any_width: there a problem's path must not depend on the others.
    bool paired = !split_any_width && nsteps >= 2 && sweep_pairable(max_nb) && !(adjoint && strided);
    for (const SweepItem &it : items)
        paired = paired && it.fac.nb == max_nb && it.fac.ar[TS_LB] && (!adjoint || it.fac.ar[TS_UTB]) &&
                 (double)(it.fac.NT + 2 * guard_rows(max_nb)) * max_nb * TILE_ELEMS * (f32 ? 4 : 8) < 4.0e9;
    // Narrow panels (at most sweep_narrow_cols columns per factor) run on the
    // vector ALUs: a single column then does not pay for a 16-column group.
    // Without split_any_width the whole launch goes narrow when every item
    // is; the alternating L U / U' L' pairs measured about half the FP32
    // error of L U steps alone (32 steps on 255^2 grids), so factors that
    // carry the UL set keep the matrix-core pass pairs.  With split_any_width
    // (Parareal) each panel's own width decides, so a problem rounds the same
    // whatever else shares the launch.
    const int ncmax = sweep_narrow_cols(f32);
    std::vector<char> is_narrow(items.size(), 0);
    if (!adjoint && !paired) {
        bool all = true;
        for (size_t i = 0; i < items.size(); ++i) {
            const int nb = items[i].fac.nb;
            is_narrow[i] = nb >= 2 && nb <= 64 && (split_any_width ? item_w[i] <= ncmax : items[i].ncols <= ncmax);
            all = all && is_narrow[i];
        }
        if (!split_any_width && !all) std::fill(is_narrow.begin(), is_narrow.end(), 0);
    }
    // narrow items (cut into <= ncmax columns) first, then the matrix-core
    // items by band class: each class runs its own kernel, so an item's
    // arithmetic depends only on its own factor's band
    const size_t esz = f32 ? 4 : 8;
    std::vector<SweepItem> nit;
    int narrow_cols = 0, narrow_nb = 1;
    std::vector<std::vector<SweepItem>> cls(7);
    auto class_of = [](int nb) { return nb <= 1 ? 0 : nb <= 4 ? 1 : nb <= 8 ? 2 : nb <= 16 ? 3 : nb <= 32 ? 4 : 5; };
    for (size_t i = 0; i < items.size(); ++i) {
        const SweepItem &it = items[i];
        if (is_narrow[i]) {
            for (int c0 = 0; c0 < it.ncols; c0 += ncmax) {
                SweepItem q = it;
                q.X = (char *)it.X + (size_t)c0 * it.ldx * esz;
                q.ncols = std::min(ncmax, it.ncols - c0);
                if (q.fcol) q.fcol = it.fcol + c0;
                if (q.fscale) q.fscale = it.fscale + (size_t)c0 * it.fsteps;
                narrow_cols = std::max(narrow_cols, q.ncols);
                narrow_nb = std::max(narrow_nb, it.fac.nb);
                nit.push_back(q);
            }
        } else {
            cls[paired ? 6 : class_of(it.fac.nb)].push_back(it);
        }
    }
    struct Launch {
        size_t at, count;
        int nb, ng;
    };
    std::vector<Launch> wide;
    xcd_order(nit);
    std::vector<SweepItem> all_items = nit;
    for (int c = 0; c < 7; ++c) {
        std::vector<SweepItem> &v = cls[c];
        if (v.empty()) continue;
        int cnb = 1;
        for (const SweepItem &it : v) cnb = std::max(cnb, it.fac.nb);
        // Several 16-column groups of one panel per workgroup: every band
        // tile read then feeds all of them (the groups' arithmetic is
        // unchanged); by default the most that still leave no compute unit
        // idle
        int ng = 1;
        if (!paired) {
            ng = ctx->tune_sweep_groups ? std::min(ctx->tune_sweep_groups, sweep_max_groups(f32, cnb))
                                        : sweep_max_groups(f32, cnb);
            while (!ctx->tune_sweep_groups && ng > 1 && (int)group_items(v, ng, esz).size() < ctx->ncu) --ng;
            if (ng > 1) v = group_items(v, ng, esz);
        }
        xcd_order(v);
        wide.push_back({all_items.size(), v.size(), cnb, ng});
        all_items.insert(all_items.end(), v.begin(), v.end());
    }
    items.swap(all_items);
    const size_t nn = nit.size();
    if (paired) {
        // [0, ni): first substitution of the first step; [ni, 2ni): second
        // substitution of an L U step; [2ni, 3ni): second substitution of a
        // U' L' step (the UL set's first-pass tiles, no source)
        const size_t ni = items.size();
        items.resize(3 * ni);
        for (size_t i = 0; i < ni; ++i) {
            items[i].passes = 1;
            items[ni + i] = items[i];
            items[ni + i].passes = 2;
            SweepItem &r = items[2 * ni + i];
            r = items[i];
            for (int k = 0; k < TS_COUNT; ++k) r.fac.a[k] = r.fac.ar[k];
            r.f = nullptr;
            r.fcol = nullptr;
            r.fscale = nullptr;
        }
    }
    SweepItem *d_items = nullptr;
    if (plan) {
        d_items = (SweepItem *)ws_get(ctx, (pre + "items").c_str(), sizeof(SweepItem) * items.size(), &e);
        if (!d_items) return hipfail(ctx, e == hipSuccess ? hipErrorOutOfMemory : e, "sweep items");
    } else {
        lrpr_status st = ensure_items(ctx, items.size());
        if (st != LRPR_OK) return st;
        d_items = ctx->d_items;
    }
    e = hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(SweepItem), hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return hipfail(ctx, e, "sweep item upload");
    lrpr_ctx_s::ProfRec rec{};
    record = record && !plan;
    if (record && ctx->prof && (e = prof_begin(ctx, npanels, panels, nsteps, f32, rec)) != hipSuccess)
        return hipfail(ctx, e, "profile event");
    std::function<hipError_t(hipStream_t)> go;
    if (!paired) {
        go = [=](hipStream_t s) {
            hipError_t ee = hipSuccess;
            if (nn > 0) ee = launch_sweep_narrow(f32, (int)nn, d_items, nsteps, narrow_nb, narrow_cols, s, step0);
            for (const Launch &L : wide)
                if (ee == hipSuccess)
                    ee = launch_sweep(adjoint, strided, f32, (int)L.count, d_items + L.at, nsteps, L.nb, s, step0,
                                      false, L.ng);
            return ee;
        };
    } else {
        // even steps (from step0) L U, odd steps U' L'; the second
        // substitution of step s runs with the first of step s+1
        const size_t ni = items.size() / 3;
        const int nii = (int)ni;
        go = [=](hipStream_t s) {
            hipError_t ee = launch_sweep(adjoint, false, f32, nii, d_items, 1, max_nb, s, step0);
            for (int q = 0; q + 1 < nsteps && ee == hipSuccess; ++q)
                ee = launch_sweep_pair(adjoint, (q & 1) != 0, f32, nii, d_items, max_nb, s, step0 + q + 1);
            if (ee == hipSuccess)
                ee = launch_sweep(adjoint, false, f32, nii, d_items + (((nsteps - 1) & 1) ? 2 * ni : ni), 1, max_nb,
                                  s, step0 + nsteps - 1);
            return ee;
        };
    }
    if (plan) {
        plan->launches.push_back(go);
    } else if ((e = go(ctx->stream)) != hipSuccess) {
        return hipfail(ctx, e, paired ? "paired sweep launch" : "sweep launch");
    }
    if (record && ctx->prof) {
        if ((e = hipEventRecord(rec.b, ctx->stream)) != hipSuccess) return hipfail(ctx, e, "profile event");
        ctx->prof_recs.push_back(rec);
    }
    return LRPR_OK;
}

lrpr_status plan_sweep(lrpr_ctx ctx, int npanels, const lrpr_panel *panels, int nsteps, lrpr_prec prec,
                       bool adjoint, bool split_any_width, const char *ws_prefix, SweepPlan *plan) {
    if (!ctx || !plan || !ws_prefix) return LRPR_ERR_ARG;
    if (npanels < 0 || (npanels > 0 && !panels) || nsteps < 0 || (prec != LRPR_F64 && prec != LRPR_F32))
        return fail(ctx, LRPR_ERR_ARG, "sweep plan: invalid arguments");
    for (int p = 0; p < npanels; ++p)
        if (!panels[p].F || (panels[p].w > 0 && panels[p].F->stepper != LRPR_STEP_EULER))
            return fail(ctx, LRPR_ERR_ARG, "sweep plan: implicit-Euler factors only");
    plan->launches.clear();
    return run_sweep_core(ctx, npanels, panels, nsteps, prec, adjoint, nsteps, 0, false, split_any_width, plan,
                          ws_prefix);
}

// Sweeps of nsteps time steps of the panels' common stepper.  Implicit
// Euler: one solve per step.  The two-stage SDIRK methods (both with a_11 =
// a_22 = g, the factored matrix M = I + g dt A): with stage values U_i
// (M U_i = r_i), the tableaus give
//   stage 1: r_1 = u + g dt f(t + c_1 dt)
//   stage 2: r_2 = u + beta (U_1 - u) + g dt f(t + c_2 dt)
//   step:    u_new = U_1 + (U_2 - u) / 2 (SDIRK2),  u_new = U_2 (SDIRK2-L)
// with beta = -1 (SDIRK2) and (1 - g) / g (SDIRK2-L).  Every linear map of
// a step is a rational function of M, so the adjoint runs the same
// combinations with M^T.
lrpr_status run_sweep(lrpr_ctx ctx, int npanels, const lrpr_panel *panels, int nsteps, lrpr_prec prec,
                      bool adjoint, bool split_any_width) {
    if (!ctx) return LRPR_ERR_ARG;
    if (npanels < 0 || (npanels > 0 && !panels) || nsteps < 0 || (prec != LRPR_F64 && prec != LRPR_F32))
        return fail(ctx, LRPR_ERR_ARG, "sweep: invalid arguments");
    int stepper = -1;
    for (int p = 0; p < npanels; ++p) {
        if (!panels[p].F) return fail(ctx, LRPR_ERR_ARG, "sweep: panel with null factor");
        if (panels[p].w <= 0) continue;
        if (stepper >= 0 && panels[p].F->stepper != stepper)
            return fail(ctx, LRPR_ERR_ARG, "sweep: the panels' factors use different time steppers");
        stepper = panels[p].F->stepper;
    }
    if (stepper <= 0) return run_sweep_core(ctx, npanels, panels, nsteps, prec, adjoint, nsteps, 0, true, split_any_width);
    if (nsteps == 0) return LRPR_OK;
    if (stepper == LRPR_STEP_SEQUENCE) {
        // step j with each panel's j-th factor; the adjoint in reverse order
        for (int p = 0; p < npanels; ++p)
            if (panels[p].w > 0 && (int)panels[p].F->seq.size() < nsteps)
                return fail(ctx, LRPR_ERR_ARG, "sweep: more steps than the factor sequence holds");
        std::vector<lrpr_panel> sp(panels, panels + npanels);
        hipError_t e = hipSuccess;
        lrpr_ctx_s::ProfRec rec{};
        if (ctx->prof && (e = prof_begin(ctx, npanels, panels, nsteps, prec == LRPR_F32, rec)) != hipSuccess)
            return hipfail(ctx, e, "profile event");
        for (int j = 0; j < nsteps; ++j) {
            const int idx = adjoint ? nsteps - 1 - j : j;
            for (int p = 0; p < npanels; ++p)
                if (panels[p].w > 0) sp[p].F = panels[p].F->seq[idx];
            lrpr_status r = run_sweep_core(ctx, npanels, sp.data(), 1, prec, adjoint, nsteps, idx, false, split_any_width);
            if (r != LRPR_OK) return r;
        }
        if (ctx->prof) {
            if ((e = hipEventRecord(rec.b, ctx->stream)) != hipSuccess) return hipfail(ctx, e, "profile event");
            ctx->prof_recs.push_back(rec);
        }
        return LRPR_OK;
    }
    const bool f32 = prec == LRPR_F32;
    const size_t esz = f32 ? 4 : 8;
    const double g = stepper == LRPR_STEP_SDIRK2L ? SDIRK2L_GAMMA : 1.0;
    const double beta = stepper == LRPR_STEP_SDIRK2L ? (1.0 - g) / g : -1.0;
    // stage workspaces: u and U_1 of every panel
    std::vector<size_t> off(npanels + 1, 0);
    for (int p = 0; p < npanels; ++p) off[p + 1] = off[p] + (size_t)panels[p].F->n * std::max(panels[p].w, 0);
    hipError_t e = hipSetDevice(ctx->dev);
    if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
    char *Wu = (char *)ws_get(ctx, "sdirk_u", off[npanels] * esz, &e);
    char *Wv = Wu ? (char *)ws_get(ctx, "sdirk_v", off[npanels] * esz, &e) : nullptr;
    if (!Wu || !Wv) return hipfail(ctx, e == hipSuccess ? hipErrorOutOfMemory : e, "SDIRK workspace");
    hipStream_t st = ctx->stream;
    // out = ca a + cb b + cc c on every panel; an operand is the panel (X) or a workspace
    enum { OX = 0, OU = 1, OV = 2 };
    auto comb = [&](int out, int a, double ca, int b, double cb, int c, double cc) -> hipError_t {
        for (int p = 0; p < npanels; ++p) {
            const lrpr_panel &P = panels[p];
            if (P.w <= 0) continue;
            auto ptr = [&](int o) -> void * {
                return o == OX ? P.X : (o == OU ? Wu : Wv) + off[p] * esz;
            };
            auto ld = [&](int o) -> int64_t { return o == OX ? P.ldx : P.F->n; };
            hipError_t ee = launch_combine3(f32, ptr(out), ld(out), ptr(a), ld(a), ca, b < 0 ? nullptr : ptr(b),
                                            b < 0 ? 0 : ld(b), cb, c < 0 ? nullptr : ptr(c), c < 0 ? 0 : ld(c), cc,
                                            P.F->n, P.w, st);
            if (ee != hipSuccess) return ee;
        }
        return hipSuccess;
    };
    lrpr_ctx_s::ProfRec rec{};
    if (ctx->prof) {
        if ((e = prof_begin(ctx, npanels, panels, nsteps, f32, rec)) != hipSuccess)
            return hipfail(ctx, e, "profile event");
        rec.flops *= 2;   // two stage solves per step
    }
    const int fstride = 2 * nsteps;
    for (int j = 0; j < nsteps; ++j) {
        lrpr_status r;
        if ((e = comb(OU, OX, 1.0, -1, 0.0, -1, 0.0)) != hipSuccess) return hipfail(ctx, e, "SDIRK copy");
        if ((r = run_sweep_core(ctx, npanels, panels, 1, prec, adjoint, fstride, 2 * j, false, split_any_width)) !=
            LRPR_OK)
            return r;
        if ((e = comb(OV, OX, 1.0, -1, 0.0, -1, 0.0)) != hipSuccess) return hipfail(ctx, e, "SDIRK copy");
        if ((e = comb(OX, OU, 1.0 - beta, OV, beta, -1, 0.0)) != hipSuccess) return hipfail(ctx, e, "SDIRK stage");
        if ((r = run_sweep_core(ctx, npanels, panels, 1, prec, adjoint, fstride, 2 * j + 1, false, split_any_width)) !=
            LRPR_OK)
            return r;
        if (stepper == LRPR_STEP_SDIRK2 && (e = comb(OX, OX, 0.5, OV, 1.0, OU, -0.5)) != hipSuccess)
            return hipfail(ctx, e, "SDIRK step");
    }
    if (ctx->prof) {
        if ((e = hipEventRecord(rec.b, st)) != hipSuccess) return hipfail(ctx, e, "profile event");
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

lrpr_status lrpr_randn(lrpr_ctx ctx, void *dst, int64_t count, lrpr_prec prec, uint64_t seed, uint64_t stream) {
    if (!ctx) return LRPR_ERR_ARG;
    if (count < 0 || (count > 0 && !dst) || (prec != LRPR_F64 && prec != LRPR_F32))
        return fail(ctx, LRPR_ERR_ARG, "lrpr_randn: invalid arguments");
    if (count == 0) return LRPR_OK;
    hipError_t e = hipSetDevice(ctx->dev);
    if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
    if ((e = launch_randn(prec == LRPR_F32, dst, count, seed, stream, ctx->stream)) != hipSuccess)
        return hipfail(ctx, e, "randn");
    return LRPR_OK;
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
