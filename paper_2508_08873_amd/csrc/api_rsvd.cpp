// Host side of the C ABI: randomized-SVD build of the coarse solvers and
// the Parareal solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>

#include "dense.h"
#include "lrpr_internal.h"

namespace lrpr {
FacView fac_view(lrpr_fac f, bool f32);

// Workspace cached per context and purpose; grows on demand.
void *ws_get(lrpr_ctx ctx, const char *key, size_t bytes, hipError_t *err);
}  // namespace lrpr

using namespace lrpr;

namespace {

// Temporaries of one call, taken from the context's cached workspaces (one
// slot per allocation, in call order): after the first call of a shape no
// call allocates or frees device memory, so independent contexts on
// separate streams never wait on each other here.
struct Scoped {
    lrpr_ctx ctx;
    const char *prefix;
    int count = 0;
    Scoped(lrpr_ctx c, const char *pre) : ctx(c), prefix(pre) {}
    template <typename T>
    hipError_t alloc(T **p, size_t n) {
        char key[48];
        snprintf(key, sizeof key, "%s%d", prefix, count++);
        hipError_t e = hipSuccess;
        void *q = ws_get(ctx, key, n * sizeof(T) > 0 ? n * sizeof(T) : 16, &e);
        *p = (T *)q;
        return q ? hipSuccess : (e == hipSuccess ? hipErrorOutOfMemory : e);
    }
};

lrpr_status herr(lrpr_ctx ctx, hipError_t e, const char *what) {
    return fail(ctx, e == hipErrorOutOfMemory ? LRPR_ERR_NOMEM : LRPR_ERR_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define CK(call, what)                                  \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return herr(ctx, e_, what); \
    } while (0)

template <typename T>
hipError_t upload(T *dst, const std::vector<T> &src, hipStream_t s) {
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

}  // namespace

namespace lrpr {

// Low-rank apply over w columns, split so that k*w fits the kernel's LDS.
hipError_t lowrank_cols(LrArgs a, double *part, double *incpart, hipStream_t s) {
    const int maxw = std::max(1, 12288 / std::max(a.k, 1));
    const int w = a.w;
    for (int c0 = 0; c0 < w; c0 += maxw) {
        LrArgs b = a;
        const int64_t off = (int64_t)c0 * a.n;
        b.w = std::min(maxw, w - c0);
        b.x = a.x ? a.x + off : nullptr;
        b.out = a.out + off;
        b.gold = a.gold ? a.gold + off : nullptr;
        b.bvec = a.bvec ? a.bvec + off : nullptr;
        b.fu64 = a.fu64 ? a.fu64 + off : nullptr;
        b.fu32 = a.fu32 ? a.fu32 + off : nullptr;
        b.active = a.active ? a.active + c0 : nullptr;
        b.part = part;
        b.incpart = incpart ? incpart + (int64_t)c0 : nullptr;   // layout [chunk][w] with stride w below
        if (incpart && b.w != w) return hipErrorInvalidValue;    // increments need all columns in one pass
        hipError_t e = launch_lowrank(b, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lrpr

// ---------------------------------------------------------------------------
// rSVD build
// ---------------------------------------------------------------------------
extern "C" {

lrpr_status lrpr_coarse_view(lrpr_coarse c, int first, int count, lrpr_coarse *out) {
    if (!c || !out || first < 0 || count < 1 || first + count > c->nslices) return LRPR_ERR_ARG;
    lrpr_coarse v = new (std::nothrow) lrpr_coarse_s();
    if (!v) return LRPR_ERR_NOMEM;
    size_t pos = 0;
    for (int s = 0; s < first; ++s) pos += (size_t)c->l[s];
    v->dev = c->dev;
    v->nslices = count;
    v->view = true;
    for (int s = first; s < first + count; ++s) {
        v->n.push_back(c->n[s]);
        v->k.push_back(c->k[s]);
        v->l.push_back(c->l[s]);
        v->U.push_back(c->U[s]);
        v->S.push_back(c->S[s]);
        v->V.push_back(c->V[s]);
        if ((size_t)s < c->F.size()) v->F.push_back(c->F[s]);
        v->sigma.insert(v->sigma.end(), c->sigma.begin() + pos, c->sigma.begin() + pos + c->l[s]);
        pos += (size_t)c->l[s];
    }
    *out = v;
    return LRPR_OK;
}

void lrpr_coarse_destroy(lrpr_coarse c) {
    if (!c) return;
    if (c->view) {
        delete c;
        return;
    }
    hipSetDevice(c->dev);
    hipDeviceSynchronize();
    if (c->block) {
        dfree(c->block, nullptr);
        for (double *b : c->more) dfree(b, nullptr);
    } else {
        for (size_t s = 0; s < c->U.size(); ++s) {
            if (c->U[s]) hipFree(c->U[s]);
            if (c->V[s]) hipFree(c->V[s]);
            if (c->S[s]) hipFree(c->S[s]);
        }
    }
    delete c;
}

lrpr_status lrpr_coarse_get(lrpr_coarse c, int s, const double **U, const double **S, const double **V, int *k,
                            int64_t *n) {
    if (!c || s < 0 || s >= c->nslices) return LRPR_ERR_ARG;
    if (U) *U = c->U[s];
    if (S) *S = c->S[s];
    if (V) *V = c->V[s];
    if (k) *k = c->k[s];
    if (n) *n = c->n[s];
    return LRPR_OK;
}

}  // extern "C"

static lrpr_status rsvd_build_impl(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices,
                                   const void *const *psi, int nsteps, int q, lrpr_prec range_prec,
                                   lrpr_coarse *out, double *sigma_host, int *fallback_host,
                                   const double *const *weights = nullptr);

extern "C" {

lrpr_status lrpr_rsvd_build(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices, int nsteps,
                            lrpr_prec range_prec, lrpr_coarse *out, double *sigma_host, int *fallback_host) {
    return lrpr_rsvd_build_q(ctx, nslices, slices, nsteps, 0, range_prec, out, sigma_host, fallback_host);
}

lrpr_status lrpr_rsvd_build_q(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices, int nsteps, int q,
                              lrpr_prec range_prec, lrpr_coarse *out, double *sigma_host, int *fallback_host) {
    return rsvd_build_impl(ctx, nslices, slices, nullptr, nsteps, q, range_prec, out, sigma_host, fallback_host);
}

lrpr_status lrpr_rsvd_build_w(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices,
                              const double *const *weights, int nsteps, int q, lrpr_prec range_prec,
                              lrpr_coarse *out, double *sigma_host, int *fallback_host) {
    if (!ctx) return LRPR_ERR_ARG;
    if (!weights) return fail(ctx, LRPR_ERR_ARG, "lrpr_rsvd_build_w: weights is null");
    return rsvd_build_impl(ctx, nslices, slices, nullptr, nsteps, q, range_prec, out, sigma_host, fallback_host,
                           weights);
}

lrpr_status lrpr_coarse_from_factors(lrpr_ctx ctx, int nslices, const lrpr_fac *F, const int *k,
                                     const double *const *U, const double *const *S, const double *const *V,
                                     lrpr_coarse *out) {
    if (!ctx) return LRPR_ERR_ARG;
    if (nslices <= 0 || !F || !k || !U || !S || !V || !out)
        return fail(ctx, LRPR_ERR_ARG, "lrpr_coarse_from_factors: invalid arguments");
    for (int s = 0; s < nslices; ++s)
        if (!F[s] || k[s] < 1 || (int64_t)k[s] > F[s]->n || !U[s] || !S[s] || !V[s] || F[s]->dev != ctx->dev)
            return fail(ctx, LRPR_ERR_ARG, "lrpr_coarse_from_factors: invalid slice");
    hipError_t e = hipSetDevice(ctx->dev);
    if (e != hipSuccess) return herr(ctx, e, "hipSetDevice");
    lrpr_coarse c = new (std::nothrow) lrpr_coarse_s();
    if (!c) return fail(ctx, LRPR_ERR_NOMEM, "coarse handle");
    c->dev = ctx->dev;
    c->nslices = nslices;
    c->n.resize(nslices);
    c->k.resize(nslices);
    c->l.resize(nslices);
    c->U.assign(nslices, nullptr);
    c->V.assign(nslices, nullptr);
    c->S.assign(nslices, nullptr);
    c->F.resize(nslices);
    auto bail = [&](lrpr_status stt, const char *msg) {
        lrpr_coarse_destroy(c);
        return fail(ctx, stt, msg);
    };
    hipStream_t st = ctx->stream;
    for (int s = 0; s < nslices; ++s) {
        const int64_t n = F[s]->n;
        c->n[s] = n;
        c->k[s] = c->l[s] = k[s];
        c->F[s] = F[s];
        const size_t nk = (size_t)n * k[s];
        if (hipMalloc(&c->U[s], nk * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->V[s], nk * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->S[s], (size_t)k[s] * sizeof(double)) != hipSuccess)
            return bail(LRPR_ERR_NOMEM, "coarse factors");
        if (hipMemcpyAsync(c->U[s], U[s], nk * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(c->V[s], V[s], nk * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(c->S[s], S[s], (size_t)k[s] * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
            return bail(LRPR_ERR_HIP, "copy factors");
    }
    size_t tot = 0;
    for (int s = 0; s < nslices; ++s) tot += (size_t)k[s];
    std::vector<double> hs(tot);   // sized before the copies are queued
    for (int s = 0, at = 0; s < nslices; at += k[s], ++s)
        if (hipMemcpyAsync(hs.data() + at, S[s], (size_t)k[s] * sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess)
            return bail(LRPR_ERR_HIP, "copy S");
    if (hipStreamSynchronize(st) != hipSuccess) return bail(LRPR_ERR_HIP, "coarse factors");
    c->sigma = hs;
    *out = c;
    return LRPR_OK;
}

lrpr_status lrpr_rsvd_build_two_sided(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices,
                                      const void *const *psi, int nsteps, lrpr_prec range_prec, lrpr_coarse *out,
                                      double *sigma_host, int *fallback_host) {
    if (!ctx) return LRPR_ERR_ARG;
    if (!psi) return fail(ctx, LRPR_ERR_ARG, "lrpr_rsvd_build_two_sided: psi is null");
    for (int s = 0; s < nslices; ++s)
        if (!psi[s]) return fail(ctx, LRPR_ERR_ARG, "lrpr_rsvd_build_two_sided: psi[s] is null");
    return rsvd_build_impl(ctx, nslices, slices, psi, nsteps, 0, range_prec, out, sigma_host, fallback_host);
}

}  // extern "C"

// Randomized SVD of every slice.  psi == null: one-sided (Sec. 2.1 steps 1-6,
// q power iterations); psi != null: the adjoint runs on the independent test
// vectors psi[s] and the core is (Psi^T Q)^{-1} (T^T Psi)^T (Sec. 2.2).
// weights (or null): per slice null or n positive doubles; the build then
// runs for W^{1/2} T W^{-1/2}: every forward sweep's input is scaled by
// W^{-1/2} and its output by W^{1/2}, every adjoint sweep's input by W^{1/2}
// and its output by W^{-1/2}, and the factors are mapped back at the end
// (U_k by W^{-1/2}, V_k by W^{1/2}) before the signs are fixed.
static lrpr_status rsvd_build_one(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices,
                                  const void *const *psi, int nsteps, int q, lrpr_prec range_prec,
                                  lrpr_coarse *out, double *sigma_host, int *fallback_host,
                                  const double *const *weights);

// The build in chunks of consecutive slices whose panels fit the budget
// (each chunk is one build; every slice's result is the same as in a build
// of all slices at once, as no step couples slices), merged into one handle.
static lrpr_status rsvd_build_impl(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices,
                                   const void *const *psi, int nsteps, int q, lrpr_prec range_prec,
                                   lrpr_coarse *out, double *sigma_host, int *fallback_host,
                                   const double *const *weights) {
    if (!ctx) return LRPR_ERR_ARG;
    if (nslices <= 0 || !slices || !out) return fail(ctx, LRPR_ERR_ARG, "lrpr_rsvd_build: invalid arguments");
    for (int s = 0; s < nslices; ++s)
        if (!slices[s].F) return fail(ctx, LRPR_ERR_ARG, "lrpr_rsvd_build: slice needs factor");
    const size_t esz = range_prec == LRPR_F32 ? sizeof(float) : sizeof(double);
    const double budget = ctx->tune_rsvd_budget ? (double)ctx->tune_rsvd_budget : 96e9;
    // panel bytes of a chunk: two arenas in the range finder's precision and
    // three in FP64, each n x (k+p) per slice
    std::vector<int> cut{0};
    double bytes = 0.0;
    for (int s = 0; s < nslices; ++s) {
        const double b = (double)slices[s].F->n * (slices[s].k + slices[s].p) * (2.0 * esz + 3.0 * 8.0);
        if (s > cut.back() && bytes + b > budget) {
            cut.push_back(s);
            bytes = 0.0;
        }
        bytes += b;
    }
    cut.push_back(nslices);
    if (cut.size() == 2)
        return rsvd_build_one(ctx, nslices, slices, psi, nsteps, q, range_prec, out, sigma_host, fallback_host,
                              weights);
    lrpr_coarse all = new (std::nothrow) lrpr_coarse_s();
    if (!all) return fail(ctx, LRPR_ERR_NOMEM, "coarse handle");
    all->dev = ctx->dev;
    size_t sig_at = 0;
    for (size_t ci = 0; ci + 1 < cut.size(); ++ci) {
        const int a = cut[ci], cnt = cut[ci + 1] - cut[ci];
        lrpr_coarse part = nullptr;
        lrpr_status st = rsvd_build_one(ctx, cnt, slices + a, psi ? psi + a : nullptr, nsteps, q, range_prec, &part,
                                        sigma_host ? sigma_host + sig_at : nullptr,
                                        fallback_host ? fallback_host + a : nullptr, weights ? weights + a : nullptr);
        if (st != LRPR_OK) {
            lrpr_coarse_destroy(all);
            return st;
        }
        all->nslices += part->nslices;
        all->n.insert(all->n.end(), part->n.begin(), part->n.end());
        all->k.insert(all->k.end(), part->k.begin(), part->k.end());
        all->l.insert(all->l.end(), part->l.begin(), part->l.end());
        all->U.insert(all->U.end(), part->U.begin(), part->U.end());
        all->S.insert(all->S.end(), part->S.begin(), part->S.end());
        all->V.insert(all->V.end(), part->V.begin(), part->V.end());
        all->sigma.insert(all->sigma.end(), part->sigma.begin(), part->sigma.end());
        all->F.insert(all->F.end(), part->F.begin(), part->F.end());
        sig_at += part->sigma.size();
        if (!all->block) all->block = part->block;
        else all->more.push_back(part->block);
        part->block = nullptr;
        part->U.clear();
        part->S.clear();
        part->V.clear();
        delete part;
    }
    *out = all;
    return LRPR_OK;
}

static lrpr_status rsvd_build_one(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices,
                                  const void *const *psi, int nsteps, int q, lrpr_prec range_prec,
                                  lrpr_coarse *out, double *sigma_host, int *fallback_host,
                                  const double *const *weights) {
    if (!ctx) return LRPR_ERR_ARG;
    if (nslices <= 0 || !slices || !out || nsteps < 0 || q < 0 ||
        (range_prec != LRPR_F64 && range_prec != LRPR_F32))
        return fail(ctx, LRPR_ERR_ARG, "lrpr_rsvd_build: invalid arguments");
    const bool f32 = range_prec == LRPR_F32;
    const size_t esz = f32 ? sizeof(float) : sizeof(double);
    int lmax = 1, kmax = 1;
    int64_t nmax = 1;
    for (int s = 0; s < nslices; ++s) {
        const lrpr_slice_desc &d = slices[s];
        const int l = d.k + d.p;
        if (!d.F || !d.Omega || d.k < 0 || d.p < 0 || l < 1 || l > LMAX || l > d.F->n)
            return fail(ctx, LRPR_ERR_ARG, "lrpr_rsvd_build: slice needs factor, Omega, 1 <= k+p <= min(96, n)");
        if (!(d.F->mask & (f32 ? LRPR_STORE_F32 : LRPR_STORE_F64)))
            return fail(ctx, LRPR_ERR_ARG, "lrpr_rsvd_build: factor lacks the copy in the range finder's precision");
        if (d.F->dev != ctx->dev) return fail(ctx, LRPR_ERR_ARG, "lrpr_rsvd_build: factor on another device");
        lmax = std::max(lmax, l);
        kmax = std::max(kmax, d.k);
        nmax = std::max(nmax, d.F->n);
    }
    CK(hipSetDevice(ctx->dev), "hipSetDevice");
    hipStream_t st = ctx->stream;
    Scoped mem(ctx, "rsvd");
    // offsets of every slice's n x l block in the tall arenas
    std::vector<int64_t> off(nslices + 1, 0);
    std::vector<int> ls(nslices);
    for (int s = 0; s < nslices; ++s) {
        ls[s] = slices[s].k + slices[s].p;
        off[s + 1] = off[s] + slices[s].F->n * ls[s];
    }
    const int64_t tot = off[nslices];
    // the five panel arenas, carved from the context's arena (the workspace
    // that the factorisation's bands and scratch used before)
    char *Y = nullptr, *Z = nullptr;
    double *Q = nullptr, *QZ = nullptr, *T2 = nullptr;
    {
        const size_t a1 = ((size_t)tot * esz + 255) / 256 * 256, a2 = ((size_t)tot * 8 + 255) / 256 * 256;
        hipError_t ea = hipSuccess;
        char *base = (char *)ws_get(ctx, "arena", 2 * a1 + 3 * a2, &ea);
        if (!base) return herr(ctx, ea == hipSuccess ? hipErrorOutOfMemory : ea, "rsvd panels");
        Y = base;
        Z = base + a1;
        Q = (double *)(base + 2 * a1);
        QZ = (double *)(base + 2 * a1 + a2);
        T2 = (double *)(base + 2 * a1 + 2 * a2);
    }
    const size_t SM = (size_t)LMAX * LMAX;
    double *G, *R1, *I1, *R2, *I2, *RY, *RZ, *Mm, *Uh, *Vh, *Sd, *part;
    int *d_ls, *stat1, *stat2, *sweeps;
    const int nchunks = gram_chunks(nmax);
    CK(mem.alloc(&G, SM * nslices), "G");
    CK(mem.alloc(&R1, SM * nslices), "R1");
    CK(mem.alloc(&I1, SM * nslices), "I1");
    CK(mem.alloc(&R2, SM * nslices), "R2");
    CK(mem.alloc(&I2, SM * nslices), "I2");
    CK(mem.alloc(&RY, SM * nslices), "RY");
    CK(mem.alloc(&RZ, SM * nslices), "RZ");
    CK(mem.alloc(&Mm, SM * nslices), "Mm");
    CK(mem.alloc(&Uh, SM * nslices), "Uh");
    CK(mem.alloc(&Vh, SM * nslices), "Vh");
    CK(mem.alloc(&Sd, (size_t)LMAX * nslices), "S");
    CK(mem.alloc(&part, SM * nslices * nchunks), "gram partials");
    CK(mem.alloc(&d_ls, nslices), "ls");
    CK(mem.alloc(&stat1, nslices), "stat1");
    CK(mem.alloc(&stat2, nslices), "stat2");
    CK(mem.alloc(&sweeps, nslices), "sweeps");
    CK(upload(d_ls, ls, st), "upload ls");

    // --- step 1: Y = T Omega (fine sweep without source) ------------------
    for (int s = 0; s < nslices; ++s)
        CK(hipMemcpyAsync((char *)Y + off[s] * esz, slices[s].Omega, (size_t)(off[s + 1] - off[s]) * esz,
                          hipMemcpyDeviceToDevice, st),
           "copy Omega");
    if (psi)   // two-sided: Z = Psi, swept with the adjoint below without waiting for Q
        for (int s = 0; s < nslices; ++s)
            CK(hipMemcpyAsync((char *)Z + off[s] * esz, psi[s], (size_t)(off[s + 1] - off[s]) * esz,
                              hipMemcpyDeviceToDevice, st),
               "copy Psi");
    // consecutive slices with the same factor form one panel (contiguous blocks)
    auto make_panels = [&](void *base) {
        std::vector<lrpr_panel> P;
        for (int s = 0; s < nslices; ++s) {
            if (!P.empty() && P.back().F == slices[s].F) {
                P.back().w += ls[s];
                continue;
            }
            lrpr_panel p{};
            p.F = slices[s].F;
            p.X = (char *)base + off[s] * esz;
            p.ldx = slices[s].F->n;
            p.w = ls[s];
            P.push_back(p);
        }
        return P;
    };
    // W^{+-1/2} row scaling of every weighted slice's block of an arena
    bool weighted = false;
    for (int s = 0; weights && s < nslices; ++s) weighted = weighted || weights[s];
    auto wscale = [&](void *base, bool up) -> hipError_t {
        for (int s = 0; weighted && s < nslices; ++s) {
            if (!weights[s]) continue;
            hipError_t he = launch_row_scale(f32, (char *)base + off[s] * esz, slices[s].F->n, ls[s], weights[s],
                                             up, st);
            if (he != hipSuccess) return he;
        }
        return hipSuccess;
    };
    // forward / adjoint sweep of the (transformed) operator on a panel arena
    auto fwd = [&](void *base) -> lrpr_status {
        if (hipError_t he = wscale(base, false); he != hipSuccess) return herr(ctx, he, "weights");
        std::vector<lrpr_panel> P = make_panels(base);
        lrpr_status rr = run_sweep(ctx, (int)P.size(), P.data(), nsteps, range_prec, false);
        if (rr != LRPR_OK) return rr;
        if (hipError_t he = wscale(base, true); he != hipSuccess) return herr(ctx, he, "weights");
        return LRPR_OK;
    };
    auto adj = [&](void *base) -> lrpr_status {
        if (hipError_t he = wscale(base, true); he != hipSuccess) return herr(ctx, he, "weights");
        std::vector<lrpr_panel> P = make_panels(base);
        lrpr_status rr = run_sweep(ctx, (int)P.size(), P.data(), nsteps, range_prec, true);
        if (rr != LRPR_OK) return rr;
        if (hipError_t he = wscale(base, false); he != hipSuccess) return herr(ctx, he, "weights");
        return LRPR_OK;
    };
    {
        lrpr_status r = fwd(Y);
        if (r != LRPR_OK) return r;
    }

    // --- CholeskyQR2 with Householder fallback ---------------------------
    std::vector<GramJob> gj(nslices);
    std::vector<RowMatJob> rj(nslices);
    GramJob *d_gj;
    RowMatJob *d_rj;
    HouseJob *d_hj;
    SignJob *d_sj;
    CK(mem.alloc(&d_gj, nslices), "jobs");
    CK(mem.alloc(&d_rj, nslices), "jobs");
    CK(mem.alloc(&d_hj, nslices), "jobs");
    CK(mem.alloc(&d_sj, nslices), "jobs");
    std::vector<int> fallback(nslices, 0);

    // orthonormalise A (T or FP64 arena) into Qout (FP64); R into Rout
    auto cholqr2 = [&](const void *A, bool a32, double *Qout, double *Rout) -> lrpr_status {
        for (int s = 0; s < nslices; ++s)
            gj[s] = GramJob{(const char *)A + off[s] * (a32 ? 4 : 8), slices[s].F->n, ls[s], 0};
        CK(upload(d_gj, gj, st), "upload");
        CK(launch_gram(a32, d_gj, nslices, nchunks, part, G, st), "gram 1");
        CK(launch_chol(d_ls, nslices, G, R1, I1, stat1, 2e-8, st), "chol 1");
        for (int s = 0; s < nslices; ++s)
            rj[s] = RowMatJob{(const char *)A + off[s] * (a32 ? 4 : 8), slices[s].F->n, I1 + SM * s,
                              T2 + off[s], slices[s].F->n, slices[s].F->n, ls[s], ls[s], 1, 0};
        CK(upload(d_rj, rj, st), "upload");
        CK(launch_rowmat(a32 ? 1 : 0, 0, d_rj, nslices, nmax, st), "Y Rinv");
        for (int s = 0; s < nslices; ++s) gj[s] = GramJob{T2 + off[s], slices[s].F->n, ls[s], 0};
        CK(upload(d_gj, gj, st), "upload");
        CK(launch_gram(false, d_gj, nslices, nchunks, part, G, st), "gram 2");
        CK(launch_chol(d_ls, nslices, G, R2, I2, stat2, 0.1, st), "chol 2");
        for (int s = 0; s < nslices; ++s)
            rj[s] = RowMatJob{T2 + off[s], slices[s].F->n, I2 + SM * s, Qout + off[s], slices[s].F->n,
                              slices[s].F->n, ls[s], ls[s], 1, 0};
        CK(upload(d_rj, rj, st), "upload");
        CK(launch_rowmat(0, 0, d_rj, nslices, nmax, st), "Q1 Rinv");
        CK(launch_trmm_upper(d_ls, nslices, R2, R1, Rout, st), "R2 R1");
        std::vector<int> h1(nslices), h2(nslices);
        CK(hipMemcpyAsync(h1.data(), stat1, sizeof(int) * nslices, hipMemcpyDeviceToHost, st), "stat");
        CK(hipMemcpyAsync(h2.data(), stat2, sizeof(int) * nslices, hipMemcpyDeviceToHost, st), "stat");
        CK(hipStreamSynchronize(st), "sync");
        std::vector<HouseJob> hj;
        for (int s = 0; s < nslices; ++s) {
            if (!h1[s] && !h2[s]) continue;
            fallback[s] = 1;
            // FP64 working copy of the panel in T2, Q into Qout, R into Rout
            const int64_t cnt = off[s + 1] - off[s];
            CK(launch_convert(a32 ? 1 : 0, 0, (const char *)A + off[s] * (a32 ? 4 : 8), T2 + off[s], cnt, st),
               "fallback copy");
            hj.push_back(HouseJob{T2 + off[s], Qout + off[s], Rout + SM * s, slices[s].F->n, ls[s], 0});
        }
        if (!hj.empty()) {
            CK(upload(d_hj, hj, st), "upload");
            CK(launch_householder(d_hj, (int)hj.size(), st), "householder");
        }
        return LRPR_OK;
    };

    lrpr_status r;
    // --- power iterations: Y <- T Qz with Qz = orth(T^T orth(Y)) ---------------
    for (int it = 0; it < q; ++it) {
        if ((r = cholqr2(Y, f32, Q, RY)) != LRPR_OK) return r;
        CK(launch_convert(0, f32 ? 1 : 0, Q, Z, tot, st), "Q -> Z");
        if ((r = adj(Z)) != LRPR_OK) return r;
        if ((r = cholqr2(Z, f32, QZ, RZ)) != LRPR_OK) return r;
        CK(launch_convert(0, f32 ? 1 : 0, QZ, Y, tot, st), "Qz -> Y");
        if ((r = fwd(Y)) != LRPR_OK) return r;
    }
    if (psi) {
        // --- two-sided: Z = T^T Psi; C = Psi^T Q; X^T = Z C^{-T}; X^T = Qx Rx ---
        if ((r = adj(Z)) != LRPR_OK) return r;
        if ((r = cholqr2(Y, f32, Q, RY)) != LRPR_OK) return r;
        double *ones, *Cg, *Bt, *lpart;
        int *stat3;
        CK(mem.alloc(&ones, LMAX), "ones");
        CK(mem.alloc(&Cg, SM * nslices), "Psi^T Q");
        CK(mem.alloc(&Bt, SM * nslices), "C^-T");
        CK(mem.alloc(&stat3, nslices), "status");
        CK(mem.alloc(&lpart, (size_t)lr_part_elems(nmax, lmax, lmax)), "cross Gram partials");
        CK(launch_fill(ones, LMAX, 1.0, st), "ones");
        // FP64 copy of Psi in T2 (the caller's Psi is untouched; Z holds T^T Psi)
        for (int s = 0; s < nslices; ++s) {
            CK(launch_convert(f32 ? 1 : 0, 0, psi[s], T2 + off[s], off[s + 1] - off[s], st), "Psi -> FP64");
            CK(launch_cross_gram(T2 + off[s], Q + off[s], slices[s].F->n, ls[s], ls[s], ones, lpart, Cg + SM * s,
                                 st),
               "Psi^T Q");
        }
        CK(launch_small_inv_t(d_ls, nslices, lmax, Cg, Bt, stat3, st), "(Psi^T Q)^-T");
        std::vector<int> h3(nslices);
        CK(hipMemcpyAsync(h3.data(), stat3, sizeof(int) * nslices, hipMemcpyDeviceToHost, st), "status");
        CK(hipStreamSynchronize(st), "sync");
        for (int s = 0; s < nslices; ++s)
            if (h3[s]) return fail(ctx, LRPR_ERR_QR_BREAKDOWN, "lrpr_rsvd_build_two_sided: Psi^T Q is singular");
        // X^T into Y (range precision, as Z in the one-sided build; Y is consumed)
        for (int s = 0; s < nslices; ++s)
            rj[s] = RowMatJob{(const char *)Z + off[s] * esz, slices[s].F->n, Bt + SM * s, (char *)Y + off[s] * esz,
                              slices[s].F->n, slices[s].F->n, ls[s], ls[s], 0, 0};
        CK(upload(d_rj, rj, st), "upload");
        CK(launch_rowmat(f32 ? 1 : 0, f32 ? 1 : 0, d_rj, nslices, nmax, st), "Z C^-T");
        if ((r = cholqr2(Y, f32, QZ, RZ)) != LRPR_OK) return r;
    } else {
        r = cholqr2(Y, f32, Q, RY);                    // step 2
        if (r != LRPR_OK) return r;
        // --- step 3: Z = T^T Q (adjoint sweep) -----------------------------
        CK(launch_convert(0, f32 ? 1 : 0, Q, Z, tot, st), "Q -> Z");
        if ((r = adj(Z)) != LRPR_OK) return r;
        r = cholqr2(Z, f32, QZ, RZ);                   // step 4
        if (r != LRPR_OK) return r;
    }
    // --- step 5: Mm = Rz^T, small SVD --------------------------------------
    CK(launch_transpose_small(d_ls, nslices, RZ, Mm, st), "Rz^T");
    CK(launch_jacobi(d_ls, nslices, lmax, Mm, Uh, Sd, Vh, sweeps, st), "jacobi");
    // --- step 6: U_k = Q Uh[:, :k], V_k = Qz Vh[:, :k] ---------------------
    lrpr_coarse c = new (std::nothrow) lrpr_coarse_s();
    if (!c) return fail(ctx, LRPR_ERR_NOMEM, "coarse handle");
    c->dev = ctx->dev;
    c->nslices = nslices;
    c->n.resize(nslices);
    c->k.resize(nslices);
    c->l.resize(nslices);
    c->U.assign(nslices, nullptr);
    c->V.assign(nslices, nullptr);
    c->S.assign(nslices, nullptr);
    c->F.resize(nslices);
    auto bail = [&](lrpr_status stt, const char *msg) {
        lrpr_coarse_destroy(c);
        return fail(ctx, stt, msg);
    };
    // every slice's U_k, V_k and S in one allocation (one device allocation
    // per build instead of three per slice)
    // (each array starts on a 256-byte boundary)
    auto pad = [](size_t e) { return (e + 31) / 32 * 32; };
    size_t elems = 0;
    for (int s = 0; s < nslices; ++s)
        elems += 2 * pad((size_t)slices[s].F->n * std::max(slices[s].k, 1)) + pad(LMAX);
    if (dmalloc((void **)&c->block, elems * sizeof(double), st) != hipSuccess)
        return bail(LRPR_ERR_NOMEM, "coarse factors");
    size_t at = 0;
    for (int s = 0; s < nslices; ++s) {
        c->n[s] = slices[s].F->n;
        c->k[s] = slices[s].k;
        c->l[s] = ls[s];
        c->F[s] = slices[s].F;
        const size_t nk = pad((size_t)c->n[s] * std::max(slices[s].k, 1));
        c->U[s] = c->block + at;
        c->V[s] = c->block + at + nk;
        c->S[s] = c->block + at + 2 * nk;
        at += 2 * nk + pad(LMAX);
        if (hipMemcpyAsync(c->S[s], Sd + (size_t)LMAX * s, LMAX * sizeof(double), hipMemcpyDeviceToDevice, st) !=
            hipSuccess)
            return bail(LRPR_ERR_HIP, "copy S");
    }
    for (int s = 0; s < nslices; ++s)
        rj[s] = RowMatJob{Q + off[s], c->n[s], Uh + SM * s, c->U[s], c->n[s], c->n[s], ls[s], slices[s].k, 0, 0};
    if (upload(d_rj, rj, st) != hipSuccess || launch_rowmat(0, 0, d_rj, nslices, nmax, st) != hipSuccess)
        return bail(LRPR_ERR_HIP, "U_k = Q Uh");
    for (int s = 0; s < nslices; ++s)
        rj[s] = RowMatJob{QZ + off[s], c->n[s], Vh + SM * s, c->V[s], c->n[s], c->n[s], ls[s], slices[s].k, 0, 0};
    if (upload(d_rj, rj, st) != hipSuccess || launch_rowmat(0, 0, d_rj, nslices, nmax, st) != hipSuccess)
        return bail(LRPR_ERR_HIP, "V_k = Qz Vh");
    for (int s = 0; weighted && s < nslices; ++s) {
        if (!weights[s]) continue;
        if (launch_row_scale(false, c->U[s], c->n[s], slices[s].k, weights[s], false, st) != hipSuccess ||
            launch_row_scale(false, c->V[s], c->n[s], slices[s].k, weights[s], true, st) != hipSuccess)
            return bail(LRPR_ERR_HIP, "weights");
    }
    std::vector<SignJob> sj(nslices);
    for (int s = 0; s < nslices; ++s) sj[s] = SignJob{c->U[s], c->V[s], c->n[s], slices[s].k, 0};
    if (upload(d_sj, sj, st) != hipSuccess || launch_signfix(d_sj, nslices, kmax, st) != hipSuccess)
        return bail(LRPR_ERR_HIP, "sign normalisation");
    std::vector<double> hs((size_t)LMAX * nslices);
    std::vector<int> hsw(nslices);
    if (hipMemcpyAsync(hs.data(), Sd, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(hsw.data(), sweeps, nslices * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return bail(LRPR_ERR_HIP, "rsvd readback");
    int pos = 0;
    for (int s = 0; s < nslices; ++s) {
        for (int j = 0; j < ls[s]; ++j) {
            const double v = hs[(size_t)LMAX * s + j];
            if (!std::isfinite(v)) return bail(LRPR_ERR_NONFINITE, "non-finite singular value");
            c->sigma.push_back(v);
            if (sigma_host) sigma_host[pos] = v;
            ++pos;
        }
        if (hsw[s] < 0) return bail(LRPR_ERR_NONFINITE, "Jacobi SVD did not converge");
    }
    if (fallback_host)
        for (int s = 0; s < nslices; ++s) fallback_host[s] = fallback[s];
    *out = c;
    return LRPR_OK;
}

extern "C" {

lrpr_status lrpr_coarse_apply(lrpr_ctx ctx, lrpr_coarse c, int s, int w, const double *Vin, double *Out) {
    if (!ctx) return LRPR_ERR_ARG;
    if (!c || s < 0 || s >= c->nslices || w < 0 || (w > 0 && (!Vin || !Out)))
        return fail(ctx, LRPR_ERR_ARG, "lrpr_coarse_apply: invalid arguments");
    if (w == 0) return LRPR_OK;
    CK(hipSetDevice(ctx->dev), "hipSetDevice");
    hipError_t e;
    const int k = c->k[s];
    double *part = (double *)ws_get(
        ctx, "lr_part", sizeof(double) * (size_t)lr_part_elems(c->n[s], k, std::min(w, std::max(1, 12288 / std::max(k, 1)))),
        &e);
    if (!part) return herr(ctx, e, "workspace");
    LrArgs a{};
    a.U = c->U[s]; a.S = c->S[s]; a.V = c->V[s];
    a.x = Vin; a.out = Out;
    a.n = c->n[s]; a.k = k; a.w = w; a.mode = 0;
    CK(lowrank_cols(a, part, nullptr, ctx->stream), "low-rank apply");
    return LRPR_OK;
}

// ---------------------------------------------------------------------------
// Parareal
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

// Device and host state of one problem of a Parareal solve.
struct PrState {
    lrpr_parareal_problem d;
    int N = 0, kcap = 0, nreq = 1;
    int64_t n = 0;
    size_t blk = 0;                // one slice's n x nreq block
    double *Ucur = nullptr, *Gold = nullptr, *Bv = nullptr;
    void *X = nullptr, *fsrc = nullptr;
    int *fcol = nullptr, *active = nullptr;
    double *fsc = nullptr, *part = nullptr, *incpart = nullptr, *inc2 = nullptr;
    int64_t nch = 0;
    std::vector<int> hact, iters, conv;
    std::vector<double> incr, last_inc, hinc;
    int nactive = 0;
};

}  // namespace

// Parareal (eq. def_Parareal) for several independent problems at once: the
// fine solves of an iteration (all problems, all slices, all requests) run
// as one batched sweep launch, then each problem's sequential coarse
// correction over its slices; problems may differ in grid, slice count,
// rank and requests.  The iteration (conversion of the iterates, the sweep
// and every problem's correction) is captured once in a HIP graph and
// replayed, when all factors use implicit Euler.
static lrpr_status parareal_impl(lrpr_ctx ctx, int nprob, const lrpr_parareal_problem *probs, int nsteps,
                                 lrpr_prec fine_prec) {
    if (!ctx) return LRPR_ERR_ARG;
    if (nprob < 1 || !probs || nsteps < 1 || (fine_prec != LRPR_F64 && fine_prec != LRPR_F32))
        return fail(ctx, LRPR_ERR_ARG, "lrpr_parareal_solve: invalid arguments");
    const bool f32 = fine_prec == LRPR_F32;
    const size_t esz = f32 ? 4 : 8;
    std::vector<PrState> ps(nprob);
    int stepper = -1;
    for (int p = 0; p < nprob; ++p) {
        const lrpr_parareal_problem &d = probs[p];
        if (!d.C || !d.F || d.nreq < 1 || !d.u0 || !d.U || !d.iters_host || d.max_iter < 1 || !(d.tol >= 0))
            return fail(ctx, LRPR_ERR_ARG, "lrpr_parareal_solve: invalid problem");
        const int N = d.C->nslices;
        const int64_t n = d.C->n[0];
        int kmax = 0;
        for (int s = 0; s < N; ++s) {
            if (!d.F[s] || d.F[s]->n != n || d.C->n[s] != n)
                return fail(ctx, LRPR_ERR_ARG, "lrpr_parareal_solve: a problem's slices must share one size n");
            if (stepper >= 0 && d.F[s]->stepper != stepper)
                return fail(ctx, LRPR_ERR_ARG, "lrpr_parareal_solve: slices must share one time stepper");
            stepper = d.F[s]->stepper;
            if ((f32 && !(d.F[s]->mask & LRPR_STORE_F32)) || (!f32 && !(d.F[s]->mask & LRPR_STORE_F64)))
                return fail(ctx, LRPR_ERR_ARG, "lrpr_parareal_solve: factor lacks the requested precision");
            if (d.F[s]->dev != ctx->dev) return fail(ctx, LRPR_ERR_ARG, "lrpr_parareal_solve: factor on another device");
            kmax = std::max(kmax, d.C->k[s]);
        }
        if ((size_t)kmax * d.nreq > 12288) return fail(ctx, LRPR_ERR_ARG, "lrpr_parareal_solve: k * nreq above 12288");
        PrState &q = ps[p];
        q.d = d;
        q.N = N;
        q.n = n;
        q.nreq = d.nreq;
        // iterations are capped at N (Parareal is exact there); max_iter
        // stays the row stride of incr_host
        q.kcap = std::min(d.max_iter, N);
        q.blk = (size_t)n * d.nreq;
        q.nch = lr_chunks(n);
        (void)kmax;
    }
    CK(hipSetDevice(ctx->dev), "hipSetDevice");
    hipStream_t st = ctx->stream;
    const int fs = fac_stages(probs[0].F[0]) * nsteps;   // source time factors per slice and column
    hipError_t e = hipSuccess;
    for (int p = 0; p < nprob; ++p) {
        PrState &q = ps[p];
        char key[48];
        auto W = [&](const char *name, size_t bytes) {
            snprintf(key, sizeof key, "pr%d_%s", p, name);
            return ws_get(ctx, key, bytes, &e);
        };
        int kmax = 0;
        for (int s = 0; s < q.N; ++s) kmax = std::max(kmax, q.d.C->k[s]);
        q.Ucur = (double *)W("u", sizeof(double) * q.blk * (q.N + 1));
        q.Gold = (double *)W("gold", sizeof(double) * q.blk * q.N);
        q.Bv = (double *)W("b", sizeof(double) * q.blk * q.N);
        q.X = W("x", esz * q.blk * q.N);
        q.fsrc = q.d.f ? W("f", esz * q.blk) : nullptr;
        q.fcol = (int *)W("fcol", sizeof(int) * (size_t)q.N * q.nreq);
        q.fsc = (double *)W("fsc", sizeof(double) * (size_t)q.N * q.nreq * fs);
        q.part = (double *)W("part", sizeof(double) * (size_t)lr_part_elems(q.n, kmax, q.nreq));
        q.incpart = (double *)W("incpart", sizeof(double) * (size_t)q.nch * q.nreq);
        q.inc2 = (double *)W("inc2", sizeof(double) * (size_t)q.N * q.nreq);
        q.active = (int *)W("active", sizeof(int) * q.nreq);
        if (e != hipSuccess || !q.Ucur || !q.Gold || !q.Bv || !q.X || !q.fcol || !q.fsc || !q.part || !q.incpart ||
            !q.inc2 || !q.active || (q.d.f && !q.fsrc))
            return herr(ctx, e == hipSuccess ? hipErrorOutOfMemory : e, "parareal workspace");
    }
    // per-column source index and time factors: column (slice s, request r)
    std::vector<lrpr_panel> P;
    for (int p = 0; p < nprob; ++p) {
        PrState &q = ps[p];
        const int N = q.N, nreq = q.nreq;
        std::vector<int> hfcol((size_t)N * nreq);
        std::vector<double> hfsc((size_t)N * nreq * fs, 1.0);
        std::vector<double> hphi;
        if (q.d.fscale) {
            hphi.resize((size_t)N * fs);
            CK(hipMemcpyAsync(hphi.data(), q.d.fscale, sizeof(double) * hphi.size(), hipMemcpyDeviceToHost, st),
               "fscale");
            CK(hipStreamSynchronize(st), "sync");
        }
        for (int s = 0; s < N; ++s)
            for (int r = 0; r < nreq; ++r) {
                hfcol[(size_t)s * nreq + r] = r;
                if (q.d.fscale)
                    for (int j = 0; j < fs; ++j) hfsc[((size_t)s * nreq + r) * fs + j] = hphi[(size_t)s * fs + j];
            }
        CK(upload(q.fcol, hfcol, st), "fcol");
        CK(upload(q.fsc, hfsc, st), "fscale");
        if (q.d.f) CK(launch_convert(0, f32 ? 1 : 0, q.d.f, q.fsrc, (int64_t)q.blk, st), "source copy");
        q.hact.assign(nreq, 1);
        CK(upload(q.active, q.hact, st), "active");
        q.nactive = nreq;
        q.iters.assign(nreq, 0);
        q.conv.assign(nreq, 0);
        q.incr.assign((size_t)nreq * q.d.max_iter, 0.0);
        q.last_inc.assign((size_t)N * nreq, 0.0);
        q.hinc.assign((size_t)N * nreq, 0.0);
        // panels: consecutive slices with the same factor share one panel
        const size_t first = P.size();
        for (int s = 0; s < N; ++s) {
            if (P.size() > first && P.back().F == q.d.F[s]) {
                P.back().w += nreq;
                continue;
            }
            lrpr_panel pn{};
            pn.F = q.d.F[s];
            pn.X = (char *)q.X + (size_t)s * q.blk * esz;
            pn.ldx = q.n;
            pn.w = nreq;
            pn.f = q.fsrc;
            pn.ldf = q.n;
            pn.fcol = q.fsrc ? q.fcol + (size_t)s * nreq : nullptr;
            pn.fscale = q.fsrc ? q.fsc + (size_t)s * nreq * fs : nullptr;
            P.push_back(pn);
        }
    }
    // b_n = F_n 0 (all problems in one sweep)
    for (PrState &q : ps) {
        if (f32) CK(launch_fillf((float *)q.X, (int64_t)q.blk * q.N, 0.0f, st), "zero");
        else CK(launch_fill((double *)q.X, (int64_t)q.blk * q.N, 0.0, st), "zero");
    }
    lrpr_status r = run_sweep(ctx, (int)P.size(), P.data(), nsteps, fine_prec, false, true);
    if (r != LRPR_OK) return r;
    // u^0: u^0_0 = u0, u^0_n = G_n' u^0_{n-1} + b_n
    for (PrState &q : ps) {
        CK(launch_convert(f32 ? 1 : 0, 0, q.X, q.Bv, (int64_t)q.blk * q.N, st), "b_n");
        CK(hipMemcpyAsync(q.Ucur, q.d.u0, sizeof(double) * q.blk, hipMemcpyDeviceToDevice, st), "u0");
        for (int s = 0; s < q.N; ++s) {
            LrArgs a{};
            a.U = q.d.C->U[s]; a.S = q.d.C->S[s]; a.V = q.d.C->V[s];
            a.x = q.Ucur + (size_t)s * q.blk;
            a.out = q.Ucur + (size_t)(s + 1) * q.blk;
            a.gold = q.Gold + (size_t)s * q.blk;
            a.bvec = q.Bv + (size_t)s * q.blk;
            a.active = q.active;
            a.n = q.n; a.k = q.d.C->k[s]; a.w = q.nreq; a.mode = 1;
            CK(lowrank_cols(a, q.part, nullptr, st), "coarse init");
        }
    }
    // one iteration's device work on stream cs: the fine solves of all
    // problems from u^k_{n-1}, then every problem's correction sweep (slice
    // by slice, the problems interleaved)
    int Nmax = 0;
    for (const PrState &q : ps) Nmax = std::max(Nmax, q.N);
    SweepPlan plan;
    const bool graph = stepper == LRPR_STEP_EULER && ctx->tune_pr_graph != 0;
    if (graph && (r = plan_sweep(ctx, (int)P.size(), P.data(), nsteps, fine_prec, false, true, "pr_it_", &plan)) !=
                     LRPR_OK)
        return r;
    auto iteration = [&](hipStream_t cs) -> lrpr_status {
        for (PrState &q : ps)
            CK(launch_convert(0, f32 ? 1 : 0, q.Ucur, q.X, (int64_t)q.blk * q.N, cs), "u -> X");
        if (graph) {
            CK(plan.run(cs), "fine sweep");
        } else {
            lrpr_status rr = run_sweep(ctx, (int)P.size(), P.data(), nsteps, fine_prec, false, true);
            if (rr != LRPR_OK) return rr;
        }
        for (int s = 0; s < Nmax; ++s)
            for (PrState &q : ps) {
                if (s >= q.N) continue;
                LrArgs a{};
                a.U = q.d.C->U[s]; a.S = q.d.C->S[s]; a.V = q.d.C->V[s];
                a.x = q.Ucur + (size_t)s * q.blk;
                a.out = q.Ucur + (size_t)(s + 1) * q.blk;
                a.gold = q.Gold + (size_t)s * q.blk;
                if (f32) a.fu32 = (const float *)q.X + (size_t)s * q.blk;
                else a.fu64 = (const double *)q.X + (size_t)s * q.blk;
                a.active = q.active;
                a.n = q.n; a.k = q.d.C->k[s]; a.w = q.nreq; a.mode = 2;
                CK(lowrank_cols(a, q.part, q.incpart, cs), "correction");
                CK(launch_inc_reduce(q.incpart, q.nch, q.nreq, q.inc2 + (size_t)s * q.nreq, cs), "increment");
            }
        return LRPR_OK;
    };
    hipGraphExec_t gexec = nullptr;
    hipGraph_t g = nullptr;
    hipStream_t cs = nullptr;
    auto release = [&]() {
        if (gexec) hipGraphExecDestroy(gexec);
        if (g) hipGraphDestroy(g);
        if (cs) hipStreamDestroy(cs);
        gexec = nullptr;
        g = nullptr;
        cs = nullptr;
    };
    if (graph) {
        // captured on a stream of its own (no work runs while capturing);
        // replayed on the context's stream
        if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed)) != hipSuccess) {
            release();
            return herr(ctx, e, "graph capture");
        }
        lrpr_status rr = iteration(cs);
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (rr != LRPR_OK) {
            release();
            return rr;
        }
        if (e2 != hipSuccess || (e2 = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0)) != hipSuccess) {
            release();
            return herr(ctx, e2, "graph instantiate");
        }
    }
    int kmax_all = 0;
    for (const PrState &q : ps) kmax_all = std::max(kmax_all, q.kcap);
    lrpr_status result = LRPR_OK;
    for (int k = 0; k < kmax_all; ++k) {
        bool any = false;
        for (const PrState &q : ps) any = any || q.nactive > 0;
        if (!any) break;
        if (graph) {
            if ((e = hipGraphLaunch(gexec, st)) != hipSuccess) {
                release();
                return herr(ctx, e, "graph launch");
            }
        } else if ((r = iteration(st)) != LRPR_OK) {
            return r;
        }
        for (PrState &q : ps)
            if ((e = hipMemcpyAsync(q.hinc.data(), q.inc2, sizeof(double) * q.hinc.size(), hipMemcpyDeviceToHost,
                                    st)) != hipSuccess)
                break;
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            release();
            return herr(ctx, e, "increments");
        }
        for (PrState &q : ps) {
            bool changed = false;
            for (int rq = 0; rq < q.nreq; ++rq) {
                if (!q.hact[rq]) continue;
                double mx = 0.0;
                bool finite = true;
                for (int s = 0; s < q.N; ++s) {
                    const double v = q.hinc[(size_t)s * q.nreq + rq];
                    q.last_inc[(size_t)s * q.nreq + rq] = std::sqrt(v);
                    finite = finite && std::isfinite(v);   // std::max would drop a NaN
                    mx = std::max(mx, v);
                }
                const double inc = std::sqrt(mx);
                if (!finite || !std::isfinite(inc)) {
                    release();
                    return fail(ctx, LRPR_ERR_NONFINITE, "non-finite Parareal increment");
                }
                q.incr[(size_t)rq * q.d.max_iter + k] = inc;
                q.iters[rq] = k + 1;
                if (inc < q.d.tol || k + 1 >= q.N) {
                    q.conv[rq] = 1;
                    q.hact[rq] = 0;
                    --q.nactive;
                    changed = true;
                } else if (k + 1 >= q.kcap) {
                    q.hact[rq] = 0;   // max_iter reached: stops without converging
                    --q.nactive;
                    changed = true;
                }
            }
            if (changed && q.nactive > 0 && (e = upload(q.active, q.hact, st)) != hipSuccess) {
                release();
                return herr(ctx, e, "active");
            }
        }
    }
    release();
    for (PrState &q : ps) {
        const int N = q.N;
        const int64_t n = q.n;
        // output layout: request r -> n x (N+1) block
        for (int rq = 0; rq < q.nreq; ++rq)
            CK(hipMemcpy2DAsync(q.d.U + (size_t)rq * n * (N + 1), sizeof(double) * n, q.Ucur + (size_t)rq * n,
                                sizeof(double) * q.blk, sizeof(double) * n, N + 1, hipMemcpyDeviceToDevice, st),
               "output");
        // a posteriori bound (eq. apost_bound) with delta = max sigma_1, eps = max sigma_{k+1}
        double delta = 0.0, eps = 0.0;
        bool have_eps = true;
        size_t pos = 0;
        for (int s = 0; s < N; ++s) {
            delta = std::max(delta, q.d.C->sigma[pos]);
            if (q.d.C->l[s] > q.d.C->k[s]) eps = std::max(eps, q.d.C->sigma[pos + q.d.C->k[s]]);
            else have_eps = false;
            pos += q.d.C->l[s];
        }
        for (int rq = 0; rq < q.nreq; ++rq) {
            q.d.iters_host[rq] = q.iters[rq];
            if (q.d.incr_host)
                for (int k = 0; k < q.d.max_iter; ++k)
                    q.d.incr_host[(size_t)rq * q.d.max_iter + k] = q.incr[(size_t)rq * q.d.max_iter + k];
            if (q.d.apost_host) {
                for (int nn = 1; nn <= N; ++nn) {
                    double sum = 0.0;
                    for (int m = 1; m < nn; ++m)
                        sum += std::pow(delta, nn - m - 1) * q.last_inc[(size_t)(m - 1) * q.nreq + rq];
                    q.d.apost_host[(size_t)rq * N + nn - 1] = have_eps ? eps * sum : NAN;
                }
            }
            if (!q.conv[rq]) result = LRPR_ERR_NOCONV;
        }
    }
    CK(hipStreamSynchronize(st), "sync");
    if (result != LRPR_OK) return fail(ctx, result, "Parareal did not reach tol within max_iter");
    return LRPR_OK;
}

extern "C" {

lrpr_status lrpr_parareal_solve(lrpr_ctx ctx, lrpr_coarse c, const lrpr_fac *F, int nsteps, lrpr_prec fine_prec,
                                int nreq, const double *u0, const double *f, const double *fscale, double tol,
                                int max_iter, double *U, int *iters_host, double *incr_host, double *apost_host) {
    if (!ctx) return LRPR_ERR_ARG;
    lrpr_parareal_problem p{};
    p.C = c;
    p.F = F;
    p.nreq = nreq;
    p.u0 = u0;
    p.f = f;
    p.fscale = fscale;
    p.tol = tol;
    p.max_iter = max_iter;
    p.U = U;
    p.iters_host = iters_host;
    p.incr_host = incr_host;
    p.apost_host = apost_host;
    return parareal_impl(ctx, 1, &p, nsteps, fine_prec);
}

lrpr_status lrpr_parareal_solve_many(lrpr_ctx ctx, int nprob, const lrpr_parareal_problem *probs, int nsteps,
                                     lrpr_prec fine_prec) {
    return parareal_impl(ctx, nprob, probs, nsteps, fine_prec);
}

}  // extern "C"

namespace lrpr {

void *ws_get(lrpr_ctx ctx, const char *key, size_t bytes, hipError_t *err) {
    auto &slot = ctx->ws[key];
    if (slot.second >= bytes && slot.first) return slot.first;
    if (slot.first) {
        hipStreamSynchronize(ctx->stream);
        hipFree(slot.first);
        slot = {nullptr, 0};
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
    if (e == hipErrorOutOfMemory) {   // give the kept handle blocks back and try once more
        lrpr_device_trim(ctx->dev);
        hipSetDevice(ctx->dev);
        e = hipMalloc(&p, bytes ? bytes : 16);
    }
    if (e != hipSuccess) {
        if (err) *err = e;
        return nullptr;
    }
    slot = {p, bytes};
    return p;
}

}  // namespace lrpr
