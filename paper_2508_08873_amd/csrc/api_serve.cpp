// Host side of the C ABI: a serving loop for Parareal solves with the
// low-rank coarse propagators (continuous batching).
//
// The coarse propagators G_n = U_k S_k V_k^T + b_n do not depend on the
// source term except through b_n = F_n 0 (eq. F_n_affine, eq. spectral_G), so
// the device-resident U_k, S_k, V_k of an operator serve every request that
// brings a new initial value u0 and source f.  Each request runs the Parareal
// iteration of eq. def_Parareal on its own; the server batches the work of
// all requests of an operator into one fine-propagator launch and one coarse
// sweep per step:
//
//   step of operator o (one HIP stream per operator):
//     admit queued requests of o while their state fits the byte budget;
//     X_r = 0 (new requests: b_n)  or  X_r[:,s] = u^k_s (running requests);
//     one batched fine sweep over the columns of every request (with its f);
//     for s = 1..N: coarse apply to all columns at once, per column either
//       u^0_s = G'_s u^0_{s-1} + b_s            (new requests), or
//       u^{k+1}_s = F_s u^k_{s-1} + G'_s u^{k+1}_{s-1} - G'_s u^k_{s-1};
//     increments max_s ||u^{k+1}_s - u^k_s|| to the host; requests below the
//     tolerance (or at k = N, where Parareal is exact) complete.
//
// Requests that arrive while a step is on the GPU join the next step of
// their operator.  Operators step independently, on their own streams, so a
// small operator is not held back by a large one.  Every column's arithmetic
// is independent of the other columns in the batch, so a request's result is
// the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "dense.h"
#include "lrpr_internal.h"

namespace lrpr {
void *ws_get(lrpr_ctx ctx, const char *key, size_t bytes, hipError_t *err);
}  // namespace lrpr

using namespace lrpr;

namespace {

struct Req {
    int64_t id;
    int op;
    const double *u0, *f;
    double *U;      // caller's n x (N+1) iterate (column s = u_s)
    double *gold;   // G'_s u_{s-1} of the previous sweep (n x N), server-owned
    double *X;      // fine-sweep panel (n x N), server-owned
    int k;          // completed iterations (0 = only u^0)
    bool init;      // u^0 not formed yet
};

struct Pipe {
    lrpr_serve_op d{};
    std::vector<lrpr_fac> F;       // slice factors (copied from d.F at create time)
    int N = 0;
    int64_t n = 0;
    int kmax = 0;
    int cap = 0;                   // max concurrent requests (k * cap fits the coarse kernel)
    size_t req_bytes = 0;
    hipStream_t stream = nullptr;
    lrpr_ctx ctx = nullptr;        // sweep items and workspaces of this pipeline
    std::deque<Req *> queue;
    std::vector<Req *> act;        // columns of the current step
    bool inflight = false;
    hipEvent_t ev = nullptr;
    double **d_cu = nullptr, **d_cgold = nullptr;
    const double **d_cfu = nullptr;
    int *d_cmode = nullptr;
    int *d_fcol = nullptr;         // N zeros: every panel column reads source column 0
    double *d_fsc = nullptr;       // N x nsteps time factors (owned copy)
    double *d_inc2 = nullptr;      // N x cap squared increments
    double *h_inc2 = nullptr;      // pinned host copy
    std::vector<double *> h_cu, h_cgold;
    std::vector<const double *> h_cfu;
    std::vector<int> h_cmode;
};

}  // namespace

struct lrpr_server_s {
    lrpr_ctx ctx = nullptr;
    int dev = 0;
    double tol = 0.0;
    size_t budget = 0, used = 0;
    int64_t next_id = 1;
    std::vector<Pipe> pipes;
    std::vector<std::pair<int64_t, int>> done;   // completed (id, iterations; -1 on failure)
    std::string err;
};

namespace {

lrpr_status sfail(lrpr_server s, lrpr_status st, const std::string &msg) {
    if (s) s->err = msg;
    if (s && s->ctx) fail(s->ctx, st, msg);
    return st;
}

#define SCK(call, what)                                                                                  \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess)                                                                            \
            return sfail(srv, e_ == hipErrorOutOfMemory ? LRPR_ERR_NOMEM : LRPR_ERR_HIP,                 \
                         std::string(what) + ": " + hipGetErrorString(e_));                              \
    } while (0)

void free_pipe(Pipe &p) {
    if (p.stream) hipStreamSynchronize(p.stream);
    for (Req *r : p.act) {
        if (r->gold) hipFree(r->gold);
        if (r->X) hipFree(r->X);
        delete r;
    }
    for (Req *r : p.queue) delete r;
    p.act.clear();
    p.queue.clear();
    void *ptrs[] = {p.d_cu, p.d_cgold, p.d_cfu, p.d_cmode, p.d_fcol, p.d_fsc, p.d_inc2};
    for (void *q : ptrs)
        if (q) hipFree(q);
    if (p.h_inc2) hipHostFree(p.h_inc2);
    if (p.ev) hipEventDestroy(p.ev);
    if (p.ctx) lrpr_ctx_destroy(p.ctx);
    if (p.stream) hipStreamDestroy(p.stream);
}

// Launch one step of pipeline p (admission, fine sweep, coarse sweep,
// increment read-back).  Called when p has no step in flight.
lrpr_status launch_step(lrpr_server srv, Pipe &p) {
    hipStream_t st = p.stream;
    // admission by footprint (FIFO per operator)
    while (!p.queue.empty() && (int)p.act.size() < p.cap && srv->used + p.req_bytes <= srv->budget) {
        Req *r = p.queue.front();
        SCK(hipMallocAsync((void **)&r->gold, sizeof(double) * (size_t)p.n * p.N, st), "request state");
        SCK(hipMallocAsync((void **)&r->X, sizeof(double) * (size_t)p.n * p.N, st), "request state");
        SCK(hipMemcpyAsync(r->U, r->u0, sizeof(double) * (size_t)p.n, hipMemcpyDeviceToDevice, st), "u0");
        p.queue.pop_front();
        srv->used += p.req_bytes;
        p.act.push_back(r);
    }
    if (p.act.empty()) return LRPR_OK;
    const int w = (int)p.act.size();
    const size_t blk = (size_t)p.n * p.N;
    // fine-sweep start states and panels (runs of slices sharing a factor)
    std::vector<lrpr_panel> panels;
    for (Req *r : p.act) {
        if (r->init) SCK(launch_fill(r->X, (int64_t)blk, 0.0, st), "zero start");
        else SCK(hipMemcpyAsync(r->X, r->U, sizeof(double) * blk, hipMemcpyDeviceToDevice, st), "start states");
        for (int s = 0; s < p.N;) {
            int e = s + 1;
            while (e < p.N && p.F[e] == p.F[s]) ++e;
            lrpr_panel q{};
            q.F = p.F[s];
            q.X = r->X + (size_t)s * p.n;
            q.ldx = p.n;
            q.w = e - s;
            q.f = r->f;
            q.ldf = p.n;
            q.fcol = p.d_fcol + s;
            q.fscale = p.d_fsc + (size_t)s * p.d.nsteps;
            panels.push_back(q);
            s = e;
        }
    }
    lrpr_status rs = run_sweep(p.ctx, (int)panels.size(), panels.data(), p.d.nsteps, LRPR_F64, false, true);
    if (rs != LRPR_OK) return sfail(srv, rs, std::string("serve sweep: ") + lrpr_last_error(p.ctx));
    // column tables of the coarse sweep
    p.h_cu.resize(w);
    p.h_cgold.resize(w);
    p.h_cfu.resize(w);
    p.h_cmode.resize(w);
    for (int c = 0; c < w; ++c) {
        p.h_cu[c] = p.act[c]->U;
        p.h_cgold[c] = p.act[c]->gold;
        p.h_cfu[c] = p.act[c]->X;
        p.h_cmode[c] = p.act[c]->init ? 1 : 2;
    }
    SCK(hipMemcpyAsync(p.d_cu, p.h_cu.data(), sizeof(double *) * w, hipMemcpyHostToDevice, st), "tables");
    SCK(hipMemcpyAsync(p.d_cgold, p.h_cgold.data(), sizeof(double *) * w, hipMemcpyHostToDevice, st), "tables");
    SCK(hipMemcpyAsync(p.d_cfu, p.h_cfu.data(), sizeof(double *) * w, hipMemcpyHostToDevice, st), "tables");
    SCK(hipMemcpyAsync(p.d_cmode, p.h_cmode.data(), sizeof(int) * w, hipMemcpyHostToDevice, st), "tables");
    const int64_t nch = lr_chunks(p.n);
    hipError_t he = hipSuccess;
    double *part = (double *)ws_get(p.ctx, "sv_part", sizeof(double) * (size_t)lr_part_elems(p.n, p.kmax, p.cap), &he);
    double *incpart = (double *)ws_get(p.ctx, "sv_incpart", sizeof(double) * (size_t)nch * p.cap, &he);
    if (!part || !incpart) SCK(he == hipSuccess ? hipErrorOutOfMemory : he, "serve workspace");
    lrpr_coarse C = p.d.C;
    for (int s = 0; s < p.N; ++s) {
        LrArgs a{};
        a.U = C->U[s];
        a.S = C->S[s];
        a.V = C->V[s];
        a.n = p.n;
        a.k = C->k[s];
        a.w = w;
        a.mode = 2;
        a.part = part;
        a.incpart = incpart;
        a.cu = p.d_cu;
        a.cgold = p.d_cgold;
        a.cfu = p.d_cfu;
        a.cmode = p.d_cmode;
        a.coff = (int64_t)s * p.n;
        SCK(launch_lowrank(a, st), "coarse sweep");
        SCK(launch_inc_reduce(incpart, nch, w, p.d_inc2 + (size_t)s * w, st), "increments");
    }
    SCK(hipMemcpyAsync(p.h_inc2, p.d_inc2, sizeof(double) * (size_t)p.N * w, hipMemcpyDeviceToHost, st), "increments");
    SCK(hipEventRecord(p.ev, st), "event");
    p.inflight = true;
    return LRPR_OK;
}

// The step of p has finished: advance every column's request.
void finish_step(lrpr_server srv, Pipe &p) {
    const int w = (int)p.act.size();
    std::vector<Req *> keep;
    for (int c = 0; c < w; ++c) {
        Req *r = p.act[c];
        if (r->init) {
            r->init = false;
            keep.push_back(r);
            continue;
        }
        double mx = 0.0;
        bool finite = true;
        for (int s = 0; s < p.N; ++s) {
            const double v = p.h_inc2[(size_t)s * w + c];
            finite = finite && std::isfinite(v);
            mx = std::max(mx, v);
        }
        r->k += 1;
        if (!finite || std::sqrt(mx) < srv->tol || r->k >= p.N) {
            hipFreeAsync(r->gold, p.stream);
            hipFreeAsync(r->X, p.stream);
            srv->used -= p.req_bytes;
            srv->done.emplace_back(r->id, finite ? r->k : -1);
            delete r;
        } else {
            keep.push_back(r);
        }
    }
    p.act.swap(keep);
    p.inflight = false;
}

}  // namespace

extern "C" {

lrpr_status lrpr_server_create(lrpr_ctx ctx, int nops, const lrpr_serve_op *ops, double tol, size_t budget_bytes,
                               int max_active_per_op, lrpr_server *out) {
    if (!ctx) return LRPR_ERR_ARG;
    if (nops < 1 || !ops || !out || !(tol >= 0) || budget_bytes == 0)
        return fail(ctx, LRPR_ERR_ARG, "lrpr_server_create: invalid arguments");
    for (int o = 0; o < nops; ++o) {
        const lrpr_serve_op &d = ops[o];
        if (!d.C || !d.F || d.nsteps < 1 || d.C->nslices < 1)
            return fail(ctx, LRPR_ERR_ARG, "lrpr_server_create: operator without coarse propagators or factors");
        for (int s = 0; s < d.C->nslices; ++s)
            if (!d.F[s] || d.F[s]->n != d.C->n[0] || d.C->n[s] != d.C->n[0] || !(d.F[s]->mask & LRPR_STORE_F64) ||
                d.F[s]->dev != ctx->dev)
                return fail(ctx, LRPR_ERR_ARG, "lrpr_server_create: slice factors must share n and keep FP64 tiles");
        for (int s = 0; s < d.C->nslices; ++s)
            if (d.F[s]->stepper != LRPR_STEP_EULER)
                return fail(ctx, LRPR_ERR_ARG, "lrpr_server_create: served operators use implicit-Euler factors");
    }
    lrpr_server srv = new (std::nothrow) lrpr_server_s();
    if (!srv) return fail(ctx, LRPR_ERR_NOMEM, "lrpr_server_create: host allocation");
    srv->ctx = ctx;
    srv->dev = ctx->dev;
    srv->tol = tol;
    srv->budget = budget_bytes;
    srv->pipes.resize(nops);
    auto bail = [&](lrpr_status st, const std::string &m) {
        for (Pipe &p : srv->pipes) free_pipe(p);
        delete srv;
        return fail(ctx, st, m);
    };
    if (hipSetDevice(ctx->dev) != hipSuccess) return bail(LRPR_ERR_HIP, "hipSetDevice");
    {
        // keep freed request state in the stream-ordered pool between steps
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, ctx->dev) == hipSuccess) {
            uint64_t keep = UINT64_MAX;
            hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        }
    }
    for (int o = 0; o < nops; ++o) {
        Pipe &p = srv->pipes[o];
        p.d = ops[o];
        p.N = p.d.C->nslices;
        p.F.assign(p.d.F, p.d.F + p.N);
        p.d.F = nullptr;
        p.n = p.d.C->n[0];
        for (int s = 0; s < p.N; ++s) p.kmax = std::max(p.kmax, p.d.C->k[s]);
        p.cap = std::max(1, 12288 / std::max(p.kmax, 1));
        if (max_active_per_op > 0) p.cap = std::min(p.cap, max_active_per_op);
        p.req_bytes = 2 * sizeof(double) * (size_t)p.n * p.N;
        hipError_t e;
        if ((e = hipStreamCreate(&p.stream)) != hipSuccess) return bail(LRPR_ERR_HIP, "stream");
        if (lrpr_ctx_create(ctx->dev, p.stream, &p.ctx) != LRPR_OK) return bail(LRPR_ERR_HIP, "pipeline context");
        if ((e = hipEventCreateWithFlags(&p.ev, hipEventDisableTiming)) != hipSuccess) return bail(LRPR_ERR_HIP, "event");
        if (hipMalloc(&p.d_cu, sizeof(double *) * p.cap) != hipSuccess ||
            hipMalloc(&p.d_cgold, sizeof(double *) * p.cap) != hipSuccess ||
            hipMalloc(&p.d_cfu, sizeof(double *) * p.cap) != hipSuccess ||
            hipMalloc(&p.d_cmode, sizeof(int) * p.cap) != hipSuccess ||
            hipMalloc(&p.d_fcol, sizeof(int) * p.N) != hipSuccess ||
            hipMalloc(&p.d_fsc, sizeof(double) * (size_t)p.N * p.d.nsteps) != hipSuccess ||
            hipMalloc(&p.d_inc2, sizeof(double) * (size_t)p.N * p.cap) != hipSuccess ||
            hipHostMalloc(&p.h_inc2, sizeof(double) * (size_t)p.N * p.cap, hipHostMallocDefault) != hipSuccess)
            return bail(LRPR_ERR_NOMEM, "lrpr_server_create: pipeline buffers");
        if (hipMemsetAsync(p.d_fcol, 0, sizeof(int) * p.N, p.stream) != hipSuccess)
            return bail(LRPR_ERR_HIP, "source columns");
        if (p.d.fscale) {
            if (hipMemcpyAsync(p.d_fsc, p.d.fscale, sizeof(double) * (size_t)p.N * p.d.nsteps, hipMemcpyDeviceToDevice,
                               p.stream) != hipSuccess)
                return bail(LRPR_ERR_HIP, "time factors");
        } else if (launch_fill(p.d_fsc, (int64_t)p.N * p.d.nsteps, 1.0, p.stream) != hipSuccess) {
            return bail(LRPR_ERR_HIP, "time factors");
        }
        if (hipStreamSynchronize(p.stream) != hipSuccess) return bail(LRPR_ERR_HIP, "sync");
    }
    *out = srv;
    return LRPR_OK;
}

void lrpr_server_destroy(lrpr_server srv) {
    if (!srv) return;
    hipSetDevice(srv->dev);
    for (Pipe &p : srv->pipes) free_pipe(p);
    delete srv;
}

lrpr_status lrpr_server_submit(lrpr_server srv, int op, const double *u0, const double *f, double *U, int64_t *id) {
    if (!srv) return LRPR_ERR_ARG;
    if (op < 0 || op >= (int)srv->pipes.size() || !u0 || !f || !U || !id)
        return sfail(srv, LRPR_ERR_ARG, "lrpr_server_submit: invalid arguments");
    Pipe &p = srv->pipes[op];
    if (p.req_bytes > srv->budget) return sfail(srv, LRPR_ERR_NOMEM, "lrpr_server_submit: request exceeds the budget");
    Req *r = new (std::nothrow) Req();
    if (!r) return sfail(srv, LRPR_ERR_NOMEM, "lrpr_server_submit: host allocation");
    r->id = srv->next_id++;
    r->op = op;
    r->u0 = u0;
    r->f = f;
    r->U = U;
    r->gold = r->X = nullptr;
    r->k = 0;
    r->init = true;
    p.queue.push_back(r);
    *id = r->id;
    return LRPR_OK;
}

lrpr_status lrpr_server_progress(lrpr_server srv, int wait, int max_done, int64_t *done_ids, int *done_iters,
                                 int *ndone) {
    if (!srv) return LRPR_ERR_ARG;
    if (!ndone || max_done < 0 || (max_done > 0 && (!done_ids || !done_iters)))
        return sfail(srv, LRPR_ERR_ARG, "lrpr_server_progress: invalid arguments");
    SCK(hipSetDevice(srv->dev), "hipSetDevice");
    for (;;) {
        bool any_inflight = false, progressed = false;
        for (Pipe &p : srv->pipes) {
            if (p.inflight) {
                hipError_t q = hipEventQuery(p.ev);
                if (q == hipSuccess) {
                    finish_step(srv, p);
                    progressed = true;
                } else if (q != hipErrorNotReady) {
                    SCK(q, "serve step");
                } else {
                    any_inflight = true;
                }
            }
            if (!p.inflight && (!p.act.empty() || !p.queue.empty())) {
                lrpr_status st = launch_step(srv, p);
                if (st != LRPR_OK) return st;
                any_inflight = any_inflight || p.inflight;
            }
        }
        if (!wait || progressed || !any_inflight || !srv->done.empty()) break;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    const int nd = std::min<int>(max_done, (int)srv->done.size());
    for (int i = 0; i < nd; ++i) {
        done_ids[i] = srv->done[i].first;
        done_iters[i] = srv->done[i].second;
    }
    srv->done.erase(srv->done.begin(), srv->done.begin() + nd);
    *ndone = nd;
    return LRPR_OK;
}

lrpr_status lrpr_server_stats(lrpr_server srv, int *queued, int *active, int64_t *bytes_in_use) {
    if (!srv) return LRPR_ERR_ARG;
    int q = 0, a = 0;
    for (Pipe &p : srv->pipes) {
        q += (int)p.queue.size();
        a += (int)p.act.size();
    }
    if (queued) *queued = q;
    if (active) *active = a;
    if (bytes_in_use) *bytes_in_use = (int64_t)srv->used;
    return LRPR_OK;
}

const char *lrpr_server_last_error(lrpr_server srv) { return srv ? srv->err.c_str() : "null server"; }

}  // extern "C"
