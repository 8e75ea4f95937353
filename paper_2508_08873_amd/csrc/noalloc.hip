// Coarse apply without device allocation: lrpr_coarse_apply_noalloc.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).  The
// low-rank apply G_n' v = U_k (S_k .* (V_k^T v)) needs a scratch buffer for
// its chunk partials and coefficients; here it is a file-scope device array
// of fixed size, one per GPU, held until the process ends.  Its device
// address is looked up once per device with hipGetSymbolAddress (at context
// creation, with that device current) and only that address is handed to
// kernels: in host code the array's name is not a device address.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "dense.h"
#include "lrpr_internal.h"

namespace {

constexpr size_t SCRATCH_DOUBLES = (size_t)16 << 17;   // 16 MiB
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

std::mutex g_mutex;
double *g_ptr[MAX_DEVICES] = {};

}  // namespace

namespace lrpr {

// Device address of this device's scratch array; the device must be
// current.  Looked up once per device.
hipError_t noalloc_scratch_init(int dev, double **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = (double *)p;
    }
    if (out) *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace lrpr

using namespace lrpr;

extern "C" {

lrpr_status lrpr_coarse_apply_noalloc(lrpr_ctx ctx, lrpr_coarse c, int s, int w, const double *Vin, double *Out) {
    if (!ctx) return LRPR_ERR_ARG;
    if (!c || s < 0 || s >= c->nslices || w < 0 || (w > 0 && (!Vin || !Out)) || c->dev != ctx->dev)
        return fail(ctx, LRPR_ERR_ARG, "lrpr_coarse_apply_noalloc: invalid arguments");
    if (w == 0) return LRPR_OK;
    const int k = c->k[s];
    const int64_t n = c->n[s];
    const int pass_w = std::min(w, std::max(1, 12288 / std::max(k, 1)));
    const int64_t need = lr_part_elems(n, k, pass_w);
    if ((size_t)need > SCRATCH_DOUBLES)
        return fail(ctx, LRPR_ERR_ARG,
                    "lrpr_coarse_apply_noalloc: scratch of " + std::to_string(need) + " doubles needed, " +
                        std::to_string(SCRATCH_DOUBLES) + " available (n, k or w too large)");
    hipError_t e = hipSetDevice(ctx->dev);
    double *part = nullptr;
    if (e == hipSuccess) e = noalloc_scratch_init(ctx->dev, &part);
    if (e != hipSuccess)
        return fail(ctx, LRPR_ERR_HIP, std::string("lrpr_coarse_apply_noalloc: ") + hipGetErrorString(e));
    LrArgs a{};
    a.U = c->U[s];
    a.S = c->S[s];
    a.V = c->V[s];
    a.x = Vin;
    a.out = Out;
    a.n = n;
    a.k = k;
    a.w = w;
    a.mode = 0;
    if ((e = lowrank_cols(a, part, nullptr, ctx->stream)) != hipSuccess)
        return fail(ctx, LRPR_ERR_HIP, std::string("lrpr_coarse_apply_noalloc: ") + hipGetErrorString(e));
    return LRPR_OK;
}

}  // extern "C"
