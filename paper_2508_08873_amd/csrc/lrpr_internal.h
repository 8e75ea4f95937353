// Internal declarations of the lrpr library (HIP, gfx950).  Not part of the
// public ABI (include/lrpr.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "lrpr.h"

namespace lrpr {

// ---------------------------------------------------------------------------
// Tiled band storage of the LU factors, used by the sweep kernels.
//
// The unknowns are cut into tile rows of 16 (NT = ceil(n/16)); the band of
// half-width b spans nb = ceil(b/16) tiles on each side of the diagonal.
//   Lb[I][j]  = L(I, I-nb+j),  j = 0..nb-1   (strictly-left band tiles of L)
//   Ub[I][j]  = U(I, I+1+j),   j = 0..nb-1   (strictly-right band tiles of U)
//   DL[I]     = inverse of the unit lower triangular diagonal tile L(I,I)
//   DU[I]     = inverse of the upper triangular diagonal tile U(I,I)
//   DLT[I], DUT[I] = transposes of DL[I], DU[I] (adjoint sweeps)
// Tiles outside the matrix are zero; the diagonal tiles of the padded rows
// beyond n are the identity.  Each tile has 256 elements.
//
// Band tiles use a 4x4 sub-block layout: element (r, c) at
//   ((c/4)*4 + r/4)*16 + (r%4)*4 + c%4,
// so that both the tile and its transpose load as MFMA A operands with
// whole 4x4 sub-blocks per cache line.
// Diagonal (D*) tiles are stored pre-arranged as MFMA A operands: chunk kc of
// lane l at [kc*64 + l] (the k index of that slot depends on the precision,
// see tiles.hip).
// ---------------------------------------------------------------------------
constexpr int TILE = 16;
constexpr int TILE_ELEMS = 256;
// zero tile rows kept before and after every tile array (beyond the band and
// the sweep's prefetch window, reads land on zeros)
inline int guard_rows(int nb) { return nb + 8; }

struct TileSet {            // device arrays of one precision (pointers to tile row 0)
    void *Lb = nullptr, *Ub = nullptr;
    void *DL = nullptr, *DU = nullptr, *DLT = nullptr, *DUT = nullptr;
    void *EL = nullptr, *EU = nullptr, *ELT = nullptr, *EUT = nullptr;
    void *zt = nullptr;    // one all-zero tile: target of loads outside the band
    void *sink = nullptr;  // one scratch tile: target of masked-off stores
    void *alloc[10] = {};  // allocations behind Lb..EUT (they start guard rows earlier)
};

// Device-side view of one factor, passed by value to the sweep kernels.
struct FacView {
    const void *Lb, *Ub, *DL, *DU, *DLT, *DUT, *EL, *EU, *ELT, *EUT, *zt;
    void *sink;
    int n, NT, nb;
    double dt;
};

// One work item of a sweep launch: up to 16 right-hand sides sharing a factor.
struct SweepItem {
    FacView fac;
    void *X;               // first column of the group
    int64_t ldx;
    int ncols;             // 1..16
    int pad_;
    const void *f;         // sources (element type of the sweep) or null
    int64_t ldf;
    const int *fcol;       // per column (offset to the group's first column) or null
    const double *fscale;  // per column x nsteps (offset) or null
};

}  // namespace lrpr

struct lrpr_factor_s {
    int dev = 0;
    lrpr_op_desc op{};
    int64_t n = 0;
    int bw = 0;
    int NT = 0, nb = 0;
    int mask = 0;
    double *lu = nullptr;          // FP64 band LU, n x (2bw+1) row-major (kept with mask bit 0)
    lrpr::TileSet t64, t32;
};

struct lrpr_coarse_s {
    int dev = 0;
    int nslices = 0;
    std::vector<int64_t> n;
    std::vector<int> k, l;
    std::vector<double *> U, S, V;  // device, per slice
    std::vector<double> sigma;      // host copy of all singular values, per slice
    std::vector<lrpr_fac> F;     // factors the slices were built from (not owned)
};

struct lrpr_ctx_s {
    int dev = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // scratch for sweep work-item arrays
    lrpr::SweepItem *d_items = nullptr;
    size_t items_cap = 0;
    // sweep timing records (lrpr_profile_enable)
    struct ProfRec {
        hipEvent_t a, b;
        double flops, bytes, rhs_steps;
    };
    bool prof = false;
    std::vector<ProfRec> prof_recs;
    // device workspaces cached by purpose (grown on demand, freed on destroy)
    std::map<std::string, std::pair<void *, size_t>> ws;
};

namespace lrpr {

// error helper: record message in ctx and return status
lrpr_status fail(lrpr_ctx ctx, lrpr_status st, const std::string &msg);

// kernels launched from the host code (defined in the .hip sources)
hipError_t launch_assemble(const lrpr_op_desc &op, int64_t n, int bw, double *band, hipStream_t s);
hipError_t launch_band_lu(int64_t n, int bw, double *band, int *info, hipStream_t s);
hipError_t launch_pack_tiles(int64_t n, int bw, int NT, int nb, const double *lu, const TileSet *t64,
                             const TileSet *t32, double *scratch, hipStream_t s);
hipError_t launch_sweep(bool adjoint, bool f32, int nitems, const SweepItem *d_items, int nsteps,
                        int max_nb, hipStream_t s);

}  // namespace lrpr
