// Internal declarations of the lrpr library (HIP, gfx950).  Not part of the
// public ABI (include/lrpr.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
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
// With DL[I], DU[I] the inverses of the diagonal tiles L(I,I), U(I,I) and
// DLT[I], DUT[I] their transposes, the band tiles are stored multiplied from
// the left by their own row's inverse:
//   Lb[I][j]  = DL[I]  L(I, I-nb+j),    j = 0..nb-1
//   Ub[I][j]  = DU[I]  U(I, I+1+j),     j = 0..nb-1
//   UTb[I][j] = DUT[I] U^T(I, I-nb+j)   (mirrored set, optional)
//   LTb[I][j] = DLT[I] L^T(I, I+1+j)    (mirrored set, optional)
// so that a substitution pass reads y_I = D_I r_I - sum_J A_IJ y_J.  The
// transposes of the forward tiles are U^T(I,J) DUT[J] and L^T(I,J) DLT[J]:
// the adjoint without a mirrored set runs the form s_I = r_I - sum_J B_IJ s_J,
// y_I = D_I s_I on them.  Tiles outside the matrix are zero; the diagonal
// tiles of the padded rows beyond n are the identity.  Each tile has 256
// elements.
//
// Every tile is stored as MFMA A operands, lane-major: the four values lane l
// feeds to the four 16x16x4 products of a 16x16x16 contraction sit together
// (one 16-byte load in FP32, two in FP64).  With g = l/16, m = l%16 and kc the
// chunk, the value is T[m][kappa(g, kc)], where the contraction index
// kappa(g, kc) = 4 kc + g (FP64) or 4 g + kc (FP32) is the row that register
// kc of an MFMA accumulator holds, so accumulators feed the next product as B
// operands directly.  Position of (l, kc) in the tile:
//   FP32: 4 l + kc;     FP64: 128 (kc/2) + 2 l + kc%2.
// ---------------------------------------------------------------------------
constexpr int TILE = 16;
constexpr int TILE_ELEMS = 256;
// zero tile rows kept before and after every tile array (beyond the band and
// the sweep's prefetch window, reads land on zeros)
inline int guard_rows(int nb) { return nb + 8; }

enum { TS_LB, TS_UB, TS_UTB, TS_LTB, TS_DL, TS_DU, TS_DLT, TS_DUT, TS_COUNT };

struct TileSet {            // device arrays of one precision (pointers to tile row 0)
    void *a[TS_COUNT] = {};      // indexed by TS_*; UTb/LTb null without the mirrored set
    void *zt = nullptr;          // one all-zero tile: target of loads outside the band
    void *sink = nullptr;        // one scratch tile: target of masked-off stores
    void *alloc[TS_COUNT] = {};  // starts of the arrays behind a[] (guard rows earlier)
    void *block = nullptr;       // one allocation holding every array, zt and sink
};

// Device-side view of one factor, passed by value to the sweep kernels.
// ar: the tiles of the UL factorisation M = U' L' in the same layout (Lb and
// DL hold L', Ub and DU hold U'), or null.
struct FacView {
    const void *a[TS_COUNT];
    const void *ar[TS_COUNT];
    const void *zt;
    void *sink;
    int n, NT, nb;
    double dt;
};

// One work item of a sweep launch: up to 16 right-hand sides sharing a factor.
struct SweepItem {
    FacView fac;
    void *X;               // first column of the group
    int64_t ldx;
    int ncols;             // 1..16 (1..16 ng in a sweep of ng-group items)
    int passes;            // bit 0: first pass (L, or U^T), bit 1: second pass (U, or L^T)
    int r0, r1;            // tile rows [r0, r1) solved; rows outside are not coupled in
    int fsteps;            // length of a column's fscale row
    int pad_;
    const void *f;         // sources (element type of the sweep) or null
    int64_t ldf;
    const int *fcol;       // per column (offset to the group's first column) or null
    const double *fscale;  // per column x fsteps (offset) or null
};

// Partitioned forward solves (narrow panels).  The tile rows are cut into P
// blocks [blk[p], blk[p+1]) of at least 2 nb rows.  A substitution pass then
// runs as: local solves of every block with its own diagonal block (the
// sweep kernel on the block's range), a chain over the blocks for the nb
// boundary tile rows, and a parallel update of every block:
//   L pass: y_p = g_p - S_p y_{p-1}^tail,  S_p = L_pp^{-1} L_{p,p-1}[:, tail]
//   U pass: x_p = h_p - T_p x_{p+1}^head,  T_p = U_pp^{-1} U_{p,p+1}[:, head]
// where tail / head are the last / first nb tile rows of a block.  S and T
// are stored like the band tiles: NT x nb tiles (MFMA A operands), row I of
// block p holding S_p(I, .) (rows of block 0 unused) and T_p(I, .) (rows of
// the last block unused).
constexpr int SPLIT_MAX_P = 64;   // most blocks of a partitioned factor

struct SplitSet {
    void *S = nullptr;
    void *T = nullptr;
};

// One 16-column group of a partitioned pass (chain and update kernels).
struct SplitGroup {
    void *X;               // first column of the group (n rows, ldx)
    int64_t ldx;
    int ncols;
    int n, NT, nb, P;
    const int *blk;        // device, P+1 block starts (tile rows)
    const void *S, *T;     // spikes of the group's factor (precision of the pass)
    void *bnd;             // P x nb tiles (accumulator order): solved tails (L) / heads (U)
};

}  // namespace lrpr

struct lrpr_factor_s {
    int dev = 0;
    lrpr_op_desc op{};
    int64_t n = 0;
    int bw = 0;
    int NT = 0, nb = 0;
    int mask = 0;                  // LRPR_STORE_* bits
    int stepper = 0;               // LRPR_STEP_*; the factored matrix is I + a_11 dt A
    double dt_step = 0;            // the step dt (op.dt is a_11 dt)
    std::vector<lrpr_factor_s *> seq;   // LRPR_STEP_SEQUENCE: the owned per-step factors
    double *lu = nullptr;          // FP64 band LU, n x (2bw+1) row-major (kept with LRPR_STORE_F64)
    lrpr::TileSet t64, t32;
    lrpr::TileSet t64r, t32r;      // UL factorisation (LRPR_STORE_UL)
    // partitioned forward solves (LRPR_STORE_SPLIT): P blocks, starts blk
    int P = 0;
    std::vector<int> blk;
    int *d_blk = nullptr;
    lrpr::SplitSet s64, s32;
};

struct lrpr_coarse_s {
    int dev = 0;
    int nslices = 0;
    std::vector<int64_t> n;
    std::vector<int> k, l;
    std::vector<double *> U, S, V;  // device, per slice (inside `block` when that is set)
    double *block = nullptr;        // one allocation holding every slice's U, S, V
    std::vector<double *> more;     // further such allocations (a build done in chunks)
    std::vector<double> sigma;      // host copy of all singular values, per slice
    std::vector<lrpr_fac> F;     // factors the slices were built from (not owned)
    bool view = false;              // slices of another handle: owns no device memory
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
    // tuned launch shapes (lrpr_tune_set / lrpr_autotune_factor), 0 = default
    int tune_lu_wgs = 0;
    size_t tune_lu_budget = 0;   // bytes of FP64 bands and LU scratch per factor_many chunk
    int tune_pr_graph = 1;       // Parareal iterations replayed from a captured HIP graph
    int tune_sweep_groups = 0;   // 16-column groups per sweep workgroup (0 = by occupancy)
    size_t tune_rsvd_budget = 0; // bytes of rSVD panels per build chunk (0 = 96e9)
    int ncu = 256;               // compute units of the device
};

namespace lrpr {

constexpr double SDIRK2L_GAMMA = 0.29289321881345247560;   // (2 - sqrt 2) / 2
// source time factors per step of a factor's stepper (one per stage)
inline int fac_stages(const lrpr_factor_s *f) { return (f->stepper == 1 || f->stepper == 2) ? 2 : 1; }

// error helper: record message in ctx and return status
lrpr_status fail(lrpr_ctx ctx, lrpr_status st, const std::string &msg);

// Device memory of handles (factor tiles and bands, spikes, coarse
// factors): blocks freed by destroy calls are kept per device and size and
// handed to the next allocation of the same size (a batch of factors
// destroyed and made again with the same shapes maps no new memory), until
// lrpr_device_trim; an allocation that fails first gives them back.  The
// current device must be the handle's.  dfree: the block must not be in use
// by queued work.
hipError_t dmalloc(void **p, size_t bytes, hipStream_t s);
void dfree(void *p, hipStream_t s);

// Device address of the fixed scratch array of lrpr_coarse_apply_noalloc on
// device dev (noalloc.hip); dev must be current.  Looked up once per device.
hipError_t noalloc_scratch_init(int dev, double **out);

// A sweep as the list of its kernel launches over work-item arrays already
// in device memory (planned and uploaded once): it can run any number of
// times, on any stream, and be captured in a HIP graph, as long as the
// panels' buffers and the workspaces it names stay in place.
struct SweepPlan {
    std::vector<std::function<hipError_t(hipStream_t)>> launches;
    hipError_t run(hipStream_t s) const {
        for (const auto &l : launches)
            if (hipError_t e = l(s); e != hipSuccess) return e;
        return hipSuccess;
    }
};
// Plan an implicit-Euler sweep (the factors' stepper must be LRPR_STEP_EULER)
// with the same path choice as run_sweep; its item arrays go to workspaces
// named after ws_prefix (so that another sweep of the context does not
// overwrite them).  The uploads are queued on the context's stream.
lrpr_status plan_sweep(lrpr_ctx ctx, int npanels, const lrpr_panel *panels, int nsteps, lrpr_prec prec,
                       bool adjoint, bool split_any_width, const char *ws_prefix, SweepPlan *plan);

// Batched sweeps of nsteps steps of the panels' stepper (api_core.cpp).
// Forward sweeps on factors that all carry spikes take the partitioned passes
// when the launch has few column groups, or always with split_any_width: a
// column's arithmetic then does not depend on how many other columns share
// the launch (Parareal and the server rely on this).
lrpr_status run_sweep(lrpr_ctx ctx, int npanels, const lrpr_panel *panels, int nsteps, lrpr_prec prec,
                      bool adjoint, bool split_any_width = false);

// kernels launched from the host code (defined in the .hip sources)
// rev: assemble J diag(M, I) J with rows = 16 NT (its LU gives the UL factorisation of M)
hipError_t launch_assemble(const lrpr_op_desc &op, int64_t n, int64_t rows, int bw, bool rev, double *band,
                           hipStream_t s);
// pipelined tile LU (lu.hip): scratch of tile_lu_scratch_bytes(NT, nb) per matrix
size_t tile_lu_scratch_bytes(int NT, int nb);
// count independent factorisations of one tile shape (rows ns[i], band and
// scratch per matrix)
// wgs: workgroups per matrix, 0 = tile_lu_wgs's choice
hipError_t launch_tile_lu_batch(int count, const int64_t *ns, int bw, int NT, int nb, double *const *bands,
                                void *const *scratch, int **info_dev, int **err_dev, void *d_args, hipStream_t s,
                                int wgs = 0);
// workgroups per matrix of a batched LU of count matrices (wgs > 0: that
// request, clipped to nb + 9 and NT); resident: tile_lu_resident(nb)
int tile_lu_wgs(int count, int NT, int nb, int wgs, int resident);
// LU workgroups per launch on the current device, all resident at once: one
// per compute unit (0 if the kernel variant for nb cannot be resident)
int tile_lu_resident(int nb);
size_t tile_lu_args_bytes(int count);
// rev: lu is the LU of the reversed matrix (16 NT rows); the sets then hold
// the UL factors (Lb / DL: the lower factor, Ub / DU: the upper one)
hipError_t launch_pack_tiles(int64_t n, int bw, int NT, int nb, const double *lu, bool rev, const TileSet *t64,
                             const TileSet *t32, double *scratch, hipStream_t s);
// adjoint sweeps read the mirrored set unless `strided` (then the forward
// tiles are read transposed); `local`: forward block solves of a partitioned
// pass (same code, launched as k_sweep_local); ng: 16-column groups per item
// (1 .. sweep_max_groups; items then hold up to 16 ng columns)
hipError_t launch_sweep(bool adjoint, bool strided, bool f32, int nitems, const SweepItem *d_items, int nsteps,
                        int max_nb, hipStream_t s, int step0 = 0, bool local = false, int ng = 1);
int sweep_max_groups(bool f32, int max_nb);
// One pass pair over full-range items whose factors all carry the UL set
// (mirrored too for the adjoint) and have nb band tiles per row, with
// sweep_pairable(nb).  Descending (asc false): the second substitution of an
// L U step with the first of the next U' L' step; ascending: the second of a
// U' L' step with the first of the next L U step.  stepB: pass B's step.
hipError_t launch_sweep_pair(bool adjoint, bool asc, bool f32, int nitems, const SweepItem *d_items, int nb,
                             hipStream_t s, int stepB);
bool sweep_pairable(int nb);
// narrow forward sweeps on the vector ALUs (narrow.hip): items of at most
// sweep_narrow_cols(f32) columns, 2..64 band tiles per row
int sweep_narrow_cols(bool f32);
bool sweep_narrow_ok(bool f32, int max_nb, int ncols);
hipError_t launch_sweep_narrow(bool f32, int nitems, const SweepItem *d_items, int nsteps, int max_nb,
                               int ncols_max, hipStream_t s, int step0);
// out = ca a + cb b + cc c on an n x w block (column-major, own leading
// dimensions; c may be null), element type of the precision (dense.hip)
hipError_t launch_combine3(bool f32, void *out, int64_t ldo, const void *a, int64_t lda, double ca, const void *b,
                           int64_t ldb, double cb, const void *c, int64_t ldc, double cc, int64_t n, int w,
                           hipStream_t s);
// Gaussian fill, Philox4x32-10 + Box-Muller (rng.hip)
hipError_t launch_randn(bool f32, void *dst, int64_t count, uint64_t seed, uint64_t stream, hipStream_t s);
// partitioned passes (split.hip)
hipError_t launch_spike_rhs(int64_t n, int bw, int NT, int nb, int P, const int *d_blk, const double *lu,
                            double *RL, double *RU, hipStream_t s);
hipError_t launch_spike_pack(bool f32, int NT, int nb, const void *dense, int64_t ld, void *tiles, hipStream_t s);
// uniform_nb: every group has nb == max_nb (enables the kernels specialised
// on the band-tile count)
hipError_t launch_split_chain(bool f32, bool upper, int ngroups, const SplitGroup *d_groups, int max_nb,
                              hipStream_t s, bool uniform_nb);
// d_runs (or null): nruns runs {first group, count} of consecutive groups on
// one factor, every group with nb == max_nb in {8, 16, 32} (the spike tiles
// are then read once per run)
hipError_t launch_split_update(bool f32, bool upper, int ngroups, const SplitGroup *d_groups, int max_P,
                               int max_rows, hipStream_t s, int max_nb, int nruns, const int2 *d_runs);

}  // namespace lrpr
