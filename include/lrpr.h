/*
 * lrpr.h -- C ABI of the MI355X (gfx950) library for Parareal with low-rank
 * coarse solvers (Gander, Ohlberger, Rave, arXiv 2508.08873).
 *
 * The library builds, on one GPU:
 *   - the fine propagator: implicit-Euler steps of a finite-difference
 *     diffusion-advection-reaction operator through a banded LU, batched over
 *     many right-hand sides (forward F_n and adjoint F_n'^*), Sec. 2 eq.
 *     (F_n_affine) and Sec. 2.1 step 3;
 *   - the randomized SVD of every slice's transfer operator F_n' (Sec. 2.1,
 *     steps 1-6), giving the low-rank coarse solvers G_n (eq. spectral_G);
 *   - the Parareal iteration with those coarse solvers (Sec. 2, eq.
 *     def_Parareal) and its a posteriori bound (Sec. 3, eq. apost_bound).
 *
 * Conventions for every call:
 *   - Matrices are column-major.  "device" pointers point to GPU memory of
 *     the context's device; "host" pointers to ordinary CPU memory.
 *   - The caller owns every array it passes.  Handles (lrpr_ctx,
 *     lrpr_factor, lrpr_coarse) own the memory they allocate and free it in
 *     their destroy call.
 *   - Work is queued on the context's HIP stream.  Calls that return host
 *     outputs synchronise that stream before returning; others are
 *     asynchronous (device outputs are valid once the stream reaches them).
 *   - Every call returns an lrpr_status.  On LRPR_ERR_ARG nothing is written.
 *     lrpr_last_error() gives a message for the last failing call of a
 *     context.  No exception crosses the ABI.
 *   - One host thread per context at a time.
 */
#ifndef LRPR_H
#define LRPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lrpr_ctx_s *lrpr_ctx;
typedef struct lrpr_factor_s *lrpr_fac;   /* factor handle (returned by lrpr_factor) */
typedef struct lrpr_coarse_s *lrpr_coarse;

/* Arithmetic precision of a fine solve: states, factors and accumulation. */
typedef enum { LRPR_F64 = 0, LRPR_F32 = 1 } lrpr_prec;

typedef enum {
    LRPR_OK = 0,
    LRPR_ERR_ARG = 1,          /* invalid argument; nothing was written        */
    LRPR_ERR_NOMEM = 2,        /* device allocation failed                     */
    LRPR_ERR_ZERO_PIVOT = 3,   /* band LU met a zero or non-finite pivot       */
    LRPR_ERR_QR_BREAKDOWN = 4, /* orthonormalisation failed even in fallback   */
    LRPR_ERR_NOCONV = 5,       /* Parareal did not reach tol within max_iter   */
    LRPR_ERR_NONFINITE = 6,    /* NaN or Inf met in a result                   */
    LRPR_ERR_HIP = 7           /* HIP runtime error                            */
} lrpr_status;

/* Operator of one time slice:  u_t = -A u + f  with A the finite-difference
 * discretisation of  -nu*Laplace(u) + beta.grad(u) + c*u  on the unit
 * interval (dim=1, n = nx points) or unit square (dim=2, n = nx*nx, index
 * i + nx*j with x fastest), first-order upwind advection.  Boundary (bc):
 *   LRPR_BC_DIRICHLET (0): homogeneous Dirichlet; the nx points per axis are
 *     interior, h = 1/(nx+1);
 *   LRPR_BC_NEUMANN (1): homogeneous Neumann (the variant of the paper's
 *     first experiment, Sec. 4); the nx >= 2 points per axis include both
 *     boundary points, h = 1/(nx-1), and the boundary condition is imposed
 *     with a mirrored ghost point (u_{-1} = u_1), so every row of A sums to
 *     c and constants are an eigenvector.
 * The fine step is implicit Euler with step dt:
 * (I + dt*A) x_new = x_old + dt*f(t_new).  Half-bandwidth b = 1 (dim=1) or
 * nx (dim=2).  (The paper discretises with finite elements; Sec. 4, first
 * paragraph.) */
enum { LRPR_BC_DIRICHLET = 0, LRPR_BC_NEUMANN = 1 };
typedef struct {
    int dim;       /* 1 or 2 */
    int nx;        /* interior points per axis, >= 1 */
    double nu;     /* diffusion, > 0 */
    double beta1;  /* advection velocity, x component */
    double beta2;  /* advection velocity, y component (ignored for dim=1) */
    double c;      /* reaction, >= 0 */
    double dt;     /* implicit-Euler step, > 0 */
    int bc;        /* LRPR_BC_DIRICHLET or LRPR_BC_NEUMANN */
} lrpr_op_desc;

/* Lumped (trapezoidal) mass of the operator's grid: the weights of the
 * discrete L^2 inner product (u, v)_W = sum_i w_i u_i v_i, the inner product
 * the paper takes for the Neumann constant mode (Sec. 4).  Dirichlet:
 * w_i = h^dim; Neumann: a factor 1/2 per axis on boundary points, so the
 * weights sum to 1.  w_host: host, n doubles.  Errors: LRPR_ERR_ARG. */
lrpr_status lrpr_mass_weights(const lrpr_op_desc *op, double *w_host);

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, queueing work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle.
 * A context caches the device workspaces its calls need (work-item arrays,
 * LU bands and scratch, spike staging, the rSVD panels and small matrices,
 * Parareal state): they grow to the largest shape met and are freed by
 * lrpr_ctx_destroy (about 7 GB for a 255^2 rSVD build of 64 slices x 50
 * columns), so that calls after the first of a shape allocate and free no
 * temporaries.  Contexts share no state: independent contexts on separate
 * streams, driven from separate host threads, run concurrently.  One context
 * must not be used from two threads at once. */
lrpr_status lrpr_ctx_create(int device, void *hip_stream, lrpr_ctx *out);
void lrpr_ctx_destroy(lrpr_ctx ctx);
/* Free every cached workspace of ctx (synchronises its stream).  Later
 * calls allocate them again; handles are not affected.  For callers that
 * need the device memory between phases of different shapes.
 * Errors: LRPR_ERR_ARG, LRPR_ERR_HIP. */
lrpr_status lrpr_ctx_release_workspaces(lrpr_ctx ctx);
/* Tunable launch shapes of a context (set by hand or by the autotuner).
 * They change how work is spread over the chip and issued, not the results:
 *   LRPR_TUNE_LU_WGS         workgroups per matrix of the batched band LU
 *                            (0 = the library's choice; clipped to nb + 9,
 *                            nb = ceil(b/16) band tiles);
 *   LRPR_TUNE_LU_BUDGET      bytes of FP64 bands and LU scratch that
 *                            lrpr_factor_many holds at once (0 = 110e9);
 *   LRPR_TUNE_PARAREAL_GRAPH 1 (default): a Parareal iteration is captured
 *                            once in a HIP graph and replayed; 0: its
 *                            kernels are launched one by one;
 *   LRPR_TUNE_SWEEP_GROUPS   sixteen-column groups that one workgroup of an
 *                            FP32 sweep (4 < nb <= 32) carries, reading
 *                            each band tile once for all of them: 0 = the
 *                            library's choice (the most, up to 3, that
 *                            still gives every compute unit a workgroup),
 *                            1..3 = that many;
 *   LRPR_TUNE_RSVD_BUDGET    bytes of panels (n (k+p) per slice, two in the
 *                            range finder's precision and three in FP64)
 *                            that one rSVD build holds at once (0 = 96e9):
 *                            larger builds run in chunks of consecutive
 *                            slices, with the same results per slice.
 * Errors: LRPR_ERR_ARG for an unknown parameter or a value out of range. */
enum {
    LRPR_TUNE_LU_WGS = 1,
    LRPR_TUNE_LU_BUDGET = 2,
    LRPR_TUNE_PARAREAL_GRAPH = 3,
    LRPR_TUNE_SWEEP_GROUPS = 4,
    LRPR_TUNE_RSVD_BUDGET = 5
};
lrpr_status lrpr_tune_set(lrpr_ctx ctx, int param, int64_t value);
lrpr_status lrpr_tune_get(lrpr_ctx ctx, int param, int64_t *value);
/* Autotuner of the batched band LU for a later lrpr_factor_many of `count`
 * operators on op's grid: factors copies of *op, as many as one chunk of
 * that call holds (store_mask as given), once per candidate number of
 * workgroups per matrix (the default choice, nb + 9 and narrower ones that
 * let more matrices share a launch), after one untimed run, timed with HIP
 * events; keeps the
 * fastest as the context's LRPR_TUNE_LU_WGS and returns it (best_wgs,
 * best_ms may be NULL).  The factors do not depend on the choice.
 * Synchronises.  Errors: as lrpr_factor_many. */
lrpr_status lrpr_autotune_factor(lrpr_ctx ctx, const lrpr_op_desc *op, int count, int store_mask, int *best_wgs,
                                 double *best_ms);
/* Device memory that destroy calls free (factor tiles and bands, spikes,
 * coarse factors) is kept by the library, per device and block size, for
 * the next handle of the same shape.  lrpr_device_trim synchronises the
 * device and frees the kept blocks (lrpr_ctx_destroy does so too, and an
 * allocation that fails retries after it), for callers that need the memory
 * otherwise.  Errors: LRPR_ERR_HIP. */
lrpr_status lrpr_device_trim(int device);
/* Replace the stream used by later calls. */
lrpr_status lrpr_ctx_set_stream(lrpr_ctx ctx, void *hip_stream);
/* Message of the last failing call on ctx (static storage owned by ctx). */
const char *lrpr_last_error(lrpr_ctx ctx);

/* Sweep timing.  While enabled, every fine/adjoint sweep launch queued by
 * this context is bracketed by HIP events on the context's stream, and its
 * algorithmic work is recorded: 4*n*b flops per right-hand-side step, and
 * 2*n*s bytes per right-hand-side step (state in and out) plus n*(2b+1)*s
 * bytes per step for each factor read (s = 8 or 4 bytes per value). */
lrpr_status lrpr_profile_enable(lrpr_ctx ctx, int enable);
/* Synchronises the stream and returns, for the launches recorded since the
 * last read: total kernel time in ms, number of launches, algorithmic flops
 * and bytes, and right-hand-side steps; then clears the record.  Any output
 * pointer may be NULL. */
lrpr_status lrpr_profile_read(lrpr_ctx ctx, double *ms, int64_t *launches, double *flops, double *bytes,
                              double *rhs_steps);

/* ---- Gaussian test matrices (Sec. 2.1, step 1) ---------------------------- */

/* Fill dst (device, count elements of type prec) with standard Gaussians of
 * the counter-based generator Philox4x32-10 (Salmon et al., SC'11) and the
 * Box-Muller transform: element pair j of (seed, stream) comes from counter
 * (j mod 2^32, j div 2^32, stream mod 2^32, stream div 2^32) and key
 * (seed mod 2^32, seed div 2^32); the words (x0, x1), (x2, x3) give uniforms
 * u = (floor((hi 2^32 + lo) / 2^11) + 1/2) 2^-53, and elements 2j, 2j+1 are
 * sqrt(-2 ln u1) cos(2 pi u2) and sqrt(-2 ln u1) sin(2 pi u2), computed in
 * FP64 (rounded once for LRPR_F32).  The result depends only on (seed,
 * stream, element index), so any slice of a test matrix can be drawn on its
 * own.  Stream-ordered on the context's stream.  Errors: LRPR_ERR_ARG. */
lrpr_status lrpr_randn(lrpr_ctx ctx, void *dst, int64_t count, lrpr_prec prec, uint64_t seed, uint64_t stream);

/* ---- operator assembly and band LU (Sec. 4.4) --------------------------- */

enum { LRPR_STORE_F64 = 1, LRPR_STORE_F32 = 2, LRPR_STORE_MIRROR = 4, LRPR_STORE_SPLIT = 8, LRPR_STORE_UL = 16 };

/* Assemble M = I + dt*A on the device and factor it M = L U by banded
 * Gaussian elimination without pivoting, in FP64 (the paper's fine solver
 * factors the backward-Euler matrix once and reuses it for all right-hand
 * sides, Sec. 4.4).  M is an M-matrix that is diagonally dominant by rows
 * and columns, so no pivoting is needed.  The factorisation is always FP64;
 * store_mask selects the copies kept for the solves (an OR of):
 *   LRPR_STORE_F64 (1)    FP64 tiles (needed for LRPR_F64 solves) and the
 *                         FP64 band LU;
 *   LRPR_STORE_F32 (2)    FP32 tiles rounded from the FP64 factors (needed
 *                         for LRPR_F32 solves);
 *   LRPR_STORE_MIRROR (4) for each precision kept, also the band tiles of
 *                         U^T and L^T, so adjoint sweeps read contiguous
 *                         tiles (faster; doubles the band-tile memory,
 *                         about 2 n (2b+1) bytes per byte of precision).
 *   LRPR_STORE_SPLIT (8)  for each precision kept, also the spikes of a
 *                         partitioned substitution (same size as the
 *                         forward band tiles), so that fine sweeps of few
 *                         right-hand sides spread each column group over
 *                         several compute units (same results up to
 *                         rounding).
 *   LRPR_STORE_UL (16)    for each precision kept (and mirrored with
 *                         MIRROR), also the tiles of the UL factorisation
 *                         M = U' L' (U' unit upper, L' lower: the LU of the
 *                         row- and column-reversed matrix, factored in the
 *                         same launch).  Implicit-Euler sweeps of two or
 *                         more steps whose factors all carry it then
 *                         alternate LU and UL steps, so that the last
 *                         substitution of one step and the first of the next
 *                         run in the same direction and share one pass over
 *                         the rows; the state between them stays on chip.
 *                         Same results up to rounding; doubles the tile
 *                         memory.
 * 0 means LRPR_STORE_F64; at least one of F64/F32 must be set.  Errors:
 * LRPR_ERR_ARG (bad descriptor or mask), LRPR_ERR_ZERO_PIVOT,
 * LRPR_ERR_NOMEM.  Synchronises the stream. */
lrpr_status lrpr_factor(lrpr_ctx ctx, const lrpr_op_desc *op, int store_mask, lrpr_fac *out);

/* Fine time steppers (the paper's study of the time discretisation, Sec. 4:
 * two-stage SDIRK methods beside implicit Euler):
 *   LRPR_STEP_EULER   implicit Euler (what lrpr_factor builds);
 *   LRPR_STEP_SDIRK2  tableau c = (1, 0), a = [[1, 0], [-1, 1]], b = (1/2, 1/2):
 *                     both stages solve with I + dt A, so the factor is the
 *                     implicit-Euler one;
 *   LRPR_STEP_SDIRK2L tableau c = (g, 1), a = [[g, 0], [1-g, g]], b = (1-g, g),
 *                     g = (2 - sqrt 2)/2 (L-stable): the factor is of I + g dt A.
 * A factor made with lrpr_factor_stepper carries its stepper: every sweep,
 * rSVD build and Parareal solve on it takes nsteps steps of that method (two
 * stage solves per step), and its source time factors hold two values per
 * step, phi(t_j + c_1 dt) then phi(t_j + c_2 dt), so a column's fscale row
 * has 2*nsteps entries (lrpr_parareal_solve: N x 2*nsteps).  The adjoint of
 * a step is the same two-stage recurrence with M^T.  The factors of one call
 * must share a stepper.  op->dt is the step size dt.  Errors: as
 * lrpr_factor; LRPR_ERR_ARG for an unknown stepper. */
enum { LRPR_STEP_EULER = 0, LRPR_STEP_SDIRK2 = 1, LRPR_STEP_SDIRK2L = 2, LRPR_STEP_SEQUENCE = 3 };
lrpr_status lrpr_factor_stepper(lrpr_ctx ctx, const lrpr_op_desc *op, int store_mask, int stepper,
                                lrpr_fac *out);

/* Per-step operators inside a slice (time-dependent coefficients, the
 * setting of the paper's later experiments, Sec. 4): one handle for m
 * implicit-Euler steps whose step j solves with M_j = I + dt_j A_j, A_j and
 * dt_j from ops[j] (all ops share dim and nx).  Each step is factored as by
 * lrpr_factor with store_mask.  A sweep of nsteps <= m steps on the handle
 * takes step j with M_j, j = 0..nsteps-1 (source time factor j of a column
 * at step j, as for lrpr_factor); the adjoint is the transpose of that
 * product, T^T = M_1^{-T} ... M_nsteps^{-T}: the transposed steps in reverse
 * order.  rSVD builds and Parareal solves on such handles use this map
 * (stepper LRPR_STEP_SEQUENCE; the server does not take them).  The handle
 * owns its step factors (lrpr_factor_destroy frees them).  Errors: as
 * lrpr_factor; LRPR_ERR_ARG for m < 1 or mismatched grids. */
lrpr_status lrpr_factor_sequence(lrpr_ctx ctx, const lrpr_op_desc *ops, int m, int store_mask, lrpr_fac *out);
/* Independent factors of count operators on one grid (e.g. one per time
 * slice when the coefficients change from slice to slice, Sec. 4): outs[j]
 * receives the factor of ops[j], as lrpr_factor would make it.  The band LUs
 * of several operators run in one launch, in chunks that bound the FP64
 * bands held at once (the matrices one launch holds together, at least
 * about 2 GB of bands).  On error no handle is returned (every outs[j] is
 * NULL).  Errors: as lrpr_factor; LRPR_ERR_ARG for count < 1 or operators
 * on different grids. */
lrpr_status lrpr_factor_many(lrpr_ctx ctx, const lrpr_op_desc *ops, int count, int store_mask, lrpr_fac *outs);
void lrpr_factor_destroy(lrpr_fac f);
/* n = unknowns, bw = half-bandwidth, dt = step (of the factor's stepper). */
lrpr_status lrpr_factor_info(lrpr_fac f, int64_t *n, int *bw, double *dt);
/* Copy the FP64 band LU (kept with LRPR_STORE_F64) to host memory:
 * lu_host is n x (2*bw+1) row-major,
 * entry (i, j) of L (j < i, unit diagonal not stored) or U (j >= i) at
 * lu_host[i*(2*bw+1) + j - i + bw].  Synchronises. */
lrpr_status lrpr_factor_copy_lu(lrpr_ctx ctx, lrpr_fac f, double *lu_host);
/* Copy the packed band tiles that the sweeps read (Sec. 4.4: the factors
 * reused by every solve), kept with LRPR_STORE_F64 or LRPR_STORE_F32:
 * set 0 = the lower factor's tiles L(I,I)^{-1} L(I, I-nb+j), set 1 = the
 * upper factor's U(I,I)^{-1} U(I, I+1+j), for tile rows I = 0..NT-1 and
 * j = 0..nb-1 (16x16 tiles, NT = ceil(n/16), nb = ceil(bw/16)).  Tile
 * (I, j) starts at element (I*nb + j)*256 of host; entry (r, k) of a tile
 * sits at 128*(k/8) + 2*(16*(k%4) + r) + (k/4)%2 (FP64) or
 * 4*(16*(k/4) + r) + k%4 (FP32), the matrix cores' A-operand order.  The
 * FP32 tiles are the FP64 products rounded row by row (a row = the 16 nb
 * entries of one matrix row) with the row sum kept: every entry rounded,
 * the FP64 sum of the rounding errors added to the largest entry, and what
 * that entry's rounding leaves added to the smallest entry of at least
 * 2^-12 of the largest (ties: the first entry in j, k order).
 * host: NT*nb*256 elements of the precision.  Synchronises.
 * Errors: LRPR_ERR_ARG (null argument, set not 0 or 1, precision not kept). */
lrpr_status lrpr_factor_copy_tiles(lrpr_ctx ctx, lrpr_fac f, int set, lrpr_prec prec, void *host);

/* ---- batched fine propagator and its adjoint (Sec. 2, Sec. 2.1) --------- */

/* One panel: w right-hand sides that share the factor F.
 *   X      device, n x w, leading dimension ldx >= n, element type by prec
 *          (double for LRPR_F64, float for LRPR_F32); in: start states,
 *          out: states after nsteps steps.
 *   f      device, n x nf source vectors (same element type), ld ldf, or
 *          NULL for no source.
 *   fcol   device int[w]: source column used by RHS c, or -1 for none;
 *          NULL means column 0 for every RHS (only read if f != NULL).
 *   fscale device double[w*nsteps]: time factor of RHS c at step j at
 *          fscale[c*nsteps + j] (the source is f(x)*phi(t) evaluated at the
 *          step's end time); NULL means 1.  */
typedef struct {
    lrpr_fac F;
    void *X;
    int64_t ldx;
    int w;
    const void *f;
    int64_t ldf;
    const int *fcol;
    const double *fscale;
} lrpr_panel;

/* Fine propagator F_n (Sec. 2, eq. F_n_affine): for every panel and every
 * column, nsteps implicit-Euler steps
 *     (I + dt*A) x_{j+1} = x_j + dt * fscale[c][j] * f[:, fcol[c]]
 * through the panel's band LU (forward then back substitution).  Without a
 * source this is the transfer operator T = M^{-nsteps} (= F_n').  All panels
 * run in one launch; panels may use different factors and sizes.  When every
 * factor keeps spikes (LRPR_STORE_SPLIT) and the launch has at most 32
 * sixteen-column groups, the partitioned passes run; otherwise the plain (or
 * paired) substitution.  The two round differently (same solve).
 * Errors: LRPR_ERR_ARG (null/mismatched arguments, missing FP32 factor). */
lrpr_status lrpr_fine_step_batched(lrpr_ctx ctx, int npanels, const lrpr_panel *panels,
                                   int nsteps, lrpr_prec prec);

/* Adjoint propagator F_n'^* (Sec. 2.1 step 3): X <- (M^T)^{-nsteps} X for
 * every panel (forward substitution with U^T, back substitution with L^T,
 * the same factors read transposed).  The panels' f/fcol/fscale are
 * ignored (the adjoint of the linear part has no source). */
lrpr_status lrpr_adjoint_step_batched(lrpr_ctx ctx, int npanels, const lrpr_panel *panels,
                                      int nsteps, lrpr_prec prec);

/* ---- randomized SVD build (Sec. 2.1) ------------------------------------- */

/* One Parareal slice for the coarse-solver build: its factor, truncation
 * rank k (R_n in the paper) and oversampling p, and its Gaussian test
 * matrix Omega (device, n x (k+p), column-major, ld n, element type of
 * range_prec).  k + p <= 128, k + p <= n. */
typedef struct {
    lrpr_fac F;
    int k;
    int p;
    const void *Omega;
} lrpr_slice_desc;

/* Randomized SVD of every slice's transfer operator T = M^{-nsteps}
 * (Sec. 2.1, steps 1-6), all slices together:
 *   Y = T Omega (fine sweep, range_prec);  Y = Q R (CholeskyQR2 with FP64
 *   Gram and Cholesky; Householder fallback on breakdown);  Z = T^T Q
 *   (adjoint sweep);  Z = Qz Rz;  Mm = Rz^T = Uh diag(S) Vh^T (one-sided
 *   Jacobi, FP64);  U_k = Q Uh[:, :k],  V_k = Qz Vh[:, :k]  (FP64).
 * Each pair (U_k[:, r], V_k[:, r]) is signed so that the largest-magnitude
 * entry of U_k[:, r] (lowest index on ties) is positive.
 * *out receives a coarse handle holding, per slice, U_k, S (all k+p
 * singular values) and V_k in device memory.
 * sigma_host: host, NULL or sum over slices of (k+p) doubles: all singular
 *   values, slice after slice.
 * fallback_host: host, NULL or int[nslices]: 1 where the Householder
 *   fallback orthonormalised Y or Z.
 * Errors: LRPR_ERR_ARG, LRPR_ERR_NOMEM, LRPR_ERR_QR_BREAKDOWN,
 * LRPR_ERR_NONFINITE.  Synchronises. */
lrpr_status lrpr_rsvd_build(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices,
                            int nsteps, lrpr_prec range_prec, lrpr_coarse *out,
                            double *sigma_host, int *fallback_host);
/* The same build with q >= 0 power iterations (Sec. 2.1, for slowly
 * decaying singular values): the range space becomes span (T T^T)^q T
 * Omega, reached by q rounds of "orthonormalise Y (CholeskyQR2), Z = T^T Q,
 * orthonormalise Z, Y = T Qz" after Y = T Omega; the steps after that are
 * those of lrpr_rsvd_build.  Costs 2q more sweeps of every slice's panel.
 * q = 0 is lrpr_rsvd_build.  fallback_host flags a slice if any of its
 * orthonormalisations fell back to Householder.  Errors: as
 * lrpr_rsvd_build; LRPR_ERR_ARG for q < 0. */
lrpr_status lrpr_rsvd_build_q(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices,
                              int nsteps, int q, lrpr_prec range_prec, lrpr_coarse *out,
                              double *sigma_host, int *fallback_host);
/* The build with the adjoint on independent test vectors (Sec. 2.2: more
 * parallelism at some loss of accuracy).  psi: host array of nslices device
 * pointers, each an n x (k+p) Gaussian matrix (column-major, ld n, element
 * type of range_prec) drawn independently of the slice's Omega; read only.
 *   Y = T Omega,  Z = T^T Psi (the adjoint sweep does not wait for Q);
 *   Y = Q R (CholeskyQR2);  C = Psi^T Q;  X^T = Z C^{-T} (Gauss-Jordan
 *   inverse of C, FP64);  X^T = Qx Rx;  Rx^T = Uh diag(S) Vh^T;
 *   U_k = Q Uh[:, :k],  V_k = Qx Vh[:, :k],
 * the rank-k truncation of Q (Psi^T Q)^{-1} Psi^T T.  Signs, outputs and
 * errors as lrpr_rsvd_build; LRPR_ERR_QR_BREAKDOWN if Psi^T Q is singular. */
lrpr_status lrpr_rsvd_build_two_sided(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices,
                                      const void *const *psi, int nsteps, lrpr_prec range_prec,
                                      lrpr_coarse *out, double *sigma_host, int *fallback_host);
/* The build in the inner product (u, v)_W = sum_i w_i u_i v_i (eq. svd with
 * the inner product on V: the generalized SVD of F_n'; Sec. 4 takes the L^2
 * inner product of the discretisation).  The result satisfies
 *   T v ~ sum_r psi_r S_r (phi_r, v)_W,  psi and phi W-orthonormal,
 * and is stored as U_k = psi, V_k = W phi, so that the coarse apply and
 * Parareal use it unchanged (G_n' v = U_k (S_k .* (V_k^T v))).  Computed as
 * the build of lrpr_rsvd_build_q for W^{1/2} T W^{-1/2} (the test matrix
 * Omega is taken in those coordinates), mapped back.  Signs: the
 * largest-magnitude entry of psi_r is positive.
 * weights: host array of nslices device pointers, each n positive doubles
 *   (not checked), or NULL entries for the Euclidean inner product.
 * Other arguments, outputs and errors as lrpr_rsvd_build_q. */
lrpr_status lrpr_rsvd_build_w(lrpr_ctx ctx, int nslices, const lrpr_slice_desc *slices,
                              const double *const *weights, int nsteps, int q, lrpr_prec range_prec,
                              lrpr_coarse *out, double *sigma_host, int *fallback_host);
/* A coarse handle from given factors: a priori coarse spaces such as the
 * rank-1 constant mode of the Neumann experiment (Sec. 4: R_n = 1, sigma =
 * 1, phi = psi = the constant function in the L^2 inner product, i.e. U = 1,
 * S = 1, V = W 1).  Per slice s: F[s] its factor (gives n), k[s] >= 1, and
 * device FP64 arrays U[s] (n x k, ld n), S[s] (k values) and V[s] (n x k, ld
 * n), copied into the handle; G_n' v = U (S .* (V^T v)).  Errors:
 * LRPR_ERR_ARG, LRPR_ERR_NOMEM.  Synchronises. */
lrpr_status lrpr_coarse_from_factors(lrpr_ctx ctx, int nslices, const lrpr_fac *F, const int *k,
                                     const double *const *U, const double *const *S, const double *const *V,
                                     lrpr_coarse *out);
void lrpr_coarse_destroy(lrpr_coarse c);
/* A handle on slices [first, first+count) of c (their U, S, V and singular
 * values, in order), for solving problems built together in one
 * lrpr_rsvd_build call one by one (Sec. 2.2: the coarse propagators of
 * different intervals are independent).  The view owns no device memory:
 * lrpr_coarse_destroy on it frees only the view, and c must outlive it.
 * Errors: LRPR_ERR_ARG (range outside c), LRPR_ERR_NOMEM. */
lrpr_status lrpr_coarse_view(lrpr_coarse c, int first, int count, lrpr_coarse *out);
/* Device pointers (owned by the handle) of slice s: U (n x k), S (k+p
 * values), V (n x k); k and n of that slice. */
lrpr_status lrpr_coarse_get(lrpr_coarse c, int s, const double **U, const double **S,
                            const double **V, int *k, int64_t *n);

/* Linear part of the coarse solver, G_n' v = U_k (S_k .* (V_k^T v))
 * (Sec. 2, eq. spectral_G without b_n; Sec. 2.2 last paragraph) for the w
 * columns of Vin (device, n x w, ld n, FP64) into Out (device, same shape).
 * Asynchronous. */
lrpr_status lrpr_coarse_apply(lrpr_ctx ctx, lrpr_coarse c, int s, int w, const double *Vin,
                              double *Out);

/* The same apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no device memory is allocated or freed.  Its scratch (chunk partials and
 * coefficients, (ceil(n/256) + 1) * k * min(w, 12288/k) doubles) lives in a
 * fixed array of 16 MiB per GPU, held until the process ends; a call whose
 * scratch would exceed it returns LRPR_ERR_ARG and writes nothing.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (from two contexts, streams or threads) race and must be serialised by
 * the caller.  Results equal lrpr_coarse_apply's.  Asynchronous. */
lrpr_status lrpr_coarse_apply_noalloc(lrpr_ctx ctx, lrpr_coarse c, int s, int w, const double *Vin,
                                      double *Out);

/* ---- Parareal with the low-rank coarse propagator (Sec. 2) -------------- */

/* Parareal with the low-rank coarse solvers of c (Sec. 2, eq.
 * def_Parareal) for nreq independent problems that share the slices'
 * operators (different initial values and sources):
 *   b_n = F_n 0 (fine sweep from zero with source);
 *   u^0_0 = u0, u^0_n = G_n' u^0_{n-1} + b_n;
 *   u^{k+1}_n = F_n u^k_{n-1} + G_n' u^{k+1}_{n-1} - G_n' u^k_{n-1}
 * (the fine solves of an iteration run as one batched launch; the
 * correction is a sequential sweep over n in FP64), stopping per problem
 * when max_n ||u^{k+1}_n - u^k_n||_2 < tol or after N = nslices
 * iterations.
 *   F        host array of nslices factors (slice n uses F[n-1]); must
 *            match the slices c was built from.
 *   u0       device, n x nreq (FP64).
 *   f        device, n x nreq sources (FP64; converted internally for FP32
 *            fine solves) or NULL.
 *   fscale   device, nslices*nsteps doubles: time factor at the end of step
 *            j of slice n at fscale[(n-1)*nsteps + j], shared by all
 *            problems; NULL means 1.
 *   U        device, output, nreq blocks of n x (N+1) (FP64): the last
 *            iterate u^K_0..u^K_N of each problem, block r at U + r*n*(N+1).
 *   iters_host  host int[nreq]: iterations K done per problem.
 *   incr_host   host double[nreq*max_iter] or NULL: increments per
 *            iteration (row r at incr_host + r*max_iter).
 *   apost_host  host double[nreq*N] or NULL: a posteriori bound (eq.
 *            apost_bound) of the last iterate, per slice, with
 *            delta = max_n sigma_{n,1}, eps = max_n sigma_{n,k+1}.
 * Fine solves on factors that keep spikes always take the partitioned
 * passes, and every column's arithmetic is independent of the others, so a
 * problem's results are the same bit for bit whatever nreq and the other
 * problems are.
 * Returns LRPR_ERR_NOCONV (with all outputs written) if some problem
 * did not reach tol within max_iter iterations (max_iter < N);
 * LRPR_ERR_NONFINITE if an increment is not finite (outputs not written).
 * Synchronises. */
lrpr_status lrpr_parareal_solve(lrpr_ctx ctx, lrpr_coarse c, const lrpr_fac *F, int nsteps,
                                lrpr_prec fine_prec, int nreq, const double *u0, const double *f,
                                const double *fscale, double tol, int max_iter, double *U,
                                int *iters_host, double *incr_host, double *apost_host);


/* Independent Parareal problems solved together (problems of uneven grid
 * size, slice count, rank and request count): per problem, the arguments of
 * lrpr_parareal_solve.  Every iteration runs the fine solves of all
 * problems, slices and requests as one batched sweep launch, then each
 * problem's sequential coarse correction; with implicit-Euler factors the
 * iteration is captured once in a HIP graph and replayed
 * (LRPR_TUNE_PARAREAL_GRAPH).  A problem stops when its own requests have
 * converged or reached its own cap; its results are the same bit for bit as
 * when it is solved alone. */
typedef struct {
    lrpr_coarse C;            /* coarse propagators of the problem's N slices */
    const lrpr_fac *F;        /* host array of N factors (slice n uses F[n-1]) */
    int nreq;                 /* requests sharing the operators */
    const double *u0;         /* device, n x nreq */
    const double *f;          /* device, n x nreq sources, or NULL */
    const double *fscale;     /* device, N*nsteps time factors, or NULL */
    double tol;
    int max_iter;
    double *U;                /* device output, nreq blocks of n x (N+1) */
    int *iters_host;          /* host int[nreq] */
    double *incr_host;        /* host double[nreq*max_iter] or NULL */
    double *apost_host;       /* host double[nreq*N] or NULL */
} lrpr_parareal_problem;

/* Solve nprob problems together (all with nsteps fine steps per slice of
 * one stepper and fine precision).  Outputs per problem as in
 * lrpr_parareal_solve.  Returns LRPR_ERR_NOCONV (all outputs written) if a
 * problem did not reach its tolerance; LRPR_ERR_NONFINITE on a non-finite
 * increment.  Synchronises. */
lrpr_status lrpr_parareal_solve_many(lrpr_ctx ctx, int nprob, const lrpr_parareal_problem *probs, int nsteps,
                                     lrpr_prec fine_prec);

/* ---- serving: continuous batching of Parareal solves (Sec. 2) ----------- */

/* The coarse propagators depend on the source only through b_n = F_n 0
 * (eq. F_n_affine, eq. spectral_G), so the device-resident U_k, S_k, V_k of
 * an operator serve every request that brings a new initial value and
 * source.  The server runs the iteration of eq. def_Parareal per request
 * (FP64 fine steps) and batches all requests of an operator into one fine
 * sweep and one coarse sweep per step; requests that arrive while a step is
 * on the GPU join the operator's next step.  Operators step independently
 * on their own streams.  A request's result does not depend on which other
 * requests share its steps: every column's arithmetic is independent of the
 * others, and on factors that keep spikes the fine sweeps take the
 * partitioned passes at any batch width.
 *
 * Threading: one host thread per server.  Calls that overlap on one server
 * are not supported. */
typedef struct lrpr_server_s *lrpr_server;

typedef struct {
    lrpr_coarse C;          /* coarse propagators of the operator's N slices */
    const lrpr_fac *F;      /* host array of N factor handles (may alias one;
                               must keep FP64 tiles, implicit-Euler stepper);
                               read at create time */
    int nsteps;             /* implicit-Euler steps per slice */
    const double *fscale;   /* device, N*nsteps source time factors (as in
                               lrpr_parareal_solve) or NULL (= 1); copied */
} lrpr_serve_op;

/* budget_bytes bounds the server's per-request device state (2*N*n doubles
 * per admitted request); requests wait in a FIFO per operator until their
 * state fits.  max_active_per_op caps the requests per step of one operator
 * (0: as many as the coarse kernel takes, 12288/k).  The handles in ops must
 * outlive the server.  Errors: LRPR_ERR_ARG, LRPR_ERR_NOMEM, LRPR_ERR_HIP. */
lrpr_status lrpr_server_create(lrpr_ctx ctx, int nops, const lrpr_serve_op *ops, double tol,
                               size_t budget_bytes, int max_active_per_op, lrpr_server *out);
/* Synchronises the server's streams and frees everything it owns. */
void lrpr_server_destroy(lrpr_server s);
/* Queue a request for operator op: u0 and f device vectors (n, FP64), U the
 * device output (n x (N+1), FP64, column s = u_s).  All three are caller
 * memory that must stay valid until the request is reported done; U holds
 * the last iterate then.  No GPU work is done here.  *id is the request's
 * handle in lrpr_server_progress.  Errors: LRPR_ERR_ARG, LRPR_ERR_NOMEM
 * (the request alone exceeds the budget). */
lrpr_status lrpr_server_submit(lrpr_server s, int op, const double *u0, const double *f, double *U,
                               int64_t *id);
/* Advance the server: finish steps that completed, admit queued requests,
 * launch the next step of every idle operator with work.  wait != 0 blocks
 * until at least one step completes (if any is in flight).  Returns up to
 * max_done completed requests (ids and iteration counts; -1 for a request
 * whose increments became non-finite); the others are returned by later
 * calls. */
lrpr_status lrpr_server_progress(lrpr_server s, int wait, int max_done, int64_t *done_ids, int *done_iters,
                                 int *ndone);
/* Requests queued / in the current steps, and the budgeted bytes in use. */
lrpr_status lrpr_server_stats(lrpr_server s, int *queued, int *active, int64_t *bytes_in_use);
const char *lrpr_server_last_error(lrpr_server s);

#ifdef __cplusplus
}
#endif
#endif /* LRPR_H */
