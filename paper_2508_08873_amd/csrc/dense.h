// Job descriptors and launchers of the dense kernels (dense.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lrpr {

constexpr int LMAX = 96;   // largest l = k + p handled by the small dense kernels

struct GramJob {           // G = A^T A, A n x l column-major (ld n)
    const void *A;
    int64_t n;
    int l;
    int pad_;
};

struct RowMatJob {         // C = A B; A n x l (ld lda), B l x nc (FP64, row-major ld LMAX)
    const void *A;
    int64_t lda;
    const double *B;
    void *C;
    int64_t ldc;
    int64_t n;
    int l, nc;
    int upper;
    int pad_;
};

struct HouseJob {          // Householder QR of A (n x l, FP64, destroyed)
    double *A;
    double *Q;             // n x l
    double *R;             // LMAX x LMAX row-major
    int64_t n;
    int l;
    int pad_;
};

struct SignJob {           // sign normalisation of U[:, r], V[:, r], r < k
    double *U, *V;
    int64_t n;
    int k;
    int pad_;
};

struct LrArgs {            // low-rank apply / Parareal correction on w columns
    const double *U, *S, *V;   // n x k, k, n x k
    const double *x;           // input vectors (n x w)
    double *out;               // output / iterate u (n x w)
    double *gold;              // cached G' u of the previous sweep (n x w)
    const double *bvec;        // b_n (n x w), mode 1
    const double *fu64;        // F_n u (n x w), mode 2 (FP64) ...
    const float *fu32;         // ... or FP32
    const int *active;         // per column flag, or null
    double *part;              // [chunks][k*w], then k*w coefficients (lr_part_elems)
    double *coef;              // set by launch_lowrank
    double *incpart;           // [chunks][w]
    int64_t n;
    int k, w;
    int mode;
    int pad_;
    // Column tables (used when cu != null, modes 1 and 2 per column): column
    // c works on slice s of its own request, x = cu[c] + coff, out = cu[c] +
    // coff + n, gold = cgold[c] + coff, bvec = Fu = cfu[c] + coff (FP64),
    // mode = cmode[c] (0 = leave the column untouched).
    double *const *cu;
    double *const *cgold;
    const double *const *cfu;
    const int *cmode;
    int64_t coff;
};

// Low-rank apply / Parareal correction over a.w columns (api_rsvd.cpp), in
// passes of at most 12288/k columns; part holds lr_part_elems(n, k, min(w,
// 12288/k)) doubles, incpart (or null) [chunks][w] increment partials.
hipError_t lowrank_cols(LrArgs a, double *part, double *incpart, hipStream_t s);
int gram_chunks(int64_t nmax);
int64_t lr_chunks(int64_t n);
// doubles of the part workspace of a low-rank apply of rank k on w columns
int64_t lr_part_elems(int64_t n, int k, int w);
hipError_t launch_gram(bool f32, const GramJob *d_jobs, int njobs, int nchunks, double *part, double *G,
                       hipStream_t s);
hipError_t launch_chol(const int *d_ls, int nslices, const double *G, double *R, double *Rinv, int *status,
                       double cond_tol, hipStream_t s);
hipError_t launch_rowmat(int ta, int tc, const RowMatJob *d_jobs, int njobs, int64_t nmax, hipStream_t s);
hipError_t launch_householder(const HouseJob *d_jobs, int njobs, hipStream_t s);
hipError_t launch_jacobi(const int *d_ls, int nslices, int lmax, const double *Mm, double *Uh, double *S,
                         double *Vh, int *sweeps, hipStream_t s);
hipError_t launch_signfix(const SignJob *d_jobs, int njobs, int kmax, hipStream_t s);
hipError_t launch_lowrank(const LrArgs &a, hipStream_t s);
hipError_t launch_inc_reduce(const double *incpart, int64_t nch, int w, double *inc2, hipStream_t s);
hipError_t launch_convert(int from, int to, const void *src, void *dst, int64_t count, hipStream_t s);
hipError_t launch_fill(double *dst, int64_t count, double v, hipStream_t s);
hipError_t launch_fillf(float *dst, int64_t count, float v, hipStream_t s);
hipError_t launch_trmm_upper(const int *d_ls, int nslices, const double *R2, const double *R1, double *R,
                             hipStream_t s);
hipError_t launch_transpose_small(const int *d_ls, int nslices, const double *R, double *Mm, hipStream_t s);
// B = C^{-T} per slice (C row-major ld l, B row-major ld LMAX, both at s*LMAX*LMAX); status[s] = 1 if singular
hipError_t launch_small_inv_t(const int *d_ls, int nslices, int lmax, const double *C, double *B, int *status,
                              hipStream_t s);
// out[r*w + c] = sum_i V[i][r] X[i][c] (V: n x k, X: n x w, FP64 column-major ld n); ones: >= k ones;
// part: lr_part_elems(n, k, w) doubles
hipError_t launch_cross_gram(const double *V, const double *X, int64_t n, int k, int w, const double *ones,
                             double *part, double *out, hipStream_t s);

// X[i, :] *= sqrt(w_i) (up) or /= sqrt(w_i); X n x cols column-major, ld n
hipError_t launch_row_scale(bool f32, void *X, int64_t n, int64_t cols, const double *w, bool up, hipStream_t s);

}  // namespace lrpr
