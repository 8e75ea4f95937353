// Tall-skinny and small dense kernels of the randomized SVD (Sec. 2.1
// steps 2, 4, 5, 6) and of the Parareal correction sweep (Sec. 2, eq.
// def_Parareal; G_n' from eq. spectral_G).  Everything here accumulates in
// FP64; inputs of the range finder may be FP32.
#include "lrpr_internal.h"
#include <algorithm>

#include "dense.h"

namespace lrpr {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline double ld_as_double(const double *p, int64_t i) { return p[i]; }
__device__ inline double ld_as_double(const float *p, int64_t i) { return (double)p[i]; }

// ---------------------------------------------------------------------------
// Gram partials: part[s][chunk] = A_chunk^T A_chunk (l x l, upper 16x16 tiles)
// for A = slice s's n x l matrix (column-major, ld n).  A 64-row block of A
// is staged in LDS as FP64; each wave owns a set of 16x16 output tiles and
// accumulates them with v_mfma_f64_16x16x4 over the chunk's rows.
// ---------------------------------------------------------------------------
constexpr int GRAM_ROWS = 64;
constexpr int GRAM_CHUNK = 4096;

template <typename T>
__global__ __launch_bounds__(256) void k_gram_partial(const GramJob *jobs, int njobs, double *part) {
    __shared__ double blk[GRAM_ROWS * (LMAX + 2)];
    const GramJob jb = jobs[blockIdx.y];
    const int chunk = blockIdx.x;
    const int64_t r0 = (int64_t)chunk * GRAM_CHUNK;
    if (r0 >= jb.n) return;
    const int64_t r1 = (r0 + GRAM_CHUNK < jb.n) ? r0 + GRAM_CHUNK : jb.n;
    const int l = jb.l;
    const int lt = (l + 15) / 16;
    const int ldb = LMAX + 2;
    const T *A = (const T *)jb.A;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    // tiles (ti <= tj) assigned round-robin to the 4 waves, at most 36/4 -> LT_MAX
    constexpr int MAXT = (LMAX / 16) * (LMAX / 16 + 1) / 2;
    constexpr int PERW = (MAXT + 3) / 4;
    d4 acc[PERW];
    int tij[PERW];
    int nt = 0;
    {
        int idx = 0;
        for (int ti = 0; ti < lt; ++ti)
            for (int tj = ti; tj < lt; ++tj, ++idx)
                if ((idx & 3) == w && nt < PERW) tij[nt++] = ti * 16 + tj;
    }
#pragma unroll
    for (int t = 0; t < PERW; ++t) acc[t] = d4{0, 0, 0, 0};
    for (int64_t rb = r0; rb < r1; rb += GRAM_ROWS) {
        __syncthreads();
        for (int e = threadIdx.x; e < GRAM_ROWS * lt * 16; e += 256) {
            const int rr = e % GRAM_ROWS, cc = e / GRAM_ROWS;
            const int64_t row = rb + rr;
            double v = 0.0;
            if (row < r1 && cc < l) v = ld_as_double(A, row + (int64_t)cc * jb.n);
            blk[rr * ldb + cc] = v;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < PERW; ++t) {
            if (t < nt) {
                const int ti = tij[t] / 16, tj = tij[t] % 16;
#pragma unroll 4
                for (int kc = 0; kc < GRAM_ROWS / 4; ++kc) {
                    const int rr = 4 * kc + g;
                    const double a = blk[rr * ldb + 16 * ti + c];
                    const double b = blk[rr * ldb + 16 * tj + c];
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
                }
            }
        }
    }
    double *P = part + ((int64_t)blockIdx.y * gridDim.x + chunk) * (LMAX * LMAX);
#pragma unroll
    for (int t = 0; t < PERW; ++t) {
        if (t < nt) {
            const int ti = tij[t] / 16, tj = tij[t] % 16;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = 4 * i + g;   // f64 D layout: row 4i + lane/16
                P[(16 * ti + m) * LMAX + 16 * tj + c] = acc[t][i];
            }
        }
    }
}

// G[s] (l x l, ld LMAX) = sum over chunks (fixed order), symmetrised.
__global__ void k_gram_reduce(const GramJob *jobs, int nchunks, const double *part, double *G) {
    const GramJob jb = jobs[blockIdx.x];
    const int l = jb.l;
    const int64_t used = (jb.n + GRAM_CHUNK - 1) / GRAM_CHUNK;
    for (int e = threadIdx.x; e < l * l; e += blockDim.x) {
        const int i = e / l, j = e % l;
        const int a = i < j ? i : j, b = i < j ? j : i;
        double s = 0.0;
        for (int64_t ch = 0; ch < used; ++ch)
            s += part[((int64_t)blockIdx.x * nchunks + ch) * (LMAX * LMAX) + a * LMAX + b];
        G[(int64_t)blockIdx.x * LMAX * LMAX + i * LMAX + j] = s;
    }
}

// ---------------------------------------------------------------------------
// Cholesky G = R^T R (R upper, FP64) of one l x l Gram matrix per workgroup,
// then Rinv = R^{-1} (one thread per column, back substitution).
// status[s]: 0 ok; 1 breakdown (non-positive/non-finite pivot or
// min_j R_jj < cond_tol * max_j R_jj).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chol(const int *ls, const double *G, double *R, double *Rinv,
                                              int *status, double cond_tol) {
    __shared__ double a[LMAX * LMAX];
    __shared__ int bad;
    const int s = blockIdx.x;
    const int l = ls[s];
    const double *Gs = G + (int64_t)s * LMAX * LMAX;
    for (int e = threadIdx.x; e < LMAX * LMAX; e += blockDim.x) a[e] = Gs[e];
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < l; ++j) {
        const double d = a[j * LMAX + j];
        if (!(d > 0.0) || !isfinite(d)) {
            if (threadIdx.x == 0) bad = 1;
            break;
        }
        const double r = sqrt(d);
        __syncthreads();
        if (threadIdx.x == 0) a[j * LMAX + j] = r;
        for (int k = j + 1 + threadIdx.x; k < l; k += blockDim.x) a[j * LMAX + k] /= r;
        __syncthreads();
        const int m = l - j - 1;
        for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
            const int i = j + 1 + e / m, k = j + 1 + e % m;
            if (k >= i) a[i * LMAX + k] -= a[j * LMAX + i] * a[j * LMAX + k];
        }
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0 && !bad) {
        double mx = 0, mn = 1e300;
        for (int j = 0; j < l; ++j) {
            const double v = a[j * LMAX + j];
            mx = v > mx ? v : mx;
            mn = v < mn ? v : mn;
        }
        if (!(mn >= cond_tol * mx)) bad = 1;
    }
    __syncthreads();
    double *Rs = R + (int64_t)s * LMAX * LMAX;
    double *Is = Rinv + (int64_t)s * LMAX * LMAX;
    for (int e = threadIdx.x; e < LMAX * LMAX; e += blockDim.x) {
        const int i = e / LMAX, k = e % LMAX;
        Rs[e] = (i < l && k < l && k >= i) ? a[e] : 0.0;
    }
    if (threadIdx.x == 0) status[s] = bad;
    if (bad) return;
    // column jc of Rinv: R x = e_jc, back substitution
    for (int jc = threadIdx.x; jc < LMAX; jc += blockDim.x) {
        for (int i = LMAX - 1; i >= 0; --i) {
            double v = 0.0;
            if (jc < l && i <= jc) {
                v = (i == jc) ? 1.0 : 0.0;
                for (int k = i + 1; k <= jc; ++k) v -= a[i * LMAX + k] * Is[k * LMAX + jc];
                v /= a[i * LMAX + i];
            }
            Is[i * LMAX + jc] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// C = A B for every job: A n x l (type TA, ld lda), B l x nc (FP64, row-major
// ld LMAX), C n x nc (type TC, ld ldc).  B is staged in LDS; one thread per
// row; outputs in chunks of 32 columns.  With upper != 0, B is upper
// triangular (only k <= j terms are summed).
// ---------------------------------------------------------------------------
// C = A B on the matrix cores, as C^T tiles: B^T (16 columns x 4 of l, from
// LDS) times A^T (4 of l x 16 rows, read along the rows of A), so a lane ends
// with one row of four output columns and the stores run along the rows.
// Each wave takes 64 of a workgroup's 256 rows (four tiles of 16) and every
// column tile of the output; with `upper` (B upper triangular) the products
// past a column tile's last column are skipped (they are zero).
constexpr int RM_ROWS = 256;   // rows per workgroup pass
constexpr int RM_CT = LMAX / 16;   // most column tiles
constexpr int RM_LD = LMAX + 2;    // LDS row stride of B (rows k and k+1 on different banks)

template <typename TA, typename TC>
__global__ __launch_bounds__(256, 2) void k_rowmat(const RowMatJob *jobs) {
    __shared__ double Bs[LMAX * RM_LD];
    const RowMatJob jb = jobs[blockIdx.y];
    {   // rows k < l of B (the only ones read), four loads in flight per thread
        const int tot = jb.l * LMAX;
        for (int e0 = 0; e0 < tot; e0 += 4 * (int)blockDim.x) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * (int)blockDim.x + (int)threadIdx.x;
                v[u] = e < tot ? jb.B[e] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * (int)blockDim.x + (int)threadIdx.x;
                if (e < tot) Bs[(e / LMAX) * RM_LD + e % LMAX] = v[u];
            }
        }
    }
    __syncthreads();
    const TA *A = (const TA *)jb.A;
    TC *C = (TC *)jb.C;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, nr = lane & 15;
    const int l = jb.l, nc = jb.nc, nct = (nc + 15) / 16;
    for (int64_t base = (int64_t)blockIdx.x * RM_ROWS; base < jb.n; base += (int64_t)gridDim.x * RM_ROWS) {
        for (int q = 0; q < RM_ROWS / 64; ++q) {
            const int64_t row = base + (int64_t)(wv * (RM_ROWS / 64) + q) * 16 + nr;
            typedef double v4 __attribute__((ext_vector_type(4)));
            v4 acc[RM_CT];
#pragma unroll
            for (int t = 0; t < RM_CT; ++t) acc[t] = v4{0, 0, 0, 0};
            // the k range that any column tile reads; this lane's values of A
            // for every k step are loaded first, all in flight together
            const int kend = jb.upper ? (nct * 16 < l ? nct * 16 : l) : l;
            // (unconditional loads of clamped, valid addresses: a load under
            // a lane condition would be waited for before the next one)
            typedef __attribute__((address_space(1))) const TA *gA;
            const int64_t rc = row < jb.n ? row : jb.n - 1;
            TA raw[LMAX / 4];
#pragma unroll
            for (int ks = 0; ks < LMAX / 4; ++ks) {
                const int k = 4 * ks + g < l ? 4 * ks + g : l - 1;
                if (4 * ks < kend) raw[ks] = *(gA)(A + rc + (int64_t)k * jb.lda);
            }
            // (rows past n read row n-1 and k past l read column l-1: finite
            // values that meet only zero entries of B or land in rows that
            // are not stored)
#pragma unroll
            for (int ks = 0; ks < LMAX / 4; ++ks) {
                if (4 * ks < kend) {
                    const int k = 4 * ks + g;
#pragma unroll
                    for (int t = 0; t < RM_CT; ++t) {
                        if (t < nct && !(jb.upper && 4 * ks > 16 * t + 15)) {
                            const int col = 16 * t + nr;
                            const double av = (k < l && col < nc) ? Bs[k * RM_LD + col] : 0.0;
                            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, (double)raw[ks], acc[t], 0, 0, 0);
                        }
                    }
                }
            }
            // element (column 16 t + 4 reg + g, row) in register reg of tile t
            if (row < jb.n) {
#pragma unroll
                for (int t = 0; t < RM_CT; ++t) {
                    if (t < nct) {
#pragma unroll
                        for (int reg = 0; reg < 4; ++reg) {
                            const int col = 16 * t + 4 * reg + g;
                            if (col < nc) C[row + (int64_t)col * jb.ldc] = (TC)acc[t][reg];
                        }
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Householder QR (fallback for numerically rank-deficient panels): one
// workgroup per job, A (n x l, FP64, in place) -> reflectors; writes R
// (row-major ld LMAX, R_jj >= 0) and Q (n x l, FP64) explicitly.
// ---------------------------------------------------------------------------
__device__ double block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}

__global__ __launch_bounds__(1024) void k_householder(const HouseJob *jobs) {
    __shared__ double red[16];
    __shared__ double beta_s[LMAX];
    __shared__ double rdiag[LMAX];
    const HouseJob jb = jobs[blockIdx.x];
    double *A = jb.A;
    const int64_t n = jb.n;
    const int l = jb.l;
    for (int j = 0; j < l; ++j) {
        double *a = A + (int64_t)j * n;
        double ss = 0.0;
        for (int64_t i = j + threadIdx.x; i < n; i += blockDim.x) ss += a[i] * a[i];
        const double nrm2 = block_sum(ss, red);
        const double nrm = sqrt(nrm2);
        const double ajj = a[j];
        __syncthreads();
        if (nrm == 0.0) {
            if (threadIdx.x == 0) { beta_s[j] = 0.0; rdiag[j] = 0.0; }
            __syncthreads();
            continue;
        }
        const double alpha = ajj >= 0 ? -nrm : nrm;
        const double v0 = ajj - alpha;
        const double vv = nrm2 - ajj * ajj + v0 * v0;
        const double beta = vv > 0 ? 2.0 / vv : 0.0;
        if (threadIdx.x == 0) { a[j] = v0; beta_s[j] = beta; rdiag[j] = alpha; }
        __syncthreads();
        for (int cc = j + 1; cc < l; ++cc) {
            double *ac = A + (int64_t)cc * n;
            double d = 0.0;
            for (int64_t i = j + threadIdx.x; i < n; i += blockDim.x) d += a[i] * ac[i];
            const double sdot = block_sum(d, red) * beta;
            for (int64_t i = j + threadIdx.x; i < n; i += blockDim.x) ac[i] -= sdot * a[i];
            __syncthreads();
        }
    }
    // R: strictly upper part from A, diagonal from rdiag; then Q
    double *R = jb.R;
    for (int e = threadIdx.x; e < LMAX * LMAX; e += blockDim.x) {
        const int r = e / LMAX, cc = e % LMAX;
        double v = 0.0;
        if (r < l && cc < l) {
            if (cc > r) v = A[r + (int64_t)cc * n];
            else if (cc == r) v = rdiag[r];
        }
        R[e] = v;
    }
    double *Q = jb.Q;
    for (int cc = 0; cc < l; ++cc)
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) Q[i + (int64_t)cc * n] = (i == cc) ? 1.0 : 0.0;
    __syncthreads();
    for (int j = l - 1; j >= 0; --j) {
        const double beta = beta_s[j];
        if (beta == 0.0) continue;
        const double *v = A + (int64_t)j * n;   // v_j = a[j] (modified), v_i = a[i], i > j
        for (int cc = j; cc < l; ++cc) {
            double *qc = Q + (int64_t)cc * n;
            double d = 0.0;
            for (int64_t i = j + threadIdx.x; i < n; i += blockDim.x) d += v[i] * qc[i];
            const double sdot = block_sum(d, red) * beta;
            for (int64_t i = j + threadIdx.x; i < n; i += blockDim.x) qc[i] -= sdot * v[i];
            __syncthreads();
        }
    }
    // sign normalisation R_jj >= 0
    for (int j = 0; j < l; ++j) {
        if (rdiag[j] < 0) {
            for (int cc = j + threadIdx.x; cc < l; cc += blockDim.x) R[j * LMAX + cc] = -R[j * LMAX + cc];
            for (int64_t i = threadIdx.x; i < n; i += blockDim.x) Q[i + (int64_t)j * n] = -Q[i + (int64_t)j * n];
        }
    }
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of M (l x l, row-major ld LMAX) per
// workgroup: Mm = Uh diag(S) Vh^T, S descending.  Columns of M and of V are
// held in LDS; a sweep visits all column pairs in l-1 rounds of l/2 disjoint
// pairs (round-robin), 16 lanes per pair; a pair is rotated when
// |a_p.a_q| > l*eps*||a_p|| ||a_q||.  Sweeps until no rotation happens.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_jacobi(const int *ls, const double *Mm, double *Uh, double *S,
                                                 double *Vh, int *sweeps_out) {
    extern __shared__ double jsm[];
    const int s = blockIdx.x;
    const int l = ls[s];
    const int le = (l + 1) & ~1;   // even count (a zero column pads odd l)
    double *A = jsm;               // column c at A + c*le
    double *V = jsm + le * le;
    __shared__ int rotated;
    __shared__ int order[LMAX + 1];
    __shared__ double nrm[LMAX + 1];
    const double *Ms = Mm + (int64_t)s * LMAX * LMAX;
    for (int e = threadIdx.x; e < le * le; e += blockDim.x) {
        const int r = e % le, cc = e / le;
        A[e] = (r < l && cc < l) ? Ms[r * LMAX + cc] : 0.0;
        V[e] = (r == cc) ? 1.0 : 0.0;
    }
    const double tol = (double)l * 2.220446049250313e-16;
    const int pair = threadIdx.x >> 4, sub = threadIdx.x & 15;
    const int npairs = le / 2;
    int sweep = 0;
    for (; sweep < 60; ++sweep) {
        if (threadIdx.x == 0) rotated = 0;
        __syncthreads();
        for (int round = 0; round < le - 1; ++round) {
            if (pair < npairs) {
                int p, q;
                if (pair == 0) {
                    p = 0;
                    q = 1 + round % (le - 1);
                } else {
                    p = 1 + (round + pair) % (le - 1);
                    q = 1 + (round - pair + le - 1) % (le - 1);
                }
                if (p > q) { const int t = p; p = q; q = t; }
                double *ap = A + p * le, *aq = A + q * le;
                double al = 0, be = 0, ga = 0;
                for (int r = sub; r < le; r += 16) {
                    al += ap[r] * ap[r];
                    be += aq[r] * aq[r];
                    ga += ap[r] * aq[r];
                }
                for (int o = 8; o > 0; o >>= 1) {
                    al += __shfl_xor(al, o, 16);
                    be += __shfl_xor(be, o, 16);
                    ga += __shfl_xor(ga, o, 16);
                }
                if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                    for (int r = sub; r < le; r += 16) {
                        const double x = ap[r], y = aq[r];
                        ap[r] = cs * x - sn * y;
                        aq[r] = sn * x + cs * y;
                    }
                    double *vp = V + p * le, *vq = V + q * le;
                    for (int r = sub; r < le; r += 16) {
                        const double x = vp[r], y = vq[r];
                        vp[r] = cs * x - sn * y;
                        vq[r] = sn * x + cs * y;
                    }
                    if (sub == 0) rotated = 1;
                }
            }
            __syncthreads();
        }
        if (!rotated) break;
        __syncthreads();
    }
    // norms and descending order (stable: lower index first on ties)
    for (int cc = threadIdx.x; cc < le; cc += blockDim.x) {
        double ss = 0;
        for (int r = 0; r < le; ++r) ss += A[cc * le + r] * A[cc * le + r];
        nrm[cc] = sqrt(ss);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < l; ++i) order[i] = i;
        for (int a = 0; a < l; ++a) {
            int best = a;
            for (int b = a + 1; b < l; ++b)
                if (nrm[order[b]] > nrm[order[best]]) best = b;
            const int t = order[a]; order[a] = order[best]; order[best] = t;
        }
        sweeps_out[s] = sweep < 60 ? sweep + 1 : -1;
    }
    __syncthreads();
    double *Us = Uh + (int64_t)s * LMAX * LMAX, *Vs = Vh + (int64_t)s * LMAX * LMAX, *Ss = S + (int64_t)s * LMAX;
    for (int e = threadIdx.x; e < LMAX * LMAX; e += blockDim.x) {
        const int r = e / LMAX, a = e % LMAX;   // row-major (r, a): column a of Uh
        double u = 0.0, v = 0.0;
        if (r < l && a < l) {
            const int cc = order[a];
            const double nv = nrm[cc];
            u = nv > 0 ? A[cc * le + r] / nv : 0.0;
            v = V[cc * le + r];
        }
        Us[e] = u;
        Vs[e] = v;
    }
    for (int a = threadIdx.x; a < LMAX; a += blockDim.x) Ss[a] = a < l ? nrm[order[a]] : 0.0;
}

// ---------------------------------------------------------------------------
// Sign normalisation: for column r of U (n x k, ld n) find the entry of
// largest magnitude (lowest index on ties); if negative flip U[:,r] and
// V[:,r].  One workgroup per (job, column).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_signfix(const SignJob *jobs) {
    __shared__ double bv[256];
    __shared__ int64_t bi[256];
    const SignJob jb = jobs[blockIdx.y];
    const int r = blockIdx.x;
    if (r >= jb.k) return;
    double *u = jb.U + (int64_t)r * jb.n;
    double *v = jb.V + (int64_t)r * jb.n;
    double best = -1.0;
    int64_t bidx = 0;
    for (int64_t i = threadIdx.x; i < jb.n; i += blockDim.x) {
        const double a = fabs(u[i]);
        if (a > best) { best = a; bidx = i; }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double b2 = bv[threadIdx.x + o];
            const int64_t i2 = bi[threadIdx.x + o];
            if (b2 > bv[threadIdx.x] || (b2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
                bv[threadIdx.x] = b2;
                bi[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    const bool flip = u[bi[0]] < 0;
    __syncthreads();
    if (flip) {
        for (int64_t i = threadIdx.x; i < jb.n; i += blockDim.x) {
            u[i] = -u[i];
            v[i] = -v[i];
        }
    }
}

// ---------------------------------------------------------------------------
// Low-rank apply and Parareal correction.
//   dots:    part[chunk][r][c] = sum_{i in chunk} V[i][r] * x[i][c]
//   coef:    coef[r][c] = S[r] * sum over chunks of part (fixed order)
//   combine: g = U coef;  then either out = g, or the correction
//            u_new = Fu + g - gold, gold = g, with per-chunk partial sums of
//            ||u_new - u_old||^2 for the increment.
// x, out, Fu, gold, u: n x w column-major (ld n).  Chunks are 256 rows, so
// that a 65025-row slice spreads over 255 workgroups; every reduction runs in
// a fixed order, independent of w and of the other columns.
// ---------------------------------------------------------------------------
constexpr int LR_CHUNK = 256;
constexpr int LR_THREADS = 256;
constexpr int LR_RED = 16;  // waves of the chunk reductions

typedef double lr_v4d __attribute__((ext_vector_type(4)));
constexpr int LR_SUB = 32;   // chunk rows staged in LDS per pass (dots)
constexpr int LR_WC = 64;    // columns per pass (dots)

// part[chunk][r*w + c] = sum over the chunk's rows of V[i][r] x[i][c], on the
// matrix cores: output tiles of 16 ranks x 16 columns, each accumulating
// V^T (16 x 4) times x (4 x 16) over the chunk's rows in order (4 rows per
// product).  The chunk's rows pass through LDS 32 at a time (loads along the
// columns, consecutive threads on consecutive rows).  An output element sums
// only its own rank's and column's products, in an order fixed by the row
// index, so it does not depend on w or on the other columns.
__global__ __launch_bounds__(LR_THREADS) void k_lr_dots(LrArgs a) {
    __shared__ double Vs[LR_SUB][LMAX + 1];
    __shared__ double Xs[LR_SUB][LR_WC + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = lane >> 4, m = lane & 15;
    const int64_t i0 = (int64_t)blockIdx.x * LR_CHUNK;
    const int K = a.k, W = a.w, nk = K * W;
    const int RT = (K + 15) / 16;
    constexpr int TPW = (LMAX / 16) * (LR_WC / 16) / (LR_THREADS / 64);   // output tiles per wave
    for (int cb = 0; cb < W; cb += LR_WC) {
        const int wc = W - cb < LR_WC ? W - cb : LR_WC;
        const int CT = (wc + 15) / 16, ntile = RT * CT;
        lr_v4d acc[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[t] = lr_v4d{0, 0, 0, 0};
        for (int sub = 0; sub < LR_CHUNK; sub += LR_SUB) {
            for (int e = tid; e < LR_SUB * K; e += LR_THREADS) {
                const int r = e / LR_SUB, ii = e % LR_SUB;
                const int64_t i = i0 + sub + ii;
                Vs[ii][r] = i < a.n ? a.V[i + (int64_t)r * a.n] : 0.0;
            }
            for (int e = tid; e < LR_SUB * wc; e += LR_THREADS) {
                const int c = e / LR_SUB, ii = e % LR_SUB;
                const int64_t i = i0 + sub + ii;
                Xs[ii][c] = i >= a.n ? 0.0 : a.cu ? a.cu[cb + c][a.coff + i] : a.x[i + (int64_t)(cb + c) * a.n];
            }
            __syncthreads();
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int tt = wv + (LR_THREADS / 64) * t;
                if (tt < ntile) {
                    const int r = (tt / CT) * 16 + m, c = (tt % CT) * 16 + m;
                    // A[m][kk] = V[row kk][rank m] in lane m + 16 kk; B[kk][n] = x[row kk][column n]
#pragma unroll
                    for (int ks = 0; ks < LR_SUB / 4; ++ks) {
                        const int row = 4 * ks + g;
                        const double av = r < K ? Vs[row][r] : 0.0;
                        const double bv = c < wc ? Xs[row][c] : 0.0;
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
                    }
                }
            }
            __syncthreads();
        }
        // D[mm][n] in lane n + 16 (mm % 4), register mm / 4
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int tt = wv + (LR_THREADS / 64) * t;
            if (tt < ntile) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int r = (tt / CT) * 16 + 4 * q + g, c = (tt % CT) * 16 + m;
                    if (r < K && c < wc) a.part[(int64_t)blockIdx.x * nk + r * W + cb + c] = acc[t][q];
                }
            }
        }
    }
}

// coef[e] = S[e / w] * sum over the nch chunks of part[ch][e]: 64 entries per
// workgroup (one per lane), LR_RED waves take the chunks round-robin, the
// wave partials add up in wave order.
__global__ __launch_bounds__(64 * LR_RED) void k_lr_coef(const double *part, int64_t nch, int nk, int w,
                                                         const double *S, double *coef) {
    __shared__ double red[LR_RED][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    double sum = 0.0;
    if (e < nk)
        for (int64_t ch = wv; ch < nch; ch += LR_RED) sum += part[ch * nk + e];
    red[wv][lane] = sum;
    __syncthreads();
    if (wv == 0 && e < nk) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < LR_RED; ++q) t += red[q][lane];
        coef[e] = S[e / w] * t;
    }
}

// g = U coef for the block's rows; mode 0: out = g; mode 1 (Parareal
// initialisation): gold = g, out = g + bvec; mode 2 (correction):
// u_new = Fu + g - gold, incpart += ||u_new - out||^2, out = u_new, gold = g.
// Columns with active[c] == 0 are left untouched (modes 1, 2).  With column
// tables the mode is per column (and 0 means untouched); increments are
// written for every column (zero unless mode 2).
// On the matrix cores: each wave takes 64 of the chunk's rows (4 tiles of 16)
// and forms g^T tile by tile, coef^T (16 columns x 4 ranks, from LDS) times
// U^T (4 ranks x 16 rows, read along the rows), so that a lane ends with one
// row of four columns and the epilogue reads and writes along the rows.
// Every element's sum and every increment's order are fixed by the rank and
// row indices alone.
__global__ __launch_bounds__(LR_THREADS) void k_lr_combine(LrArgs a) {
    extern __shared__ double coef[];   // [k*w]
    __shared__ double red[LR_THREADS / 64][16];
    const int K = a.k, W = a.w, nk = K * W;
    for (int e = threadIdx.x; e < nk; e += LR_THREADS) coef[e] = a.coef[e];
    __syncthreads();
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = lane >> 4, nr = lane & 15;
    const int64_t i0 = (int64_t)blockIdx.x * LR_CHUNK;
    const bool incs = a.mode == 2 || a.cu;
    for (int c0 = 0; c0 < W; c0 += 16) {
        double incv[4] = {0.0, 0.0, 0.0, 0.0};
        for (int q = 0; q < LR_CHUNK / 64; ++q) {
            const int64_t rbase = i0 + (int64_t)(wv * (LR_CHUNK / 64) + q) * 16;
            lr_v4d acc = {0, 0, 0, 0};
            // this lane's U values for every rank step, all loads in flight
            const int64_t iu = rbase + nr;
            const int64_t iuc = iu < a.n ? iu : a.n - 1;
            typedef __attribute__((address_space(1))) const double *gD;
            double raw[LMAX / 4];
#pragma unroll
            for (int ks = 0; ks < LMAX / 4; ++ks) {
                const int r = 4 * ks + g < K ? 4 * ks + g : K - 1;
                if (4 * ks < K) raw[ks] = *(gD)(a.U + iuc + (int64_t)r * a.n);
            }
            // (rows past n read row n-1 and ranks past k rank k-1: finite
            // values that meet zero coefficients or land in rows not written)
#pragma unroll
            for (int ks = 0; ks < LMAX / 4; ++ks) {
                if (4 * ks < K) {
                    const int r = 4 * ks + g;
                    const double av = (r < K && c0 + nr < W) ? coef[r * W + c0 + nr] : 0.0;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, raw[ks], acc, 0, 0, 0);
                }
            }
            // element (column c0 + 4 reg + g, row rbase + nr) in register reg
            const int64_t i = rbase + nr;
            if (i >= a.n) continue;
#pragma unroll
            for (int reg = 0; reg < 4; ++reg) {
                const int c = c0 + 4 * reg + g;
                if (c >= W) continue;
                const double gs = acc[reg];
                double *outp, *goldp;
                const double *bp;
                const float *fp32 = nullptr;
                int md;
                if (a.cu) {
                    outp = a.cu[c] + a.coff + a.n;
                    goldp = a.cgold[c] + a.coff;
                    bp = a.cfu[c] + a.coff;
                    md = a.cmode[c];
                    if (md == 0) continue;
                } else {
                    const int64_t o = (int64_t)c * a.n;
                    outp = a.out + o;
                    goldp = a.gold ? a.gold + o : nullptr;
                    bp = a.mode == 1 ? (a.bvec ? a.bvec + o : nullptr) : (a.fu64 ? a.fu64 + o : nullptr);
                    fp32 = a.fu32 ? a.fu32 + o : nullptr;
                    md = (a.mode != 0 && a.active && !a.active[c]) ? -1 : a.mode;
                    if (md < 0) continue;
                }
                if (!a.cu && md == 0) {
                    outp[i] = gs;
                } else if (md == 1) {
                    goldp[i] = gs;
                    outp[i] = gs + (bp ? bp[i] : 0.0);
                } else {
                    const double fu = fp32 ? (double)fp32[i] : bp[i];
                    const double un = fu + gs - goldp[i];
                    const double d = un - outp[i];
                    incv[reg] += d * d;
                    outp[i] = un;
                    goldp[i] = gs;
                }
            }
        }
        if (incs) {
            // sum over the 16 rows of a lane group, then over the waves
#pragma unroll
            for (int reg = 0; reg < 4; ++reg) {
                double v = incv[reg];
                for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o);
                if (nr == 0) red[wv][4 * reg + g] = v;
            }
            __syncthreads();
            if (tid < 16 && c0 + tid < W) {
                double sum = 0.0;
                for (int t = 0; t < LR_THREADS / 64; ++t) sum += red[t][tid];
                a.incpart[(int64_t)blockIdx.x * W + c0 + tid] = sum;
            }
            __syncthreads();
        }
    }
}

// per column: inc2[c] = sum over chunks of incpart (LR_RED waves round-robin
// over the chunks, lanes over columns, wave partials in wave order)
__global__ __launch_bounds__(64 * LR_RED) void k_inc_reduce(const double *incpart, int64_t nch, int w,
                                                            double *inc2) {
    __shared__ double red[LR_RED][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c0 = 0; c0 < w; c0 += 64) {
        const int cc = c0 + lane;
        double s = 0.0;
        if (cc < w)
            for (int64_t ch = wv; ch < nch; ch += LR_RED) s += incpart[ch * w + cc];
        red[wv][lane] = s;
        __syncthreads();
        if (wv == 0 && cc < w) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < LR_RED; ++q) t += red[q][lane];
            inc2[cc] = t;
        }
        __syncthreads();
    }
}

// elementwise helpers
template <typename TS, typename TD>
__global__ void k_convert(const TS *src, TD *dst, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (TD)src[i];
}

__global__ void k_fill(double *dst, int64_t count, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = v;
}

__global__ void k_fillf(float *dst, int64_t count, float v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = v;
}

// R = R2 * R1 (both upper triangular, l x l row-major ld LMAX), one block per slice
__global__ void k_trmm_upper(const int *ls, const double *R2, const double *R1, double *R) {
    const int s = blockIdx.x;
    const int l = ls[s];
    const int64_t off = (int64_t)s * LMAX * LMAX;
    for (int e = threadIdx.x; e < LMAX * LMAX; e += blockDim.x) {
        const int i = e / LMAX, j = e % LMAX;
        double v = 0.0;
        if (i < l && j < l && j >= i)
            for (int k = i; k <= j; ++k) v += R2[off + i * LMAX + k] * R1[off + k * LMAX + j];
        R[off + e] = v;
    }
}

// Mm = R^T for each slice (l x l, row-major ld LMAX)
__global__ void k_transpose_small(const int *ls, const double *R, double *Mm) {
    const int s = blockIdx.x;
    const int l = ls[s];
    const int64_t off = (int64_t)s * LMAX * LMAX;
    for (int e = threadIdx.x; e < LMAX * LMAX; e += blockDim.x) {
        const int i = e / LMAX, j = e % LMAX;
        Mm[off + e] = (i < l && j < l) ? R[off + j * LMAX + i] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// B = C^{-T} for one small l x l matrix per slice (Gauss-Jordan elimination
// with partial pivoting in LDS, one workgroup per slice).  C: row-major ld l
// at s*LMAX*LMAX; B: row-major ld LMAX at the same offset.  status[s] = 1 if
// a pivot is zero or not finite (B is then not written).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_small_inv_t(const int *ls, const double *C, double *B, int *status) {
    extern __shared__ double sm[];
    const int s = blockIdx.x;
    const int l = ls[s];
    const int64_t off = (int64_t)s * LMAX * LMAX;
    double *A = sm;              // l x l, row-major
    double *V = sm + l * l;      // becomes C^{-1}
    double *fac = V + l * l;     // column multipliers
    __shared__ int piv;
    __shared__ int bad;
    const int tid = threadIdx.x, lane = tid & 63;
    for (int e = tid; e < l * l; e += blockDim.x) {
        A[e] = C[off + e];
        V[e] = (e / l == e % l) ? 1.0 : 0.0;
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int c = 0; c < l; ++c) {
        if (tid < 64) {   // pivot row: largest |A[r][c]|, r >= c (lowest index on ties)
            int best = -1;
            double bv = -1.0;
            for (int r = c + lane; r < l; r += 64) {
                const double v = fabs(A[r * l + c]);
                if (v > bv) { bv = v; best = r; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv, o);
                const int ob = __shfl_xor(best, o);
                if (ov > bv || (ov == bv && ob >= 0 && (best < 0 || ob < best))) { bv = ov; best = ob; }
            }
            if (lane == 0) {
                piv = best;
                if (!(bv > 0.0) || !isfinite(bv)) bad = 1;
            }
        }
        __syncthreads();
        if (bad) break;   // uniform: every thread reads the same flag after the barrier
        const int pr = piv;
        if (pr != c)
            for (int j = tid; j < l; j += blockDim.x) {
                double t = A[c * l + j];
                A[c * l + j] = A[pr * l + j];
                A[pr * l + j] = t;
                t = V[c * l + j];
                V[c * l + j] = V[pr * l + j];
                V[pr * l + j] = t;
            }
        __syncthreads();
        const double inv = 1.0 / A[c * l + c];
        for (int r = tid; r < l; r += blockDim.x) fac[r] = r == c ? 0.0 : A[r * l + c];
        __syncthreads();
        for (int j = tid; j < l; j += blockDim.x) {
            A[c * l + j] *= inv;
            V[c * l + j] *= inv;
        }
        __syncthreads();
        for (int e = tid; e < l * l; e += blockDim.x) {
            const int r = e / l, j = e % l;
            if (r != c) {
                A[e] -= fac[r] * A[c * l + j];
                V[e] -= fac[r] * V[c * l + j];
            }
        }
        __syncthreads();
    }
    if (tid == 0) status[s] = bad;
    if (bad) return;
    for (int e = tid; e < LMAX * LMAX; e += blockDim.x) {
        const int i = e / LMAX, j = e % LMAX;
        B[off + e] = (i < l && j < l) ? V[j * l + i] : 0.0;
    }
}

// out = ca a + cb b + cc c, column by column (the stage combinations of the
// SDIRK steppers)
template <typename T>
__global__ __launch_bounds__(256) void k_combine3(T *out, int64_t ldo, const T *a, int64_t lda, T ca, const T *b,
                                                  int64_t ldb, T cb, const T *c, int64_t ldc, T cc, int64_t n, int w) {
    const int64_t total = n * w;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t col = e / n, i = e - col * n;
        T v = ca * a[i + col * lda];
        if (b) v += cb * b[i + col * ldb];
        if (c) v += cc * c[i + col * ldc];
        out[i + col * ldo] = v;
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static unsigned blocks_for(int64_t count, int threads) {
    int64_t b = (count + threads - 1) / threads;
    if (b > 65535) b = 65535;
    if (b < 1) b = 1;
    return (unsigned)b;
}

int gram_chunks(int64_t nmax) { return (int)((nmax + GRAM_CHUNK - 1) / GRAM_CHUNK); }

hipError_t launch_gram(bool f32, const GramJob *d_jobs, int njobs, int nchunks, double *part, double *G,
                       hipStream_t s) {
    dim3 grid(nchunks, njobs);
    if (f32)
        hipLaunchKernelGGL(k_gram_partial<float>, grid, dim3(256), 0, s, d_jobs, njobs, part);
    else
        hipLaunchKernelGGL(k_gram_partial<double>, grid, dim3(256), 0, s, d_jobs, njobs, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_reduce, dim3(njobs), dim3(256), 0, s, d_jobs, nchunks, part, G);
    return hipGetLastError();
}

hipError_t launch_chol(const int *d_ls, int nslices, const double *G, double *R, double *Rinv, int *status,
                       double cond_tol, hipStream_t s) {
    hipLaunchKernelGGL(k_chol, dim3(nslices), dim3(256), 0, s, d_ls, G, R, Rinv, status, cond_tol);
    return hipGetLastError();
}

hipError_t launch_rowmat(int ta, int tc, const RowMatJob *d_jobs, int njobs, int64_t nmax, hipStream_t s) {
    dim3 grid(blocks_for(nmax, RM_ROWS) > 2048 ? 2048 : blocks_for(nmax, RM_ROWS), njobs);
    if (ta == 0 && tc == 0) hipLaunchKernelGGL((k_rowmat<double, double>), grid, dim3(256), 0, s, d_jobs);
    else if (ta == 1 && tc == 0) hipLaunchKernelGGL((k_rowmat<float, double>), grid, dim3(256), 0, s, d_jobs);
    else if (ta == 0 && tc == 1) hipLaunchKernelGGL((k_rowmat<double, float>), grid, dim3(256), 0, s, d_jobs);
    else hipLaunchKernelGGL((k_rowmat<float, float>), grid, dim3(256), 0, s, d_jobs);
    return hipGetLastError();
}

hipError_t launch_householder(const HouseJob *d_jobs, int njobs, hipStream_t s) {
    hipLaunchKernelGGL(k_householder, dim3(njobs), dim3(1024), 0, s, d_jobs);
    return hipGetLastError();
}

hipError_t launch_jacobi(const int *d_ls, int nslices, int lmax, const double *Mm, double *Uh, double *S,
                         double *Vh, int *sweeps, hipStream_t s) {
    const int le = (lmax + 1) & ~1;
    const size_t lds = sizeof(double) * 2 * (size_t)le * le;
    hipLaunchKernelGGL(k_jacobi, dim3(nslices), dim3(1024), lds, s, d_ls, Mm, Uh, S, Vh, sweeps);
    return hipGetLastError();
}

hipError_t launch_signfix(const SignJob *d_jobs, int njobs, int kmax, hipStream_t s) {
    hipLaunchKernelGGL(k_signfix, dim3(kmax, njobs), dim3(256), 0, s, d_jobs);
    return hipGetLastError();
}

int64_t lr_chunks(int64_t n) { return (n + LR_CHUNK - 1) / LR_CHUNK; }
int64_t lr_part_elems(int64_t n, int k, int w) { return (lr_chunks(n) + 1) * (int64_t)(k > 1 ? k : 1) * w; }

hipError_t launch_lowrank(const LrArgs &a, hipStream_t s) {
    const unsigned nch = (unsigned)lr_chunks(a.n);
    const int nk = a.k * a.w;
    LrArgs b = a;
    b.coef = a.part + (int64_t)nch * nk;   // after the chunk partials
    if (a.k > 0) {
        hipLaunchKernelGGL(k_lr_dots, dim3(nch), dim3(LR_THREADS), 0, s, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_lr_coef, dim3((nk + 63) / 64), dim3(64 * LR_RED), 0, s, (const double *)b.part,
                           (int64_t)nch, nk, a.w, a.S, b.coef);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_lr_combine, dim3(nch), dim3(LR_THREADS), sizeof(double) * (size_t)(nk + 1), s, b);
    return hipGetLastError();
}

hipError_t launch_inc_reduce(const double *incpart, int64_t nch, int w, double *inc2, hipStream_t s) {
    hipLaunchKernelGGL(k_inc_reduce, dim3(1), dim3(64 * LR_RED), 0, s, incpart, nch, w, inc2);
    return hipGetLastError();
}

hipError_t launch_convert(int from, int to, const void *src, void *dst, int64_t count, hipStream_t s) {
    const unsigned b = blocks_for(count, 256);
    if (from == 0 && to == 1) hipLaunchKernelGGL((k_convert<double, float>), dim3(b), dim3(256), 0, s, (const double *)src, (float *)dst, count);
    else if (from == 1 && to == 0) hipLaunchKernelGGL((k_convert<float, double>), dim3(b), dim3(256), 0, s, (const float *)src, (double *)dst, count);
    else if (from == 0) hipLaunchKernelGGL((k_convert<double, double>), dim3(b), dim3(256), 0, s, (const double *)src, (double *)dst, count);
    else hipLaunchKernelGGL((k_convert<float, float>), dim3(b), dim3(256), 0, s, (const float *)src, (float *)dst, count);
    return hipGetLastError();
}

hipError_t launch_fill(double *dst, int64_t count, double v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(count, 256)), dim3(256), 0, s, dst, count, v);
    return hipGetLastError();
}

hipError_t launch_fillf(float *dst, int64_t count, float v, hipStream_t s) {
    hipLaunchKernelGGL(k_fillf, dim3(blocks_for(count, 256)), dim3(256), 0, s, dst, count, v);
    return hipGetLastError();
}

hipError_t launch_trmm_upper(const int *d_ls, int nslices, const double *R2, const double *R1, double *R,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_trmm_upper, dim3(nslices), dim3(256), 0, s, d_ls, R2, R1, R);
    return hipGetLastError();
}

hipError_t launch_small_inv_t(const int *d_ls, int nslices, int lmax, const double *C, double *B, int *status,
                              hipStream_t s) {
    const size_t lds = sizeof(double) * (2 * (size_t)lmax * lmax + lmax);
    hipLaunchKernelGGL(k_small_inv_t, dim3(nslices), dim3(256), lds, s, d_ls, C, B, status);
    return hipGetLastError();
}

hipError_t launch_cross_gram(const double *V, const double *X, int64_t n, int k, int w, const double *ones,
                             double *part, double *out, hipStream_t s) {
    LrArgs a{};
    a.V = V;
    a.x = X;
    a.n = n;
    a.k = k;
    a.w = w;
    a.part = part;
    const unsigned nch = (unsigned)lr_chunks(n);
    const int nk = k * w;
    hipLaunchKernelGGL(k_lr_dots, dim3(nch), dim3(LR_THREADS), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lr_coef, dim3((nk + 63) / 64), dim3(64 * LR_RED), 0, s, (const double *)part, (int64_t)nch,
                       nk, w, ones, out);
    return hipGetLastError();
}

hipError_t launch_combine3(bool f32, void *out, int64_t ldo, const void *a, int64_t lda, double ca, const void *b,
                           int64_t ldb, double cb, const void *c, int64_t ldc, double cc, int64_t n, int w,
                           hipStream_t s) {
    const int64_t total = n * w;
    if (total <= 0) return hipSuccess;
    unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
    if (f32)
        hipLaunchKernelGGL(k_combine3<float>, dim3(blocks), dim3(256), 0, s, (float *)out, ldo, (const float *)a, lda,
                           (float)ca, (const float *)b, ldb, (float)cb, (const float *)c, ldc, (float)cc, n, w);
    else
        hipLaunchKernelGGL(k_combine3<double>, dim3(blocks), dim3(256), 0, s, (double *)out, ldo, (const double *)a,
                           lda, ca, (const double *)b, ldb, cb, (const double *)c, ldc, cc, n, w);
    return hipGetLastError();
}

hipError_t launch_transpose_small(const int *d_ls, int nslices, const double *R, double *Mm, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose_small, dim3(nslices), dim3(256), 0, s, d_ls, R, Mm);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row scaling by the square roots of positive weights: X[i, j] *= sqrt(w_i)
// (up) or /= sqrt(w_i), X n x cols column-major with leading dimension n, in
// the element type of the panel (FP32 panels scale in FP64 and round).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_row_scale(T *X, int64_t n, int64_t cols, const double *w, int up) {
    const int64_t total = n * cols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double s = sqrt(w[e % n]);
        const double x = (double)X[e];
        X[e] = (T)(up ? x * s : x / s);
    }
}

hipError_t launch_row_scale(bool f32, void *X, int64_t n, int64_t cols, const double *w, bool up, hipStream_t s) {
    const int64_t total = n * cols;
    if (total <= 0) return hipSuccess;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (f32)
        hipLaunchKernelGGL(k_row_scale<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float *)X, n, cols, w,
                           up ? 1 : 0);
    else
        hipLaunchKernelGGL(k_row_scale<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double *)X, n, cols, w,
                           up ? 1 : 0);
    return hipGetLastError();
}

}  // namespace lrpr
