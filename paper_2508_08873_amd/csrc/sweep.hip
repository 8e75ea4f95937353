// Batched implicit-Euler sweeps through a banded LU on gfx950 (CDNA4).
//
// One implicit-Euler step of the fine propagator solves (I + dt A) x_new =
// x_old + dt f(t_new) with M = L U: a forward substitution with L then a
// back substitution with U (Sec. 2, eq. F_n_affine; the paper's solver reuses
// one factorisation for all right-hand sides of a step, Sec. 4.4).  The
// adjoint (Sec. 2.1 step 3) solves M^T z = x: forward with U^T, back with L^T.
//
// Blocking.  Rows are cut into tile rows of 16.  For tile row I the solve is
//     y_I = D_I (r_I - sum_J B_IJ y_J)
// where the B_IJ are the nb band tiles on the already-solved side and D_I the
// inverse of the diagonal tile.  Both products are 16x16x16 contractions on
// the matrix cores (v_mfma_*_16x16x4), one wave per 16 right-hand sides.
// The last nb solved tiles of the group live in an LDS ring; the band tiles
// stream from L2/HBM straight into VGPRs.  KW waves split the nb band tiles
// of a tile row, their partial sums meet in LDS, and wave 0 finishes the row
// (source term, diagonal inverse, store).  The state stays column-major in
// HBM and is read/written once per substitution pass.
#include "lrpr_internal.h"

namespace lrpr {

template <typename T> struct Mf;

// f64 16x16x4: A[m][k] in lane m+16k, B[k][n] in lane n+16k,
// D[m][n] in lane n+16(m%4), register m/4.
template <> struct Mf<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int g, int i) { return 4 * i + g; }
};

// f32 16x16x4: A and B as above, D[m][n] in lane n+16(m/4), register m%4.
template <> struct Mf<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int g, int i) { return 4 * g + i; }
};

// One substitution pass over all tile rows of one 16-column group.
//   ASC   : ascending tile rows (forward substitution) or descending.
//   TRANS : band tiles are read transposed from the other triangle's
//           storage (adjoint).
template <typename T, int KW, int TPW, bool ASC, bool TRANS>
__device__ __forceinline__ void sweep_pass(const SweepItem &it, const T *__restrict__ band,
                                           const T *__restrict__ dtile, T *ring, T *red,
                                           bool with_src, int step, int nsteps) {
    typedef typename Mf<T>::v4 v4;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int c = lane & 15;
    const int n = it.fac.n, NT = it.fac.NT, nb = it.fac.nb;
    const int RS = nb + 1;
    // A-operand offsets of a band tile in the 4x4 sub-block layout
    const int off_fwd = ((c >> 2) * 16) + ((c & 3) * 4) + g;   // + 64*kc; lane's row = c
    const int off_adj = ((c >> 2) * 64) + (g * 4) + (c & 3);   // + 16*kc
    T *X = (T *)it.X;
    const int64_t ldx = it.ldx;
    const bool colok = c < it.ncols;
    const T *fsrc = nullptr;
    T fs = 0;
    if (with_src && w == 0 && colok) {
        int fc = it.fcol ? it.fcol[c] : 0;
        if (fc >= 0) {
            fsrc = (const T *)it.f + (int64_t)fc * it.ldf;
            double sc = it.fscale ? it.fscale[(int64_t)c * nsteps + step] : 1.0;
            fs = (T)(it.fac.dt * sc);
        }
    }
    for (int q = 0; q < NT; ++q) {
        const int I = ASC ? q : NT - 1 - q;
        // wave 0 fetches its right-hand side early so the load overlaps the MFMAs
        v4 r = {0, 0, 0, 0};
        if (w == 0 && colok) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = I * TILE + Mf<T>::row(g, i);
                if (row < n) {
                    T x = X[row + (int64_t)c * ldx];
                    if (fsrc) x += fs * fsrc[row];
                    r[i] = x;
                }
            }
        }
        v4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int j = w + KW * t;
            if (j < nb) {
                const int J = ASC ? I - nb + j : I + 1 + j;
                if (J >= 0 && J < NT) {
                    const T *tile;
                    if (TRANS)
                        tile = band + ((int64_t)J * nb + (nb - 1 - j)) * TILE_ELEMS;
                    else
                        tile = band + ((int64_t)I * nb + j) * TILE_ELEMS;
                    const T *rj = ring + (J % RS) * TILE_ELEMS;
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc) {
                        const T a = TRANS ? tile[16 * kc + off_adj] : tile[64 * kc + off_fwd];
                        const T b = rj[64 * kc + lane];
                        acc = Mf<T>::mma(a, b, acc);
                    }
                }
            }
        }
        if (KW > 1) {
            if (w > 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i) red[(w - 1) * TILE_ELEMS + i * 64 + lane] = acc[i];
            }
            __syncthreads();
        }
        if (w == 0) {
#pragma unroll
            for (int ww = 1; ww < KW; ++ww)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[i] += red[(ww - 1) * TILE_ELEMS + i * 64 + lane];
            v4 s;
#pragma unroll
            for (int i = 0; i < 4; ++i) s[i] = r[i] - acc[i];
            const T *D = dtile + (int64_t)I * TILE_ELEMS;
            v4 y = {0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) y = Mf<T>::mma(D[kc * 64 + lane], s[kc], y);
            T *ri = ring + (I % RS) * TILE_ELEMS;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int rr = Mf<T>::row(g, i);
                ri[rr * TILE + c] = y[i];
                const int row = I * TILE + rr;
                if (colok && row < n) X[row + (int64_t)c * ldx] = y[i];
            }
        }
        __syncthreads();
    }
}

template <typename T, int KW, int TPW, bool ADJ>
__global__ __launch_bounds__(64 * KW) void k_sweep(const SweepItem *__restrict__ items, int nitems,
                                                   int nsteps) {
    extern __shared__ __align__(16) unsigned char smem[];
    for (int idx = blockIdx.x; idx < nitems; idx += gridDim.x) {
        const SweepItem it = items[idx];
        T *ring = (T *)smem;
        T *red = ring + (it.fac.nb + 1) * TILE_ELEMS;
        const T *Lb = (const T *)it.fac.Lb, *Ub = (const T *)it.fac.Ub;
        for (int step = 0; step < nsteps; ++step) {
            if (!ADJ) {
                sweep_pass<T, KW, TPW, true, false>(it, Lb, (const T *)it.fac.DL, ring, red,
                                                    it.f != nullptr, step, nsteps);
                sweep_pass<T, KW, TPW, false, false>(it, Ub, (const T *)it.fac.DU, ring, red, false,
                                                     step, nsteps);
            } else {
                sweep_pass<T, KW, TPW, true, true>(it, Ub, (const T *)it.fac.DUT, ring, red, false,
                                                   step, nsteps);
                sweep_pass<T, KW, TPW, false, true>(it, Lb, (const T *)it.fac.DLT, ring, red, false,
                                                    step, nsteps);
            }
        }
    }
}

template <typename T, int KW, int TPW>
static hipError_t launch_t(bool adjoint, int nitems, const SweepItem *d_items, int nsteps, int max_nb,
                           hipStream_t s) {
    const size_t lds = (size_t)(max_nb + 1 + (KW - 1)) * TILE_ELEMS * sizeof(T);
    const int grid = nitems < 65536 ? nitems : 65536;
    if (adjoint)
        hipLaunchKernelGGL((k_sweep<T, KW, TPW, true>), dim3(grid), dim3(64 * KW), lds, s, d_items,
                           nitems, nsteps);
    else
        hipLaunchKernelGGL((k_sweep<T, KW, TPW, false>), dim3(grid), dim3(64 * KW), lds, s, d_items,
                           nitems, nsteps);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_prec(bool adjoint, int nitems, const SweepItem *d_items, int nsteps,
                              int max_nb, hipStream_t s) {
    if (max_nb <= 4) return launch_t<T, 1, 4>(adjoint, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 8) return launch_t<T, 4, 2>(adjoint, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 16) return launch_t<T, 4, 4>(adjoint, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 32) return launch_t<T, 4, 8>(adjoint, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 64) return launch_t<T, 4, 16>(adjoint, nitems, d_items, nsteps, max_nb, s);
    return hipErrorInvalidValue;
}

hipError_t launch_sweep(bool adjoint, bool f32, int nitems, const SweepItem *d_items, int nsteps,
                        int max_nb, hipStream_t s) {
    if (nitems <= 0 || nsteps <= 0) return hipSuccess;
    if (f32) return launch_prec<float>(adjoint, nitems, d_items, nsteps, max_nb, s);
    return launch_prec<double>(adjoint, nitems, d_items, nsteps, max_nb, s);
}

}  // namespace lrpr
