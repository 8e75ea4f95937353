// Operator assembly and packing of the LU factors into the tiled layout read
// by the sweep kernels (the LU itself is in lu.hip).
#include <climits>

#include "lrpr_internal.h"
#include "tile_ops.h"

namespace lrpr {

// ---------------------------------------------------------------------------
// Assembly of M = I + dt*A into band storage n x (2b+1), row-major, entry
// (i, j) at i*(2b+1) + j - i + b.  A: finite differences of
// -nu*Laplace + beta.grad + c on the unit interval/square, first-order
// upwind (the upwind neighbour is the west/south one for a positive velocity
// component); homogeneous Dirichlet (h = 1/(nx+1), interior points) or
// Neumann (h = 1/(nx-1), boundary points included, mirrored ghost points)
// boundary.  One thread per band entry.
//
// Reversed assembly (rev): the matrix J Mp J of N = 16 NT rows, with Mp =
// diag(M, I) padded to whole tile rows and J the row reversal.  Its LU,
// J Mp J = Lr Ur, gives the UL factorisation Mp = (J Lr J)(J Ur J): an upper
// factor with unit diagonal times a lower one.
// ---------------------------------------------------------------------------
__device__ inline double dirichlet_entry(const lrpr_op_desc &op, int64_t n, int64_t i, int64_t jcol) {
    if (jcol < 0 || jcol >= n) return 0.0;
    const double h = 1.0 / (double)(op.nx + 1);
    const double dif = op.nu / (h * h);
    const double b1 = op.beta1, b2 = op.dim == 2 ? op.beta2 : 0.0;
    if (op.dim == 1) {
        if (jcol == i) return 1.0 + op.dt * (2.0 * dif + fabs(b1) / h + op.c);
        if (jcol == i - 1) return op.dt * (-dif - fmax(b1, 0.0) / h);
        if (jcol == i + 1) return op.dt * (-dif - fmax(-b1, 0.0) / h);
        return 0.0;
    }
    const int nx = op.nx;
    const int64_t ix = i % nx;
    if (jcol == i) return 1.0 + op.dt * (4.0 * dif + (fabs(b1) + fabs(b2)) / h + op.c);
    if (jcol == i - 1 && ix > 0) return op.dt * (-dif - fmax(b1, 0.0) / h);
    if (jcol == i + 1 && ix < nx - 1) return op.dt * (-dif - fmax(-b1, 0.0) / h);
    if (jcol == i - nx) return op.dt * (-dif - fmax(b2, 0.0) / h);
    if (jcol == i + nx) return op.dt * (-dif - fmax(-b2, 0.0) / h);
    return 0.0;
}

// Neumann: the 1D stencil of point p on an axis of nx points, with the
// coefficient of a neighbour beyond the boundary moved onto the mirrored one
// (ghost point u_{-1} = u_1, u_{nx} = u_{nx-2}); off = -1 / +1 for the lower /
// upper neighbour, 0 for the diagonal part.
__device__ inline double neumann_axis(int p, int nx, double dif, double beta, double h, int off) {
    const double lo = -dif - fmax(beta, 0.0) / h, hi = -dif - fmax(-beta, 0.0) / h;
    if (off == 0) return 2.0 * dif + fabs(beta) / h;
    if (off < 0) return p == 0 ? 0.0 : (p == nx - 1 ? lo + hi : lo);
    return p == nx - 1 ? 0.0 : (p == 0 ? hi + lo : hi);
}

__device__ inline double neumann_entry(const lrpr_op_desc &op, int64_t n, int64_t i, int64_t jcol) {
    if (jcol < 0 || jcol >= n) return 0.0;
    const int nx = op.nx;
    const double h = 1.0 / (double)(nx - 1);
    const double dif = op.nu / (h * h);
    if (op.dim == 1) {
        const int d = (int)(jcol - i);
        if (d < -1 || d > 1) return 0.0;
        const double a = neumann_axis((int)i, nx, dif, op.beta1, h, d);
        return d == 0 ? 1.0 + op.dt * (a + op.c) : op.dt * a;
    }
    const int ix = (int)(i % nx), iy = (int)(i / nx);
    if (jcol == i)
        return 1.0 + op.dt * (neumann_axis(ix, nx, dif, op.beta1, h, 0) + neumann_axis(iy, nx, dif, op.beta2, h, 0) +
                              op.c);
    if (jcol == i - 1 && ix > 0) return op.dt * neumann_axis(ix, nx, dif, op.beta1, h, -1);
    if (jcol == i + 1 && ix < nx - 1) return op.dt * neumann_axis(ix, nx, dif, op.beta1, h, 1);
    if (jcol == i - nx) return op.dt * neumann_axis(iy, nx, dif, op.beta2, h, -1);
    if (jcol == i + nx) return op.dt * neumann_axis(iy, nx, dif, op.beta2, h, 1);
    return 0.0;
}

__device__ inline double m_entry(const lrpr_op_desc &op, int64_t n, int64_t i, int64_t jcol) {
    return op.bc == LRPR_BC_NEUMANN ? neumann_entry(op, n, i, jcol) : dirichlet_entry(op, n, i, jcol);
}

// rows: n (plain) or N (reversed); n is the operator's size
__global__ void k_assemble(lrpr_op_desc op, int64_t n, int64_t rows, int bw, bool rev, double *band) {
    const int W = 2 * bw + 1;
    const int64_t total = rows * W;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / W;
        const int d = (int)(e - r * W);
        const int64_t cidx = r - bw + d;
        double v = 0.0;
        if (!rev) {
            v = m_entry(op, n, r, cidx);
        } else if (cidx >= 0 && cidx < rows) {
            const int64_t i = rows - 1 - r, j = rows - 1 - cidx;
            v = (i < n && j < n) ? m_entry(op, n, i, j) : (i == j ? 1.0 : 0.0);
        }
        band[e] = v;
    }
}

hipError_t launch_assemble(const lrpr_op_desc &op, int64_t n, int64_t rows, int bw, bool rev, double *band,
                           hipStream_t s) {
    const int64_t total = rows * (2 * bw + 1);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)blocks), dim3(256), 0, s, op, n, rows, bw, rev, band);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Packing into the lane-major MFMA A-operand layout of every tile: the value
// lane l feeds as chunk kc is T[m][k] with m = l%16 and the contraction index
// k = 4 kc + l/16 (FP64) or 4 (l/16) + kc (FP32), the row that register kc
// of an accumulator holds.  Position of (l, kc): FP32 4 l + kc (one 16-byte
// load per lane), FP64 128 (kc/2) + 2 l + kc%2 (two 16-byte loads, each a
// contiguous 1 KiB across the wave).
// ---------------------------------------------------------------------------
__device__ inline double lu_at(const double *lu, int64_t n, int bw, int64_t i, int64_t j) {
    if (i < 0 || j < 0 || i >= n || j >= n) return 0.0;
    const int64_t d = j - i;
    if (d < -bw || d > bw) return 0.0;
    return lu[i * (2 * bw + 1) + d + bw];
}

// The two triangular factors of a band LU of `rows` rows, in the operator's
// row order.  Plain (M = L U): lower = L (unit diagonal), upper = U, rows
// beyond n padded with the identity.  Reversed (the LU Lr Ur of J Mp J):
// upper = J Lr J (unit diagonal), lower = J Ur J, so that Mp = upper * lower.
struct LuAcc {
    const double *lu;
    int64_t n, rows;
    int bw;
    bool rev;
    __device__ double at(int64_t i, int64_t j) const {
        return rev ? lu_at(lu, rows, bw, rows - 1 - i, rows - 1 - j) : lu_at(lu, n, bw, i, j);
    }
    // element (i, j) of the lower factor, j <= i
    __device__ double lower(int64_t i, int64_t j) const {
        if (j == i && !rev) return 1.0;
        return at(i, j);
    }
    // element (i, j) of the upper factor, j >= i
    __device__ double upper(int64_t i, int64_t j) const {
        if (j == i && (rev || i >= n)) return 1.0;
        return at(i, j);
    }
};

// position of element (row m, contraction k) of an A-operand tile
__device__ inline int aslot(bool f32, int m, int k) {
    if (f32) return 4 * (16 * (k >> 2) + m) + (k & 3);                 // g = k/4, kc = k%4
    const int kc = k >> 2, l = 16 * (k & 3) + m;                       // g = k%4, kc = k/4
    return 128 * (kc >> 1) + 2 * l + (kc & 1);
}

// Band tiles multiplied from the left by their row's diagonal-tile inverse
// (Linv, Uinv: FP64, row-major per tile row, from k_diag_inv):
//   Lb[I][j]  = L(I,I)^{-1}   L(I, I-nb+j)
//   Ub[I][j]  = U(I,I)^{-1}   U(I, I+1+j)
// and, when requested, the mirrored set
//   UTb[I][j] = U(I,I)^{-T}   U(I-nb+j, I)^T
//   LTb[I][j] = L(I,I)^{-T}   L(I+1+j, I)^T.
struct BandOut {
    void *b[4];   // Lb, Ub, UTb, LTb (null: not stored)
};

// Element (row r, column q) of band tile j of tile row I in set a (0 Lb,
// 1 Ub, 2 UTb, 3 LTb), FP64.
__device__ inline double band_elem(const LuAcc &F, int nb, const double *Linv, const double *Uinv, int64_t I,
                                   int j, int r, int q, int a) {
    const int64_t base = I * TILE;
    const int64_t jl = (I - nb + j) * TILE + q;   // column in tile row I-nb+j
    const int64_t ju = (I + 1 + j) * TILE + q;    // column in tile row I+1+j
    const double *Li = Linv + I * TILE_ELEMS, *Ui = Uinv + I * TILE_ELEMS;
    double v = 0.0;
    for (int k = 0; k < TILE; ++k) {
        const int64_t i = base + k;
        switch (a) {
            case 0: v += Li[r * TILE + k] * F.lower(i, jl); break;   // L(I, J)[k][q]
            case 1: v += Ui[r * TILE + k] * F.upper(i, ju); break;   // U(I, J)[k][q]
            case 2: v += Ui[k * TILE + r] * F.upper(jl, i); break;   // U(J, I)[q][k]
            default: v += Li[k * TILE + r] * F.lower(ju, i); break;  // L(J, I)[q][k]
        }
    }
    return v;
}

// FP64 band tiles: one thread per element (tile row I, band index j, row r,
// column q).
__global__ void k_pack_band(LuAcc F, int NT, int nb, const double *Linv, const double *Uinv, BandOut o64) {
    const int64_t total = (int64_t)NT * nb * TILE_ELEMS;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t tileidx = e / TILE_ELEMS;
        const int o = (int)(e % TILE_ELEMS);
        const int64_t I = tileidx / nb;
        const int j = (int)(tileidx % nb);
        const int r = o >> 4, q = o & 15;
        const int64_t dst = tileidx * TILE_ELEMS + aslot(false, r, q);
        for (int a = 0; a < 4; ++a)
            if (o64.b[a]) ((double *)o64.b[a])[dst] = band_elem(F, nb, Linv, Uinv, I, j, r, q, a);
    }
}

// Row-sum-keeping FP32 rounding of one row of `count` entries; elem(t)
// returns the FP64 value and the FP32 destination of entry t.  Every entry
// is rounded; the FP64 sum of the rounding errors goes into the largest
// entry, and what that entry's rounding leaves into the smallest entry of
// at least 2^-12 of the largest, whose finer spacing holds it to about
// 2^-12 of one rounding of the largest.
template <class Elem>
__device__ inline void round_row_keep_sum(float *out, int count, Elem elem) {
    double err = 0.0, vmax = 0.0;
    int64_t at = -1;
    for (int t = 0; t < count; ++t) {
        int64_t dst;
        const double v = elem(t, dst);
        const float f = (float)v;
        out[dst] = f;
        err += v - (double)f;
        if (fabs(v) > fabs(vmax)) { vmax = v; at = dst; }
    }
    if (at < 0) return;
    const double want = (double)out[at] + err;
    out[at] = (float)want;
    const double res = want - (double)out[at];
    if (res == 0.0) return;
    const double lo = fabs(vmax) * (1.0 / 4096.0);
    double best = fabs(vmax);
    int64_t at2 = -1;
    for (int t = 0; t < count; ++t) {
        int64_t dst;
        const double a = fabs(elem(t, dst));
        if (dst != at && a >= lo && a < best) { best = a; at2 = dst; }
    }
    if (at2 >= 0) out[at2] = (float)((double)out[at2] + res);
}

// FP32 copies keep every row's sum.  A substitution row computes
// x_i = sum_k D[i][k] r_k - sum_c B[i][c] x_c; on smooth vectors only the row
// sums of D and B act, and for a constant-coefficient operator the factor
// entries, hence their FP32 rounding errors, are the same in every interior
// row, so plain rounding shifts the smooth modes' decay rate coherently,
// once per step.  Each row is rounded by round_row_keep_sum.
//
// Band tiles: one thread per (set, tile row I, row r) walks the nb x 16
// entries of its row, read from the FP64 tiles of the set when they are
// stored (src64), else computed as k_pack_band does (the same values).
__global__ void k_pack_band32(LuAcc F, int NT, int nb, const double *Linv, const double *Uinv, BandOut src64,
                              BandOut o32) {
    const int64_t rows = (int64_t)NT * TILE;
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (tid >= 4 * rows) return;
    const int a = (int)(tid / rows);
    if (!o32.b[a]) return;
    const int64_t I = (tid % rows) / TILE;
    const int r = (int)(tid % TILE);
    round_row_keep_sum((float *)o32.b[a], nb * TILE, [&](int t, int64_t &dst) {
        const int j = t / TILE, q = t % TILE;
        const int64_t tile = (I * nb + j) * TILE_ELEMS;
        dst = tile + aslot(true, r, q);
        return src64.b[a] ? ((const double *)src64.b[a])[tile + aslot(false, r, q)]
                          : band_elem(F, nb, Linv, Uinv, I, j, r, q, a);
    });
}

// Band tiles of one tile row per workgroup (256 threads, one per element of
// a tile), for every requested set (blockIdx.y).  The nb 16x16 factor blocks
// of the row are loaded 16 at a time (every load of a chunk in flight
// together, the next chunk's while the current one is used) and staged in
// LDS; thread (r, q) forms entry (r, q) of every block's product with the
// row's diagonal-tile inverse (the same sums in the same order as band_elem:
// one independent chain per block) and keeps them in registers.  Row r's
// 16 nb values then sit in the 16 threads (r, 0..15), thread q holding
// entries q, q + 16, ...: the FP32 row is rounded by round_row_keep_sum's
// rule with the rounding errors summed over those threads and the largest
// and smallest entries reduced across them (ties going to the lower entry
// index), and every thread writes its own entries.
template <int NBMAX>
__global__ __launch_bounds__(256) void k_pack_rows(LuAcc F, int NT, int nb, const double *Linv, const double *Uinv,
                                                   BandOut o64, BandOut o32) {
    constexpr int CH = 16;               // blocks staged at once
    extern __shared__ double lds[];      // [CH][16][16]: element (k, q) of block u at u*256 + 16 k + q
    const int a = blockIdx.y;
    if (!o64.b[a] && !o32.b[a]) return;
    const int64_t I = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t base = I * TILE;
    const int r = t >> 4, q = t & 15;
    // this thread's element of block j, read along the contiguous direction
    // of the band storage, staged at (sk, sq)
    const int sk = a < 2 ? (t >> 4) : (t & 15), sq = a < 2 ? (t & 15) : (t >> 4);
    auto fetch = [&](int j) -> double {
        const int64_t jl = (I - nb + j) * TILE, ju = (I + 1 + j) * TILE;
        if (a < 2) return a == 0 ? F.lower(base + sk, jl + sq) : F.upper(base + sk, ju + sq);
        return a == 2 ? F.upper(jl + sq, base + sk) : F.lower(ju + sq, base + sk);
    };
    double m[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) m[u] = u < nb ? fetch(u) : 0.0;
    // row r of the diagonal-tile inverse (column r for the transposed sets)
    const double *Di = ((a == 0 || a == 3) ? Linv : Uinv) + I * TILE_ELEMS;
    double d[TILE];
#pragma unroll
    for (int k = 0; k < TILE; ++k) d[k] = a < 2 ? Di[r * TILE + k] : Di[k * TILE + r];
    double v[NBMAX];
#pragma unroll
    for (int c0 = 0; c0 < NBMAX; c0 += CH) {
        if (c0 < nb) {   // workgroup-uniform
            if (c0 > 0) lds_barrier();   // the previous chunk's reads are done
#pragma unroll
            for (int u = 0; u < CH; ++u)
                if (c0 + u < nb) lds[u * TILE_ELEMS + sk * TILE + sq] = m[u];
            if (c0 + CH < nb) {
#pragma unroll
                for (int u = 0; u < CH; ++u) m[u] = c0 + CH + u < nb ? fetch(c0 + CH + u) : 0.0;
            }
            lds_barrier();   // LDS only: the next chunk's loads stay in flight
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int j = c0 + u;
            double x = 0.0;
            if (j < nb) {
#pragma unroll
                for (int k = 0; k < TILE; ++k) x += d[k] * lds[u * TILE_ELEMS + k * TILE + q];
            }
            v[j] = x;
        }
    }
    if (o64.b[a]) {
#pragma unroll
        for (int j = 0; j < NBMAX; ++j)
            if (j < nb) ((double *)o64.b[a])[(I * nb + j) * TILE_ELEMS + aslot(false, r, q)] = v[j];
    }
    if (!o32.b[a]) return;
    // rounding of row r by its 16 threads (entry c = 16 j + q in thread q)
    double err = 0.0, amax = 0.0, xmax = 0.0;
    int imax = INT_MAX;   // none: every entry is zero (or NaN)
#pragma unroll
    for (int j = 0; j < NBMAX; ++j)
        if (j < nb) {
            const double x = v[j];
            err += x - (double)(float)x;
            if (fabs(x) > amax) { amax = fabs(x); xmax = x; imax = TILE * j + q; }
        }
#pragma unroll
    for (int s = 8; s >= 1; s >>= 1) {
        err += __shfl_xor(err, s, TILE);
        const double oa = __shfl_xor(amax, s, TILE), ox = __shfl_xor(xmax, s, TILE);
        const int oi = __shfl_xor(imax, s, TILE);
        if (oa > amax || (oa == amax && oi < imax)) { amax = oa; xmax = ox; imax = oi; }
    }
    int at2 = INT_MAX;
    float fat = 0.f, f2 = 0.f;
    if (imax != INT_MAX) {
        const double want = (double)(float)xmax + err;
        fat = (float)want;
        const double res = want - (double)fat;
        if (res != 0.0) {   // row-uniform
            const double lo = amax * (1.0 / 4096.0);
            double best = amax, x2 = 0.0;
#pragma unroll
            for (int j = 0; j < NBMAX; ++j)
                if (j < nb) {
                    const double ax = fabs(v[j]);
                    if (TILE * j + q != imax && ax >= lo && ax < best) { best = ax; x2 = v[j]; at2 = TILE * j + q; }
                }
#pragma unroll
            for (int s = 8; s >= 1; s >>= 1) {
                const double ob = __shfl_xor(best, s, TILE), ox = __shfl_xor(x2, s, TILE);
                const int oi = __shfl_xor(at2, s, TILE);
                if (ob < best || (ob == best && oi < at2)) { best = ob; x2 = ox; at2 = oi; }
            }
            if (at2 != INT_MAX) f2 = (float)((double)(float)x2 + res);
        }
    }
    float *const out = (float *)o32.b[a] + I * nb * TILE_ELEMS;
#pragma unroll
    for (int j = 0; j < NBMAX; ++j)
        if (j < nb) {
            const int c = TILE * j + q;
            out[j * TILE_ELEMS + aslot(true, r, q)] = c == imax ? fat : c == at2 ? f2 : (float)v[j];
        }
}

// Phase 1: FP64 inverses of the diagonal tiles, natural row-major 16x16 per
// tile row (scratch).  One thread per (tile row, column of the inverse).
__global__ void k_diag_inv(LuAcc F, int NT, double *Linv, double *Uinv) {
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (tid >= (int64_t)NT * TILE) return;
    const int64_t I = tid / TILE;
    const int col = (int)(tid % TILE);
    const int64_t base = I * TILE;
    double xl[TILE], xu[TILE];
    // column `col` of L_II^{-1}: forward substitution on e_col
    for (int r = 0; r < TILE; ++r) {
        double v = (r == col) ? 1.0 : 0.0;
        for (int q = 0; q < r; ++q) v -= F.lower(base + r, base + q) * xl[q];
        xl[r] = v / F.lower(base + r, base + r);
    }
    // column `col` of U_II^{-1}: back substitution
    for (int r = TILE - 1; r >= 0; --r) {
        double v = (r == col) ? 1.0 : 0.0;
        for (int q = r + 1; q < TILE; ++q) v -= F.upper(base + r, base + q) * xu[q];
        xu[r] = v / F.upper(base + r, base + r);
    }
    for (int r = 0; r < TILE; ++r) {
        Linv[I * TILE_ELEMS + r * TILE + col] = xl[r];
        Uinv[I * TILE_ELEMS + r * TILE + col] = xu[r];
    }
}

// Phase 2: diagonal inverses DL = L(I,I)^{-1}, DU = U(I,I)^{-1} and their
// transposes as MFMA A operands (aslot layout), FP64 and/or FP32.
struct DiagOut {
    void *D[4];   // DL, DU, DLT, DUT
};

// Element (r, c) of diagonal set a (0 DL, 1 DU, 2 DLT, 3 DUT) of tile row I.
__device__ inline double diag_elem(const double *Linv, const double *Uinv, int64_t I, int r, int c, int a) {
    const double *Li = Linv + I * TILE_ELEMS, *Ui = Uinv + I * TILE_ELEMS;
    switch (a) {
        case 0: return Li[r * TILE + c];
        case 1: return Ui[r * TILE + c];
        case 2: return Li[c * TILE + r];
        default: return Ui[c * TILE + r];
    }
}

// One thread per (tile row, row r): FP64 copies as they are, FP32 copies
// with the row sum kept (as k_pack_band32).
__global__ void k_pack_diag(int NT, const double *Linv, const double *Uinv, DiagOut o64, DiagOut o32) {
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (tid >= (int64_t)NT * TILE) return;
    const int64_t I = tid / TILE;
    const int r = (int)(tid % TILE);
    const int64_t off = I * TILE_ELEMS;
    for (int a = 0; a < 4; ++a) {
        if (o64.D[a])
            for (int c = 0; c < TILE; ++c)
                ((double *)o64.D[a])[off + aslot(false, r, c)] = diag_elem(Linv, Uinv, I, r, c, a);
        if (o32.D[a])
            round_row_keep_sum((float *)o32.D[a], TILE, [&](int c, int64_t &dst) {
                dst = off + aslot(true, r, c);
                return diag_elem(Linv, Uinv, I, r, c, a);
            });
    }
}

hipError_t launch_pack_tiles(int64_t n, int bw, int NT, int nb, const double *lu, bool rev, const TileSet *t64,
                             const TileSet *t32, double *scratch, hipStream_t s) {
    const int64_t th = (int64_t)NT * TILE;
    double *Linv = scratch, *Uinv = scratch + (size_t)NT * TILE_ELEMS;
    const LuAcc F{lu, n, (int64_t)NT * TILE, bw, rev};
    hipLaunchKernelGGL(k_diag_inv, dim3((unsigned)((th + 127) / 128)), dim3(128), 0, s, F, NT, Linv, Uinv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)NT * nb * TILE_ELEMS;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    BandOut b64{}, b32{};
    const int bidx[4] = {TS_LB, TS_UB, TS_UTB, TS_LTB};
    for (int a = 0; a < 4; ++a) {
        b64.b[a] = t64 ? t64->a[bidx[a]] : nullptr;
        b32.b[a] = t32 ? t32->a[bidx[a]] : nullptr;
    }
    if (nb <= 64) {
        const size_t lds = sizeof(double) * TILE_ELEMS * 16;
        if (nb <= 32)
            hipLaunchKernelGGL(k_pack_rows<32>, dim3((unsigned)NT, 4), dim3(256), lds, s, F, NT, nb, Linv, Uinv, b64,
                               b32);
        else
            hipLaunchKernelGGL(k_pack_rows<64>, dim3((unsigned)NT, 4), dim3(256), lds, s, F, NT, nb, Linv, Uinv, b64,
                               b32);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        if (t64) {
            hipLaunchKernelGGL(k_pack_band, dim3((unsigned)blocks), dim3(256), 0, s, F, NT, nb, Linv, Uinv, b64);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (t32) {
            hipLaunchKernelGGL(k_pack_band32, dim3((unsigned)((4 * th + 127) / 128)), dim3(128), 0, s, F, NT, nb,
                               Linv, Uinv, b64, b32);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    DiagOut o64{}, o32{};
    const int didx[4] = {TS_DL, TS_DU, TS_DLT, TS_DUT};
    for (int a = 0; a < 4; ++a) {
        o64.D[a] = t64 ? t64->a[didx[a]] : nullptr;
        o32.D[a] = t32 ? t32->a[didx[a]] : nullptr;
    }
    hipLaunchKernelGGL(k_pack_diag, dim3((unsigned)((th + 127) / 128)), dim3(128), 0, s, NT, Linv, Uinv, o64, o32);
    return hipGetLastError();
}

}  // namespace lrpr
