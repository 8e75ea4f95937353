// Batched implicit-Euler sweeps through a banded LU on gfx950 (CDNA4).
//
// One implicit-Euler step of the fine propagator solves (I + dt A) x_new =
// x_old + dt f(t_new) with M = L U: a forward substitution with L, then a
// back substitution with U (Sec. 2, eq. F_n_affine; the paper's solver reuses
// one factorisation for all right-hand sides of a step, Sec. 4.4).  The
// adjoint (Sec. 2.1, step 3) solves M^T z = x with M^T = U^T L^T: forward
// with U^T, back with L^T.  Both are the same two-pass sweep over band tiles:
// the forward set holds L and U, the mirrored set U^T and L^T of the same LU.
// Without a mirrored set the adjoint reads the forward tiles transposed.
//
// Blocking.  Rows are cut into tile rows of 16.  For tile row I of a pass
//     y_I = D_I s_I,   s_I = r_I - sum_{bulk J} B_IJ y_J - E_I s_{I-1}
// where the B_IJ are the nb-1 older band tiles, D_I is the inverse of the
// diagonal tile and E_I = B_{I,I-1} D_{I-1} is the newest band tile times the
// neighbour's inverse, so the row-to-row recurrence only runs through s.
// Every product is a 16x16x16 contraction on the matrix cores
// (v_mfma_*_16x16x4), 16 right-hand sides per workgroup.
//
// Waves of a workgroup (KW = 8):
//   wave 0        finisher: s, t = E s, y = D s, ring and HBM store;
//   waves 1..5    bulk: partial sums over the older band tiles, operands
//                 prefetched PD-1 tile rows ahead into registers;
//   wave 6        factor helper: prefetches D and E of coming rows;
//   wave 7        state helper: prefetches the right-hand side rows.
// The last nb solved tiles live in an LDS ring; helpers hand their operands
// to the finisher through a triple-buffered LDS area.  One barrier per tile
// row orders LDS traffic only, so prefetches stay in flight across it.
// Narrow bands (nb <= 4) run one wave that does everything.
#include "lrpr_internal.h"

namespace lrpr {

// Loads and stores through address space 1 compile to global_* instructions
// (flat_* would also count against the LDS counter and be drained by every
// LDS barrier, cancelling the prefetch).
template <typename T> using gptr = __attribute__((address_space(1))) const T *;
template <typename T> using gptr_mut = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ T gld(const T *p) { return *(gptr<T>)p; }
template <typename T> __device__ __forceinline__ void gst(T *p, T v) { *(gptr_mut<T>)p = v; }

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T> struct Mf;

// f64 16x16x4: A[m][k] in lane m+16k, B[k][n] in lane n+16k,
// D[m][n] in lane n+16(m%4), register m/4.
template <> struct Mf<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // row held by register i of lane group g
    __device__ static inline int row(int g, int i) { return 4 * i + g; }
    // position of (lane l, chunk kc) in a lane-major tile
    __device__ static inline int slot(int l, int kc) { return 128 * (kc >> 1) + 2 * l + (kc & 1); }
    // (lane group, chunk) whose contraction index is k
    __device__ static inline void gk(int k, int &g, int &kc) { g = k & 3; kc = k >> 2; }
    __device__ static inline void ld4(const double *tile, int l, double (&v)[4]) {
        const d2v a = *(gptr<d2v>)(tile + 2 * l), b = *(gptr<d2v>)(tile + 128 + 2 * l);
        v[0] = a[0]; v[1] = a[1]; v[2] = b[0]; v[3] = b[1];
    }
};

// f32 16x16x4: A and B as above, D[m][n] in lane n+16(m/4), register m%4.
template <> struct Mf<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static inline v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int row(int g, int i) { return 4 * g + i; }
    __device__ static inline int slot(int l, int kc) { return 4 * l + kc; }
    __device__ static inline void gk(int k, int &g, int &kc) { g = k >> 2; kc = k & 3; }
    __device__ static inline void ld4(const float *tile, int l, float (&v)[4]) {
        const f4v a = *(gptr<f4v>)(tile + 4 * l);
        v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3];
    }
};

// Barrier that orders LDS traffic only: outstanding global loads (the
// prefetches of later tile rows) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One pass (ascending or descending tile rows) over one 16-column group.
//   band  : band tiles of the pass, nb per tile row (row I, index j)
//   dtile : diagonal inverses; etile: newest-tile products (one per row)
//   STRIDED: the band tiles are the forward set's, read transposed: tile
//            (row J, index nb-1-j), each lane gathering its four values.
// Registers and LDS hold 16x16 blocks in accumulator order: value i of lane
// l is row Mf::row(l/16, i), column l%16 — the B operand of chunk i.
template <typename T, int KW, int TPW, int PD, bool ASC, bool STRIDED>
struct Pass {
    typedef typename Mf<T>::v4 v4;
    static constexpr int NBW = KW > 1 ? KW - 3 : 1;   // bulk waves
    const T *__restrict__ band;
    const T *__restrict__ dtile;
    const T *__restrict__ etile;
    const T *__restrict__ zt;
    T *ring;
    int lane, w, g, c, n, NT, nb, RS, nbulk;
    int soff[4];   // STRIDED: position of this lane's chunk values in a forward tile

    __device__ Pass(const SweepItem &it, const T *band_, const T *dtile_, const T *etile_, T *ring_)
        : band(band_), dtile(dtile_), etile(etile_), zt((const T *)it.fac.zt), ring(ring_) {
        lane = threadIdx.x & 63;
        w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform (scalar)
        g = lane >> 4;
        c = lane & 15;
        n = it.fac.n;
        NT = it.fac.NT;
        nb = it.fac.nb;
        RS = nb + 1;
        nbulk = nb - 1;
        // transposed: A'[c][k] = T[k][c] with k = row(g, kc); element (k, c) of
        // the forward tile is held by lane 16 g' + k, chunk kc' where the
        // contraction index of (g', kc') is c
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            int gp, kcp;
            Mf<T>::gk(c, gp, kcp);
            soff[kc] = Mf<T>::slot(16 * gp + Mf<T>::row(g, kc), kcp);
        }
    }
    __device__ __forceinline__ int row_of(int q) const { return ASC ? q : NT - 1 - q; }
    __device__ __forceinline__ const T *tile_ptr(int I, int j, int J) const {
        if (STRIDED) return band + ((int64_t)J * nb + (nb - 1 - j)) * TILE_ELEMS;
        return band + ((int64_t)I * nb + j) * TILE_ELEMS;
    }
    // bulk tile t of bulk wave wb.  Tile rows outside [0, NT) are zero guard
    // rows of the tile arrays, so every address within the prefetch window is
    // valid; surplus slots (idx >= nb-1) read the zero tile.
    __device__ __forceinline__ bool bulk(int q, int wb, int t, int &j, int &J) const {
        const int I = row_of(q);
        const int idx = wb + NBW * t;
        j = ASC ? idx : idx + 1;
        J = ASC ? I - nb + j : I + 1 + j;
        return idx < nbulk;
    }
    __device__ __forceinline__ void ld_tile(const T *tp, T (&v)[4]) const {
        if (STRIDED) {
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) v[kc] = gld(tp + soff[kc]);
        } else {
            Mf<T>::ld4(tp, lane, v);
        }
    }
    template <int NTP>
    __device__ __forceinline__ void load_bulk(int q, int wb, T (&ab)[NTP][4]) const {
        const int I = row_of(q);
#pragma unroll
        for (int t = 0; t < NTP; ++t) {
            int j, J;
            ld_tile(bulk(q, wb, t, j, J) ? tile_ptr(I, j, J) : zt, ab[t]);
        }
    }
    // ring slot of tile row J given sI = slot of the current row I (J within
    // nb rows of I); invalid tiles read any slot (their A operand is zero and
    // every slot holds finite values)
    __device__ __forceinline__ int slot_of(int sI, int j) const {
        int sJ = ASC ? sI - nb + j : sI + 1 + j;
        sJ = (sJ < 0) ? sJ + RS : sJ;
        sJ = (sJ >= RS) ? sJ - RS : sJ;
        return sJ;
    }
    // two independent accumulator chains (they interleave on the matrix core)
    template <int NTP>
    __device__ __forceinline__ v4 bulk_mma(int q, int wb, int sI, const T (&ab)[NTP][4]) const {
        constexpr int NA = NTP < 2 ? NTP : 2;
        v4 acc[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) acc[a] = v4{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < NTP; ++t) {
            int j, J;
            bulk(q, wb, t, j, J);
            const T *rj = ring + slot_of(sI, j) * TILE_ELEMS;
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) acc[t % NA] = Mf<T>::mma(ab[t][kc], rj[64 * kc + lane], acc[t % NA]);
        }
#pragma unroll
        for (int a = 1; a < NA; ++a) acc[0] += acc[a];
        return acc[0];
    }
    __device__ __forceinline__ int next_slot(int sI) const {
        return ASC ? (sI + 1 == RS ? 0 : sI + 1) : (sI == 0 ? RS - 1 : sI - 1);
    }
    // diagonal inverse of row q and newest-tile product of row q+1 (guard
    // rows are zero)
    __device__ __forceinline__ void load_de(int q, T (&dbv)[4], T (&ebv)[4]) const {
        Mf<T>::ld4(dtile + (int64_t)row_of(q) * TILE_ELEMS, lane, dbv);
        Mf<T>::ld4(etile + (int64_t)row_of(q + 1) * TILE_ELEMS, lane, ebv);
    }
    // right-hand side rows of row q (accumulator order), clamped into the
    // arrays: rows >= n, columns >= ncols and rows of q >= NT are never stored
    // and meet only zero band entries, so any finite value serves
    __device__ __forceinline__ void load_state(int q, const T *X, int64_t ldx, int col, const T *fsrc,
                                               int64_t fstride, T (&xbv)[4], T (&fbv)[4]) const {
        const int I = row_of(q);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int row = I * TILE + Mf<T>::row(g, i);
            row = row < 0 ? 0 : (row >= n ? n - 1 : row);
            xbv[i] = gld(X + row + (int64_t)col * ldx);
            fbv[i] = gld(fsrc + row * fstride);
        }
    }
};

template <typename T, int KW, int TPW, int PD, bool ASC, bool STRIDED>
__device__ __forceinline__ void sweep_pass(const SweepItem &it, const T *__restrict__ band,
                                           const T *__restrict__ dtile, const T *__restrict__ etile, T *ring,
                                           T *red, T *hand, bool with_src, int step, int nsteps) {
    typedef typename Mf<T>::v4 v4;
    typedef Pass<T, KW, TPW, PD, ASC, STRIDED> PS;
    PS P(it, band, dtile, etile, ring);
    const int NT = P.NT, lane = P.lane, g = P.g, c = P.c, n = P.n;
    const int NTp = (NT + PD - 1) / PD * PD;   // rows beyond NT are zero work
    T *X = (T *)it.X;
    const int64_t ldx = it.ldx;
    const bool colok = c < it.ncols;
    const int col = colok ? c : 0;
    // source of this lane's column: f(x) * dt * phi(t_step), or the zero tile
    const T *fsrc = P.zt;
    int64_t fstride = 0;
    T fs = 0;
    if (with_src && colok) {
        const int fc = it.fcol ? it.fcol[c] : 0;
        if (fc >= 0) {
            fsrc = (const T *)it.f + (int64_t)fc * it.ldf;
            fstride = 1;
            const double sc = it.fscale ? it.fscale[(int64_t)c * nsteps + step] : 1.0;
            fs = (T)(it.fac.dt * sc);
        }
    }
    T *sink = (T *)it.fac.sink;
    const int w = P.w;
    // y of tile row Irow: into ring slot ri (accumulator order) and into X
    auto store_y = [&](const v4 &y, T *ri, int Irow, bool ok) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ri[i * 64 + lane] = y[i];
            const int row = Irow * TILE + Mf<T>::row(g, i);
            gst((ok && colok && row < n) ? X + row + (int64_t)c * ldx : sink + lane, y[i]);
        }
    };
    if (KW == 1) {
        // ---- single wave: everything, prefetching PD-1 rows ahead
        T abuf[PD][TPW][4];
        T dbuf[PD][4], ebuf[PD][4], xbuf[PD][4], fbuf[PD][4];
#pragma unroll
        for (int u = 0; u < PD - 1; ++u) {
            P.load_bulk(u, 0, abuf[u]);
            P.load_de(u, dbuf[u], ebuf[u]);
            P.load_state(u, X, ldx, col, fsrc, fstride, xbuf[u], fbuf[u]);
        }
        v4 tnext = {0, 0, 0, 0};
        int sI = P.row_of(0) % P.RS;
        for (int q0 = 0; q0 < NTp; q0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int q = q0 + u;
                const int un = (u + PD - 1) % PD;
                P.load_bulk(q + PD - 1, 0, abuf[un]);
                P.load_de(q + PD - 1, dbuf[un], ebuf[un]);
                P.load_state(q + PD - 1, X, ldx, col, fsrc, fstride, xbuf[un], fbuf[un]);
                __builtin_amdgcn_sched_barrier(0);
                const bool okq = q < NT;
                const int I = P.row_of(q);
                const v4 a = P.bulk_mma(q, 0, sI, abuf[u]);
                v4 sv;
#pragma unroll
                for (int i = 0; i < 4; ++i) sv[i] = (xbuf[u][i] + fs * fbuf[u][i]) - (a[i] + tnext[i]);
                v4 y = {0, 0, 0, 0}, tn = {0, 0, 0, 0};
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) {
                    y = Mf<T>::mma(dbuf[u][kc], sv[kc], y);
                    tn = Mf<T>::mma(ebuf[u][kc], sv[kc], tn);
                }
                tnext = tn;
                store_y(y, ring + (okq ? sI : P.RS) * TILE_ELEMS, I, okq);
                sI = P.next_slot(sI);
                lds_barrier();
            }
        }
    } else if (w == 0) {
        // ---- finisher.  With s_q = r_q - (bulk partials) - E_q s_{q-1}, the
        //      row's solution is y_q = D_q s_q; the recurrence only needs
        //      t_{q+1} = E_{q+1} s_q, and y_q is formed during the next row,
        //      before the barrier that publishes it to the bulk waves.
        v4 tnext = {0, 0, 0, 0};
        v4 sprev = {0, 0, 0, 0};
        T dprev[4] = {0, 0, 0, 0};
        int sprev_slot = P.RS, Iprev = 0;
        bool okprev = false;
        int sI = P.row_of(0) % P.RS;
        lds_barrier();   // hand-off of row 0 is ready
        for (int q = 0; q < NTp; ++q) {
            const bool okq = q < NT;
            const int I = P.row_of(q);
            const T *h = hand + (q % 3) * 4 * TILE_ELEMS;
            {
                v4 y = {0, 0, 0, 0};
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) y = Mf<T>::mma(dprev[kc], sprev[kc], y);
                store_y(y, ring + sprev_slot * TILE_ELEMS, Iprev, okprev);
            }
            T dcur[4], ecur[4], rcur[4];
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                dcur[kc] = h[kc * 64 + lane];
                ecur[kc] = h[TILE_ELEMS + kc * 64 + lane];
            }
            lds_barrier();
#pragma unroll
            for (int i = 0; i < 4; ++i) rcur[i] = h[2 * TILE_ELEMS + i * 64 + lane];
            v4 sv;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                T a = tnext[i];
#pragma unroll
                for (int ww = 0; ww < PS::NBW; ++ww) a += red[((q & 1) * PS::NBW + ww) * TILE_ELEMS + i * 64 + lane];
                sv[i] = rcur[i] - a;
            }
            v4 tn = {0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) tn = Mf<T>::mma(ecur[kc], sv[kc], tn);
            tnext = tn;
            sprev = sv;
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) dprev[kc] = dcur[kc];
            sprev_slot = okq ? sI : P.RS;
            Iprev = I;
            okprev = okq;
            sI = P.next_slot(sI);
        }
        {
            v4 y = {0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) y = Mf<T>::mma(dprev[kc], sprev[kc], y);
            store_y(y, ring + sprev_slot * TILE_ELEMS, Iprev, okprev);
        }
    } else if (w <= PS::NBW) {
        // ---- bulk waves
        const int wb = w - 1;
        T abuf[PD][TPW][4];
#pragma unroll
        for (int u = 0; u < PD - 1; ++u) P.load_bulk(u, wb, abuf[u]);
        lds_barrier();
        int sI = P.row_of(0) % P.RS;
        for (int q0 = 0; q0 < NTp; q0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int q = q0 + u;
                const int un = (u + PD - 1) % PD;
                P.load_bulk(q + PD - 1, wb, abuf[un]);
                __builtin_amdgcn_sched_barrier(0);
                const v4 acc = P.bulk_mma(q, wb, sI, abuf[u]);
#pragma unroll
                for (int i = 0; i < 4; ++i) red[((q & 1) * PS::NBW + wb) * TILE_ELEMS + i * 64 + lane] = acc[i];
                sI = P.next_slot(sI);
                lds_barrier();
            }
        }
    } else {
        // ---- helpers: stage the finisher's operands of row q+1 in hand[(q+1)%3]
        //      (D and E from the factor helper, r = x + dt phi f from the state helper)
        constexpr int PDH = 4;
        T b0[PDH][4], b1[PDH][4];
        const bool facw = (w == PS::NBW + 1);
        const int NTh = (NTp + PDH - 1) / PDH * PDH;
        if (facw) {
            auto post = [&](int q, const T (&v0)[4], const T (&v1)[4]) {
                T *h = hand + (q % 3) * 4 * TILE_ELEMS;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    h[i * 64 + lane] = v0[i];
                    h[TILE_ELEMS + i * 64 + lane] = v1[i];
                }
            };
#pragma unroll
            for (int u = 0; u < PDH - 1; ++u) P.load_de(u, b0[u], b1[u]);
            post(0, b0[0], b1[0]);
            lds_barrier();
            for (int q0 = 0; q0 < NTh; q0 += PDH) {
#pragma unroll
                for (int u = 0; u < PDH; ++u) {
                    const int q = q0 + u;
                    P.load_de(q + PDH - 1, b0[(u + PDH - 1) % PDH], b1[(u + PDH - 1) % PDH]);
                    __builtin_amdgcn_sched_barrier(0);
                    if (q < NTp) {
                        post(q + 1, b0[(u + 1) % PDH], b1[(u + 1) % PDH]);
                        lds_barrier();
                    }
                }
            }
        } else {
            auto post = [&](int q, const T (&x)[4], const T (&fv)[4]) {
                T *h = hand + (q % 3) * 4 * TILE_ELEMS + 2 * TILE_ELEMS;
#pragma unroll
                for (int i = 0; i < 4; ++i) h[i * 64 + lane] = x[i] + fs * fv[i];
            };
#pragma unroll
            for (int u = 0; u < PDH - 1; ++u) P.load_state(u, X, ldx, col, fsrc, fstride, b0[u], b1[u]);
            post(0, b0[0], b1[0]);
            lds_barrier();
            for (int q0 = 0; q0 < NTh; q0 += PDH) {
#pragma unroll
                for (int u = 0; u < PDH; ++u) {
                    const int q = q0 + u;
                    P.load_state(q + PDH - 1, X, ldx, col, fsrc, fstride, b0[(u + PDH - 1) % PDH],
                                 b1[(u + PDH - 1) % PDH]);
                    __builtin_amdgcn_sched_barrier(0);
                    if (q < NTp) {
                        post(q + 1, b0[(u + 1) % PDH], b1[(u + 1) % PDH]);
                        lds_barrier();
                    }
                }
            }
        }
    }
    // end of pass: the next pass reads X rows stored by wave 0
    __syncthreads();
}

// ADJ: adjoint sweep, on the mirrored set or (STRIDED) the transposed
// forward tiles.
template <typename T, int KW, int TPW, int PD, bool ADJ, bool STRIDED>
__global__ __launch_bounds__(64 * KW) void k_sweep(const SweepItem *__restrict__ items, int nitems,
                                                   int nsteps) {
    extern __shared__ __align__(16) unsigned char smem[];
    for (int idx = blockIdx.x; idx < nitems; idx += gridDim.x) {
        const SweepItem it = items[idx];
        T *ring = (T *)smem;
        // the ring must hold finite values only: zero tiles multiply stale slots
        for (int e = threadIdx.x; e < (it.fac.nb + 2) * TILE_ELEMS; e += blockDim.x) ring[e] = (T)0;
        __syncthreads();
        T *red = ring + (it.fac.nb + 2) * TILE_ELEMS;              // [2][KW-3][256]
        T *hand = red + 2 * (KW > 1 ? KW - 3 : 1) * TILE_ELEMS;     // [3][4][256]
        const void *const *a = it.fac.a;
        for (int step = 0; step < nsteps; ++step) {
            if (!ADJ) {
                sweep_pass<T, KW, TPW, PD, true, false>(it, (const T *)a[TS_LB], (const T *)a[TS_DL],
                                                        (const T *)a[TS_EL], ring, red, hand, it.f != nullptr,
                                                        step, nsteps);
                sweep_pass<T, KW, TPW, PD, false, false>(it, (const T *)a[TS_UB], (const T *)a[TS_DU],
                                                         (const T *)a[TS_EU], ring, red, hand, false, step, nsteps);
            } else if (!STRIDED) {
                sweep_pass<T, KW, TPW, PD, true, false>(it, (const T *)a[TS_UTB], (const T *)a[TS_DUT],
                                                        (const T *)a[TS_EUT], ring, red, hand, false, step, nsteps);
                sweep_pass<T, KW, TPW, PD, false, false>(it, (const T *)a[TS_LTB], (const T *)a[TS_DLT],
                                                         (const T *)a[TS_ELT], ring, red, hand, false, step, nsteps);
            } else {
                sweep_pass<T, KW, TPW, PD, true, true>(it, (const T *)a[TS_UB], (const T *)a[TS_DUT],
                                                       (const T *)a[TS_EUT], ring, red, hand, false, step, nsteps);
                sweep_pass<T, KW, TPW, PD, false, true>(it, (const T *)a[TS_LB], (const T *)a[TS_DLT],
                                                        (const T *)a[TS_ELT], ring, red, hand, false, step, nsteps);
            }
        }
    }
}

template <typename T, int KW, int TPW, int PD>
static hipError_t launch_t(bool adjoint, bool strided, int nitems, const SweepItem *d_items, int nsteps,
                           int max_nb, hipStream_t s) {
    // LDS: ring of nb+1 solved tiles (+1 dummy slot), double-buffered partial
    // sums of the bulk waves, triple-buffered hand-off (D, E, r)
    const size_t lds = (size_t)(max_nb + 2 + 2 * (KW > 1 ? KW - 3 : 1) + 12) * TILE_ELEMS * sizeof(T);
    const int grid = nitems < 65536 ? nitems : 65536;
    if (!adjoint)
        hipLaunchKernelGGL((k_sweep<T, KW, TPW, PD, false, false>), dim3(grid), dim3(64 * KW), lds, s, d_items,
                           nitems, nsteps);
    else if (!strided)
        hipLaunchKernelGGL((k_sweep<T, KW, TPW, PD, true, false>), dim3(grid), dim3(64 * KW), lds, s, d_items,
                           nitems, nsteps);
    else
        hipLaunchKernelGGL((k_sweep<T, KW, TPW, PD, true, true>), dim3(grid), dim3(64 * KW), lds, s, d_items,
                           nitems, nsteps);
    return hipGetLastError();
}

// KW > 1: wave 0 finishes tile rows, KW-3 bulk waves share the nb-1 older
// band tiles (TPW = ceil((nb-1)/(KW-3)) each), two helper waves prefetch the
// finisher's operands.  Narrow bands run on one wave.
template <typename T>
static hipError_t launch_prec(bool adjoint, bool strided, int nitems, const SweepItem *d_items, int nsteps,
                              int max_nb, hipStream_t s) {
    if (max_nb <= 1) return launch_t<T, 1, 1, 3>(adjoint, strided, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 4) return launch_t<T, 1, 3, 3>(adjoint, strided, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 8)
        return launch_t<T, 8, 2, sizeof(T) == 8 ? 4 : 6>(adjoint, strided, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 16)
        return launch_t<T, 8, 3, sizeof(T) == 8 ? 4 : 5>(adjoint, strided, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 32) return launch_t<T, 8, 7, 3>(adjoint, strided, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 64) return launch_t<T, 8, 13, 2>(adjoint, strided, nitems, d_items, nsteps, max_nb, s);
    return hipErrorInvalidValue;
}

hipError_t launch_sweep(bool adjoint, bool strided, bool f32, int nitems, const SweepItem *d_items, int nsteps,
                        int max_nb, hipStream_t s) {
    if (nitems <= 0 || nsteps <= 0) return hipSuccess;
    if (f32) return launch_prec<float>(adjoint, strided, nitems, d_items, nsteps, max_nb, s);
    return launch_prec<double>(adjoint, strided, nitems, d_items, nsteps, max_nb, s);
}

}  // namespace lrpr
