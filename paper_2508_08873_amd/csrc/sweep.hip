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

// Loads and stores through address space 1 compile to global_* instructions
// (flat_* would also count against the LDS counter and be drained by every
// LDS barrier, cancelling the prefetch).
template <typename T> using gptr = __attribute__((address_space(1))) const T *;
template <typename T> using gptr_mut = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ T gld(const T *p) { return *(gptr<T>)p; }
template <typename T> __device__ __forceinline__ void gst(T *p, T v) { *(gptr_mut<T>)p = v; }

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
// Per tile row I the nb band tiles split into the "newest" one (J = I-1 when
// ascending, I+1 when descending), whose right-hand factor y_J wave 0 still
// holds in registers, and nb-1 "bulk" tiles (J further away) that all KW
// waves share, reading y_J from the LDS ring.  Operands of the next PD tile
// rows are prefetched into registers, so global-memory latency overlaps the
// matrix-core work.  One barrier per tile row: before it the waves post their
// bulk partial sums (double-buffered), after it wave 0 finishes the row
// (source term, newest tile, diagonal inverse, ring and HBM store).
template <typename T> struct NewestOff;
// f64: the accumulator register kc holds rows 4kc + lane/16, i.e. the B
// operand of chunk kc in the standard k order, same A offsets as bulk tiles.
template <> struct NewestOff<double> {
    __device__ static inline void get(bool trans, int c, int g, int off_fwd, int off_adj, int &off, int &stride) {
        off = trans ? off_adj : off_fwd;
        stride = trans ? 16 : 64;
    }
};
// f32: register kc holds rows 4*(lane/16) + kc, so chunk kc contracts over
// k = 4*(lane/16) + kc; in the sub-block layout a lane's four chunks are
// adjacent (forward) or 4 apart (transposed).
template <> struct NewestOff<float> {
    __device__ static inline void get(bool trans, int c, int g, int, int, int &off, int &stride) {
        if (!trans) {
            off = (g * 4 + (c >> 2)) * 16 + (c & 3) * 4;
            stride = 1;
        } else {
            off = ((c >> 2) * 4 + g) * 16 + (c & 3);
            stride = 4;
        }
    }
};

// Barrier that orders LDS traffic only: outstanding global loads (the
// prefetches of later tile rows) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Roles of the waves of a workgroup (KW > 1):
//   wave 0          finisher: newest tile, source term, diagonal inverse,
//                   ring and HBM store of each tile row; no global loads;
//   waves 1..NBW    bulk: partial sums over the nb-1 older band tiles;
//   wave NBW+1      factor helper: prefetches the newest band tile and the
//                   diagonal inverse of coming rows, hands them to wave 0
//                   through LDS;
//   wave NBW+2      state helper: prefetches the right-hand side rows (state
//                   and source) the same way.
// With KW == 1 (narrow bands) the single wave does everything.
template <typename T, int KW, int TPW, int PD, bool ASC, bool TRANS>
struct Pass {
    typedef typename Mf<T>::v4 v4;
    static constexpr int NBW = KW > 1 ? KW - 3 : 1;   // bulk waves
    const SweepItem &it;
    const T *__restrict__ band;
    const T *__restrict__ dtile;
    const T *__restrict__ etile;
    const T *__restrict__ zt;
    T *ring;
    T *red;   // [2][NBW][256]
    T *hand;  // [3][4][256]: newest, D, x, f
    int lane, w, g, c, n, NT, nb, RS, nbulk;
    int boff, bstr, noff, nstr;

    __device__ Pass(const SweepItem &it_, const T *band_, const T *dtile_, const T *etile_, T *ring_, T *red_,
                    T *hand_)
        : it(it_), band(band_), dtile(dtile_), etile(etile_), zt((const T *)it_.fac.zt), ring(ring_), red(red_),
          hand(hand_) {
        lane = threadIdx.x & 63;
        w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform (scalar)
        g = lane >> 4;
        c = lane & 15;
        n = it.fac.n;
        NT = it.fac.NT;
        nb = it.fac.nb;
        RS = nb + 1;
        nbulk = nb - 1;
        const int off_fwd = ((c >> 2) * 16) + ((c & 3) * 4) + g;   // + 64*kc; lane's row = c
        const int off_adj = ((c >> 2) * 64) + (g * 4) + (c & 3);   // + 16*kc
        boff = TRANS ? off_adj : off_fwd;
        bstr = TRANS ? 16 : 64;
        NewestOff<T>::get(TRANS, c, g, off_fwd, off_adj, noff, nstr);
    }
    __device__ __forceinline__ int row_of(int q) const { return ASC ? q : NT - 1 - q; }
    __device__ __forceinline__ const T *tile_ptr(int I, int j, int J) const {
        if (TRANS) return band + ((int64_t)J * nb + (nb - 1 - j)) * TILE_ELEMS;
        return band + ((int64_t)I * nb + j) * TILE_ELEMS;
    }
    // bulk tile t of this wave (wb = index among the bulk waves).  Tile rows
    // outside [0, NT) are zero guard rows of the tile arrays, so every address
    // within the prefetch window is valid; only surplus slots (idx >= nb-1)
    // read the zero tile.
    __device__ __forceinline__ bool bulk(int q, int wb, int t, int &j, int &J) const {
        const int I = row_of(q);
        const int idx = wb + NBW * t;
        j = ASC ? idx : idx + 1;
        J = ASC ? I - nb + j : I + 1 + j;
        return idx < nbulk;
    }
    template <int NTP>
    __device__ __forceinline__ void load_bulk(int q, int wb, T (&ab)[NTP][4]) const {
        const int I = row_of(q);
#pragma unroll
        for (int t = 0; t < NTP; ++t) {
            int j, J;
            const T *tp = bulk(q, wb, t, j, J) ? tile_ptr(I, j, J) : zt;
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) ab[t][kc] = gld(tp + boff + bstr * kc);
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
    // operands of the finisher for row q: newest band tile and diagonal inverse
    __device__ __forceinline__ void load_fac(int q, T (&nbv)[4], T (&dbv)[4]) const {
        const int I = row_of(q);
        const int jn = ASC ? nb - 1 : 0;
        const int Jn = ASC ? I - 1 : I + 1;
        const T *tn = tile_ptr(I, jn, Jn);           // guard rows are zero
        const T *D = dtile + (int64_t)I * TILE_ELEMS;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            nbv[kc] = gld(tn + noff + nstr * kc);
            dbv[kc] = gld(D + kc * 64 + lane);
        }
    }
    // finisher operands staged for row q: diagonal inverse of row q and the
    // newest-tile product E of row q+1 (applied to the residual s of row q)
    __device__ __forceinline__ void load_de(int q, T (&dbv)[4], T (&ebv)[4]) const {
        const T *D = dtile + (int64_t)row_of(q) * TILE_ELEMS;
        const T *E = etile + (int64_t)row_of(q + 1) * TILE_ELEMS;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            dbv[kc] = gld(D + kc * 64 + lane);
            ebv[kc] = gld(E + kc * 64 + lane);
        }
    }
    // right-hand side rows of row q: state x and source f (D-layout rows)
    __device__ __forceinline__ void load_state(int q, const T *X, int64_t ldx, bool colok, const T *fsrc,
                                               int64_t fstride, T (&xbv)[4], T (&fbv)[4]) const {
        const int I = row_of(q);
        const bool okq = q < NT;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = I * TILE + Mf<T>::row(g, i);
            const bool okr = okq && colok && row < n;
            xbv[i] = gld(okr ? X + row + (int64_t)c * ldx : zt);
            fbv[i] = gld(okr ? fsrc + row * fstride : zt);
        }
    }
};

template <typename T, int KW, int TPW, int PD, bool ASC, bool TRANS>
__device__ __forceinline__ void sweep_pass(const SweepItem &it, const T *__restrict__ band,
                                           const T *__restrict__ dtile, const T *__restrict__ etile, T *ring,
                                           T *red, T *hand, bool with_src, int step, int nsteps) {
    typedef typename Mf<T>::v4 v4;
    typedef Pass<T, KW, TPW, PD, ASC, TRANS> PS;
    PS P(it, band, dtile, etile, ring, red, hand);
    const int NT = P.NT, lane = P.lane, g = P.g, c = P.c, n = P.n;
    const int NTp = (NT + PD - 1) / PD * PD;   // rows beyond NT are zero work
    T *X = (T *)it.X;
    const int64_t ldx = it.ldx;
    const bool colok = c < it.ncols;
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
    if (KW == 1) {
        // ---- single wave: everything, prefetching PD-1 rows ahead
        T abuf[PD][TPW][4];
        T nbuf[PD][4], dbuf[PD][4], xbuf[PD][4], fbuf[PD][4];
#pragma unroll
        for (int u = 0; u < PD - 1; ++u) {
            P.load_bulk(u, 0, abuf[u]);
            P.load_fac(u, nbuf[u], dbuf[u]);
            P.load_state(u, X, ldx, colok, fsrc, fstride, xbuf[u], fbuf[u]);
        }
        v4 yprev = {0, 0, 0, 0};
        int sI = P.row_of(0) % P.RS;
        for (int q0 = 0; q0 < NTp; q0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int q = q0 + u;
                const int un = (u + PD - 1) % PD;
                P.load_bulk(q + PD - 1, 0, abuf[un]);
                P.load_fac(q + PD - 1, nbuf[un], dbuf[un]);
                P.load_state(q + PD - 1, X, ldx, colok, fsrc, fstride, xbuf[un], fbuf[un]);
                __builtin_amdgcn_sched_barrier(0);
                const bool okq = q < NT;
                const int I = P.row_of(q);
                v4 a = P.bulk_mma(q, 0, sI, abuf[u]);
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) a = Mf<T>::mma(nbuf[u][kc], yprev[kc], a);
                v4 sv;
#pragma unroll
                for (int i = 0; i < 4; ++i) sv[i] = (xbuf[u][i] + fs * fbuf[u][i]) - a[i];
                v4 y = {0, 0, 0, 0};
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) y = Mf<T>::mma(dbuf[u][kc], sv[kc], y);
                T *ri = ring + (okq ? sI : P.RS) * TILE_ELEMS;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int rr = Mf<T>::row(g, i);
                    ri[rr * TILE + c] = y[i];
                    const int row = I * TILE + rr;
                    gst((okq && colok && row < n) ? X + row + (int64_t)c * ldx : sink + lane, y[i]);
                }
                yprev = y;
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
            // y_{q-1} = D_{q-1} s_{q-1}: ring and HBM
            {
                v4 y = {0, 0, 0, 0};
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) y = Mf<T>::mma(dprev[kc], sprev[kc], y);
                T *ri = ring + sprev_slot * TILE_ELEMS;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int rr = Mf<T>::row(g, i);
                    ri[rr * TILE + c] = y[i];
                    const int row = Iprev * TILE + rr;
                    gst((okprev && colok && row < n) ? X + row + (int64_t)c * ldx : sink + lane, y[i]);
                }
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
        // last row's solution
        {
            v4 y = {0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) y = Mf<T>::mma(dprev[kc], sprev[kc], y);
            T *ri = ring + sprev_slot * TILE_ELEMS;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int rr = Mf<T>::row(g, i);
                ri[rr * TILE + c] = y[i];
                const int row = Iprev * TILE + rr;
                gst((okprev && colok && row < n) ? X + row + (int64_t)c * ldx : sink + lane, y[i]);
            }
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
                v4 acc = P.bulk_mma(q, wb, sI, abuf[u]);
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
        if (w == PS::NBW + 1) {
            T b0[PDH][4], b1[PDH][4];
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
            const int NTh = (NTp + PDH - 1) / PDH * PDH;
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
            T b0[PDH][4], b1[PDH][4];
            auto post = [&](int q, const T (&x)[4], const T (&fv)[4]) {
                T *h = hand + (q % 3) * 4 * TILE_ELEMS + 2 * TILE_ELEMS;
#pragma unroll
                for (int i = 0; i < 4; ++i) h[i * 64 + lane] = x[i] + fs * fv[i];
            };
#pragma unroll
            for (int u = 0; u < PDH - 1; ++u) P.load_state(u, X, ldx, colok, fsrc, fstride, b0[u], b1[u]);
            post(0, b0[0], b1[0]);
            lds_barrier();
            const int NTh = (NTp + PDH - 1) / PDH * PDH;
            for (int q0 = 0; q0 < NTh; q0 += PDH) {
#pragma unroll
                for (int u = 0; u < PDH; ++u) {
                    const int q = q0 + u;
                    P.load_state(q + PDH - 1, X, ldx, colok, fsrc, fstride, b0[(u + PDH - 1) % PDH],
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

template <typename T, int KW, int TPW, int PD, bool ADJ>
__global__ __launch_bounds__(64 * KW) void k_sweep(const SweepItem *__restrict__ items, int nitems,
                                                   int nsteps) {
    extern __shared__ __align__(16) unsigned char smem[];
    for (int idx = blockIdx.x; idx < nitems; idx += gridDim.x) {
        const SweepItem it = items[idx];
        T *ring = (T *)smem;
        // the ring must hold finite values only: zero tiles multiply stale slots
        for (int e = threadIdx.x; e < (it.fac.nb + 2) * TILE_ELEMS; e += blockDim.x) ring[e] = (T)0;
        __syncthreads();
        T *red = ring + (it.fac.nb + 2) * TILE_ELEMS;   // [2][KW-3][256]
        T *hand = red + 2 * (KW > 1 ? KW - 3 : 1) * TILE_ELEMS;   // [3][4][256]
        const T *Lb = (const T *)it.fac.Lb, *Ub = (const T *)it.fac.Ub;
        for (int step = 0; step < nsteps; ++step) {
            if (!ADJ) {
                sweep_pass<T, KW, TPW, PD, true, false>(it, Lb, (const T *)it.fac.DL, (const T *)it.fac.EL, ring, red, hand,
                                                    it.f != nullptr, step, nsteps);
                sweep_pass<T, KW, TPW, PD, false, false>(it, Ub, (const T *)it.fac.DU, (const T *)it.fac.EU, ring, red, hand, false,
                                                     step, nsteps);
            } else {
                sweep_pass<T, KW, TPW, PD, true, true>(it, Ub, (const T *)it.fac.DUT, (const T *)it.fac.EUT, ring, red, hand, false,
                                                   step, nsteps);
                sweep_pass<T, KW, TPW, PD, false, true>(it, Lb, (const T *)it.fac.DLT, (const T *)it.fac.ELT, ring, red, hand, false,
                                                    step, nsteps);
            }
        }
    }
}

template <typename T, int KW, int TPW, int PD>
static hipError_t launch_t(bool adjoint, int nitems, const SweepItem *d_items, int nsteps, int max_nb,
                           hipStream_t s) {
    // LDS: ring of nb+1 solved tiles + double-buffered partial sums of KW-1 waves
    const size_t lds = (size_t)(max_nb + 2 + 2 * (KW > 1 ? KW - 3 : 1) + 12) * TILE_ELEMS * sizeof(T);
    const int grid = nitems < 65536 ? nitems : 65536;
    if (adjoint)
        hipLaunchKernelGGL((k_sweep<T, KW, TPW, PD, true>), dim3(grid), dim3(64 * KW), lds, s, d_items,
                           nitems, nsteps);
    else
        hipLaunchKernelGGL((k_sweep<T, KW, TPW, PD, false>), dim3(grid), dim3(64 * KW), lds, s, d_items,
                           nitems, nsteps);
    return hipGetLastError();
}

// KW > 1: wave 0 finishes tile rows, KW-3 bulk waves share the nb-1 older
// band tiles (TPW = ceil((nb-1)/(KW-3)) each), two helper waves prefetch the
// finisher's operands.  Narrow bands run on one wave.
template <typename T>
static hipError_t launch_prec(bool adjoint, int nitems, const SweepItem *d_items, int nsteps,
                              int max_nb, hipStream_t s) {
    if (max_nb <= 1) return launch_t<T, 1, 1, 3>(adjoint, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 4) return launch_t<T, 1, 3, 3>(adjoint, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 8) return launch_t<T, 8, 2, sizeof(T) == 8 ? 4 : 6>(adjoint, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 16) return launch_t<T, 8, 3, sizeof(T) == 8 ? 4 : 5>(adjoint, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 32) return launch_t<T, 8, 7, 3>(adjoint, nitems, d_items, nsteps, max_nb, s);
    if (max_nb <= 64) return launch_t<T, 8, 13, 2>(adjoint, nitems, d_items, nsteps, max_nb, s);
    return hipErrorInvalidValue;
}

hipError_t launch_sweep(bool adjoint, bool f32, int nitems, const SweepItem *d_items, int nsteps,
                        int max_nb, hipStream_t s) {
    if (nitems <= 0 || nsteps <= 0) return hipSuccess;
    if (f32) return launch_prec<float>(adjoint, nitems, d_items, nsteps, max_nb, s);
    return launch_prec<double>(adjoint, nitems, d_items, nsteps, max_nb, s);
}

}  // namespace lrpr
