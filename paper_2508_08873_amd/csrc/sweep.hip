// Batched implicit-Euler sweeps through a banded LU on gfx950 (CDNA4).
//
// One implicit-Euler step of the fine propagator solves (I + dt A) x_new =
// x_old + dt f(t_new) with M = L U: a forward substitution with L, then a
// back substitution with U (Sec. 2, eq. F_n_affine; the paper's solver reuses
// one factorisation for all right-hand sides of a step, Sec. 4.4).  The
// adjoint (Sec. 2.1, step 3) solves M^T z = x with M^T = U^T L^T: forward
// with U^T, back with L^T.  Both are the same two-pass sweep over band tiles:
// the forward set holds L and U, the mirrored set U^T and L^T of the same LU.
//
// Blocking.  Rows are cut into tile rows of 16.  The band tiles are stored
// multiplied from the left by their row's diagonal-tile inverse D_I, so a
// pass reads, per tile row I,
//     v_I = D_I r_I - sum_{bulk J} A_IJ v_J - A_{I,I-1} v_{I-1}      (left)
// with v the pass's solution.  Without a mirrored set the adjoint reads the
// forward tiles transposed, which are multiplied from the right instead:
//     v_I = r_I - sum_{bulk J} B_IJ v_J - B_{I,I-1} v_{I-1},  y_I = D_I v_I
// (right).  Either way the row-to-row recurrence runs through one 16x16x16
// product with the newest tile; every product runs on the matrix cores
// (v_mfma_*_16x16x4), 16 right-hand sides per workgroup.
//
// Waves of a workgroup (KW = 8), one LDS barrier per tile row:
//   wave 0        finisher: v = r - partials - t, ring store, t = E v;
//   waves 1..5    bulk: partial sums over the nb-1 older band tiles, operands
//                 prefetched PD-1 tile rows ahead into registers;
//   wave 6        factor helper: hands the newest tile E of the coming row to
//                 the finisher; writes the pass output (v, or D v) to HBM;
//   wave 7        state helper: hands r (D (x + dt phi f), or x) to the
//                 finisher.
// The finisher computes row q after barrier q+1 from the bulk partials of row
// q (computed between barriers q and q+1) and the hand-off of row q.  The last
// nb solved tiles live in an LDS ring.  Narrow bands (nb <= 4) run one wave.
#include "lrpr_internal.h"
#include "tile_ops.h"

namespace lrpr {

constexpr int max5(int a, int b, int c, int d, int e) {
    int m = a;
    m = b > m ? b : m;
    m = c > m ? c : m;
    m = d > m ? d : m;
    return e > m ? e : m;
}

// Distribution of the nb-1 older ("bulk") band tiles of a tile row over the
// five bulk waves 1..5: wave w takes the contiguous range after the counts of
// the waves before it.  Waves w and w+4 share a SIMD (and so its matrix core);
// wave 0 (finisher) sits on SIMD 0 and the helpers on SIMDs 2 and 3.
template <int C1, int C2, int C3, int C4, int C5>
struct Split {
    static constexpr int c1 = C1, c2 = C2, c3 = C3, c4 = C4, c5 = C5;
    static constexpr int cmax = max5(C1, C2, C3, C4, C5);
    __host__ __device__ static constexpr int cn(int wb) {
        return wb == 0 ? C1 : wb == 1 ? C2 : wb == 2 ? C3 : wb == 3 ? C4 : C5;
    }
    __host__ __device__ static constexpr int st(int wb) {
        return (wb > 0 ? C1 : 0) + (wb > 1 ? C2 : 0) + (wb > 2 ? C3 : 0) + (wb > 3 ? C4 : 0);
    }
};

// One pass (ascending or descending tile rows) over one 16-column group.
//   band  : band tiles of the pass, nb per tile row (row I, index j)
//   dtile : diagonal-tile inverses (one per row)
//   STRIDED: the band tiles are the forward set's, read transposed (tile (row
//            J, index nb-1-j), each lane gathering its four values); the pass
//            then runs the right form, otherwise the left form.
// Registers and LDS hold 16x16 blocks in accumulator order: value i of lane
// l is row Mf::row(l/16, i), column l%16 — the B operand of chunk i.
template <typename T, int KW, int PD, bool ASC, bool STRIDED>
struct Pass {
    typedef typename Mf<T>::v4 v4;
    static constexpr int NBW = KW > 1 ? KW - 3 : 1;   // bulk waves
    const T *__restrict__ band;
    const T *__restrict__ dtile;
    const T *__restrict__ zt;
    T *ring;
    int lane, w, g, c, n, NT, nb, RS, nbulk;   // NT: tile rows of the item's range
    int r0, r1;                                 // the range [r0, r1) of tile rows
    int soff[4];   // STRIDED: position of this lane's chunk values in a forward tile

    __device__ Pass(const SweepItem &it, const T *band_, const T *dtile_, T *ring_)
        : band(band_), dtile(dtile_), zt((const T *)it.fac.zt), ring(ring_) {
        lane = threadIdx.x & 63;
        w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform (scalar)
        g = lane >> 4;
        c = lane & 15;
        n = it.fac.n;
        r0 = it.r0;
        r1 = it.r1;
        NT = r1 - r0;
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
    __device__ __forceinline__ int row_of(int q) const { return ASC ? r0 + q : r1 - 1 - q; }
    __device__ __forceinline__ const T *tile_ptr(int I, int j, int J) const {
        if (STRIDED) return band + ((int64_t)J * nb + (nb - 1 - j)) * TILE_ELEMS;
        return band + ((int64_t)I * nb + j) * TILE_ELEMS;
    }
    // bulk tile idx (0..nb-2) of row q.  Tile rows outside [0, NT) are zero
    // guard rows of the tile arrays, so every address within the prefetch
    // window is valid; surplus slots (idx >= nb-1, on factors with fewer band
    // tiles than the launch's widest) read the zero tile and take the first
    // bulk tile's index, so that their ring slot stays inside the ring.
    __device__ __forceinline__ bool bulk(int q, int idx, int &j, int &J) const {
        const int I = row_of(q);
        const bool ok = idx < nbulk;
        const int id = ok ? idx : 0;
        j = ASC ? id : id + 1;
        J = ASC ? I - nb + j : I + 1 + j;
        return ok;
    }
    __device__ __forceinline__ void ld_tile(const T *tp, T (&v)[4]) const {
        if (STRIDED) {
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) v[kc] = gld(tp + soff[kc]);
        } else {
            Mf<T>::ld4(tp, lane, v);
        }
    }
    // tiles st..st+cn-1 of row q into slots 0..cn-1 (loads are unconditional:
    // slots >= cn read the zero tile)
    template <int NTP>
    __device__ __forceinline__ void load_bulk(int q, int st, int cn, T (&ab)[NTP][4]) const {
        const int I = row_of(q);
#pragma unroll
        for (int t = 0; t < NTP; ++t) {
            int j, J;
            const bool ok = bulk(q, st + t, j, J) && t < cn;
            ld_tile(ok ? tile_ptr(I, j, J) : zt, ab[t]);
        }
    }
    // newest band tile of row q (J = I-1 ascending, I+1 descending)
    __device__ __forceinline__ void load_newest(int q, T (&v)[4]) const {
        const int I = row_of(q);
        ld_tile(ASC ? tile_ptr(I, nb - 1, I - 1) : tile_ptr(I, 0, I + 1), v);
    }
    __device__ __forceinline__ void load_d(int q, T (&v)[4]) const {
        Mf<T>::ld4(dtile + (int64_t)row_of(q) * TILE_ELEMS, lane, v);
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
    // products of slots t < cn (a wave-uniform branch skips the rest); two
    // accumulator chains interleave on the matrix core
    template <int NTP>
    __device__ __forceinline__ v4 bulk_mma(int q, int sI, int st, int cn, const T (&ab)[NTP][4]) const {
        constexpr int NA = NTP < 2 ? NTP : 2;
        v4 acc[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) acc[a] = v4{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < NTP; ++t) {
            if (t < cn) {
                int j, J;
                bulk(q, st + t, j, J);
                T bv[4];
                ring_ld(ring + slot_of(sI, j) * TILE_ELEMS, bv);
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) acc[t % NA] = Mf<T>::mma(ab[t][kc], bv[kc], acc[t % NA]);
            }
        }
#pragma unroll
        for (int a = 1; a < NA; ++a) acc[0] += acc[a];
        return acc[0];
    }
    // ring tiles keep a lane's four values together (one wide LDS access)
    __device__ __forceinline__ void ring_ld(const T *tile, T (&v)[4]) const {
        const v4 x = *(const v4 *)(tile + 4 * lane);
        v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
    }
    __device__ __forceinline__ void ring_st(T *tile, const v4 &v) const { *(v4 *)(tile + 4 * lane) = v; }
    __device__ __forceinline__ int next_slot(int sI) const {
        return ASC ? (sI + 1 == RS ? 0 : sI + 1) : (sI == 0 ? RS - 1 : sI - 1);
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
    // (D t) for t in accumulator order (t as B operand)
    __device__ __forceinline__ v4 dmul(const T (&d)[4], const v4 &t) const {
        v4 y = {0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) y = Mf<T>::mma(d[kc], t[kc], y);
        return y;
    }
};

// Bulk wave WB of a sweep: tiles [ST, ST+CN) of row q between barriers q
// and q+1, operands prefetched PD-1 rows ahead.  Products accumulate in two
// chains per group (even and odd tiles), as in Pass::bulk_mma.
template <typename T, typename PS, typename SP, int PD, int NG, int WB>
__device__ __forceinline__ void sweep_bulk(const PS &P, int NTp, T *red, int grs) {
    typedef typename Mf<T>::v4 v4;
    constexpr int CN = SP::cn(WB), ST = SP::st(WB), NBW = PS::NBW;
    constexpr int NA = SP::cmax < 2 ? SP::cmax : 2;
    const int lane = P.lane;
    if constexpr (CN == 0) {
        lds_barrier();
        for (int q = 0; q < NTp; ++q) {
            T *rd = red + ((q & 1) * NBW + WB) * NG * TILE_ELEMS;
#pragma unroll
            for (int k = 0; k < NG; ++k)
#pragma unroll
                for (int i = 0; i < 4; ++i) rd[k * TILE_ELEMS + i * 64 + lane] = (T)0;
            lds_barrier();
        }
        __syncthreads();
        return;
    } else {
        T abuf[PD][CN][4];
#pragma unroll
        for (int u = 0; u < PD - 1; ++u) P.template load_bulk<CN>(u, ST, CN, abuf[u]);
        lds_barrier();
        int sI = P.row_of(0) % P.RS;
        for (int q0 = 0; q0 < NTp; q0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int q = q0 + u;
                const int un = (u + PD - 1) % PD;
                P.template load_bulk<CN>(q + PD - 1, ST, CN, abuf[un]);
                __builtin_amdgcn_sched_barrier(0);
                // ring operands of tile t+1 are read while tile t's products run
                auto ring_read = [&](int t, T (&bv)[NG][4]) {
                    int j, J;
                    P.bulk(q, ST + t, j, J);
                    const T *rj = P.ring + P.slot_of(sI, j) * TILE_ELEMS;
#pragma unroll
                    for (int k = 0; k < NG; ++k) P.ring_ld(rj + k * grs, bv[k]);
                };
                v4 acc[NA][NG];
#pragma unroll
                for (int a = 0; a < NA; ++a)
#pragma unroll
                    for (int k = 0; k < NG; ++k) acc[a][k] = v4{0, 0, 0, 0};
                T bv[2][NG][4];
                ring_read(0, bv[0]);
#pragma unroll
                for (int t = 0; t < CN; ++t) {
                    if (t + 1 < CN) ring_read(t + 1, bv[(t + 1) & 1]);
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc)
#pragma unroll
                        for (int k = 0; k < NG; ++k)
                            acc[t % NA][k] = Mf<T>::mma(abuf[u][t][kc], bv[t & 1][k][kc], acc[t % NA][k]);
                }
                T *rd = red + ((q & 1) * NBW + WB) * NG * TILE_ELEMS;
#pragma unroll
                for (int k = 0; k < NG; ++k) {
                    v4 r = acc[0][k];
#pragma unroll
                    for (int a = 1; a < NA; ++a) r += acc[a][k];
#pragma unroll
                    for (int i = 0; i < 4; ++i) rd[k * TILE_ELEMS + i * 64 + lane] = r[i];
                }
                sI = P.next_slot(sI);
                lds_barrier();
            }
        }
        __syncthreads();
    }
}

// One pass over NG 16-column groups of one item (columns 16 i .. 16 i + 15
// of the item in group i).  Every band tile loaded by a bulk wave multiplies
// the solved tiles of all NG groups, so the factor streams from HBM once per
// NG groups; the finisher runs NG independent chains.  LDS: ring [NG][nb+2],
// partial sums [2][bulk waves][NG], hand-off [2][1 + NG] (E, then r of each
// group), all in tiles.
template <typename T, int KW, typename SP, int PD, bool ASC, bool STRIDED, int NG>
__device__ __forceinline__ void sweep_pass(const SweepItem &it, const T *__restrict__ band,
                                           const T *__restrict__ dtile, T *ring, T *red, T *hand, bool with_src,
                                           int step, int nsteps) {
    static_assert(KW > 1 || NG == 1, "the single-wave sweep handles one column group");
    typedef typename Mf<T>::v4 v4;
    typedef Pass<T, KW, PD, ASC, STRIDED> PS;
    constexpr int TPW = SP::cmax;
    constexpr bool LEFT = !STRIDED;   // left form: r = D (x + dt phi f); right form: y = D v
    constexpr int HS = (1 + NG) * TILE_ELEMS;   // one hand-off buffer
    PS P(it, band, dtile, ring);
    const int NT = P.NT, lane = P.lane, g = P.g, c = P.c, n = P.n;
    const int NTp = (NT + PD - 1) / PD * PD;   // rows beyond NT are zero work
    const int grs = (P.nb + 2) * TILE_ELEMS;    // ring stride between groups
    T *X = (T *)it.X;
    const int64_t ldx = it.ldx;
    bool colok[NG];
    int col[NG];
    // source of this lane's columns: f(x) * dt * phi(t_step), or the zero tile
    const T *fsrc[NG];
    int64_t fstride[NG];
    T fs[NG];
#pragma unroll
    for (int i = 0; i < NG; ++i) {
        const int cc = 16 * i + c;
        colok[i] = cc < it.ncols;
        col[i] = colok[i] ? cc : 0;
        fsrc[i] = P.zt;
        fstride[i] = 0;
        fs[i] = 0;
        if (with_src && colok[i]) {
            const int fc = it.fcol ? gld(it.fcol + cc) : 0;
            if (fc >= 0) {
                fsrc[i] = (const T *)it.f + (int64_t)fc * it.ldf;
                fstride[i] = 1;
                const double sc = it.fscale ? gld(it.fscale + (int64_t)cc * it.fsteps + step) : 1.0;
                fs[i] = (T)(it.fac.dt * sc);
            }
        }
    }
    T *sink = (T *)it.fac.sink;
    const int w = P.w;
    // pass output of tile row q (accumulator order) of group i to X
    auto store_out = [&](const v4 &y, int q, int i) {
        const int Irow = P.row_of(q);
        const bool ok = q < NT && colok[i];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = Irow * TILE + Mf<T>::row(g, e);
            gst((ok && row < n) ? X + row + (int64_t)col[i] * ldx : sink + lane, y[e]);
        }
    };
    if constexpr (KW == 1) {
        // ---- single wave: everything, prefetching PD-1 rows ahead
        T abuf[PD][TPW][4];
        T ebuf[PD][4], dbuf[PD][4], xbuf[PD][4], fbuf[PD][4];
#pragma unroll
        for (int u = 0; u < PD - 1; ++u) {
            P.template load_bulk<TPW>(u, 0, TPW, abuf[u]);
            P.load_newest(u + 1, ebuf[u]);
            P.load_d(u, dbuf[u]);
            P.load_state(u, X, ldx, col[0], fsrc[0], fstride[0], xbuf[u], fbuf[u]);
        }
        v4 t = {0, 0, 0, 0};
        int sI = P.row_of(0) % P.RS;
        for (int q0 = 0; q0 < NTp; q0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int q = q0 + u;
                const int un = (u + PD - 1) % PD;
                P.template load_bulk<TPW>(q + PD - 1, 0, TPW, abuf[un]);
                P.load_newest(q + PD, ebuf[un]);
                P.load_d(q + PD - 1, dbuf[un]);
                P.load_state(q + PD - 1, X, ldx, col[0], fsrc[0], fstride[0], xbuf[un], fbuf[un]);
                __builtin_amdgcn_sched_barrier(0);
                const v4 a = P.template bulk_mma<TPW>(q, sI, 0, TPW, abuf[u]);
                v4 r;
#pragma unroll
                for (int i = 0; i < 4; ++i) r[i] = xbuf[u][i] + fs[0] * fbuf[u][i];
                if (LEFT) r = P.dmul(dbuf[u], r);
                v4 v;
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = r[i] - (a[i] + t[i]);
                P.ring_st(ring + (q < NT ? sI : P.RS) * TILE_ELEMS, v);
                t = P.dmul(ebuf[u], v);
                store_out(LEFT ? v : P.dmul(dbuf[u], v), q, 0);
                sI = P.next_slot(sI);
                lds_barrier();
            }
        }
    } else if (w == 0) {
        // ---- finisher: row q after barrier q+1
        v4 t[NG];
#pragma unroll
        for (int k = 0; k < NG; ++k) t[k] = v4{0, 0, 0, 0};
        int sI = P.row_of(0) % P.RS;
        lds_barrier();
        for (int q = 0; q < NTp; ++q) {
            lds_barrier();
            const T *h = hand + (q & 1) * HS;
            T ecur[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) ecur[i] = h[i * 64 + lane];
            const int so = (q < NT ? sI : P.RS) * TILE_ELEMS;
#pragma unroll
            for (int k = 0; k < NG; ++k) {
                v4 v;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    T a = t[k][i];
#pragma unroll
                    for (int ww = 0; ww < PS::NBW; ++ww)
                        a += red[(((q & 1) * PS::NBW + ww) * NG + k) * TILE_ELEMS + i * 64 + lane];
                    v[i] = h[(1 + k) * TILE_ELEMS + i * 64 + lane] - a;
                }
                P.ring_st(ring + k * grs + so, v);
                t[k] = P.dmul(ecur, v);
            }
            sI = P.next_slot(sI);
        }
        __syncthreads();
    } else if (w <= PS::NBW) {
        // ---- bulk waves (compile-time share of each wave)
        switch (w) {
            case 1: sweep_bulk<T, PS, SP, PD, NG, 0>(P, NTp, red, grs); break;
            case 2: sweep_bulk<T, PS, SP, PD, NG, 1>(P, NTp, red, grs); break;
            case 3: sweep_bulk<T, PS, SP, PD, NG, 2>(P, NTp, red, grs); break;
            case 4: sweep_bulk<T, PS, SP, PD, NG, 3>(P, NTp, red, grs); break;
            default: sweep_bulk<T, PS, SP, PD, NG, 4>(P, NTp, red, grs); break;
        }
    } else {
        // ---- helpers: between barriers q and q+1 they hand over row q's r and
        //      row q+1's newest tile; the factor helper also writes the output
        //      of row q-2 (in the ring since barrier q)
#ifndef LRPR_PDH
#define LRPR_PDH 3
#endif
        constexpr int PDH = LRPR_PDH;   // helpers' prefetch depth
        const int NTh = (NTp + PDH - 1) / PDH * PDH;
        // output of ring slot so (tile row qo) of every group; D of the row
        // in the right form
        auto write_rows = [&](int so, int qo, const T (&d)[4]) {
#pragma unroll
            for (int k = 0; k < NG; ++k) {
                T x[4];
                P.ring_ld(ring + k * grs + so * TILE_ELEMS, x);
                const v4 v = {x[0], x[1], x[2], x[3]};
                store_out(LEFT ? v : P.dmul(d, v), qo, k);
            }
        };
        if (w == PS::NBW + 1) {
            // b0: newest tile of row q+1, b1: D of row q-2 (right form)
            T b0[PDH][4], b1[PDH][4];
#pragma unroll
            for (int u = 0; u < PDH - 1; ++u) {
                P.load_newest(u + 1, b0[u]);
                if (!LEFT) P.load_d(u - 2, b1[u]);
            }
            lds_barrier();
            int so = P.row_of(0) % P.RS;   // ring slot of the next row to write out
            for (int q0 = 0; q0 < NTh; q0 += PDH) {
#pragma unroll
                for (int u = 0; u < PDH; ++u) {
                    const int q = q0 + u;
                    const int un = (u + PDH - 1) % PDH;
                    P.load_newest(q + PDH, b0[un]);
                    if (!LEFT) P.load_d(q + PDH - 3, b1[un]);
                    __builtin_amdgcn_sched_barrier(0);
                    if (q < NTp) {
                        T *h = hand + (q & 1) * HS;
#pragma unroll
                        for (int i = 0; i < 4; ++i) h[i * 64 + lane] = b0[u][i];
                        if (q >= 2) {
                            write_rows(so, q - 2, b1[u]);
                            so = P.next_slot(so);
                        }
                        lds_barrier();
                    }
                }
            }
            // rows NTp-2 (in the ring since barrier NTp) and NTp-1 (after the
            // finisher's last row, one barrier later)
            {
                T d2[4];
                if (!LEFT) P.load_d(NTp - 2, d2);
                write_rows(so, NTp - 2, d2);
                so = P.next_slot(so);
            }
            __syncthreads();
            {
                T d1[4];
                if (!LEFT) P.load_d(NTp - 1, d1);
                write_rows(so, NTp - 1, d1);
            }
        } else {
            // state helper: b0 x, b1 f (per group), b2 D of row q
            T b0[PDH][NG][4], b1[PDH][NG][4], b2[PDH][4];
#pragma unroll
            for (int u = 0; u < PDH - 1; ++u) {
#pragma unroll
                for (int k = 0; k < NG; ++k)
                    P.load_state(u, X, ldx, col[k], fsrc[k], fstride[k], b0[u][k], b1[u][k]);
                if (LEFT) P.load_d(u, b2[u]);
            }
            lds_barrier();
            for (int q0 = 0; q0 < NTh; q0 += PDH) {
#pragma unroll
                for (int u = 0; u < PDH; ++u) {
                    const int q = q0 + u;
                    const int un = (u + PDH - 1) % PDH;
#pragma unroll
                    for (int k = 0; k < NG; ++k)
                        P.load_state(q + PDH - 1, X, ldx, col[k], fsrc[k], fstride[k], b0[un][k], b1[un][k]);
                    if (LEFT) P.load_d(q + PDH - 1, b2[un]);
                    __builtin_amdgcn_sched_barrier(0);
                    if (q < NTp) {
                        T *h = hand + (q & 1) * HS + TILE_ELEMS;
#pragma unroll
                        for (int k = 0; k < NG; ++k) {
                            v4 r;
#pragma unroll
                            for (int i = 0; i < 4; ++i) r[i] = b0[u][k][i] + fs[k] * b1[u][k][i];
                            if (LEFT) r = P.dmul(b2[u], r);
#pragma unroll
                            for (int i = 0; i < 4; ++i) h[k * TILE_ELEMS + i * 64 + lane] = r[i];
                        }
                        lds_barrier();
                    }
                }
            }
            __syncthreads();
        }
    }
    // end of pass: the next pass reads X rows written by this one
    __syncthreads();
}

// Zero the LDS rings before a pass: they must hold finite values only (zero
// tiles multiply stale slots), and rows before the item's range must read as
// zero (they are not coupled in).
template <typename T>
__device__ __forceinline__ void clear_ring(T *ring, int tiles) {
    for (int e = threadIdx.x; e < tiles * TILE_ELEMS; e += blockDim.x) ring[e] = (T)0;
    __syncthreads();
}

// LDS tiles of a sweep workgroup: NG rings of nb+1 solved tiles (+1 dummy
// slot), double-buffered partial sums of the bulk waves, double-buffered
// hand-offs (E and one r per group)
__host__ __device__ constexpr int sweep_lds_tiles(int nb, int kw, int ng) {
    return ng * (nb + 2) + 2 * (kw > 1 ? kw - 3 : 1) * ng + 2 * (1 + ng);
}

// ADJ: adjoint sweep, on the mirrored set or (STRIDED) the transposed
// forward tiles.  Steps step0 .. step0+nsteps-1 (the step picks the source's
// time factor); each item runs the passes its mask selects.
template <typename T, int KW, typename SP, int PD, bool ADJ, bool STRIDED, int NG>
__device__ __forceinline__ void sweep_items(const SweepItem *__restrict__ items, int nitems, int nsteps,
                                            int step0) {
    extern __shared__ __align__(16) unsigned char smem[];
    for (int idx = blockIdx.x; idx < nitems; idx += gridDim.x) {
        const SweepItem it = items[idx];
        const int nrt = NG * (it.fac.nb + 2);
        T *ring = (T *)smem;
        T *red = ring + nrt * TILE_ELEMS;                                // [2][KW-3][NG][256]
        T *hand = red + 2 * (KW > 1 ? KW - 3 : 1) * NG * TILE_ELEMS;     // [2][1+NG][256]: E, r
        const void *const *a = it.fac.a;
        for (int s = 0; s < nsteps; ++s) {
            const int step = step0 + s;
            if (it.passes & 1) {
                clear_ring(ring, nrt);
                if (!ADJ)
                    sweep_pass<T, KW, SP, PD, true, false, NG>(it, (const T *)a[TS_LB], (const T *)a[TS_DL], ring,
                                                               red, hand, it.f != nullptr, step, nsteps);
                else if (!STRIDED)
                    sweep_pass<T, KW, SP, PD, true, false, NG>(it, (const T *)a[TS_UTB], (const T *)a[TS_DUT], ring,
                                                               red, hand, false, step, nsteps);
                else
                    sweep_pass<T, KW, SP, PD, true, true, NG>(it, (const T *)a[TS_UB], (const T *)a[TS_DUT], ring,
                                                              red, hand, false, step, nsteps);
            }
            if (it.passes & 2) {
                clear_ring(ring, nrt);
                if (!ADJ)
                    sweep_pass<T, KW, SP, PD, false, false, NG>(it, (const T *)a[TS_UB], (const T *)a[TS_DU], ring,
                                                                red, hand, false, step, nsteps);
                else if (!STRIDED)
                    sweep_pass<T, KW, SP, PD, false, false, NG>(it, (const T *)a[TS_LTB], (const T *)a[TS_DLT], ring,
                                                                red, hand, false, step, nsteps);
                else
                    sweep_pass<T, KW, SP, PD, false, true, NG>(it, (const T *)a[TS_LB], (const T *)a[TS_DLT], ring,
                                                               red, hand, false, step, nsteps);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Pass pairs.  With both M = L U and M = U' L' stored, consecutive steps
// alternate between the two factorisations, so that the second substitution
// of one step and the first of the next run in the same direction:
//   forward: U (step s) with U' (step s+1), then L' (s+1) with L (s+2);
//   adjoint: L^T with L'^T, then U'^T with U^T.
// Pass B (the first substitution of the later step) solves tile row q-2 in
// the period where pass A solves row q.  Its right-hand side D_B (v_A + dt phi
// f) is formed from pass A's solution while that is still in LDS, so the
// state between the two passes never goes to HBM, and every barrier period
// carries the matrix-core work of two tile rows.
//
// Waves (KW = 8), one LDS barrier per period; iteration q ends with barrier
// q+1 (bulk, helpers) or starts with it (finisher):
//   wave 0      finisher: rows q of A and q-2 of B, the two chains interleaved;
//   waves 1..5  bulk: partial sums of rows q (A) and q-2 (B) over the older
//               band tiles, each a fixed share of the 2 (nb-1) tiles;
//   wave 6      factor helper: hands over the newest tiles of rows q+1 (A)
//               and q-1 (B); writes B's solution of row q-4 to HBM;
//   wave 7      state helper: hands over r_A = D_A x of row q (x from HBM)
//               and r_B = D_B (v_A + dt phi f) of row q-2 (v_A from A's ring).
// ---------------------------------------------------------------------------

// Shares of the 2 (NB-1) combined bulk tiles (A's tiles first, then B's) of
// the five bulk waves; waves w and w+4 share a SIMD, the finisher sits with
// wave 4 and the state helper (two tile products per period) with wave 3.
template <int C1, int C2, int C3, int C4, int C5>
struct Split2 {
    __host__ __device__ static constexpr int cn(int wb) {
        return wb == 0 ? C1 : wb == 1 ? C2 : wb == 2 ? C3 : wb == 3 ? C4 : C5;
    }
    __host__ __device__ static constexpr int st(int wb) {
        return (wb > 0 ? C1 : 0) + (wb > 1 ? C2 : 0) + (wb > 2 ? C3 : 0) + (wb > 3 ? C4 : 0);
    }
    __host__ __device__ static constexpr int total() { return C1 + C2 + C3 + C4 + C5; }
    __host__ __device__ static constexpr bool hasA(int wb) { return cn(wb) > 0 && st(wb) < total() / 2; }
    __host__ __device__ static constexpr bool hasB(int wb) { return cn(wb) > 0 && st(wb) + cn(wb) > total() / 2; }
    // bit wb: bulk wave wb has tiles of pass A (maskA) / pass B (maskB)
    static constexpr unsigned maskA =
        (hasA(0) ? 1u : 0u) | (hasA(1) ? 2u : 0u) | (hasA(2) ? 4u : 0u) | (hasA(3) ? 8u : 0u) | (hasA(4) ? 16u : 0u);
    static constexpr unsigned maskB =
        (hasB(0) ? 1u : 0u) | (hasB(1) ? 2u : 0u) | (hasB(2) ? 4u : 0u) | (hasB(3) ? 8u : 0u) | (hasB(4) ? 16u : 0u);
};

constexpr int PAIR_PDH = 3;   // helpers' prefetch depth in pass pairs
// tiles whose ring operands a bulk wave reads ahead of its products
#ifndef LRPR_PAIR_RA32
#define LRPR_PAIR_RA32 16
#endif
// prefetch depth (tile rows) of the bulk waves in pass pairs
#ifndef LRPR_PAIR_PD32
#define LRPR_PAIR_PD32 6
#endif
#ifndef LRPR_PAIR_PD64
#define LRPR_PAIR_PD64 2
#endif
#ifndef LRPR_PAIR_RA64
#define LRPR_PAIR_RA64 16
#endif
constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

// Buffer loads of lane-major tiles: an SGPR resource over a whole tile
// array, one VGPR lane offset shared by every load, the tile's byte offset
// in an SGPR (no per-lane 64-bit addresses to keep live across the prefetch).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
// (The 128-bit result is reinterpreted as a whole vector: casting its
// elements one by one lets the compiler shrink the load to one dword.)
template <typename T> struct BufTile;
template <> struct BufTile<float> {
    __device__ static inline void ld4(rsrc_t r, uint32_t voff, uint32_t soff, float (&v)[4]) {
        const f4v x = __builtin_bit_cast(f4v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
        v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
    }
};
template <> struct BufTile<double> {
    __device__ static inline void ld4(rsrc_t r, uint32_t voff, uint32_t soff, double (&v)[4]) {
        const d2v x = __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
        const d2v y =
            __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff + 1024, 0));
        v[0] = x[0]; v[1] = x[1]; v[2] = y[0]; v[3] = y[1];
    }
};

// One pass of a pair (left form, full range, every factor of the launch
// with NB band tiles per row).  Tile rows outside [0, NT) are clamped to
// rows -1 and NT, guard rows of zero tiles.
template <typename T, int NB, bool ASC>
struct PairPass {
    typedef typename Mf<T>::v4 v4;
    static constexpr int RS = NB + 1;          // ring slots (+1 dummy slot at RS)
    static constexpr int G = NB + 8;           // guard tile rows before and after the arrays
    static constexpr uint32_t TB = TILE_ELEMS * sizeof(T);   // bytes per tile
    rsrc_t rband, rdiag;                       // from guard row -G on
    T *ring;
    int NT, n, lane, g;
    uint32_t voff;                             // this lane's byte offset in a tile
    __device__ PairPass(const SweepItem &it, const T *band, const T *dtile, T *ring_) : ring(ring_) {
        NT = it.fac.NT;
        n = it.fac.n;
        lane = threadIdx.x & 63;
        g = lane >> 4;
        voff = 16u * (uint32_t)lane;
        const uint32_t rows = (uint32_t)(NT + 2 * G);
        rband = make_rsrc(band - (int64_t)G * NB * TILE_ELEMS, rows * NB * TB);
        rdiag = make_rsrc(dtile - (int64_t)G * TILE_ELEMS, rows * TB);
    }
    __device__ __forceinline__ int row_of(int q) const { return ASC ? q : NT - 1 - q; }
    __device__ __forceinline__ int row_clamped(int q) const {
        q = q < -1 ? -1 : (q > NT ? NT : q);
        return row_of(q);
    }
    // byte offset of the band tiles of row q (bulk tile idx: j = idx ascending, idx + 1 descending)
    __device__ __forceinline__ uint32_t row_off(int q) const { return (uint32_t)(row_clamped(q) + G) * NB * TB; }
    static constexpr uint32_t bulk_off(int idx) { return (uint32_t)(ASC ? idx : idx + 1) * TB; }
    // tile at byte offset `toff` within row offset `roff` (the row offset in
    // the scalar operand, the tile's position in the lane's vector offset)
    __device__ __forceinline__ void ld_band(uint32_t roff, uint32_t toff, T (&v)[4]) const {
        BufTile<T>::ld4(rband, voff + toff, roff, v);
    }
    // ring slot of bulk tile idx, sI being the slot of the row being solved
    __device__ __forceinline__ int slot(int sI, int idx) const {
        const int s = sI + (ASC ? 1 : 2) + idx;
        return s >= RS ? s - RS : s;
    }
    __device__ __forceinline__ int first_slot() const { return row_of(0) % RS; }
    __device__ __forceinline__ int next_slot(int sI) const {
        return ASC ? (sI + 1 == RS ? 0 : sI + 1) : (sI == 0 ? RS - 1 : sI - 1);
    }
    __device__ __forceinline__ void load_newest(int q, T (&v)[4]) const {
        ld_band(row_off(q), (uint32_t)(ASC ? NB - 1 : 0) * TB, v);
    }
    __device__ __forceinline__ void load_d(int q, T (&v)[4]) const {
        BufTile<T>::ld4(rdiag, voff, (uint32_t)(row_clamped(q) + G) * TB, v);
    }
    // rows of one column of a state array (accumulator order), clamped into [0, n)
    __device__ __forceinline__ void load_rows(int q, const T *base, int64_t stride, T (&v)[4]) const {
        const int I = row_of(q);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int row = I * TILE + Mf<T>::row(g, i);
            row = row < 0 ? 0 : (row >= n ? n - 1 : row);
            v[i] = gld(base + (int64_t)row * stride);
        }
    }
    __device__ __forceinline__ v4 dmul(const T (&d)[4], const v4 &t) const {
        v4 y = {0, 0, 0, 0};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) y = Mf<T>::mma(d[kc], t[kc], y);
        return y;
    }
};

template <typename T, int NB, typename SP, int PD, bool ASC, int WB>
__device__ __forceinline__ void pair_bulk(const PairPass<T, NB, ASC> &PA, const PairPass<T, NB, ASC> &PB, T *red,
                                          int NQ) {
    typedef typename Mf<T>::v4 v4;
    constexpr int ST = SP::st(WB), CN = SP::cn(WB), NBM = NB - 1, NBW = 5;
    constexpr int RA = sizeof(T) == 8 ? LRPR_PAIR_RA64 : LRPR_PAIR_RA32;   // ring read-ahead (tiles)
    static_assert(SP::total() == 2 * NBM, "the shares must cover both passes' bulk tiles");
    const int lane = PA.lane;
    T ab[PD][CN][4];
    typedef PairPass<T, NB, ASC> PS;
    // tiles of A's row q and B's row q-2
    auto load = [&](int q, T (&buf)[CN][4]) {
        const uint32_t oa = PA.row_off(q), ob = PB.row_off(q - 2);
#pragma unroll
        for (int t = 0; t < CN; ++t) {
            const bool isB = ST + t >= NBM;
            const int idx = isB ? ST + t - NBM : ST + t;
            if (isB) PB.ld_band(ob, PS::bulk_off(idx), buf[t]);
            else PA.ld_band(oa, PS::bulk_off(idx), buf[t]);
        }
    };
#pragma unroll
    for (int u = 0; u < PD - 1; ++u) load(u, ab[u]);
    lds_barrier();
    int sA = PA.first_slot(), sB = sA;
    for (int q0 = 0; q0 < NQ; q0 += PD) {
#pragma unroll
        for (int u = 0; u < PD; ++u) {
            const int q = q0 + u;
            load(q + PD - 1, ab[(u + PD - 1) % PD]);
            __builtin_amdgcn_sched_barrier(0);
            // ring operands (B operands, accumulator order) of the wave's tiles
            T bv[CN][4];
            auto ring_read = [&](int t) {
                const bool isB = ST + t >= NBM;
                const int idx = isB ? ST + t - NBM : ST + t;
                const T *rj = isB ? PB.ring + PB.slot(sB, idx) * TILE_ELEMS : PA.ring + PA.slot(sA, idx) * TILE_ELEMS;
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) bv[t][kc] = rj[64 * kc + lane];
            };
            v4 a2[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, b2[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
            auto tile_mma = [&](int t, int kc) {
                if (ST + t >= NBM) b2[t & 1] = Mf<T>::mma(ab[u][t][kc], bv[t][kc], b2[t & 1]);
                else a2[t & 1] = Mf<T>::mma(ab[u][t][kc], bv[t][kc], a2[t & 1]);
            };
#pragma unroll
            for (int t = 0; t < CN; ++t) ring_read(t);
            if constexpr (RA >= CN) {
                // every ring read issued before the first product
                __builtin_amdgcn_sched_barrier(0);
            } else {
                // ring reads RA tiles ahead of the products (two LDS reads
                // and four products per tile)
                __builtin_amdgcn_sched_group_barrier(0x100, 2 * RA, 0);
#pragma unroll
                for (int t = 0; t + RA < CN; ++t) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
                    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x008, 4 * RA, 0);
            }
            // tiles t and t+1 accumulate into different registers: their
            // products alternate, so no product waits on the one before it
#pragma unroll
            for (int t = 0; t < CN; t += 2) {
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) {
                    tile_mma(t, kc);
                    if (t + 1 < CN) tile_mma(t + 1, kc);
                }
            }
            T *rd = red + (q & 1) * 2 * NBW * TILE_ELEMS;
            if constexpr ((SP::maskA >> WB) & 1u) {
                const v4 acc = a2[0] + a2[1];
#pragma unroll
                for (int i = 0; i < 4; ++i) rd[WB * TILE_ELEMS + i * 64 + lane] = acc[i];
            }
            if constexpr ((SP::maskB >> WB) & 1u) {
                const v4 acc = b2[0] + b2[1];
#pragma unroll
                for (int i = 0; i < 4; ++i) rd[(NBW + WB) * TILE_ELEMS + i * 64 + lane] = acc[i];
            }
            sA = PA.next_slot(sA);
            if (q >= 2) sB = PB.next_slot(sB);
            lds_barrier();
        }
    }
}

template <typename T, int NB, typename SP, int PD, bool ASC>
__device__ __forceinline__ void sweep_pair(const SweepItem &it, const T *__restrict__ bandA,
                                           const T *__restrict__ dA, const T *__restrict__ bandB,
                                           const T *__restrict__ dB, T *ringA, T *ringB, T *red, T *hand,
                                           bool with_src, int stepB) {
    typedef typename Mf<T>::v4 v4;
    typedef PairPass<T, NB, ASC> PS;
    constexpr int NBW = 5, PDH = PAIR_PDH, RS = PS::RS;
    constexpr int PQ = PD / gcd_c(PD, PDH) * PDH;   // both unroll depths divide the period count
    PS PA(it, bandA, dA, ringA), PB(it, bandB, dB, ringB);
    const int NT = PA.NT, lane = PA.lane, g = PA.g, n = PA.n;
    const int c = lane & 15;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // A's rows 0..NT-1; B's rows trail by 2, and its output by 2 more
    const int NQ = (NT + 4 + PQ - 1) / PQ * PQ;
    T *X = (T *)it.X;
    const int64_t ldx = it.ldx;
    const bool colok = c < it.ncols;
    const int col = colok ? c : 0;
    // pass B's source: f(x) * dt * phi(t_stepB), or the zero tile
    const T *fsrc = (const T *)it.fac.zt;
    int64_t fstride = 0;
    T fs = 0;
    if (with_src && colok) {
        const int fc = it.fcol ? gld(it.fcol + c) : 0;
        if (fc >= 0) {
            fsrc = (const T *)it.f + (int64_t)fc * it.ldf;
            fstride = 1;
            const double sc = it.fscale ? gld(it.fscale + (int64_t)c * it.fsteps + stepB) : 1.0;
            fs = (T)(it.fac.dt * sc);
        }
    }
    if (w == 0) {
        v4 tA = {0, 0, 0, 0}, tB = {0, 0, 0, 0};
        int sA = PA.first_slot(), sB = sA;
        lds_barrier();
        for (int q = 0; q < NQ; ++q) {
            lds_barrier();
            const T *h = hand + (q & 1) * 4 * TILE_ELEMS;   // E_A, r_A, E_B, r_B
            const T *rd = red + (q & 1) * 2 * NBW * TILE_ELEMS;
            T eA[4], eB[4];
            v4 vA, vB;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                T a = tA[i], b = tB[i];
#pragma unroll
                for (int wb = 0; wb < NBW; ++wb) {
                    if ((SP::maskA >> wb) & 1u) a += rd[wb * TILE_ELEMS + i * 64 + lane];
                    if ((SP::maskB >> wb) & 1u) b += rd[(NBW + wb) * TILE_ELEMS + i * 64 + lane];
                }
                vA[i] = h[TILE_ELEMS + i * 64 + lane] - a;
                vB[i] = h[3 * TILE_ELEMS + i * 64 + lane] - b;
                eA[i] = h[i * 64 + lane];
                eB[i] = h[2 * TILE_ELEMS + i * 64 + lane];
            }
            T *ra = ringA + (q < NT ? sA : RS) * TILE_ELEMS;
            T *rb = ringB + ((q >= 2 && q - 2 < NT) ? sB : RS) * TILE_ELEMS;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ra[i * 64 + lane] = vA[i];
                rb[i * 64 + lane] = vB[i];
            }
            // t = E v for both chains, interleaved on the matrix core
            v4 ya = {0, 0, 0, 0}, yb = {0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                ya = Mf<T>::mma(eA[kc], vA[kc], ya);
                yb = Mf<T>::mma(eB[kc], vB[kc], yb);
            }
            tA = ya;
            tB = yb;
            sA = PA.next_slot(sA);
            if (q >= 2) sB = PB.next_slot(sB);
        }
        __syncthreads();
    } else if (w <= NBW) {
        switch (w) {
            case 1: pair_bulk<T, NB, SP, PD, ASC, 0>(PA, PB, red, NQ); break;
            case 2: pair_bulk<T, NB, SP, PD, ASC, 1>(PA, PB, red, NQ); break;
            case 3: pair_bulk<T, NB, SP, PD, ASC, 2>(PA, PB, red, NQ); break;
            case 4: pair_bulk<T, NB, SP, PD, ASC, 3>(PA, PB, red, NQ); break;
            default: pair_bulk<T, NB, SP, PD, ASC, 4>(PA, PB, red, NQ); break;
        }
        __syncthreads();
    } else if (w == NBW + 1) {
        // factor helper
        T bA[PDH][4], bB[PDH][4];
#pragma unroll
        for (int u = 0; u < PDH - 1; ++u) {
            PA.load_newest(u + 1, bA[u]);
            PB.load_newest(u - 1, bB[u]);
        }
        lds_barrier();
        T *sink = (T *)it.fac.sink;
        int so = PB.first_slot();
        for (int q0 = 0; q0 < NQ; q0 += PDH) {
#pragma unroll
            for (int u = 0; u < PDH; ++u) {
                const int q = q0 + u;
                const int un = (u + PDH - 1) % PDH;
                PA.load_newest(q + PDH, bA[un]);
                PB.load_newest(q + PDH - 2, bB[un]);
                __builtin_amdgcn_sched_barrier(0);
                T *h = hand + (q & 1) * 4 * TILE_ELEMS;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    h[i * 64 + lane] = bA[u][i];
                    h[2 * TILE_ELEMS + i * 64 + lane] = bB[u][i];
                }
                if (q >= 4) {
                    // B's row q-4: in its ring since this period's barrier
                    const int qo = q - 4;
                    const T *ro = ringB + so * TILE_ELEMS;
                    const int Irow = PB.row_of(qo);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = Irow * TILE + Mf<T>::row(g, i);
                        const T v = ro[i * 64 + lane];
                        gst((qo < NT && colok && row < n) ? X + row + (int64_t)c * ldx : sink + lane, v);
                    }
                    so = PB.next_slot(so);
                }
                lds_barrier();
            }
        }
        __syncthreads();
    } else {
        // state helper
        const T *xcol = X + (int64_t)col * ldx;
        T xb[PDH][4], da[PDH][4], fb[PDH][4], db[PDH][4];
#pragma unroll
        for (int u = 0; u < PDH - 1; ++u) {
            PA.load_rows(u, xcol, 1, xb[u]);
            PA.load_d(u, da[u]);
            PB.load_rows(u - 2, fsrc, fstride, fb[u]);
            PB.load_d(u - 2, db[u]);
        }
        lds_barrier();
        int so = PA.first_slot();
        for (int q0 = 0; q0 < NQ; q0 += PDH) {
#pragma unroll
            for (int u = 0; u < PDH; ++u) {
                const int q = q0 + u;
                const int un = (u + PDH - 1) % PDH;
                PA.load_rows(q + PDH - 1, xcol, 1, xb[un]);
                PA.load_d(q + PDH - 1, da[un]);
                PB.load_rows(q + PDH - 3, fsrc, fstride, fb[un]);
                PB.load_d(q + PDH - 3, db[un]);
                __builtin_amdgcn_sched_barrier(0);
                v4 x;
#pragma unroll
                for (int i = 0; i < 4; ++i) x[i] = xb[u][i];
                // r_A = D_A x and r_B = D_B (v_A + dt phi f), products interleaved
                // (B's row q-2 is negative, so D_B is the zero tile, before q = 2)
                const T *ro = ringA + so * TILE_ELEMS;   // A's row q-2, in its ring since this barrier
                v4 y;
#pragma unroll
                for (int i = 0; i < 4; ++i) y[i] = ro[i * 64 + lane] + fs * fb[u][i];
                v4 rA = {0, 0, 0, 0}, rB = {0, 0, 0, 0};
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) {
                    rA = Mf<T>::mma(da[u][kc], x[kc], rA);
                    rB = Mf<T>::mma(db[u][kc], y[kc], rB);
                }
                if (q >= 2) so = PA.next_slot(so);
                T *h = hand + (q & 1) * 4 * TILE_ELEMS;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    h[TILE_ELEMS + i * 64 + lane] = rA[i];
                    h[3 * TILE_ELEMS + i * 64 + lane] = rB[i];
                }
                lds_barrier();
            }
        }
        __syncthreads();
    }
    // end of the pair: the next pass reads X rows written by this one
    __syncthreads();
}

// One pass pair over every item (each item's factor carries the UL set and
// has NB band tiles per row).  Descending pairs join the second substitution
// of an L U step with the first of the following U' L' step; ascending pairs
// the second substitution of a U' L' step with the first of the following
// L U step.  stepB: the step of pass B (its source's time factor).
// minimum waves per SIMD of the FP32 pair kernels (4 fits two workgroups per
// compute unit at prefetch depth 2; measured slower than one at depth 5 or 6)
#ifndef LRPR_PAIR_WG32
#define LRPR_PAIR_WG32 1
#endif
template <typename T, int NB, typename SP, int PD, bool ASC, bool ADJ>
__global__ __launch_bounds__(512, sizeof(T) == 4 ? LRPR_PAIR_WG32 : 1) void k_sweep_pair(const SweepItem *__restrict__ items, int nitems, int stepB) {
    extern __shared__ __align__(16) unsigned char smem[];
    for (int idx = blockIdx.x; idx < nitems; idx += gridDim.x) {
        const SweepItem &it = items[idx];
        T *ringA = (T *)smem;
        T *ringB = ringA + (NB + 2) * TILE_ELEMS;
        T *red = ringB + (NB + 2) * TILE_ELEMS;      // [2][2][5]
        T *hand = red + 20 * TILE_ELEMS;             // [2][4]
        const T *const *a = (const T *const *)it.fac.a;
        const T *const *ar = (const T *const *)it.fac.ar;
        // forward: U with U' (descending), L' with L (ascending);
        // adjoint: L^T with L'^T (descending), U'^T with U^T (ascending)
        const T *bA, *dA, *bB, *dB;
        if (!ADJ) {
            bA = ASC ? ar[TS_LB] : a[TS_UB];
            dA = ASC ? ar[TS_DL] : a[TS_DU];
            bB = ASC ? a[TS_LB] : ar[TS_UB];
            dB = ASC ? a[TS_DL] : ar[TS_DU];
        } else {
            bA = ASC ? ar[TS_UTB] : a[TS_LTB];
            dA = ASC ? ar[TS_DUT] : a[TS_DLT];
            bB = ASC ? a[TS_UTB] : ar[TS_LTB];
            dB = ASC ? a[TS_DUT] : ar[TS_DLT];
        }
        clear_ring(ringA, 2 * NB + 4);   // both rings
        sweep_pair<T, NB, SP, PD, ASC>(it, bA, dA, bB, dB, ringA, ringB, red, hand, !ADJ && it.f != nullptr, stepB);
    }
}

template <typename T, int KW, typename SP, int PD, bool ADJ, bool STRIDED, int NG>
__global__ __launch_bounds__(64 * KW) void k_sweep(const SweepItem *__restrict__ items, int nitems, int nsteps,
                                                   int step0) {
    sweep_items<T, KW, SP, PD, ADJ, STRIDED, NG>(items, nitems, nsteps, step0);
}

// The local block solves of partitioned passes (forward items on row ranges):
// the same code under its own name, so that profiles keep them apart from the
// full-length sweeps.
template <typename T, int KW, typename SP, int PD>
__global__ __launch_bounds__(64 * KW) void k_sweep_local(const SweepItem *__restrict__ items, int nitems,
                                                         int nsteps, int step0) {
    sweep_items<T, KW, SP, PD, false, false, 1>(items, nitems, nsteps, step0);
}

template <typename T, int KW, typename SP, int PD, int NG = 1>
static hipError_t launch_t(bool adjoint, bool strided, int nitems, const SweepItem *d_items, int nsteps,
                           int max_nb, hipStream_t s, int step0, bool local) {
    const size_t lds = (size_t)sweep_lds_tiles(max_nb, KW, NG) * TILE_ELEMS * sizeof(T);
    const int grid = nitems < 65536 ? nitems : 65536;
    if (local && NG == 1)
        hipLaunchKernelGGL((k_sweep_local<T, KW, SP, PD>), dim3(grid), dim3(64 * KW), lds, s, d_items, nitems,
                           nsteps, step0);
    else if (local)
        return hipErrorInvalidValue;
    else if (!adjoint)
        hipLaunchKernelGGL((k_sweep<T, KW, SP, PD, false, false, NG>), dim3(grid), dim3(64 * KW), lds, s, d_items,
                           nitems, nsteps, step0);
    else if (!strided)
        hipLaunchKernelGGL((k_sweep<T, KW, SP, PD, true, false, NG>), dim3(grid), dim3(64 * KW), lds, s, d_items,
                           nitems, nsteps, step0);
    else
        hipLaunchKernelGGL((k_sweep<T, KW, SP, PD, true, true, NG>), dim3(grid), dim3(64 * KW), lds, s, d_items,
                           nitems, nsteps, step0);
    return hipGetLastError();
}

// Tile split and prefetch depth of the nb <= 16 class (compile-time tuning).
#ifndef LRPR_SPLIT16_F64
#define LRPR_SPLIT16_F64 2, 4, 4, 3, 2
#endif
#ifndef LRPR_PD16_F64
#define LRPR_PD16_F64 3
#endif
#ifndef LRPR_SPLIT16_F32
#define LRPR_SPLIT16_F32 2, 4, 4, 3, 2
#endif
#ifndef LRPR_PD16_F32
#define LRPR_PD16_F32 5
#endif

// KW > 1: wave 0 finishes tile rows, five bulk waves share the nb-1 older
// band tiles (Split: tiles per bulk wave), two helper waves stage the
// finisher's operands and write the output.  Narrow bands run on one wave.
template <typename T, int NB, typename SP, int PD>
static hipError_t launch_pair_t(bool adjoint, bool asc, int nitems, const SweepItem *d_items, hipStream_t s,
                                int stepB) {
    // LDS: two rings, double-buffered partial sums of both passes, hand-offs
    const size_t lds = (size_t)(2 * (NB + 2) + 20 + 8) * TILE_ELEMS * sizeof(T);
    const int grid = nitems < 65536 ? nitems : 65536;
    if (!adjoint && !asc)
        hipLaunchKernelGGL((k_sweep_pair<T, NB, SP, PD, false, false>), dim3(grid), dim3(512), lds, s, d_items, nitems,
                           stepB);
    else if (!adjoint)
        hipLaunchKernelGGL((k_sweep_pair<T, NB, SP, PD, true, false>), dim3(grid), dim3(512), lds, s, d_items, nitems,
                           stepB);
    else if (!asc)
        hipLaunchKernelGGL((k_sweep_pair<T, NB, SP, PD, false, true>), dim3(grid), dim3(512), lds, s, d_items, nitems,
                           stepB);
    else
        hipLaunchKernelGGL((k_sweep_pair<T, NB, SP, PD, true, true>), dim3(grid), dim3(512), lds, s, d_items, nitems,
                           stepB);
    return hipGetLastError();
}

hipError_t launch_sweep_pair(bool adjoint, bool asc, bool f32, int nitems, const SweepItem *d_items, int nb,
                             hipStream_t s, int stepB) {
    if (nitems <= 0) return hipSuccess;
    if (nb == 8) {
        if (f32) return launch_pair_t<float, 8, Split2<2, 4, 3, 3, 2>, 5>(adjoint, asc, nitems, d_items, s, stepB);
        return launch_pair_t<double, 8, Split2<2, 4, 3, 3, 2>, 3>(adjoint, asc, nitems, d_items, s, stepB);
    }
    if (nb == 16) {
        // FP32 shares as in FP64: with (5, 8, 7, 6, 4), equally fast, every
        // ascending FP32 pair shrank smooth modes by a further 3e-7 to 6e-7
        // (deterministically; the prefetch depth leaves results bit for bit)
        if (f32)
            return launch_pair_t<float, 16, Split2<4, 7, 7, 7, 5>, LRPR_PAIR_PD32>(adjoint, asc, nitems, d_items, s,
                                                                                   stepB);
        return launch_pair_t<double, 16, Split2<4, 7, 7, 7, 5>, LRPR_PAIR_PD64>(adjoint, asc, nitems, d_items, s,
                                                                                 stepB);
    }
    return hipErrorInvalidValue;
}

bool sweep_pairable(int nb) { return nb == 8 || nb == 16; }

template <typename T>
static hipError_t launch_prec(bool adjoint, bool strided, int nitems, const SweepItem *d_items, int nsteps,
                              int max_nb, hipStream_t s, int step0, bool local) {
    constexpr bool F64 = sizeof(T) == 8;
    if (max_nb <= 1) return launch_t<T, 1, Split<1, 0, 0, 0, 0>, 3>(adjoint, strided, nitems, d_items, nsteps, max_nb, s, step0, local);
    if (max_nb <= 4) return launch_t<T, 1, Split<3, 0, 0, 0, 0>, 3>(adjoint, strided, nitems, d_items, nsteps, max_nb, s, step0, local);
    if (max_nb <= 8)
        return launch_t<T, 8, Split<1, 2, 2, 1, 1>, F64 ? 4 : 6>(adjoint, strided, nitems, d_items, nsteps, max_nb, s, step0, local);
    if (max_nb <= 16) {
        if constexpr (F64)
            return launch_t<T, 8, Split<LRPR_SPLIT16_F64>, LRPR_PD16_F64>(adjoint, strided, nitems, d_items, nsteps,
                                                                          max_nb, s, step0, local);
        else
            return launch_t<T, 8, Split<LRPR_SPLIT16_F32>, LRPR_PD16_F32>(adjoint, strided, nitems, d_items, nsteps,
                                                                          max_nb, s, step0, local);
    }
    if (max_nb <= 32) {
        // FP32: the shares of the multi-group sweeps (the same arithmetic
        // for every group count)
        if constexpr (F64)
            return launch_t<T, 8, Split<6, 7, 6, 6, 6>, 2>(adjoint, strided, nitems, d_items, nsteps, max_nb, s,
                                                           step0, local);
        else
            return launch_t<T, 8, Split<4, 8, 8, 7, 4>, 3>(adjoint, strided, nitems, d_items, nsteps, max_nb, s,
                                                           step0, local);
    }
    if (max_nb <= 64)
        return launch_t<T, 8, Split<13, 13, 13, 13, 11>, 2>(adjoint, strided, nitems, d_items, nsteps, max_nb, s, step0, local);
    return hipErrorInvalidValue;
}

// Column groups per item (FP32, 4 < nb <= 32): one band tile feeds the
// matrix-core products of NG groups, with the bulk shares of the one-group
// sweep of the same band class (so the same arithmetic per column).  For
// nb <= 32 those shares favour the SIMDs that run no finisher or helper
// wave besides their bulk waves (waves 1 and 5 share SIMD 1).
int sweep_max_groups(bool f32, int max_nb) { return (f32 && max_nb > 4 && max_nb <= 32) ? 3 : 1; }

static hipError_t launch_groups_f32(bool adjoint, bool strided, int nitems, const SweepItem *d_items, int nsteps,
                                   int max_nb, hipStream_t s, int step0, int ng) {
    if (max_nb <= 8) {
        if (ng == 2)
            return launch_t<float, 8, Split<1, 2, 2, 1, 1>, 4, 2>(adjoint, strided, nitems, d_items, nsteps, max_nb,
                                                                  s, step0, false);
        return launch_t<float, 8, Split<1, 2, 2, 1, 1>, 4, 3>(adjoint, strided, nitems, d_items, nsteps, max_nb, s,
                                                              step0, false);
    }
    if (max_nb <= 16) {
        if (ng == 2)
            return launch_t<float, 8, Split<LRPR_SPLIT16_F32>, 3, 2>(adjoint, strided, nitems, d_items, nsteps, max_nb,
                                                                  s, step0, false);
        return launch_t<float, 8, Split<LRPR_SPLIT16_F32>, 3, 3>(adjoint, strided, nitems, d_items, nsteps, max_nb, s,
                                                              step0, false);
    }
    if (ng == 2)
        return launch_t<float, 8, Split<4, 8, 8, 7, 4>, 3, 2>(adjoint, strided, nitems, d_items, nsteps, max_nb, s,
                                                              step0, false);
    return launch_t<float, 8, Split<4, 8, 8, 7, 4>, 3, 3>(adjoint, strided, nitems, d_items, nsteps, max_nb, s,
                                                          step0, false);
}

hipError_t launch_sweep(bool adjoint, bool strided, bool f32, int nitems, const SweepItem *d_items, int nsteps,
                        int max_nb, hipStream_t s, int step0, bool local, int ng) {
    if (nitems <= 0 || nsteps <= 0) return hipSuccess;
    if (local && adjoint) return hipErrorInvalidValue;
    if (ng < 1 || ng > sweep_max_groups(f32, max_nb) || (local && ng > 1)) return hipErrorInvalidValue;
    if (ng > 1) return launch_groups_f32(adjoint, strided, nitems, d_items, nsteps, max_nb, s, step0, ng);
    if (f32) return launch_prec<float>(adjoint, strided, nitems, d_items, nsteps, max_nb, s, step0, local);
    return launch_prec<double>(adjoint, strided, nitems, d_items, nsteps, max_nb, s, step0, local);
}

}  // namespace lrpr
