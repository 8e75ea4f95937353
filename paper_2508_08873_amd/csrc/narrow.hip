// Fine sweeps of narrow panels (1 to 4 right-hand sides per factor) on the
// vector ALUs.  The matrix-core sweep multiplies 16x16 tiles by 16-column
// groups, so one right-hand side costs it as much as sixteen; with one
// column per factor (the Parareal sweeps of problems whose slices each have
// their own operator) a tile row needs only nb tile-vector products, and
// the pass is bound by streaming the factor tiles from HBM.
//
// Same blocking and tile layout as the matrix-core sweep (lrpr_internal.h):
// per tile row I of a pass, with the band tiles premultiplied by their row's
// diagonal-tile inverse D_I,
//     v_I = D_I r_I - sum_{bulk J} A_IJ v_J - A_{I,I-1} v_{I-1}
// (forward passes, left form; r = x + dt phi f in the L pass, r = x in the U
// pass, which runs the tile rows in descending order).
//
// Waves of a workgroup (8), one LDS barrier per period p:
//   waves 1..7  bulk: partial sums of row p over the nb-1 older band tiles
//               (solved rows p-nb..p-2, in an LDS ring), wave 1 also D_p r_p;
//               operands prefetched PD rows ahead; each wave reduces its four
//               lane groups and writes 16 x NC values;
//   wave 0      finisher: row p-1 = D r - (sum of the bulk partials of row
//               p-1 + A_newest v_{p-2}); ring store, output to HBM.
// Lane l holds row m = l % 16 of a tile and the four contraction indices
// k = Mf::row(l / 16, kc), kc = 0..3 (the A-operand layout of the tiles).
#include "lrpr_internal.h"
#include "tile_ops.h"

namespace lrpr {

namespace {

constexpr int NW = 8;          // waves per workgroup
constexpr int NBULK = NW - 1;  // bulk waves

// reduce over the four lane groups (lanes m, m+16, m+32, m+48) with the
// row-swapping permutes of the vector ALU (no LDS round trip): after the
// 16-lane swap every lane holds x_r + x_(r^1) of its row pair, after the
// 32-lane swap (x_0 + x_1) + (x_2 + x_3), the order of a butterfly over
// lane distances 16 and 32
__device__ __forceinline__ float group_sum(float v) {
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    const float s = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(s), __float_as_uint(s), false, false);
    return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}
__device__ __forceinline__ double group_sum(double v) {
    auto swap_add = [](double x, bool wide) {
        const unsigned lo = (unsigned)(__double_as_longlong(x) & 0xffffffffull);
        const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(x) >> 32);
        const auto a = wide ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                            : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto b = wide ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                            : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        const double x0 = __longlong_as_double((long long)(((unsigned long long)b[0] << 32) | a[0]));
        const double x1 = __longlong_as_double((long long)(((unsigned long long)b[1] << 32) | a[1]));
        return x0 + x1;
    };
    return swap_add(swap_add(v, false), true);
}

template <typename T, int NC, int TMAX, int PD, bool ASC>
__device__ __forceinline__ void narrow_pass(const SweepItem &it, const T *__restrict__ band,
                                            const T *__restrict__ dtile, T *ring, T *red, bool with_src, int step) {
    static_assert(PD % 2 == 0 && PD >= 2, "even prefetch depth");
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, m = lane & 15;
    const int nb = it.fac.nb, n = it.fac.n;
    const int r0 = it.r0, r1 = it.r1, NT = r1 - r0;
    const int RS = nb + 1;
    const T *zt = (const T *)it.fac.zt;
    T *X = (T *)it.X;
    const int64_t ldx = it.ldx;
    auto row_of = [&](int q) { return ASC ? r0 + q : r1 - 1 - q; };
    // ring slot of tile row position q (q may be negative: rows before the
    // range read the zero-initialised slots)
    auto slot = [&](int q) { return ((q % RS) + RS) % RS; };
    T *rslot = ring;   // [RS][16][NC]
    auto ring_at = [&](int s, int row, int c) -> T & { return rslot[(s * 16 + row) * NC + c]; };

    if (w == 0) {
        // ---- finisher
        T vprev[NC][4];   // v_{p-2} at this lane's contraction indices
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) vprev[c][kc] = 0;
        T eb[PD][4];   // newest tiles, prefetched
        auto ld_new = [&](int q, T (&e)[4]) {
            if (q < NT) {
                const int I = row_of(q);
                const T *tp = band + ((int64_t)I * nb + (ASC ? nb - 1 : 0)) * TILE_ELEMS;
                Mf<T>::ld4(tp, lane, e);
            } else {
                Mf<T>::ld4(zt, lane, e);
            }
        };
#pragma unroll
        for (int u = 0; u < PD - 1; ++u) ld_new(u, eb[u]);
        lds_barrier();   // period 0: the bulk waves compute row 0
        for (int q0 = 0; q0 < NT; q0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int q = q0 + u;   // row finished in period q + 1
                ld_new(q + PD - 1, eb[(u + PD - 1) % PD]);
                if (q < NT) {
                    const T *rd = red + (q & 1) * (NBULK + 1) * 16 * NC;
                    T v[NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        T t = 0;
#pragma unroll
                        for (int kc = 0; kc < 4; ++kc) t += eb[u][kc] * vprev[c][kc];
                        t = group_sum(t);
                        T a = 0;
#pragma unroll
                        for (int b = 0; b < NBULK; ++b) a += rd[(m * (NBULK + 1) + b) * NC + c];
                        v[c] = rd[(m * (NBULK + 1) + NBULK) * NC + c] - (a + t);   // D r - (partials + newest)
                    }
                    const int sq = slot(q);
                    if (lane < 16) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) ring_at(sq, m, c) = v[c];
                        const int row = row_of(q) * TILE + m;
                        if (row < n)
#pragma unroll
                            for (int c = 0; c < NC; ++c)
                                if (c < it.ncols) gst(X + row + (int64_t)c * ldx, v[c]);
                    }
                    // this wave's ring writes before its own reads below (LDS
                    // only: the prefetched tile loads stay in flight)
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
#pragma unroll
                    for (int c = 0; c < NC; ++c)
#pragma unroll
                        for (int kc = 0; kc < 4; ++kc) vprev[c][kc] = ring_at(sq, Mf<T>::row(g, kc), c);
                    lds_barrier();
                }
            }
        }
    } else {
        // ---- bulk waves: tiles [st, st+cn) of the nb-1 older ones; wave 1
        //      also forms D r
        const int wb = w - 1;
        const int nbulk = nb - 1;
        const int per = (nbulk + NBULK - 1) / NBULK;
        const int st = wb * per;
        const int cn = st >= nbulk ? 0 : (nbulk - st < per ? nbulk - st : per);   // <= TMAX
        const bool dr = wb == 0;
        // source column of every right-hand side
        // (no source: the zero tile with stride 0, so that every load is
        // unconditional and none has to complete before the next is issued)
        const T *fsrc[NC];
        int fstr[NC];
        T fs[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            fsrc[c] = zt;
            fstr[c] = 0;
            fs[c] = 0;
            if (with_src && c < it.ncols) {
                const int fc = it.fcol ? gld(it.fcol + c) : 0;
                if (fc >= 0) {
                    fsrc[c] = (const T *)it.f + (int64_t)fc * it.ldf;
                    fstr[c] = 1;
                    const double sc = it.fscale ? gld(it.fscale + (int64_t)c * it.fsteps + step) : 1.0;
                    fs[c] = (T)(it.fac.dt * sc);
                }
            }
        }
        // tiles PD-1 rows ahead; the state (x, f) and D of wave 1 SD-1 rows
        // ahead (SD divides PD: state slot q % SD)
        constexpr int SD = PD / 2 < 2 ? 2 : PD / 2;
        static_assert(PD % SD == 0, "state slots must repeat within the unrolled period");
        T ab[PD][TMAX][4];
        T db[SD][4], xb[SD][NC][4], fb[SD][NC][4];
        auto ld_tiles = [&](int q, T (&abu)[TMAX][4]) {
            const int I = row_of(q < NT ? q : NT - 1);
#pragma unroll
            for (int t = 0; t < TMAX; ++t) {
                const T *tp = zt;
                if (q < NT && t < cn) {
                    const int j = ASC ? st + t : st + t + 1;
                    tp = band + ((int64_t)I * nb + j) * TILE_ELEMS;
                }
                Mf<T>::ld4(tp, lane, abu[t]);
            }
        };
        auto ld_state = [&](int q, T (&d)[4], T (&xv)[NC][4], T (&fv)[NC][4]) {
            if (!dr) return;
            const int I = row_of(q < NT ? q : NT - 1);
            Mf<T>::ld4(dtile + (int64_t)I * TILE_ELEMS, lane, d);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int col = c < it.ncols ? c : 0;
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) {
                    int row = I * TILE + Mf<T>::row(g, kc);
                    row = row >= n ? n - 1 : row;
                    xv[c][kc] = gld(X + row + (int64_t)col * ldx);
                    fv[c][kc] = gld(fsrc[c] + row * fstr[c]);
                }
            }
        };
#pragma unroll
        for (int u = 0; u < PD - 1; ++u) ld_tiles(u, ab[u]);
#pragma unroll
        for (int u = 0; u < SD - 1; ++u) ld_state(u, db[u], xb[u], fb[u]);
        for (int q0 = 0; q0 < NT; q0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int q = q0 + u;   // row computed in period q
                ld_tiles(q + PD - 1, ab[(u + PD - 1) % PD]);
                ld_state(q + SD - 1, db[(u + SD - 1) % SD], xb[(u + SD - 1) % SD], fb[(u + SD - 1) % SD]);
                if (q < NT) {
                    T p[NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c) p[c] = 0;
#pragma unroll
                    for (int t = 0; t < TMAX; ++t) {
                        if (t < cn) {
                            // older tile j of row q multiplies v of row position q - nb + j
                            // (ascending) or q - 1 - j (descending): solved in period <= q - 1
                            const int j = ASC ? st + t : st + t + 1;
                            const int sJ = slot(ASC ? q - nb + j : q - 1 - j);
#pragma unroll
                            for (int c = 0; c < NC; ++c)
#pragma unroll
                                for (int kc = 0; kc < 4; ++kc)
                                    p[c] += ab[u][t][kc] * ring_at(sJ, Mf<T>::row(g, kc), c);
                        }
                    }
                    T *rd = red + (q & 1) * (NBULK + 1) * 16 * NC;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const T s = group_sum(p[c]);
                        if (lane < 16) rd[(m * (NBULK + 1) + wb) * NC + c] = s;
                    }
                    if (dr) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            T d = 0;
#pragma unroll
                            for (int kc = 0; kc < 4; ++kc)
                                d += db[u % SD][kc] * (xb[u % SD][c][kc] + fs[c] * fb[u % SD][c][kc]);
                            d = group_sum(d);
                            if (lane < 16) rd[(m * (NBULK + 1) + NBULK) * NC + c] = d;
                        }
                    }
                    lds_barrier();
                }
            }
        }
        lds_barrier();   // period NT: the finisher completes the last row
    }
    __syncthreads();   // the next pass reads X rows written by this one
}

template <typename T, int NC, int TMAX, int PD>
__global__ __launch_bounds__(64 * NW) void k_sweep_narrow(const SweepItem *__restrict__ items, int nitems,
                                                          int nsteps, int step0) {
    extern __shared__ __align__(16) unsigned char smem[];
    for (int idx = blockIdx.x; idx < nitems; idx += gridDim.x) {
        const SweepItem it = items[idx];
        T *ring = (T *)smem;
        T *red = ring + (it.fac.nb + 1) * 16 * NC;
        const void *const *a = it.fac.a;
        for (int s = 0; s < nsteps; ++s) {
            const int step = step0 + s;
            for (int e = threadIdx.x; e < (it.fac.nb + 1) * 16 * NC; e += blockDim.x) ring[e] = (T)0;
            __syncthreads();
            if (it.passes & 1)
                narrow_pass<T, NC, TMAX, PD, true>(it, (const T *)a[TS_LB], (const T *)a[TS_DL], ring, red,
                                             it.f != nullptr, step);
            for (int e = threadIdx.x; e < (it.fac.nb + 1) * 16 * NC; e += blockDim.x) ring[e] = (T)0;
            __syncthreads();
            if (it.passes & 2)
                narrow_pass<T, NC, TMAX, PD, false>(it, (const T *)a[TS_UB], (const T *)a[TS_DU], ring, red, false,
                                                    step);
        }
    }
}

}  // namespace

int sweep_narrow_cols(bool f32) { return f32 ? 4 : 2; }
bool sweep_narrow_ok(bool f32, int max_nb, int ncols) {
    return max_nb >= 2 && max_nb <= 64 && ncols >= 1 && ncols <= sweep_narrow_cols(f32);
}

// Forward sweep of items with at most sweep_narrow_cols columns each
// (ncols_max) on factors with 2..64 band tiles per row.  A column's
// arithmetic does not depend on the other columns of its item.
hipError_t launch_sweep_narrow(bool f32, int nitems, const SweepItem *d_items, int nsteps, int max_nb,
                               int ncols_max, hipStream_t s, int step0) {
    if (nitems <= 0 || nsteps <= 0) return hipSuccess;
    if (!sweep_narrow_ok(f32, max_nb, ncols_max)) return hipErrorInvalidValue;
    const int grid = nitems < 65536 ? nitems : 65536;
    const int nc = ncols_max <= 1 ? 1 : (ncols_max <= 2 ? 2 : 4);
    const size_t esz = f32 ? 4 : 8;
    const size_t lds = esz * 16 * nc * ((size_t)(max_nb + 1) + 2 * (NBULK + 1));
#define LRPR_NARROW(TT, NCV, TMV, PDV)                                                                         \
    hipLaunchKernelGGL((k_sweep_narrow<TT, NCV, TMV, PDV>), dim3(grid), dim3(64 * NW), lds, s, d_items, nitems,    \
                       nsteps, step0)
    // bulk tiles per wave: 3 (nb <= 16), 5 (nb <= 32), 9 (nb <= 64); prefetch
    // depth (even) for at most about 150 registers of tiles and state per lane
#define LRPR_NARROW_NB(TT, NCV, P16, P32, P64)                                                                 \
    if (max_nb <= 16) LRPR_NARROW(TT, NCV, 3, P16);                                                            \
    else if (max_nb <= 32) LRPR_NARROW(TT, NCV, 5, P32);                                                       \
    else LRPR_NARROW(TT, NCV, 9, P64);
    if (f32) {
        if (nc == 1) { LRPR_NARROW_NB(float, 1, 8, 6, 4) }
        else if (nc == 2) { LRPR_NARROW_NB(float, 2, 6, 4, 2) }
        else { LRPR_NARROW_NB(float, 4, 4, 2, 2) }
    } else {
        if (nc == 1) { LRPR_NARROW_NB(double, 1, 4, 2, 2) }
        else { LRPR_NARROW_NB(double, 2, 2, 2, 2) }
    }
#undef LRPR_NARROW_NB
#undef LRPR_NARROW
    return hipGetLastError();
}

}  // namespace lrpr
