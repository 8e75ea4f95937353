// Partitioned forward solves for narrow panels (few 16-column groups).
//
// A substitution pass is sequential in its tile rows, so a group of 16
// right-hand sides keeps one compute unit busy for NT tile rows.  Cutting the
// rows into P blocks lets P compute units work on one group (the classical
// spike partitioning of a banded triangular solve):
//   local:  g_p = L_pp^{-1} r_p for every block p (the sweep kernel on the
//           block's range; rows before the block read as zero),
//   chain:  y_p^tail = g_p^tail - S_p^tail y_{p-1}^tail, p = 1..P-1, with
//           S_p = L_pp^{-1} L_{p,p-1}[:, tail] (tail: last nb tile rows),
//   update: y_p = g_p - S_p y_{p-1}^tail for every row of every block,
// and the mirror image for the back substitution with U (blocks from the
// last one down, heads = first nb tile rows, T_p = U_pp^{-1} U_{p,p+1}[:, head]).
// In exact arithmetic this is the same solve; every product runs on the
// matrix cores (v_mfma_*_16x16x4).  The spikes S_p, T_p are computed once per
// factor with the same local sweeps.
#include "lrpr_internal.h"
#include "tile_ops.h"

namespace lrpr {

__device__ inline double band_at(const double *lu, int64_t n, int bw, int64_t i, int64_t j) {
    if (i < 0 || j < 0 || i >= n || j >= n) return 0.0;
    const int64_t d = j - i;
    if (d < -bw || d > bw) return 0.0;
    return lu[i * (2 * bw + 1) + d + bw];
}

__device__ inline int block_of(const int *blk, int P, int I) {
    int lo = 0, hi = P - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk[mid] <= I) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Right-hand sides of the spike solves, dense column-major (NT*16 rows, ld),
// nb*16 columns: RL(i, j) = L(i, (blk[p]-nb)*16 + j) for the first nb tile
// rows of each block p >= 1; RU(i, j) = U(i, blk[p+1]*16 + j) for the last nb
// tile rows of each block p <= P-2; zero elsewhere.
__global__ void k_spike_rhs(int64_t n, int bw, int NT, int nb, int P, const int *blk, const double *lu,
                            double *RL, double *RU) {
    const int64_t ld = (int64_t)NT * TILE;
    const int64_t total = ld * nb * TILE;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % ld;
        const int j = (int)(e / ld);
        const int I = (int)(i / TILE);
        const int p = block_of(blk, P, I);
        double l = 0.0, u = 0.0;
        if (p >= 1 && I < blk[p] + nb) l = band_at(lu, n, bw, i, (int64_t)(blk[p] - nb) * TILE + j);
        if (p <= P - 2 && I >= blk[p + 1] - nb) u = band_at(lu, n, bw, i, (int64_t)blk[p + 1] * TILE + j);
        RL[e] = l;
        RU[e] = u;
    }
}

hipError_t launch_spike_rhs(int64_t n, int bw, int NT, int nb, int P, const int *d_blk, const double *lu,
                            double *RL, double *RU, hipStream_t s) {
    const int64_t total = (int64_t)NT * TILE * nb * TILE;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_spike_rhs, dim3((unsigned)blocks), dim3(256), 0, s, n, bw, NT, nb, P, d_blk, lu, RL, RU);
    return hipGetLastError();
}

// dense (NT*16 x nb*16, column-major, ld) -> NT x nb tiles, lane-major MFMA A
// operands: element (m, k) of tile (I, s) is dense(I*16 + m, s*16 + k)
template <typename T>
__global__ void k_spike_pack(int NT, int nb, const T *dense, int64_t ld, T *tiles) {
    const int64_t total = (int64_t)NT * nb * TILE_ELEMS;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t tile = e / TILE_ELEMS;
        const int o = (int)(e % TILE_ELEMS);
        const int64_t I = tile / nb;
        const int s = (int)(tile % nb);
        const int m = o >> 4, k = o & 15;
        int g, kc;
        Mf<T>::gk(k, g, kc);
        tiles[tile * TILE_ELEMS + Mf<T>::slot(16 * g + m, kc)] = dense[(I * TILE + m) + (int64_t)(s * TILE + k) * ld];
    }
}

hipError_t launch_spike_pack(bool f32, int NT, int nb, const void *dense, int64_t ld, void *tiles, hipStream_t s) {
    const int64_t total = (int64_t)NT * nb * TILE_ELEMS;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (f32)
        hipLaunchKernelGGL(k_spike_pack<float>, dim3((unsigned)blocks), dim3(256), 0, s, NT, nb, (const float *)dense,
                           ld, (float *)tiles);
    else
        hipLaunchKernelGGL(k_spike_pack<double>, dim3((unsigned)blocks), dim3(256), 0, s, NT, nb,
                           (const double *)dense, ld, (double *)tiles);
    return hipGetLastError();
}

// tile row I of the group's columns, accumulator order (rows clamped into the
// array: padded rows never feed a stored value)
template <typename T>
__device__ __forceinline__ void load_rows(const SplitGroup &G, int I, int lane, T (&v)[4]) {
    const int g = lane >> 4, c = lane & 15;
    const int col = c < G.ncols ? c : 0;
    const T *X = (const T *)G.X;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int row = I * TILE + Mf<T>::row(g, i);
        row = row < G.n ? row : G.n - 1;
        v[i] = gld(X + row + (int64_t)col * G.ldx);
    }
}

template <typename T>
__device__ __forceinline__ void store_rows(const SplitGroup &G, int I, int lane, const typename Mf<T>::v4 &v) {
    const int g = lane >> 4, c = lane & 15;
    if (c >= G.ncols) return;
    T *X = (T *)G.X;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = I * TILE + Mf<T>::row(g, i);
        if (row < G.n) gst(X + row + (int64_t)c * G.ldx, v[i]);
    }
}

// Chain over the blocks of one group (one workgroup of 4 waves per group).
// L (upper = false): bnd[0] = tail of block 0, bnd[p] = g_p^tail - S_p^tail
// bnd[p-1], p = 1..P-1.  U: bnd[P-1] = head of the last block, bnd[p] =
// h_p^head - T_p^head bnd[p+1].  Wave w computes the boundary tile rows
// t = w, w+4, ...; the spike tiles (A operands, independent of the chain
// values) stream through a PF-deep register ring across the steps, the
// previous step's boundary tiles (B operands) sit in LDS, double-buffered.
constexpr int CPF = 4;
constexpr int CHAIN_WAVES = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_split_chain(const SplitGroup *groups, int upper) {
    typedef typename Mf<T>::v4 v4;
    extern __shared__ __align__(16) unsigned char smem[];
    const SplitGroup G = groups[blockIdx.x];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ int sblk[SPLIT_MAX_P + 1];
    const int nb = G.nb, P = G.P;
    T *prev = (T *)smem;   // [2][nb] tiles, accumulator order
    const T *A = (const T *)(upper ? G.T : G.S);
    T *bnd = (T *)G.bnd;
    for (int i = threadIdx.x; i <= P; i += 256) sblk[i] = gld(G.blk + i);
    __syncthreads();
    // boundary rows of the chain's k-th block
    auto base_of = [&](int k) {
        const int p = upper ? P - 1 - k : k;
        return upper ? sblk[p] : sblk[p + 1] - nb;
    };
    auto block_of_k = [&](int k) { return upper ? P - 1 - k : k; };
    // first block: its own solution
    for (int t = w; t < nb; t += 4) {
        T x[4];
        load_rows(G, base_of(0) + t, lane, x);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            prev[t * TILE_ELEMS + i * 64 + lane] = x[i];
            gst(bnd + ((int64_t)block_of_k(0) * nb + t) * TILE_ELEMS + i * 64 + lane, x[i]);
        }
    }
    const int share = (nb + 3) / 4;                      // output tiles per wave (some may be void)
    const int ips = (share * nb + CPF - 1) / CPF * CPF;  // items per step, ring-aligned
    const int total = (P - 1) * ips;
    // A operand of item idx (void items read the block's first spike tile)
    auto a_ptr = [&](int idx) {
        const int k = 1 + idx / ips;
        const int i = idx % ips;
        const int j = i / nb, s = i % nb;
        const int t = w + 4 * j;
        const int kk = k < P ? k : P - 1;
        const int I = base_of(kk) + (t < nb && i < share * nb ? t : 0);
        return A + ((int64_t)I * nb + (t < nb && i < share * nb ? s : 0)) * TILE_ELEMS;
    };
    T abuf[CPF][4];
#pragma unroll
    for (int u = 0; u < CPF - 1; ++u) Mf<T>::ld4(a_ptr(u < total ? u : 0), lane, abuf[u]);
    v4 acc = {0, 0, 0, 0};
    T x[4] = {0, 0, 0, 0};
    for (int k = 1; k < P; ++k) {
        __syncthreads();   // step k-1's boundary tiles are in prev[(k-1)&1]
        const T *pin = prev + ((k - 1) & 1) * nb * TILE_ELEMS;
        T *pout = prev + (k & 1) * nb * TILE_ELEMS;
        const int base = base_of(k);
        const int p = block_of_k(k);
        for (int i0 = 0; i0 < ips; i0 += CPF) {
#pragma unroll
            for (int u = 0; u < CPF; ++u) {
                const int idx = (k - 1) * ips + i0 + u;
                const int nx = idx + CPF - 1;
                Mf<T>::ld4(a_ptr(nx < total ? nx : 0), lane, abuf[(u + CPF - 1) % CPF]);
                const int i = i0 + u;
                const int j = i / nb, s = i % nb;
                const int t = w + 4 * j;
                const bool valid = i < share * nb && t < nb;
                if (valid) {
                    if (s == 0) load_rows(G, base + t, lane, x);
                    const T *bs = pin + s * TILE_ELEMS;
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc) acc = Mf<T>::mma(abuf[u][kc], bs[kc * 64 + lane], acc);
                    if (s == nb - 1) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const T o = x[q] - acc[q];
                            pout[t * TILE_ELEMS + q * 64 + lane] = o;
                            gst(bnd + ((int64_t)p * nb + t) * TILE_ELEMS + q * 64 + lane, o);
                        }
                        acc = v4{0, 0, 0, 0};
                    }
                }
            }
        }
    }
}

// Chain for a compile-time band-tile count NB: CHAIN_WAVES waves (two per
// SIMD) take the NB output tiles of a step round-robin.  The spike tiles (A
// operands: they do not depend on the chain values) stream through a
// register ring of CHAIN_RING chunks of two tiles that runs ahead across
// output tiles and steps; the barrier between steps orders LDS only, so the
// prefetches stay in flight across it.  The previous step's boundary tiles
// (B operands) sit in LDS, double-buffered.
constexpr int CHAIN_RING = 4;

template <typename T, int NB>
__global__ __launch_bounds__(64 * CHAIN_WAVES) void k_split_chain_nb(const SplitGroup *groups, int upper) {
    typedef typename Mf<T>::v4 v4;
    constexpr int NW = CHAIN_WAVES;
    constexpr int NTW = (NB + NW - 1) / NW;   // output tiles per wave per step
    constexpr int CH = 2;                     // spike tiles per ring chunk
    constexpr int NCH = NB / CH;              // chunks per output tile (a multiple of the ring depth)
    constexpr int D = CHAIN_RING;
    static_assert(NCH % D == 0, "ring depth must divide the chunks of an output tile");
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int sblk[SPLIT_MAX_P + 1];     // block starts (LDS: no wait on the operand loads)
    const SplitGroup G = groups[blockIdx.x];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int P = G.P;
    T *prev = (T *)smem;   // [2][NB] tiles, accumulator order
    const T *A = (const T *)(upper ? G.T : G.S);
    T *bnd = (T *)G.bnd;
    for (int i = threadIdx.x; i <= P; i += 64 * NW) sblk[i] = gld(G.blk + i);
    __syncthreads();
    auto base_of = [&](int k) {
        const int p = upper ? P - 1 - k : k;
        return upper ? sblk[p] : sblk[p + 1] - NB;
    };
    auto block_of_k = [&](int k) { return upper ? P - 1 - k : k; };
    for (int t = w; t < NB; t += NW) {
        T x[4];
        load_rows(G, base_of(0) + t, lane, x);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            prev[t * TILE_ELEMS + i * 64 + lane] = x[i];
            gst(bnd + ((int64_t)block_of_k(0) * NB + t) * TILE_ELEMS + i * 64 + lane, x[i]);
        }
    }
    const int nq = (P - 1) * NTW;   // output tiles of this wave over the chain (some void)
    // spike row of output item q (void and past-the-end items read a valid row)
    auto a_row = [&](int q) {
        const int qq = q < nq ? q : 0;
        const int k = 1 + qq / NTW, t = w + NW * (qq % NTW);
        return A + (int64_t)(base_of(k) + (t < NB ? t : 0)) * NB * TILE_ELEMS;
    };
    auto load_chunk = [&](const T *row, int c, T (&buf)[CH][4]) {
#pragma unroll
        for (int s = 0; s < CH; ++s) Mf<T>::ld4(row + (int64_t)(c * CH + s) * TILE_ELEMS, lane, buf[s]);
    };
    T ring[D][CH][4];
    {
        const T *r0 = a_row(0);
#pragma unroll
        for (int c = 0; c < D - 1; ++c) load_chunk(r0, c, ring[c]);
    }
    for (int q = 0; q < nq; ++q) {
        const int k = 1 + q / NTW, j = q % NTW;
        if (j == 0) lds_barrier();   // step k-1's tiles are in prev[(k-1)&1]
        const int t = w + NW * j;
        const bool live = t < NB;
        const T *pin = prev + ((k - 1) & 1) * NB * TILE_ELEMS;
        const int I = base_of(k) + (live ? t : 0);
        T x[4];
        load_rows(G, I, lane, x);
        const T *row_cur = a_row(q), *row_nxt = a_row(q + 1);
        v4 acc = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};   // two accumulators: no product waits on the previous one
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            // prefetch the chunk D-1 ahead in the wave's stream (next output tile past the end)
            const int cn = c + D - 1;
            if (cn < NCH) load_chunk(row_cur, cn, ring[cn % D]);
            else load_chunk(row_nxt, cn - NCH, ring[cn % D]);
            if (live) {
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) {
                    acc = Mf<T>::mma(ring[c % D][0][kc], pin[(c * CH) * TILE_ELEMS + kc * 64 + lane], acc);
                    acc1 = Mf<T>::mma(ring[c % D][1][kc], pin[(c * CH + 1) * TILE_ELEMS + kc * 64 + lane], acc1);
                }
            }
        }
        if (live) {
            T *pout = prev + (k & 1) * NB * TILE_ELEMS;
            const int p = block_of_k(k);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const T o = x[i] - (acc[i] + acc1[i]);
                pout[t * TILE_ELEMS + i * 64 + lane] = o;
                gst(bnd + ((int64_t)p * NB + t) * TILE_ELEMS + i * 64 + lane, o);
            }
        }
    }
}

// nb of every group of a launch equals the launch's max_nb for the
// specialised kernels (checked by the host)
hipError_t launch_split_chain(bool f32, bool upper, int ngroups, const SplitGroup *d_groups, int max_nb,
                              hipStream_t s, bool uniform_nb) {
    if (ngroups <= 0) return hipSuccess;
    const size_t lds = 2 * (size_t)max_nb * TILE_ELEMS * (f32 ? 4 : 8);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const int up = upper ? 1 : 0;
#define LRPR_CHAIN_NB(NBV)                                                                                     \
    if (uniform_nb && max_nb == NBV) {                                                                         \
        if (f32)                                                                                               \
            hipLaunchKernelGGL((k_split_chain_nb<float, NBV>), dim3(ngroups), dim3(64 * CHAIN_WAVES), lds, s,  \
                               d_groups, up);                                                                  \
        else                                                                                                   \
            hipLaunchKernelGGL((k_split_chain_nb<double, NBV>), dim3(ngroups), dim3(64 * CHAIN_WAVES), lds, s, \
                               d_groups, up);                                                                  \
        return hipGetLastError();                                                                              \
    }
    LRPR_CHAIN_NB(8)
    LRPR_CHAIN_NB(16)
    LRPR_CHAIN_NB(32)
#undef LRPR_CHAIN_NB
    if (f32)
        hipLaunchKernelGGL(k_split_chain<float>, dim3(ngroups), dim3(256), lds, s, d_groups, up);
    else
        hipLaunchKernelGGL(k_split_chain<double>, dim3(ngroups), dim3(256), lds, s, d_groups, up);
    return hipGetLastError();
}

// Update of every block with a neighbour: one workgroup (4 waves) per
// (group, block, 4 tile rows); wave w updates tile row blk[p] + 4*chunk + w:
// X(I) -= sum_s A(I, s) bnd[neighbour][s], operands through a CPF-deep ring.
template <typename T>
__global__ __launch_bounds__(256) void k_split_update(const SplitGroup *groups, int upper, int maxP, int chunks) {
    typedef typename Mf<T>::v4 v4;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t unit = blockIdx.x;
    const int64_t per_group = (int64_t)maxP * chunks;
    const SplitGroup G = groups[unit / per_group];
    const int rest = (int)(unit % per_group);
    const int p = rest / chunks, chunk = rest % chunks;
    if (p >= G.P) return;
    if (upper ? p == G.P - 1 : p == 0) return;
    const int I = gld(G.blk + p) + 4 * chunk + w;
    if (I >= gld(G.blk + p + 1)) return;
    const int nb = G.nb;
    const T *A = (const T *)(upper ? G.T : G.S) + (int64_t)I * nb * TILE_ELEMS;
    const T *b = (const T *)G.bnd + (int64_t)(upper ? p + 1 : p - 1) * nb * TILE_ELEMS;
    T x[4];
    load_rows(G, I, lane, x);
    T abuf[CPF][4], bbuf[CPF][4];
    auto fetch = [&](int s, T (&av)[4], T (&bv)[4]) {
        const int ss = s < nb ? s : 0;
        Mf<T>::ld4(A + (int64_t)ss * TILE_ELEMS, lane, av);
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) bv[kc] = gld(b + (int64_t)ss * TILE_ELEMS + kc * 64 + lane);
    };
#pragma unroll
    for (int u = 0; u < CPF - 1; ++u) fetch(u, abuf[u], bbuf[u]);
    v4 acc = {0, 0, 0, 0};
    const int nsp = (nb + CPF - 1) / CPF * CPF;
    for (int s0 = 0; s0 < nsp; s0 += CPF) {
#pragma unroll
        for (int u = 0; u < CPF; ++u) {
            const int s = s0 + u;
            fetch(s + CPF - 1, abuf[(u + CPF - 1) % CPF], bbuf[(u + CPF - 1) % CPF]);
            if (s < nb) {
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) acc = Mf<T>::mma(abuf[u][kc], bbuf[u][kc], acc);
            }
        }
    }
    v4 o;
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = x[q] - acc[q];
    store_rows<T>(G, I, lane, o);
}

// Update for a compile-time band-tile count NB, one workgroup per (run of
// groups on the same factor, block, 4 tile rows): the spike tiles of a row
// (the same for every group of the run) are read once, the neighbour's
// boundary tiles of each group are staged in LDS (the next group's are loaded
// into registers while the current group multiplies).  Wave w updates tile row
// blk[p] + 4*chunk + w of every group of the run.
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_split_update_nb(const SplitGroup *groups, const int2 *runs, int upper,
                                                         int maxP, int chunks) {
    typedef typename Mf<T>::v4 v4;
    constexpr bool AREG = NB <= 16;   // spike row held in registers across the run
    extern __shared__ __align__(16) unsigned char smem[];
    T *bl = (T *)smem;   // NB tiles
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t unit = blockIdx.x;
    const int64_t per_run = (int64_t)maxP * chunks;
    const int2 run = runs[unit / per_run];
    const int rest = (int)(unit % per_run);
    const int p = rest / chunks, chunk = rest % chunks;
    const SplitGroup &G0 = groups[run.x];
    const int P = G0.P;
    if (p >= P) return;
    if (upper ? p == P - 1 : p == 0) return;
    const int b0 = gld(G0.blk + p), b1 = gld(G0.blk + p + 1);
    if (b0 + 4 * chunk >= b1) return;   // whole workgroup: uniform exit
    const int I = b0 + 4 * chunk + w;
    const bool valid = I < b1;          // waves past the block still take part in the staging
    const T *A = (const T *)(upper ? G0.T : G0.S) + (int64_t)(valid ? I : b0) * NB * TILE_ELEMS;
    T a[AREG ? NB : 1][4];
    if constexpr (AREG) {
#pragma unroll
        for (int s = 0; s < NB; ++s) Mf<T>::ld4(A + (int64_t)s * TILE_ELEMS, lane, a[s]);
    }
    const int nbr = upper ? p + 1 : p - 1;
    // the neighbour's boundary tiles of a group: NB values per thread, all
    // loads in flight together; the next group's load while this one multiplies
    constexpr int PER = NB * TILE_ELEMS / 256;
    T stg[PER];
    auto stage_load = [&](int g) {
        const T *b = (const T *)groups[g].bnd + (int64_t)nbr * NB * TILE_ELEMS;
#pragma unroll
        for (int i = 0; i < PER; ++i) stg[i] = gld(b + threadIdx.x + i * 256);
    };
    constexpr bool PRE = PER * sizeof(T) <= 128;   // next group's tiles held in registers while they fit
    if (PRE) stage_load(run.x);
    for (int g = run.x; g < run.x + run.y; ++g) {
        const SplitGroup &G = groups[g];
        if (!PRE) stage_load(g);
        if (g != run.x) __syncthreads();   // previous group's tiles consumed
#pragma unroll
        for (int i = 0; i < PER; ++i) bl[threadIdx.x + i * 256] = stg[i];
        __syncthreads();
        if (PRE && g + 1 < run.x + run.y) stage_load(g + 1);
        if (!valid) continue;
        T x[4];
        load_rows(G, I, lane, x);
        v4 acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};   // even / odd spike tiles
#pragma unroll
        for (int s = 0; s < NB; ++s) {
            T as[4];
            if constexpr (AREG) {
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) as[kc] = a[s][kc];
            } else {
                Mf<T>::ld4(A + (int64_t)s * TILE_ELEMS, lane, as);
            }
#pragma unroll
            for (int kc = 0; kc < 4; ++kc)
                acc[s & 1] = Mf<T>::mma(as[kc], bl[s * TILE_ELEMS + kc * 64 + lane], acc[s & 1]);
        }
        v4 o;
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = x[q] - (acc[0][q] + acc[1][q]);
        store_rows<T>(G, I, lane, o);
    }
}

hipError_t launch_split_update(bool f32, bool upper, int ngroups, const SplitGroup *d_groups, int max_P,
                               int max_rows, hipStream_t s, int max_nb, int nruns, const int2 *d_runs) {
    if (ngroups <= 0) return hipSuccess;
    const int chunks = (max_rows + 3) / 4;
    const int up = upper ? 1 : 0;
    const size_t lds = (size_t)max_nb * TILE_ELEMS * (f32 ? 4 : 8);
    if (d_runs) {
        const int64_t grid = (int64_t)nruns * max_P * chunks;
        if (grid > 0x7fffffff) return hipErrorInvalidValue;
#define LRPR_UPDATE_NB(NBV)                                                                                    \
        if (max_nb == NBV) {                                                                                   \
            if (f32)                                                                                           \
                hipLaunchKernelGGL((k_split_update_nb<float, NBV>), dim3((unsigned)grid), dim3(256), lds, s,   \
                                   d_groups, d_runs, up, max_P, chunks);                                       \
            else                                                                                               \
                hipLaunchKernelGGL((k_split_update_nb<double, NBV>), dim3((unsigned)grid), dim3(256), lds, s,  \
                                   d_groups, d_runs, up, max_P, chunks);                                       \
            return hipGetLastError();                                                                          \
        }
        LRPR_UPDATE_NB(8)
        LRPR_UPDATE_NB(16)
        LRPR_UPDATE_NB(32)
#undef LRPR_UPDATE_NB
        return hipErrorInvalidValue;
    }
    const int64_t grid = (int64_t)ngroups * max_P * chunks;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    if (f32)
        hipLaunchKernelGGL(k_split_update<float>, dim3((unsigned)grid), dim3(256), 0, s, d_groups, up, max_P, chunks);
    else
        hipLaunchKernelGGL(k_split_update<double>, dim3((unsigned)grid), dim3(256), 0, s, d_groups, up, max_P, chunks);
    return hipGetLastError();
}

}  // namespace lrpr
