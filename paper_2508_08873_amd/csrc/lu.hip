// Banded LU without pivoting, M = L U, as a pipelined tile factorisation on
// the matrix cores (FP64).  The paper's fine solver factors the implicit-Euler
// matrix once and reuses it for every right-hand side (Sec. 4.4); M is a
// row- and column-diagonally dominant M-matrix, so elimination without
// pivoting is stable.
//
// Tiles of 16x16: tile column J holds tile rows I = J-nb..J+nb (nb =
// ceil(b/16)).  Right-looking elimination in tile form:
//   for K < J (K >= J-nb):  U(K,J) = L(K,K)^{-1} A(K,J)
//                           A(I,J) -= L(I,K) U(K,J),   K < I <= K+nb
//   then                    A(J,J) = L(J,J) U(J,J)     (unblocked, in LDS)
//                           L(I,J) = A(I,J) U(J,J)^{-1},  J < I <= J+nb
// Entries outside the band stay exactly zero (each of their update terms has
// a zero factor), so only in-band entries are stored back.
//
// Workgroup p owns tile columns J = p, p+P, p+2P, ... and keeps the 2nb+1
// tiles of its current column in registers (accumulator layout, tiles dealt
// round-robin to the waves).  When column J is done it publishes L(J,J)^{-1}
// and the L(I,J) tiles (MFMA A-operand layout) and raises flag[J]; the owner
// of a later column waits for flag[K] before applying panel K.  Every wait
// is bounded: on time-out it raises *err and the kernel runs to its end.
// All P workgroups are resident together (a launch holds no more workgroups
// than the device keeps resident at once), and every wait is for a lower
// column, so the pipeline always drains.
#include <algorithm>
#include <vector>

#include "lrpr_internal.h"
#include "tile_ops.h"

namespace lrpr {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ v4d mfma64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// MFMA A-operand tiles, lane-major: chunk kc of lane l at 128 (kc/2) + 2 l +
// kc%2; lane l = 16 g + m holds row m, contraction index k = 4 kc + g.
__device__ __forceinline__ int apos(int m, int k) { return 128 * ((k >> 2) >> 1) + 2 * (16 * (k & 3) + m) + ((k >> 2) & 1); }
typedef __attribute__((address_space(1))) const d2v *gd2p;
__device__ __forceinline__ void ld_a(const double *tile, int lane, double (&v)[4]) {
    const d2v x = *(gd2p)(tile + 2 * lane), y = *(gd2p)(tile + 128 + 2 * lane);
    v[0] = x[0]; v[1] = x[1]; v[2] = y[0]; v[3] = y[1];
}

struct LuArgs {
    int64_t n;
    int bw, NT, nb;
    double *band;   // n x (2bw+1) row-major: in M, out L (strict lower) and U
    double *Lt;     // [NT][nb] tiles: L(K+1+d, K), A-operand layout
    double *Li;     // [NT] tiles: L(K,K)^{-1}, A-operand layout
    int *flag;      // [NT], zero on entry
    int *info;      // min over bad pivots of (row + 1); 0x7f7f7f7f if none
    int *err;       // nonzero after a wait timed out
    int spin_limit;
};

// wait until column K is published, then take every later column up to
// Kmax that is published too with the same acquire; returns the last of them
// (workgroup-uniform).  One cache invalidation then covers several panels.
__device__ __forceinline__ int wait_upto(const LuArgs &a, int K, int Kmax, int *shared_last) {
    if (threadIdx.x == 0) {
        int spins = 0;
        while (__hip_atomic_load(a.flag + K, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
            if (++spins > a.spin_limit) {
                __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        int last = K;
        while (last < Kmax && __hip_atomic_load(a.flag + last + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            ++last;
        *shared_last = last;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *shared_last;
}

// Panels staged through LDS (one buffer of nb tiles, filled by direct
// global-to-LDS loads) for nb <= 32 with one wave per SIMD; wider bands read
// the L tiles from memory as they are applied.  The diagonal tile's buffers
// share the dynamic LDS with the panel (they are used after a column's panel
// loop).  No register buffer holds a panel, which leaves the registers to the
// column's tiles.
constexpr int PANEL_NB = 32;
constexpr int PANEL_VECS = PANEL_NB * (TILE_ELEMS / 2) / 256;   // 16-byte vectors per thread (256 threads)
static bool lu_ldsp(int NW, int nb) { return NW == 4 && nb <= PANEL_NB; }
size_t tile_lu_lds_bytes(int NW, int nb) {
    const size_t panel = lu_ldsp(NW, nb) ? (size_t)nb * TILE_ELEMS : 0, diag = (size_t)(4 + NW) * TILE_ELEMS;
    return 8 * std::max(panel, diag);
}

// Linear workgroup order in which each XCD holds a contiguous range: the
// chip deals workgroup b to XCD b % 8, and each XCD has its own L2, so a
// matrix's workgroups (consecutive in this order) read its panels through
// one L2.  A bijection on [0, G).
__device__ __forceinline__ int lu_xcd_linear(int b, int G) {
    const int q = G >> 3, r = G & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

template <int NW, int TPW>
__global__ __launch_bounds__(64 * NW, NW == 4 ? 2 : 1) void k_tile_lu(const LuArgs *args, int P) {
    constexpr bool LDSP = NW == 4;
    // dynamic LDS: the panel [nb][256] while the panels are applied (LDSP),
    // then the diagonal tile's buffers, all row-major 16x16: sd, sd2 (the two
    // buffers of the diagonal elimination), sli = L(J,J)^{-1},
    // sui = U(J,J)^{-1}, st[w] (wave w's transposition buffer)
    extern __shared__ __align__(16) double lu_lds[];
    double *const sd = lu_lds, *const sd2 = lu_lds + 256, *const sli = lu_lds + 512, *const sui = lu_lds + 768;
    __shared__ double ubuf[2][256];   // U(K,J), accumulator order
    __shared__ int s_last;            // last published column seen by wait_upto
    // workgroups [P*i, P*i + P) of the XCD-contiguous order factor matrix i
    const int lin = lu_xcd_linear(blockIdx.x, gridDim.x);
    const int wg = lin % P;
    const LuArgs a = args[lin / P];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, c = lane & 15;
    const int nb = a.nb, NT = a.NT, bw = a.bw;
    const int64_t n = a.n, W = 2 * bw + 1;
    double *band = a.band;

    for (int J = wg; J < NT; J += P) {
        // ---- load tile column J (tile t = I - J + nb, owned by wave t % NW)
        v4d acc[TPW];
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            const int t = w + NW * s;
            const int I = J - nb + t;
            const bool ex = t <= 2 * nb && I >= 0 && I < NT;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t row = (int64_t)I * TILE + 4 * i + g, col = (int64_t)J * TILE + c;
                double v = 0.0;
                if (ex) {
                    if (row >= n || col >= n) v = (row == col) ? 1.0 : 0.0;   // padding: identity
                    else if (col - row <= bw && row - col <= bw) v = band[row * W + (col - row) + bw];
                }
                acc[s][i] = v;
            }
        }
        // ---- apply panels K = J-nb .. J-1
        const int K0 = J - nb > 0 ? J - nb : 0;
        int avail = K0 - 1;   // columns up to avail are published and acquired
        // U(K,J) = L(K,K)^{-1} A(K,J) by the wave holding tile K, to LDS
        auto form_u = [&](int K) {
            const int tK = K - J + nb;
            double *ub = ubuf[K & 1];
            if (w == tK % NW) {
                double li[4];
                ld_a(a.Li + (int64_t)K * TILE_ELEMS, lane, li);
#pragma unroll
                for (int s = 0; s < TPW; ++s) {
                    if (s == tK / NW) {
                        v4d u = {0, 0, 0, 0};
#pragma unroll
                        for (int kc = 0; kc < 4; ++kc) u = mfma64(li[kc], acc[s][kc], u);
                        acc[s] = u;
#pragma unroll
                        for (int i = 0; i < 4; ++i) ub[i * 64 + lane] = u[i];
                    }
                }
            }
        };
        // A(I,J) -= L(I,K) U(K,J) for the wave's tiles in rows K+1..K+nb
        auto apply = [&](int K, auto &&ltile) {
            const double *ub = ubuf[K & 1];
            double ubv[4];
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) ubv[kc] = ub[kc * 64 + lane];
#pragma unroll
            for (int s = 0; s < TPW; ++s) {
                const int t = w + NW * s;
                const int I = J - nb + t;
                if (t <= 2 * nb && I > K && I <= K + nb && I < NT) {
                    double l[4];
                    ltile(I - K - 1, l);
#pragma unroll
                    for (int kc = 0; kc < 4; ++kc) acc[s] = mfma64(-l[kc], ubv[kc], acc[s]);
                }
            }
        };
        if constexpr (LDSP) {
            // the nb L tiles of a panel are contiguous in Lt: copied to LDS by
            // direct global-to-LDS loads (16 bytes a lane, one contiguous KB
            // a wave instruction), in flight while U(K,J) is formed; the
            // first barrier orders the previous panel's LDS reads before the
            // copy, the second waits for every wave's copy
            double *const pb = lu_lds;
            const int nv = nb * (TILE_ELEMS / 2);   // 16-byte vectors per panel (a multiple of 128)
            typedef __attribute__((address_space(3))) void *lds_ptr;
            for (int K = K0; K < J; ++K) {
                if (K > avail) avail = wait_upto(a, K, J - 1, &s_last);
                lds_barrier();
                const double *src = a.Lt + (int64_t)K * nb * TILE_ELEMS;
#pragma unroll
                for (int i = 0; i < PANEL_VECS; ++i) {
                    const int e0 = 256 * i + 64 * w;   // wave-uniform; e0 < nv implies e0 + 64 <= nv
                    if (e0 < nv)
                        __builtin_amdgcn_global_load_lds((const void *)(src + 2 * (e0 + lane)), (lds_ptr)(pb + 2 * e0),
                                                         16, 0, 0);
                }
                form_u(K);
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                apply(K, [&](int d, double (&l)[4]) {
                    const d2v x = *(const d2v *)(pb + d * TILE_ELEMS + 2 * lane);
                    const d2v y = *(const d2v *)(pb + d * TILE_ELEMS + 128 + 2 * lane);
                    l[0] = x[0]; l[1] = x[1]; l[2] = y[0]; l[3] = y[1];
                });
            }
            lds_barrier();   // the diagonal tile's buffers overwrite the panel
        } else {
            for (int K = K0; K < J; ++K) {
                if (K > avail) avail = wait_upto(a, K, J - 1, &s_last);
                form_u(K);
                lds_barrier();
                apply(K, [&](int d, double (&l)[4]) {
                    ld_a(a.Lt + ((int64_t)K * nb + d) * TILE_ELEMS, lane, l);
                });
            }
        }
        // ---- diagonal tile: unblocked LU in LDS
        if (w == nb % NW) {
#pragma unroll
            for (int s = 0; s < TPW; ++s)
                if (s == nb / NW) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) sd[(4 * i + g) * TILE + c] = acc[s][i];
                }
        }
        __syncthreads();
        const int r = (tid >> 4) & 15, q = tid & 15;
        // one barrier per pivot: step p reads buffer p%2 and writes the other
        // (the multiplier l = A(r,p)/A(p,p) is recomputed by every thread of
        // row r, bit-identical to the stored one)
        for (int p = 0; p < TILE; ++p) {
            const double *cur = (p & 1) ? sd2 : sd;
            double *nxt = (p & 1) ? sd : sd2;
            const double piv = cur[p * TILE + p];
            if (tid == 0 && (int64_t)J * TILE + p < n && !(piv != 0.0 && isfinite(piv)))
                atomicMin(a.info, J * TILE + p + 1);
            if (tid < 256) {
                double v = cur[r * TILE + q];
                if (r > p) {
                    const double l = cur[r * TILE + p] / piv;
                    if (q == p) v = l;
                    else if (q > p) v -= l * cur[p * TILE + q];
                }
                nxt[r * TILE + q] = v;
            }
            __syncthreads();
        }
        // ---- inverses of the unit-lower L(J,J) (wave 0) and of U(J,J) (wave 1)
        //      on the matrix cores.  With L = I + N (N strictly lower, N^16 = 0):
        //      L^{-1} = (I - N)(I + N^2)(I + N^4)(I + N^8), an exact finite product;
        //      U = D (I + N') with N' = D^{-1}(U - D) strictly upper, so
        //      U^{-1} = (I - N')(I + N'^2)(I + N'^4)(I + N'^8) D^{-1}.
        if (w < 2) {
            const bool up = w == 1;
            double *buf = lu_lds + (4 + w) * 256;   // st[w]
            // N (or N') in accumulator layout
            v4d N;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 4 * i + g;
                const double x = sd[row * TILE + c];
                N[i] = up ? (c > row ? x / sd[row * TILE + row] : 0.0) : (row > c ? x : 0.0);
            }
            // X * Y with Y in accumulator layout (B operand), X staged through LDS
            auto mm = [&](const v4d &X, const v4d &Y) {
#pragma unroll
                for (int i = 0; i < 4; ++i) buf[(4 * i + g) * TILE + c] = X[i];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                double xa[4];
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) xa[kc] = buf[c * TILE + 4 * kc + g];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                v4d o = {0, 0, 0, 0};
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) o = mfma64(xa[kc], Y[kc], o);
                return o;
            };
            v4d I4;
#pragma unroll
            for (int i = 0; i < 4; ++i) I4[i] = (4 * i + g == c) ? 1.0 : 0.0;
            const v4d N2 = mm(N, N);
            v4d P = I4 - N;                       // (I - N)
            P = P + mm(P, N2);                    // (I - N)(I + N^2)
            const v4d N4 = mm(N2, N2);
            P = P + mm(P, N4);
            const v4d N8 = mm(N4, N4);
            P = P + mm(P, N8);
            double *dst = up ? sui : sli;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 4 * i + g;
                // U^{-1} = (I + N')^{-1} D^{-1}: column c scaled by 1 / U(c,c)
                dst[row * TILE + c] = up ? P[i] / sd[c * TILE + c] : P[i];
            }
        }
        __syncthreads();
        if (tid < 256) a.Li[(int64_t)J * TILE_ELEMS + apos(r, q)] = sli[r * TILE + q];
        // ---- L(I,J) = A(I,J) U(J,J)^{-1}: A(I,J) as A operand via the wave's
        //      transposition buffer, U^{-1} as B operand
        double uiv[4];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) uiv[kc] = sui[(4 * kc + g) * TILE + c];
        double *stw = lu_lds + (4 + w) * 256;   // st[w]
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            const int t = w + NW * s;
            const int I = J - nb + t;
            if (t > nb && t <= 2 * nb && I < NT) {
#pragma unroll
                for (int i = 0; i < 4; ++i) stw[(4 * i + g) * TILE + c] = acc[s][i];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                v4d l = {0, 0, 0, 0};
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) l = mfma64(stw[c * TILE + 4 * kc + g], uiv[kc], l);
                acc[s] = l;
                double *dst = a.Lt + ((int64_t)J * nb + (t - nb - 1)) * TILE_ELEMS;
#pragma unroll
                for (int i = 0; i < 4; ++i) dst[apos(4 * i + g, c)] = l[i];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        // ---- publish panel J
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) __hip_atomic_store(a.flag + J, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // ---- store the column's factors into the band (in-band entries)
#pragma unroll
        for (int s = 0; s < TPW; ++s) {
            const int t = w + NW * s;
            const int I = J - nb + t;
            if (t <= 2 * nb && t != nb && I >= 0 && I < NT) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int64_t row = (int64_t)I * TILE + 4 * i + g, col = (int64_t)J * TILE + c;
                    if (row < n && col < n && col - row <= bw && row - col <= bw)
                        band[row * W + (col - row) + bw] = acc[s][i];
                }
            }
        }
        if (tid < 256) {
            const int64_t row = (int64_t)J * TILE + r, col = (int64_t)J * TILE + q;
            if (row < n && col < n && col - row <= bw && row - col <= bw) band[row * W + (col - row) + bw] = sd[r * TILE + q];
        }
        __syncthreads();   // sd, sli, sui, ubuf are reused by the next column
    }
}

size_t tile_lu_scratch_bytes(int NT, int nb) {
    return sizeof(double) * ((size_t)NT * nb + NT) * TILE_ELEMS + sizeof(int) * ((size_t)NT + 2);
}

// the kernel variant for nb band tiles per row (f gets the kernel and its
// waves per workgroup)
template <typename F>
static hipError_t with_lu_kernel(int nb, F &&f) {
    if (nb <= 4) return f(k_tile_lu<4, 3>, 4);
    if (nb <= 16) return f(k_tile_lu<4, 9>, 4);
    if (nb <= 32) return f(k_tile_lu<4, 17>, 4);
    if (nb <= 64) return f(k_tile_lu<8, 17>, 8);
    return hipErrorInvalidValue;
}

// One workgroup per compute unit: every variant keeps at least one resident
// per compute unit (an occupancy query confirms it), and two per compute unit
// (P = 16 for 32 matrices of 511^2: 2.14 s) were slower than one (P = 8:
// 1.84 s): the compute unit's throughput, not load latency, bounds a column.
int tile_lu_resident(int nb) {
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        return 256;
    const hipError_t e = with_lu_kernel(nb, [&](auto kern, int NW) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * NW, tile_lu_lds_bytes(NW, nb));
    });
    if (e != hipSuccess || per_cu < 1) return 0;   // the launch reports the error
    return ncu;
}

int tile_lu_wgs(int count, int NT, int nb, int wgs, int resident) {
    const int full = std::min(nb + 9, NT);
    if (wgs > 0) return std::max(1, std::min(wgs, full));
    // one matrix's P workgroups own every P-th tile column; a column's owner
    // applies its nb panels as they are published, about nb*(nb+1) tile
    // products, and must be done before the chain reaches its next column
    // P columns later.  nb + 9 leaves wide slack; when a batch would need
    // more launches at that width, fewer workgroups per matrix let more
    // matrices share a launch (at least 6 each)
    if ((int64_t)count * full <= resident) return full;
    const int lo = std::min(full, 6);
    return std::max(lo, std::min(full, resident / count));
}

// Several independent factorisations of one shape in one launch: P workgroups
// per matrix (tile_lu_wgs), no more workgroups per launch than the device
// keeps resident at once (tile_lu_resident), so that every matrix's
// workgroups are resident together (their waits only involve each other).  Each matrix i has its band, scratch (tile_lu_scratch_bytes) and
// on return info_dev[i] / err_dev[i] point into its scratch (pivot info:
// 0x7f7f7f7f if all pivots are fine, else the first bad row + 1; err:
// nonzero on a wait time-out).  d_args: device space for count LuArgs.
// The factors do not depend on P: every column applies its panels in the
// same order whichever workgroup owns it.
hipError_t launch_tile_lu_batch(int count, const int64_t *ns, int bw, int NT, int nb, double *const *bands,
                                void *const *scratch, int **info_dev, int **err_dev, void *d_args, hipStream_t s,
                                int wgs) {
    std::vector<LuArgs> hv(count);
    for (int i = 0; i < count; ++i) {
        LuArgs &a = hv[i];
        a.n = ns[i];
        a.bw = bw;
        a.NT = NT;
        a.nb = nb;
        a.band = bands[i];
        a.Lt = (double *)scratch[i];
        a.Li = a.Lt + (size_t)NT * nb * TILE_ELEMS;
        a.flag = (int *)(a.Li + (size_t)NT * TILE_ELEMS);
        a.info = a.flag + NT;
        a.err = a.info + 1;
        a.spin_limit = 1 << 22;
        info_dev[i] = a.info;
        err_dev[i] = a.err;
        hipError_t e;
        if ((e = hipMemsetAsync(a.flag, 0, sizeof(int) * (size_t)NT, s)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(a.info, 0x7f, sizeof(int), s)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(a.err, 0, sizeof(int), s)) != hipSuccess) return e;
    }
    if (nb > 64) return hipErrorInvalidValue;
    const int resident = tile_lu_resident(nb);
    if (resident < 1) return hipErrorInvalidConfiguration;
    const int P = tile_lu_wgs(count, NT, nb, wgs, resident);
    const int per = P > resident ? 1 : resident / P;   // matrices per launch
    LuArgs *dA = (LuArgs *)d_args;
    hipError_t e = hipMemcpyAsync(dA, hv.data(), sizeof(LuArgs) * (size_t)count, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    for (int i0 = 0; i0 < count; i0 += per) {
        const int c = count - i0 < per ? count - i0 : per;
        const dim3 grid((unsigned)(c * P));
        e = with_lu_kernel(nb, [&](auto kern, int NW) {
            hipLaunchKernelGGL(kern, grid, dim3(64 * NW), tile_lu_lds_bytes(NW, nb), s, dA + i0, P);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t tile_lu_args_bytes(int count) { return sizeof(LuArgs) * (size_t)count; }

}  // namespace lrpr
