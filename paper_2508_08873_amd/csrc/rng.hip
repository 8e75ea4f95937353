// On-device Gaussian test matrices: Philox4x32-10 (Salmon, Moraes, Dror,
// Shaw, SC'11) with the Box-Muller transform, so that the random test vectors
// of the range finder (Sec. 2.1, step 1) can be drawn where they are used.
//
// Gaussian pair j of stream s under seed k: counter (j mod 2^32, j div 2^32,
// s mod 2^32, s div 2^32), key (k mod 2^32, k div 2^32), ten rounds; the
// output words (x0, x1) and (x2, x3) give two 53-bit uniforms
// u = (floor((hi 2^32 + lo) / 2^11) + 1/2) 2^-53 in (0, 1), and elements 2j,
// 2j+1 are r cos(2 pi u2), r sin(2 pi u2) with r = sqrt(-2 ln u1), in FP64
// (rounded once for an FP32 destination).
#include "lrpr_internal.h"

namespace lrpr {

namespace {
constexpr uint32_t PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;
constexpr uint32_t PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(PH_M0, c[0]), lo0 = PH_M0 * c[0];
        const uint32_t hi1 = __umulhi(PH_M1, c[2]), lo1 = PH_M1 * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += PH_W0;
        k1 += PH_W1;
    }
}

__device__ __forceinline__ double u53(uint32_t hi, uint32_t lo) {
    const uint64_t k = ((uint64_t)hi << 32 | lo) >> 11;
    return ((double)k + 0.5) * 0x1.0p-53;
}
}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void k_randn(T *dst, int64_t count, uint64_t seed, uint64_t stream) {
    const int64_t npairs = (count + 1) / 2;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < npairs;
         j += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c[4] = {(uint32_t)j, (uint32_t)((uint64_t)j >> 32), (uint32_t)stream, (uint32_t)(stream >> 32)};
        philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
        const double r = sqrt(-2.0 * log(u1));
        const double a = 2.0 * M_PI * u2;
        dst[2 * j] = (T)(r * cos(a));
        if (2 * j + 1 < count) dst[2 * j + 1] = (T)(r * sin(a));
    }
}

hipError_t launch_randn(bool f32, void *dst, int64_t count, uint64_t seed, uint64_t stream, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t npairs = (count + 1) / 2;
    int64_t blocks = (npairs + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (f32)
        hipLaunchKernelGGL(k_randn<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float *)dst, count, seed, stream);
    else
        hipLaunchKernelGGL(k_randn<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double *)dst, count, seed,
                           stream);
    return hipGetLastError();
}

}  // namespace lrpr
