// Device helpers shared by the sweep kernels: global loads/stores and the
// 16x16x4 MFMA operand layouts for FP64 and FP32 (lrpr_internal.h describes
// the lane-major tile layout they read).
#pragma once
#include <hip/hip_runtime.h>

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

// Barrier that orders LDS traffic only: outstanding global loads (prefetches
// of operands needed later) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace lrpr
