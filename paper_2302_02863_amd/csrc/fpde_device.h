// Device-side helpers shared by the HIP translation units: launch shapes,
// vector loads of the caller's x, the Chebyshev transfer products of the
// nested bases, and the (dim, points per dim) dispatch of templated kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_internal.h"

#define FPDE_KERNEL __global__ __launch_bounds__(256)

namespace fpde {

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline unsigned grid1(int64_t n, int bs = 256) {
    int64_t g = cdiv(n, bs);
    return (unsigned)(g < 1 ? 1 : (g > 2147483647 ? 2147483647 : g));
}

// element i of a caller vector of dtype 0 (double) or 1 (float)
__device__ __forceinline__ double ldx(const void* x, int64_t i, int dtype) {
    return dtype == 0 ? ((const double*)x)[i] : (double)((const float*)x)[i];
}

// |d|^{-e} from |d|^2: exp(-e/2 * log(r2))
__device__ __forceinline__ double rpow(double r2, double e) { return exp(-0.5 * e * log(r2)); }

// Stores and loads of values that another block of the same launch reads:
// agent-scope atomics, coherent across the XCDs' L2 caches.  A block hands
// such values over by waiting for its stores (s_waitcnt 0), a barrier, then one
// agent-scope counter increment; the block that sees the final count reads
// them with get().
template <typename T>
__device__ __forceinline__ void put(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T get(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroups of a launch go to the 8 XCDs round-robin by linear id (x fastest).
// xcd_block maps that id to a logical block so that XCD j runs the j-th
// contiguous eighth of the logical range: blocks that run at the same time on
// one XCD then work on neighbouring clusters and share their gathered rows in
// that XCD's L2.  Identity when the grid is not a multiple of 8.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t hw, int64_t total) {
    if (total % kXcds) return hw;
    return (hw % kXcds) * (total / kXcds) + hw / kXcds;
}

// sum over the 64 lanes of a wavefront
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Chebyshev rank and transfer size of a (dim, points per dim) tree
template <int D, int P>
struct KR {
    static constexpr int K = D == 2 ? P * P : P;
    static constexpr int EP = D * P * P;   // transfer entries per cluster: D matrices [b][a]
};

// Parent coefficient alpha from its two children (Sec. 5.3, nested bases):
// x_parent[alpha] = sum_c sum_beta E_c[beta][alpha] x_c[beta], E_c the Kronecker
// product of per-dimension P x P transfers stored [D][b][a]; x strided by R.
template <int D, int P, typename T>
__device__ __forceinline__ T up_t(const T* E1, const T* E2, const T* x1, const T* x2, int alpha, int R) {
    const int a0 = alpha % P, a1 = alpha / P;
    T acc = 0;
#pragma unroll
    for (int b1 = 0; b1 < (D == 2 ? P : 1); ++b1) {
        const T f1 = D == 2 ? E1[P * P + b1 * P + a1] : T(1);
        const T f2 = D == 2 ? E2[P * P + b1 * P + a1] : T(1);
        T s1 = 0, s2 = 0;
#pragma unroll
        for (int b0 = 0; b0 < P; ++b0) {
            s1 += E1[b0 * P + a0] * x1[(int64_t)(b0 + P * b1) * R];
            s2 += E2[b0 * P + a0] * x2[(int64_t)(b0 + P * b1) * R];
        }
        acc += f1 * s1 + f2 * s2;
    }
    return acc;
}

// Child coefficient beta of the downward transfer: (E_c y_parent)[beta]
template <int D, int P, typename T>
__device__ __forceinline__ T down_t(const T* Ec, const T* yp, int beta, int R) {
    const int b0 = beta % P, b1 = beta / P;
    T acc = 0;
#pragma unroll
    for (int a1 = 0; a1 < (D == 2 ? P : 1); ++a1) {
        const T f = D == 2 ? Ec[P * P + b1 * P + a1] : T(1);
        T s = 0;
#pragma unroll
        for (int a0 = 0; a0 < P; ++a0) s += Ec[b0 * P + a0] * yp[(int64_t)(a0 + P * a1) * R];
        acc += f * s;
    }
    return acc;
}

}  // namespace fpde

// Instantiate FN<D, P>(...) for the runtime dimension (1, 2) and points per dimension (1..8).
#define FPDE_DISPATCH_DP(dim, p, FN, ...)                                   \
    do {                                                                    \
        if (dim == 1) {                                                     \
            switch (p) {                                                    \
                case 1: FN<1, 1>(__VA_ARGS__); break;                       \
                case 2: FN<1, 2>(__VA_ARGS__); break;                       \
                case 3: FN<1, 3>(__VA_ARGS__); break;                       \
                case 4: FN<1, 4>(__VA_ARGS__); break;                       \
                case 5: FN<1, 5>(__VA_ARGS__); break;                       \
                case 6: FN<1, 6>(__VA_ARGS__); break;                       \
                case 7: FN<1, 7>(__VA_ARGS__); break;                       \
                default: FN<1, 8>(__VA_ARGS__); break;                      \
            }                                                               \
        } else {                                                            \
            switch (p) {                                                    \
                case 1: FN<2, 1>(__VA_ARGS__); break;                       \
                case 2: FN<2, 2>(__VA_ARGS__); break;                       \
                case 3: FN<2, 3>(__VA_ARGS__); break;                       \
                case 4: FN<2, 4>(__VA_ARGS__); break;                       \
                case 5: FN<2, 5>(__VA_ARGS__); break;                       \
                case 6: FN<2, 6>(__VA_ARGS__); break;                       \
                case 7: FN<2, 7>(__VA_ARGS__); break;                       \
                default: FN<2, 8>(__VA_ARGS__); break;                      \
            }                                                               \
        }                                                                   \
    } while (0)
