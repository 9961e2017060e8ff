// Device steps of the far field's algebraic recompression (Sec. 5.3, closing
// remark), FP64, K <= 32.  The host orthogonalises and truncates the bases
// (fpde_recompress.cpp); these kernels do the per-pair work over every field:
//   k_rc_weights  H_t = sum_f sum_{(t,s) far} S C_s S^T   (per target cluster)
//   k_rc_project  S' = P_t S P_s^T                         (per far pair and field)
// St[f][e][beta][alpha] = S_e[alpha][beta] in both the input and the output.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_device.h"
#include "fpde_recompress.h"

namespace fpde {

namespace {
constexpr int kP = 32, kPS = kP + 1;   // padded LDS rows
}

// One block per target cluster t; the thread owns H_t entries tid + 256 m.
FPDE_KERNEL void k_rc_weights(int K, int F, int64_t nfar, const int64_t* __restrict__ far_ptr,
                              const int64_t* __restrict__ far_src, const double* __restrict__ St,
                              const double* __restrict__ C, double* __restrict__ H) {
    __shared__ double sS[kP * kPS];   // S[alpha][beta]
    __shared__ double sC[kP * kPS];   // C_s[beta][beta']
    __shared__ double sW[kP * kPS];   // (S C_s)[alpha][beta']
    const int64_t t = blockIdx.x;
    const int tid = threadIdx.x, KK = K * K;
    double h[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t e = far_ptr[t]; e < far_ptr[t + 1]; ++e) {
        const int64_t s = far_src[e];
        for (int i = tid; i < KK; i += blockDim.x) sC[(i / K) * kPS + i % K] = C[s * KK + i];
        for (int f = 0; f < F; ++f) {
            __syncthreads();   // the previous pair's products are done with sS / sW
            const double* Se = St + ((int64_t)f * nfar + e) * KK;
            for (int i = tid; i < KK; i += blockDim.x) sS[(i % K) * kPS + i / K] = Se[i];   // Se[beta][alpha]
            __syncthreads();
            for (int i = tid; i < KK; i += blockDim.x) {
                const int al = i / K, bp = i % K;
                double w = 0.0;
                for (int b = 0; b < K; ++b) w += sS[al * kPS + b] * sC[b * kPS + bp];
                sW[al * kPS + bp] = w;
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int i = tid + 256 * m;
                if (i >= KK) break;
                const int al = i / K, ap = i % K;
                double v = 0.0;
                for (int b = 0; b < K; ++b) v += sW[al * kPS + b] * sS[ap * kPS + b];
                h[m] += v;
            }
        }
        __syncthreads();   // sC is reloaded for the next pair
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int i = tid + 256 * m;
        if (i < KK) H[t * KK + i] = h[m];
    }
}

hipError_t launch_rc_weights(int64_t ncl, int K, int F, int64_t nfar, const int64_t* far_ptr, const int64_t* far_src,
                             const double* St, const double* C, double* H, hipStream_t st) {
    if (K > kP) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rc_weights, dim3((unsigned)ncl), dim3(256), 0, st, K, F, nfar, far_ptr, far_src, St, C, H);
    return hipGetLastError();
}

// One block per (far pair e, field f): T = P_t S (r x K), S' = T P_s^T (r x r).
FPDE_KERNEL void k_rc_project(int K, int r, int64_t nfar, const int64_t* __restrict__ far_tgt,
                              const int64_t* __restrict__ far_src, const double* __restrict__ St,
                              const double* __restrict__ P, double* __restrict__ Sr) {
    __shared__ double sS[kP * kPS];    // S[alpha][beta]
    __shared__ double sPt[kP * kPS];   // P_t[i][alpha]
    __shared__ double sPs[kP * kPS];   // P_s[j][beta]
    __shared__ double sT[kP * kPS];    // (P_t S)[i][beta]
    const int64_t e = blockIdx.x;
    const int f = blockIdx.y, tid = threadIdx.x, KK = K * K;
    const int64_t t = far_tgt[e], s = far_src[e];
    const double* Se = St + ((int64_t)f * nfar + e) * KK;
    for (int i = tid; i < KK; i += blockDim.x) sS[(i % K) * kPS + i / K] = Se[i];
    for (int i = tid; i < r * K; i += blockDim.x) {
        sPt[(i / K) * kPS + i % K] = P[t * r * K + i];
        sPs[(i / K) * kPS + i % K] = P[s * r * K + i];
    }
    __syncthreads();
    for (int i = tid; i < r * K; i += blockDim.x) {
        const int ii = i / K, b = i % K;
        double v = 0.0;
        for (int a = 0; a < K; ++a) v += sPt[ii * kPS + a] * sS[a * kPS + b];
        sT[ii * kPS + b] = v;
    }
    __syncthreads();
    double* So = Sr + ((int64_t)f * nfar + e) * r * r;
    for (int i = tid; i < r * r; i += blockDim.x) {
        const int jj = i / r, ii = i % r;   // output [beta = jj][alpha = ii]
        double v = 0.0;
        for (int b = 0; b < K; ++b) v += sT[ii * kPS + b] * sPs[jj * kPS + b];
        So[i] = v;
    }
}

hipError_t launch_rc_project(int64_t ncl, int K, int r, int F, int64_t nfar, const int64_t* far_tgt,
                             const int64_t* far_src, const double* St, const double* P, double* Sr, hipStream_t st) {
    (void)ncl;
    if (K > kP || r > kP || r < 1) return hipErrorInvalidValue;
    if (nfar <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rc_project, dim3((unsigned)nfar, F), dim3(256), 0, st, K, r, nfar, far_tgt, far_src, St, P,
                       Sr);
    return hipGetLastError();
}

}  // namespace fpde
