// Far field of the apply for many right-hand sides (Sec. 5.3, nested bases),
// with the operator data in FP64 or FP32.  Coefficients are [F][cluster][K][R]
// (right-hand sides fastest).  Each stage is a batch of small dense products:
//   k_bup_leaf     X^_leaf = U_leaf^T X_leaf            (per leaf, 64 rhs)
//   k_bup_level    X^_parent = sum_c E_c^T X^_c          (per level)
//   k_bcoupling    Y^_S = sum_{S' far S} S_(S,S') X^_S'  (MFMA, per target cluster)
//   k_bdown_level  Y^_c += E_c Y^_parent                 (per level)
//   k_bout_leaf    y_leaf += U_leaf Y^_leaf              (per leaf, added to y)
// The coupling products, 2 K^2 R flops per far pair and field, are the bulk
// of the work: FP32 operator data uses v_mfma_f32_32x32x2f32, FP64 uses
// v_mfma_f64_16x16x4f64 (lane layouts as in the near-panel GEMM).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_device.h"

namespace fpde {

namespace {
typedef float bf32x16 __attribute__((ext_vector_type(16)));
typedef double bf64x4 __attribute__((ext_vector_type(4)));
constexpr int kRC = 64;   // right-hand sides per block
}  // namespace

// X^_leaf[alpha][r] = sum_j U[j][alpha] x[perm[j]][r]; one block per (leaf, rhs chunk, field)
template <typename T>
__global__ __launch_bounds__(256) void k_bup_leaf(ApplyPlan a, H2Tree t, int F, int R, const T* U, int dtype,
                                                  const void* x, T* xh) {
    extern __shared__ __align__(16) unsigned char sraw[];
    const int K = t.k;
    const int64_t nrc = (R + kRC - 1) / kRC;
    const int64_t li = blockIdx.x / nrc;
    const int r0 = (int)(blockIdx.x % nrc) * kRC;
    const int f = blockIdx.y;
    const int64_t lb = a.leaf_beg[li], n = a.leaf_beg[li + 1] - lb;
    T* sU = (T*)sraw;          // [n][K]
    T* sX = sU + n * K;        // [n][kRC]
    for (int64_t i = threadIdx.x; i < n * K; i += blockDim.x) sU[i] = U[lb * K + i];
    for (int64_t i = threadIdx.x; i < n * kRC; i += blockDim.x) {
        const int64_t j = i / kRC;
        const int r = r0 + (int)(i % kRC);
        sX[i] = r < R ? (T)ldx(x, ((int64_t)f * a.N + a.perm[lb + j]) * R + r, dtype) : T(0);
    }
    __syncthreads();
    const int64_t c = t.first_leaf + li;
    for (int i = threadIdx.x; i < K * kRC; i += blockDim.x) {
        const int al = i / kRC, rr = i % kRC;
        if (r0 + rr >= R) continue;
        T acc = 0;
        for (int64_t j = 0; j < n; ++j) acc += sU[j * K + al] * sX[j * kRC + rr];
        xh[(((int64_t)f * t.ncl + c) * K + al) * R + r0 + rr] = acc;
    }
}

// one level of the upsweep: parent coefficients from both children
template <int D, int P, typename T>
FPDE_KERNEL void k_bup_level(H2Tree t, int64_t c0, int64_t nlev, int F, int R, const T* E, T* xh) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)F * nlev * K * R) return;
    const int r = (int)(i % R);
    const int al = (int)((i / R) % K);
    const int64_t cl = (i / ((int64_t)R * K)) % nlev;
    const int f = (int)(i / ((int64_t)R * K * nlev));
    const int64_t c = c0 + cl, ch1 = 2 * c + 1, ch2 = 2 * c + 2;
    const T* xf = xh + (int64_t)f * t.ncl * K * R;
    xh[(((int64_t)f * t.ncl + c) * K + al) * R + r] =
        up_t<D, P, T>(E + ch1 * EP, E + ch2 * EP, xf + ch1 * K * R + r, xf + ch2 * K * R + r, al, R);
}

// one level of the downsweep: children += E_c parent
template <int D, int P, typename T>
FPDE_KERNEL void k_bdown_level(H2Tree t, int64_t c0, int64_t nlev, int F, int R, const T* E, T* yh) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)F * nlev * K * R) return;
    const int r = (int)(i % R);
    const int be = (int)((i / R) % K);
    const int64_t cl = (i / ((int64_t)R * K)) % nlev;
    const int f = (int)(i / ((int64_t)R * K * nlev));
    const int64_t c = c0 + cl, par = (c - 1) / 2;
    T* yf = yh + (int64_t)f * t.ncl * K * R;
    yf[(c * K + be) * R + r] += down_t<D, P, T>(E + c * EP, yf + par * K * R + r, be, R);
}

// Y^_S[alpha][r] = sum_{e in far(S)} sum_beta S_e[alpha][beta] X^_src(e)[beta][r],
// St[f][e][beta][alpha] = S_e[alpha][beta].  One block (two waves, 32 rhs each) per
// (target cluster, rhs chunk, field); S_e and X^_src(e) are staged in LDS per pair.
// K <= 32: alpha and beta are padded to 32 with zeros.
template <typename T>
__global__ __launch_bounds__(128) void k_bcoupling(H2Tree t, int F, int R, const T* St, const T* xh, T* yh) {
    constexpr int KP = 32, SS = KP + 1, XS = kRC + 1;
    __shared__ T sS[KP * SS];    // [beta][alpha]
    __shared__ T sX[KP * XS];    // [beta][r]
    const int K = t.k;
    const int64_t nrc = (R + kRC - 1) / kRC;
    const int64_t S = blockIdx.x / nrc;
    const int r0 = (int)(blockIdx.x % nrc) * kRC;
    const int f = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t nfar = t.far_ptr[t.ncl];
    bf32x16 c32 = {0};
    bf64x4 c64[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
    for (int64_t e = t.far_ptr[S]; e < t.far_ptr[S + 1]; ++e) {
        const int64_t src = t.far_src[e];
        const T* Se = St + ((int64_t)f * nfar + e) * K * K;
        const T* Xe = xh + (((int64_t)f * t.ncl + src) * K) * R;
        __syncthreads();
        for (int i = tid; i < KP * KP; i += blockDim.x) {
            const int be = i / KP, al = i % KP;
            sS[be * SS + al] = (be < K && al < K) ? Se[be * K + al] : T(0);
        }
        for (int i = tid; i < KP * kRC; i += blockDim.x) {
            const int be = i / kRC, rr = i % kRC;
            sX[be * XS + rr] = (be < K && r0 + rr < R) ? Xe[(int64_t)be * R + r0 + rr] : T(0);
        }
        __syncthreads();
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int k = 0; k < KP; k += 2) {
                const float av = sS[(k + (lane >> 5)) * SS + (lane & 31)];
                const float bv = sX[(k + (lane >> 5)) * XS + wv * 32 + (lane & 31)];
                c32 = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, c32, 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int k = 0; k < KP; k += 4) {
                double av[2], bv[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    av[i] = sS[(k + (lane >> 4)) * SS + 16 * i + (lane & 15)];
                    bv[i] = sX[(k + (lane >> 4)) * XS + wv * 32 + 16 * i + (lane & 15)];
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        c64[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], c64[i][j], 0, 0, 0);
            }
        }
    }
    T* Yo = yh + (((int64_t)f * t.ncl + S) * K) * R;
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int al = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const int r = r0 + wv * 32 + (lane & 31);
            if (al < K && r < R) Yo[(int64_t)al * R + r] = c32[v];
        }
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int al = 16 * i + (lane >> 4) + 4 * v;
                    const int r = r0 + wv * 32 + 16 * j + (lane & 15);
                    if (al < K && r < R) Yo[(int64_t)al * R + r] = c64[i][j][v];
                }
    }
}

// y[perm[row]][r] += sum_alpha U[row][alpha] Y^_leaf[alpha][r]; one block per (leaf, rhs chunk, field)
template <typename T>
__global__ __launch_bounds__(256) void k_bout_leaf(ApplyPlan a, H2Tree t, int F, int R, const T* U, const T* yh,
                                                   int dtype, void* y) {
    extern __shared__ __align__(16) unsigned char sraw[];
    const int K = t.k;
    const int64_t nrc = (R + kRC - 1) / kRC;
    const int64_t li = blockIdx.x / nrc;
    const int r0 = (int)(blockIdx.x % nrc) * kRC;
    const int f = blockIdx.y;
    const int64_t lb = a.leaf_beg[li], n = a.leaf_beg[li + 1] - lb;
    const int64_t c = t.first_leaf + li;
    T* sU = (T*)sraw;          // [n][K]
    T* sY = sU + n * K;        // [K][kRC]
    for (int64_t i = threadIdx.x; i < n * K; i += blockDim.x) sU[i] = U[lb * K + i];
    for (int i = threadIdx.x; i < K * kRC; i += blockDim.x) {
        const int al = i / kRC, rr = i % kRC;
        sY[i] = r0 + rr < R ? yh[(((int64_t)f * t.ncl + c) * K + al) * R + r0 + rr] : T(0);
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n * kRC; i += blockDim.x) {
        const int64_t j = i / kRC;
        const int rr = (int)(i % kRC);
        if (r0 + rr >= R) continue;
        T acc = 0;
        for (int al = 0; al < K; ++al) acc += sU[j * K + al] * sY[al * kRC + rr];
        const int64_t dst = ((int64_t)f * a.N + a.perm[lb + j]) * R + r0 + rr;
        if (dtype == 0) ((double*)y)[dst] += (double)acc;
        else ((float*)y)[dst] = (float)((double)((float*)y)[dst] + (double)acc);
    }
}

namespace {

template <typename T>
struct Batched {
    template <int D, int P>
    static void up(const H2Tree& t, int F, int R, const T* E, T* xh, hipStream_t st) {
        for (int lev = t.L - 1; lev >= 0; --lev) {
            const int64_t c0 = (int64_t(1) << lev) - 1, n = int64_t(1) << lev;
            hipLaunchKernelGGL((k_bup_level<D, P, T>), dim3(grid1((int64_t)F * n * t.k * R)), dim3(256), 0, st, t, c0,
                               n, F, R, E, xh);
        }
    }
    template <int D, int P>
    static void down(const H2Tree& t, int F, int R, const T* E, T* yh, hipStream_t st) {
        for (int lev = 1; lev <= t.L; ++lev) {
            const int64_t c0 = (int64_t(1) << lev) - 1, n = int64_t(1) << lev;
            hipLaunchKernelGGL((k_bdown_level<D, P, T>), dim3(grid1((int64_t)F * n * t.k * R)), dim3(256), 0, st, t,
                               c0, n, F, R, E, yh);
        }
    }
};

template <typename T>
hipError_t far_batched_t(const ApplyPlan& a, const H2Tree& t, int F, int R, const OpData<T>& od, int dtype,
                         const void* x, T* xh, T* yh, hipStream_t st) {
    const int64_t nrc = (R + kRC - 1) / kRC;
    const size_t lds_up = sizeof(T) * (size_t)(a.cap * t.k + a.cap * kRC);
    hipLaunchKernelGGL(k_bup_leaf<T>, dim3((unsigned)(a.nleaf * nrc), F), dim3(256), lds_up, st, a, t, F, R, od.U,
                       dtype, x, xh);
    FPDE_DISPATCH_DP(t.dim, t.p, Batched<T>::template up, t, F, R, od.E, xh, st);
    hipLaunchKernelGGL(k_bcoupling<T>, dim3((unsigned)(t.ncl * nrc), F), dim3(128), 0, st, t, F, R, od.St, xh, yh);
    FPDE_DISPATCH_DP(t.dim, t.p, Batched<T>::template down, t, F, R, od.E, yh, st);
    return hipGetLastError();
}

template <typename T>
hipError_t far_out_batched_t(const ApplyPlan& a, const H2Tree& t, int F, int R, const T* U, const T* yh, int dtype,
                             void* y, hipStream_t st) {
    const int64_t nrc = (R + kRC - 1) / kRC;
    const size_t lds = sizeof(T) * (size_t)(a.cap * t.k + t.k * kRC);
    hipLaunchKernelGGL(k_bout_leaf<T>, dim3((unsigned)(a.nleaf * nrc), F), dim3(256), lds, st, a, t, F, R, U, yh,
                       dtype, y);
    return hipGetLastError();
}

template <typename T>
hipError_t apply_batched_t(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, int parts, int F, int R,
                           const double* csr_val, const OpData<T>& od, T* xh, T* yh, int dtype, const void* x, void* y,
                           hipStream_t st, hipStream_t side, hipEvent_t fork, hipEvent_t join, hipEvent_t* ev) {
    const bool far = (parts & 8) != 0;
    if (ev) hipEventRecord(ev[0], st);
    hipStream_t fs = st;
    if (far && side != st) {
        hipEventRecord(fork, st);
        hipStreamWaitEvent(side, fork, 0);
        fs = side;
    }
    hipError_t e = hipSuccess;
    if (far && (e = far_batched_t<T>(a, t, F, R, od, dtype, x, xh, yh, fs)) != hipSuccess) return e;
    if (ev) hipEventRecord(ev[1], fs);
    e = launch_near_mm(a, pp, od.panel, (parts & 4) != 0, csr_val, F, R, dtype, x, y, st, ev ? ev[2] : nullptr,
                       ev ? ev[3] : nullptr);
    if (e != hipSuccess) return e;
    if (far) {
        if (fs != st) {
            hipEventRecord(join, fs);
            hipStreamWaitEvent(st, join, 0);
        }
        if ((e = far_out_batched_t<T>(a, t, F, R, od.U, yh, dtype, y, st)) != hipSuccess) return e;
    }
    if (ev) hipEventRecord(ev[4], st);
    return hipGetLastError();
}

}  // namespace

bool batched_fits(const H2Tree& t, int64_t cap, int prec) {
    const size_t es = prec == 0 ? 8 : 4;
    const size_t lds = es * (size_t)(cap * t.k + cap * kRC);
    return t.k <= 32 && lds <= 64 * 1024;
}

hipError_t launch_apply_batched(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, int parts, int F, int R,
                                const double* csr_val, const OpData<double>& od, double* xh, double* yh, int dtype,
                                const void* x, void* y, hipStream_t st, hipStream_t side, hipEvent_t fork,
                                hipEvent_t join, hipEvent_t* ev) {
    return apply_batched_t<double>(a, t, pp, parts, F, R, csr_val, od, xh, yh, dtype, x, y, st, side, fork, join, ev);
}

hipError_t launch_apply_batched(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, int parts, int F, int R,
                                const double* csr_val, const OpData<float>& od, float* xh, float* yh, int dtype,
                                const void* x, void* y, hipStream_t st, hipStream_t side, hipEvent_t fork,
                                hipEvent_t join, hipEvent_t* ev) {
    return apply_batched_t<float>(a, t, pp, parts, F, R, csr_val, od, xh, yh, dtype, x, y, st, side, fork, join, ev);
}

}  // namespace fpde
