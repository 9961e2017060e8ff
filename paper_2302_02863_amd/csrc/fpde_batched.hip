// Far field of the apply for many right-hand sides (Sec. 5.3, nested bases),
// with the operator data in FP64 or FP32.  Coefficients are [F][cluster][K][R]
// (right-hand sides fastest).  Each stage is a batch of small dense products:
//   k_bup_leaf     X^_leaf = U_leaf^T X_leaf            (per leaf, 64 rhs)
//   k_blevel       X^_parent = sum_c E_c^T X^_c          (per level)
//   k_bcoupling    Y^_S = sum_{S' far S} S_(S,S') X^_S'  (MFMA, per target cluster)
//   k_blevel       Y^_c += E_c Y^_parent                 (per level)
// and the near kernel (fpde_near.hip) adds y_leaf += U_leaf Y^_leaf to its rows.
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

// X^_leaf[alpha][r] = sum_j U[j][alpha] x[perm[j]][r]: a (K <= 32) x 64 x n GEMM per
// (leaf, rhs chunk, field) on MFMA, two waves of 32 right-hand sides, leaf rows
// staged in LDS 32 at a time (alpha and the row count padded with zeros).
template <typename T>
__global__ __launch_bounds__(128) void k_bup_leaf(ApplyPlan a, H2Tree t, int F, int R, const T* U, int dtype,
                                                  const void* x, T* xh) {
    constexpr int JC = 32, US = 33, XS = kRC + 1;
    __shared__ T sU[JC * US];    // [row][alpha]
    __shared__ T sX[JC * XS];    // [row][r]
    const int K = t.k;
    const int64_t nrc = (R + kRC - 1) / kRC;
    const int64_t li = blockIdx.x / nrc;
    const int r0 = (int)(blockIdx.x % nrc) * kRC;
    const int f = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t lb = a.leaf_beg[li], n = a.leaf_beg[li + 1] - lb;
    bf32x16 c32 = {0};
    bf64x4 c64[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
    for (int64_t j0 = 0; j0 < n; j0 += JC) {
        // all of this thread's loads in flight before the first wait: U rows (alpha = tid % 32,
        // rows tid / 32 + 4m), the permutation, then x (rhs = tid % 64, rows tid / 64 + 2m)
        T uv[JC * 32 / 128], xv[JC * kRC / 128];
        int64_t pv[JC * kRC / 128];
#pragma unroll
        for (int m = 0; m < JC * 32 / 128; ++m) {
            const int j = (tid >> 5) + 4 * m, al = tid & 31;
            uv[m] = (j0 + j < n && al < K) ? U[(lb + j0 + j) * K + al] : T(0);
        }
#pragma unroll
        for (int m = 0; m < JC * kRC / 128; ++m) {
            const int j = (tid >> 6) + 2 * m;
            pv[m] = j0 + j < n ? a.perm[lb + j0 + j] : -1;
        }
#pragma unroll
        for (int m = 0; m < JC * kRC / 128; ++m) {
            const int rr = tid & 63;
            xv[m] = (pv[m] >= 0 && r0 + rr < R) ? (T)ldx(x, ((int64_t)f * a.N + pv[m]) * R + r0 + rr, dtype) : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < JC * 32 / 128; ++m) sU[((tid >> 5) + 4 * m) * US + (tid & 31)] = uv[m];
#pragma unroll
        for (int m = 0; m < JC * kRC / 128; ++m) sX[((tid >> 6) + 2 * m) * XS + (tid & 63)] = xv[m];
        __syncthreads();
        if constexpr (sizeof(T) == 4) {
#pragma unroll 8
            for (int k = 0; k < JC; k += 2) {
                const float av = sU[(k + (lane >> 5)) * US + (lane & 31)];
                const float bv = sX[(k + (lane >> 5)) * XS + wv * 32 + (lane & 31)];
                c32 = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, c32, 0, 0, 0);
            }
        } else {
#pragma unroll 4
            for (int k = 0; k < JC; k += 4) {
                double av[2], bv[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    av[i] = sU[(k + (lane >> 4)) * US + 16 * i + (lane & 15)];
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
    T* Xo = xh + (((int64_t)f * t.ncl + t.first_leaf + li) * K) * R;
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int al = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const int r = r0 + wv * 32 + (lane & 31);
            if (al < K && r < R) Xo[(int64_t)al * R + r] = c32[v];
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
                    if (al < K && r < R) Xo[(int64_t)al * R + r] = c64[i][j][v];
                }
    }
}

// One level of the nested transfers, per (parent cluster, rhs chunk, field), with the
// Kronecker transfer applied one dimension at a time in LDS:
//   up:   X^_p[a0 + P a1] = sum_c sum_b1 E_c1[b1][a1] sum_b0 E_c0[b0][a0] X^_c[b0 + P b1]
//   down: Y^_c[b0 + P b1] += sum_a1 E_c1[b1][a1] sum_a0 E_c0[b0][a0] Y^_p[a0 + P a1]
template <int D, int P, typename T, bool UP>
__global__ __launch_bounds__(256) void k_blevel(H2Tree t, int64_t c0, int F, int R, const T* E, T* xh) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    __shared__ T sE[2 * EP];
    __shared__ T sA[(UP ? 2 : 1) * K * kRC];   // up: both children; down: the parent
    __shared__ T sT[2 * K * kRC];   // after the first dimension
    const int64_t nrc = (R + kRC - 1) / kRC;
    const int64_t c = c0 + blockIdx.x / nrc;
    const int r0 = (int)(blockIdx.x % nrc) * kRC;
    const int f = blockIdx.y;
    const int tid = threadIdx.x;
    const int64_t ch[2] = {2 * c + 1, 2 * c + 2};
    T* xf = xh + (int64_t)f * t.ncl * K * R;
    constexpr int nin = UP ? 2 : 1, NE = (2 * EP + 255) / 256, NA = (nin * K * kRC + 255) / 256;
    T ve[NE], va[NA];
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        const int i = tid + 256 * m;
        ve[m] = i < 2 * EP ? E[ch[i / EP] * EP + i % EP] : T(0);
    }
#pragma unroll
    for (int m = 0; m < NA; ++m) {
        const int i = tid + 256 * m;
        const int s = i / (K * kRC), al = (i / kRC) % K, rr = i % kRC;
        const int64_t src = UP ? ch[s < 2 ? s : 1] : c;
        va[m] = (i < nin * K * kRC && r0 + rr < R) ? xf[(src * K + al) * R + r0 + rr] : T(0);
    }
    // down: the children's current coefficients, read now so that the final
    // read-modify-write costs no round trip after the sums
    constexpr int NO = UP ? 1 : (2 * K * kRC + 255) / 256;
    T vo[NO];
    if constexpr (!UP) {
#pragma unroll
        for (int m = 0; m < NO; ++m) {
            const int i = tid + 256 * m;
            const int s = i / (K * kRC), q = (i / kRC) % K, rr = i % kRC;
            vo[m] = (i < 2 * K * kRC && r0 + rr < R) ? xf[(ch[s < 2 ? s : 1] * K + q) * R + r0 + rr] : T(0);
        }
    }
#pragma unroll
    for (int m = 0; m < NE; ++m)
        if (tid + 256 * m < 2 * EP) sE[tid + 256 * m] = ve[m];
#pragma unroll
    for (int m = 0; m < NA; ++m)
        if (tid + 256 * m < nin * K * kRC) sA[tid + 256 * m] = va[m];
    __syncthreads();
    // first dimension (dim 0: index % P): sT[s][i0][i1][r], both children
    for (int i = tid; i < 2 * K * kRC; i += blockDim.x) {
        const int s = i / (K * kRC), q = (i / kRC) % K, rr = i % kRC;
        const int i0 = q % P, i1 = q / P;
        const T* Ed = sE + s * EP;   // dim-0 factor [b][a]
        const T* src = sA + (UP ? s : 0) * K * kRC;
        T acc = 0;
#pragma unroll
        for (int m = 0; m < P; ++m)   // up: sum_b0 E[b0][a0 = i0] X[b0 + P i1];  down: sum_a0 E[b0 = i0][a0] Y[a0 + P i1]
            acc += (UP ? Ed[m * P + i0] : Ed[i0 * P + m]) * src[(m + P * i1) * kRC + rr];
        sT[i] = acc;
    }
    __syncthreads();
    // second dimension (2D), then store
#pragma unroll
    for (int m = 0; m < (UP ? (K * kRC + 255) / 256 : NO); ++m) {
        const int i = tid + 256 * m;
        if (i >= (UP ? 1 : 2) * K * kRC) break;
        const int s = i / (K * kRC), q = (i / kRC) % K, rr = i % kRC;
        if (r0 + rr >= R) continue;
        const int i0 = q % P, i1 = q / P;
        T acc = 0;
        for (int s2 = 0; s2 < 2; ++s2) {
            if (!UP && s2 != s) continue;
            if (D == 1) {
                acc += sT[(s2 * K + q) * kRC + rr];
            } else {
                const T* Ed = sE + s2 * EP + P * P;   // dim-1 factor [b][a]
#pragma unroll
                for (int m = 0; m < P; ++m)
                    acc += (UP ? Ed[m * P + i1] : Ed[i1 * P + m]) * sT[(s2 * K + i0 + P * m) * kRC + rr];
            }
        }
        if constexpr (UP) xf[(c * K + q) * R + r0 + rr] = acc;
        else xf[(ch[s] * K + q) * R + r0 + rr] = vo[m] + acc;
    }
}

// One level of dense transfers (recompressed bases, K <= 32), per (parent cluster, rhs
// chunk, field), Ed[c][b][a] = E_c[b][a] (child index b, parent index a):
//   up:   X^_p[a] = sum_c sum_b E_c[b][a] X^_c[b]
//   down: Y^_c[b] += sum_a E_c[b][a] Y^_p[a]
template <typename T, bool UP>
__global__ __launch_bounds__(256) void k_blevel_dense(H2Tree t, int64_t c0, int F, int R, const T* Ed, T* xh) {
    constexpr int KP = 32, ES = KP + 1, XS = kRC + 1;
    __shared__ T sE[2 * KP * ES];
    __shared__ T sA[(UP ? 2 : 1) * KP * XS];   // up: both children; down: the parent
    const int K = t.k;
    const int64_t nrc = (R + kRC - 1) / kRC;
    const int64_t c = c0 + blockIdx.x / nrc;
    const int r0 = (int)(blockIdx.x % nrc) * kRC;
    const int f = blockIdx.y;
    const int tid = threadIdx.x;
    const int64_t ch[2] = {2 * c + 1, 2 * c + 2};
    T* xf = xh + (int64_t)f * t.ncl * K * R;
    for (int i = tid; i < 2 * K * K; i += 256) {
        const int s = i / (K * K), q = i % (K * K);
        sE[s * KP * ES + (q / K) * ES + q % K] = Ed[ch[s] * K * K + q];
    }
    constexpr int nin = UP ? 2 : 1;
    for (int i = tid; i < nin * K * kRC; i += 256) {
        const int s = i / (K * kRC), al = (i / kRC) % K, rr = i % kRC;
        const int64_t src = UP ? ch[s] : c;
        sA[s * KP * XS + al * XS + rr] = r0 + rr < R ? xf[(src * K + al) * R + r0 + rr] : T(0);
    }
    __syncthreads();
    if (UP) {
        for (int i = tid; i < K * kRC; i += 256) {
            const int a = i / kRC, rr = i % kRC;
            if (r0 + rr >= R) continue;
            T acc = 0;
            for (int s = 0; s < 2; ++s)
                for (int b = 0; b < K; ++b) acc += sE[s * KP * ES + b * ES + a] * sA[s * KP * XS + b * XS + rr];
            xf[(c * K + a) * R + r0 + rr] = acc;
        }
    } else {
        for (int i = tid; i < 2 * K * kRC; i += 256) {
            const int s = i / (K * kRC), b = (i / kRC) % K, rr = i % kRC;
            if (r0 + rr >= R) continue;
            T acc = 0;
            for (int a = 0; a < K; ++a) acc += sE[s * KP * ES + b * ES + a] * sA[a * XS + rr];
            xf[(ch[s] * K + b) * R + r0 + rr] += acc;
        }
    }
}

// Y^_S[alpha][r] = sum_{e in far(S)} sum_beta S_e[alpha][beta] X^_src(e)[beta][r],
// St[f][e][beta][alpha] = S_e[alpha][beta].  One block (two waves, 32 rhs each) per
// (target cluster, rhs chunk, field); S_e and X^_src(e) are staged in LDS per pair.
// K <= 32: alpha and beta are padded to 32 with zeros.
template <typename T>
__device__ __forceinline__ void bcoupling_body(const H2Tree& t, int F, int R, const T* St, const T* xh, T* yh) {
    constexpr int KP = 32, SS = KP + 1, XS = kRC + 1;
    // far pairs staged per iteration (two measured slower: registers halve the occupancy)
    constexpr int NP = 1;
    __shared__ T sS[NP][KP * SS];    // [beta][alpha]
    __shared__ T sX[NP][KP * XS];    // [beta][r]
    const int K = t.k;
    const int64_t nrc = (R + kRC - 1) / kRC;
    const int64_t lb = xcd_block((int64_t)blockIdx.y * gridDim.x + blockIdx.x, (int64_t)gridDim.x * gridDim.y);
    const int f = (int)(lb / gridDim.x);
    const int64_t S = (lb % gridDim.x) / nrc;
    const int r0 = (int)((lb % gridDim.x) % nrc) * kRC;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t nfar = t.far_ptr[t.ncl];
    bf32x16 c32 = {0};
    bf64x4 c64[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
    // operands of a pair: S_e (thread -> alpha = tid % 32, beta = tid / 32 + 4m) and
    // X^ of its source (rhs = tid % 64, beta = tid / 64 + 2m), fetched into registers
    // one stage ahead so that the loads overlap the MFMAs; a missing pair loads zeros
    constexpr int NS = KP * KP / 128, NX = KP * kRC / 128;
    T rs[NP][NS], rx[NP][NX];
    const int64_t e0 = t.far_ptr[S], e1 = t.far_ptr[S + 1];
    auto fetch = [&](int64_t eb) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int64_t e = eb + p;
            const bool ok = e < e1;
            const int64_t src = ok ? t.far_src[e] : 0;
            const T* Se = St + ((int64_t)f * nfar + (ok ? e : 0)) * K * K;
            const T* Xe = xh + (((int64_t)f * t.ncl + src) * K) * R;
#pragma unroll
            for (int m = 0; m < NS; ++m) {
                const int be = (tid >> 5) + 4 * m, al = tid & 31;
                rs[p][m] = (ok && be < K && al < K) ? Se[be * K + al] : T(0);
            }
#pragma unroll
            for (int m = 0; m < NX; ++m) {
                const int be = (tid >> 6) + 2 * m, rr = tid & 63;
                rx[p][m] = (ok && be < K && r0 + rr < R) ? Xe[(int64_t)be * R + r0 + rr] : T(0);
            }
        }
    };
    if (e0 < e1) fetch(e0);
    for (int64_t e = e0; e < e1; e += NP) {
        __syncthreads();
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int m = 0; m < NS; ++m) sS[p][((tid >> 5) + 4 * m) * SS + (tid & 31)] = rs[p][m];
#pragma unroll
            for (int m = 0; m < NX; ++m) sX[p][((tid >> 6) + 2 * m) * XS + (tid & 63)] = rx[p][m];
        }
        __syncthreads();
        if (e + NP < e1) fetch(e + NP);
        const int np = e1 - e < NP ? (int)(e1 - e) : NP;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (p >= np) break;   // block-uniform
            if constexpr (sizeof(T) == 4) {
#pragma unroll
                for (int k = 0; k < KP; k += 2) {   // beta past K is zero padding: skipped
                    if (k >= K) break;
                    const float av = sS[p][(k + (lane >> 5)) * SS + (lane & 31)];
                    const float bv = sX[p][(k + (lane >> 5)) * XS + wv * 32 + (lane & 31)];
                    c32 = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, c32, 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int k = 0; k < KP; k += 4) {
                    if (k >= K) break;
                    double av[2], bv[2];
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        av[i] = sS[p][(k + (lane >> 4)) * SS + 16 * i + (lane & 15)];
                        bv[i] = sX[p][(k + (lane >> 4)) * XS + wv * 32 + 16 * i + (lane & 15)];
                    }
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
                            c64[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], c64[i][j], 0, 0, 0);
                }
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

template <typename T>
__global__ __launch_bounds__(128) void k_bcoupling(H2Tree t, int F, int R, const T* St, const T* xh, T* yh) {
    bcoupling_body<T>(t, F, R, St, xh, yh);
}
// FP64: 200 VGPRs unconstrained (two waves per SIMD); held to three waves per SIMD
template <>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3))) void k_bcoupling<double>(
    H2Tree t, int F, int R, const double* St, const double* xh, double* yh) {
    bcoupling_body<double>(t, F, R, St, xh, yh);
}

namespace {

template <typename T>
struct Batched {
    template <int D, int P>
    static void up(const H2Tree& t, int F, int R, const T* E, T* xh, hipStream_t st) {
        const int64_t nrc = (R + kRC - 1) / kRC;
        for (int lev = t.L - 1; lev >= 0; --lev) {
            const int64_t c0 = (int64_t(1) << lev) - 1, n = int64_t(1) << lev;
            hipLaunchKernelGGL((k_blevel<D, P, T, true>), dim3((unsigned)(n * nrc), F), dim3(256), 0, st, t, c0, F, R,
                               E, xh);
        }
    }
    template <int D, int P>
    static void down(const H2Tree& t, int F, int R, const T* E, T* yh, hipStream_t st) {
        const int64_t nrc = (R + kRC - 1) / kRC;
        for (int lev = 0; lev < t.L; ++lev) {   // parents at lev -> children at lev + 1
            const int64_t c0 = (int64_t(1) << lev) - 1, n = int64_t(1) << lev;
            hipLaunchKernelGGL((k_blevel<D, P, T, false>), dim3((unsigned)(n * nrc), F), dim3(256), 0, st, t, c0, F,
                               R, E, yh);
        }
    }
};

template <typename T>
void dense_levels(const H2Tree& t, int F, int R, const T* Ed, T* xh, bool up, hipStream_t st) {
    const int64_t nrc = (R + kRC - 1) / kRC;
    for (int i = 0; i < t.L; ++i) {
        const int lev = up ? t.L - 1 - i : i;   // parents at lev
        const int64_t c0 = (int64_t(1) << lev) - 1, n = int64_t(1) << lev;
        if (up)
            hipLaunchKernelGGL((k_blevel_dense<T, true>), dim3((unsigned)(n * nrc), F), dim3(256), 0, st, t, c0, F, R,
                               Ed, xh);
        else
            hipLaunchKernelGGL((k_blevel_dense<T, false>), dim3((unsigned)(n * nrc), F), dim3(256), 0, st, t, c0, F,
                               R, Ed, xh);
    }
}

template <typename T>
hipError_t far_batched_t(const ApplyPlan& a, const H2Tree& t, int F, int R, const OpData<T>& od, int dtype,
                         const void* x, T* xh, T* yh, hipStream_t st) {
    const int64_t nrc = (R + kRC - 1) / kRC;
    hipLaunchKernelGGL(k_bup_leaf<T>, dim3((unsigned)(a.nleaf * nrc), F), dim3(128), 0, st, a, t, F, R, od.U, dtype, x,
                       xh);
    if (od.Ed) dense_levels<T>(t, F, R, od.Ed, xh, true, st);
    else FPDE_DISPATCH_DP(t.dim, t.p, Batched<T>::template up, t, F, R, od.E, xh, st);
    hipLaunchKernelGGL(k_bcoupling<T>, dim3((unsigned)(t.ncl * nrc), F), dim3(128), 0, st, t, F, R, od.St, xh, yh);
    if (od.Ed) dense_levels<T>(t, F, R, od.Ed, yh, false, st);
    else FPDE_DISPATCH_DP(t.dim, t.p, Batched<T>::template down, t, F, R, od.E, yh, st);
    return hipGetLastError();
}

template <typename T>
hipError_t apply_batched_t(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, int parts, int F, int R,
                           const double* csr_val, const OpData<T>& od, T* xh, T* yh, int dtype, const void* x, void* y,
                           hipStream_t st, hipEvent_t* ev) {
    // The far chain first, then the near kernel, which adds U_leaf Y^_leaf to its rows:
    // run beside the near kernel on a second stream, the chain's small dependent launches
    // wait behind the near kernel's blocks and end up on the critical path.
    const bool far = (parts & 8) != 0;
    if (ev) (void)hipEventRecord(ev[0], st);
    hipError_t e = hipSuccess;
    if (far && (e = far_batched_t<T>(a, t, F, R, od, dtype, x, xh, yh, st)) != hipSuccess) return e;
    if (ev) (void)hipEventRecord(ev[1], st);
    MmFar<T> fo{};
    if (far) fo = MmFar<T>{yh, od.Upad, t.ncl, t.first_leaf, t.k};   // t.k: the (recompressed) rank
    e = launch_near_mm(a, pp, od.panel, (parts & 4) != 0, csr_val, F, R, dtype, x, y, st, ev ? ev[2] : nullptr,
                       ev ? ev[3] : nullptr, fo);
    if (e != hipSuccess) return e;
    if (ev) (void)hipEventRecord(ev[4], st);
    return hipGetLastError();
}

}  // namespace

bool batched_fits(const H2Tree& t, int64_t cap, int prec) {
    (void)cap;
    (void)prec;
    return t.k <= 32;
}

hipError_t launch_apply_batched(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, int parts, int F, int R,
                                const double* csr_val, const OpData<double>& od, double* xh, double* yh, int dtype,
                                const void* x, void* y, hipStream_t st, hipEvent_t* ev) {
    return apply_batched_t<double>(a, t, pp, parts, F, R, csr_val, od, xh, yh, dtype, x, y, st, ev);
}

hipError_t launch_apply_batched(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, int parts, int F, int R,
                                const double* csr_val, const OpData<float>& od, float* xh, float* yh, int dtype,
                                const void* x, void* y, hipStream_t st, hipEvent_t* ev) {
    return apply_batched_t<float>(a, t, pp, parts, F, R, csr_val, od, xh, yh, dtype, x, y, st, ev);
}

}  // namespace fpde
