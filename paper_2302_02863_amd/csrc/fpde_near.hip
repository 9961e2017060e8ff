// Near field of the apply: dense near leaf blocks of K~ packed per target leaf
// into row-major panels (FP64, and additionally FP32 for a mixed-precision
// operator), and the MFMA near-field kernel for several right-hand sides.  The
// one-vector near rows run inside the fused near/upsweep launch of the apply.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_device.h"

namespace fpde {

// Repack the near blocks of each target leaf into one row-major panel
// panel[f][poff[li] + it*pstride[li] + col], columns = concatenated source leaves.
FPDE_KERNEL void k_pack_panels(int64_t nleaf, int64_t cap, int64_t npairs, const int64_t* near_ptr,
                               const int64_t* near_src, const int64_t* leaf_beg, const int64_t* pcol_off,
                               const int64_t* poff, const int64_t* pstride, const int64_t* pcols_ptr, const double* nb,
                               int F, double* panel) {
    // one block per (leaf, field); threads stride over (row, column)
    const int64_t li = blockIdx.x;
    const int f = blockIdx.y;
    const int64_t nt = leaf_beg[li + 1] - leaf_beg[li];
    const int64_t ps = pstride[li];
    for (int64_t e = near_ptr[li]; e < near_ptr[li + 1]; ++e) {
        const int64_t ls_ = near_src[e];
        const int64_t ns = leaf_beg[ls_ + 1] - leaf_beg[ls_];
        const int64_t co = pcol_off[e];
        const double* blk = nb + ((int64_t)f * npairs + e) * cap * cap;
        for (int64_t i = threadIdx.x; i < cap * ns; i += blockDim.x) {
            const int64_t it = i / ns, j = i % ns;
            panel[(int64_t)f * poff[nleaf] + poff[li] + it * ps + co + j] = it < nt ? blk[it * cap + j] : 0.0;
        }
    }
    // zero the alignment padding of each row
    const int64_t ncols = pcols_ptr[li + 1] - pcols_ptr[li];
    for (int64_t i = threadIdx.x; i < cap * (ps - ncols); i += blockDim.x) {
        const int64_t it = i / (ps - ncols), j = ncols + i % (ps - ncols);
        panel[(int64_t)f * poff[nleaf] + poff[li] + it * ps + j] = 0.0;
    }
}

hipError_t launch_pack_panels(int64_t nleaf, int64_t cap, int64_t npairs, const int64_t* near_ptr,
                              const int64_t* near_src, const int64_t* leaf_beg, const int64_t* pcol_off,
                              const int64_t* poff, const int64_t* pstride, const int64_t* pcols_ptr, const double* nb,
                              int F, double* panel, hipStream_t st) {
    hipLaunchKernelGGL(k_pack_panels, dim3((unsigned)nleaf, F), dim3(256), 0, st, nleaf, cap, npairs, near_ptr, near_src,
                       leaf_beg, pcol_off, poff, pstride, pcols_ptr, nb, F, panel);
    return hipGetLastError();
}

// ------------------------------------------------------------ several right-hand sides: MFMA panels
//
// Y[rows, r0:r0+64] = Panel[rows, :] X[cols, r0:r0+64] + (B+M)[rows, :] X, one
// block per (leaf, 64-row tile, 64-column tile of right-hand sides, field).
// The panel times the gathered rows of X is a dense GEMM of 64 x 64 x
// pstride; four waves each own a 32 x 32 quarter of the tile:
//   FP32 operator data: v_mfma_f32_32x32x2f32 (lane l supplies A[l%32][l/32],
//     B[l/32][l%32]; accumulator v holds C[8(v/4) + 4(l/32) + v%4][l%32]);
//   FP64: 2 x 2 tiles of v_mfma_f64_16x16x4f64 (A[l%16][l/16], B[l/16][l%16];
//     accumulator v holds C[l/16 + 4v][l%16]).
// Chunks of 32 panel columns and the matching 32 rows of X are staged in LDS.
// The tile is then written to LDS and each thread adds the CSR row of B + M
// (FP64) for one right-hand side and writes y.
typedef float fpde_f32x16 __attribute__((ext_vector_type(16)));
typedef double fpde_f64x4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int kMT = 64, kNT = 64, kKC = 32;
constexpr int kApS = kKC + 1;   // LDS row strides (padding against bank conflicts)
constexpr int kBxS = kNT + 1;
constexpr int kCS = kNT + 1;

template <typename T>
__device__ __forceinline__ T ldt(const void* x, int64_t i, int dtype) {
    return dtype == 0 ? (T)((const double*)x)[i] : (T)((const float*)x)[i];
}
}  // namespace

template <typename T>
__global__ __launch_bounds__(256) void k_near_mm(ApplyPlan a, PanelPlan pp, const T* panel, int use_near,
                                                 const double* csr_val, int F, int R, int dtype, const void* x,
                                                 void* y) {
    extern __shared__ __align__(16) unsigned char sraw[];
    T* Ap = (T*)sraw;                       // [kMT][kApS]
    T* Bx = Ap + kMT * kApS;                // [kKC][kBxS]
    T* Cs = Ap;                             // [kMT][kCS] after the GEMM
    const int f = blockIdx.y;
    const int64_t nrt = (a.cap + kMT - 1) / kMT, nct = (R + kNT - 1) / kNT;
    const int64_t li = blockIdx.x / (nrt * nct);
    const int64_t rem = blockIdx.x % (nrt * nct);
    const int64_t row0 = (rem / nct) * kMT;   // first panel row of the tile
    const int r0 = (int)(rem % nct) * kNT;    // first right-hand side
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;   // the wave's quarter
    const int64_t lb = a.leaf_beg[li], nt = a.leaf_beg[li + 1] - lb;
    const int64_t xo = (int64_t)f * a.N * R;
    fpde_f32x16 c32 = {0};
    fpde_f64x4 c64[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
    if (use_near) {
        const int64_t ps = pp.pstride[li];
        const int64_t cb = pp.pcols_ptr[li], ncols = pp.pcols_ptr[li + 1] - cb;
        const T* pl = panel + (int64_t)f * pp.poff[a.nleaf] + pp.poff[li];
        // this thread's share of a chunk: panel row tid/4, columns (tid%4)*8..+8;
        // X row for column tid/8, right-hand sides (tid%8)*8..+8
        const int pr_ = tid >> 2, pc_ = (tid & 3) * 8;
        const int xk_ = tid >> 3, xr_ = (tid & 7) * 8;
        const int64_t prow = row0 + pr_;
        T pa[8], xa[8];
        auto fetch = [&](int64_t k0) {   // global -> registers (next chunk, in flight during the MFMAs)
            const int64_t col = k0 + pc_;
            if (prow < a.cap && col + 8 <= ps) {
#pragma unroll
                for (int j = 0; j < 8; ++j) pa[j] = pl[prow * ps + col + j];
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) pa[j] = (prow < a.cap && col + j < ps) ? pl[prow * ps + col + j] : T(0);
            }
            const int64_t xc = k0 + xk_;
            const int64_t dof = xc < ncols ? pp.pcols[cb + xc] : -1;
            const int64_t xi = xo + dof * R + r0 + xr_;
#pragma unroll
            for (int j = 0; j < 8; ++j) xa[j] = (dof >= 0 && r0 + xr_ + j < R) ? ldt<T>(x, xi + j, dtype) : T(0);
        };
        fetch(0);
        for (int64_t k0 = 0; k0 < ps; k0 += kKC) {
            __syncthreads();   // the previous chunk's MFMAs are done with the LDS tiles
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                Ap[pr_ * kApS + pc_ + j] = pa[j];
                Bx[xk_ * kBxS + xr_ + j] = xa[j];
            }
            __syncthreads();
            if (k0 + kKC < ps) fetch(k0 + kKC);
            if constexpr (sizeof(T) == 4) {
#pragma unroll
                for (int k = 0; k < kKC; k += 2) {
                    const float av = Ap[(wr + (lane & 31)) * kApS + k + (lane >> 5)];
                    const float bv = Bx[(k + (lane >> 5)) * kBxS + wc + (lane & 31)];
                    c32 = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, c32, 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int k = 0; k < kKC; k += 4) {
                    double av[2], bv[2];
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        av[i] = Ap[(wr + 16 * i + (lane & 15)) * kApS + k + (lane >> 4)];
                        bv[i] = Bx[(k + (lane >> 4)) * kBxS + wc + 16 * i + (lane & 15)];
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
    __syncthreads();
    // the tile to LDS
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int v = 0; v < 16; ++v)
            Cs[(wr + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)) * kCS + wc + (lane & 31)] = c32[v];
    } else {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Cs[(wr + 16 * i + (lane >> 4) + 4 * v) * kCS + wc + 16 * j + (lane & 15)] = c64[i][j][v];
    }
    __syncthreads();
    // CSR rows of B + M and the output: thread -> one rhs, rows strided by 4 (a wave
    // shares each row, so the column and value loads are uniform across it)
    const int rc = tid & 63;
    const int r = r0 + rc;
    if (r >= R) return;
    for (int rr = tid >> 6; rr < kMT; rr += 4) {
        const int64_t it = row0 + rr;
        if (it >= nt) break;
        const int64_t row = lb + it;
        double acc = (double)Cs[rr * kCS + rc];
        if (csr_val) {
            const double* v = csr_val + (int64_t)f * a.nnz;
            const int64_t e1 = a.csr_ptr[row + 1];
            int64_t e = a.csr_ptr[row];
            double s1 = 0.0, s2 = 0.0, s3 = 0.0;
            for (; e + 4 <= e1; e += 4) {   // four independent gathers in flight
                acc += v[e] * ldx(x, xo + (int64_t)pp.csr_col_dof[e] * R + r, dtype);
                s1 += v[e + 1] * ldx(x, xo + (int64_t)pp.csr_col_dof[e + 1] * R + r, dtype);
                s2 += v[e + 2] * ldx(x, xo + (int64_t)pp.csr_col_dof[e + 2] * R + r, dtype);
                s3 += v[e + 3] * ldx(x, xo + (int64_t)pp.csr_col_dof[e + 3] * R + r, dtype);
            }
            for (; e < e1; ++e) acc += v[e] * ldx(x, xo + (int64_t)pp.csr_col_dof[e] * R + r, dtype);
            acc += (s1 + s2) + s3;
        }
        const int64_t dst = xo + (int64_t)a.perm[row] * R + r;
        if (dtype == 0) ((double*)y)[dst] = acc;
        else ((float*)y)[dst] = (float)acc;
    }
}

template <typename T>
static hipError_t near_mm_t(const ApplyPlan& a, const PanelPlan& pp, const T* panel, int use_near,
                            const double* csr_val, int F, int R, int dtype, const void* x, void* y, hipStream_t st,
                            hipEvent_t e0, hipEvent_t e1) {
    const int64_t nrt = (a.cap + kMT - 1) / kMT, nct = (R + kNT - 1) / kNT;
    const size_t lds = sizeof(T) * (size_t)((kMT * kApS + kKC * kBxS) > kMT * kCS ? (kMT * kApS + kKC * kBxS)
                                                                                   : kMT * kCS);
    const dim3 grid((unsigned)(a.nleaf * nrt * nct), F);
    if (e0)
        hipExtLaunchKernelGGL(k_near_mm<T>, grid, dim3(256), lds, st, e0, e1, 0, a, pp, panel, use_near, csr_val, F, R,
                              dtype, x, y);
    else
        hipLaunchKernelGGL(k_near_mm<T>, grid, dim3(256), lds, st, a, pp, panel, use_near, csr_val, F, R, dtype, x, y);
    return hipGetLastError();
}

hipError_t launch_near_mm(const ApplyPlan& a, const PanelPlan& pp, const double* panel, int use_near,
                          const double* csr_val, int F, int R, int dtype, const void* x, void* y, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1) {
    return near_mm_t<double>(a, pp, panel, use_near, csr_val, F, R, dtype, x, y, st, e0, e1);
}

hipError_t launch_near_mm(const ApplyPlan& a, const PanelPlan& pp, const float* panel, int use_near,
                          const double* csr_val, int F, int R, int dtype, const void* x, void* y, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1) {
    return near_mm_t<float>(a, pp, panel, use_near, csr_val, F, R, dtype, x, y, st, e0, e1);
}

// FP32 copy of FP64 operator data (mixed precision)
FPDE_KERNEL void k_to_float(int64_t n, const double* src, float* dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

hipError_t launch_to_float(int64_t n, const double* src, float* dst, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_float, dim3(grid1(n)), dim3(256), 0, st, n, src, dst);
    return hipGetLastError();
}

}  // namespace fpde
