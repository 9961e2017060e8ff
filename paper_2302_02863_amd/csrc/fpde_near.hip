// Near field of the apply: dense near leaf blocks of K~ packed per target leaf
// into row-major panels, streamed together with the CSR rows of B + M.
// This is the HBM-bound kernel of the apply (one right-hand side).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_internal.h"

#define FPDE_KERNEL __global__ __launch_bounds__(256)

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

// y[f][perm[row]] = (B+M)_row . xt + panel_row . xt[cols]; one block per (leaf, 16-row block),
// one right-hand side.  The leaf's panel columns of x are staged in LDS once per block.
FPDE_KERNEL void k_near_panel(ApplyPlan a, const int64_t* poff, const int64_t* pstride, const int32_t* pcols,
                              const int64_t* pcols_ptr, const double* panel, int use_near, const double* csr_val, int F,
                              const double* xt, int dtype, void* y) {
    extern __shared__ double xs[];
    const int f = blockIdx.y;
    const int64_t nrb = (a.cap + 15) / 16;
    const int64_t li = blockIdx.x / nrb;
    const int rb = (int)(blockIdx.x % nrb);
    const double* xf = xt + (int64_t)f * a.N;
    const int64_t c0 = pcols_ptr[li], ncols = pcols_ptr[li + 1] - c0;
    if (use_near)   // padding columns of the row stride hold 0 in the panel and in xs
        for (int64_t c = threadIdx.x; c < pstride[li]; c += blockDim.x) xs[c] = c < ncols ? xf[pcols[c0 + c]] : 0.0;
    __syncthreads();
    const int g = threadIdx.x & 15;
    const int64_t it = (int64_t)rb * 16 + (threadIdx.x >> 4);
    const int64_t lb = a.leaf_beg[li], nt = a.leaf_beg[li + 1] - lb;
    if (it >= nt) return;
    const int64_t row = lb + it;
    double acc = 0.0;
    if (csr_val) {
        const double* v = csr_val + (int64_t)f * a.nnz;
        for (int64_t e = a.csr_ptr[row] + g; e < a.csr_ptr[row + 1]; e += 16) acc += v[e] * xf[a.csr_col[e]];
    }
    if (use_near) {
        const int64_t ps = pstride[li];
        const double* pr = panel + (int64_t)f * poff[a.nleaf] + poff[li] + it * ps;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int64_t c = 2 * g;
        // 4 x 16-byte loads per lane in flight
        for (; c + 96 + 2 <= ps; c += 128) {
            const double2 p0 = *(const double2*)(pr + c);
            const double2 p1 = *(const double2*)(pr + c + 32);
            const double2 p2 = *(const double2*)(pr + c + 64);
            const double2 p3 = *(const double2*)(pr + c + 96);
            a0 += p0.x * xs[c] + p0.y * xs[c + 1];
            a1 += p1.x * xs[c + 32] + p1.y * xs[c + 33];
            a2 += p2.x * xs[c + 64] + p2.y * xs[c + 65];
            a3 += p3.x * xs[c + 96] + p3.y * xs[c + 97];
        }
        for (; c + 2 <= ps; c += 32) {
            const double2 p0 = *(const double2*)(pr + c);
            a0 += p0.x * xs[c] + p0.y * xs[c + 1];
        }
        acc += (a0 + a1) + (a2 + a3);
    }
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
    if (g == 0) {
        const int64_t dst = (int64_t)f * a.N + a.perm[row];
        if (dtype == 0) ((double*)y)[dst] = acc;
        else ((float*)y)[dst] = (float)acc;
    }
}

hipError_t launch_near_panel(const ApplyPlan& a, const int64_t* poff, const int64_t* pstride, const int32_t* pcols,
                             const int64_t* pcols_ptr, int64_t max_stride, const double* panel, int use_near,
                             const double* csr_val, int F, const double* xt, int dtype, void* y, hipStream_t st,
                             hipEvent_t e0, hipEvent_t e1) {
    const int64_t nrb = (a.cap + 15) / 16;
    const size_t lds = sizeof(double) * (max_stride > 0 ? max_stride : 1);
    if (e0)
        hipExtLaunchKernelGGL(k_near_panel, dim3((unsigned)(a.nleaf * nrb), F), dim3(256), lds, st, e0, e1, 0, a, poff,
                              pstride, pcols, pcols_ptr, panel, use_near, csr_val, F, xt, dtype, y);
    else
        hipLaunchKernelGGL(k_near_panel, dim3((unsigned)(a.nleaf * nrb), F), dim3(256), lds, st, a, poff, pstride, pcols,
                           pcols_ptr, panel, use_near, csr_val, F, xt, dtype, y);
    return hipGetLastError();
}

}  // namespace fpde
