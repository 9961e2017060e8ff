// Operator apply for several right-hand sides per field (R > 1): main stream:
// near panels as MFMA GEMMs with the CSR rows of B + M (k_near_mm, fpde_near.hip,
// FP64 or FP32 operator data); side stream: the far field in FP64 (subtree
// upsweep, top levels, coupling products per far pair, or per-level sweeps
// when R is too wide for LDS); join: the far output added per leaf.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_device.h"

namespace fpde {

// levels ls-1 .. 0 with every transfer of levels 1..ls resident in LDS; one block per field
template <int D, int P>
__global__ __launch_bounds__(1024) void k_up_top_m(H2Tree t, int ls, int F, int R, double* xh) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    extern __shared__ double sm[];
    const int f = blockIdx.x;
    const int64_t ntop = (int64_t(2) << ls) - 1;
    const int64_t KRr = (int64_t)K * R;
    double* sx = sm;                     // [ntop][K][R]
    double* sE = sx + ntop * KRr;        // [ntop][EP] (index = heap id)
    for (int64_t i = threadIdx.x + ((int64_t(1) << ls) - 1) * KRr; i < ntop * KRr; i += blockDim.x)
        sx[i] = xh[(int64_t)f * t.ncl * KRr + i];
    for (int64_t i = threadIdx.x + EP; i < ntop * EP; i += blockDim.x) sE[i] = t.E[i];
    __syncthreads();
    for (int lev = ls - 1; lev >= 0; --lev) {
        const int64_t c0 = (int64_t(1) << lev) - 1, w = int64_t(1) << lev;
        for (int64_t i = threadIdx.x; i < w * KRr; i += blockDim.x) {
            const int64_t cc = c0 + i / KRr;
            const int al = (int)((i / R) % K), r = (int)(i % R);
            const int64_t ch1 = 2 * cc + 1, ch2 = 2 * cc + 2;
            const double v = up_t<D, P>(sE + ch1 * EP, sE + ch2 * EP, sx + ch1 * KRr + r, sx + ch2 * KRr + r, al, R);
            sx[cc * KRr + (int64_t)al * R + r] = v;
            xh[((int64_t)f * t.ncl + cc) * KRr + (int64_t)al * R + r] = v;
        }
        __syncthreads();
    }
}

template <int D, int P>
FPDE_KERNEL void k_coupling_pairs_m(H2Tree t, int64_t nfar, int F, int R, const double* St, const double* xh,
                                    double* tmp) {
    constexpr int K = KR<D, P>::K;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)K * R;
    if (i >= (int64_t)F * nfar * per) return;
    const int f = (int)(i / (nfar * per));
    int64_t rem = i - (int64_t)f * nfar * per;
    const int64_t e = rem / per;
    rem %= per;
    const int al = (int)(rem / R), r = (int)(rem % R);
    const double* S = St + ((int64_t)f * nfar + e) * K * K + al;
    const double* xs = xh + (((int64_t)f * t.ncl + t.far_src[e]) * K) * R + r;
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < K; ++b) acc += S[b * K] * xs[(int64_t)b * R];
    tmp[i] = acc;
}

// LDS needed by the v2 far chain; false when the per-level path must be used
bool multi_fits(const H2Tree& t, int ls, int R) {
    const int64_t K = t.k, EP = (int64_t)t.dim * t.p * t.p;
    const int64_t ncs = (int64_t(2) << (t.L - ls)) - 1, ntop = (int64_t(2) << ls) - 1;
    const int64_t lim = 64 * 1024 / 8;
    return ncs * K * R + ncs * EP <= lim && ntop * K * R + ntop * EP <= lim &&
           (int64_t)(t.L + 1) * (K * R + EP) <= lim && K <= 64;
}
// One wave per leaf (up to 8 leaves per 512-thread block); x read once per row.
template <int D, int P>
__global__ __launch_bounds__(512) void k_up_sub_m(ApplyPlan a, H2Tree t, int ls, int F, int R, int dtype,
                                                  const void* x, double* xh) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    constexpr int CH = K < 16 ? K : 16;
    constexpr int MAXROWS = 4;   // rows per lane held in registers (leaf <= 256 rows)
    extern __shared__ double sm[];
    const int f = blockIdx.y;
    const int64_t c = ((int64_t(1) << ls) - 1) + blockIdx.x;
    const int depth = t.L - ls;
    const int64_t ncs = (int64_t(2) << depth) - 1;
    double* sc = sm;
    double* sE = sc + ncs * K * R;
    auto gid = [&](int64_t l) -> int64_t {
        int lev = 0;
        while (((int64_t(2) << lev) - 1) <= l) ++lev;
        const int64_t w = int64_t(1) << lev;
        return (c + 1) * w - 1 + (l - (w - 1));
    };
    for (int64_t i = threadIdx.x; i < ncs * EP; i += blockDim.x) sE[i] = t.E[gid(i / EP) * EP + i % EP];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int64_t nl = int64_t(1) << depth;
    const int64_t l0 = ((c + 1) << depth) - 1;
    for (int64_t li = wv; li < nl; li += nw) {
        const int64_t cc = l0 + li;
        const int64_t rb = t.beg[cc], re = t.end[cc];
        for (int r = 0; r < R; ++r) {
            double xv[MAXROWS];
#pragma unroll
            for (int m = 0; m < MAXROWS; ++m) {
                const int64_t j = rb + lane + 64 * m;
                xv[m] = j < re ? ldx(x, ((int64_t)f * a.N + a.perm[j]) * R + r, dtype) : 0.0;
            }
            for (int a0 = 0; a0 < K; a0 += CH) {
                double acc[CH];
#pragma unroll
                for (int q = 0; q < CH; ++q) acc[q] = 0.0;
#pragma unroll
                for (int m = 0; m < MAXROWS; ++m) {
                    const int64_t j = rb + lane + 64 * m;
                    if (j < re) {
                        const double* u = a.U + j * K + a0;
#pragma unroll
                        for (int q = 0; q < CH; ++q)
                            if (a0 + q < K) acc[q] += u[q] * xv[m];
                    }
                }
#pragma unroll
                for (int q = 0; q < CH; ++q) {
                    const double v = wave_sum(acc[q]);
                    if (lane == q && a0 + q < K) {
                        sc[((nl - 1 + li) * K + a0 + q) * R + r] = v;
                        xh[(((int64_t)f * t.ncl + cc) * K + a0 + q) * R + r] = v;
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int lev = t.L - 1; lev >= ls; --lev) {
        const int64_t w = int64_t(1) << (lev - ls);
        const int64_t lfirst = w - 1;
        for (int64_t i = threadIdx.x; i < w * K * R; i += blockDim.x) {
            const int64_t lc = lfirst + i / ((int64_t)K * R);
            const int al = (int)((i / R) % K), r = (int)(i % R);
            const int64_t l1 = 2 * lc + 1, l2 = 2 * lc + 2;
            const double v = up_t<D, P>(sE + l1 * EP, sE + l2 * EP, sc + l1 * K * R + r, sc + l2 * K * R + r, al, R);
            sc[(lc * K + al) * R + r] = v;
            xh[(((int64_t)f * t.ncl + gid(lc)) * K + al) * R + r] = v;
        }
        __syncthreads();
    }
}

// y[perm[row]] += U[row] . yh_total(leaf), yh(c) = sum of the pair products of far(c)
template <int D, int P>
FPDE_KERNEL void k_far_out_m(ApplyPlan a, H2Tree t, int F, int R, const double* tmp, int dtype, void* y) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    extern __shared__ double sm[];
    const int f = blockIdx.y;
    const int64_t nrb = (a.cap * R + 63) / 64;
    const int64_t li = blockIdx.x / nrb;
    const int rb = (int)(blockIdx.x % nrb);
    const int64_t leafc = t.first_leaf + li;
    const int64_t KRr = (int64_t)K * R;
    const int L = t.L;
    const int64_t nfar = t.far_ptr[t.ncl];
    double* sy = sm;
    double* sE = sy + (int64_t)(L + 1) * KRr;
    // output row of this thread and its basis row, fetched before the walk
    const int64_t lb = a.leaf_beg[li], nt = a.leaf_beg[li + 1] - lb;
    const int g = threadIdx.x & 3;
    const int64_t item = (int64_t)rb * 64 + (threadIdx.x >> 2);
    const int64_t it = item / R;
    const int r = (int)(item % R);
    const bool ok = it < nt;
    double u[(K + 3) / 4];
#pragma unroll
    for (int q = 0; q < (K + 3) / 4; ++q) u[q] = (ok && 4 * q + g < K) ? a.U[(lb + it) * K + 4 * q + g] : 0.0;
    for (int64_t i = threadIdx.x; i < (int64_t)(L + 1) * KRr; i += blockDim.x) {
        const int lev = (int)(i / KRr);
        const int64_t cc = ((leafc + 1) >> (L - lev)) - 1;
        const int64_t w = i % KRr;
        const int64_t e0 = t.far_ptr[cc], e1 = t.far_ptr[cc + 1];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int64_t e = e0;
        for (; e + 4 <= e1; e += 4) {   // four independent loads in flight
            s0 += tmp[((int64_t)f * nfar + e) * KRr + w];
            s1 += tmp[((int64_t)f * nfar + e + 1) * KRr + w];
            s2 += tmp[((int64_t)f * nfar + e + 2) * KRr + w];
            s3 += tmp[((int64_t)f * nfar + e + 3) * KRr + w];
        }
        for (; e < e1; ++e) s0 += tmp[((int64_t)f * nfar + e) * KRr + w];
        sy[i] = (s0 + s1) + (s2 + s3);
    }
    for (int64_t i = threadIdx.x; i < (int64_t)(L + 1) * EP; i += blockDim.x) {
        const int lev = (int)(i / EP);
        const int64_t cc = ((leafc + 1) >> (L - lev)) - 1;
        sE[i] = lev == 0 ? 0.0 : t.E[cc * EP + i % EP];
    }
    __syncthreads();
    for (int lev = 1; lev <= L; ++lev) {
        for (int64_t i = threadIdx.x; i < KRr; i += blockDim.x) {
            const int be = (int)(i / R), rr = (int)(i % R);
            sy[lev * KRr + i] += down_t<D, P>(sE + lev * EP, sy + (lev - 1) * KRr + rr, be, R);
        }
        __syncthreads();
    }
    const double* cur = sy + L * KRr;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < (K + 3) / 4; ++q)
        if (4 * q + g < K) acc += u[q] * cur[(int64_t)(4 * q + g) * R + r];
    acc += __shfl_xor(acc, 1, 4);
    acc += __shfl_xor(acc, 2, 4);
    if (ok && g == 0) {
        const int64_t dst = ((int64_t)f * a.N + a.perm[lb + it]) * R + r;
        if (dtype == 0) ((double*)y)[dst] += acc;
        else ((float*)y)[dst] = (float)((double)((float*)y)[dst] + acc);
    }
}

template <int D, int P>
static void far_m_t(const ApplyPlan& a, const H2Tree& t, int ls, int F, int R, const double* St, int64_t nfar,
                     int dtype, const void* x, double* xh, double* tmp, hipStream_t fs) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    const int depth = t.L - ls;
    const int64_t ncs = (int64_t(2) << depth) - 1;
    const int64_t nl = int64_t(1) << depth;
    const int threads = 64 * (int)(nl < 8 ? nl : 8);
    const size_t lds_sub = sizeof(double) * (ncs * K * R + ncs * EP);
    hipLaunchKernelGGL((k_up_sub_m<D, P>), dim3((unsigned)(int64_t(1) << ls), F), dim3(threads), lds_sub, fs, a, t,
                       ls, F, R, dtype, x, xh);
    if (ls > 0) {
        const int64_t ntop = (int64_t(2) << ls) - 1;
        const size_t lds_top = sizeof(double) * (ntop * K * R + ntop * EP);
        hipLaunchKernelGGL((k_up_top_m<D, P>), dim3(F), dim3(1024), lds_top, fs, t, ls, F, R, xh);
    }
    if (nfar > 0)
        hipLaunchKernelGGL((k_coupling_pairs_m<D, P>), dim3(grid1((int64_t)F * nfar * K * R)), dim3(256), 0, fs, t,
                           nfar, F, R, St, xh, tmp);
}

template <int D, int P>
static void far_out_m_t(const ApplyPlan& a, const H2Tree& t, int F, int R, const double* tmp, int dtype, void* y,
                         hipStream_t st) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    const int64_t nrb = (a.cap * R + 63) / 64;
    const size_t lds = sizeof(double) * ((int64_t)(t.L + 1) * K * R + (int64_t)(t.L + 1) * EP);
    hipLaunchKernelGGL((k_far_out_m<D, P>), dim3((unsigned)(a.nleaf * nrb), F), dim3(256), lds, st, a, t, F, R, tmp,
                       dtype, y);
}

// main stream: near panels (MFMA GEMMs) and the CSR rows of B + M; side stream:
// subtree upsweep, top levels and coupling products; join; per-leaf downsweep
// walk fused with the output.
hipError_t launch_apply_multi(const ApplyPlan& a, const H2Tree& t, int ls, const PanelPlan& pp, const void* panel,
                              int panel_f32, int parts, int F, int R, const double* csr_val, const double* St,
                              int64_t nfar, int dtype, const void* x, double* xh, double* tmp, void* y,
                              hipStream_t st, hipStream_t side, hipEvent_t fork, hipEvent_t join, hipEvent_t* ev) {
    const bool far = (parts & 8) != 0;
    if (ev) (void)hipEventRecord(ev[0], st);
    hipStream_t fs = st;
    if (far && side != st) {
        hipError_t e0 = hipEventRecord(fork, st);
        if (e0 == hipSuccess) e0 = hipStreamWaitEvent(side, fork, 0);
        if (e0 != hipSuccess) return e0;
        fs = side;
    }
    if (far) FPDE_DISPATCH_DP(t.dim, t.p, far_m_t, a, t, ls, F, R, St, nfar, dtype, x, xh, tmp, fs);
    if (ev) (void)hipEventRecord(ev[1], fs);
    hipError_t e = panel_f32 ? launch_near_mm(a, pp, (const float*)panel, (parts & 4) != 0, csr_val, F, R, dtype, x, y,
                                              st, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr)
                             : launch_near_mm(a, pp, (const double*)panel, (parts & 4) != 0, csr_val, F, R, dtype, x,
                                              y, st, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
    if (e != hipSuccess) return e;
    if (far) {
        if (fs != st) {
            hipError_t e1 = hipEventRecord(join, fs);
            if (e1 == hipSuccess) e1 = hipStreamWaitEvent(st, join, 0);
            if (e1 != hipSuccess) return e1;
        }
        FPDE_DISPATCH_DP(t.dim, t.p, far_out_m_t, a, t, F, R, tmp, dtype, y, st);
    }
    if (ev) (void)hipEventRecord(ev[4], st);
    return hipGetLastError();
}

// Wide R (subtrees do not fit LDS): the far field by per-level sweeps on the side
// stream, near panels on the main stream, then y += U y^ per leaf.
hipError_t launch_apply_wide(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, const void* panel, int panel_f32,
                             int parts, int F, int R, const double* csr_val, const double* St, int dtype,
                             const void* x, double* xt, double* xh, double* yh, void* y, hipStream_t st,
                             hipStream_t side, hipEvent_t fork, hipEvent_t join, hipEvent_t* ev) {
    const bool far = (parts & 8) != 0;
    if (ev) (void)hipEventRecord(ev[0], st);
    hipStream_t fs = st;
    if (far && side != st) {
        hipError_t e0 = hipEventRecord(fork, st);
        if (e0 == hipSuccess) e0 = hipStreamWaitEvent(side, fork, 0);
        if (e0 != hipSuccess) return e0;
        fs = side;
    }
    hipError_t e = hipSuccess;
    if (far) {
        if ((e = launch_gather(a, F, R, dtype, x, xt, fs)) != hipSuccess) return e;
        if ((e = launch_leaf_up(a, t, F, R, xt, xh, fs)) != hipSuccess) return e;
        for (int lev = t.L - 1; lev >= 0; --lev)
            if ((e = launch_up_level(t, lev, F, R, xh, fs)) != hipSuccess) return e;
        if ((e = launch_coupling_apply(t, F, R, St, xh, yh, fs)) != hipSuccess) return e;
        for (int lev = 0; lev < t.L; ++lev)
            if ((e = launch_down_level(t, lev, F, R, yh, fs)) != hipSuccess) return e;
    }
    if (ev) (void)hipEventRecord(ev[1], fs);
    e = panel_f32 ? launch_near_mm(a, pp, (const float*)panel, (parts & 4) != 0, csr_val, F, R, dtype, x, y, st,
                                   ev ? ev[2] : nullptr, ev ? ev[3] : nullptr)
                  : launch_near_mm(a, pp, (const double*)panel, (parts & 4) != 0, csr_val, F, R, dtype, x, y, st,
                                   ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
    if (e != hipSuccess) return e;
    if (far) {
        if (fs != st) {
            hipError_t e1 = hipEventRecord(join, fs);
            if (e1 == hipSuccess) e1 = hipStreamWaitEvent(st, join, 0);
            if (e1 != hipSuccess) return e1;
        }
        if ((e = launch_leaf_out(a, t, 8, F, R, nullptr, xt, yh, dtype, y, st, 1)) != hipSuccess) return e;
    }
    if (ev) (void)hipEventRecord(ev[4], st);
    return hipGetLastError();
}

}  // namespace fpde
