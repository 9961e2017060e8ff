// Operator apply for one right-hand side per field (Sec. 3 and 5: y = (B+M)x +
// K~x), with the operator data in FP64 or FP32 (mixed precision: the CSR of
// B + M stays FP64, the near leaf blocks, bases, transfers and coupling
// matrices are FP32 and their products accumulate in FP32).
//
// One apply is three launches on one stream:
//   k_near_up    blocks [0, nup): the upsweep, whole subtrees of depth d0 per
//                block (leaf coefficients, then the nested transfers);
//                blocks [nup, ...): the near rows (CSR row of B + M and the
//                packed near panel row).
//   k_couple, k_far_out (fpde_far1.hip): coupling sums per far target, then
//                the downsweep walk fused with the output.
// The far list of this path has its sources moved down to the subtree levels
// at build (coupling matrices S M_r^T), so on the usual trees no upsweep block
// reads another's coefficients.  On deeper trees the levels still above the
// subtree roots are chained by tickets: the subtree roots one block hands to
// another are stored and loaded as agent-scope atomics, which bypass the
// per-XCD L2 copies; every wave waits for its stores to be acknowledged before
// the block's barrier and its one ticket increment, so no cache writeback or
// invalidate is needed, and no block ever waits for another (the last arrival
// goes on), so the launch always drains.  (The far chain on a second stream
// beside the near rows was measured slower: the streams did not overlap and
// the event fork/join added its own cost.)
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_device.h"

namespace fpde {


template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
    using type = double2;
};
template <>
struct Vec2<float> {
    using type = float2;
};

// heap id -> level
__device__ __forceinline__ int heap_level(int64_t c) {
    int lev = 0;
    while (((int64_t(2) << lev) - 1) <= c) ++lev;
    return lev;
}

// Upsweep (nested bases, Sec. 5.3) from the leaves up to level lmin.
// Stage 0: upsweep block b owns the subtree of depth d0 rooted at level L - d0
// (2^d0 leaves, at most one per wave): leaf coefficients x^_leaf = U_leaf^T
// x_leaf, the leaf's rows split over the waves of the leaf (x rows staged in
// LDS, partial sums combined in a fixed order), then the subtree's levels in
// LDS.  Upper stages: every
// group of subtrees under one ancestor ds levels up counts its finished blocks
// with a ticket; the last block of the group computes the ancestor's subtree
// levels from the other blocks' subtree roots, resets the ticket and goes on to
// the next group.  Loads that do not depend on other blocks (U rows,
// transfers) are issued before the dependent ones.
template <int D, int P, typename T>
__device__ __forceinline__ void up_tree(const ApplyPlan& a, const H2Tree& t, const UpPlan& up, int dtype,
                                        const void* x, const T* U, const T* E, T* xh, unsigned int* tickets, int f,
                                        int64_t bid, T* sm) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    constexpr int kRows = 16;   // rows per half-wave held in registers (32 rows per wave)
    __shared__ unsigned int s_ticket;
    const int L = t.L;
    int lc = L - up.d0;                          // root level of the current subtree
    int64_t c = ((int64_t(1) << lc) - 1) + bid;  // its heap id
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    T* xf = xh + (int64_t)f * t.ncl * K;
    // local heap index l of a subtree rooted at r -> global heap id
    auto gid = [](int64_t r, int64_t l) -> int64_t {
        const int lev = heap_level(l);
        const int64_t w = int64_t(1) << lev;
        return (r + 1) * w - 1 + (l - (w - 1));
    };
    {
        const int depth = up.d0;                     // 2^depth leaves, at most one per wave
        const int64_t ncs = (int64_t(2) << depth) - 1;
        const int nl = 1 << depth, wpl = nw / nl;    // waves per leaf
        T* sc = sm;                          // [ncs][K]
        T* sE = sc + ncs * K;                // [ncs][EP]
        T* sp = sE + ncs * EP;               // [waves][K] partial sums
        T* sx = sp + nw * K;                 // [waves][cap]
        for (int64_t i = threadIdx.x + EP; i < ncs * EP; i += blockDim.x) sE[i] = E[gid(c, i / EP) * EP + i % EP];
        const int64_t l0 = ((c + 1) << depth) - 1;
        T* sxw = sx + (int64_t)wv * a.cap;
        {
            const int64_t cc = l0 + wv / wpl;
            const int wi = wv % wpl;
            const int64_t rl = t.beg[cc], nll = t.end[cc] - rl;
            // this wave's share of the leaf's rows
            const int64_t rb = rl + nll * wi / wpl, n = rl + nll * (wi + 1) / wpl - rb;
            // lanes (half, alpha): with K <= 32 the two half-waves split the rows
            const int half = K <= 32 ? (lane >> 5) : 0;
            const int al = K <= 32 ? (lane & 31) : lane;
            const int64_t jb = K <= 32 ? (half ? (n + 1) / 2 : 0) : 0;
            const int64_t je = K <= 32 ? (half ? n : (n + 1) / 2) : n;
            const T* u = U + rb * K + al;
            const bool regs = K <= 32 && n <= 2 * kRows && al < K;
            T uv[kRows];
            if (regs) {   // the U rows of this lane, all in flight before the x gather
#pragma unroll
                for (int q = 0; q < kRows; ++q) uv[q] = jb + q < je ? u[(jb + q) * K] : T(0);
            }
            for (int64_t j = lane; j < n; j += 64) sxw[j] = (T)ldx(x, (int64_t)f * a.N + a.perm[rb + j], dtype);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            T v = 0;
            if (regs) {
                T s[4] = {0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < kRows; ++q) s[q & 3] += uv[q] * (jb + q < je ? sxw[jb + q] : T(0));
                v = (s[0] + s[1]) + (s[2] + s[3]);
            } else if (al < K) {
                T s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                int64_t j = jb;
                for (; j + 8 <= je; j += 8) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) s[q] += u[(j + q) * K] * sxw[j + q];
                }
                for (; j < je; ++j) s[0] += u[j * K] * sxw[j];
                v = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
            }
            if (K <= 32) v += __shfl_xor(v, 32, 64);
            if (lane < K) sp[wv * K + lane] = v;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < nl * K; i += blockDim.x) {   // the waves of a leaf, in a fixed order
            const int l = i / K, al = i % K;
            T s = 0;
            for (int w = 0; w < wpl; ++w) s += sp[(l * wpl + w) * K + al];
            sc[(nl - 1 + l) * K + al] = s;
            put(&xf[(l0 + l) * K + al], s);
        }
        __syncthreads();
        for (int lev = depth - 1; lev >= 0; --lev) {
            const int64_t w = int64_t(1) << lev, lfirst = w - 1;
            for (int64_t i = threadIdx.x; i < w * K; i += blockDim.x) {
                const int64_t lcl = lfirst + i / K;
                const int al = (int)(i % K);
                const int64_t l1 = 2 * lcl + 1, l2 = 2 * lcl + 2;
                const T v = up_t<D, P, T>(sE + l1 * EP, sE + l2 * EP, sc + l1 * K, sc + l2 * K, al, 1);
                sc[lcl * K + al] = v;
                put(&xf[gid(c, lcl) * K + al], v);
            }
            __syncthreads();
        }
    }
    while (lc > up.lmin) {
        const int ln = lc - up.ds > up.lmin ? lc - up.ds : up.lmin;
        const int depth = lc - ln;
        const int64_t g = ((c + 1) >> depth) - 1;     // ancestor at level ln
        const int64_t ncs = (int64_t(2) << depth) - 1, w0 = int64_t(1) << depth;
        T* sc = sm;
        T* sE = sc + ncs * K;
        // transfers of the group's subtree do not depend on other blocks: load them first
        for (int64_t i = threadIdx.x + EP; i < ncs * EP; i += blockDim.x) sE[i] = E[gid(g, i / EP) * EP + i % EP];
        // publish: the root's agent-scope stores of every wave are acknowledged
        // before the barrier, then one ticket per block
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0)
            s_ticket = __hip_atomic_fetch_add(&tickets[(int64_t)f * t.ncl + g], 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        if (s_ticket != (unsigned int)((1u << depth) - 1)) return;
        if (threadIdx.x == 0)   // every group's blocks have arrived: reset for the next launch
            __hip_atomic_store(&tickets[(int64_t)f * t.ncl + g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int64_t i = threadIdx.x; i < w0 * K; i += blockDim.x)
            sc[(w0 - 1) * K + i] = get(&xf[(((g + 1) << depth) - 1) * K + i]);
        __syncthreads();
        for (int lev = depth - 1; lev >= 0; --lev) {
            const int64_t w = int64_t(1) << lev, lfirst = w - 1;
            for (int64_t i = threadIdx.x; i < w * K; i += blockDim.x) {
                const int64_t lcl = lfirst + i / K;
                const int al = (int)(i % K);
                const int64_t l1 = 2 * lcl + 1, l2 = 2 * lcl + 2;
                const T v = up_t<D, P, T>(sE + l1 * EP, sE + l2 * EP, sc + l1 * K, sc + l2 * K, al, 1);
                sc[lcl * K + al] = v;
                put(&xf[gid(g, lcl) * K + al], v);
            }
            __syncthreads();
        }
        lc = ln;
        c = g;
    }
}

// Near rows: y[f][perm[row]] = (B+M)_row . x + panel_row . x_near for the
// rows of block rb of leaf li, 16 lanes per row (blockDim / 16 rows).  Rows are
// addressed by leaf slot (li * cap + row in the leaf), so every index a lane
// needs is one load away: the padded panel column list, the ELL row of B + M
// and the output index.  The x entries of the leaf's near columns are staged in
// LDS once per block.  Each lane keeps 12 vector loads of its panel row in
// flight (384 columns a batch, so a leaf with 3 x 3 near leaves of 64 rows
// takes two batches); the first 12 are issued before the x staging and the B + M row, so
// their latency overlaps those gathers.
template <typename T>
__device__ __forceinline__ void near_rows(const ApplyPlan& a, const PanelPlan& pp, const T* panel, int use_near,
                                          const double* csr_val, int dtype, const void* x, void* y, int f,
                                          int64_t bid, T* xs) {
    using V2 = typename Vec2<T>::type;
    constexpr int NB = 12;   // vector loads in flight per lane (32 columns apart)
    const int rpb = blockDim.x / 16;   // rows per block
    const int64_t nrb = (a.cap + rpb - 1) / rpb;
    const int64_t li = bid / nrb;
    const int rb = (int)(bid % nrb);
    const int64_t xo = (int64_t)f * a.N;
    const int g = threadIdx.x & 15;
    const int64_t it = (int64_t)rb * rpb + (threadIdx.x >> 4);
    const bool in = it < a.cap;   // panels hold cap rows per leaf; rows past the leaf's are never stored
    const int64_t slot = li * a.cap + it;
    const int64_t ps = use_near ? pp.pstride[li] : 0;
    const T* pr = panel + (int64_t)f * pp.poff[a.nleaf] + pp.poff[li] + it * ps + 2 * g;
    V2 q[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k)
        if (in && 2 * g + 32 * k + 2 <= ps) q[k] = *(const V2*)(pr + 32 * k);
    if (use_near) {   // padding columns of the row stride hold 0 in the panel and in xs
        const int32_t* pc = pp.pcols_pad + li * pp.max_stride;
        for (int64_t c = threadIdx.x; c < ps; c += blockDim.x) {
            const int j = pc[c];
            xs[c] = j >= 0 ? (T)ldx(x, xo + j, dtype) : T(0);
        }
    }
    const int64_t dst = in ? pp.perm_pad[slot] : -1;
    double acc = 0.0;
    if (pp.ell_val) {   // B + M in ELL form, entries in CSR order
        if (in) {
            const int w = pp.ell_w;
            const int32_t* ec = pp.ell_col + slot * w;
            const double* ev = pp.ell_val + ((int64_t)f * a.nleaf * a.cap + slot) * w;
            for (int e = g; e < w; e += 16) {
                const int j = ec[e];
                if (j >= 0) acc += ev[e] * ldx(x, xo + j, dtype);
            }
        }
    } else if (in && csr_val && dst >= 0) {
        const double* v = csr_val + (int64_t)f * a.nnz;
        const int64_t row = a.leaf_beg[li] + it;
        for (int64_t e = a.csr_ptr[row] + g; e < a.csr_ptr[row + 1]; e += 16)
            acc += v[e] * ldx(x, xo + pp.csr_col_dof[e], dtype);
    }
    __syncthreads();
    if (dst < 0) return;
    if (use_near) {
        T s[4] = {0, 0, 0, 0};
        const T* xl = xs + 2 * g;
        int64_t c = 0;   // column offset of q[0] relative to 2g
        for (;;) {
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (2 * g + c + 32 * k + 2 <= ps)
                    s[k & 3] += q[k].x * xl[c + 32 * k] + q[k].y * xl[c + 32 * k + 1];
            c += 32 * NB;
            if (2 * g + c + 2 > ps) break;
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (2 * g + c + 32 * k + 2 <= ps) q[k] = *(const V2*)(pr + c + 32 * k);
        }
        acc += (double)((s[0] + s[1]) + (s[2] + s[3]));
    }
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
    if (g == 0) {
        if (dtype == 0) ((double*)y)[xo + dst] = acc;
        else ((float*)y)[xo + dst] = (float)acc;
    }
}

// Upsweep blocks first, then the near rows.  The upsweep blocks are
// dispatched first, so their dependent chain (one subtree of depth d0 per
// block: 2^d0 leaves, two waves each) runs beside the near rows' HBM stream.
constexpr int kUpThreads = 512;
template <int D, int P, typename T>
__global__ __launch_bounds__(kUpThreads) void k_near_up(ApplyPlan a, H2Tree t, PanelPlan pp, UpPlan up, int nup,
                                                        const T* panel, int use_near, const double* csr_val,
                                                        int dtype, const void* x, void* y, const T* U, const T* E,
                                                        T* xh, unsigned int* tickets) {
    extern __shared__ __align__(16) unsigned char sraw[];
    const int f = blockIdx.y;
    if ((int)blockIdx.x < nup)
        up_tree<D, P, T>(a, t, up, dtype, x, U, E, xh, tickets, f, blockIdx.x, (T*)sraw);
    else
        near_rows<T>(a, pp, panel, use_near, csr_val, dtype, x, y, f, (int64_t)blockIdx.x - nup, (T*)sraw);
}

template <int D, int P, typename T>
static size_t up_tree_lds(int64_t cap, int d0, int ds) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    constexpr int64_t waves = kUpThreads / 64;
    const int64_t s0 = ((int64_t(2) << d0) - 1) * (K + EP) + waves * (K + cap);
    const int64_t s1 = ((int64_t(2) << ds) - 1) * (K + EP);
    return sizeof(T) * (size_t)(s0 > s1 ? s0 : s1);
}

// (dim, points) dispatch of the templates above for one operator precision T
template <typename T>
struct Single {
    template <int D, int P>
    static void near_up(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, const UpPlan& up, bool far,
                        int use_near, const double* csr_val, int F, int dtype, const void* x, void* y,
                        const OpData<T>& od, unsigned int* tickets, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
        const int nup = far ? (int)(int64_t(1) << (t.L - up.d0)) : 0;
        const int64_t nrb = (a.cap + kUpThreads / 16 - 1) / (kUpThreads / 16);
        size_t lds = sizeof(T) * (pp.max_stride > 0 ? pp.max_stride : 1);
        if (far) {
            const size_t lu = up_tree_lds<D, P, T>(a.cap, up.d0, up.ds);
            if (lu > lds) lds = lu;
        }
        const dim3 grid((unsigned)(nup + a.nleaf * nrb), F);
        if (e0)   // start/stop timestamps of exactly this kernel
            hipExtLaunchKernelGGL((k_near_up<D, P, T>), grid, dim3(kUpThreads), lds, st, e0, e1, 0, a, t, pp, up,
                                  nup, od.panel, use_near, csr_val, dtype, x, y, od.U, od.E, od.xh, tickets);
        else
            hipLaunchKernelGGL((k_near_up<D, P, T>), grid, dim3(kUpThreads), lds, st, a, t, pp, up, nup, od.panel,
                               use_near, csr_val, dtype, x, y, od.U, od.E, od.xh, tickets);
    }
    // leaf-stage depth d0 (2: four leaves, two waves each) and the upper-stage
    // depth ds: the levels above the stage-0 roots up to lmin in one stage if
    // they fit 64 KB of LDS
    template <int D, int P>
    static void plan(const H2Tree& t, int64_t cap, int lmin, UpPlan* up) {
        const size_t lim = 64 * 1024;
        up->lmin = lmin;
        up->d0 = t.L < 2 ? t.L : 2;
        while (up->d0 > 0 && up_tree_lds<D, P, T>(cap, up->d0, 1) > lim) --up->d0;
        const int need = t.L - up->d0 - lmin > 1 ? t.L - up->d0 - lmin : 1;
        up->ds = 1;
        while (up->ds < need && up_tree_lds<D, P, T>(cap, up->d0, up->ds + 1) <= lim) ++up->ds;
        up->path_lds = sizeof(T) * (size_t)((int64_t)(t.L + 1) * (KR<D, P>::K + KR<D, P>::EP));
        up->ok = up_tree_lds<D, P, T>(cap, up->d0, up->ds) <= lim && up->path_lds <= lim &&
                 KR<D, P>::K <= 64 && cap <= 256;
    }
};

UpPlan plan_up_tree(const H2Tree& t, int64_t cap, int lmin, int prec) {
    UpPlan up{};
    if (prec == 0) FPDE_DISPATCH_DP(t.dim, t.p, Single<double>::template plan, t, cap, lmin, &up);
    else FPDE_DISPATCH_DP(t.dim, t.p, Single<float>::template plan, t, cap, lmin, &up);
    return up;
}

template <typename T>
static hipError_t apply_single_t(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, const UpPlan& up,
                                 const FarPlan& fp, int parts, int F, const double* csr_val, const OpData<T>& od,
                                 int dtype, const void* x, void* y, unsigned int* tickets, hipStream_t st,
                                 hipEvent_t* ev) {
    const bool far = (parts & 8) != 0 && fp.ntgt > 0;
    if (ev) {
        (void)hipEventRecord(ev[0], st);
        (void)hipEventRecord(ev[1], st);
    }
    FPDE_DISPATCH_DP(t.dim, t.p, Single<T>::template near_up, a, t, pp, up, far, (parts & 4) != 0, csr_val, F, dtype,
                     x, y, od, tickets, st, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (far) {
        if ((e = launch_couple_single(t, fp, F, od, st)) != hipSuccess) return e;
        if ((e = launch_out_single(a, t, fp, F, od, dtype, y, st)) != hipSuccess) return e;
    }
    if (ev) (void)hipEventRecord(ev[4], st);
    return hipGetLastError();
}

hipError_t launch_apply_single(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, const UpPlan& up,
                               const FarPlan& fp, int parts, int F, const double* csr_val, const OpData<double>& od,
                               int dtype, const void* x, void* y, unsigned int* tickets, hipStream_t st,
                               hipEvent_t* ev) {
    return apply_single_t<double>(a, t, pp, up, fp, parts, F, csr_val, od, dtype, x, y, tickets, st, ev);
}

hipError_t launch_apply_single(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, const UpPlan& up,
                               const FarPlan& fp, int parts, int F, const double* csr_val, const OpData<float>& od,
                               int dtype, const void* x, void* y, unsigned int* tickets, hipStream_t st,
                               hipEvent_t* ev) {
    return apply_single_t<float>(a, t, pp, up, fp, parts, F, csr_val, od, dtype, x, y, tickets, st, ev);
}

}  // namespace fpde
