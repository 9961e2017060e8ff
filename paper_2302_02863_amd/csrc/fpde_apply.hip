// Operator apply for one right-hand side per field (Sec. 3 and 5: y = (B+M)x +
// K~x), with the operator data in FP64 or FP32 (mixed precision: the CSR of
// B + M stays FP64, the near leaf blocks, bases, transfers and coupling
// matrices are FP32 and their products accumulate in FP32).
//
// One apply is a fork/join of five kernels:
//   main stream:  k_near_panel   CSR row of B + M and the packed near panel row
//   side stream:  k_up_tree      leaf coefficients and the whole upsweep
//                 k_coupling1    S x^ for every far pair
//   after join:   k_far_out1     per-leaf downsweep walk fused with the output
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_device.h"

namespace fpde {

// Upsweep of the whole tree in one launch (nested bases, Sec. 5.3).
// Stage 0: block b owns the subtree of depth d0 rooted at level L - d0: leaf
// coefficients x^_leaf = U_leaf^T x_leaf (one wave per leaf, the leaf's x rows
// staged in LDS), then the subtree's levels in LDS.  Upper stages: every group
// of subtrees under one ancestor ds levels up counts its finished blocks with a
// ticket (agent-scope release fence of every thread, block barrier, one atomic
// per block, agent-scope acquire fence in the last block); the last block of the group
// computes the ancestor's subtree levels from the published coefficients,
// resets the ticket and goes on to the next group.  No block ever waits for
// another, so the launch always drains.  Loads that do not depend on other
// blocks (U rows, transfers) are issued before the dependent ones.
template <int D, int P, typename T>
__global__ __launch_bounds__(512) void k_up_tree(ApplyPlan a, H2Tree t, UpPlan up, int F, int dtype, const void* x,
                                                 const T* U, const T* E, T* xh, unsigned int* tickets) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    constexpr int kRows = 32;   // rows per half-wave held in registers (leaves of up to 64 rows)
    extern __shared__ __align__(16) unsigned char sraw[];
    T* sm = (T*)sraw;
    __shared__ unsigned int s_ticket;
    const int f = blockIdx.y;
    const int L = t.L;
    int lc = L - up.d0;                                 // root level of the current subtree
    int64_t c = ((int64_t(1) << lc) - 1) + blockIdx.x;  // its heap id
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    T* xf = xh + (int64_t)f * t.ncl * K;
    // local heap index l of a subtree rooted at r -> global heap id
    auto gid = [](int64_t r, int64_t l) -> int64_t {
        int lev = 0;
        while (((int64_t(2) << lev) - 1) <= l) ++lev;
        const int64_t w = int64_t(1) << lev;
        return (r + 1) * w - 1 + (l - (w - 1));
    };
    {
        const int depth = up.d0;
        const int64_t ncs = (int64_t(2) << depth) - 1;
        T* sc = sm;                          // [ncs][K]
        T* sE = sc + ncs * K;                // [ncs][EP]
        T* sx = sE + ncs * EP;               // [waves][cap]
        for (int64_t i = threadIdx.x + EP; i < ncs * EP; i += blockDim.x) sE[i] = E[gid(c, i / EP) * EP + i % EP];
        const int64_t nl = int64_t(1) << depth;
        const int64_t l0 = ((c + 1) << depth) - 1;
        T* sxw = sx + (int64_t)wv * a.cap;
        for (int64_t li = wv; li < nl; li += nw) {
            const int64_t cc = l0 + li;
            const int64_t rb = t.beg[cc], n = t.end[cc] - rb;
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
            if (lane < K) {
                sc[(nl - 1 + li) * K + lane] = v;
                xf[cc * K + lane] = v;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
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
                xf[gid(c, lcl) * K + al] = v;
            }
            __syncthreads();
        }
    }
    while (lc > 0) {
        const int ln = lc - up.ds > 0 ? lc - up.ds : 0;
        const int depth = lc - ln;
        const int64_t g = ((c + 1) >> depth) - 1;     // ancestor at level ln
        const int64_t ncs = (int64_t(2) << depth) - 1, w0 = int64_t(1) << depth;
        T* sc = sm;
        T* sE = sc + ncs * K;
        // transfers of the group's subtree do not depend on other blocks: load them first
        for (int64_t i = threadIdx.x + EP; i < ncs * EP; i += blockDim.x) sE[i] = E[gid(g, i / EP) * EP + i % EP];
        // publish: every thread's coefficient stores are released at agent scope before
        // the barrier; one ticket per block; the last block acquires the others' stores
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0)
            s_ticket = __hip_atomic_fetch_add(&tickets[(int64_t)f * t.ncl + g], 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        if (s_ticket != (unsigned int)((1u << depth) - 1)) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (threadIdx.x == 0)   // every group's blocks have arrived: reset for the next launch
            __hip_atomic_store(&tickets[(int64_t)f * t.ncl + g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int64_t i = threadIdx.x; i < w0 * K; i += blockDim.x)
            sc[(w0 - 1) * K + i] = __builtin_nontemporal_load(&xf[(((g + 1) << depth) - 1) * K + i]);
        __syncthreads();
        for (int lev = depth - 1; lev >= 0; --lev) {
            const int64_t w = int64_t(1) << lev, lfirst = w - 1;
            for (int64_t i = threadIdx.x; i < w * K; i += blockDim.x) {
                const int64_t lcl = lfirst + i / K;
                const int al = (int)(i % K);
                const int64_t l1 = 2 * lcl + 1, l2 = 2 * lcl + 2;
                const T v = up_t<D, P, T>(sE + l1 * EP, sE + l2 * EP, sc + l1 * K, sc + l2 * K, al, 1);
                sc[lcl * K + al] = v;
                xf[gid(g, lcl) * K + al] = v;
            }
            __syncthreads();
        }
        lc = ln;
        c = g;
    }
}

// tmp[f][e][alpha] = sum_beta S_e[alpha][beta] x^[f][src(e)][beta]; St holds S_e transposed
// ([beta][alpha]) so that consecutive threads (alpha) read consecutive entries.
template <int D, int P, typename T>
FPDE_KERNEL void k_coupling1(H2Tree t, int64_t nfar, int F, const T* St, const T* xh, T* tmp) {
    constexpr int K = KR<D, P>::K;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)F * nfar * K) return;
    const int64_t fe = i / K;
    const int al = (int)(i % K);
    const int f = (int)(fe / nfar);
    const int64_t e = fe - (int64_t)f * nfar;
    const T* S = St + fe * K * K + al;
    const T* xs = xh + ((int64_t)f * t.ncl + t.far_src[e]) * K;
    T acc = 0;
#pragma unroll
    for (int b = 0; b < K; ++b) acc += S[b * K] * xs[b];
    tmp[i] = acc;
}

// y[perm[row]] += U[row] . y^_leaf, where y^_leaf accumulates, from the root
// down, y^(c) = sum_{e in far(c)} tmp[e] plus the transfer of the parent's.
// One block per (leaf, 64 rows, field); the root-to-leaf walk is redone per block.
template <int D, int P, typename T>
FPDE_KERNEL void k_far_out1(ApplyPlan a, H2Tree t, int F, const T* tmp, const T* U, const T* E, int dtype, void* y) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    extern __shared__ __align__(16) unsigned char sraw[];
    T* sy = (T*)sraw;
    const int f = blockIdx.y;
    const int64_t nrb = (a.cap + 63) / 64;
    const int64_t li = blockIdx.x / nrb;
    const int rb = (int)(blockIdx.x % nrb);
    const int64_t leafc = t.first_leaf + li;
    const int L = t.L;
    const int64_t nfar = t.far_ptr[t.ncl];
    T* sE = sy + (int64_t)(L + 1) * K;
    // output row of this thread (4 lanes per row) and its basis row, fetched before the walk
    const int64_t lb = a.leaf_beg[li], nt = a.leaf_beg[li + 1] - lb;
    const int g = threadIdx.x & 3;
    const int64_t it = (int64_t)rb * 64 + (threadIdx.x >> 2);
    const bool ok = it < nt;
    T u[(K + 3) / 4];
#pragma unroll
    for (int q = 0; q < (K + 3) / 4; ++q) u[q] = (ok && 4 * q + g < K) ? U[(lb + it) * K + 4 * q + g] : T(0);
    for (int64_t i = threadIdx.x; i < (int64_t)(L + 1) * K; i += blockDim.x) {
        const int lev = (int)(i / K);
        const int64_t cc = ((leafc + 1) >> (L - lev)) - 1;
        const int w = (int)(i % K);
        const int64_t e0 = t.far_ptr[cc], e1 = t.far_ptr[cc + 1];
        const T* tp = tmp + ((int64_t)f * nfar) * K + w;
        T s[4] = {0, 0, 0, 0};
        for (int64_t e = e0; e < e1; e += 16) {   // sixteen independent loads in flight
            T v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = e + q < e1 ? tp[(e + q) * K] : T(0);
#pragma unroll
            for (int q = 0; q < 16; ++q) s[q & 3] += v[q];
        }
        sy[i] = (s[0] + s[1]) + (s[2] + s[3]);
    }
    for (int64_t i = threadIdx.x; i < (int64_t)(L + 1) * EP; i += blockDim.x) {
        const int lev = (int)(i / EP);
        const int64_t cc = ((leafc + 1) >> (L - lev)) - 1;
        sE[i] = lev == 0 ? T(0) : E[cc * EP + i % EP];
    }
    __syncthreads();
    for (int lev = 1; lev <= L; ++lev) {
        for (int i = threadIdx.x; i < K; i += blockDim.x)
            sy[lev * K + i] += down_t<D, P, T>(sE + lev * EP, sy + (lev - 1) * K, i, 1);
        __syncthreads();
    }
    const T* cur = sy + L * K;
    T acc = 0;
#pragma unroll
    for (int q = 0; q < (K + 3) / 4; ++q)
        if (4 * q + g < K) acc += u[q] * cur[4 * q + g];
    acc += __shfl_xor(acc, 1, 4);
    acc += __shfl_xor(acc, 2, 4);
    if (ok && g == 0) {
        const int64_t dst = (int64_t)f * a.N + a.perm[lb + it];
        if (dtype == 0) ((double*)y)[dst] += (double)acc;
        else ((float*)y)[dst] = (float)((double)((float*)y)[dst] + (double)acc);
    }
}

template <int D, int P, typename T>
static size_t up_tree_lds(const H2Tree& t, int64_t cap, int d0, int ds) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    (void)t;
    const int64_t nl = int64_t(1) << d0;
    const int64_t waves = nl < 8 ? nl : 8;
    const int64_t s0 = ((int64_t(2) << d0) - 1) * (K + EP) + waves * cap;
    const int64_t s1 = ((int64_t(2) << ds) - 1) * (K + EP);
    return sizeof(T) * (size_t)(s0 > s1 ? s0 : s1);
}

template <int D, int P, typename T>
static void far_chain1(const ApplyPlan& a, const H2Tree& t, const UpPlan& up, int F, int64_t nfar, int dtype,
                       const void* x, const OpData<T>& od, unsigned int* tickets, hipStream_t fs) {
    constexpr int K = KR<D, P>::K;
    const int64_t nl = int64_t(1) << up.d0;
    const int waves = (int)(nl < 8 ? nl : 8);
    const size_t lds = up_tree_lds<D, P, T>(t, a.cap, up.d0, up.ds);
    hipLaunchKernelGGL((k_up_tree<D, P, T>), dim3((unsigned)(int64_t(1) << (t.L - up.d0)), F), dim3(64 * waves), lds,
                       fs, a, t, up, F, dtype, x, od.U, od.E, od.xh, tickets);
    if (nfar > 0)
        hipLaunchKernelGGL((k_coupling1<D, P, T>), dim3(grid1((int64_t)F * nfar * K)), dim3(256), 0, fs, t, nfar, F,
                           od.St, od.xh, od.tmp);
}

template <int D, int P, typename T>
static void far_out1(const ApplyPlan& a, const H2Tree& t, int F, const OpData<T>& od, int dtype, void* y,
                     hipStream_t st) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    const int64_t nrb = (a.cap + 63) / 64;
    const size_t lds = sizeof(T) * ((int64_t)(t.L + 1) * (K + EP));
    hipLaunchKernelGGL((k_far_out1<D, P, T>), dim3((unsigned)(a.nleaf * nrb), F), dim3(256), lds, st, a, t, F, od.tmp,
                       od.U, od.E, dtype, y);
}

// (dim, points) dispatch of the templates above for one operator precision T
template <typename T>
struct Single {
    template <int D, int P>
    static void chain(const ApplyPlan& a, const H2Tree& t, const UpPlan& up, int F, int64_t nfar, int dtype,
                      const void* x, const OpData<T>& od, unsigned int* tickets, hipStream_t fs) {
        far_chain1<D, P, T>(a, t, up, F, nfar, dtype, x, od, tickets, fs);
    }
    template <int D, int P>
    static void out(const ApplyPlan& a, const H2Tree& t, int F, const OpData<T>& od, int dtype, void* y,
                    hipStream_t st) {
        far_out1<D, P, T>(a, t, F, od, dtype, y, st);
    }
    // leaf-stage depth d0 (at most 3: 8 leaves, one wave each) and the deepest
    // upper-stage depth ds whose subtree fits 64 KB of LDS
    template <int D, int P>
    static void plan(const H2Tree& t, int64_t cap, UpPlan* up) {
        const size_t lim = 64 * 1024;
        up->d0 = t.L < 3 ? t.L : 3;
        while (up->d0 > 0 && up_tree_lds<D, P, T>(t, cap, up->d0, 1) > lim) --up->d0;
        up->ds = 1;
        while (up->ds < 16 && up_tree_lds<D, P, T>(t, cap, up->d0, up->ds + 1) <= lim) ++up->ds;
        up->ok = up_tree_lds<D, P, T>(t, cap, up->d0, up->ds) <= lim && KR<D, P>::K <= 64 && cap <= 256;
    }
};

UpPlan plan_up_tree(const H2Tree& t, int64_t cap, int prec) {
    UpPlan up{};
    if (prec == 0) FPDE_DISPATCH_DP(t.dim, t.p, Single<double>::template plan, t, cap, &up);
    else FPDE_DISPATCH_DP(t.dim, t.p, Single<float>::template plan, t, cap, &up);
    return up;
}

template <typename T>
static hipError_t apply_single_t(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, const UpPlan& up, int parts,
                                 int F, const double* csr_val, int64_t nfar, const OpData<T>& od, int dtype,
                                 const void* x, void* y, unsigned int* tickets, hipStream_t st, hipStream_t side,
                                 hipEvent_t fork, hipEvent_t join, hipEvent_t* ev) {
    const bool far = (parts & 8) != 0;
    if (ev) hipEventRecord(ev[0], st);
    hipStream_t fs = st;
    if (far && side != st) {
        hipEventRecord(fork, st);
        hipStreamWaitEvent(side, fork, 0);
        fs = side;
    }
    if (far) FPDE_DISPATCH_DP(t.dim, t.p, Single<T>::template chain, a, t, up, F, nfar, dtype, x, od, tickets, fs);
    if (ev) hipEventRecord(ev[1], fs);
    hipError_t e = launch_near_panel(a, pp, od.panel, (parts & 4) != 0, csr_val, F, dtype, x, y, st,
                                     ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
    if (e != hipSuccess) return e;
    if (far) {
        if (fs != st) {
            hipEventRecord(join, fs);
            hipStreamWaitEvent(st, join, 0);
        }
        FPDE_DISPATCH_DP(t.dim, t.p, Single<T>::template out, a, t, F, od, dtype, y, st);
    }
    if (ev) hipEventRecord(ev[4], st);
    return hipGetLastError();
}

hipError_t launch_apply_single(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, const UpPlan& up, int parts,
                               int F, const double* csr_val, int64_t nfar, const OpData<double>& od, int dtype,
                               const void* x, void* y, unsigned int* tickets, hipStream_t st, hipStream_t side,
                               hipEvent_t fork, hipEvent_t join, hipEvent_t* ev) {
    return apply_single_t<double>(a, t, pp, up, parts, F, csr_val, nfar, od, dtype, x, y, tickets, st, side, fork,
                                  join, ev);
}

hipError_t launch_apply_single(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, const UpPlan& up, int parts,
                               int F, const double* csr_val, int64_t nfar, const OpData<float>& od, int dtype,
                               const void* x, void* y, unsigned int* tickets, hipStream_t st, hipStream_t side,
                               hipEvent_t fork, hipEvent_t join, hipEvent_t* ev) {
    return apply_single_t<float>(a, t, pp, up, parts, F, csr_val, nfar, od, dtype, x, y, tickets, st, side, fork,
                                 join, ev);
}

}  // namespace fpde
