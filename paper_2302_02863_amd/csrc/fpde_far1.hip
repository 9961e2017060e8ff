// Far field of the one-vector apply after its upsweep: coupling sums per far
// target cluster, then the downsweep fused with the output (Sec. 5.2-5.3).
// Both run in the operator's precision T (FP32 data of a mixed operator
// accumulate in FP32 and are added to y in FP64).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_device.h"

namespace fpde {

constexpr int kFarThreads = 256;

// Coupling of far target cluster c (Sec. 5.2): z^(c) = sum over the far pairs
// (c, s) of S x^(s).  Pair slots of G lanes (lane alpha) each take every NS-th
// pair of c and accumulate S[alpha][beta] x^(s)[beta]; St holds S transposed
// ([beta][alpha]) so that the lanes read consecutive entries, and x^(s)[beta]
// is broadcast from lane beta of the slot.  The source index is loaded first
// (the x^ gather waits only for it), and the next pair's S is in flight while
// the current one is summed.  The slots are summed in a fixed order.  z^ of
// clusters that are not targets stays zero.
constexpr int kCoupleThreads = 512;
template <int D, int P, typename T>
__device__ __forceinline__ void couple(const H2Tree& t, int64_t c, int f, const T* St, const T* xh, T* zh, T* sred) {
    constexpr int K = KR<D, P>::K;
    constexpr int G = K <= 32 ? 32 : 64;   // lanes of a pair slot
    constexpr int NS = kCoupleThreads / G; // pair slots
    const int64_t nfar = t.far_ptr[t.ncl];
    const int64_t e0 = t.far_ptr[c], e1 = t.far_ptr[c + 1];
    const int sl = threadIdx.x / G, al = threadIdx.x % G;
    const int alc = al < K ? al : 0;
    const int base = (threadIdx.x & 63) & ~(G - 1);   // first lane of the slot within the wave
    const T* xf = xh + (int64_t)f * t.ncl * K;
    const T* Sf = St + (int64_t)f * nfar * K * K + alc;
    T acc = 0;
    int64_t e = e0 + sl;
    if (e < e1) {
        int64_t src = t.far_src[e];
        T sv[K];
#pragma unroll
        for (int b = 0; b < K; ++b) sv[b] = Sf[(e * K + b) * K];
        for (;;) {   // the lanes of a slot share e
            const T xv = al < K ? xf[src * K + al] : T(0);
            const int64_t en = e + NS;
            const bool more = en < e1;
            int64_t srcn = 0;
            T svn[K];
            if (more) {
                srcn = t.far_src[en];
#pragma unroll
                for (int b = 0; b < K; ++b) svn[b] = Sf[(en * K + b) * K];
            }
#pragma unroll
            for (int b = 0; b < K; ++b) acc += sv[b] * __shfl(xv, base + b, 64);
            if (!more) break;
            e = en;
            src = srcn;
#pragma unroll
            for (int b = 0; b < K; ++b) sv[b] = svn[b];
        }
    }
    sred[sl * G + al] = acc;
    __syncthreads();
    if (threadIdx.x < K) {
        T z = 0;
        for (int s = 0; s < NS; ++s) z += sred[s * G + threadIdx.x];
        zh[((int64_t)f * t.ncl + c) * K + threadIdx.x] = z;
    }
}

// One block per far target cluster tgt[b].
template <int D, int P, typename T>
__global__ __launch_bounds__(kCoupleThreads) void k_couple(H2Tree t, FarPlan fp, const T* St, const T* xh, T* zh) {
    __shared__ T sred[kCoupleThreads];
    couple<D, P, T>(t, fp.tgt[blockIdx.x], blockIdx.y, St, xh, zh, sred);
}

// Downsweep and output (Sec. 5.3): y[perm[row]] += U[row] . y^_leaf, where
// y^ of a cluster is its z^ plus the transfer of its parent's y^, from level
// ltop (the shallowest target) down.  One block per (leaf, 64 rows, field),
// 4 lanes per row; the basis rows, output indices, old y values, transfers
// and z^ of the root path are all fetched before the walk.
template <int D, int P, typename T>
__global__ __launch_bounds__(kFarThreads) void k_far_out(ApplyPlan a, H2Tree t, int ltop, const T* zh, const T* U,
                                                           const T* E, int dtype, void* y) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    extern __shared__ __align__(16) unsigned char sraw[];
    const int L = t.L, nlev = L + 1 - ltop;
    T* sy = (T*)sraw;                       // [nlev][K]
    T* sE = sy + (int64_t)nlev * K;         // [nlev][EP]
    const int f = blockIdx.y;
    const int64_t nrb = (a.cap + 63) / 64;
    const int64_t li = blockIdx.x / nrb;
    const int rb = (int)(blockIdx.x % nrb);
    const int64_t leafc = t.first_leaf + li;
    const int64_t lb = a.leaf_beg[li], nt = a.leaf_beg[li + 1] - lb;
    const int g = threadIdx.x & 3;
    const int64_t it = (int64_t)rb * 64 + (threadIdx.x >> 2);
    const bool ok = it < nt;
    T u[(K + 3) / 4];
#pragma unroll
    for (int q = 0; q < (K + 3) / 4; ++q) u[q] = (ok && 4 * q + g < K) ? U[(lb + it) * K + 4 * q + g] : T(0);
    int64_t dst = 0;
    double yold = 0.0;
    if (ok && g == 0) {
        dst = (int64_t)f * a.N + a.perm[lb + it];
        yold = ldx(y, dst, dtype);
    }
    const T* zf = zh + (int64_t)f * t.ncl * K;
    for (int i = threadIdx.x; i < nlev * K; i += blockDim.x) {
        const int lev = ltop + i / K;
        sy[i] = zf[(((leafc + 1) >> (L - lev)) - 1) * K + i % K];
    }
    for (int i = threadIdx.x; i < nlev * EP; i += blockDim.x) {
        const int lev = ltop + i / EP;
        sE[i] = E[(((leafc + 1) >> (L - lev)) - 1) * EP + i % EP];
    }
    __syncthreads();
    for (int l = 1; l < nlev; ++l) {
        for (int i = threadIdx.x; i < K; i += blockDim.x)
            sy[l * K + i] += down_t<D, P, T>(sE + l * EP, sy + (l - 1) * K, i, 1);
        __syncthreads();
    }
    const T* cur = sy + (int64_t)(nlev - 1) * K;
    T acc = 0;
#pragma unroll
    for (int q = 0; q < (K + 3) / 4; ++q)
        if (4 * q + g < K) acc += u[q] * cur[4 * q + g];
    acc += __shfl_xor(acc, 1, 4);
    acc += __shfl_xor(acc, 2, 4);
    if (ok && g == 0) {
        if (dtype == 0) ((double*)y)[dst] = yold + (double)acc;
        else ((float*)y)[dst] = (float)(yold + (double)acc);
    }
}

// far-field part of a near block: y^ and transfers of the root path from ltop
template <int D, int P, typename T>
static size_t path_lds(const H2Tree& t, int ltop) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    return sizeof(T) * (size_t)((int64_t)(t.L + 1 - ltop) * (K + EP));
}

template <typename T>
struct Far1 {
    template <int D, int P>
    static void far_out(const ApplyPlan& a, const H2Tree& t, const FarPlan& fp, int F, const OpData<T>& od, int dtype,
                        void* y, hipStream_t st) {
        hipLaunchKernelGGL((k_couple<D, P, T>), dim3((unsigned)fp.ntgt, F), dim3(kCoupleThreads), 0, st, t, fp, od.St,
                           od.xh, od.zh);
        const int64_t nrb = (a.cap + 63) / 64;
        const size_t lds = path_lds<D, P, T>(t, fp.ltop);
        hipLaunchKernelGGL((k_far_out<D, P, T>), dim3((unsigned)(a.nleaf * nrb), F), dim3(kFarThreads), lds, st, a,
                           t, fp.ltop, od.zh, od.U, od.E, dtype, y);
    }
};

template <typename T>
static hipError_t far_single_t(const ApplyPlan& a, const H2Tree& t, const FarPlan& fp, int F, const OpData<T>& od,
                               int dtype, void* y, hipStream_t st) {
    FPDE_DISPATCH_DP(t.dim, t.p, Far1<T>::template far_out, a, t, fp, F, od, dtype, y, st);
    return hipGetLastError();
}

hipError_t launch_far_single(const ApplyPlan& a, const H2Tree& t, const FarPlan& fp, int F, const OpData<double>& od,
                             int dtype, void* y, hipStream_t st) {
    return far_single_t<double>(a, t, fp, F, od, dtype, y, st);
}

hipError_t launch_far_single(const ApplyPlan& a, const H2Tree& t, const FarPlan& fp, int F, const OpData<float>& od,
                             int dtype, void* y, hipStream_t st) {
    return far_single_t<float>(a, t, fp, F, od, dtype, y, st);
}

}  // namespace fpde
