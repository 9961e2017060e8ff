// Far field of the one-vector apply after its upsweep: coupling sums per far
// target cluster, then the downsweep fused with the output (Sec. 5.2-5.3).
// Partial coupling sums that one block hands to another are stored and loaded
// as agent-scope atomics (put / get), coherent across the XCDs' L2 caches.
// Both run in the operator's precision T (FP32 data of a mixed operator
// accumulate in FP32 and are added to y in FP64).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_device.h"

namespace fpde {

constexpr int kFarThreads = 256;

// Coupling (Sec. 5.2): z^(c) = sum over the far pairs (c, s) of S x^(s) for
// every far target c.  The pairs of a target are cut into chunks of at most
// NS pairs (their source clusters in the chunk record, so that the x^ gather
// goes out with the S loads), one block per chunk, one pair per slot of G
// lanes (lane alpha):
// S[alpha][beta] x^(s)[beta] summed over beta, St holding S transposed
// ([beta][alpha]) so that the lanes read consecutive entries, x^(s)[beta]
// broadcast from lane beta of the slot.  The slots are summed in a fixed
// order.  A target with one chunk writes z^ at once; otherwise each chunk
// stores its partial at agent scope, counts itself on the target's ticket,
// and the last one sums the partials in chunk order and resets the ticket.
// z^ of clusters that are not targets stays zero.
constexpr int kCoupleThreads = 512;
template <int D, int P, typename T>
__global__ __launch_bounds__(kCoupleThreads) void k_couple(H2Tree t, FarPlan fp, const T* St, const T* xh, T* zh,
                                                           T* zp) {
    constexpr int K = KR<D, P>::K;
    constexpr int G = K <= 32 ? 32 : 64;   // lanes of a pair slot
    constexpr int NS = kCoupleThreads / G; // pair slots
    __shared__ T sred[kCoupleThreads];
    __shared__ int s_last;
    const int f = blockIdx.y;
    const int64_t* ck = fp.chunks + kChunkWords * (int64_t)blockIdx.x;
    const int64_t c = ck[0], e0 = ck[1], e1 = ck[2];
    const int ci = (int)(ck[3] >> 32), nch = (int)(ck[3] & 0xffffffff);
    const int64_t nfar = t.far_ptr[t.ncl];
    const int sl = threadIdx.x / G, al = threadIdx.x % G;
    const int base = (threadIdx.x & 63) & ~(G - 1);   // first lane of the slot within the wave
    const int64_t e = e0 + sl;
    T acc = 0;
    if (e < e1) {   // the lanes of a slot share e
        const int64_t src = ck[4 + sl];   // the source cluster, carried by the chunk record
        const T* S = St + ((int64_t)f * nfar + e) * K * K + (al < K ? al : 0);
        T sv[K];
#pragma unroll
        for (int b = 0; b < K; ++b) sv[b] = S[b * K];
        const T xv = al < K ? xh[((int64_t)f * t.ncl + src) * K + al] : T(0);
#pragma unroll
        for (int b = 0; b < K; ++b) acc += sv[b] * __shfl(xv, base + b, 64);
    }
    sred[sl * G + al] = acc;
    __syncthreads();
    T z = 0;
    if (threadIdx.x < K)
        for (int s = 0; s < NS; ++s) z += sred[s * G + threadIdx.x];
    T* zc = zh + ((int64_t)f * t.ncl + c) * K;
    if (nch == 1) {
        if (threadIdx.x < K) zc[threadIdx.x] = z;
        return;
    }
    T* zpf = zp + (int64_t)f * fp.nchunks * K;
    if (threadIdx.x < K) put(&zpf[(int64_t)blockIdx.x * K + threadIdx.x], z);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    unsigned int* tk = &fp.ctk[(int64_t)f * t.ncl + c];
    if (threadIdx.x == 0)
        s_last = __hip_atomic_fetch_add(tk, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned int)nch - 1;
    __syncthreads();
    if (!s_last) return;
    if (threadIdx.x == 0) __hip_atomic_store(tk, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x < K) {
        const int64_t first = (int64_t)blockIdx.x - ci;   // chunks of a target are consecutive
        T s = 0;
        for (int j = 0; j < nch; ++j) s += get(&zpf[(first + j) * K + threadIdx.x]);
        zc[threadIdx.x] = s;
    }
}

// Downsweep and output (Sec. 5.3): y[perm[row]] += U[row] . y^_leaf, where
// y^ of a cluster is its z^ plus the transfer of its parent's y^, from level
// ltop (the shallowest target) down.  One block per (leaf, 64 rows, field),
// 256 threads, 4 lanes per row.  Rows are addressed by leaf slot (leaf li,
// row i: slot li * cap + i, padded), so the basis rows (Upad) and output
// indices (perm_pad, -1 for padding) are loaded at once; they, the old y
// values, the transfers and z^ of the root path are all fetched before the
// walk.
template <int D, int P, typename T>
__global__ __launch_bounds__(kFarThreads) void k_far_out(ApplyPlan a, H2Tree t, int ltop, const T* zh,
                                                           const T* Upad, const int64_t* perm_pad, const T* E,
                                                           int dtype, void* y, CgFuse cg) {
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
    // z^ and transfers of the root path depend on no load: fetched first, into
    // registers, and written to LDS once the dependent loads are in flight
    const T* zf = zh + (int64_t)f * t.ncl * K;
    constexpr int kZR = 2, kER = 4;   // entries per thread held in registers
    T zr[kZR], er[kER];
#pragma unroll
    for (int q = 0; q < kZR; ++q) {
        const int i = threadIdx.x + q * kFarThreads;
        zr[q] = i < nlev * K ? zf[(((leafc + 1) >> (L - (ltop + i / K))) - 1) * K + i % K] : T(0);
    }
#pragma unroll
    for (int q = 0; q < kER; ++q) {
        const int i = threadIdx.x + q * kFarThreads;
        er[q] = i < nlev * EP ? E[(((leafc + 1) >> (L - (ltop + i / EP))) - 1) * EP + i % EP] : T(0);
    }
    // leaf slot rows: the basis rows and output indices need no leaf range first
    const int g = threadIdx.x & 3;
    const int64_t it = (int64_t)rb * 64 + (threadIdx.x >> 2);
    const int64_t slot = li * a.cap + it;
    const bool in = it < a.cap;
    T u[(K + 3) / 4];
#pragma unroll
    for (int q = 0; q < (K + 3) / 4; ++q) u[q] = (in && 4 * q + g < K) ? Upad[slot * K + 4 * q + g] : T(0);
    const int64_t pr = in ? perm_pad[slot] : -1;
    const bool ok = pr >= 0;
    int64_t dst = 0;
    double yold = 0.0, pv = 0.0;
    if (ok && g == 0) {
        dst = (int64_t)f * a.N + pr;
        yold = ldx(y, dst, dtype);
        if (cg.p) pv = cg.p[dst];
    }
#pragma unroll
    for (int q = 0; q < kZR; ++q) {
        const int i = threadIdx.x + q * kFarThreads;
        if (i < nlev * K) sy[i] = zr[q];
    }
#pragma unroll
    for (int q = 0; q < kER; ++q) {
        const int i = threadIdx.x + q * kFarThreads;
        if (i < nlev * EP) sE[i] = er[q];
    }
    for (int i = threadIdx.x + kZR * kFarThreads; i < nlev * K; i += blockDim.x)   // very deep trees
        sy[i] = zf[(((leafc + 1) >> (L - (ltop + i / K))) - 1) * K + i % K];
    for (int i = threadIdx.x + kER * kFarThreads; i < nlev * EP; i += blockDim.x)
        sE[i] = E[(((leafc + 1) >> (L - (ltop + i / EP))) - 1) * EP + i % EP];
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
    double yn = 0.0;
    if (ok && g == 0) {
        yn = yold + (double)acc;
        if (dtype == 0) {
            ((double*)y)[dst] = yn;
        } else {
            ((float*)y)[dst] = (float)yn;
            yn = (double)(float)yn;
        }
    }
    if (cg.p) {   // fused CG iteration: the block's share of p . y (tree in LDS, fixed order)
        __shared__ double red[kFarThreads];
        red[threadIdx.x] = yn * pv;
        __syncthreads();
        for (int s = kFarThreads / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            cg.part[(int64_t)f * gridDim.x + blockIdx.x] = red[0];
            if (blockIdx.x == 0) {
                cg.rr[f] = cg.rr_next[f];
                cg.active[f] = cg.active_next[f];
                if (f == 0) cg.n_active[0] = 0;
            }
        }
    }
}

// far-field part of a near block: y^ and transfers of the root path from ltop
template <int D, int P, typename T>
static size_t path_lds(const H2Tree& t, int ltop) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    return sizeof(T) * (size_t)((int64_t)(t.L + 1 - ltop) * (K + EP));
}

// Leaf-slot copies for the output kernel: Upad[li * cap + i] = U[leaf_beg[li] + i]
// and perm_pad[li * cap + i] = perm[leaf_beg[li] + i] for i < the leaf's rows,
// zeros and -1 beyond.
FPDE_KERNEL void k_pad_rows(int64_t nleaf, int64_t cap, int k, const int64_t* leaf_beg, const double* U,
                            const int64_t* perm, double* Upad, int64_t* perm_pad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaf * cap) return;
    const int64_t li = i / cap, it = i % cap;
    const int64_t lb = leaf_beg[li], nt = leaf_beg[li + 1] - lb;
    const bool ok = it < nt;
    perm_pad[i] = ok ? perm[lb + it] : -1;
    for (int q = 0; q < k; ++q) Upad[i * k + q] = ok ? U[(lb + it) * k + q] : 0.0;
}

// ELL values of B + M by leaf slot: out[f][i] = val[f][src[i]], 0 where src[i] < 0
FPDE_KERNEL void k_ell_values(int64_t n, int F, int64_t nnz, const int64_t* src, const double* val, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t e = src[i];
    for (int f = 0; f < F; ++f) out[(int64_t)f * n + i] = e >= 0 ? val[(int64_t)f * nnz + e] : 0.0;
}

hipError_t launch_ell_values(int64_t n, int F, int64_t nnz, const int64_t* src, const double* val, double* out,
                             hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ell_values, dim3(grid1(n)), dim3(256), 0, st, n, F, nnz, src, val, out);
    return hipGetLastError();
}

hipError_t launch_pad_rows(int64_t nleaf, int64_t cap, int k, const int64_t* leaf_beg, const double* U,
                           const int64_t* perm, double* Upad, int64_t* perm_pad, hipStream_t st) {
    if (nleaf * cap == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pad_rows, dim3(grid1(nleaf * cap)), dim3(256), 0, st, nleaf, cap, k, leaf_beg, U, perm, Upad,
                       perm_pad);
    return hipGetLastError();
}

template <typename T>
struct Far1 {
    template <int D, int P>
    static void couple(const H2Tree& t, const FarPlan& fp, int F, const OpData<T>& od, hipStream_t st) {
        hipLaunchKernelGGL((k_couple<D, P, T>), dim3((unsigned)fp.nchunks, F), dim3(kCoupleThreads), 0, st, t, fp,
                           od.St, od.xh, od.zh, od.zp);
    }
    template <int D, int P>
    static void out(const ApplyPlan& a, const H2Tree& t, const FarPlan& fp, int F, const OpData<T>& od, int dtype,
                    void* y, hipStream_t st) {
        const int64_t nrb = (a.cap + 63) / 64;
        const size_t lds = path_lds<D, P, T>(t, fp.ltop);
        hipLaunchKernelGGL((k_far_out<D, P, T>), dim3((unsigned)(a.nleaf * nrb), F), dim3(kFarThreads), lds, st, a,
                           t, fp.ltop, od.zh, od.Upad, fp.perm_pad, od.E, dtype, y, fp.cg);
    }
};

hipError_t launch_couple_single(const H2Tree& t, const FarPlan& fp, int F, const OpData<double>& od, hipStream_t st) {
    FPDE_DISPATCH_DP(t.dim, t.p, Far1<double>::template couple, t, fp, F, od, st);
    return hipGetLastError();
}
hipError_t launch_couple_single(const H2Tree& t, const FarPlan& fp, int F, const OpData<float>& od, hipStream_t st) {
    FPDE_DISPATCH_DP(t.dim, t.p, Far1<float>::template couple, t, fp, F, od, st);
    return hipGetLastError();
}
hipError_t launch_out_single(const ApplyPlan& a, const H2Tree& t, const FarPlan& fp, int F, const OpData<double>& od,
                             int dtype, void* y, hipStream_t st) {
    FPDE_DISPATCH_DP(t.dim, t.p, Far1<double>::template out, a, t, fp, F, od, dtype, y, st);
    return hipGetLastError();
}
hipError_t launch_out_single(const ApplyPlan& a, const H2Tree& t, const FarPlan& fp, int F, const OpData<float>& od,
                             int dtype, void* y, hipStream_t st) {
    FPDE_DISPATCH_DP(t.dim, t.p, Far1<float>::template out, a, t, fp, F, od, dtype, y, st);
    return hipGetLastError();
}

}  // namespace fpde
