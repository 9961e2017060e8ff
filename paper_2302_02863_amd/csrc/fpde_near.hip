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
// Y[rows, r0:r0+64] = Panel[rows, :] X[cols, r0:r0+64] + (B+M)[rows, :] X
// (+ U[rows, :] Y^_leaf[:, r0:r0+64] when the far field's coefficients are given),
// one block per (leaf, 64-row tile, 64-column tile of right-hand sides, field).
// The panel times the gathered rows of X is a dense GEMM of 64 x 64 x
// pstride; four waves each own a 32 x 32 quarter of the tile:
//   FP32 operator data: v_mfma_f32_32x32x2f32, two k per step (lane l supplies
//     A[l%32][l/32], B[l/32][l%32]; accumulator v holds C[8(v/4) + 4(l/32) + v%4][l%32]);
//   FP64: 2 x 2 tiles of v_mfma_f64_16x16x4f64, four k per step (A[l%16][l/16],
//     B[l/16][l%16]; accumulator v holds C[l/16 + 4v][l%16]).
// Chunks of 32 panel columns and the matching 32 rows of X go global ->
// registers -> LDS with 16-byte loads, so that every wave instruction reads
// whole cache lines; the next chunk's loads are in flight during the MFMAs.
// The panel chunk is stored in LDS with its columns permuted (column KS*s + g
// of the chunk at position g*(32/KS) + s, KS = k per step), so each lane reads
// the A values of all its steps with 16-byte LDS reads; X stays row-major.  The
// leaf's panel column list is staged in LDS once.  The far field's leaf output
// U Y^ is one more chunk of the same GEMM (A = the tile's basis rows by leaf
// slot, B = the leaf's coefficients, both padded to 32).  The tile then goes to
// LDS and each thread adds the B + M row (FP64; the ELL form by leaf slot when
// the operator holds it) for one right-hand side and writes y.
typedef float fpde_f32x16 __attribute__((ext_vector_type(16)));
typedef double fpde_f64x4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int kMT = 64, kNT = 64, kKC = 32;
constexpr int kCS = kNT + 1;          // LDS row stride of the output tile
constexpr int kStageCols = 4096;      // longest panel column list staged in LDS
template <typename T>
struct MM;
template <>
struct MM<float> {
    static constexpr int KS = 2;          // k per MFMA step
    static constexpr int SA = kKC + 4;    // LDS row strides: 16-byte aligned rows, no bank
    static constexpr int SB = kNT + 32;   // conflicts for the MFMA operand reads
    using V = float4;
};
template <>
struct MM<double> {
    static constexpr int KS = 4;
    static constexpr int SA = kKC + 2;
    static constexpr int SB = kNT + 16;
    using V = double2;
};
template <typename T>
constexpr size_t mm_tile_elems() {
    const size_t g = (size_t)kMT * MM<T>::SA + (size_t)kKC * MM<T>::SB;
    const size_t c = (size_t)kMT * kCS;
    return g > c ? g : c;
}

__device__ __forceinline__ double bcast(double v, int l) {   // v of lane l (wave-uniform l)
    const int64_t b = __double_as_longlong(v);
    return __longlong_as_double((int64_t)(uint32_t)__builtin_amdgcn_readlane((int)b, l) |
                                ((int64_t)__builtin_amdgcn_readlane((int)(b >> 32), l) << 32));
}
}  // namespace

// B + M rows of a tile from the ELL form by leaf slot, W entries a row (W <= 32;
// a row's padding entries repeat its first column with the value 0):
// lane e < W of the wave loads entry e (column and value) of the row, so one
// load round trip fetches a whole row; the wave then broadcasts the entries
// with readlane and issues all W gathers of x at once, and the next row's
// entries load while this row's gathers are in flight.  Rows rr = wv, wv + 4,
// ... of the tile; lane = right-hand side r0 + lane (stored only when < R).
template <int W, typename XT, typename T>
__device__ __forceinline__ void ell_rows(const ApplyPlan& a, const PanelPlan& pp, const int32_t* __restrict__ ell_col,
                                         const double* __restrict__ ell_val, const T* Cs, int64_t li, int64_t row0,
                                         int wv, int lane, int f, int R, int r0, int64_t xo,
                                         const XT* __restrict__ x, XT* __restrict__ y) {
    const int64_t nslot = a.nleaf * a.cap;
    const int r = r0 + lane;
    const bool rok = r < R;
    const int rx = rok ? r : r0;   // lanes past R gather a valid entry and store nothing
    auto load = [&](int rr, int& jc, double& vv, int64_t& dst) {
        const int64_t it = row0 + rr;
        jc = -1;
        vv = 0.0;
        dst = -1;
        if (rr < kMT && it < a.cap) {
            const int64_t slot = li * a.cap + it;
            dst = pp.perm_pad[slot];
            if (lane < W) {
                jc = ell_col[slot * W + lane];
                vv = ell_val[((int64_t)f * nslot + slot) * W + lane];
            }
        }
    };
    int jc;
    double vv;
    int64_t dst;
    load(wv, jc, vv, dst);
    for (int rr = wv; rr < kMT; rr += 4) {
        if (dst < 0) break;   // the same in every lane; slots past the leaf's rows come last
        XT xg[W];
#pragma unroll
        for (int e = 0; e < W; ++e) xg[e] = x[xo + (int64_t)__builtin_amdgcn_readlane(jc, e) * R + rx];
        const int64_t d = dst;
        const double v0 = vv;
        load(rr + 4, jc, vv, dst);   // the next row's entries, in flight during the sums
        double acc[4] = {(double)Cs[rr * kCS + lane], 0.0, 0.0, 0.0};
#pragma unroll
        for (int e = 0; e < W; ++e) acc[e & 3] += bcast(v0, e) * (double)xg[e];
        if (rok) y[xo + d * R + r] = (XT)(acc[0] + ((acc[1] + acc[2]) + acc[3]));
    }
}

template <int W, typename T>
__device__ __forceinline__ bool ell_rows_w(int w, const ApplyPlan& a, const PanelPlan& pp,
                                           const int32_t* __restrict__ ell_col, const double* __restrict__ ell_val,
                                           const T* Cs, int64_t li, int64_t row0, int wv, int lane, int f, int R,
                                           int r0, int64_t xo, int dtype, const void* x, void* y) {
    if (w != W) return false;
    if (dtype == 0)
        ell_rows<W, double, T>(a, pp, ell_col, ell_val, Cs, li, row0, wv, lane, f, R, r0, xo, (const double*)x,
                               (double*)y);
    else
        ell_rows<W, float, T>(a, pp, ell_col, ell_val, Cs, li, row0, wv, lane, f, R, r0, xo, (const float*)x,
                              (float*)y);
    return true;
}

template <typename T>
__global__ __launch_bounds__(256, 3) void k_near_mm(ApplyPlan a, PanelPlan pp, const T* __restrict__ panel,
                                                 int use_near, const double* __restrict__ csr_val,
                                                 const int32_t* __restrict__ ell_col,
                                                 const double* __restrict__ ell_val, int F, int R, int dtype,
                                                 const void* __restrict__ x, void* __restrict__ y, MmFar<T> fo) {
    constexpr int KS = MM<T>::KS, NS = kKC / KS, SA = MM<T>::SA, SB = MM<T>::SB;
    constexpr int VW = 16 / sizeof(T);               // elements of a 16-byte vector
    constexpr int NA = kMT * kKC / VW / 256;          // panel vectors per thread and chunk
    using V = typename MM<T>::V;
    extern __shared__ __align__(16) unsigned char sraw[];
    T* Ap = (T*)sraw;                       // [kMT][SA], permuted columns
    T* Bx = Ap + kMT * SA;                  // [kKC][SB]
    T* Cs = (T*)sraw;                       // [kMT][kCS] after the GEMM
    int32_t* pcs = (int32_t*)(sraw + sizeof(T) * mm_tile_elems<T>());   // staged panel column dofs
    const int64_t nrt = (a.cap + kMT - 1) / kMT, nct = (R + kNT - 1) / kNT;
    const int64_t lb = xcd_block((int64_t)blockIdx.y * gridDim.x + blockIdx.x, (int64_t)gridDim.x * gridDim.y);
    const int f = (int)(lb / gridDim.x);
    const int64_t bx = lb % gridDim.x;
    const int64_t li = bx / (nrt * nct);
    const int64_t rem = bx % (nrt * nct);
    const int64_t row0 = (rem / nct) * kMT;   // first panel row of the tile
    const int r0 = (int)(rem % nct) * kNT;    // first right-hand side
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;   // the wave's quarter
    const int64_t xo = (int64_t)f * a.N * R;
    fpde_f32x16 c32 = {0};
    fpde_f64x4 c64[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
    // MFMA steps over the chunk in LDS (32 columns of A, 32 rows of B)
    auto mma = [&]() {
        if constexpr (sizeof(T) == 4) {
            const int g = lane >> 5, i32 = lane & 31;
            const float4* ar = (const float4*)(Ap + (wr + i32) * SA + g * NS);
            float4 a4[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) a4[q] = ar[q];
            const float av[16] = {a4[0].x, a4[0].y, a4[0].z, a4[0].w, a4[1].x, a4[1].y, a4[1].z, a4[1].w,
                                  a4[2].x, a4[2].y, a4[2].z, a4[2].w, a4[3].x, a4[3].y, a4[3].z, a4[3].w};
#pragma unroll
            for (int st = 0; st < NS; ++st) {
                const float bv = Bx[(KS * st + g) * SB + wc + i32];
                c32 = __builtin_amdgcn_mfma_f32_32x32x2f32(av[st], bv, c32, 0, 0, 0);
            }
        } else {
            const int g = lane >> 4, i16 = lane & 15;
            const double2* ar0 = (const double2*)(Ap + (wr + i16) * SA + g * NS);
            const double2* ar1 = (const double2*)(Ap + (wr + 16 + i16) * SA + g * NS);
#pragma unroll
            for (int q = 0; q < NS / 2; ++q) {   // two steps per 16-byte read of A
                const double2 a0 = ar0[q], a1 = ar1[q];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int st = 2 * q + h;
                    const double av[2] = {h ? a0.y : a0.x, h ? a1.y : a1.x};
                    double bv[2];
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj) bv[tj] = Bx[(KS * st + g) * SB + wc + 16 * tj + i16];
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                        for (int tj = 0; tj < 2; ++tj)
                            c64[ti][tj] =
                                __builtin_amdgcn_mfma_f64_16x16x4f64(av[ti], bv[tj], c64[ti][tj], 0, 0, 0);
                }
            }
        }
    };
    if (use_near) {
        const int64_t ps = pp.pstride[li];
        const int32_t* pcg = pp.pcols_pad + li * pp.max_stride;   // -1 past the leaf's columns
        const bool staged = pp.max_stride <= kStageCols;
        if (staged) {
            for (int64_t c = tid; c < ps; c += 256) pcs[c] = pcg[c];
            __syncthreads();
        }
        const T* pl = panel + (int64_t)f * pp.poff[a.nleaf] + pp.poff[li];
        const bool xv = (R & 3) == 0;   // X rows start 16-byte aligned
        V pa[NA];
        T xa[8];
        // X chunk element k of this thread: FP32 source (and the scalar fallback)
        // 2 x 4 consecutive right-hand sides, FP64 source 4 x 2
        auto xpos32 = [&](int i, int& xr, int& rv) { const int v = tid + 256 * i; xr = v >> 4; rv = (v & 15) * 4; };
        auto xpos64 = [&](int i, int& xr, int& rv) { const int v = tid + 256 * i; xr = v >> 5; rv = (v & 31) * 2; };
        auto fetch = [&](int64_t k0) {   // global -> registers (next chunk, in flight during the MFMAs)
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int v = tid + 256 * i;
                const int64_t row = row0 + v / (kKC / VW), col = k0 + (v % (kKC / VW)) * VW;
                if (row < a.cap && col < ps) pa[i] = *(const V*)(pl + row * ps + col);
                else pa[i] = V{};
            }
            if (xv && dtype == 1) {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    int xr, rv;
                    xpos32(i, xr, rv);
                    const int64_t c = k0 + xr;
                    const int dof = c < ps ? (staged ? pcs[c] : pcg[c]) : -1;
                    float4 q = {0.f, 0.f, 0.f, 0.f};
                    if (dof >= 0 && r0 + rv < R) q = *(const float4*)((const float*)x + xo + (int64_t)dof * R + r0 + rv);
                    xa[4 * i] = (T)q.x; xa[4 * i + 1] = (T)q.y; xa[4 * i + 2] = (T)q.z; xa[4 * i + 3] = (T)q.w;
                }
            } else if (xv) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int xr, rv;
                    xpos64(i, xr, rv);
                    const int64_t c = k0 + xr;
                    const int dof = c < ps ? (staged ? pcs[c] : pcg[c]) : -1;
                    double2 q = {0.0, 0.0};
                    if (dof >= 0 && r0 + rv < R) q = *(const double2*)((const double*)x + xo + (int64_t)dof * R + r0 + rv);
                    xa[2 * i] = (T)q.x; xa[2 * i + 1] = (T)q.y;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    int xr, rv;
                    xpos32(i, xr, rv);
                    const int64_t c = k0 + xr;
                    const int dof = c < ps ? (staged ? pcs[c] : pcg[c]) : -1;
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        xa[4 * i + j] = (dof >= 0 && r0 + rv + j < R)
                                            ? (T)ldx(x, xo + (int64_t)dof * R + r0 + rv + j, dtype) : T(0);
                }
            }
        };
        fetch(0);
        for (int64_t k0 = 0; k0 < ps; k0 += kKC) {
            __syncthreads();   // the previous chunk's MFMAs are done with the LDS tiles
            // panel chunk -> LDS, columns permuted
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int v = tid + 256 * i;
                const int row = v / (kKC / VW), c = (v % (kKC / VW)) * VW;
                if constexpr (sizeof(T) == 4) {   // columns c..c+3 = (g 0, s), (1, s), (0, s+1), (1, s+1)
                    const int s0 = c / 2;
                    *(float2*)(Ap + row * SA + s0) = float2{pa[i].x, pa[i].z};
                    *(float2*)(Ap + row * SA + NS + s0) = float2{pa[i].y, pa[i].w};
                } else {                          // columns c, c+1 = (c%4, c/4), (c%4 + 1, c/4)
                    Ap[row * SA + (c % 4) * NS + c / 4] = pa[i].x;
                    Ap[row * SA + (c % 4 + 1) * NS + c / 4] = pa[i].y;
                }
            }
            // X chunk -> LDS, row-major
            if (xv && dtype != 1) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int xr, rv;
                    xpos64(i, xr, rv);
                    Bx[xr * SB + rv] = xa[2 * i];
                    Bx[xr * SB + rv + 1] = xa[2 * i + 1];
                }
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    int xr, rv;
                    xpos32(i, xr, rv);
#pragma unroll
                    for (int j = 0; j < 4; ++j) Bx[xr * SB + rv + j] = xa[4 * i + j];
                }
            }
            __syncthreads();
            if (k0 + kKC < ps) fetch(k0 + kKC);
            mma();
        }
    }
    if (fo.yh) {
        // the far field's leaf output U_leaf Y^_leaf as one more chunk: A = the tile's rows of
        // the bases by leaf slot, B = the leaf's coefficients Y^ (alpha, beta padded to 32, K <= 32)
        const T* yl = fo.yh + (((int64_t)f * fo.ncl + fo.first_leaf + li) * fo.K) * R + r0;
        const int ar_ = tid >> 2, ac_ = (tid & 3) * 8;    // A: row, first of 8 columns
        const int br_ = tid >> 3, bc_ = (tid & 7) * 8;    // B: row (alpha), first of 8 right-hand sides
        const int64_t urow = row0 + ar_;
        T ua[8], ya[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            ua[j] = (urow < a.cap && ac_ + j < fo.K) ? fo.Upad[(li * a.cap + urow) * fo.K + ac_ + j] : T(0);
            ya[j] = (br_ < fo.K && r0 + bc_ + j < R) ? yl[(int64_t)br_ * R + bc_ + j] : T(0);
        }
        __syncthreads();   // the last panel chunk's MFMAs are done with the LDS tiles
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int col = ac_ + j;
            Ap[ar_ * SA + (col % KS) * NS + col / KS] = ua[j];
            Bx[br_ * SB + bc_ + j] = ya[j];
        }
        __syncthreads();
        mma();
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
    // B + M rows and the output: thread -> one right-hand side, rows strided by
    // 4; a wave shares each row
    if (ell_val) {
        const int w = pp.ell_w;
#define FPDE_ELL_W(W_) ell_rows_w<W_, T>(w, a, pp, ell_col, ell_val, Cs, li, row0, wv, lane, f, R, r0, xo, dtype, x, y)
        if (FPDE_ELL_W(4) || FPDE_ELL_W(8) || FPDE_ELL_W(12) || FPDE_ELL_W(16) || FPDE_ELL_W(20) || FPDE_ELL_W(24) ||
            FPDE_ELL_W(28) || FPDE_ELL_W(32))
            return;
#undef FPDE_ELL_W
    }
    const int rc = tid & 63;
    const int r = r0 + rc;
    if (r >= R) return;
    const int64_t nslot = a.nleaf * a.cap;
    for (int rr = wv; rr < kMT; rr += 4) {
        const int64_t it = row0 + rr;
        if (it >= a.cap) break;
        const int64_t slot = li * a.cap + it;
        const int64_t dst = pp.perm_pad[slot];
        if (dst < 0) break;   // slots past the leaf's rows come last
        double acc = (double)Cs[rr * kCS + rc];
        if (ell_val) {
            const int w = pp.ell_w;   // a multiple of 4
            const int32_t* ec = ell_col + slot * w;
            const double* ev = ell_val + ((int64_t)f * nslot + slot) * w;
            double s1 = 0.0, s2 = 0.0, s3 = 0.0;
            for (int e = 0; e < w; e += 4) {   // four independent gathers in flight
                const int j0 = ec[e], j1 = ec[e + 1], j2 = ec[e + 2], j3 = ec[e + 3];
                if (j0 >= 0) acc += ev[e] * ldx(x, xo + (int64_t)j0 * R + r, dtype);
                if (j1 >= 0) s1 += ev[e + 1] * ldx(x, xo + (int64_t)j1 * R + r, dtype);
                if (j2 >= 0) s2 += ev[e + 2] * ldx(x, xo + (int64_t)j2 * R + r, dtype);
                if (j3 >= 0) s3 += ev[e + 3] * ldx(x, xo + (int64_t)j3 * R + r, dtype);
            }
            acc += (s1 + s2) + s3;
        } else if (csr_val) {
            const double* v = csr_val + (int64_t)f * a.nnz;
            const int64_t row = a.leaf_beg[li] + it;
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
        const int64_t o = xo + dst * R + r;
        if (dtype == 0) ((double*)y)[o] = acc;
        else ((float*)y)[o] = (float)acc;
    }
}

template <typename T>
static hipError_t near_mm_t(const ApplyPlan& a, const PanelPlan& pp, const T* panel, int use_near,
                            const double* csr_val, int F, int R, int dtype, const void* x, void* y, hipStream_t st,
                            hipEvent_t e0, hipEvent_t e1, const MmFar<T>& fo) {
    const int64_t nrt = (a.cap + kMT - 1) / kMT, nct = (R + kNT - 1) / kNT;
    size_t lds = sizeof(T) * mm_tile_elems<T>();
    if (use_near && pp.max_stride <= kStageCols) lds += sizeof(int32_t) * (size_t)pp.max_stride;
    const dim3 grid((unsigned)(a.nleaf * nrt * nct), F);
    // the ELL rows hold B + M; other subsets of the near field read the CSR
    const int32_t* ec = pp.ell_val ? pp.ell_col : nullptr;
    if (e0)
        hipExtLaunchKernelGGL(k_near_mm<T>, grid, dim3(256), lds, st, e0, e1, 0, a, pp, panel, use_near, csr_val, ec,
                              pp.ell_val, F, R, dtype, x, y, fo);
    else
        hipLaunchKernelGGL(k_near_mm<T>, grid, dim3(256), lds, st, a, pp, panel, use_near, csr_val, ec, pp.ell_val,
                           F, R, dtype, x, y, fo);
    return hipGetLastError();
}

hipError_t launch_near_mm(const ApplyPlan& a, const PanelPlan& pp, const double* panel, int use_near,
                          const double* csr_val, int F, int R, int dtype, const void* x, void* y, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1, const MmFar<double>& fo) {
    return near_mm_t<double>(a, pp, panel, use_near, csr_val, F, R, dtype, x, y, st, e0, e1, fo);
}

hipError_t launch_near_mm(const ApplyPlan& a, const PanelPlan& pp, const float* panel, int use_near,
                          const double* csr_val, int F, int R, int dtype, const void* x, void* y, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1, const MmFar<float>& fo) {
    return near_mm_t<float>(a, pp, panel, use_near, csr_val, F, R, dtype, x, y, st, e0, e1, fo);
}

// FP32 panels with B + M added: p32[f][off[e]] = p64[f][off[e]] + val[f][e] for every
// nonzero e of B + M (off: its position in its row's panel; the positions are distinct)
FPDE_KERNEL void k_panel_add_csr(int64_t nnz, int F, int64_t total, const int64_t* off, const double* val,
                                 const double* p64, float* p32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)F * nnz) return;
    const int64_t f = i / nnz, e = i % nnz;
    const int64_t o = f * total + off[e];
    p32[o] = (float)(p64[o] + val[i]);
}

hipError_t launch_panel_add_csr(int64_t nnz, int F, int64_t total, const int64_t* off, const double* val,
                                const double* p64, float* p32, hipStream_t st) {
    const int64_t n = (int64_t)F * nnz;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_panel_add_csr, dim3(grid1(n)), dim3(256), 0, st, nnz, F, total, off, val, p64, p32);
    return hipGetLastError();
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
