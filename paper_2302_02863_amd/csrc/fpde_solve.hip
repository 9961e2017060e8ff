// Vector kernels of the batched conjugate-gradient solve and of the outer
// iterative refinement (Sec. 7: the Galerkin system is solved by CG).
//
// Vectors are [F][N][R] FP64 (right-hand sides fastest); system s = f*R + r is
// solved independently.  Dot products are reduced in a fixed order (rows of a
// block in an LDS tree, then the per-block partials in block order), so a
// solve is bitwise reproducible.  The per-system scalars stay on the device:
// each block that needs alpha or beta sums the partials itself (same order,
// same value in every block), so one CG iteration is the operator apply and
// three row-block kernels, launched back to back with no host round trip; with
// one right-hand side per field the apply's output kernel computes p . Ap and
// does CG_DOT's commit, and CG_DOT is not launched.
// State that the blocks of a kernel read (|r|^2, activity) is only committed
// by the next kernel, so no block reads a value another block of the same
// kernel writes.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fpde_internal.h"

namespace fpde {

namespace {

constexpr int kBS = 256;

__host__ __device__ inline int pow2_floor(int v) {
    int p = 1;
    while (2 * p <= v) p *= 2;
    return p;
}

// Column chunk width of the row-block passes: the largest power of two
// <= min(R, 256); the other threads of the block stride over rows.
__device__ inline int col_chunk(int R) { return pow2_floor(R < kBS ? R : kBS); }

// Sum the per-thread values of one column chunk over the row lanes (tree in
// LDS, fixed order) and store the block partial.
__device__ inline void reduce_store(double* red, double v, int RC, int col, int R, double* out) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    const int nrl = kBS / RC;
    for (int s = nrl / 2; s >= 1; s >>= 1) {
        if (t / RC < s) red[t] += red[t + s * RC];
        __syncthreads();
    }
    if (t < RC && col < R) out[col] = red[t];
    __syncthreads();
}

__device__ inline double sum_parts(const double* part, int64_t nb, int R, int64_t s) {
    const int64_t f = s / R, r = s % R;
    double v = 0.0;
    for (int64_t b = 0; b < nb; ++b) v += part[(f * nb + b) * R + r];
    return v;
}

// Row-block pass over all (row, r) of field f = blockIdx.y, rows
// [blockIdx.x * rpb, ...):
//   CG_DOT:       part1 = p . Ap                                        (a=p, b=Ap)
//                 the first block of the field commits |r|^2 and activity of the
//                 previous iteration (rr = rr_next, active = active_next); the
//                 first block of field 0 clears the active-system counter
//   CG_UPDATE_UR: alpha = rr / p.Ap (p.Ap summed from the nb_in partials of part_in: CG_DOT's, or
//                 those of the apply's output kernel when the iteration is fused); a system with a
//                 non-positive p.Ap takes alpha = 0 and is flagged (breakdown);
//                 u += alpha p, r -= alpha Ap, part1 = r . r             (a=p, b=Ap)
//   CG_UPDATE_P:  rr_new = r.r from part_in, beta = rr_new / rr, p = r + beta p;
//                 the first block of the field records rr_next, the iteration
//                 count, active_next and adds its field's active systems to n_active
//   CG_RESID:     r = b - Ap, part1 = r . r, part2 = b . b              (a=Ap, b=b)
//   CG_COPY_RP:   r = b, p = b, u = 0, part1 = b . b                    (b=b)
//   with the Jacobi preconditioner (dinv, z = D^-1 r): CG_UPDATE_UR part1 = r . z and
//   part2 = r . r; CG_UPDATE_P p = z + beta p with beta from the r . z partials and the
//   stopping test on the r . r partials part_in2; CG_COPY_RP p = D^-1 b, part1 = b . z,
//   part2 = b . b.  The Lanczos coefficients alpha_k, beta_k are recorded when asked.
//   V: the type of the CG vectors (FP64, or FP32 for the inner CG of a mixed-precision
//   solve); CG_RESID works on the outer FP64 vectors and CG_COPY_RP reads the FP64 outer
//   residual.  Values are read into FP64 and the dot products use the stored values.
template <int OP, typename V>
__global__ __launch_bounds__(kBS) void k_rowblock(int64_t N, int R, int64_t rpb, const void* __restrict__ a_,
                                                  const void* __restrict__ b_, void* __restrict__ u_,
                                                  void* __restrict__ r_, void* __restrict__ p_,
                                                  double* __restrict__ part1, double* __restrict__ part2,
                                                  const double* __restrict__ part_in, int64_t nb_in, CgScalars c,
                                                  const double* __restrict__ dinv,
                                                  const double* __restrict__ part_in2) {
    using TA = std::conditional_t<OP == CG_RESID, double, V>;
    using TB = std::conditional_t<OP == CG_RESID || OP == CG_COPY_RP, double, V>;
    using TR = std::conditional_t<OP == CG_RESID, double, V>;
    const TA* a = (const TA*)a_;
    const TB* b = (const TB*)b_;
    V* u = (V*)u_;
    TR* r = (TR*)r_;
    V* p = (V*)p_;
    __shared__ double red[kBS];
    __shared__ double coef[kBS];
    __shared__ int nact;
    const int f = blockIdx.y;
    const int64_t nb = gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = r0 + rpb < N ? r0 + rpb : N;
    const int RC = col_chunk(R);
    const int t = threadIdx.x;
    const int cl = t % RC, rl = t / RC, nrl = kBS / RC;
    const bool first = blockIdx.x == 0;
    constexpr bool kCoef = OP == CG_UPDATE_UR || OP == CG_UPDATE_P;
    if (OP == CG_DOT && first) {
        for (int col = t; col < R; col += kBS) {
            const int64_t sys = (int64_t)f * R + col;
            c.rr[sys] = c.rr_next[sys];
            c.active[sys] = c.active_next[sys];
        }
        if (f == 0 && t == 0) c.n_active[0] = 0;   // rebuilt by this iteration's CG_UPDATE_P
    }
    if (OP == CG_UPDATE_P && t == 0) nact = 0;
    for (int c0 = 0; c0 < R; c0 += RC) {
        const int col = c0 + cl;
        const int64_t sys = (int64_t)f * R + col;
        if (kCoef) {
            // the partials of the previous pass, summed by the whole block: row lanes
            // stride over the blocks, then a fixed-order tree (same value in every block)
            double pv = 0.0;
            if (col < R)
#pragma unroll 8
                for (int64_t b = rl; b < nb_in; b += nrl) pv += part_in[((int64_t)f * nb_in + b) * R + col];
            red[t] = pv;
            __syncthreads();
            for (int s = nrl / 2; s >= 1; s >>= 1) {
                if (rl < s) red[t] += red[t + s * RC];
                __syncthreads();
            }
            double v2 = 0.0;   // r . r of the new residual (preconditioned CG_UPDATE_P)
            if (OP == CG_UPDATE_P && part_in2) {
                const double v1 = red[cl];
                __syncthreads();
                double pw = 0.0;
                if (col < R)
#pragma unroll 8
                    for (int64_t b = rl; b < nb_in; b += nrl) pw += part_in2[((int64_t)f * nb_in + b) * R + col];
                red[t] = pw;
                __syncthreads();
                for (int s = nrl / 2; s >= 1; s >>= 1) {
                    if (rl < s) red[t] += red[t + s * RC];
                    __syncthreads();
                }
                v2 = red[cl];
                __syncthreads();
                if (rl == 0) red[cl] = v1;
                __syncthreads();
            }
            if (rl == 0) {   // per-system coefficient, once per column
                double cf = 0.0;
                if (col < R) {
                    const double v = red[cl];
                    const double vs = (OP == CG_UPDATE_P && part_in2) ? v2 : v;
                    const bool act = c.active[sys] != 0;
                    if (OP == CG_UPDATE_UR) {
                        const bool ok = act && v > 0.0 && v == v;
                        cf = ok ? c.rr[sys] / v : 0.0;
                        if (first) {
                            c.alpha[sys] = cf;
                            if (act && !ok) c.flags[sys] = 1;
                            const int k = c.iters[sys];
                            if (act && c.hist_a && k < c.hist_cap) c.hist_a[(int64_t)k * gridDim.y * R + sys] = cf;
                        }
                    } else {
                        const bool moved = act && c.alpha[sys] != 0.0;
                        cf = moved ? v / c.rr[sys] : 0.0;
                        if (first) {
                            c.beta[sys] = cf;
                            c.rr_next[sys] = moved ? v : c.rr[sys];
                            const int k = c.iters[sys];
                            if (moved && c.hist_b && k < c.hist_cap) c.hist_b[(int64_t)k * gridDim.y * R + sys] = cf;
                            if (moved) c.iters[sys] += 1;
                            const int still = (moved && vs > c.tol2[sys]) ? 1 : 0;
                            c.active_next[sys] = still;
                            atomicAdd(&nact, still);
                        }
                    }
                }
                coef[cl] = cf;
            }
            __syncthreads();
        }
        double acc1 = 0.0, acc2 = 0.0;
        if (col < R) {
            const double cf = kCoef ? coef[cl] : 0.0;
#pragma unroll 4   // four rows of loads in flight per thread
            for (int64_t row = r0 + rl; row < r1; row += nrl) {
                const int64_t i = ((int64_t)f * N + row) * R + col;
                if (OP == CG_DOT) {
                    acc1 += (double)a[i] * (double)b[i];
                } else if (OP == CG_UPDATE_UR) {
                    u[i] = (V)((double)u[i] + cf * (double)a[i]);
                    const double rn = (double)(V)((double)r[i] - cf * (double)b[i]);   // as stored
                    r[i] = (V)rn;
                    if (dinv) {
                        acc1 += rn * rn * dinv[(int64_t)f * N + row];
                        acc2 += rn * rn;
                    } else {
                        acc1 += rn * rn;
                    }
                } else if (OP == CG_UPDATE_P) {
                    const double av = (double)a[i];
                    p[i] = (V)((dinv ? av * dinv[(int64_t)f * N + row] : av) + cf * (double)p[i]);
                } else if (OP == CG_RESID) {
                    const double rn = b[i] - a[i];
                    r[i] = rn;
                    acc1 += rn * rn;
                    acc2 += b[i] * b[i];
                } else {
                    const double bv = (double)(V)b[i];   // as stored in r
                    const double di = dinv ? dinv[(int64_t)f * N + row] : 1.0;
                    r[i] = (V)bv;
                    p[i] = (V)(bv * di);
                    u[i] = (V)0;
                    acc1 += bv * (double)(V)(bv * di);
                    acc2 += bv * bv;
                }
            }
        }
        if (OP == CG_UPDATE_P) {
            __syncthreads();   // coef[] is rewritten by the next column chunk
        } else {
            reduce_store(red, acc1, RC, col, R, part1 + ((int64_t)f * nb + blockIdx.x) * R);
            if (OP == CG_RESID || ((OP == CG_UPDATE_UR || OP == CG_COPY_RP) && part2))
                reduce_store(red, acc2, RC, col, R, part2 + ((int64_t)f * nb + blockIdx.x) * R);
        }
    }
    if (OP == CG_UPDATE_P && first && t == 0) atomicAdd(c.n_active, nact);
}

// Start of a CG run on A d = b from d = 0 (after CG_COPY_RP): |r|^2 and the
// stopping threshold tol2_s = max(tau_in^2 |r_s|^2, rtol^2 |b0_s|^2), where bb0
// holds |b0|^2 of the outer system; the committed and the next state agree.
__global__ __launch_bounds__(kBS) void k_cg_start(int64_t S, int64_t nb, int R, const double* part, const double* bb0,
                                                   double tau_in, double rtol, CgScalars c, const double* part_rr) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int mine = 0;
    for (int64_t s = threadIdx.x; s < S; s += blockDim.x) {
        const double rz = sum_parts(part, nb, R, s);
        const double rn = part_rr ? sum_parts(part_rr, nb, R, s) : rz;
        const double t_in = tau_in * tau_in * rn, t_out = rtol * rtol * bb0[s];
        const double tol2 = t_in > t_out ? t_in : t_out;
        const int act = rn > tol2 ? 1 : 0;
        c.rr[s] = rz;
        c.rr_next[s] = rz;
        c.tol2[s] = tol2;
        c.active[s] = act;
        c.active_next[s] = act;
        c.alpha[s] = 0.0;
        c.beta[s] = 0.0;
        c.iters[s] = 0;
        c.flags[s] = 0;
        mine += act;
    }
    atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) c.n_active[0] = cnt;
}

// |r|^2 and |b|^2 of the outer residual r = b - A u per system
__global__ __launch_bounds__(kBS) void k_sum2(int64_t S, int64_t nb, int R, const double* part1, const double* part2,
                                               double* o1, double* o2) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    o1[s] = sum_parts(part1, nb, R, s);
    if (o2) o2[s] = sum_parts(part2, nb, R, s);
}

template <typename V>
__global__ __launch_bounds__(kBS) void k_add(int64_t n, const V* d, double* u) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] += (double)d[i];
}

unsigned grid_of(int64_t n) {
    const int64_t g = (n + kBS - 1) / kBS;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

int64_t cg_row_blocks(int64_t N, int R, int F) {
    // one element per thread, N * R / 256 blocks per field, but about 2048 blocks in all:
    // every block of a pass sums all the partials of the previous one (F * nb^2 * R
    // loads), so many fields or right-hand sides take fewer, larger blocks
    int64_t nb = (N * (int64_t)R + kBS - 1) / kBS;
    const int64_t cap = F > 0 ? (2048 + F - 1) / F : 2048;
    if (nb > cap) nb = cap;
    if (nb > 1024) nb = 1024;
    if (nb > N) nb = N;
    if (nb < 1) nb = 1;
    return nb;
}

hipError_t launch_cg_rowblock(int op, const CgDims& d, const void* a, const void* b, void* u, void* r, void* p,
                              double* part1, double* part2, const double* part_in, const CgScalars& c, hipStream_t st,
                              int64_t nb_in, const double* dinv, const double* part_in2, bool v32) {
    const int64_t rpb = (d.N + d.nb - 1) / d.nb;
    if (nb_in < 0) nb_in = d.nb;
    const dim3 g((unsigned)d.nb, (unsigned)d.F);
    if (v32 && op == CG_RESID) return hipErrorInvalidValue;   // the outer residual is FP64
#define FPDE_ROWBLOCK(OPV)                                                                                          \
    do {                                                                                                            \
        if (v32)                                                                                                    \
            hipLaunchKernelGGL((k_rowblock<OPV, float>), g, dim3(kBS), 0, st, d.N, d.R, rpb, a, b, u, r, p, part1,  \
                               part2, part_in, nb_in, c, dinv, part_in2);                                          \
        else                                                                                                        \
            hipLaunchKernelGGL((k_rowblock<OPV, double>), g, dim3(kBS), 0, st, d.N, d.R, rpb, a, b, u, r, p, part1, \
                               part2, part_in, nb_in, c, dinv, part_in2);                                          \
    } while (0)
    switch (op) {
        case CG_DOT: FPDE_ROWBLOCK(CG_DOT); break;
        case CG_UPDATE_UR: FPDE_ROWBLOCK(CG_UPDATE_UR); break;
        case CG_RESID: FPDE_ROWBLOCK(CG_RESID); break;
        case CG_COPY_RP: FPDE_ROWBLOCK(CG_COPY_RP); break;
        case CG_UPDATE_P: FPDE_ROWBLOCK(CG_UPDATE_P); break;
        default: return hipErrorInvalidValue;
    }
#undef FPDE_ROWBLOCK
    return hipGetLastError();
}

hipError_t launch_cg_start(const CgDims& d, const double* part, const double* bb0, double tau_in, double rtol,
                           const CgScalars& c, hipStream_t st, const double* part_rr) {
    const int64_t S = (int64_t)d.F * d.R;
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kBS), 0, st, S, d.nb, d.R, part, bb0, tau_in, rtol, c, part_rr);
    return hipGetLastError();
}

hipError_t launch_cg_sum2(const CgDims& d, const double* part1, const double* part2, double* o1, double* o2,
                          hipStream_t st) {
    const int64_t S = (int64_t)d.F * d.R;
    hipLaunchKernelGGL(k_sum2, dim3(grid_of(S)), dim3(kBS), 0, st, S, d.nb, d.R, part1, part2, o1, o2);
    return hipGetLastError();
}

// 1 / diag(A_h) per field and dof
__global__ __launch_bounds__(kBS) void k_jacobi_diag(int64_t N, int F, int64_t nnz, const int64_t* bm_idx,
                                                      const double* bm, int64_t ptot, const int64_t* p_idx,
                                                      const double* panel, double* dinv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int f = 0; f < F; ++f) {
        const double d = bm[(int64_t)f * nnz + bm_idx[i]] + (p_idx[i] >= 0 ? panel[(int64_t)f * ptot + p_idx[i]] : 0.0);
        dinv[(int64_t)f * N + i] = 1.0 / d;
    }
}

hipError_t launch_jacobi_diag(int64_t N, int F, int64_t nnz, const int64_t* bm_idx, const double* bm, int64_t ptot,
                              const int64_t* p_idx, const double* panel, double* dinv, hipStream_t st) {
    hipLaunchKernelGGL(k_jacobi_diag, dim3(grid_of(N)), dim3(kBS), 0, st, N, F, nnz, bm_idx, bm, ptot, p_idx, panel,
                       dinv);
    return hipGetLastError();
}

hipError_t launch_vec_add(int64_t n, const void* d, double* u, hipStream_t st, bool v32) {
    if (v32) hipLaunchKernelGGL(k_add<float>, dim3(grid_of(n)), dim3(kBS), 0, st, n, (const float*)d, u);
    else hipLaunchKernelGGL(k_add<double>, dim3(grid_of(n)), dim3(kBS), 0, st, n, (const double*)d, u);
    return hipGetLastError();
}

}  // namespace fpde
