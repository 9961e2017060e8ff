// Vector kernels of the batched conjugate-gradient solve and of the outer
// iterative refinement (Sec. 7: the Galerkin system is solved by CG).
//
// Vectors are [F][N][R] FP64 (right-hand sides fastest); system s = f*R + r is
// solved independently.  Every dot product is reduced in a fixed order
// (row blocks -> per-block partials -> one pass over the partials), so a solve
// is bitwise reproducible.  Scalars (alpha, beta, |r|^2, activity flags) stay
// on the device: an iteration needs no host round trip and is captured in a
// graph together with the operator apply.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_internal.h"

namespace fpde {

namespace {

constexpr int kBS = 256;

__host__ __device__ inline int pow2_floor(int v) {
    int p = 1;
    while (2 * p <= v) p *= 2;
    return p;
}

// Column chunk width of the row-block reductions: the largest power of two
// <= min(R, 256); the remaining threads of the block stride over rows.
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

enum { OP_DOT = 0, OP_UPDATE_UR = 1, OP_RESID = 2, OP_COPY_RP = 3 };

// Row-block pass over all (f, row, r) of field f = blockIdx.y, rows
// [blockIdx.x * rpb, ...):
//   OP_DOT:       partial1 += a . b
//   OP_UPDATE_UR: u += alpha p, r -= alpha Ap, partial1 += r . r      (a=p, b=Ap)
//   OP_RESID:     r = b - Ap, partial1 += r . r, partial2 += b . b   (a=Ap, b=b)
//   OP_COPY_RP:   r = b, p = b, u = 0, partial1 += b . b             (b=b)
template <int OP>
__global__ __launch_bounds__(kBS) void k_rowblock(int64_t N, int R, int64_t rpb, const double* a, const double* b,
                                                  const double* alpha, double* u, double* r, double* p,
                                                  double* part1, double* part2) {
    __shared__ double red[kBS];
    const int f = blockIdx.y;
    const int64_t nb = gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = r0 + rpb < N ? r0 + rpb : N;
    const int RC = col_chunk(R);
    const int t = threadIdx.x;
    const int cl = t % RC, rl = t / RC, nrl = kBS / RC;
    for (int c0 = 0; c0 < R; c0 += RC) {
        const int col = c0 + cl;
        double acc1 = 0.0, acc2 = 0.0;
        if (col < R) {
            const double al = (OP == OP_UPDATE_UR) ? alpha[(int64_t)f * R + col] : 0.0;
            for (int64_t row = r0 + rl; row < r1; row += nrl) {
                const int64_t i = ((int64_t)f * N + row) * R + col;
                if (OP == OP_DOT) {
                    acc1 += a[i] * b[i];
                } else if (OP == OP_UPDATE_UR) {
                    u[i] += al * a[i];
                    const double rn = r[i] - al * b[i];
                    r[i] = rn;
                    acc1 += rn * rn;
                } else if (OP == OP_RESID) {
                    const double rn = b[i] - a[i];
                    r[i] = rn;
                    acc1 += rn * rn;
                    acc2 += b[i] * b[i];
                } else {
                    const double bv = b[i];
                    r[i] = bv;
                    p[i] = bv;
                    u[i] = 0.0;
                    acc1 += bv * bv;
                }
            }
        }
        reduce_store(red, acc1, RC, col, R, part1 + ((int64_t)f * nb + blockIdx.x) * R);
        if (OP == OP_RESID) reduce_store(red, acc2, RC, col, R, part2 + ((int64_t)f * nb + blockIdx.x) * R);
    }
}

__device__ inline double sum_parts(const double* part, int64_t nb, int R, int64_t s) {
    const int64_t f = s / R, r = s % R;
    double v = 0.0;
    for (int64_t b = 0; b < nb; ++b) v += part[(f * nb + b) * R + r];
    return v;
}

// alpha_s = |r|^2 / p.Ap for active systems; a non-positive p.Ap (breakdown)
// deactivates the system and flags it.
__global__ __launch_bounds__(kBS) void k_cg_alpha(int64_t S, int64_t nb, int R, const double* part, const double* rr,
                                                   double* alpha, int* active, int* flags) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double pap = sum_parts(part, nb, R, s);
    double al = 0.0;
    if (active[s]) {
        if (pap > 0.0 && pap == pap) al = rr[s] / pap;
        else {
            active[s] = 0;
            flags[s] = 1;
        }
    }
    alpha[s] = al;
}

// New |r|^2, beta, iteration count, activity; one block counts the active systems.
__global__ __launch_bounds__(kBS) void k_cg_beta(int64_t S, int64_t nb, int R, const double* part, double* rr,
                                                  double* beta, const double* tol2, int* active, int* iters,
                                                  int* n_active) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int mine = 0;
    for (int64_t s = threadIdx.x; s < S; s += blockDim.x) {
        const double rn = sum_parts(part, nb, R, s);
        double be = 0.0;
        if (active[s]) {
            be = rn / rr[s];
            rr[s] = rn;
            iters[s] += 1;
            if (!(rn > tol2[s])) active[s] = 0;
        }
        beta[s] = be;
        mine += active[s];
    }
    atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) n_active[0] = cnt;
}

// Start of a CG run on (rhs b, solution x = 0) or on the residual of the
// current x: |r|^2 and the stopping threshold
//   tol2_s = max(tau_in^2 |r_s|^2, (rtol_abs_s)^2),  rtol_abs_s = rtol * |b0_s|
// where b0 holds |b|^2 of the outer system.
__global__ __launch_bounds__(kBS) void k_cg_start(int64_t S, int64_t nb, int R, const double* part, const double* bb0,
                                                   double tau_in, double rtol, double* rr, double* tol2, int* active,
                                                   int* iters, int* flags, int* n_active) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int mine = 0;
    for (int64_t s = threadIdx.x; s < S; s += blockDim.x) {
        const double rn = sum_parts(part, nb, R, s);
        rr[s] = rn;
        const double t_in = tau_in * tau_in * rn, t_out = rtol * rtol * bb0[s];
        tol2[s] = t_in > t_out ? t_in : t_out;
        active[s] = rn > tol2[s] ? 1 : 0;
        iters[s] = 0;
        flags[s] = 0;
        mine += active[s];
    }
    atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) n_active[0] = cnt;
}

// |b|^2 and |r|^2 of the outer residual r = b - A u per system
__global__ __launch_bounds__(kBS) void k_sum2(int64_t S, int64_t nb, int R, const double* part1, const double* part2,
                                               double* o1, double* o2) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    o1[s] = sum_parts(part1, nb, R, s);
    if (o2) o2[s] = sum_parts(part2, nb, R, s);
}

__global__ __launch_bounds__(kBS) void k_add(int64_t n, const double* d, double* u) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] += d[i];
}

// p = r + beta[f*R + r] p over [F][N][R]
__global__ __launch_bounds__(kBS) void k_cg_pupdate(int64_t N, int R, const double* beta, const double* r, double* p) {
    const int f = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N * R) return;
    const int64_t i = (int64_t)f * N * R + j;
    p[i] = r[i] + beta[(int64_t)f * R + (int)(j % R)] * p[i];
}

unsigned grid_of(int64_t n) {
    const int64_t g = (n + kBS - 1) / kBS;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

int64_t cg_row_blocks(int64_t N, int R) {
    // about 16 K elements per block, at most 1024 blocks per field
    int64_t nb = (N * (int64_t)R + 16383) / 16384;
    if (nb < 1) nb = 1;
    if (nb > 1024) nb = 1024;
    if (nb > N) nb = N;
    return nb;
}

hipError_t launch_cg_rowblock(int op, const CgDims& d, const double* a, const double* b, const double* alpha,
                              double* u, double* r, double* p, double* part1, double* part2, hipStream_t st) {
    const int64_t rpb = (d.N + d.nb - 1) / d.nb;
    const dim3 g((unsigned)d.nb, (unsigned)d.F);
    switch (op) {
        case 0: hipLaunchKernelGGL(k_rowblock<OP_DOT>, g, dim3(kBS), 0, st, d.N, d.R, rpb, a, b, alpha, u, r, p, part1,
                                   part2); break;
        case 1: hipLaunchKernelGGL(k_rowblock<OP_UPDATE_UR>, g, dim3(kBS), 0, st, d.N, d.R, rpb, a, b, alpha, u, r, p,
                                   part1, part2); break;
        case 2: hipLaunchKernelGGL(k_rowblock<OP_RESID>, g, dim3(kBS), 0, st, d.N, d.R, rpb, a, b, alpha, u, r, p,
                                   part1, part2); break;
        default: hipLaunchKernelGGL(k_rowblock<OP_COPY_RP>, g, dim3(kBS), 0, st, d.N, d.R, rpb, a, b, alpha, u, r, p,
                                    part1, part2); break;
    }
    return hipGetLastError();
}

hipError_t launch_cg_alpha(const CgDims& d, const double* part, const CgScalars& c, hipStream_t st) {
    const int64_t S = (int64_t)d.F * d.R;
    hipLaunchKernelGGL(k_cg_alpha, dim3(grid_of(S)), dim3(kBS), 0, st, S, d.nb, d.R, part, c.rr, c.alpha, c.active,
                       c.flags);
    return hipGetLastError();
}

hipError_t launch_cg_beta(const CgDims& d, const double* part, const CgScalars& c, hipStream_t st) {
    const int64_t S = (int64_t)d.F * d.R;
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(kBS), 0, st, S, d.nb, d.R, part, c.rr, c.beta, c.tol2, c.active,
                       c.iters, c.n_active);
    return hipGetLastError();
}

hipError_t launch_cg_p(const CgDims& d, const CgScalars& c, const double* r, double* p, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_pupdate, dim3(grid_of(d.N * d.R), (unsigned)d.F), dim3(kBS), 0, st, d.N, d.R, c.beta, r,
                       p);
    return hipGetLastError();
}

hipError_t launch_cg_start(const CgDims& d, const double* part, const double* bb0, double tau_in, double rtol,
                           const CgScalars& c, hipStream_t st) {
    const int64_t S = (int64_t)d.F * d.R;
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kBS), 0, st, S, d.nb, d.R, part, bb0, tau_in, rtol, c.rr, c.tol2,
                       c.active, c.iters, c.flags, c.n_active);
    return hipGetLastError();
}

hipError_t launch_cg_sum2(const CgDims& d, const double* part1, const double* part2, double* o1, double* o2,
                          hipStream_t st) {
    const int64_t S = (int64_t)d.F * d.R;
    hipLaunchKernelGGL(k_sum2, dim3(grid_of(S)), dim3(kBS), 0, st, S, d.nb, d.R, part1, part2, o1, o2);
    return hipGetLastError();
}

hipError_t launch_vec_add(int64_t n, const double* d, double* u, hipStream_t st) {
    hipLaunchKernelGGL(k_add, dim3(grid_of(n)), dim3(kBS), 0, st, n, d, u);
    return hipGetLastError();
}

}  // namespace fpde
