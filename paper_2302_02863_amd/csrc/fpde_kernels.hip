// HIP kernels for gfx950 (MI355X): build-time quadrature (singular near field,
// near leaf blocks, Chebyshev bases and transfers, point-collocation density,
// weighted mass) and the operator apply (CSR + near blocks + H2 sweeps).
//
// All floating point here is FP64.  64-wide wavefronts: reductions use
// cross-lane shuffles; every output element has exactly one writer, so the
// results are bitwise reproducible from run to run.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_internal.h"

namespace fpde {

#define FPDE_KERNEL __global__ __launch_bounds__(256)

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline unsigned grid1(int64_t n, int bs = 256) {
    int64_t g = cdiv(n, bs);
    return (unsigned)(g < 1 ? 1 : (g > 2147483647 ? 2147483647 : g));
}

// |d|^{-e} from |d|^2: exp(-e/2 * log(r2))
__device__ __forceinline__ double rpow(double r2, double e) { return exp(-0.5 * e * log(r2)); }

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ============================================================ singular pairs

struct Reg2 {
    double a0, a1, b0, b1, jac;
};

// Region maps of the touching cases written as x^ = xi*a(eta), y^ = xi*b(eta)
// (vertex/edge) and the Jacobian factor after extracting xi^3.
__device__ __forceinline__ Reg2 vertex_region(int r, double e1, double e2, double e3) {
    Reg2 g;
    if (r == 0) { g.a0 = 1.0; g.a1 = e1; g.b0 = e2; g.b1 = e2 * e3; }
    else        { g.a0 = e2; g.a1 = e2 * e3; g.b0 = 1.0; g.b1 = e1; }
    g.jac = e2;
    return g;
}

__device__ __forceinline__ Reg2 edge_region(int r, double e1, double e2, double e3) {
    Reg2 g;
    const double e12 = e1 * e2, e123 = e12 * e3;
    switch (r) {
        case 0: g.a0 = 1.0; g.a1 = e1 * e3; g.b0 = 1.0 - e12; g.b1 = e1 * (1.0 - e2); g.jac = e1 * e1; break;
        case 1: g.a0 = 1.0; g.a1 = e1; g.b0 = 1.0 - e123; g.b1 = e12 * (1.0 - e3); g.jac = e1 * e1 * e2; break;
        case 2: g.a0 = 1.0 - e12; g.a1 = e1 * (1.0 - e2); g.b0 = 1.0; g.b1 = e123; g.jac = e1 * e1 * e2; break;
        case 3: g.a0 = 1.0 - e123; g.a1 = e12 * (1.0 - e3); g.b0 = 1.0; g.b1 = e1; g.jac = e1 * e1 * e2; break;
        default: g.a0 = 1.0 - e123; g.a1 = e1 * (1.0 - e2 * e3); g.b0 = 1.0; g.b1 = e12; g.jac = e1 * e1 * e2; break;
    }
    return g;
}

// identical case: x^ = xi*a, y^ = xi*b, x^-y^ = xi*eta1*eta2*dhat
__device__ __forceinline__ void identical_region(int r, double e1, double e2, double e3, double* a,
                                                 double* b, double* dh) {
    if (r == 0) {
        a[0] = 1.0; a[1] = 1.0 - e1 + e1 * e2; b[0] = 1.0 - e1 * e2 * e3; b[1] = 1.0 - e1;
        dh[0] = e3; dh[1] = 1.0;
    } else if (r == 1) {
        a[0] = 1.0; a[1] = e1 * (1.0 - e2 + e2 * e3); b[0] = 1.0 - e1 * e2; b[1] = e1 * (1.0 - e2);
        dh[0] = 1.0; dh[1] = e3;
    } else {
        a[0] = 1.0 - e1 * e2 * e3; a[1] = e1 * (1.0 - e2 * e3); b[0] = 1.0; b[1] = e1 * (1.0 - e2);
        dh[0] = -e3; dh[1] = 1.0 - e3;
    }
}

struct SingArgs {
    int64_t np;
    const int32_t* pairs;
    const double* X;
    int64_t M;
    const double* s;
    const double* kap;
    double a_scale, s_bar;
    int nq;
    const double* g;
    const double* w;
    double* out;
};

// one 64-lane wave per pair; lanes stride over the tensor Gauss points of all regions
FPDE_KERNEL void k_singular2d(SingArgs A, int f) {
    const int lane = threadIdx.x & 63;
    const int64_t pid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pid >= A.np) return;
    const int32_t* P = A.pairs + pid * 8;
    const int kind = P[0];
    const double* s = A.s + (int64_t)f * A.M;
    const double* kp = A.kap + (int64_t)f * A.M;
    // canonical vertices of both cells: row layout (kind, cell0 v0..v2, cell1 v0..v2, pad)
    double X0[3][2], X1[3][2], s0[3], s1[3], k0[3], k1[3];
    const int vv0[3] = {P[1], P[2], P[3]};
    const int vv1[3] = {P[4], P[5], P[6]};
    for (int a = 0; a < 3; ++a) {
        X0[a][0] = A.X[vv0[a]]; X0[a][1] = A.X[A.M + vv0[a]];
        X1[a][0] = A.X[vv1[a]]; X1[a][1] = A.X[A.M + vv1[a]];
        s0[a] = s[vv0[a]]; s1[a] = s[vv1[a]];
        k0[a] = kp[vv0[a]]; k1[a] = kp[vv1[a]];
    }
    const double J0[2][2] = {{X0[1][0] - X0[0][0], X0[2][0] - X0[1][0]}, {X0[1][1] - X0[0][1], X0[2][1] - X0[1][1]}};
    const double J1[2][2] = {{X1[1][0] - X1[0][0], X1[2][0] - X1[1][0]}, {X1[1][1] - X1[0][1], X1[2][1] - X1[1][1]}};
    const double det0 = fabs(J0[0][0] * J0[1][1] - J0[0][1] * J0[1][0]);
    const double det1 = fabs(J1[0][0] * J1[1][1] - J1[0][1] * J1[1][0]);
    const int nd = kind == 0 ? 3 : (kind == 1 ? 4 : 5);
    const int nreg = kind == 0 ? 3 : (kind == 1 ? 5 : 2);
    const int nq = A.nq;
    const int n4 = nq * nq * nq * nq;
    const double sb = A.s_bar;
    const double inv4 = 1.0 / (4.0 - 2.0 * sb);
    const double inv2 = 1.0 / (2.0 - 2.0 * sb);
    double acc[15];
#pragma unroll
    for (int e = 0; e < 15; ++e) acc[e] = 0.0;
    for (int idx = lane; idx < nreg * n4; idx += 64) {
        const int r = idx / n4;
        int q = idx - r * n4;
        const int i3 = q % nq; q /= nq;
        const int i2 = q % nq; q /= nq;
        const int i1 = q % nq;
        const int i0 = q / nq;
        const double z = A.g[i0], e1 = A.g[i1], t2 = A.g[i2], e3 = A.g[i3];
        const double wt = (A.w[i0] * A.w[i1]) * (A.w[i2] * A.w[i3]);
        const double lz = log(z);
        double phi[5];
        double xa0, xa1, yb0, yb1, r2, fac, sx, sy, kx, ky;
        if (kind == 0) {
            const double e2 = exp(inv2 * log(t2));      // eta2 = t^{1/(2-2 s_bar)}
            const double xi = exp(inv4 * lz);
            double a[2], b[2], dh[2];
            identical_region(r, e1, e2, e3, a, b, dh);
            xa0 = xi * a[0]; xa1 = xi * a[1]; yb0 = xi * b[0]; yb1 = xi * b[1];
            phi[0] = -dh[0]; phi[1] = dh[0] - dh[1]; phi[2] = dh[1];
            const double d0 = J0[0][0] * dh[0] + J0[0][1] * dh[1];
            const double d1 = J0[1][0] * dh[0] + J0[1][1] * dh[1];
            r2 = d0 * d0 + d1 * d1;
            sx = (1.0 - xa0) * s0[0] + (xa0 - xa1) * s0[1] + xa1 * s0[2];
            sy = (1.0 - yb0) * s0[0] + (yb0 - yb1) * s0[1] + yb1 * s0[2];
            kx = (1.0 - xa0) * k0[0] + (xa0 - xa1) * k0[1] + xa1 * k0[2];
            ky = (1.0 - yb0) * k0[0] + (yb0 - yb1) * k0[1] + yb1 * k0[2];
            const double ss = sx + sy;
            fac = exp((2.0 * sb - ss) * inv4 * lz) * exp((2.0 - ss) * log(e1)) *
                  exp((2.0 * sb - ss) * inv2 * log(t2));
        } else {
            const double xi = exp(inv4 * lz);
            Reg2 g = kind == 1 ? edge_region(r, e1, t2, e3) : vertex_region(r, e1, t2, e3);
            xa0 = xi * g.a0; xa1 = xi * g.a1; yb0 = xi * g.b0; yb1 = xi * g.b1;
            // linear parts of the reference shape functions: (-z0, z0-z1, z1)
            const double la0 = -g.a0, la1 = g.a0 - g.a1, la2 = g.a1;
            const double lb0 = -g.b0, lb1 = g.b0 - g.b1, lb2 = g.b1;
            if (kind == 1) {
                phi[0] = la0 - lb0; phi[1] = la1 - lb1; phi[2] = la2; phi[3] = -lb2;
            } else {
                phi[0] = la0 - lb0; phi[1] = la1; phi[2] = la2; phi[3] = -lb1; phi[4] = -lb2;
            }
            const double d0 = (J0[0][0] * g.a0 + J0[0][1] * g.a1) - (J1[0][0] * g.b0 + J1[0][1] * g.b1);
            const double d1 = (J0[1][0] * g.a0 + J0[1][1] * g.a1) - (J1[1][0] * g.b0 + J1[1][1] * g.b1);
            r2 = d0 * d0 + d1 * d1;
            sx = (1.0 - xa0) * s0[0] + (xa0 - xa1) * s0[1] + xa1 * s0[2];
            sy = (1.0 - yb0) * s1[0] + (yb0 - yb1) * s1[1] + yb1 * s1[2];
            kx = (1.0 - xa0) * k0[0] + (xa0 - xa1) * k0[1] + xa1 * k0[2];
            ky = (1.0 - yb0) * k1[0] + (yb0 - yb1) * k1[1] + yb1 * k1[2];
            fac = exp((2.0 * sb - (sx + sy)) * inv4 * lz) * g.jac;
        }
        const double val = wt * A.a_scale * sqrt(kx * ky) * fac * rpow(r2, 2.0 + sx + sy);
        int e = 0;
        for (int i = 0; i < 5; ++i)
            for (int j = i; j < 5; ++j, ++e)
                if (i < nd && j < nd) acc[e] += val * phi[i] * phi[j];
    }
    double pre = kind == 0 ? det0 * det0 / ((2.0 - sb) * (2.0 - 2.0 * sb)) : det0 * det1 * inv4;
    if (kind != 0) pre *= 2.0;   // both orderings of a distinct touching pair
    double* o = A.out + ((int64_t)f * A.np + pid) * 25;
    int e = 0;
    for (int i = 0; i < 5; ++i)
        for (int j = i; j < 5; ++j, ++e) {
            double v = wave_sum(acc[e]);
            if (lane == 0) o[i * 5 + j] = v * pre;
        }
}

FPDE_KERNEL void k_singular1d(SingArgs A, int f) {
    const int lane = threadIdx.x & 63;
    const int64_t pid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pid >= A.np) return;
    const int32_t* P = A.pairs + pid * 8;
    const int kind = P[0];
    const double* s = A.s + (int64_t)f * A.M;
    const double* kp = A.kap + (int64_t)f * A.M;
    const int nq = A.nq;
    const double sb = A.s_bar;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (kind == 0) {
        const int v0 = P[1], v1 = P[2];
        const double J = A.X[v1] - A.X[v0];
        const double aJ = fabs(J);
        const double inv = 1.0 / (2.0 - 2.0 * sb);
        for (int idx = lane; idx < nq * nq; idx += 64) {
            const int i0 = idx / nq, i1 = idx % nq;
            const double z = A.g[i0], u = A.g[i1];
            const double wt = A.w[i0] * A.w[i1];
            const double t = exp(inv * log(z));
            const double yh = (1.0 - t) * u;
            const double xh = yh + t;
            const double sx = (1.0 - xh) * s[v0] + xh * s[v1];
            const double sy = (1.0 - yh) * s[v0] + yh * s[v1];
            const double kx = (1.0 - xh) * kp[v0] + xh * kp[v1];
            const double ky = (1.0 - yh) * kp[v0] + yh * kp[v1];
            const double ss = sx + sy;
            acc[0] += wt * A.a_scale * sqrt(kx * ky) * exp((1.0 - ss) * log(aJ)) *
                      exp((2.0 * sb - ss) * inv * log(z)) * (1.0 - t);
        }
        double v = wave_sum(acc[0]) * 2.0 * inv;
        if (lane == 0) {
            double* o = A.out + ((int64_t)f * A.np + pid) * 25;
            o[0] = v; o[1] = -v; o[6] = v;
        }
        return;
    }
    // vertex pair: cell0 = (P, A), cell1 = (P, B)
    const int vp = P[1], va = P[2], vb = P[5];
    const double h1 = fabs(A.X[va] - A.X[vp]);
    const double h2 = fabs(A.X[vb] - A.X[vp]);
    const double inv = 1.0 / (3.0 - 2.0 * sb);
    for (int idx = lane; idx < 2 * nq * nq; idx += 64) {
        const int r = idx / (nq * nq);
        const int q = idx % (nq * nq);
        const int i0 = q / nq, i1 = q % nq;
        const double z = A.g[i0], u = A.g[i1];
        const double wt = A.w[i0] * A.w[i1];
        const double xi = exp(inv * log(z));
        const double at = r == 0 ? 1.0 : u;
        const double bt = r == 0 ? u : 1.0;
        const double al = xi * at, be = xi * bt;
        const double sx = (1.0 - al) * s[vp] + al * s[va];
        const double sy = (1.0 - be) * s[vp] + be * s[vb];
        const double kx = (1.0 - al) * kp[vp] + al * kp[va];
        const double ky = (1.0 - be) * kp[vp] + be * kp[vb];
        const double D = h1 * at + h2 * bt;
        const double val = wt * A.a_scale * sqrt(kx * ky) * exp((2.0 * sb - (sx + sy)) * inv * log(z)) *
                           exp(-(1.0 + sx + sy) * log(D));
        const double phi[3] = {bt - at, at, -bt};
        int e = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j, ++e) acc[e] += val * phi[i] * phi[j];
    }
    const double pre = 2.0 * h1 * h2 * inv;
    double* o = A.out + ((int64_t)f * A.np + pid) * 25;
    int e = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j, ++e) {
            double v = wave_sum(acc[e]);
            if (lane == 0) o[i * 5 + j] = v * pre;
        }
}

hipError_t launch_singular(int dim, int64_t np, const int32_t* pairs, const double* coords,
                           int64_t n_nodes, int F, const double* s, const double* kappa,
                           double a_scale, double s_bar, int nq, const double* g01,
                           const double* w01, double* out, hipStream_t st) {
    if (np == 0) return hipSuccess;
    SingArgs A{np, pairs, coords, n_nodes, s, kappa, a_scale, s_bar, nq, g01, w01, out};
    for (int f = 0; f < F; ++f) {
        if (dim == 2)
            hipLaunchKernelGGL(k_singular2d, dim3(grid1(np, 4)), dim3(256), 0, st, A, f);
        else
            hipLaunchKernelGGL(k_singular1d, dim3(grid1(np, 4)), dim3(256), 0, st, A, f);
    }
    return hipGetLastError();
}

// ============================================================ segmented sums

FPDE_KERNEL void k_segsum(int64_t n, const int64_t* ptr, const int64_t* idx, const double* w,
                          const double* src, int64_t src_stride, double* out, int f) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* sf = src + (int64_t)f * src_stride;
    double acc = 0.0;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) acc += (w ? w[e] : 1.0) * sf[idx[e]];
    out[(int64_t)f * n + i] = acc;
}

hipError_t launch_segsum(int64_t nslots, const int64_t* ptr, const int64_t* idx, const double* w,
                         int F, const double* src, int64_t src_stride, double* out,
                         hipStream_t st) {
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(k_segsum, dim3(grid1(nslots)), dim3(256), 0, st, nslots, ptr, idx, w, src,
                           src_stride, out, f);
    return hipGetLastError();
}

// ============================================================ quadrature fields

FPDE_KERNEL void k_quad_fields(int dim, int64_t nc, int nqe, const int32_t* cells, const double* lam,
                               int64_t M, const double* s, const double* kap, double* qs, double* qk,
                               int f) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nc * nqe) return;
    const int64_t c = q / nqe;
    const int l = (int)(q - c * nqe);
    const double* sf = s + (int64_t)f * M;
    const double* kf = kap + (int64_t)f * M;
    double sv = 0.0, kv = 0.0;
    for (int a = 0; a <= dim; ++a) {
        const int v = cells[a * nc + c];
        sv += lam[a * nqe + l] * sf[v];
        kv += lam[a * nqe + l] * kf[v];
    }
    qs[(int64_t)f * nc * nqe + q] = sv;
    qk[(int64_t)f * nc * nqe + q] = sqrt(kv);
}

hipError_t launch_quad_fields(int dim, int64_t nc, int nqe, const int32_t* cells, const double* lam,
                              int F, int64_t n_nodes, const double* s, const double* kappa,
                              double* qs, double* qk, hipStream_t st) {
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(k_quad_fields, dim3(grid1(nc * nqe)), dim3(256), 0, st, dim, nc, nqe, cells,
                           lam, n_nodes, s, kappa, qs, qk, f);
    return hipGetLastError();
}

// ============================================================ Chebyshev helpers

// 1D Lagrange basis value L_a(x) on the axis points t[0..p)
__device__ __forceinline__ double lag1(const double* t, int p, int a, double x) {
    double v = 1.0;
    const double ta = t[a];
    for (int b = 0; b < p; ++b)
        if (b != a) v *= (x - t[b]) / (ta - t[b]);
    return v;
}

// tensor basis l_alpha(x), alpha = a0 + p*a1
__device__ __forceinline__ double lagk(const double* axes, int dim, int p, int alpha, const double* x) {
    double v = lag1(axes, p, alpha % p, x[0]);
    if (dim == 2) v *= lag1(axes + p, p, alpha / p, x[1]);
    return v;
}

FPDE_KERNEL void k_transfer(H2Tree t, double* E) {
    // E[c][d][b][a] = L^{parent(c), d}_a(t^{c,d}_b)
    const int p = t.p;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)t.dim * p * p;
    if (i >= t.ncl * per) return;
    const int64_t c = i / per;
    int r = (int)(i - c * per);
    const int d = r / (p * p);
    r -= d * p * p;
    const int b = r / p, a = r % p;
    if (c == 0) { E[i] = 0.0; return; }
    const int64_t par = (c - 1) / 2;
    const double* tp = t.axes + (par * t.dim + d) * p;
    const double* tc = t.axes + (c * t.dim + d) * p;
    E[i] = lag1(tp, p, a, tc[b]);
}

hipError_t launch_transfer(const H2Tree& t, double* E, hipStream_t st) {
    int64_t n = t.ncl * t.dim * t.p * t.p;
    hipLaunchKernelGGL(k_transfer, dim3(grid1(n)), dim3(256), 0, st, t, E);
    return hipGetLastError();
}

// parent at `level`: xh[f][par][alpha][r] = sum_{c} sum_beta E_c[beta][alpha] xh[f][c][beta][r]
FPDE_KERNEL void k_up_level(H2Tree t, int64_t c0, int64_t nc_lev, int F, int R, double* xh) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = t.k, p = t.p;
    const int64_t per = (int64_t)k * R;
    if (i >= (int64_t)F * nc_lev * per) return;
    const int f = (int)(i / (nc_lev * per));
    int64_t rem = i - (int64_t)f * nc_lev * per;
    const int64_t par = c0 + rem / per;
    rem %= per;
    const int alpha = (int)(rem / R), r = (int)(rem % R);
    const int a0 = alpha % p, a1 = alpha / p;
    double acc = 0.0;
    for (int ch = 1; ch <= 2; ++ch) {
        const int64_t c = 2 * par + ch;
        const double* Ec = t.E + c * t.dim * p * p;
        const double* xc = xh + (((int64_t)f * t.ncl + c) * k) * R + r;
        for (int beta = 0; beta < k; ++beta) {
            const int b0 = beta % p, b1 = beta / p;
            double e = Ec[b0 * p + a0];
            if (t.dim == 2) e *= Ec[p * p + b1 * p + a1];
            acc += e * xc[(int64_t)beta * R];
        }
    }
    xh[(((int64_t)f * t.ncl + par) * k + alpha) * R + r] = acc;
}

hipError_t launch_up_level(const H2Tree& t, int level, int F, int R, double* xh, hipStream_t st) {
    const int64_t c0 = (int64_t(1) << level) - 1, n = int64_t(1) << level;
    const int64_t tot = (int64_t)F * n * t.k * R;
    hipLaunchKernelGGL(k_up_level, dim3(grid1(tot)), dim3(256), 0, st, t, c0, n, F, R, xh);
    return hipGetLastError();
}

// children of clusters at `level`: yh[f][c][beta][r] += sum_alpha E_c[beta][alpha] yh[f][par][alpha][r]
FPDE_KERNEL void k_down_level(H2Tree t, int64_t c0, int64_t nc_lev, int F, int R, double* yh) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = t.k, p = t.p;
    const int64_t per = (int64_t)k * R;
    const int64_t nch = 2 * nc_lev;
    if (i >= (int64_t)F * nch * per) return;
    const int f = (int)(i / (nch * per));
    int64_t rem = i - (int64_t)f * nch * per;
    const int64_t c = 2 * c0 + 1 + rem / per;
    rem %= per;
    const int beta = (int)(rem / R), r = (int)(rem % R);
    const int64_t par = (c - 1) / 2;
    const double* Ec = t.E + c * t.dim * p * p;
    const int b0 = beta % p, b1 = beta / p;
    const double* yp = yh + (((int64_t)f * t.ncl + par) * k) * R + r;
    double acc = 0.0;
    for (int alpha = 0; alpha < k; ++alpha) {
        const int a0 = alpha % p, a1 = alpha / p;
        double e = Ec[b0 * p + a0];
        if (t.dim == 2) e *= Ec[p * p + b1 * p + a1];
        acc += e * yp[(int64_t)alpha * R];
    }
    yh[(((int64_t)f * t.ncl + c) * k + beta) * R + r] += acc;
}

hipError_t launch_down_level(const H2Tree& t, int level, int F, int R, double* yh, hipStream_t st) {
    const int64_t c0 = (int64_t(1) << level) - 1, n = int64_t(1) << level;
    const int64_t tot = (int64_t)F * 2 * n * t.k * R;
    hipLaunchKernelGGL(k_down_level, dim3(grid1(tot)), dim3(256), 0, st, t, c0, n, F, R, yh);
    return hipGetLastError();
}

// coupling with the kernel generated on the fly at the Chebyshev nodes
FPDE_KERNEL void k_coupling(H2Tree t, int F, int R, double fac, double a_scale, const double* xh,
                            double* yh) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = t.k, p = t.p, dim = t.dim;
    const int64_t per = (int64_t)k * R;
    if (i >= (int64_t)F * t.ncl * per) return;
    const int f = (int)(i / (t.ncl * per));
    int64_t rem = i - (int64_t)f * t.ncl * per;
    const int64_t c = rem / per;
    rem %= per;
    const int alpha = (int)(rem / R), r = (int)(rem % R);
    const double* ax = t.axes + c * dim * p;
    const double x0 = ax[alpha % p];
    const double x1 = dim == 2 ? ax[p + alpha / p] : 0.0;
    const double sa = t.node_s[((int64_t)f * t.ncl + c) * k + alpha];
    const double ka = t.node_k[((int64_t)f * t.ncl + c) * k + alpha];
    double acc = 0.0;
    for (int64_t e = t.far_ptr[c]; e < t.far_ptr[c + 1]; ++e) {
        const int64_t cs = t.far_src[e];
        const double* bx = t.axes + cs * dim * p;
        const double* ns = t.node_s + ((int64_t)f * t.ncl + cs) * k;
        const double* nk = t.node_k + ((int64_t)f * t.ncl + cs) * k;
        const double* xs = xh + (((int64_t)f * t.ncl + cs) * k) * R + r;
        for (int beta = 0; beta < k; ++beta) {
            const double d0 = x0 - bx[beta % p];
            const double d1 = dim == 2 ? x1 - bx[p + beta / p] : 0.0;
            const double r2 = d0 * d0 + d1 * d1;
            const double g = ka * nk[beta] * rpow(r2, (double)dim + sa + ns[beta]);
            acc += g * xs[(int64_t)beta * R];
        }
    }
    yh[(((int64_t)f * t.ncl + c) * k + alpha) * R + r] = fac * a_scale * acc;
}

hipError_t launch_coupling(const H2Tree& t, int F, int R, double fac, double a_scale,
                           const double* xh, double* yh, hipStream_t st) {
    const int64_t tot = (int64_t)F * t.ncl * t.k * R;
    hipLaunchKernelGGL(k_coupling, dim3(grid1(tot)), dim3(256), 0, st, t, F, R, fac, a_scale, xh, yh);
    return hipGetLastError();
}

// ============================================================ density (point H2)

FPDE_KERNEL void k_rho_moments(H2Tree t, const int64_t* perm, const double* qx, const double* qw,
                               int64_t nq, int F, double* xh) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = t.k;
    if (i >= t.nleaf * k) return;
    const int64_t c = t.first_leaf + i / k;
    const int beta = (int)(i % k);
    const double* ax = t.axes + c * t.dim * t.p;
    double acc = 0.0;
    for (int64_t j = t.beg[c]; j < t.end[c]; ++j) {
        const int64_t q = perm[j];
        double x[2] = {qx[q], t.dim == 2 ? qx[nq + q] : 0.0};
        acc += lagk(ax, t.dim, t.p, beta, x) * qw[q];
    }
    for (int f = 0; f < F; ++f) xh[((int64_t)f * t.ncl + c) * k + beta] = acc;
}

hipError_t launch_rho_moments(const H2Tree& t, const int64_t* perm, const double* qx,
                              const double* qw, int64_t nq_all, int F, double* xh, hipStream_t st) {
    hipLaunchKernelGGL(k_rho_moments, dim3(grid1(t.nleaf * t.k)), dim3(256), 0, st, t, perm, qx, qw,
                       nq_all, F, xh);
    return hipGetLastError();
}

FPDE_KERNEL void k_rho_eval(H2Tree t, const int64_t* perm, const int64_t* leaf_of, const double* qx,
                            const uint8_t* q_int, int64_t nq, int F, const double* yh, double* rho) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nq) return;
    const int64_t q = perm[j];
    if (!q_int[q]) return;
    const int64_t c = leaf_of[j];
    const double* ax = t.axes + c * t.dim * t.p;
    double x[2] = {qx[q], t.dim == 2 ? qx[nq + q] : 0.0};
    for (int f = 0; f < F; ++f) {
        const double* y = yh + ((int64_t)f * t.ncl + c) * t.k;
        double acc = 0.0;
        for (int a = 0; a < t.k; ++a) acc += lagk(ax, t.dim, t.p, a, x) * y[a];
        rho[(int64_t)f * nq + q] += acc;
    }
}

// leaf index of each tree position (needed by rho_eval); computed on the fly here
FPDE_KERNEL void k_leaf_of(H2Tree t, int64_t n, int64_t* leaf_of) {
    int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (li >= t.nleaf) return;
    const int64_t c = t.first_leaf + li;
    for (int64_t j = t.beg[c]; j < t.end[c]; ++j) leaf_of[j] = c;
}

hipError_t launch_rho_eval(const H2Tree& t, const int64_t* perm, const double* qx,
                           const uint8_t* q_int, int64_t nq_all, int F, const double* yh,
                           double* rho, hipStream_t st) {
    int64_t* leaf_of = nullptr;
    hipError_t e = hipMallocAsync((void**)&leaf_of, sizeof(int64_t) * nq_all, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_leaf_of, dim3(grid1(t.nleaf)), dim3(256), 0, st, t, nq_all, leaf_of);
    hipLaunchKernelGGL(k_rho_eval, dim3(grid1(nq_all)), dim3(256), 0, st, t, perm, leaf_of, qx, q_int,
                       nq_all, F, yh, rho);
    e = hipGetLastError();
    hipFreeAsync(leaf_of, st);
    return e;
}

// near sums: one 64-thread block per target leaf; source leaves staged in LDS
FPDE_KERNEL void k_rho_near(H2Tree t, const int64_t* perm, const int64_t* near_ptr,
                            const int64_t* near_src, const double* qx, const double* qw,
                            const double* qs, const double* qk, const uint8_t* q_int, int nqe,
                            const int32_t* cells, int64_t nc, int64_t nq, int f, double a_scale,
                            double* rho) {
    __shared__ double sx[64], sy[64], sw[64], ss[64], sk[64];
    __shared__ int sv[64][3];
    const int64_t li = blockIdx.x;
    const int64_t c = t.first_leaf + li;
    const int tid = threadIdx.x;
    const int64_t j = t.beg[c] + tid;
    const bool have = j < t.end[c];
    int64_t q = have ? perm[j] : 0;
    const bool act = have && q_int[q];
    double x0 = 0, x1 = 0, s0 = 0, k0 = 0;
    int tv[3] = {-1, -1, -1};
    if (act) {
        x0 = qx[q];
        x1 = t.dim == 2 ? qx[nq + q] : 0.0;
        s0 = qs[(int64_t)f * nq + q];
        k0 = qk[(int64_t)f * nq + q];
        const int64_t cq = q / nqe;
        for (int a = 0; a <= t.dim; ++a) tv[a] = cells[a * nc + cq];
    }
    double acc = 0.0;
    for (int64_t e = near_ptr[li]; e < near_ptr[li + 1]; ++e) {
        const int64_t cs = near_src[e];
        const int64_t b = t.beg[cs], n = t.end[cs] - t.beg[cs];
        __syncthreads();
        if (tid < n) {
            const int64_t q2 = perm[b + tid];
            sx[tid] = qx[q2];
            sy[tid] = t.dim == 2 ? qx[nq + q2] : 0.0;
            sw[tid] = qw[q2];
            ss[tid] = qs[(int64_t)f * nq + q2];
            sk[tid] = qk[(int64_t)f * nq + q2];
            const int64_t c2 = q2 / nqe;
            for (int a = 0; a < 3; ++a) sv[tid][a] = a <= t.dim ? cells[a * nc + c2] : -2;
        }
        __syncthreads();
        if (act) {
            for (int m = 0; m < n; ++m) {
                bool touch = false;
                for (int a = 0; a <= t.dim; ++a)
                    for (int bb = 0; bb <= t.dim; ++bb) touch |= (tv[a] == sv[m][bb]);
                if (touch) continue;
                const double d0 = x0 - sx[m], d1 = x1 - sy[m];
                acc += k0 * sk[m] * rpow(d0 * d0 + d1 * d1, (double)t.dim + s0 + ss[m]) * sw[m];
            }
        }
    }
    if (act) rho[(int64_t)f * nq + q] += a_scale * acc;
}

hipError_t launch_rho_near(const H2Tree& t, const int64_t* perm, const int64_t* near_ptr,
                           const int64_t* near_src, const double* qx, const double* qw,
                           const double* qs, const double* qk, const uint8_t* q_int, int nqe,
                           const int32_t* cells, int64_t nc, int64_t nq_all, int F, double a_scale,
                           double* rho, hipStream_t st) {
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(k_rho_near, dim3((unsigned)t.nleaf), dim3(64), 0, st, t, perm, near_ptr,
                           near_src, qx, qw, qs, qk, q_int, nqe, cells, nc, nq_all, f, a_scale, rho);
    return hipGetLastError();
}

FPDE_KERNEL void k_rho_exterior(int dim, int64_t nq, const double* qx, const double* qs,
                                const double* qk, const uint8_t* q_int, double R, double s_out,
                                double k_out, double a_scale, int n_theta, double* rho, int f) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq || !q_int[q]) return;
    const double sx = qs[(int64_t)f * nq + q];
    const double sig = sx + s_out;
    const double a = a_scale * qk[(int64_t)f * nq + q] * k_out;
    double val;
    if (dim == 1) {
        const double x = qx[q];
        val = a / sig * (exp(-sig * log(R - x)) + exp(-sig * log(R + x)));
    } else {
        const double x0 = qx[q], x1 = qx[nq + q];
        const double r2 = x0 * x0 + x1 * x1;
        double acc = 0.0;
        const double dth = 2.0 * M_PI / n_theta;
        for (int i = 0; i < n_theta; ++i) {
            double sn, cs;
            sincos(dth * i, &sn, &cs);
            const double mu = x0 * cs + x1 * sn;
            const double tt = sqrt(mu * mu + R * R - r2) - mu;
            acc += exp(-sig * log(tt));
        }
        val = a / sig * acc * dth;
    }
    rho[(int64_t)f * nq + q] += val;
}

hipError_t launch_rho_exterior(int dim, int64_t nq_all, const double* qx, const double* qs,
                               const double* qk, const uint8_t* q_int, int F, double R,
                               double s_out, double k_out_sqrt, double a_scale, int n_theta,
                               double* rho, hipStream_t st) {
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(k_rho_exterior, dim3(grid1(nq_all)), dim3(256), 0, st, dim, nq_all, qx, qs,
                           qk, q_int, R, s_out, k_out_sqrt, a_scale, n_theta, rho, f);
    return hipGetLastError();
}

// ============================================================ weighted mass

FPDE_KERNEL void k_mass_local(int dim, int64_t nci, const int64_t* icells, int nqe, const double* lam,
                              const double* qw, const double* rho, int64_t nq, int F, double* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)F * nci) return;
    const int f = (int)(i / nci);
    const int64_t ci = i - (int64_t)f * nci;
    const int64_t c = icells[ci];
    const int nv = dim + 1;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int l = 0; l < nqe; ++l) {
        const int64_t q = c * nqe + l;
        const double wr = qw[q] * rho[(int64_t)f * nq + q];
        for (int a = 0; a < nv; ++a)
            for (int b = a; b < nv; ++b) acc[a * 3 + b] += wr * lam[a * nqe + l] * lam[b * nqe + l];
    }
    double* o = out + ((int64_t)f * nci + ci) * 9;
    for (int a = 0; a < 9; ++a) o[a] = 2.0 * acc[a];
}

hipError_t launch_mass_local(int dim, int64_t n_int_cells, const int64_t* int_cells, int nqe,
                             const double* lam, const double* qw, const double* rho, int64_t nq_all,
                             int F, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_mass_local, dim3(grid1((int64_t)F * n_int_cells)), dim3(256), 0, st, dim,
                       n_int_cells, int_cells, nqe, lam, qw, rho, nq_all, F, out);
    return hipGetLastError();
}

// ============================================================ leaf bases

FPDE_KERNEL void k_basis(H2Tree t, const int64_t* perm, const int64_t* leaf_of, const int64_t* nc_ptr,
                         const int64_t* nc_cell, const int8_t* nc_slot, int nqe, const double* qx,
                         const double* qw, const double* lam, int64_t nq, int64_t N, double* U) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = t.k;
    if (i >= N * k) return;
    const int64_t j = i / k;
    const int alpha = (int)(i % k);
    const int64_t node = perm[j];
    const int64_t c = leaf_of[j];
    const double* ax = t.axes + c * t.dim * t.p;
    double acc = 0.0;
    for (int64_t e = nc_ptr[node]; e < nc_ptr[node + 1]; ++e) {
        const int64_t cell = nc_cell[e];
        const int slot = nc_slot[e];
        for (int l = 0; l < nqe; ++l) {
            const int64_t q = cell * nqe + l;
            double x[2] = {qx[q], t.dim == 2 ? qx[nq + q] : 0.0};
            acc += qw[q] * lam[slot * nqe + l] * lagk(ax, t.dim, t.p, alpha, x);
        }
    }
    U[j * k + alpha] = acc;
}

hipError_t launch_basis_n(const H2Tree& t, int64_t N, const int64_t* perm, const int64_t* nc_ptr,
                          const int64_t* nc_cell, const int8_t* nc_slot, int nqe, const double* qx,
                          const double* qw, const double* lam, int64_t nq_all, double* U,
                          hipStream_t st) {
    int64_t* leaf_of = nullptr;
    hipError_t e = hipMallocAsync((void**)&leaf_of, sizeof(int64_t) * N, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_leaf_of, dim3(grid1(t.nleaf)), dim3(256), 0, st, t, N, leaf_of);
    hipLaunchKernelGGL(k_basis, dim3(grid1(N * t.k)), dim3(256), 0, st, t, perm, leaf_of, nc_ptr,
                       nc_cell, nc_slot, nqe, qx, qw, lam, nq_all, N, U);
    e = hipGetLastError();
    hipFreeAsync(leaf_of, st);
    return e;
}

// ============================================================ near leaf blocks of K~

// Block per (near pair, chunk of JC source columns).
// Phase A: R[lc][a][jj] = sum_{tau' in S_j, tau' not touching tau_lc} sum_q sum_q'
//                         w w' gamma(q,q') lam_a(q) psi_j(q')
// Phase B: blk[it][j] = -2 sum_{(lc,slot) around row node} R[lc][slot][jj]
constexpr int kJC = 8;

FPDE_KERNEL void k_near_blocks(H2Tree t, NearPlan P, const int64_t* perm, const int32_t* cells, int nqe,
                               int64_t nc, const double* qx, const double* qw, const double* qs,
                               const double* qk, const double* lam, int64_t nq, int f, double a_scale,
                               double* nb) {
    extern __shared__ double R[];
    const int64_t nchunk = (P.cap + kJC - 1) / kJC;
    const int64_t pr = blockIdx.x / nchunk;
    const int j0 = (int)(blockIdx.x % nchunk) * kJC;
    const int64_t ct = P.tgt[pr], cs = P.src[pr];
    const int64_t lt = ct - t.first_leaf;
    const int64_t pb = P.patch_ptr[lt], npc = P.patch_ptr[lt + 1] - pb;
    const int64_t sb = t.beg[cs], ns = t.end[cs] - t.beg[cs];
    const int nv = t.dim + 1;
    const double* qsf = qs + (int64_t)f * nq;
    const double* qkf = qk + (int64_t)f * nq;
    // phase A
    for (int64_t item = threadIdx.x; item < npc * kJC; item += blockDim.x) {
        const int64_t lc = item / kJC;
        const int jj = (int)(item % kJC);
        double acc[3] = {0.0, 0.0, 0.0};
        if (j0 + jj < ns) {
            const int64_t cell = P.patch_cell[pb + lc];
            const int64_t jn = perm[sb + j0 + jj];
            int tv[3];
            for (int a = 0; a < nv; ++a) tv[a] = cells[a * nc + cell];
            for (int64_t e = P.nc_ptr[jn]; e < P.nc_ptr[jn + 1]; ++e) {
                const int64_t c2 = P.nc_cell[e];
                const int slot = P.nc_slot[e];
                bool touch = false;
                for (int a = 0; a < nv; ++a)
                    for (int b = 0; b < nv; ++b) touch |= (tv[a] == cells[b * nc + c2]);
                if (touch) continue;
                for (int l = 0; l < nqe; ++l) {
                    const int64_t q = cell * nqe + l;
                    const double x0 = qx[q], x1 = t.dim == 2 ? qx[nq + q] : 0.0;
                    const double s0 = qsf[q], k0 = qkf[q];
                    double g = 0.0;
                    for (int l2 = 0; l2 < nqe; ++l2) {
                        const int64_t q2 = c2 * nqe + l2;
                        const double d0 = x0 - qx[q2];
                        const double d1 = t.dim == 2 ? x1 - qx[nq + q2] : 0.0;
                        g += qw[q2] * lam[slot * nqe + l2] * qkf[q2] *
                             rpow(d0 * d0 + d1 * d1, (double)t.dim + s0 + qsf[q2]);
                    }
                    g *= qw[q] * k0;
                    for (int a = 0; a < nv; ++a) acc[a] += g * lam[a * nqe + l];
                }
            }
        }
        for (int a = 0; a < nv; ++a) R[(lc * 3 + a) * kJC + jj] = acc[a];
    }
    __syncthreads();
    // phase B
    const int64_t tb = t.beg[ct], nt = t.end[ct] - t.beg[ct];
    double* out = nb + (((int64_t)f * P.npairs + pr) * P.cap) * P.cap;
    for (int64_t item = threadIdx.x; item < P.cap * kJC; item += blockDim.x) {
        const int64_t it = item / kJC;
        const int jj = (int)(item % kJC);
        if (j0 + jj >= P.cap) continue;
        double v = 0.0;
        if (it < nt && j0 + jj < ns) {
            const int64_t row = tb + it;
            for (int64_t e = P.row_ptr[row]; e < P.row_ptr[row + 1]; ++e)
                v += R[(P.row_lcell[e] * 3 + P.row_slot[e]) * kJC + jj];
            v *= -2.0 * a_scale;
        }
        out[it * P.cap + j0 + jj] = v;
    }
}

hipError_t launch_near_blocks_lds(const H2Tree& t, const NearPlan& np, int64_t max_patch,
                                  const int64_t* perm, const int32_t* cells, int nqe, int64_t nc,
                                  const double* qx, const double* qw, const double* qs,
                                  const double* qk, const double* lam, int64_t nq_all, int F,
                                  double a_scale, double* nb, hipStream_t st) {
    if (np.npairs == 0) return hipSuccess;
    const size_t lds = (size_t)max_patch * 3 * kJC * sizeof(double);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const int64_t nchunk = (np.cap + kJC - 1) / kJC;
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(k_near_blocks, dim3((unsigned)(np.npairs * nchunk)), dim3(256), lds, st, t, np,
                           perm, cells, nqe, nc, qx, qw, qs, qk, lam, nq_all, f, a_scale, nb);
    return hipGetLastError();
}

// ============================================================ load vector

FPDE_KERNEL void k_load(int64_t N, const int64_t* nc_ptr, const int64_t* nc_cell, const int8_t* nc_slot,
                        const int32_t* cells, int64_t nc, int nqe, int nv, const double* lam,
                        const double* qw, const uint8_t* cell_int, const double* f_nodal, double* F) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (int64_t e = nc_ptr[i]; e < nc_ptr[i + 1]; ++e) {
        const int64_t c = nc_cell[e];
        if (!cell_int[c]) continue;
        const int slot = nc_slot[e];
        for (int l = 0; l < nqe; ++l) {
            double fq = 0.0;
            for (int a = 0; a < nv; ++a) fq += lam[a * nqe + l] * f_nodal[cells[a * nc + c]];
            acc += qw[c * nqe + l] * lam[slot * nqe + l] * fq;
        }
    }
    F[i] = acc;
}

hipError_t launch_load_nv(int64_t N, int nv, const int64_t* nc_ptr, const int64_t* nc_cell,
                          const int8_t* nc_slot, const int32_t* cells, int64_t nc, int nqe,
                          const double* lam, const double* qw, const uint8_t* cell_int,
                          const double* f_nodal, double* F, hipStream_t st) {
    hipLaunchKernelGGL(k_load, dim3(grid1(N)), dim3(256), 0, st, N, nc_ptr, nc_cell, nc_slot, cells, nc,
                       nqe, nv, lam, qw, cell_int, f_nodal, F);
    return hipGetLastError();
}

// ============================================================ apply

FPDE_KERNEL void k_gather(int64_t N, const int64_t* perm, int F, int R, int dtype, const void* x,
                          double* xt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)F * N * R) return;
    const int f = (int)(i / (N * R));
    int64_t rem = i - (int64_t)f * N * R;
    const int64_t t = rem / R;
    const int r = (int)(rem % R);
    const int64_t src = ((int64_t)f * N + perm[t]) * R + r;
    const double v = dtype == 0 ? ((const double*)x)[src] : (double)((const float*)x)[src];
    xt[i] = v;
}

hipError_t launch_gather(const ApplyPlan& a, int F, int R, int dtype, const void* x, double* xt,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3(grid1((int64_t)F * a.N * R)), dim3(256), 0, st, a.N, a.perm, F, R,
                       dtype, x, xt);
    return hipGetLastError();
}

FPDE_KERNEL void k_leaf_up(ApplyPlan a, H2Tree t, int F, int R, const double* xt, double* xh) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = t.k;
    const int64_t per = (int64_t)k * R;
    if (i >= (int64_t)F * t.nleaf * per) return;
    const int f = (int)(i / (t.nleaf * per));
    int64_t rem = i - (int64_t)f * t.nleaf * per;
    const int64_t li = rem / per;
    rem %= per;
    const int alpha = (int)(rem / R), r = (int)(rem % R);
    const int64_t c = t.first_leaf + li;
    double acc = 0.0;
    for (int64_t j = t.beg[c]; j < t.end[c]; ++j)
        acc += a.U[j * k + alpha] * xt[((int64_t)f * a.N + j) * R + r];
    xh[(((int64_t)f * t.ncl + c) * k + alpha) * R + r] = acc;
}

hipError_t launch_leaf_up(const ApplyPlan& a, const H2Tree& t, int F, int R, const double* xt,
                          double* xh, hipStream_t st) {
    hipLaunchKernelGGL(k_leaf_up, dim3(grid1((int64_t)F * t.nleaf * t.k * R)), dim3(256), 0, st, a, t, F,
                       R, xt, xh);
    return hipGetLastError();
}

// Output per tree row: one 16-lane group per (row, rhs); lanes split the columns
// of the near blocks (row-major [cap][cap]) and the CSR row, then reduce.
FPDE_KERNEL void k_leaf_out(ApplyPlan a, H2Tree t, int parts, int F, int R, const double* csr_val,
                            const double* xt, const double* yh, int dtype, void* y) {
    const int g = threadIdx.x & 15;
    const int64_t item = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    if (item >= (int64_t)F * a.N * R) return;
    const int f = (int)(item / (a.N * R));
    int64_t rem = item - (int64_t)f * a.N * R;
    const int64_t row = rem / R;
    const int r = (int)(rem % R);
    const double* xf = xt + (int64_t)f * a.N * R;
    double acc = 0.0;
    if (csr_val) {
        const double* v = csr_val + (int64_t)f * a.nnz;
        for (int64_t e = a.csr_ptr[row] + g; e < a.csr_ptr[row + 1]; e += 16)
            acc += v[e] * xf[(int64_t)a.csr_col[e] * R + r];
    }
    // leaf of this row: binary search over leaf_beg
    int64_t lo = 0, hi = a.nleaf;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (a.leaf_beg[mid] <= row) lo = mid; else hi = mid;
    }
    const int64_t li = lo;
    const int64_t it = row - a.leaf_beg[li];
    if (parts & 4) {
        for (int64_t e = a.near_ptr[li]; e < a.near_ptr[li + 1]; ++e) {
            const int64_t ls = a.near_src[e];
            const int64_t sb = a.leaf_beg[ls], ns = a.leaf_beg[ls + 1] - sb;
            const double* blk = a.near_blk + (((int64_t)f * a.npairs + e) * a.cap + it) * a.cap;
            for (int64_t jc = g; jc < ns; jc += 16) acc += blk[jc] * xf[(sb + jc) * R + r];
        }
    }
    if ((parts & 8) && g == 0) {
        const double* yl = yh + (((int64_t)f * t.ncl + t.first_leaf + li) * t.k) * R + r;
        const double* u = a.U + row * t.k;
        for (int al = 0; al < t.k; ++al) acc += u[al] * yl[(int64_t)al * R];
    }
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
    if (g == 0) {
        const int64_t dst = ((int64_t)f * a.N + a.perm[row]) * R + r;
        if (dtype == 0) ((double*)y)[dst] = acc;
        else ((float*)y)[dst] = (float)acc;
    }
}

hipError_t launch_leaf_out(const ApplyPlan& a, const H2Tree& t, int parts, int F, int R,
                           const double* csr_val_override, const double* xt, const double* yh,
                           int dtype, void* y, hipStream_t st) {
    const int64_t items = (int64_t)F * a.N * R;
    hipLaunchKernelGGL(k_leaf_out, dim3(grid1(items, 16)), dim3(256), 0, st, a, t, parts, F, R,
                       csr_val_override, xt, yh, dtype, y);
    return hipGetLastError();
}

// ============================================================ small vector kernels

FPDE_KERNEL void k_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = a * x[i] + b * y[i];
}

hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_axpby, dim3(grid1(n)), dim3(256), 0, st, n, a, x, b, y, z);
    return hipGetLastError();
}

FPDE_KERNEL void k_fill(int64_t n, double v, double* x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

hipError_t launch_fill(int64_t n, double v, double* x, hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3(grid1(n)), dim3(256), 0, st, n, v, x);
    return hipGetLastError();
}

}  // namespace fpde

// ============================================================ apply, fused far field

namespace fpde {

// Coupling matrices of the far pairs, stored transposed: St[f][e][beta][alpha]
// = fac * a_scale * sqrt(kappa_a kappa_b) |xi_a - xi'_b|^{-(d + s_a + s'_b)}
FPDE_KERNEL void k_coupling_store(H2Tree t, int64_t nfar, const int64_t* far_tgt, int F, double fac,
                                  double a_scale, double* St) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = t.k, p = t.p, dim = t.dim;
    const int64_t kk = (int64_t)k * k;
    if (i >= (int64_t)F * nfar * kk) return;
    const int f = (int)(i / (nfar * kk));
    int64_t rem = i - (int64_t)f * nfar * kk;
    const int64_t e = rem / kk;
    rem %= kk;
    const int beta = (int)(rem / k), alpha = (int)(rem % k);
    const int64_t c = far_tgt[e], cs = t.far_src[e];
    const double* ax = t.axes + c * dim * p;
    const double* bx = t.axes + cs * dim * p;
    const double d0 = ax[alpha % p] - bx[beta % p];
    const double d1 = dim == 2 ? ax[p + alpha / p] - bx[p + beta / p] : 0.0;
    const double sa = t.node_s[((int64_t)f * t.ncl + c) * k + alpha];
    const double ka = t.node_k[((int64_t)f * t.ncl + c) * k + alpha];
    const double sb = t.node_s[((int64_t)f * t.ncl + cs) * k + beta];
    const double kb = t.node_k[((int64_t)f * t.ncl + cs) * k + beta];
    St[i] = fac * a_scale * ka * kb * rpow(d0 * d0 + d1 * d1, (double)dim + sa + sb);
}

hipError_t launch_coupling_store(const H2Tree& t, int64_t nfar, const int64_t* far_tgt, int F, double fac,
                                 double a_scale, double* St, hipStream_t st) {
    const int64_t n = (int64_t)F * nfar * t.k * t.k;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_coupling_store, dim3(grid1(n)), dim3(256), 0, st, t, nfar, far_tgt, F, fac, a_scale, St);
    return hipGetLastError();
}

// yh[f][c][alpha][r] = sum_{e in far(c)} sum_beta St[f][e][beta][alpha] xh[f][src(e)][beta][r]
// one block per (cluster, field); threads = (alpha lane in 0..63) x (4 pair groups), k <= 64
FPDE_KERNEL void k_coupling_apply(H2Tree t, int F, int R, const double* St, const double* xh, double* yh) {
    __shared__ double red[4][64];
    const int64_t c = blockIdx.x;
    const int f = blockIdx.y;
    const int k = t.k;
    const int al = threadIdx.x & 63, pg = threadIdx.x >> 6;
    const int64_t e0 = t.far_ptr[c], e1 = t.far_ptr[c + 1];
    const int64_t kk = (int64_t)k * k;
    const int64_t nfar = t.far_ptr[t.ncl];
    for (int r = 0; r < R; ++r) {
        double acc = 0.0;
        if (al < k) {
            for (int64_t e = e0 + pg; e < e1; e += 4) {
                const double* S = St + ((int64_t)f * nfar + e) * kk + al;
                const double* xs = xh + (((int64_t)f * t.ncl + t.far_src[e]) * k) * R + r;
                for (int b = 0; b < k; ++b) acc += S[(int64_t)b * k] * xs[(int64_t)b * R];
            }
        }
        red[pg][al] = acc;
        __syncthreads();
        if (threadIdx.x < 64 && al < k) {
            const double v = (red[0][al] + red[1][al]) + (red[2][al] + red[3][al]);
            yh[(((int64_t)f * t.ncl + c) * k + al) * R + r] = v;
        }
        __syncthreads();
    }
}

hipError_t launch_coupling_apply(const H2Tree& t, int F, int R, const double* St, const double* xh, double* yh,
                                 hipStream_t st) {
    hipLaunchKernelGGL(k_coupling_apply, dim3((unsigned)t.ncl, F), dim3(256), 0, st, t, F, R, St, xh, yh);
    return hipGetLastError();
}

// Parent coefficients from two children with the Kronecker transfers (one output)
__device__ __forceinline__ double up_one(const H2Tree& t, const double* Ec1, const double* Ec2, const double* x1,
                                         const double* x2, int alpha, int R) {
    const int p = t.p, k = t.k;
    const int a0 = alpha % p, a1 = alpha / p;
    double acc = 0.0;
    for (int beta = 0; beta < k; ++beta) {
        const int b0 = beta % p, b1 = beta / p;
        double e1 = Ec1[b0 * p + a0], e2 = Ec2[b0 * p + a0];
        if (t.dim == 2) {
            e1 *= Ec1[p * p + b1 * p + a1];
            e2 *= Ec2[p * p + b1 * p + a1];
        }
        acc += e1 * x1[(int64_t)beta * R];
        acc += e2 * x2[(int64_t)beta * R];
    }
    return acc;
}

// gather x into tree order + leaf upsweep + levels below the subtree root, one block per
// (subtree root at level ls, field).  LDS: U rows of the subtree, x rows, coefficients.
FPDE_KERNEL void k_up_sub(ApplyPlan a, H2Tree t, int ls, int F, int R, int dtype, const void* x, double* xt,
                          double* xh) {
    extern __shared__ double sm[];
    const int f = blockIdx.y;
    const int64_t c = ((int64_t(1) << ls) - 1) + blockIdx.x;   // subtree root
    const int64_t b = t.beg[c], n = t.end[c] - t.beg[c];
    const int k = t.k;
    double* sU = sm;                       // [n][k]
    double* sx = sU + n * k;               // [n][R]
    const int depth = t.L - ls;
    double* sc = sx + n * R;               // coefficients of the subtree clusters [(2^{depth+1}-1)][k][R]
    const double* xf_in = (const double*)x;
    for (int64_t i = threadIdx.x; i < n * R; i += blockDim.x) {
        const int64_t row = i / R;
        const int r = (int)(i % R);
        const int64_t src = ((int64_t)f * a.N + a.perm[b + row]) * R + r;
        const double v = dtype == 0 ? xf_in[src] : (double)((const float*)x)[src];
        sx[i] = v;
        xt[((int64_t)f * a.N + b) * R + i] = v;
    }
    for (int64_t i = threadIdx.x; i < n * k; i += blockDim.x) sU[i] = a.U[b * k + i];
    __syncthreads();
    // local heap index of cluster cc in the subtree: l = (cc+1) - (c+1)*2^{lev-ls} + (2^{lev-ls} - 1)
    auto local = [&](int64_t cc, int lev) -> int64_t {
        const int64_t w = int64_t(1) << (lev - ls);
        return (w - 1) + (cc + 1 - (c + 1) * w);
    };
    // leaves
    const int64_t nl = int64_t(1) << depth;
    const int64_t l0 = ((c + 1) << depth) - 1;   // first leaf of the subtree
    for (int64_t i = threadIdx.x; i < nl * k * R; i += blockDim.x) {
        const int64_t li = i / ((int64_t)k * R);
        const int al = (int)((i / R) % k), r = (int)(i % R);
        const int64_t cc = l0 + li;
        double acc = 0.0;
        for (int64_t j = t.beg[cc] - b; j < t.end[cc] - b; ++j) acc += sU[j * k + al] * sx[j * R + r];
        sc[(local(cc, t.L) * k + al) * R + r] = acc;
        xh[(((int64_t)f * t.ncl + cc) * k + al) * R + r] = acc;
    }
    __syncthreads();
    for (int lev = t.L - 1; lev >= ls; --lev) {
        const int64_t w = int64_t(1) << (lev - ls);
        const int64_t cfirst = ((c + 1) << (lev - ls)) - 1;
        for (int64_t i = threadIdx.x; i < w * k * R; i += blockDim.x) {
            const int64_t cc = cfirst + i / ((int64_t)k * R);
            const int al = (int)((i / R) % k), r = (int)(i % R);
            const int64_t ch1 = 2 * cc + 1, ch2 = 2 * cc + 2;
            const double* x1 = sc + (local(ch1, lev + 1) * k) * R + r;
            const double* x2 = sc + (local(ch2, lev + 1) * k) * R + r;
            const double v = up_one(t, t.E + ch1 * t.dim * t.p * t.p, t.E + ch2 * t.dim * t.p * t.p, x1, x2, al, R);
            sc[(local(cc, lev) * k + al) * R + r] = v;
            xh[(((int64_t)f * t.ncl + cc) * k + al) * R + r] = v;
        }
        __syncthreads();
    }
}

// levels ls-1 .. 0 in one block per field (1024 threads)
__global__ __launch_bounds__(1024) void k_up_top(H2Tree t, int ls, int F, int R, double* xh) {
    const int f = blockIdx.x;
    const int k = t.k;
    for (int lev = ls - 1; lev >= 0; --lev) {
        const int64_t c0 = (int64_t(1) << lev) - 1, w = int64_t(1) << lev;
        for (int64_t i = threadIdx.x; i < w * k * R; i += blockDim.x) {
            const int64_t cc = c0 + i / ((int64_t)k * R);
            const int al = (int)((i / R) % k), r = (int)(i % R);
            const int64_t ch1 = 2 * cc + 1, ch2 = 2 * cc + 2;
            const double* x1 = xh + (((int64_t)f * t.ncl + ch1) * k) * R + r;
            const double* x2 = xh + (((int64_t)f * t.ncl + ch2) * k) * R + r;
            xh[(((int64_t)f * t.ncl + cc) * k + al) * R + r] =
                up_one(t, t.E + ch1 * t.dim * t.p * t.p, t.E + ch2 * t.dim * t.p * t.p, x1, x2, al, R);
        }
        __syncthreads();
    }
}

// yh(c) += E_c yh(parent) for levels 1..ls (top-down), one block per field (1024 threads)
__global__ __launch_bounds__(1024) void k_down_top(H2Tree t, int ls, int F, int R, double* yh) {
    const int f = blockIdx.x;
    const int k = t.k, p = t.p;
    for (int lev = 1; lev <= ls; ++lev) {
        const int64_t c0 = (int64_t(1) << lev) - 1, w = int64_t(1) << lev;
        for (int64_t i = threadIdx.x; i < w * k * R; i += blockDim.x) {
            const int64_t cc = c0 + i / ((int64_t)k * R);
            const int be = (int)((i / R) % k), r = (int)(i % R);
            const int64_t par = (cc - 1) / 2;
            const double* Ec = t.E + cc * t.dim * p * p;
            const double* yp = yh + (((int64_t)f * t.ncl + par) * k) * R + r;
            const int b0 = be % p, b1 = be / p;
            double acc = 0.0;
            for (int al = 0; al < k; ++al) {
                double e = Ec[b0 * p + al % p];
                if (t.dim == 2) e *= Ec[p * p + b1 * p + al / p];
                acc += e * yp[(int64_t)al * R];
            }
            yh[(((int64_t)f * t.ncl + cc) * k + be) * R + r] += acc;
        }
        __syncthreads();
    }
}

// Output: one block per (field, leaf, 16-row block).  The block first completes the
// downsweep from the level-ls ancestor to its leaf (in LDS), then 16 lanes per row
// accumulate the CSR row, the near blocks (4 contiguous columns per lane) and U yh.
FPDE_KERNEL void k_out(ApplyPlan a, H2Tree t, int ls, int parts, int F, int R, const double* csr_val,
                       const double* xt, const double* yh, int dtype, void* y) {
    extern __shared__ double sy[];          // [2][k][R] ping-pong for the walk
    const int f = blockIdx.y;
    const int64_t nrb = (a.cap + 15) / 16;
    const int64_t li = blockIdx.x / nrb;
    const int rb = (int)(blockIdx.x % nrb);
    const int k = t.k, p = t.p;
    const int64_t leafc = t.first_leaf + li;
    const int64_t kR = (int64_t)k * R;
    double* cur = sy;
    double* nxt = sy + kR;
    const bool far = (parts & 8) != 0;
    if (far) {
        // ancestor at level ls (or the leaf itself if ls == L)
        const int64_t anc = ((leafc + 1) >> (t.L - ls)) - 1;
        for (int64_t i = threadIdx.x; i < kR; i += blockDim.x) cur[i] = yh[((int64_t)f * t.ncl + anc) * kR + i];
        __syncthreads();
        for (int lev = ls + 1; lev <= t.L; ++lev) {
            const int64_t cc = ((leafc + 1) >> (t.L - lev)) - 1;
            const double* Ec = t.E + cc * t.dim * p * p;
            for (int64_t i = threadIdx.x; i < kR; i += blockDim.x) {
                const int be = (int)(i / R), r = (int)(i % R);
                const int b0 = be % p, b1 = be / p;
                double acc = yh[((int64_t)f * t.ncl + cc) * kR + i];
                for (int al = 0; al < k; ++al) {
                    double e = Ec[b0 * p + al % p];
                    if (t.dim == 2) e *= Ec[p * p + b1 * p + al / p];
                    acc += e * cur[(int64_t)al * R + r];
                }
                nxt[i] = acc;
            }
            __syncthreads();
            double* tmp = cur; cur = nxt; nxt = tmp;
        }
    }
    const int g = threadIdx.x & 15;
    const int64_t it = (int64_t)rb * 16 + (threadIdx.x >> 4);
    const int64_t lb = a.leaf_beg[li], nt = a.leaf_beg[li + 1] - lb;
    if (it >= nt) return;
    const int64_t row = lb + it;
    const double* xf = xt + (int64_t)f * a.N * R;
    for (int r = 0; r < R; ++r) {
        double acc = 0.0;
        if (csr_val) {
            const double* v = csr_val + (int64_t)f * a.nnz;
            for (int64_t e = a.csr_ptr[row] + g; e < a.csr_ptr[row + 1]; e += 16)
                acc += v[e] * xf[(int64_t)a.csr_col[e] * R + r];
        }
        if (parts & 4) {
            const int64_t cap = a.cap;
            for (int64_t e = a.near_ptr[li]; e < a.near_ptr[li + 1]; ++e) {
                const int64_t ls_ = a.near_src[e];
                const int64_t sb = a.leaf_beg[ls_], ns = a.leaf_beg[ls_ + 1] - sb;
                const double* blk = a.near_blk + (((int64_t)f * a.npairs + e) * cap + it) * cap;
                const int64_t c0 = 4 * g;
                if (R == 1 && (cap & 3) == 0 && c0 + 4 <= ns) {
                    const double2 b01 = *(const double2*)(blk + c0);
                    const double2 b23 = *(const double2*)(blk + c0 + 2);
                    const double* xs = xf + sb + c0;
                    acc += b01.x * xs[0] + b01.y * xs[1] + b23.x * xs[2] + b23.y * xs[3];
                } else {
                    for (int64_t jc = c0; jc < c0 + 4 && jc < ns; ++jc) acc += blk[jc] * xf[(sb + jc) * R + r];
                }
                // columns beyond 64 when cap > 64
                for (int64_t jc = 64 + g; jc < ns; jc += 16) acc += blk[jc] * xf[(sb + jc) * R + r];
            }
        }
        if (far) {
            const double* u = a.U + row * k;
            for (int al = g; al < k; al += 16) acc += u[al] * cur[(int64_t)al * R + r];
        }
        for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
        if (g == 0) {
            const int64_t dst = ((int64_t)f * a.N + a.perm[row]) * R + r;
            if (dtype == 0) ((double*)y)[dst] = acc;
            else ((float*)y)[dst] = (float)acc;
        }
    }
}

hipError_t launch_apply_fused(const ApplyPlan& a, const H2Tree& t, int ls, int parts, int F, int R,
                              const double* csr_val, const double* St, int dtype, const void* x, double* xt,
                              double* xh, double* yh, void* y, hipStream_t st, hipEvent_t* ev) {
    const int k = t.k;
    if (ev) hipEventRecord(ev[0], st);
    if (parts & 8) {
        const int64_t nsub = int64_t(1) << ls;
        // subtree of (2^{L-ls}) leaves holds at most 2^{L-ls} * cap rows
        const int64_t rows = (int64_t(1) << (t.L - ls)) * a.cap;
        const int64_t ncl_sub = (int64_t(2) << (t.L - ls)) - 1;
        const size_t lds = sizeof(double) * (rows * k + rows * R + ncl_sub * k * R);
        hipLaunchKernelGGL(k_up_sub, dim3((unsigned)nsub, F), dim3(256), lds, st, a, t, ls, F, R, dtype, x, xt, xh);
        if (ev) hipEventRecord(ev[1], st);
        if (ls > 0) hipLaunchKernelGGL(k_up_top, dim3(F), dim3(1024), 0, st, t, ls, F, R, xh);
        hipLaunchKernelGGL(k_coupling_apply, dim3((unsigned)t.ncl, F), dim3(256), 0, st, t, F, R, St, xh, yh);
        if (ls > 0) hipLaunchKernelGGL(k_down_top, dim3(F), dim3(1024), 0, st, t, ls, F, R, yh);
    } else {
        hipLaunchKernelGGL(k_gather, dim3(grid1((int64_t)F * a.N * R)), dim3(256), 0, st, a.N, a.perm, F, R, dtype, x,
                           xt);
        if (ev) hipEventRecord(ev[1], st);
    }
    if (ev) hipEventRecord(ev[2], st);
    const int64_t nrb = (a.cap + 15) / 16;
    const size_t lds_out = sizeof(double) * 2 * k * R;
    hipLaunchKernelGGL(k_out, dim3((unsigned)(a.nleaf * nrb), F), dim3(256), lds_out, st, a, t, ls, parts, F, R,
                       csr_val, xt, yh, dtype, y);
    if (ev) hipEventRecord(ev[3], st);
    return hipGetLastError();
}

}  // namespace fpde

// ============================================================ apply, fork/join variant

namespace fpde {

// tmp[f][e][alpha][r] = sum_beta St[f][e][beta][alpha] xh[f][src(e)][beta][r]   (one thread per output)
FPDE_KERNEL void k_coupling_pairs(H2Tree t, int64_t nfar, int F, int R, const double* St, const double* xh,
                                  double* tmp) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = t.k;
    const int64_t per = (int64_t)k * R;
    if (i >= (int64_t)F * nfar * per) return;
    const int f = (int)(i / (nfar * per));
    int64_t rem = i - (int64_t)f * nfar * per;
    const int64_t e = rem / per;
    rem %= per;
    const int al = (int)(rem / R), r = (int)(rem % R);
    const double* S = St + ((int64_t)f * nfar + e) * k * k + al;
    const double* xs = xh + (((int64_t)f * t.ncl + t.far_src[e]) * k) * R + r;
    double acc = 0.0;
#pragma unroll 5
    for (int b = 0; b < k; ++b) acc += S[(int64_t)b * k] * xs[(int64_t)b * R];
    tmp[i] = acc;
}

// yh[f][c][alpha][r] = sum_{e in far(c)} tmp[f][e][alpha][r]   (fixed order)
FPDE_KERNEL void k_coupling_reduce(H2Tree t, int64_t nfar, int F, int R, const double* tmp, double* yh) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = t.k;
    const int64_t per = (int64_t)k * R;
    if (i >= (int64_t)F * t.ncl * per) return;
    const int f = (int)(i / (t.ncl * per));
    int64_t rem = i - (int64_t)f * t.ncl * per;
    const int64_t c = rem / per;
    rem %= per;
    double acc = 0.0;
    for (int64_t e = t.far_ptr[c]; e < t.far_ptr[c + 1]; ++e) acc += tmp[((int64_t)f * nfar + e) * per + rem];
    yh[i] = acc;
}

// subtree upsweep from x already in tree order
FPDE_KERNEL void k_up_sub_xt(ApplyPlan a, H2Tree t, int ls, int F, int R, const double* xt, double* xh) {
    extern __shared__ double sm[];
    const int f = blockIdx.y;
    const int64_t c = ((int64_t(1) << ls) - 1) + blockIdx.x;
    const int64_t b = t.beg[c], n = t.end[c] - t.beg[c];
    const int k = t.k;
    double* sU = sm;
    double* sx = sU + n * k;
    const int depth = t.L - ls;
    double* sc = sx + n * R;
    for (int64_t i = threadIdx.x; i < n * R; i += blockDim.x) sx[i] = xt[((int64_t)f * a.N + b) * R + i];
    for (int64_t i = threadIdx.x; i < n * k; i += blockDim.x) sU[i] = a.U[b * k + i];
    __syncthreads();
    auto local = [&](int64_t cc, int lev) -> int64_t {
        const int64_t w = int64_t(1) << (lev - ls);
        return (w - 1) + (cc + 1 - (c + 1) * w);
    };
    const int64_t nl = int64_t(1) << depth;
    const int64_t l0 = ((c + 1) << depth) - 1;
    for (int64_t i = threadIdx.x; i < nl * k * R; i += blockDim.x) {
        const int64_t li = i / ((int64_t)k * R);
        const int al = (int)((i / R) % k), r = (int)(i % R);
        const int64_t cc = l0 + li;
        double acc = 0.0;
        for (int64_t j = t.beg[cc] - b; j < t.end[cc] - b; ++j) acc += sU[j * k + al] * sx[j * R + r];
        sc[(local(cc, t.L) * k + al) * R + r] = acc;
        xh[(((int64_t)f * t.ncl + cc) * k + al) * R + r] = acc;
    }
    __syncthreads();
    for (int lev = t.L - 1; lev >= ls; --lev) {
        const int64_t w = int64_t(1) << (lev - ls);
        const int64_t cfirst = ((c + 1) << (lev - ls)) - 1;
        for (int64_t i = threadIdx.x; i < w * k * R; i += blockDim.x) {
            const int64_t cc = cfirst + i / ((int64_t)k * R);
            const int al = (int)((i / R) % k), r = (int)(i % R);
            const int64_t ch1 = 2 * cc + 1, ch2 = 2 * cc + 2;
            const double* x1 = sc + (local(ch1, lev + 1) * k) * R + r;
            const double* x2 = sc + (local(ch2, lev + 1) * k) * R + r;
            const double v = up_one(t, t.E + ch1 * t.dim * t.p * t.p, t.E + ch2 * t.dim * t.p * t.p, x1, x2, al, R);
            sc[(local(cc, lev) * k + al) * R + r] = v;
            xh[(((int64_t)f * t.ncl + cc) * k + al) * R + r] = v;
        }
        __syncthreads();
    }
}

// y[f][perm[row]][r] = (CSR row + near blocks) . x   (one 16-lane group per row; 16 rows per block)
FPDE_KERNEL void k_near_out(ApplyPlan a, int parts, int F, int R, const double* csr_val, const double* xt,
                            int dtype, void* y) {
    const int f = blockIdx.y;
    const int64_t nrb = (a.cap + 15) / 16;
    const int64_t li = blockIdx.x / nrb;
    const int rb = (int)(blockIdx.x % nrb);
    const int g = threadIdx.x & 15;
    const int64_t it = (int64_t)rb * 16 + (threadIdx.x >> 4);
    const int64_t lb = a.leaf_beg[li], nt = a.leaf_beg[li + 1] - lb;
    if (it >= nt) return;
    const int64_t row = lb + it;
    const double* xf = xt + (int64_t)f * a.N * R;
    const int64_t cap = a.cap;
    const int64_t e0 = a.near_ptr[li], e1 = a.near_ptr[li + 1];
    const int64_t c0 = 4 * g;
    for (int r = 0; r < R; ++r) {
        double acc = 0.0;
        if (csr_val) {
            const double* v = csr_val + (int64_t)f * a.nnz;
            for (int64_t e = a.csr_ptr[row] + g; e < a.csr_ptr[row + 1]; e += 16)
                acc += v[e] * xf[(int64_t)a.csr_col[e] * R + r];
        }
        if (parts & 4) {
            if (R == 1 && (cap & 3) == 0) {
                int64_t e = e0;
                // four blocks in flight per lane
                for (; e + 4 <= e1; e += 4) {
                    double2 b0[4], b1[4];
                    int64_t sb[4], ns[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t ls_ = a.near_src[e + u];
                        sb[u] = a.leaf_beg[ls_];
                        ns[u] = a.leaf_beg[ls_ + 1] - sb[u];
                        const double* blk = a.near_blk + (((int64_t)f * a.npairs + e + u) * cap + it) * cap + c0;
                        if (c0 < ns[u]) {
                            b0[u] = *(const double2*)(blk);
                            b1[u] = *(const double2*)(blk + 2);
                        } else {
                            b0[u] = make_double2(0.0, 0.0);
                            b1[u] = make_double2(0.0, 0.0);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const double* xs = xf + sb[u] + c0;
                        const int64_t m = ns[u] - c0;
                        if (m >= 4) acc += b0[u].x * xs[0] + b0[u].y * xs[1] + b1[u].x * xs[2] + b1[u].y * xs[3];
                        else if (m > 0) {
                            double v4[4] = {b0[u].x, b0[u].y, b1[u].x, b1[u].y};
                            for (int j = 0; j < m; ++j) acc += v4[j] * xs[j];
                        }
                    }
                }
                for (; e < e1; ++e) {
                    const int64_t ls_ = a.near_src[e];
                    const int64_t sb = a.leaf_beg[ls_], ns = a.leaf_beg[ls_ + 1] - sb;
                    const double* blk = a.near_blk + (((int64_t)f * a.npairs + e) * cap + it) * cap;
                    for (int64_t jc = c0; jc < c0 + 4 && jc < ns; ++jc) acc += blk[jc] * xf[sb + jc];
                }
                for (e = e0; e < e1 && cap > 64; ++e) {
                    const int64_t ls_ = a.near_src[e];
                    const int64_t sb = a.leaf_beg[ls_], ns = a.leaf_beg[ls_ + 1] - sb;
                    const double* blk = a.near_blk + (((int64_t)f * a.npairs + e) * cap + it) * cap;
                    for (int64_t jc = 64 + g; jc < ns; jc += 16) acc += blk[jc] * xf[sb + jc];
                }
            } else {
                for (int64_t e = e0; e < e1; ++e) {
                    const int64_t ls_ = a.near_src[e];
                    const int64_t sb = a.leaf_beg[ls_], ns = a.leaf_beg[ls_ + 1] - sb;
                    const double* blk = a.near_blk + (((int64_t)f * a.npairs + e) * cap + it) * cap;
                    for (int64_t jc = g; jc < ns; jc += 16) acc += blk[jc] * xf[(sb + jc) * R + r];
                }
            }
        }
        for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
        if (g == 0) {
            const int64_t dst = ((int64_t)f * a.N + a.perm[row]) * R + r;
            if (dtype == 0) ((double*)y)[dst] = acc;
            else ((float*)y)[dst] = (float)acc;
        }
    }
}

// y[f][perm[row]][r] += U[row] . (downsweep walk from the level-ls ancestor to the leaf)
FPDE_KERNEL void k_far_out(ApplyPlan a, H2Tree t, int ls, int F, int R, const double* yh, int dtype, void* y) {
    extern __shared__ double sy[];
    const int f = blockIdx.y;
    const int64_t nrb = (a.cap + 63) / 64;
    const int64_t li = blockIdx.x / nrb;
    const int rb = (int)(blockIdx.x % nrb);
    const int k = t.k, p = t.p;
    const int64_t leafc = t.first_leaf + li;
    const int64_t kR = (int64_t)k * R;
    double* cur = sy;
    double* nxt = sy + kR;
    const int64_t anc = ((leafc + 1) >> (t.L - ls)) - 1;
    for (int64_t i = threadIdx.x; i < kR; i += blockDim.x) cur[i] = yh[((int64_t)f * t.ncl + anc) * kR + i];
    __syncthreads();
    for (int lev = ls + 1; lev <= t.L; ++lev) {
        const int64_t cc = ((leafc + 1) >> (t.L - lev)) - 1;
        const double* Ec = t.E + cc * t.dim * p * p;
        for (int64_t i = threadIdx.x; i < kR; i += blockDim.x) {
            const int be = (int)(i / R), r = (int)(i % R);
            const int b0 = be % p, b1 = be / p;
            double acc = yh[((int64_t)f * t.ncl + cc) * kR + i];
            for (int al = 0; al < k; ++al) {
                double e = Ec[b0 * p + al % p];
                if (t.dim == 2) e *= Ec[p * p + b1 * p + al / p];
                acc += e * cur[(int64_t)al * R + r];
            }
            nxt[i] = acc;
        }
        __syncthreads();
        double* tmp = cur; cur = nxt; nxt = tmp;
    }
    // 4 lanes per (row, r) item; 64 items per block
    const int64_t lb = a.leaf_beg[li], nt = a.leaf_beg[li + 1] - lb;
    const int g = threadIdx.x & 3;
    {
        const int64_t item = (int64_t)rb * 64 + (threadIdx.x >> 2);
        const int64_t it = item / R;
        const int r = (int)(item % R);
        const bool ok = it < nt;
        double acc = 0.0;
        if (ok) {
            const double* u = a.U + (lb + it) * k;
            for (int al = g; al < k; al += 4) acc += u[al] * cur[(int64_t)al * R + r];
        }
        acc += __shfl_xor(acc, 1, 4);
        acc += __shfl_xor(acc, 2, 4);
        if (ok && g == 0) {
            const int64_t dst = ((int64_t)f * a.N + a.perm[lb + it]) * R + r;
            if (dtype == 0) ((double*)y)[dst] += acc;
            else ((float*)y)[dst] = (float)((double)((float*)y)[dst] + acc);
        }
    }
}

// Fork/join apply.  main: gather -> near_out ---------------------------\
//                    side:          up_sub -> up_top -> coupling -> down_top -> (join) far_out
// ev (optional, 6 events on the main stream when side == main): see fpde_host.cpp
hipError_t launch_apply_forkjoin(const ApplyPlan& a, const H2Tree& t, int ls, int parts, int F, int R,
                                 const double* csr_val, const double* St, int64_t nfar, int dtype, const void* x,
                                 double* xt, double* xh, double* yh, double* tmp, void* y, hipStream_t st,
                                 hipStream_t side, hipEvent_t fork, hipEvent_t join, hipEvent_t* ev) {
    const int k = t.k;
    const bool far = (parts & 8) != 0;
    if (ev) hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(k_gather, dim3(grid1((int64_t)F * a.N * R)), dim3(256), 0, st, a.N, a.perm, F, R, dtype, x,
                       xt);
    if (ev) hipEventRecord(ev[1], st);
    hipStream_t fs = st;
    if (far && side != st) {
        hipEventRecord(fork, st);
        hipStreamWaitEvent(side, fork, 0);
        fs = side;
    }
    if (far) {
        const int64_t nsub = int64_t(1) << ls;
        const int64_t rows = (int64_t(1) << (t.L - ls)) * a.cap;
        const int64_t ncl_sub = (int64_t(2) << (t.L - ls)) - 1;
        const size_t lds = sizeof(double) * (rows * k + rows * R + ncl_sub * k * R);
        hipLaunchKernelGGL(k_up_sub_xt, dim3((unsigned)nsub, F), dim3(256), lds, fs, a, t, ls, F, R, xt, xh);
        if (ls > 0) hipLaunchKernelGGL(k_up_top, dim3(F), dim3(1024), 0, fs, t, ls, F, R, xh);
        if (nfar > 0)
            hipLaunchKernelGGL(k_coupling_pairs, dim3(grid1((int64_t)F * nfar * k * R)), dim3(256), 0, fs, t, nfar, F,
                               R, St, xh, tmp);
        hipLaunchKernelGGL(k_coupling_reduce, dim3(grid1((int64_t)F * t.ncl * k * R)), dim3(256), 0, fs, t, nfar, F,
                           R, tmp, yh);
        if (ls > 0) hipLaunchKernelGGL(k_down_top, dim3(F), dim3(1024), 0, fs, t, ls, F, R, yh);
    }
    if (ev) hipEventRecord(ev[2], fs);
    const int64_t nrb = (a.cap + 15) / 16;
    hipLaunchKernelGGL(k_near_out, dim3((unsigned)(a.nleaf * nrb), F), dim3(256), 0, st, a, parts, F, R, csr_val, xt,
                       dtype, y);
    if (ev) hipEventRecord(ev[3], st);
    if (far) {
        if (fs != st) {
            hipEventRecord(join, fs);
            hipStreamWaitEvent(st, join, 0);
        }
        const int64_t nrb2 = (a.cap * R + 63) / 64;
        hipLaunchKernelGGL(k_far_out, dim3((unsigned)(a.nleaf * nrb2), F), dim3(256), sizeof(double) * 2 * k * R, st,
                           a, t, ls, F, R, yh, dtype, y);
    }
    if (ev) hipEventRecord(ev[4], st);
    return hipGetLastError();
}

}  // namespace fpde

// ============================================================ templated far-field kernels

namespace fpde {

template <int D, int P>
struct KR {
    static constexpr int K = D == 2 ? P * P : P;
    static constexpr int EP = D * P * P;   // transfer entries per cluster
};

// parent coefficient alpha from two children; E1, E2: [D][P][P] ([b][a]); x stride R
template <int D, int P>
__device__ __forceinline__ double up_t(const double* E1, const double* E2, const double* x1, const double* x2,
                                       int alpha, int R) {
    const int a0 = alpha % P, a1 = alpha / P;
    double acc = 0.0;
#pragma unroll
    for (int b1 = 0; b1 < (D == 2 ? P : 1); ++b1) {
        const double f1 = D == 2 ? E1[P * P + b1 * P + a1] : 1.0;
        const double f2 = D == 2 ? E2[P * P + b1 * P + a1] : 1.0;
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int b0 = 0; b0 < P; ++b0) {
            s1 += E1[b0 * P + a0] * x1[(int64_t)(b0 + P * b1) * R];
            s2 += E2[b0 * P + a0] * x2[(int64_t)(b0 + P * b1) * R];
        }
        acc += f1 * s1 + f2 * s2;
    }
    return acc;
}

// child coefficient beta += (E y_parent)[beta]
template <int D, int P>
__device__ __forceinline__ double down_t(const double* Ec, const double* yp, int beta, int R) {
    const int b0 = beta % P, b1 = beta / P;
    double acc = 0.0;
#pragma unroll
    for (int a1 = 0; a1 < (D == 2 ? P : 1); ++a1) {
        const double f = D == 2 ? Ec[P * P + b1 * P + a1] : 1.0;
        double s = 0.0;
#pragma unroll
        for (int a0 = 0; a0 < P; ++a0) s += Ec[b0 * P + a0] * yp[(int64_t)(a0 + P * a1) * R];
        acc += f * s;
    }
    return acc;
}

template <int D, int P>
FPDE_KERNEL void k_up_sub_t(ApplyPlan a, H2Tree t, int ls, int F, int R, const double* xt, double* xh) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    extern __shared__ double sm[];
    const int f = blockIdx.y;
    const int64_t c = ((int64_t(1) << ls) - 1) + blockIdx.x;
    const int64_t b = t.beg[c], n = t.end[c] - t.beg[c];
    const int depth = t.L - ls;
    const int64_t ncs = (int64_t(2) << depth) - 1;
    double* sU = sm;                   // [n][K]
    double* sx = sU + n * K;           // [n][R]
    double* sc = sx + n * R;           // [ncs][K][R]
    double* sE = sc + ncs * K * R;     // [ncs][EP]
    auto gid = [&](int64_t l) -> int64_t {   // subtree-local heap index -> global heap index
        int lev = 0;
        while (((int64_t(2) << lev) - 1) <= l) ++lev;
        const int64_t w = int64_t(1) << lev;
        return (c + 1) * w - 1 + (l - (w - 1));
    };
    for (int64_t i = threadIdx.x; i < n * R; i += blockDim.x) sx[i] = xt[((int64_t)f * a.N + b) * R + i];
    for (int64_t i = threadIdx.x; i < n * K; i += blockDim.x) sU[i] = a.U[b * K + i];
    for (int64_t i = threadIdx.x; i < ncs * EP; i += blockDim.x) sE[i] = t.E[gid(i / EP) * EP + i % EP];
    __syncthreads();
    const int64_t nl = int64_t(1) << depth;
    const int64_t l0 = ((c + 1) << depth) - 1;
    const int64_t loc0 = nl - 1;   // local index of the first leaf
    for (int64_t i = threadIdx.x; i < nl * K * R; i += blockDim.x) {
        const int64_t li = i / ((int64_t)K * R);
        const int al = (int)((i / R) % K), r = (int)(i % R);
        const int64_t cc = l0 + li;
        double acc = 0.0;
        const int64_t j1 = t.end[cc] - b;
        for (int64_t j = t.beg[cc] - b; j < j1; ++j) acc += sU[j * K + al] * sx[j * R + r];
        sc[((loc0 + li) * K + al) * R + r] = acc;
        xh[(((int64_t)f * t.ncl + cc) * K + al) * R + r] = acc;
    }
    __syncthreads();
    for (int lev = t.L - 1; lev >= ls; --lev) {
        const int64_t w = int64_t(1) << (lev - ls);
        const int64_t lfirst = w - 1;               // local index of the first cluster of this level
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

// levels lt-1 .. 0 from level lt, all in LDS; one block per field
template <int D, int P>
__global__ __launch_bounds__(1024) void k_up_top_t(H2Tree t, int lt, int F, int R, double* xh) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    extern __shared__ double sm[];
    const int f = blockIdx.x;
    const int64_t ntop = (int64_t(2) << lt) - 1;
    double* sx = sm;                       // [ntop][K][R] heap indexed
    double* sE = sx + ntop * K * R;        // [2^lt][EP] transfers of one level's children
    const int64_t KRr = (int64_t)K * R;
    for (int64_t i = threadIdx.x + ((int64_t(1) << lt) - 1) * KRr; i < ntop * KRr; i += blockDim.x)
        sx[i] = xh[(int64_t)f * t.ncl * KRr + i];
    for (int lev = lt - 1; lev >= 0; --lev) {
        const int64_t ch0 = (int64_t(2) << lev) - 1, nch = int64_t(2) << lev;
        for (int64_t i = threadIdx.x; i < nch * EP; i += blockDim.x) sE[i] = t.E[ch0 * EP + i];
        __syncthreads();
        const int64_t c0 = (int64_t(1) << lev) - 1, w = int64_t(1) << lev;
        for (int64_t i = threadIdx.x; i < w * KRr; i += blockDim.x) {
            const int64_t cc = c0 + i / KRr;
            const int al = (int)((i / R) % K), r = (int)(i % R);
            const int64_t ch1 = 2 * cc + 1, ch2 = 2 * cc + 2;
            const double v = up_t<D, P>(sE + (ch1 - ch0) * EP, sE + (ch2 - ch0) * EP, sx + ch1 * KRr + r,
                                        sx + ch2 * KRr + r, al, R);
            sx[cc * KRr + (int64_t)al * R + r] = v;
            xh[((int64_t)f * t.ncl + cc) * KRr + (int64_t)al * R + r] = v;
        }
        __syncthreads();
    }
}

// levels 1..lt: yh(c) += E_c yh(parent), all in LDS; one block per field
template <int D, int P>
__global__ __launch_bounds__(1024) void k_down_top_t(H2Tree t, int lt, int F, int R, double* yh) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    extern __shared__ double sm[];
    const int f = blockIdx.x;
    const int64_t ntop = (int64_t(2) << lt) - 1;
    const int64_t KRr = (int64_t)K * R;
    double* sy = sm;
    double* sE = sy + ntop * KRr;
    for (int64_t i = threadIdx.x; i < ntop * KRr; i += blockDim.x) sy[i] = yh[(int64_t)f * t.ncl * KRr + i];
    for (int lev = 1; lev <= lt; ++lev) {
        const int64_t c0 = (int64_t(1) << lev) - 1, w = int64_t(1) << lev;
        for (int64_t i = threadIdx.x; i < w * EP; i += blockDim.x) sE[i] = t.E[c0 * EP + i];
        __syncthreads();
        for (int64_t i = threadIdx.x; i < w * KRr; i += blockDim.x) {
            const int64_t cc = c0 + i / KRr;
            const int be = (int)((i / R) % K), r = (int)(i % R);
            const int64_t par = (cc - 1) / 2;
            const double v = sy[cc * KRr + (int64_t)be * R + r] +
                             down_t<D, P>(sE + (cc - c0) * EP, sy + par * KRr + r, be, R);
            sy[cc * KRr + (int64_t)be * R + r] = v;
            yh[((int64_t)f * t.ncl + cc) * KRr + (int64_t)be * R + r] = v;
        }
        __syncthreads();
    }
}

template <int D, int P>
FPDE_KERNEL void k_coupling_pairs_t(H2Tree t, int64_t nfar, int F, int R, const double* St, const double* xh,
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

template <int D, int P>
FPDE_KERNEL void k_far_out_t(ApplyPlan a, H2Tree t, int ls, int F, int R, const double* yh, int dtype, void* y) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    extern __shared__ double sy[];
    const int f = blockIdx.y;
    const int64_t nrb = (a.cap * R + 63) / 64;
    const int64_t li = blockIdx.x / nrb;
    const int rb = (int)(blockIdx.x % nrb);
    const int64_t leafc = t.first_leaf + li;
    const int64_t KRr = (int64_t)K * R;
    double* cur = sy;
    double* nxt = sy + KRr;
    double* sE = sy + 2 * KRr;
    const int64_t anc = ((leafc + 1) >> (t.L - ls)) - 1;
    for (int64_t i = threadIdx.x; i < KRr; i += blockDim.x) cur[i] = yh[((int64_t)f * t.ncl + anc) * KRr + i];
    for (int lev = ls + 1; lev <= t.L; ++lev) {
        const int64_t cc = ((leafc + 1) >> (t.L - lev)) - 1;
        for (int i = threadIdx.x; i < EP; i += blockDim.x) sE[i] = t.E[cc * EP + i];
        __syncthreads();
        for (int64_t i = threadIdx.x; i < KRr; i += blockDim.x) {
            const int be = (int)(i / R), r = (int)(i % R);
            nxt[i] = yh[((int64_t)f * t.ncl + cc) * KRr + i] + down_t<D, P>(sE, cur + r, be, R);
        }
        __syncthreads();
        double* tmp = cur; cur = nxt; nxt = tmp;
    }
    __syncthreads();
    const int64_t lb = a.leaf_beg[li], nt = a.leaf_beg[li + 1] - lb;
    const int g = threadIdx.x & 3;
    const int64_t item = (int64_t)rb * 64 + (threadIdx.x >> 2);
    const int64_t it = item / R;
    const int r = (int)(item % R);
    const bool ok = it < nt;
    double acc = 0.0;
    if (ok) {
        const double* u = a.U + (lb + it) * K;
#pragma unroll
        for (int al = 0; al < K; al += 4)
            if (al + g < K) acc += u[al + g] * cur[(int64_t)(al + g) * R + r];
    }
    acc += __shfl_xor(acc, 1, 4);
    acc += __shfl_xor(acc, 2, 4);
    if (ok && g == 0) {
        const int64_t dst = ((int64_t)f * a.N + a.perm[lb + it]) * R + r;
        if (dtype == 0) ((double*)y)[dst] += acc;
        else ((float*)y)[dst] = (float)((double)((float*)y)[dst] + acc);
    }
}

template <int D, int P>
static hipError_t far_chain_t(const ApplyPlan& a, const H2Tree& t, const FarLaunch& fl, int F, int R,
                              const double* St, int64_t nfar, double* xt, double* xh, double* yh, double* tmp,
                              hipStream_t fs) {
    constexpr int K = KR<D, P>::K;
    const int64_t nsub = int64_t(1) << fl.ls;
    hipLaunchKernelGGL((k_up_sub_t<D, P>), dim3((unsigned)nsub, F), dim3(256), fl.lds_sub, fs, a, t, fl.ls, F, R, xt,
                       xh);
    for (int lev = fl.ls - 1; lev >= fl.lt; --lev) {
        hipError_t e = launch_up_level(t, lev, F, R, xh, fs);
        if (e != hipSuccess) return e;
    }
    if (fl.lt > 0) hipLaunchKernelGGL((k_up_top_t<D, P>), dim3(F), dim3(1024), fl.lds_top, fs, t, fl.lt, F, R, xh);
    if (nfar > 0)
        hipLaunchKernelGGL((k_coupling_pairs_t<D, P>), dim3(grid1((int64_t)F * nfar * K * R)), dim3(256), 0, fs, t,
                           nfar, F, R, St, xh, tmp);
    hipLaunchKernelGGL(k_coupling_reduce, dim3(grid1((int64_t)F * t.ncl * K * R)), dim3(256), 0, fs, t, nfar, F, R,
                       tmp, yh);
    if (fl.lt > 0) hipLaunchKernelGGL((k_down_top_t<D, P>), dim3(F), dim3(1024), fl.lds_down, fs, t, fl.lt, F, R, yh);
    for (int lev = fl.lt; lev < fl.ls; ++lev) {
        hipError_t e = launch_down_level(t, lev, F, R, yh, fs);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

template <int D, int P>
static void far_out_t(const ApplyPlan& a, const H2Tree& t, const FarLaunch& fl, int F, int R, const double* yh,
                      int dtype, void* y, hipStream_t st) {
    const int64_t nrb = (a.cap * R + 63) / 64;
    hipLaunchKernelGGL((k_far_out_t<D, P>), dim3((unsigned)(a.nleaf * nrb), F), dim3(256), fl.lds_out, st, a, t,
                       fl.ls, F, R, yh, dtype, y);
}

#define FPDE_DISPATCH_DP(dim, p, FN, ...)                                   \
    do {                                                                    \
        if (dim == 1) {                                                     \
            switch (p) {                                                    \
                case 1: FN<1, 1>(__VA_ARGS__); break;                       \
                case 2: FN<1, 2>(__VA_ARGS__); break;                       \
                case 3: FN<1, 3>(__VA_ARGS__); break;                       \
                case 4: FN<1, 4>(__VA_ARGS__); break;                       \
                case 5: FN<1, 5>(__VA_ARGS__); break;                       \
                case 6: FN<1, 6>(__VA_ARGS__); break;                       \
                case 7: FN<1, 7>(__VA_ARGS__); break;                       \
                default: FN<1, 8>(__VA_ARGS__); break;                      \
            }                                                               \
        } else {                                                            \
            switch (p) {                                                    \
                case 1: FN<2, 1>(__VA_ARGS__); break;                       \
                case 2: FN<2, 2>(__VA_ARGS__); break;                       \
                case 3: FN<2, 3>(__VA_ARGS__); break;                       \
                case 4: FN<2, 4>(__VA_ARGS__); break;                       \
                case 5: FN<2, 5>(__VA_ARGS__); break;                       \
                case 6: FN<2, 6>(__VA_ARGS__); break;                       \
                case 7: FN<2, 7>(__VA_ARGS__); break;                       \
                default: FN<2, 8>(__VA_ARGS__); break;                      \
            }                                                               \
        }                                                                   \
    } while (0)

// LDS plan of the far chain for R right-hand sides; returns false if the subtree does not fit
bool far_launch_plan(const H2Tree& t, int64_t cap, int ls, int R, FarLaunch* fl) {
    const int64_t K = t.k, EP = (int64_t)t.dim * t.p * t.p;
    const int depth = t.L - ls;
    const int64_t rows = (int64_t(1) << depth) * cap, ncs = (int64_t(2) << depth) - 1;
    fl->ls = ls;
    fl->lds_sub = sizeof(double) * (rows * K + rows * R + ncs * K * R + ncs * EP);
    fl->lds_out = sizeof(double) * (2 * K * R + EP);
    if (fl->lds_sub > 64 * 1024 || fl->lds_out > 64 * 1024) return false;
    int lt = ls;
    while (lt > 0) {
        const int64_t ntop = (int64_t(2) << lt) - 1;
        const size_t up = sizeof(double) * (ntop * K * R + (int64_t(2) << lt) * EP);
        if (up <= 64 * 1024) break;
        --lt;
    }
    fl->lt = lt;
    const int64_t ntop = (int64_t(2) << lt) - 1;
    fl->lds_top = sizeof(double) * (ntop * K * R + (int64_t(2) << lt) * EP);
    fl->lds_down = sizeof(double) * (ntop * K * R + (int64_t(1) << lt) * EP);
    return true;
}

hipError_t launch_apply_forkjoin_t(const ApplyPlan& a, const H2Tree& t, const FarLaunch& fl, int parts, int F, int R,
                                   const double* csr_val, const double* St, int64_t nfar, int dtype, const void* x,
                                   double* xt, double* xh, double* yh, double* tmp, void* y, hipStream_t st,
                                   hipStream_t side, hipEvent_t fork, hipEvent_t join, hipEvent_t* ev) {
    const bool far = (parts & 8) != 0;
    if (ev) hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(k_gather, dim3(grid1((int64_t)F * a.N * R)), dim3(256), 0, st, a.N, a.perm, F, R, dtype, x,
                       xt);
    if (ev) hipEventRecord(ev[1], st);
    hipStream_t fs = st;
    if (far && side != st) {
        hipEventRecord(fork, st);
        hipStreamWaitEvent(side, fork, 0);
        fs = side;
    }
    if (far) FPDE_DISPATCH_DP(t.dim, t.p, far_chain_t, a, t, fl, F, R, St, nfar, xt, xh, yh, tmp, fs);
    if (ev) hipEventRecord(ev[2], fs);
    const int64_t nrb = (a.cap + 15) / 16;
    hipLaunchKernelGGL(k_near_out, dim3((unsigned)(a.nleaf * nrb), F), dim3(256), 0, st, a, parts, F, R, csr_val, xt,
                       dtype, y);
    if (ev) hipEventRecord(ev[3], st);
    if (far) {
        if (fs != st) {
            hipEventRecord(join, fs);
            hipStreamWaitEvent(st, join, 0);
        }
        FPDE_DISPATCH_DP(t.dim, t.p, far_out_t, a, t, fl, F, R, yh, dtype, y, st);
    }
    if (ev) hipEventRecord(ev[4], st);
    return hipGetLastError();
}

}  // namespace fpde

// ============================================================ apply v2: no gather, short far chain

namespace fpde {

__device__ __forceinline__ double ldx(const void* x, int64_t i, int dtype) {
    return dtype == 0 ? ((const double*)x)[i] : (double)((const float*)x)[i];
}

// Subtree upsweep reading the caller's x through the permutation.  One block per
// (subtree root at level ls, field); each wave owns leaves, lane = row, partial
// products reduced with cross-lane sums; levels below ls in LDS.
template <int D, int P>
FPDE_KERNEL void k_up_sub_v2(ApplyPlan a, H2Tree t, int ls, int F, int R, int dtype, const void* x, double* xh) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    constexpr int CH = K < 16 ? K : 16;               // coefficients accumulated per pass
    extern __shared__ double sm[];
    const int f = blockIdx.y;
    const int64_t c = ((int64_t(1) << ls) - 1) + blockIdx.x;
    const int depth = t.L - ls;
    const int64_t ncs = (int64_t(2) << depth) - 1;
    double* sc = sm;                   // [ncs][K][R]
    double* sE = sc + ncs * K * R;     // [ncs][EP]
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
            for (int a0 = 0; a0 < K; a0 += CH) {
                double acc[CH];
#pragma unroll
                for (int q = 0; q < CH; ++q) acc[q] = 0.0;
                for (int64_t j = rb + lane; j < re; j += 64) {
                    const double xv = ldx(x, ((int64_t)f * a.N + a.perm[j]) * R + r, dtype);
                    const double* u = a.U + j * K + a0;
#pragma unroll
                    for (int q = 0; q < CH; ++q)
                        if (a0 + q < K) acc[q] += u[q] * xv;
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

// levels ls-1 .. 0 with every transfer of levels 1..ls resident in LDS; one block per field
template <int D, int P>
__global__ __launch_bounds__(1024) void k_up_top_v2(H2Tree t, int ls, int F, int R, double* xh) {
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

// yh[f][c] = sum_{e in far(c)} S_e xh[f][src(e)]: one block per (target cluster, field);
// 64 alpha lanes x 4 pair groups, transposed S rows are coalesced across alpha.
template <int D, int P>
FPDE_KERNEL void k_coupling_v2(H2Tree t, int F, int R, const double* St, const double* xh, double* yh) {
    constexpr int K = KR<D, P>::K;
    __shared__ double red[4][64];
    const int64_t c = blockIdx.x;
    const int f = blockIdx.y;
    const int al = threadIdx.x & 63, pg = threadIdx.x >> 6;
    const int64_t e0 = t.far_ptr[c], e1 = t.far_ptr[c + 1];
    const int64_t nfar = t.far_ptr[t.ncl];
    for (int r = 0; r < R; ++r) {
        double acc = 0.0;
        if (al < K) {
            for (int64_t e = e0 + pg; e < e1; e += 4) {
                const double* S = St + ((int64_t)f * nfar + e) * K * K + al;
                const double* xs = xh + (((int64_t)f * t.ncl + t.far_src[e]) * K) * R + r;
#pragma unroll
                for (int b = 0; b < K; ++b) acc += S[b * K] * xs[(int64_t)b * R];
            }
        }
        red[pg][al] = acc;
        __syncthreads();
        if (threadIdx.x < K) {
            const double v = (red[0][al] + red[1][al]) + (red[2][al] + red[3][al]);
            yh[(((int64_t)f * t.ncl + c) * K + al) * R + r] = v;
        }
        __syncthreads();
    }
}

// y[perm[row]] += U[row] . yh_total(leaf): each block walks the downsweep from the root
// to its leaf (ancestor coefficients and transfers prefetched into LDS in one pass).
template <int D, int P>
FPDE_KERNEL void k_far_out_v2(ApplyPlan a, H2Tree t, int F, int R, const double* yh, int dtype, void* y) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    extern __shared__ double sm[];
    const int f = blockIdx.y;
    const int64_t nrb = (a.cap * R + 63) / 64;
    const int64_t li = blockIdx.x / nrb;
    const int rb = (int)(blockIdx.x % nrb);
    const int64_t leafc = t.first_leaf + li;
    const int64_t KRr = (int64_t)K * R;
    const int L = t.L;
    double* sy = sm;                          // [L+1][K][R] coefficients of the ancestors (level order)
    double* sE = sy + (int64_t)(L + 1) * KRr; // [L+1][EP]
    for (int64_t i = threadIdx.x; i < (int64_t)(L + 1) * KRr; i += blockDim.x) {
        const int lev = (int)(i / KRr);
        const int64_t cc = ((leafc + 1) >> (L - lev)) - 1;
        sy[i] = yh[((int64_t)f * t.ncl + cc) * KRr + i % KRr];
    }
    for (int64_t i = threadIdx.x; i < (int64_t)(L + 1) * EP; i += blockDim.x) {
        const int lev = (int)(i / EP);
        const int64_t cc = ((leafc + 1) >> (L - lev)) - 1;
        sE[i] = lev == 0 ? 0.0 : t.E[cc * EP + i % EP];
    }
    __syncthreads();
    for (int lev = 1; lev <= L; ++lev) {
        for (int64_t i = threadIdx.x; i < KRr; i += blockDim.x) {
            const int be = (int)(i / R), r = (int)(i % R);
            sy[lev * KRr + i] += down_t<D, P>(sE + lev * EP, sy + (lev - 1) * KRr + r, be, R);
        }
        __syncthreads();
    }
    const double* cur = sy + L * KRr;
    const int64_t lb = a.leaf_beg[li], nt = a.leaf_beg[li + 1] - lb;
    const int g = threadIdx.x & 3;
    const int64_t item = (int64_t)rb * 64 + (threadIdx.x >> 2);
    const int64_t it = item / R;
    const int r = (int)(item % R);
    const bool ok = it < nt;
    double acc = 0.0;
    if (ok) {
        const double* u = a.U + (lb + it) * K;
#pragma unroll
        for (int al = 0; al < K; al += 4)
            if (al + g < K) acc += u[al + g] * cur[(int64_t)(al + g) * R + r];
    }
    acc += __shfl_xor(acc, 1, 4);
    acc += __shfl_xor(acc, 2, 4);
    if (ok && g == 0) {
        const int64_t dst = ((int64_t)f * a.N + a.perm[lb + it]) * R + r;
        if (dtype == 0) ((double*)y)[dst] += acc;
        else ((float*)y)[dst] = (float)((double)((float*)y)[dst] + acc);
    }
}

// Near field + CSR reading the caller's x: CSR columns are dof indices (csr_col_dof),
// near-block columns map through perm.  One 16-lane group per row, 16 rows per block.
FPDE_KERNEL void k_near_out_v2(ApplyPlan a, const int32_t* csr_col_dof, int parts, int F, int R,
                               const double* csr_val, int dtype, const void* x, void* y) {
    const int f = blockIdx.y;
    const int64_t nrb = (a.cap + 15) / 16;
    const int64_t li = blockIdx.x / nrb;
    const int rb = (int)(blockIdx.x % nrb);
    const int g = threadIdx.x & 15;
    const int64_t it = (int64_t)rb * 16 + (threadIdx.x >> 4);
    const int64_t lb = a.leaf_beg[li], nt = a.leaf_beg[li + 1] - lb;
    if (it >= nt) return;
    const int64_t row = lb + it;
    const int64_t xo = (int64_t)f * a.N * R;
    const int64_t cap = a.cap;
    const int64_t e0 = a.near_ptr[li], e1 = a.near_ptr[li + 1];
    const int64_t c0 = 4 * g;
    for (int r = 0; r < R; ++r) {
        double acc = 0.0;
        if (csr_val) {
            const double* v = csr_val + (int64_t)f * a.nnz;
            for (int64_t e = a.csr_ptr[row] + g; e < a.csr_ptr[row + 1]; e += 16)
                acc += v[e] * ldx(x, xo + (int64_t)csr_col_dof[e] * R + r, dtype);
        }
        if (parts & 4) {
            if ((cap & 3) == 0) {
                int64_t e = e0;
                for (; e + 4 <= e1; e += 4) {
                    double2 b0[4], b1[4];
                    int64_t sb[4], ns[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t ls_ = a.near_src[e + u];
                        sb[u] = a.leaf_beg[ls_];
                        ns[u] = a.leaf_beg[ls_ + 1] - sb[u];
                        const double* blk = a.near_blk + (((int64_t)f * a.npairs + e + u) * cap + it) * cap + c0;
                        if (c0 < ns[u]) {
                            b0[u] = *(const double2*)(blk);
                            b1[u] = *(const double2*)(blk + 2);
                        } else {
                            b0[u] = make_double2(0.0, 0.0);
                            b1[u] = make_double2(0.0, 0.0);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t m = ns[u] - c0;
                        const double v4[4] = {b0[u].x, b0[u].y, b1[u].x, b1[u].y};
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (j < m) acc += v4[j] * ldx(x, xo + a.perm[sb[u] + c0 + j] * R + r, dtype);
                    }
                }
                for (; e < e1; ++e) {
                    const int64_t ls_ = a.near_src[e];
                    const int64_t sb = a.leaf_beg[ls_], ns = a.leaf_beg[ls_ + 1] - sb;
                    const double* blk = a.near_blk + (((int64_t)f * a.npairs + e) * cap + it) * cap;
                    for (int64_t jc = c0; jc < c0 + 4 && jc < ns; ++jc)
                        acc += blk[jc] * ldx(x, xo + a.perm[sb + jc] * R + r, dtype);
                }
                for (e = e0; e < e1 && cap > 64; ++e) {
                    const int64_t ls_ = a.near_src[e];
                    const int64_t sb = a.leaf_beg[ls_], ns = a.leaf_beg[ls_ + 1] - sb;
                    const double* blk = a.near_blk + (((int64_t)f * a.npairs + e) * cap + it) * cap;
                    for (int64_t jc = 64 + g; jc < ns; jc += 16) acc += blk[jc] * ldx(x, xo + a.perm[sb + jc] * R + r, dtype);
                }
            } else {
                for (int64_t e = e0; e < e1; ++e) {
                    const int64_t ls_ = a.near_src[e];
                    const int64_t sb = a.leaf_beg[ls_], ns = a.leaf_beg[ls_ + 1] - sb;
                    const double* blk = a.near_blk + (((int64_t)f * a.npairs + e) * cap + it) * cap;
                    for (int64_t jc = g; jc < ns; jc += 16) acc += blk[jc] * ldx(x, xo + a.perm[sb + jc] * R + r, dtype);
                }
            }
        }
        for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
        if (g == 0) {
            const int64_t dst = ((int64_t)f * a.N + a.perm[row]) * R + r;
            if (dtype == 0) ((double*)y)[dst] = acc;
            else ((float*)y)[dst] = (float)acc;
        }
    }
}

template <int D, int P>
static void far_v2_t(const ApplyPlan& a, const H2Tree& t, int ls, int F, int R, const double* St, int dtype,
                     const void* x, double* xh, double* yh, hipStream_t fs, hipEvent_t ev_mid) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    const int depth = t.L - ls;
    const int64_t ncs = (int64_t(2) << depth) - 1;
    const size_t lds_sub = sizeof(double) * (ncs * K * R + ncs * EP);
    hipLaunchKernelGGL((k_up_sub_v2<D, P>), dim3((unsigned)(int64_t(1) << ls), F), dim3(256), lds_sub, fs, a, t, ls, F,
                       R, dtype, x, xh);
    if (ls > 0) {
        const int64_t ntop = (int64_t(2) << ls) - 1;
        const size_t lds_top = sizeof(double) * (ntop * K * R + ntop * EP);
        hipLaunchKernelGGL((k_up_top_v2<D, P>), dim3(F), dim3(1024), lds_top, fs, t, ls, F, R, xh);
    }
    hipLaunchKernelGGL((k_coupling_v2<D, P>), dim3((unsigned)t.ncl, F), dim3(256), 0, fs, t, F, R, St, xh, yh);
    if (ev_mid) hipEventRecord(ev_mid, fs);
}

template <int D, int P>
static void far_out_v2_t(const ApplyPlan& a, const H2Tree& t, int F, int R, const double* yh, int dtype, void* y,
                         hipStream_t st) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    const int64_t nrb = (a.cap * R + 63) / 64;
    const size_t lds = sizeof(double) * ((int64_t)(t.L + 1) * K * R + (int64_t)(t.L + 1) * EP);
    hipLaunchKernelGGL((k_far_out_v2<D, P>), dim3((unsigned)(a.nleaf * nrb), F), dim3(256), lds, st, a, t, F, R, yh,
                       dtype, y);
}

// LDS needed by the v2 far chain; false when the per-level path must be used
bool far_v2_fits(const H2Tree& t, int ls, int R) {
    const int64_t K = t.k, EP = (int64_t)t.dim * t.p * t.p;
    const int64_t ncs = (int64_t(2) << (t.L - ls)) - 1, ntop = (int64_t(2) << ls) - 1;
    const int64_t lim = 64 * 1024 / 8;
    return ncs * K * R + ncs * EP <= lim && ntop * K * R + ntop * EP <= lim &&
           (int64_t)(t.L + 1) * (K * R + EP) <= lim && K <= 64;
}

// Apply: main stream near-field + CSR (reads x directly); side stream far chain;
// join; far output.  ev (optional, 5 events, side == st): start, (unused) , after far
// chain, after near output, after far output.
hipError_t launch_apply_v2(const ApplyPlan& a, const H2Tree& t, int ls, const int32_t* csr_col_dof, int parts, int F,
                           int R, const double* csr_val, const double* St, int dtype, const void* x, double* xh,
                           double* yh, void* y, hipStream_t st, hipStream_t side, hipEvent_t fork, hipEvent_t join,
                           hipEvent_t* ev) {
    const bool far = (parts & 8) != 0;
    if (ev) {
        hipEventRecord(ev[0], st);
        hipEventRecord(ev[1], st);
    }
    hipStream_t fs = st;
    if (far && side != st) {
        hipEventRecord(fork, st);
        hipStreamWaitEvent(side, fork, 0);
        fs = side;
    }
    if (far) FPDE_DISPATCH_DP(t.dim, t.p, far_v2_t, a, t, ls, F, R, St, dtype, x, xh, yh, fs, (hipEvent_t) nullptr);
    if (ev) hipEventRecord(ev[2], fs);
    const int64_t nrb = (a.cap + 15) / 16;
    hipLaunchKernelGGL(k_near_out_v2, dim3((unsigned)(a.nleaf * nrb), F), dim3(256), 0, st, a, csr_col_dof, parts, F, R,
                       csr_val, dtype, x, y);
    if (ev) hipEventRecord(ev[3], st);
    if (far) {
        if (fs != st) {
            hipEventRecord(join, fs);
            hipStreamWaitEvent(st, join, 0);
        }
        FPDE_DISPATCH_DP(t.dim, t.p, far_out_v2_t, a, t, F, R, yh, dtype, y, st);
    }
    if (ev) hipEventRecord(ev[4], st);
    return hipGetLastError();
}

}  // namespace fpde

// ============================================================ apply v3 kernels

namespace fpde {

// One wave per leaf (up to 8 leaves per 512-thread block); x read once per row.
template <int D, int P>
__global__ __launch_bounds__(512) void k_up_sub_v3(ApplyPlan a, H2Tree t, int ls, int F, int R, int dtype,
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
FPDE_KERNEL void k_far_out_v3(ApplyPlan a, H2Tree t, int F, int R, const double* tmp, int dtype, void* y) {
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
static void far_v3_t(const ApplyPlan& a, const H2Tree& t, int ls, int F, int R, const double* St, int64_t nfar,
                     int dtype, const void* x, double* xh, double* tmp, hipStream_t fs) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    const int depth = t.L - ls;
    const int64_t ncs = (int64_t(2) << depth) - 1;
    const int64_t nl = int64_t(1) << depth;
    const int threads = 64 * (int)(nl < 8 ? nl : 8);
    const size_t lds_sub = sizeof(double) * (ncs * K * R + ncs * EP);
    hipLaunchKernelGGL((k_up_sub_v3<D, P>), dim3((unsigned)(int64_t(1) << ls), F), dim3(threads), lds_sub, fs, a, t,
                       ls, F, R, dtype, x, xh);
    if (ls > 0) {
        const int64_t ntop = (int64_t(2) << ls) - 1;
        const size_t lds_top = sizeof(double) * (ntop * K * R + ntop * EP);
        hipLaunchKernelGGL((k_up_top_v2<D, P>), dim3(F), dim3(1024), lds_top, fs, t, ls, F, R, xh);
    }
    if (nfar > 0)
        hipLaunchKernelGGL((k_coupling_pairs_t<D, P>), dim3(grid1((int64_t)F * nfar * K * R)), dim3(256), 0, fs, t,
                           nfar, F, R, St, xh, tmp);
}

template <int D, int P>
static void far_out_v3_t(const ApplyPlan& a, const H2Tree& t, int F, int R, const double* tmp, int dtype, void* y,
                         hipStream_t st) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    const int64_t nrb = (a.cap * R + 63) / 64;
    const size_t lds = sizeof(double) * ((int64_t)(t.L + 1) * K * R + (int64_t)(t.L + 1) * EP);
    hipLaunchKernelGGL((k_far_out_v3<D, P>), dim3((unsigned)(a.nleaf * nrb), F), dim3(256), lds, st, a, t, F, R, tmp,
                       dtype, y);
}

hipError_t launch_apply_v3(const ApplyPlan& a, const H2Tree& t, int ls, const int32_t* csr_col_dof, int parts, int F,
                           int R, const double* csr_val, const double* St, int64_t nfar, int dtype, const void* x,
                           double* xh, double* tmp, void* y, hipStream_t st, hipStream_t side, hipEvent_t fork,
                           hipEvent_t join, hipEvent_t* ev) {
    const bool far = (parts & 8) != 0;
    if (ev) hipEventRecord(ev[0], st);
    hipStream_t fs = st;
    if (far && side != st) {
        hipEventRecord(fork, st);
        hipStreamWaitEvent(side, fork, 0);
        fs = side;
    }
    if (far) FPDE_DISPATCH_DP(t.dim, t.p, far_v3_t, a, t, ls, F, R, St, nfar, dtype, x, xh, tmp, fs);
    if (ev) hipEventRecord(ev[1], fs);
    const int64_t nrb = (a.cap + 15) / 16;
    if (ev)   // start/stop timestamps of exactly this kernel
        hipExtLaunchKernelGGL(k_near_out_v2, dim3((unsigned)(a.nleaf * nrb), F), dim3(256), 0, st, ev[2], ev[3], 0, a,
                              csr_col_dof, parts, F, R, csr_val, dtype, x, y);
    else
        hipLaunchKernelGGL(k_near_out_v2, dim3((unsigned)(a.nleaf * nrb), F), dim3(256), 0, st, a, csr_col_dof, parts,
                           F, R, csr_val, dtype, x, y);
    if (far) {
        if (fs != st) {
            hipEventRecord(join, fs);
            hipStreamWaitEvent(st, join, 0);
        }
        FPDE_DISPATCH_DP(t.dim, t.p, far_out_v3_t, a, t, F, R, tmp, dtype, y, st);
    }
    if (ev) hipEventRecord(ev[4], st);
    return hipGetLastError();
}

}  // namespace fpde

// ============================================================ near field as packed leaf panels
// (k_pack_panels, k_near_panel: fpde_near.hip)

namespace fpde {

// Apply with panels (one right-hand side): main stream gather + panel near field,
// side stream far chain (x read in place), join, far output.
hipError_t launch_apply_v4(const ApplyPlan& a, const H2Tree& t, int ls, const int64_t* poff, const int64_t* pstride,
                           const int32_t* pcols, const int64_t* pcols_ptr, int64_t max_stride, const double* panel,
                           int parts, int F, const double* csr_val, const double* St, int64_t nfar, int dtype,
                           const void* x, double* xt, double* xh, double* tmp, void* y, hipStream_t st,
                           hipStream_t side, hipEvent_t fork, hipEvent_t join, hipEvent_t* ev) {
    const int R = 1;
    const bool far = (parts & 8) != 0;
    if (ev) hipEventRecord(ev[0], st);
    hipStream_t fs = st;
    if (far && side != st) {
        hipEventRecord(fork, st);
        hipStreamWaitEvent(side, fork, 0);
        fs = side;
    }
    if (far) FPDE_DISPATCH_DP(t.dim, t.p, far_v3_t, a, t, ls, F, R, St, nfar, dtype, x, xh, tmp, fs);
    if (ev) hipEventRecord(ev[1], fs);
    hipLaunchKernelGGL(k_gather, dim3(grid1((int64_t)F * a.N)), dim3(256), 0, st, a.N, a.perm, F, R, dtype, x, xt);
    hipError_t e = launch_near_panel(a, poff, pstride, pcols, pcols_ptr, max_stride, panel, (parts & 4) != 0, csr_val, F,
                                     xt, dtype, y, st, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
    if (e != hipSuccess) return e;
    if (far) {
        if (fs != st) {
            hipEventRecord(join, fs);
            hipStreamWaitEvent(st, join, 0);
        }
        FPDE_DISPATCH_DP(t.dim, t.p, far_out_v3_t, a, t, F, R, tmp, dtype, y, st);
    }
    if (ev) hipEventRecord(ev[4], st);
    return hipGetLastError();
}

}  // namespace fpde

// ============================================================ apply v5: one-kernel upsweep

namespace fpde {

// Upsweep of the whole tree in one launch.  Block b owns the subtree rooted at
// cluster (2^ls - 1 + b): leaf coefficients (one lane per coefficient, the
// leaf's x rows staged in LDS), then the subtree levels in LDS.  Each block
// publishes its results with a device-scope release fence and takes a ticket;
// the block holding the last ticket (acquire fence) computes levels ls-1..0 and
// resets the ticket counter.  No block ever waits for another.
template <int D, int P>
__global__ __launch_bounds__(512) void k_up_all(ApplyPlan a, H2Tree t, int ls, int F, int dtype, const void* x,
                                                double* xh, unsigned int* tickets) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    extern __shared__ double sm[];
    __shared__ unsigned int s_ticket;
    const int f = blockIdx.y;
    const int64_t c = ((int64_t(1) << ls) - 1) + blockIdx.x;
    const int depth = t.L - ls;
    const int64_t ncs = (int64_t(2) << depth) - 1;
    double* sc = sm;                          // [ncs][K]
    double* sE = sc + ncs * K;                // [ncs][EP]
    double* sx = sE + ncs * EP;               // [waves][a.cap] x rows of the leaf being processed
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
    double* sxw = sx + (int64_t)wv * a.cap;
    for (int64_t li = wv; li < nl; li += nw) {
        const int64_t cc = l0 + li;
        const int64_t rb = t.beg[cc], n = t.end[cc] - rb;
        for (int64_t j = lane; j < n; j += 64) sxw[j] = ldx(x, (int64_t)f * a.N + a.perm[rb + j], dtype);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // lanes (half, alpha): with K <= 32 the two half-waves split the rows
        const int half = K <= 32 ? (lane >> 5) : 0;
        const int al = K <= 32 ? (lane & 31) : lane;
        const int64_t jb = K <= 32 ? (half ? (n + 1) / 2 : 0) : 0;
        const int64_t je = K <= 32 ? (half ? n : (n + 1) / 2) : n;
        double v = 0.0;
        if (al < K) {
            const double* u = a.U + rb * K + al;
            double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
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
            xh[((int64_t)f * t.ncl + cc) * K + lane] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    __syncthreads();
    for (int lev = t.L - 1; lev >= ls; --lev) {
        const int64_t w = int64_t(1) << (lev - ls);
        const int64_t lfirst = w - 1;
        for (int64_t i = threadIdx.x; i < w * K; i += blockDim.x) {
            const int64_t lc = lfirst + i / K;
            const int al = (int)(i % K);
            const int64_t l1 = 2 * lc + 1, l2 = 2 * lc + 2;
            const double v = up_t<D, P>(sE + l1 * EP, sE + l2 * EP, sc + l1 * K, sc + l2 * K, al, 1);
            sc[lc * K + al] = v;
            xh[((int64_t)f * t.ncl + gid(lc)) * K + al] = v;
        }
        __syncthreads();
    }
    if (ls == 0) return;
    // publish, take a ticket
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_ticket = atomicAdd(&tickets[f], 1u);
    __syncthreads();
    if (s_ticket != (unsigned int)((int64_t(1) << ls) - 1)) return;
    __threadfence();
    if (threadIdx.x == 0) atomicExch(&tickets[f], 0u);
    // top levels ls-1..0 from every block's level-ls coefficients (LDS reused)
    const int64_t ntop = (int64_t(2) << ls) - 1;
    double* tx = sm;                     // [ntop][K]
    double* tE = tx + ntop * K;          // [ntop][EP]
    __syncthreads();
    for (int64_t i = threadIdx.x + ((int64_t(1) << ls) - 1) * K; i < ntop * K; i += blockDim.x)
        tx[i] = __builtin_nontemporal_load(&xh[(int64_t)f * t.ncl * K + i]);
    for (int64_t i = threadIdx.x + EP; i < ntop * EP; i += blockDim.x) tE[i] = t.E[i];
    __syncthreads();
    for (int lev = ls - 1; lev >= 0; --lev) {
        const int64_t c0 = (int64_t(1) << lev) - 1, w = int64_t(1) << lev;
        for (int64_t i = threadIdx.x; i < w * K; i += blockDim.x) {
            const int64_t cc = c0 + i / K;
            const int al = (int)(i % K);
            const int64_t ch1 = 2 * cc + 1, ch2 = 2 * cc + 2;
            const double v = up_t<D, P>(tE + ch1 * EP, tE + ch2 * EP, tx + ch1 * K, tx + ch2 * K, al, 1);
            tx[cc * K + al] = v;
            xh[((int64_t)f * t.ncl + cc) * K + al] = v;
        }
        __syncthreads();
    }
}

template <int D, int P>
static void up_all_t(const ApplyPlan& a, const H2Tree& t, int ls, int F, int dtype, const void* x, double* xh,
                     unsigned int* tickets, hipStream_t fs) {
    constexpr int K = KR<D, P>::K, EP = KR<D, P>::EP;
    const int64_t ncs = (int64_t(2) << (t.L - ls)) - 1, ntop = (int64_t(2) << ls) - 1;
    const int64_t nl = int64_t(1) << (t.L - ls);
    const int waves = (int)(nl < 8 ? nl : 8);
    const int64_t sub = ncs * (K + EP) + waves * a.cap, top = ntop * (K + EP);
    const size_t lds = sizeof(double) * (sub > top ? sub : top);
    hipLaunchKernelGGL((k_up_all<D, P>), dim3((unsigned)(int64_t(1) << ls), F), dim3(64 * waves), lds, fs, a, t, ls, F,
                       dtype, x, xh, tickets);
}

template <int D, int P>
static void pairs_t(const H2Tree& t, int64_t nfar, int F, const double* St, const double* xh, double* tmp,
                    hipStream_t fs) {
    constexpr int K = KR<D, P>::K;
    if (nfar > 0)
        hipLaunchKernelGGL((k_coupling_pairs_t<D, P>), dim3(grid1((int64_t)F * nfar * K)), dim3(256), 0, fs, t, nfar, F,
                           1, St, xh, tmp);
}

// LDS budget of k_up_all
bool up_all_fits(const H2Tree& t, int64_t cap, int ls) {
    const int64_t K = t.k, EP = (int64_t)t.dim * t.p * t.p;
    const int64_t ncs = (int64_t(2) << (t.L - ls)) - 1, ntop = (int64_t(2) << ls) - 1;
    const int64_t sub = ncs * (K + EP) + 8 * cap, top = ntop * (K + EP);
    return (sub > top ? sub : top) * 8 <= 64 * 1024 && K <= 64;
}

hipError_t launch_apply_v5(const ApplyPlan& a, const H2Tree& t, int ls, const int64_t* poff, const int64_t* pstride,
                           const int32_t* pcols, const int64_t* pcols_ptr, int64_t max_stride, const double* panel,
                           int parts, int F, const double* csr_val, const double* St, int64_t nfar, int dtype,
                           const void* x, double* xt, double* xh, double* tmp, unsigned int* tickets, void* y,
                           hipStream_t st, hipStream_t side, hipEvent_t fork, hipEvent_t join, hipEvent_t* ev) {
    const bool far = (parts & 8) != 0;
    if (ev) hipEventRecord(ev[0], st);
    hipStream_t fs = st;
    if (far && side != st) {
        hipEventRecord(fork, st);
        hipStreamWaitEvent(side, fork, 0);
        fs = side;
    }
    if (far) {
        FPDE_DISPATCH_DP(t.dim, t.p, up_all_t, a, t, ls, F, dtype, x, xh, tickets, fs);
        FPDE_DISPATCH_DP(t.dim, t.p, pairs_t, t, nfar, F, St, xh, tmp, fs);
    }
    if (ev) hipEventRecord(ev[1], fs);
    hipLaunchKernelGGL(k_gather, dim3(grid1((int64_t)F * a.N)), dim3(256), 0, st, a.N, a.perm, F, 1, dtype, x, xt);
    hipError_t e = launch_near_panel(a, poff, pstride, pcols, pcols_ptr, max_stride, panel, (parts & 4) != 0, csr_val, F,
                                     xt, dtype, y, st, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
    if (e != hipSuccess) return e;
    if (far) {
        if (fs != st) {
            hipEventRecord(join, fs);
            hipStreamWaitEvent(st, join, 0);
        }
        FPDE_DISPATCH_DP(t.dim, t.p, far_out_v3_t, a, t, F, 1, tmp, dtype, y, st);
    }
    if (ev) hipEventRecord(ev[4], st);
    return hipGetLastError();
}

}  // namespace fpde
