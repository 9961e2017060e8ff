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

#include "fpde_device.h"

namespace fpde {




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

// ------------------------------------------------------------ adjoint of the singular pairs
//
// d/ds_j and d/dkappa_j of sum_r w_r^T L u_r for one touching pair, L its local
// matrix.  The substituted integrand is gamma(x, y) Phi Phi^T times factors
// that do not depend on s (the substitutions of Sec. 4 only rewrite the power
// |x - y|^{-(2 + s(x) + s(y))}), so with s(x) = sum_a lambda_a(x^) s_a:
//   d/ds_a  (x side) = integrand * (-ln|x - y|) * lambda_a(x^)   (y side alike),
//   d/dkappa_a       = integrand * lambda_a(x^) / (2 kappa(x)).
// |x - y| = xi |J0 a - J1 b| (vertex, edge), xi eta1 eta2 |J0 dhat| (identical).
// out[f][pair][12]: slots 0..5 d/ds at cell0 v0..v2, cell1 v0..v2 (canonical
// order), slots 6..11 the same for kappa; multiplied by the pair weight.
struct AdjVecs {
    const double* w;   // [F][N][R]
    const double* u;
    int64_t N;
    int R;
};

FPDE_KERNEL void k_adj_singular2d(SingArgs A, AdjVecs V, int f) {
    const int lane = threadIdx.x & 63;
    const int64_t pid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pid >= A.np) return;
    const int32_t* P = A.pairs + pid * 8;
    const int kind = P[0];
    const double* s = A.s + (int64_t)f * A.M;
    const double* kp = A.kap + (int64_t)f * A.M;
    double X0[3][2], X1[3][2], s0[3], s1[3], k0[3], k1[3];
    const int vv0[3] = {P[1], P[2], P[3]};
    const int vv1[3] = {P[4], P[5], P[6]};
    for (int a = 0; a < 3; ++a) {
        X0[a][0] = A.X[vv0[a]]; X0[a][1] = A.X[A.M + vv0[a]];
        X1[a][0] = A.X[vv1[a]]; X1[a][1] = A.X[A.M + vv1[a]];
        s0[a] = s[vv0[a]]; s1[a] = s[vv1[a]];
        k0[a] = kp[vv0[a]]; k1[a] = kp[vv1[a]];
    }
    // local dofs of the case (same order as the forward kernel's Phi) and
    // C[a][b] = sum_r w_r[a] u_r[b] over them
    const int nd = kind == 0 ? 3 : (kind == 1 ? 4 : 5);
    int loc[5] = {P[1], P[2], P[3], kind == 1 ? P[6] : P[5], P[6]};
    double C[5][5];
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) {
            double v = 0.0;
            if (a < nd && b < nd && loc[a] < V.N && loc[b] < V.N)
                for (int r = 0; r < V.R; ++r)
                    v += V.w[((int64_t)f * V.N + loc[a]) * V.R + r] * V.u[((int64_t)f * V.N + loc[b]) * V.R + r];
            C[a][b] = v;
        }
    const double J0[2][2] = {{X0[1][0] - X0[0][0], X0[2][0] - X0[1][0]}, {X0[1][1] - X0[0][1], X0[2][1] - X0[1][1]}};
    const double J1[2][2] = {{X1[1][0] - X1[0][0], X1[2][0] - X1[1][0]}, {X1[1][1] - X1[0][1], X1[2][1] - X1[1][1]}};
    const double det0 = fabs(J0[0][0] * J0[1][1] - J0[0][1] * J0[1][0]);
    const double det1 = fabs(J1[0][0] * J1[1][1] - J1[0][1] * J1[1][0]);
    const int nreg = kind == 0 ? 3 : (kind == 1 ? 5 : 2);
    const int nq = A.nq;
    const int n4 = nq * nq * nq * nq;
    const double sb = A.s_bar;
    const double inv4 = 1.0 / (4.0 - 2.0 * sb);
    const double inv2 = 1.0 / (2.0 - 2.0 * sb);
    double acc[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) acc[e] = 0.0;
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
        double phi[5] = {0, 0, 0, 0, 0};
        double xa0, xa1, yb0, yb1, r2, fac, sx, sy, kx, ky, lnr;
        if (kind == 0) {
            const double e2 = exp(inv2 * log(t2));
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
            lnr = inv4 * lz + log(e1) + inv2 * log(t2) + 0.5 * log(r2);
        } else {
            const double xi = exp(inv4 * lz);
            Reg2 g = kind == 1 ? edge_region(r, e1, t2, e3) : vertex_region(r, e1, t2, e3);
            xa0 = xi * g.a0; xa1 = xi * g.a1; yb0 = xi * g.b0; yb1 = xi * g.b1;
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
            lnr = inv4 * lz + 0.5 * log(r2);
        }
        double qf = 0.0;
        for (int a = 0; a < 5; ++a) {
            double ca = 0.0;
            for (int b = 0; b < 5; ++b) ca += C[a][b] * phi[b];
            qf += phi[a] * ca;
        }
        const double val = wt * A.a_scale * sqrt(kx * ky) * fac * rpow(r2, 2.0 + sx + sy) * qf;
        const double vs = -lnr * val;
        const double lx[3] = {1.0 - xa0, xa0 - xa1, xa1};
        const double ly[3] = {1.0 - yb0, yb0 - yb1, yb1};
        const double hx = 0.5 * val / kx, hy = 0.5 * val / ky;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc[a] += vs * lx[a];
            acc[3 + a] += vs * ly[a];
            acc[6 + a] += hx * lx[a];
            acc[9 + a] += hy * ly[a];
        }
    }
    double pre = kind == 0 ? det0 * det0 / ((2.0 - sb) * (2.0 - 2.0 * sb)) : det0 * det1 * inv4;
    if (kind != 0) pre *= 2.0;   // both orderings of a distinct touching pair
    double* o = A.out + ((int64_t)f * A.np + pid) * 12;
    for (int e = 0; e < 12; ++e) {
        const double v = wave_sum(acc[e]);
        if (lane == 0) o[e] = v * pre;
    }
}

FPDE_KERNEL void k_adj_singular1d(SingArgs A, AdjVecs V, int f) {
    const int lane = threadIdx.x & 63;
    const int64_t pid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pid >= A.np) return;
    const int32_t* P = A.pairs + pid * 8;
    const int kind = P[0];
    const double* s = A.s + (int64_t)f * A.M;
    const double* kp = A.kap + (int64_t)f * A.M;
    const int nq = A.nq;
    const double sb = A.s_bar;
    auto val_of = [&](const double* x, int node, int r) -> double {
        return node < V.N ? x[((int64_t)f * V.N + node) * V.R + r] : 0.0;
    };
    double acc[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) acc[e] = 0.0;
    double pre;
    if (kind == 0) {
        const int v0 = P[1], v1 = P[2];
        double cq = 0.0;   // sum_r (w1 - w0)(u1 - u0): the local matrix is sigma sigma^T
        for (int r = 0; r < V.R; ++r)
            cq += (val_of(V.w, v1, r) - val_of(V.w, v0, r)) * (val_of(V.u, v1, r) - val_of(V.u, v0, r));
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
            const double val = cq * wt * A.a_scale * sqrt(kx * ky) * exp((1.0 - ss) * log(aJ)) *
                               exp((2.0 * sb - ss) * inv * log(z)) * (1.0 - t);
            const double vs = -(inv * log(z) + log(aJ)) * val;   // |x - y| = t |J|
            acc[0] += vs * (1.0 - xh); acc[1] += vs * xh;
            acc[3] += vs * (1.0 - yh); acc[4] += vs * yh;
            acc[6] += 0.5 * val / kx * (1.0 - xh); acc[7] += 0.5 * val / kx * xh;
            acc[9] += 0.5 * val / ky * (1.0 - yh); acc[10] += 0.5 * val / ky * yh;
        }
        pre = 2.0 * inv;
    } else {
        // vertex pair: cell0 = (P, A), cell1 = (P, B); local dofs (P, A, B)
        const int vp = P[1], va = P[2], vb = P[5];
        double C[3][3];
        const int loc[3] = {vp, va, vb};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double v = 0.0;
                for (int r = 0; r < V.R; ++r) v += val_of(V.w, loc[a], r) * val_of(V.u, loc[b], r);
                C[a][b] = v;
            }
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
            const double phi[3] = {bt - at, at, -bt};
            double qf = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) qf += phi[a] * C[a][b] * phi[b];
            const double val = qf * wt * A.a_scale * sqrt(kx * ky) * exp((2.0 * sb - (sx + sy)) * inv * log(z)) *
                               exp(-(1.0 + sx + sy) * log(D));
            const double vs = -(inv * log(z) + log(D)) * val;   // |x - y| = xi D
            acc[0] += vs * (1.0 - al); acc[1] += vs * al;
            acc[3] += vs * (1.0 - be); acc[4] += vs * be;
            acc[6] += 0.5 * val / kx * (1.0 - al); acc[7] += 0.5 * val / kx * al;
            acc[9] += 0.5 * val / ky * (1.0 - be); acc[10] += 0.5 * val / ky * be;
        }
        pre = 2.0 * h1 * h2 * inv;
    }
    double* o = A.out + ((int64_t)f * A.np + pid) * 12;
    for (int e = 0; e < 12; ++e) {
        const double v = wave_sum(acc[e]);
        if (lane == 0) o[e] = v * pre;
    }
}

hipError_t launch_adj_singular(int dim, int64_t np, const int32_t* pairs, const double* coords, int64_t n_nodes,
                               int F, const double* s, const double* kappa, double a_scale, double s_bar, int nq,
                               const double* g01, const double* w01, const double* w, const double* u, int64_t N,
                               int R, double* out, hipStream_t st) {
    if (np == 0) return hipSuccess;
    SingArgs A{np, pairs, coords, n_nodes, s, kappa, a_scale, s_bar, nq, g01, w01, out};
    AdjVecs V{w, u, N, R};
    for (int f = 0; f < F; ++f) {
        if (dim == 2)
            hipLaunchKernelGGL(k_adj_singular2d, dim3(grid1(np, 4)), dim3(256), 0, st, A, V, f);
        else
            hipLaunchKernelGGL(k_adj_singular1d, dim3(grid1(np, 4)), dim3(256), 0, st, A, V, f);
    }
    return hipGetLastError();
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

// P1 values of s and sqrt(kappa) at the Chebyshev nodes of the clusters: the stencil
// entries summed in order, each product rounded on its own (no contraction)
FPDE_KERNEL void k_node_fields(int64_t nn, int64_t M, const int64_t* st_node, const double* st_w,
                               const double* s, const double* kappa, double* ns, double* nk, int f) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    const double* sf = s + (int64_t)f * M;
    const double* kf = kappa + (int64_t)f * M;
    double sv = 0.0, kv = 0.0;
    for (int a = 0; a < 3; ++a) {
        const int64_t v = st_node[i * 3 + a];
        if (v < 0) continue;
        const double w = st_w[i * 3 + a];
        const double ps = sf[v] * w, pk = kf[v] * w;
        sv = a == 0 ? ps : sv + ps;
        kv = a == 0 ? pk : kv + pk;
    }
    ns[(int64_t)f * nn + i] = sv;
    nk[(int64_t)f * nn + i] = sqrt(kv);
}

hipError_t launch_node_fields(int64_t nn, int F, int64_t M, const int64_t* st_node, const double* st_w,
                              const double* s, const double* kappa, double* ns, double* nk, hipStream_t st) {
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(k_node_fields, dim3(grid1(nn)), dim3(256), 0, st, nn, M, st_node, st_w, s, kappa, ns, nk,
                           f);
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
    const hipError_t ef = hipFreeAsync(leaf_of, st);
    return e != hipSuccess ? e : ef;
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
    const hipError_t ef = hipFreeAsync(leaf_of, st);
    return e != hipSuccess ? e : ef;
}

// ============================================================ near leaf blocks of K~

// Block per (computed near pair, chunk of JC source columns).
// Phase A: R[lc][a][jj] = sum_{tau' in S_j, tau' not touching tau_lc} sum_q sum_q'
//                         w w' gamma(q,q') lam_a(q) psi_j(q')
// Phase B: blk[it][j] = -2 sum_{(lc,slot) around row node} R[lc][slot][jj], stored
//          also as entry [j][it] of the mirrored pair's block when there is one
//          (gamma is symmetric and so is the touching test, so both blocks hold the
//          same integrals)
constexpr int kJC = 8;

// NQE > 0: the NQE points of the target cell stay in registers and each source point
// is loaded once per cell pair; the sums over the target points close the item.
// NQE = 0: any rule size, the points reloaded in the inner loops.
template <int NQE>
FPDE_KERNEL void k_near_blocks(H2Tree t, NearPlan P, const int64_t* perm, const int32_t* cells, int nqe,
                               int64_t nc, const double* qx, const double* qw, const double* qs,
                               const double* qk, const double* lam, int64_t nq, int f, double a_scale,
                               double* nb) {
    extern __shared__ double R[];
    const int64_t nchunk = (P.cap + kJC - 1) / kJC;
    const int64_t pr = P.own[blockIdx.x / nchunk], pm = P.mirror[blockIdx.x / nchunk];
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
            if constexpr (NQE > 0) {
                double tx0[NQE], tx1[NQE], te[NQE], g[NQE];
#pragma unroll
                for (int l = 0; l < NQE; ++l) {
                    const int64_t q = cell * NQE + l;
                    tx0[l] = qx[q];
                    tx1[l] = t.dim == 2 ? qx[nq + q] : 0.0;
                    te[l] = (double)t.dim + qsf[q];
                    g[l] = 0.0;
                }
                for (int64_t e = P.nc_ptr[jn]; e < P.nc_ptr[jn + 1]; ++e) {
                    const int64_t c2 = P.nc_cell[e];
                    const int slot = P.nc_slot[e];
                    bool touch = false;
                    for (int a = 0; a < nv; ++a)
                        for (int b = 0; b < nv; ++b) touch |= (tv[a] == cells[b * nc + c2]);
                    if (touch) continue;
                    for (int l2 = 0; l2 < NQE; ++l2) {
                        const int64_t q2 = c2 * NQE + l2;
                        const double y0 = qx[q2], y1 = t.dim == 2 ? qx[nq + q2] : 0.0;
                        const double w2 = qw[q2] * lam[slot * NQE + l2] * qkf[q2], s2 = qsf[q2];
#pragma unroll
                        for (int l = 0; l < NQE; ++l) {
                            const double d0 = tx0[l] - y0, d1 = tx1[l] - y1;
                            g[l] += w2 * rpow(d0 * d0 + d1 * d1, te[l] + s2);
                        }
                    }
                }
#pragma unroll
                for (int l = 0; l < NQE; ++l) {
                    const int64_t q = cell * NQE + l;
                    const double gl = g[l] * (qw[q] * qkf[q]);
                    for (int a = 0; a < nv; ++a) acc[a] += gl * lam[a * NQE + l];
                }
            } else {
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
        }
        for (int a = 0; a < nv; ++a) R[(lc * 3 + a) * kJC + jj] = acc[a];
    }
    __syncthreads();
    // phase B
    const int64_t tb = t.beg[ct], nt = t.end[ct] - t.beg[ct];
    double* out = nb + (((int64_t)f * P.npairs + pr) * P.cap) * P.cap;
    double* outm = nb + (((int64_t)f * P.npairs + pm) * P.cap) * P.cap;
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
        if (pm != pr) outm[(j0 + jj) * P.cap + it] = v;
    }
}

hipError_t launch_near_blocks_lds(const H2Tree& t, const NearPlan& np, int64_t max_patch,
                                  const int64_t* perm, const int32_t* cells, int nqe, int64_t nc,
                                  const double* qx, const double* qw, const double* qs,
                                  const double* qk, const double* lam, int64_t nq_all, int F,
                                  double a_scale, double* nb, hipStream_t st) {
    if (np.npairs == 0 || np.nown == 0) return hipSuccess;
    const size_t lds = (size_t)max_patch * 3 * kJC * sizeof(double);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const int64_t nchunk = (np.cap + kJC - 1) / kJC;
    auto kern = nqe == 9 ? k_near_blocks<9> : nqe == 3 ? k_near_blocks<3> : k_near_blocks<0>;
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(kern, dim3((unsigned)(np.nown * nchunk)), dim3(256), lds, st, t, np, perm, cells, nqe, nc,
                           qx, qw, qs, qk, lam, nq_all, f, a_scale, nb);
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
                            const double* xt, const double* yh, int dtype, void* y, int accumulate) {
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
        if (dtype == 0) ((double*)y)[dst] = accumulate ? ((double*)y)[dst] + acc : acc;
        else ((float*)y)[dst] = (float)(accumulate ? (double)((float*)y)[dst] + acc : acc);
    }
}

hipError_t launch_leaf_out(const ApplyPlan& a, const H2Tree& t, int parts, int F, int R,
                           const double* csr_val_override, const double* xt, const double* yh,
                           int dtype, void* y, hipStream_t st, int accumulate) {
    const int64_t items = (int64_t)F * a.N * R;
    hipLaunchKernelGGL(k_leaf_out, dim3(grid1(items, 16)), dim3(256), 0, st, a, t, parts, F, R,
                       csr_val_override, xt, yh, dtype, y, accumulate);
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

// Coupling matrices of far pairs whose source is moved down the tree (nested
// bases, Sec. 5.3).  x^(s) = sum over the descendants r of s at a deeper
// level of M_r^T x^(r), M_r = E_r E_parent(r) ... (the child-to-parent
// transfers from r up to the child of s; per dimension, Kronecker), so
// S x^(s) = sum_r (S M_r^T) x^(r).  Entry j of the new list takes pair orig[j]
// with source r = src1[j], dd = depth[j] levels below the original source:
//   St1[f][j][delta][alpha] = sum_beta S[alpha][beta] M_r[delta][beta]
// (transposed like St; M_r = I for dd = 0).
FPDE_KERNEL void k_expand_coupling(H2Tree t, int64_t n1, const int64_t* orig, const int64_t* src1,
                                   const int32_t* depth, int F, int64_t nfar, const double* St, double* St1) {
    const int k = t.k, p = t.p, dim = t.dim;
    const int64_t kk = (int64_t)k * k;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)F * n1 * kk) return;
    const int f = (int)(i / (n1 * kk));
    int64_t rem = i - (int64_t)f * n1 * kk;
    const int64_t j = rem / kk;
    rem %= kk;
    const int delta = (int)(rem / k), alpha = (int)(rem % k);
    const int64_t e = orig[j];
    const double* S = St + ((int64_t)f * nfar + e) * kk;   // S[beta * k + alpha] = S_e[alpha][beta]
    const int dd = depth[j];
    if (dd == 0) {
        St1[i] = S[(int64_t)delta * k + alpha];
        return;
    }
    // row delta_d of the per-dimension chain E_r E_parent(r) ... (dd factors)
    double v[2][8];
    int64_t c = src1[j];
    for (int d = 0; d < dim; ++d) {
        const int dl = d == 0 ? delta % p : delta / p;
        for (int a = 0; a < p; ++a) v[d][a] = t.E[(c * dim + d) * p * p + dl * p + a];
    }
    for (int s = 1; s < dd; ++s) {
        c = (c - 1) / 2;
        for (int d = 0; d < dim; ++d) {
            double w[8];
            for (int a2 = 0; a2 < p; ++a2) {
                double acc = 0.0;
                for (int a = 0; a < p; ++a) acc += v[d][a] * t.E[(c * dim + d) * p * p + a * p + a2];
                w[a2] = acc;
            }
            for (int a2 = 0; a2 < p; ++a2) v[d][a2] = w[a2];
        }
    }
    double acc = 0.0;
    for (int beta = 0; beta < k; ++beta) {
        const double m = dim == 2 ? v[0][beta % p] * v[1][beta / p] : v[0][beta];
        acc += S[(int64_t)beta * k + alpha] * m;
    }
    St1[i] = acc;
}

hipError_t launch_expand_coupling(const H2Tree& t, int64_t n1, const int64_t* orig, const int64_t* src1,
                                  const int32_t* depth, int F, int64_t nfar, const double* St, double* St1,
                                  hipStream_t st) {
    const int64_t n = (int64_t)F * n1 * t.k * t.k;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand_coupling, dim3(grid1(n)), dim3(256), 0, st, t, n1, orig, src1, depth, F, nfar, St,
                       St1);
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

}  // namespace fpde
