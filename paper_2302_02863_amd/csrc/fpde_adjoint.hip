// Adjoint of the stiffness operator: the gradient of
//   J(s, kappa) = sum_r w_r^T A_h(s, kappa) u_r
// with respect to the nodal order s_j and diffusivity kappa_j of every mesh
// node (both fields are P1, Sec. 2).  Every dependence of A_h = B + K~ + M~ on
// them goes through the kernel gamma = a_scale sqrt(kappa(x) kappa(y))
// |x - y|^{-(d + s(x) + s(y))} at quadrature or Chebyshev points, so
//   d gamma / d s_j     = gamma (-ln|x - y|) (phi_j(x) + phi_j(y)),
//   d gamma / d kappa_j = gamma (phi_j(x) / (2 kappa(x)) + phi_j(y) / (2 kappa(y))),
// phi_j the P1 weight of node j at the point (the nearest-node indicator at a
// Chebyshev point outside the mesh).  The near and far relations of both
// trees are symmetric, so each pair sum is rewritten target-major:
//   sum_{x,y} c(x, y) (phi_j(x) + phi_j(y)) = sum_x phi_j(x) sum_y (c(x, y) + c(y, x)),
// which needs no scatter across blocks: every output has one writer and the
// gradient is bitwise reproducible.
//
// Parts (the singular pairs are in fpde_kernels.hip next to their forward rules):
//   K~ near blocks      k_adj_knear      per interior cell, per quadrature point
//   density, near       k_adj_rho_near   per point of a density leaf
//   density, exterior   k_adj_rho_ext    per interior point (eq. e:rho)
//   points -> nodes     k_adj_points     sum_q phi_j(q) D(q)
//   far blocks          k_adj_far        per Chebyshev node of a cluster (both trees)
//   nodes of clusters   k_adj_gather     through the P1 stencils of the Chebyshev nodes
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fpde_device.h"

namespace fpde {

namespace {

constexpr int kMaxQE = 16;   // quadrature points per cell handled by k_adj_knear

// c(q) = 2 omega_q sum_r W_r(q) U_r(q) at interior points (0 elsewhere): the weight
// with which the density at q enters w^T M~ u = 2 sum_q omega_q W(q) U(q) rho(q)
// (eq. e:m), W, U the P1 interpolants of the dof vectors w, u.
FPDE_KERNEL void k_adj_c(int dim, int64_t nc, int nqe, const int32_t* cells, const uint8_t* cell_int,
                         const double* lam, const double* qw, const double* w, const double* u, int64_t N, int R,
                         int f, int64_t nq, double* c) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nc * nqe) return;
    const int64_t cell = q / nqe;
    const int l = (int)(q - cell * nqe);
    double v = 0.0;
    if (cell_int[cell]) {
        for (int r = 0; r < R; ++r) {
            double W = 0.0, U = 0.0;
            for (int a = 0; a <= dim; ++a) {
                const int64_t node = cells[a * nc + cell];
                if (node < N) {
                    W += lam[a * nqe + l] * w[((int64_t)f * N + node) * R + r];
                    U += lam[a * nqe + l] * u[((int64_t)f * N + node) * R + r];
                }
            }
            v += W * U;
        }
        v *= 2.0 * qw[q];
    }
    c[(int64_t)f * nq + q] = v;
}

}  // namespace

// ------------------------------------------------------------------ K~ near blocks
//
// w^T K~_near u = -2 sum_{(S, S') near} sum_{tau in P(S), tau' in P(S'), disjoint}
//                 sum_{q, q'} omega omega' gamma(q, q') W_S(q) U_S'(q'),
// P(S) the cells touching the dofs of leaf S, W_S the interpolant of w
// restricted to the dofs of S (eq. e:k-near).  Target-major with the symmetric
// near relation: for q in an interior cell tau,
//   D(q) = sum_{S: tau in P(S)} sum_{S' near S} sum_{q'} -2 omega omega' gamma
//          [W_S(q) U_S'(q') + U_S(q) W_S'(q')] x {-ln r | 1 / (2 kappa(q))}.
// One block per interior cell, one right-hand side r per launch; the threads
// take the (source leaf, patch cell) items of a target leaf in turn, so every
// lane has work however small each patch is.  NQE > 0 fixes the rule size at
// compile time (the accumulators then take NQE registers, not kMaxQE).

template <int NQE>
FPDE_KERNEL void k_adj_knear(AdjKnear P, int f, double* Ds, double* Dk) {
    constexpr int NL = NQE > 0 ? NQE : kMaxQE;
    __shared__ double tx[kMaxQE], ty[kMaxQE], ts[kMaxQE], tk[kMaxQE], tw[kMaxQE], tW[kMaxQE], tU[kMaxQE];
    __shared__ double red[256];
    const int64_t ci = blockIdx.x;
    const int64_t cell = P.icells[ci];
    const int nqe = NQE > 0 ? NQE : P.nqe, nv = P.dim + 1;
    const int tid = threadIdx.x;
    const double* qs = P.qs + (int64_t)f * P.nq;
    const double* qk = P.qk + (int64_t)f * P.nq;
    int tv[3] = {-1, -1, -1}, tl[3] = {-1, -1, -1};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (a < nv) {
            tv[a] = P.cells[a * P.nc + cell];
            tl[a] = P.leaf_of_node[tv[a]];
        }
    if (tid < nqe) {
        const int64_t q = cell * nqe + tid;
        tx[tid] = P.qx[q];
        ty[tid] = P.dim == 2 ? P.qx[P.nq + q] : 0.0;
        ts[tid] = qs[q];
        tk[tid] = qk[q];
        tw[tid] = P.qw[q];
    }
    double accS[NL], accK[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) accS[l] = accK[l] = 0.0;
    const double dd = (double)P.dim;
    for (int64_t e0 = P.cell_leaf_ptr[ci]; e0 < P.cell_leaf_ptr[ci + 1]; ++e0) {
        const int S = P.cell_leaf[e0];
        __syncthreads();
        if (tid < nqe) {   // W_S, U_S at the target points
            double W = 0.0, U = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (a < nv && tl[a] == S) {
                    const double la = P.lam[a * nqe + tid];
                    W += la * P.w[((int64_t)f * P.N + tv[a]) * P.R + P.r];
                    U += la * P.u[((int64_t)f * P.N + tv[a]) * P.R + P.r];
                }
            tW[tid] = W;
            tU[tid] = U;
        }
        __syncthreads();
        int64_t base = 0;   // items of the earlier source leaves
        for (int64_t e = P.near_ptr[S]; e < P.near_ptr[S + 1]; ++e) {
            const int64_t S2 = P.near_src[e];
            const int64_t pb = P.patch_ptr[S2], pn = P.patch_ptr[S2 + 1] - pb;
            const int64_t k0 = ((tid - base) % blockDim.x + blockDim.x) % blockDim.x;   // (base + k0) % nt == tid
            base += pn;
            for (int64_t k = k0; k < pn; k += blockDim.x) {
                const int64_t c2 = P.patch_cell[pb + k];
                int sv[3] = {-2, -2, -2}, sl[3] = {-1, -1, -1};
                bool touch = false;
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    if (b < nv) {
                        sv[b] = P.cells[b * P.nc + c2];
                        sl[b] = P.leaf_of_node[sv[b]];
#pragma unroll
                        for (int a = 0; a < 3; ++a) touch |= (a < nv && tv[a] == sv[b]);
                    }
                if (touch) continue;
                double wv[3] = {0, 0, 0}, uv[3] = {0, 0, 0};
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    if (b < nv && sl[b] == (int)S2) {
                        wv[b] = P.w[((int64_t)f * P.N + sv[b]) * P.R + P.r];
                        uv[b] = P.u[((int64_t)f * P.N + sv[b]) * P.R + P.r];
                    }
                for (int l2 = 0; l2 < nqe; ++l2) {
                    const int64_t q2 = c2 * nqe + l2;
                    double W2 = 0.0, U2 = 0.0;
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        if (b < nv) {
                            W2 += P.lam[b * nqe + l2] * wv[b];
                            U2 += P.lam[b * nqe + l2] * uv[b];
                        }
                    const double x2 = P.qx[q2], y2 = P.dim == 2 ? P.qx[P.nq + q2] : 0.0;
                    const double s2 = qs[q2], k2 = qk[q2], w2 = P.qw[q2];
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        if (NQE == 0 && l >= nqe) break;
                        const double d0 = tx[l] - x2, d1 = ty[l] - y2;
                        const double r2 = d0 * d0 + d1 * d1;
                        const double lr2 = log(r2);
                        const double g = tk[l] * k2 * exp(-0.5 * (dd + ts[l] + s2) * lr2);
                        const double cf = w2 * g * (tW[l] * U2 + tU[l] * W2);
                        accS[l] += -0.5 * lr2 * cf;
                        accK[l] += cf;
                    }
                }
            }
        }
    }
    // block sums in a fixed order
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        if (NQE == 0 && l >= nqe) break;
        for (int pass = 0; pass < 2; ++pass) {
            red[tid] = pass == 0 ? accS[l] : accK[l];
            __syncthreads();
            for (int s = blockDim.x / 2; s >= 1; s >>= 1) {
                if (tid < s) red[tid] += red[tid + s];
                __syncthreads();
            }
            if (tid == 0) {
                const int64_t q = cell * nqe + l;
                const double v = -2.0 * P.a_scale * tw[l] * red[0];
                if (pass == 0) Ds[(int64_t)f * P.nq + q] += v;
                else Dk[(int64_t)f * P.nq + q] += v / (2.0 * tk[l] * tk[l]);
            }
            __syncthreads();
        }
    }
}

// The same sums with the target point fixed per thread (rule sizes known at compile
// time): thread tid owns point l = tid % NQE of the cell and takes the source items
// of group tid / NQE, G = 256 / NQE groups in turn.  Each thread keeps its point's
// data and two sums in registers; the groups' sums are added in group order.
template <int NQE>
FPDE_KERNEL void k_adj_knear_pt(AdjKnear P, int f, double* Ds, double* Dk) {
    constexpr int G = 256 / NQE;
    __shared__ double redS[256], redK[256];
    const int64_t ci = blockIdx.x;
    const int64_t cell = P.icells[ci];
    const int nv = P.dim + 1;
    const int tid = threadIdx.x, l = tid % NQE, g = tid / NQE;
    const double* qs = P.qs + (int64_t)f * P.nq;
    const double* qk = P.qk + (int64_t)f * P.nq;
    int tv[3] = {-1, -1, -1}, tl[3] = {-1, -1, -1};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (a < nv) {
            tv[a] = P.cells[a * P.nc + cell];
            tl[a] = P.leaf_of_node[tv[a]];
        }
    const int64_t q = cell * NQE + l;
    const double tx = P.qx[q], ty = P.dim == 2 ? P.qx[P.nq + q] : 0.0;
    const double ts = qs[q], tk = qk[q];
    const double dd = (double)P.dim;
    double accS = 0.0, accK = 0.0;
    if (g < G) {
        for (int64_t e0 = P.cell_leaf_ptr[ci]; e0 < P.cell_leaf_ptr[ci + 1]; ++e0) {
            const int S = P.cell_leaf[e0];
            double tW = 0.0, tU = 0.0;   // W_S, U_S at the point
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (a < nv && tl[a] == S) {
                    const double la = P.lam[a * NQE + l];
                    tW += la * P.w[((int64_t)f * P.N + tv[a]) * P.R + P.r];
                    tU += la * P.u[((int64_t)f * P.N + tv[a]) * P.R + P.r];
                }
            int64_t base = 0;   // items of the earlier source leaves
            for (int64_t e = P.near_ptr[S]; e < P.near_ptr[S + 1]; ++e) {
                const int64_t S2 = P.near_src[e];
                const int64_t pb = P.patch_ptr[S2], pn = P.patch_ptr[S2 + 1] - pb;
                const int64_t k0 = ((g - base) % G + G) % G;   // (base + k0) % G == g
                base += pn;
                for (int64_t k = k0; k < pn; k += G) {
                    const int64_t c2 = P.patch_cell[pb + k];
                    int sv[3] = {-2, -2, -2}, sl[3] = {-1, -1, -1};
                    bool touch = false;
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        if (b < nv) {
                            sv[b] = P.cells[b * P.nc + c2];
                            sl[b] = P.leaf_of_node[sv[b]];
#pragma unroll
                            for (int a = 0; a < 3; ++a) touch |= (a < nv && tv[a] == sv[b]);
                        }
                    if (touch) continue;
                    double wv[3] = {0, 0, 0}, uv[3] = {0, 0, 0};
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        if (b < nv && sl[b] == (int)S2) {
                            wv[b] = P.w[((int64_t)f * P.N + sv[b]) * P.R + P.r];
                            uv[b] = P.u[((int64_t)f * P.N + sv[b]) * P.R + P.r];
                        }
#pragma unroll 3
                    for (int l2 = 0; l2 < NQE; ++l2) {
                        const int64_t q2 = c2 * NQE + l2;
                        double W2 = 0.0, U2 = 0.0;
#pragma unroll
                        for (int b = 0; b < 3; ++b)
                            if (b < nv) {
                                W2 += P.lam[b * NQE + l2] * wv[b];
                                U2 += P.lam[b * NQE + l2] * uv[b];
                            }
                        const double x2 = P.qx[q2], y2 = P.dim == 2 ? P.qx[P.nq + q2] : 0.0;
                        const double s2 = qs[q2], k2 = qk[q2], w2 = P.qw[q2];
                        const double d0 = tx - x2, d1 = ty - y2;
                        const double lr2 = log(d0 * d0 + d1 * d1);
                        const double gm = tk * k2 * exp(-0.5 * (dd + ts + s2) * lr2);
                        const double cf = w2 * gm * (tW * U2 + tU * W2);
                        accS += -0.5 * lr2 * cf;
                        accK += cf;
                    }
                }
            }
        }
    }
    redS[tid] = accS;
    redK[tid] = accK;
    __syncthreads();
    if (tid < NQE) {   // point tid: the groups' sums in group order
        double vs = 0.0, vk = 0.0;
        for (int gg = 0; gg < G; ++gg) {
            vs += redS[gg * NQE + tid];
            vk += redK[gg * NQE + tid];
        }
        const double c = -2.0 * P.a_scale * P.qw[q];
        Ds[(int64_t)f * P.nq + q] += c * vs;
        Dk[(int64_t)f * P.nq + q] += c * vk / (2.0 * tk * tk);
    }
}

hipError_t launch_adj_knear(const AdjKnear& P, int64_t n_icells, int F, double* Ds, double* Dk, hipStream_t st) {
    if (P.nqe > kMaxQE) return hipErrorInvalidValue;
    if (n_icells == 0) return hipSuccess;
    auto kern = P.nqe == 9 ? k_adj_knear_pt<9> : P.nqe == 3 ? k_adj_knear_pt<3> : k_adj_knear<0>;
    for (int f = 0; f < F; ++f) hipLaunchKernelGGL(kern, dim3((unsigned)n_icells), dim3(256), 0, st, P, f, Ds, Dk);
    return hipGetLastError();
}

// ------------------------------------------------------------------ density: near point sums
//
// w^T M~ u depends on rho through sum_q c(q) rho(q); the near part of rho is
// rho_near(q) = sum_{q' near, cells disjoint} omega' gamma(q, q') (eq. e:tgt-sum).
// Target-major over every point q of a density leaf (interior or not):
//   D(q) += sum_{q'} gamma(q, q') [c(q) omega' + omega_q c(q')] x {-ln r | 1 / (2 kappa(q))}.
FPDE_KERNEL void k_adj_rho_near(H2Tree t, const int64_t* perm, const int64_t* near_ptr, const int64_t* near_src,
                                const double* qx, const double* qw, const double* qs, const double* qk,
                                const double* cq, int nqe, const int32_t* cells, int64_t nc, int64_t nq, int f,
                                double a_scale, double* Ds, double* Dk) {
    __shared__ double sx[64], sy[64], sw[64], ss[64], sk[64], sc[64];
    __shared__ int sv[64][3];
    const int64_t li = blockIdx.x;
    const int64_t c = t.first_leaf + li;
    const int tid = threadIdx.x;
    const int64_t j = t.beg[c] + tid;
    const bool act = j < t.end[c];
    const int64_t q = act ? perm[j] : 0;
    double x0 = 0, x1 = 0, s0 = 0, k0 = 0, w0 = 0, c0 = 0;
    int tv[3] = {-1, -1, -1};
    if (act) {
        x0 = qx[q];
        x1 = t.dim == 2 ? qx[nq + q] : 0.0;
        s0 = qs[(int64_t)f * nq + q];
        k0 = qk[(int64_t)f * nq + q];
        w0 = qw[q];
        c0 = cq[(int64_t)f * nq + q];
        const int64_t cell = q / nqe;
        for (int a = 0; a <= t.dim; ++a) tv[a] = cells[a * nc + cell];
    }
    double accS = 0.0, accK = 0.0;
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
            sc[tid] = cq[(int64_t)f * nq + q2];
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
                const double lr2 = log(d0 * d0 + d1 * d1);
                const double g = k0 * sk[m] * exp(-0.5 * ((double)t.dim + s0 + ss[m]) * lr2);
                const double cf = g * (c0 * sw[m] + w0 * sc[m]);
                accS += -0.5 * lr2 * cf;
                accK += cf;
            }
        }
    }
    if (act) {
        Ds[(int64_t)f * nq + q] += a_scale * accS;
        Dk[(int64_t)f * nq + q] += a_scale * accK / (2.0 * k0 * k0);
    }
}

hipError_t launch_adj_rho_near(const H2Tree& t, const int64_t* perm, const int64_t* near_ptr, const int64_t* near_src,
                               const double* qx, const double* qw, const double* qs, const double* qk,
                               const double* cq, int nqe, const int32_t* cells, int64_t nc, int64_t nq, int F,
                               double a_scale, double* Ds, double* Dk, hipStream_t st) {
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(k_adj_rho_near, dim3((unsigned)t.nleaf), dim3(64), 0, st, t, perm, near_ptr, near_src, qx,
                           qw, qs, qk, cq, nqe, cells, nc, nq, f, a_scale, Ds, Dk);
    return hipGetLastError();
}

// ------------------------------------------------------------------ density: exterior beyond R
//
// rho_B(q) = a(q) / sig int t(theta)^{-sig} d theta (2D; 1D: the two end terms),
// sig = s(q) + s_out, a = a_scale sqrt(kappa(q) kappa_out) (eq. e:rho), so
//   d rho_B / d s(q)     = a int t^{-sig} (-ln t / sig - 1 / sig^2) d theta,
//   d rho_B / d kappa(q) = rho_B / (2 kappa(q)).
// Same periodic trapezoid rule in theta as the forward density.
FPDE_KERNEL void k_adj_rho_ext(int dim, int64_t nq, const double* qx, const double* qs, const double* qk,
                               const uint8_t* q_int, const double* cq, double R, double s_out, double k_out,
                               double a_scale, int n_theta, int f, double* Ds, double* Dk) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq || !q_int[q]) return;
    const double sx = qs[(int64_t)f * nq + q];
    const double sig = sx + s_out;
    const double kq = qk[(int64_t)f * nq + q];
    const double a = a_scale * kq * k_out;
    double i0 = 0.0, i1 = 0.0;   // int t^{-sig}, int t^{-sig} ln t
    if (dim == 1) {
        const double x = qx[q];
        const double la = log(R - x), lb = log(R + x);
        const double ta = exp(-sig * la), tb = exp(-sig * lb);
        i0 = ta + tb;
        i1 = ta * la + tb * lb;
    } else {
        const double x0 = qx[q], x1 = qx[nq + q];
        const double r2 = x0 * x0 + x1 * x1;
        const double dth = 2.0 * M_PI / n_theta;
        for (int i = 0; i < n_theta; ++i) {
            double sn, cs;
            sincos(dth * i, &sn, &cs);
            const double mu = x0 * cs + x1 * sn;
            const double lt = log(sqrt(mu * mu + R * R - r2) - mu);
            const double v = exp(-sig * lt);
            i0 += v;
            i1 += v * lt;
        }
        i0 *= dth;
        i1 *= dth;
    }
    const double c = cq[(int64_t)f * nq + q];
    const double rho_b = a / sig * i0;
    Ds[(int64_t)f * nq + q] += c * a * (-i1 / sig - i0 / (sig * sig));
    Dk[(int64_t)f * nq + q] += c * rho_b / (2.0 * kq * kq);
}

hipError_t launch_adj_rho_ext(int dim, int64_t nq, const double* qx, const double* qs, const double* qk,
                              const uint8_t* q_int, const double* cq, int F, double R, double s_out,
                              double k_out_sqrt, double a_scale, int n_theta, double* Ds, double* Dk,
                              hipStream_t st) {
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(k_adj_rho_ext, dim3(grid1(nq)), dim3(256), 0, st, dim, nq, qx, qs, qk, q_int, cq, R, s_out,
                           k_out_sqrt, a_scale, n_theta, f, Ds, Dk);
    return hipGetLastError();
}

hipError_t launch_adj_c(int dim, int64_t nc, int nqe, const int32_t* cells, const uint8_t* cell_int,
                        const double* lam, const double* qw, const double* w, const double* u, int64_t N, int R,
                        int F, double* c, hipStream_t st) {
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(k_adj_c, dim3(grid1(nc * nqe)), dim3(256), 0, st, dim, nc, nqe, cells, cell_int, lam, qw, w,
                           u, N, R, f, nc * nqe, c);
    return hipGetLastError();
}

// ------------------------------------------------------------------ points -> nodes
// gs[f][v] += sum_{cells c of v} sum_l lambda_slot(l) Ds[f][c nqe + l]  (likewise gk)
FPDE_KERNEL void k_adj_points(int64_t M, const int64_t* nc_ptr, const int64_t* nc_cell, const int8_t* nc_slot,
                              int nqe, const double* lam, const double* Ds, const double* Dk, int64_t nq, int f,
                              double* gs, double* gk) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= M) return;
    double as = 0.0, ak = 0.0;
    for (int64_t e = nc_ptr[v]; e < nc_ptr[v + 1]; ++e) {
        const int64_t c = nc_cell[e];
        const int slot = nc_slot[e];
        for (int l = 0; l < nqe; ++l) {
            const double la = lam[slot * nqe + l];
            as += la * Ds[(int64_t)f * nq + c * nqe + l];
            ak += la * Dk[(int64_t)f * nq + c * nqe + l];
        }
    }
    gs[(int64_t)f * M + v] += as;
    gk[(int64_t)f * M + v] += ak;
}

hipError_t launch_adj_points(int64_t M, const int64_t* nc_ptr, const int64_t* nc_cell, const int8_t* nc_slot, int nqe,
                             const double* lam, const double* Ds, const double* Dk, int64_t nq, int F, double* gs,
                             double* gk, hipStream_t st) {
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(k_adj_points, dim3(grid1(M)), dim3(256), 0, st, M, nc_ptr, nc_cell, nc_slot, nqe, lam, Ds,
                           Dk, nq, f, gs, gk);
    return hipGetLastError();
}

// ------------------------------------------------------------------ far blocks
//
// A far block (S, S') of either tree contributes fac * a_S^T Gamma b_S' with
// Gamma_{alpha beta} = gamma(xi_alpha, xi'_beta) at the Chebyshev nodes and
// a, b the nested-basis coefficients: (w^, u^) with fac = -2 for K~ (eq.
// eq:triple_product_factored), (c^, m) with fac = 1 for the density (eq.
// eq:matvec; c^ the upsweep of c, m the moments of the quadrature weights).
// Target-major with the symmetric far relation, per node alpha of cluster S:
//   G(S, alpha) = fac sum_{S' far S} sum_beta Gamma_{alpha beta}
//                 sum_r [a_S,alpha b_S',beta + b_S,alpha a_S',beta] x {-ln r | 1 / (2 kappa(xi_alpha))}.
// Coefficients are [f][cluster][alpha][r] (f strides af, bf); one block per
// (cluster, field): 64 alpha lanes x 4 groups of far pairs.
template <int D, int P>
FPDE_KERNEL void k_adj_far(H2Tree t, double fac, double a_scale, const double* a, int64_t af, const double* b,
                           int64_t bf, int R, int f, double* Gs, double* Gk) {
    constexpr int K = KR<D, P>::K;
    __shared__ double rs[4][64], rk[4][64];
    const int64_t S = blockIdx.x;
    const int al = threadIdx.x & 63, pg = threadIdx.x >> 6;
    double accS = 0.0, accK = 0.0;
    const double* ax = t.axes + S * D * P;
    const double xa = ax[al % P], ya = D == 2 ? ax[P + (al / P) % P] : 0.0;
    const double sa = al < K ? t.node_s[((int64_t)f * t.ncl + S) * K + al] : 0.0;
    const double ka = al < K ? t.node_k[((int64_t)f * t.ncl + S) * K + al] : 1.0;
    const double* aS = a + (int64_t)f * af + (S * K + al) * R;
    const double* bS = b + (int64_t)f * bf + (S * K + al) * R;
    if (al < K) {
        for (int64_t e = t.far_ptr[S] + pg; e < t.far_ptr[S + 1]; e += 4) {
            const int64_t S2 = t.far_src[e];
            const double* bx = t.axes + S2 * D * P;
            const double* aS2 = a + (int64_t)f * af + S2 * K * R;
            const double* bS2 = b + (int64_t)f * bf + S2 * K * R;
            for (int be = 0; be < K; ++be) {
                const double d0 = xa - bx[be % P];
                const double d1 = D == 2 ? ya - bx[P + be / P] : 0.0;
                const double lr2 = log(d0 * d0 + d1 * d1);
                const double sb = t.node_s[((int64_t)f * t.ncl + S2) * K + be];
                const double kb = t.node_k[((int64_t)f * t.ncl + S2) * K + be];
                const double g = ka * kb * exp(-0.5 * ((double)D + sa + sb) * lr2);
                double br = 0.0;
                for (int r = 0; r < R; ++r) br += aS[r] * bS2[be * R + r] + bS[r] * aS2[be * R + r];
                accS += -0.5 * lr2 * g * br;
                accK += g * br;
            }
        }
    }
    rs[pg][al] = accS;
    rk[pg][al] = accK;
    __syncthreads();
    if (pg == 0 && al < K) {
        const double vs = (rs[0][al] + rs[1][al]) + (rs[2][al] + rs[3][al]);
        const double vk = (rk[0][al] + rk[1][al]) + (rk[2][al] + rk[3][al]);
        Gs[((int64_t)f * t.ncl + S) * K + al] = fac * a_scale * vs;
        Gk[((int64_t)f * t.ncl + S) * K + al] = fac * a_scale * vk / (2.0 * ka * ka);
    }
}

template <int D, int P>
static void adj_far_t(const H2Tree& t, double fac, double a_scale, const double* a, int64_t af, const double* b,
                      int64_t bf, int R, int F, double* Gs, double* Gk, hipStream_t st) {
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL((k_adj_far<D, P>), dim3((unsigned)t.ncl), dim3(256), 0, st, t, fac, a_scale, a, af, b, bf, R,
                           f, Gs, Gk);
}

hipError_t launch_adj_far(const H2Tree& t, double fac, double a_scale, const double* a, int64_t af, const double* b,
                          int64_t bf, int R, int F, double* Gs, double* Gk, hipStream_t st) {
    if (t.k > 64) return hipErrorInvalidValue;
    FPDE_DISPATCH_DP(t.dim, t.p, adj_far_t, t, fac, a_scale, a, af, b, bf, R, F, Gs, Gk, st);
    return hipGetLastError();
}

// out[f][i] += sum_{e in [ptr[i], ptr[i+1])} wts[e] src[f][idx[e]]
FPDE_KERNEL void k_adj_gather(int64_t n, const int64_t* ptr, const int64_t* idx, const double* wts, const double* src,
                              int64_t src_f, double* out, int64_t out_f, int f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) acc += (wts ? wts[e] : 1.0) * src[(int64_t)f * src_f + idx[e]];
    out[(int64_t)f * out_f + i] += acc;
}

hipError_t launch_adj_gather(int64_t n, const int64_t* ptr, const int64_t* idx, const double* wts, const double* src,
                             int64_t src_f, int F, double* out, int64_t out_f, hipStream_t st) {
    for (int f = 0; f < F; ++f)
        hipLaunchKernelGGL(k_adj_gather, dim3(grid1(n)), dim3(256), 0, st, n, ptr, idx, wts, src, src_f, out, out_f, f);
    return hipGetLastError();
}

// x[i] *= alpha (the scale of the adjoint's output)
FPDE_KERNEL void k_scale(int64_t n, double alpha, double* x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] *= alpha;
}

hipError_t launch_scale(int64_t n, double alpha, double* x, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale, dim3(grid1(n)), dim3(256), 0, st, n, alpha, x);
    return hipGetLastError();
}

}  // namespace fpde
