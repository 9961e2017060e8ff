// Algebraic recompression of the Chebyshev H2 far field (Sec. 5.3, closing
// remark: the generic polynomial bases do not have optimal constants, so the
// ranks can be reduced algebraically).  Host side, FP64, K <= 32:
//
//  1. orthogonalise the nested bases (leaf QR U_t = Q_t R_t; parents: QR of
//     the stacked [R_c1 E_c1; R_c2 E_c2], whose Q blocks become orthonormal
//     transfers), so every far block U_t S U_s^T = Q_t (R_t S R_s^T) Q_s^T;
//  2. total cluster weights, top down: G_t = R_t H_t R_t^T + Eo_t G_parent Eo_t^T
//     with H_t = sum over fields and far pairs (t, s) of S C_s S^T, C_s = R_s^T R_s
//     (the device computes H_t);
//  3. truncate bottom up: leaves keep the eigenvectors of G_t whose eigenvalues
//     exceed tol^2 times the largest weight eigenvalue of the tree; a parent is
//     re-expressed in its children's truncated bases (QR of the projected
//     stacked transfers) and truncated with its weight in those coordinates;
//  4. new leaf bases U'_t = Q_t T_t, transfers E'_c (r_c x r_parent), and the
//     projections P_t = Pi_t R_t that turn each coupling matrix S into
//     P_t S P_s^T (the device applies them).
// Every rank is padded with zeros to the largest one, r, so the apply kernels
// see one uniform rank.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "fpde_recompress.h"
#include "fpde_threads.h"

namespace fpde {

namespace {

// Thin Householder QR of a row-major m x n matrix A: A = Q R with Q (m x n, orthonormal
// columns; columns past min(m, n) zero) and R (n x n, upper triangular; rows past
// min(m, n) zero).
void qr_thin(int m, int n, const double* A, double* Q, double* R) {
    std::vector<double> W(A, A + (size_t)m * n);
    const int kmax = std::min(m, n);
    std::vector<double> V((size_t)kmax * m, 0.0), beta(kmax, 0.0);
    for (int j = 0; j < kmax; ++j) {
        double nrm = 0.0;
        for (int i = j; i < m; ++i) nrm += W[(size_t)i * n + j] * W[(size_t)i * n + j];
        nrm = std::sqrt(nrm);
        double* v = &V[(size_t)j * m];
        if (nrm == 0.0) continue;   // beta = 0: identity reflector
        const double a = W[(size_t)j * n + j];
        const double alpha = a >= 0.0 ? -nrm : nrm;
        for (int i = j; i < m; ++i) v[i] = W[(size_t)i * n + j];
        v[j] -= alpha;
        double vv = 0.0;
        for (int i = j; i < m; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        beta[j] = 2.0 / vv;
        for (int c = j; c < n; ++c) {
            double s = 0.0;
            for (int i = j; i < m; ++i) s += v[i] * W[(size_t)i * n + c];
            s *= beta[j];
            for (int i = j; i < m; ++i) W[(size_t)i * n + c] -= s * v[i];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < n; ++c) R[(size_t)i * n + c] = (i < kmax && c >= i) ? W[(size_t)i * n + c] : 0.0;
    // Q = H_0 ... H_{kmax-1} applied to the first n columns of the identity
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < n; ++c) Q[(size_t)i * n + c] = (i == c && c < kmax) ? 1.0 : 0.0;
    for (int j = kmax - 1; j >= 0; --j) {
        if (beta[j] == 0.0) continue;
        const double* v = &V[(size_t)j * m];
        for (int c = 0; c < n; ++c) {
            double s = 0.0;
            for (int i = j; i < m; ++i) s += v[i] * Q[(size_t)i * n + c];
            s *= beta[j];
            for (int i = j; i < m; ++i) Q[(size_t)i * n + c] -= s * v[i];
        }
    }
}

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major):
// eigenvalues descending in lam, eigenvectors in the columns of V.
void eig_sym(int n, const double* S, double* lam, double* V) {
    std::vector<double> A(S, S + (size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[(size_t)i * n + j] = i == j ? 1.0 : 0.0;
    double fro = 0.0;
    for (int i = 0; i < n * n; ++i) fro += A[i] * A[i];
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
        if (off <= 1e-30 * fro || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double th = (aqq - app) / (2.0 * apq);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {   // A <- J^T A J, rows and columns p, q
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int a, int b) { return A[(size_t)a * n + a] > A[(size_t)b * n + b]; });
    std::vector<double> Vs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        lam[j] = A[(size_t)ord[j] * n + ord[j]];
        for (int i = 0; i < n; ++i) Vs[(size_t)i * n + j] = V[(size_t)i * n + ord[j]];
    }
    std::copy(Vs.begin(), Vs.end(), V);
}

// C (m x n) = A (m x k) B (k x n), all row-major; tA / tB: use the transpose
void gemm(int m, int n, int k, const double* A, bool tA, const double* B, bool tB, double* C) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int l = 0; l < k; ++l)
                s += (tA ? A[(size_t)l * m + i] : A[(size_t)i * k + l]) * (tB ? B[(size_t)j * k + l] : B[(size_t)l * n + j]);
            C[(size_t)i * n + j] = s;
        }
}

}  // namespace

void rc_dense_transfers(const RcTree& t, int dim, int p, const double* Esep, std::vector<double>& Ed) {
    const int K = t.K;
    Ed.assign((size_t)t.ncl * K * K, 0.0);
    for (int64_t c = 1; c < t.ncl; ++c) {
        const double* e = Esep + (size_t)c * dim * p * p;   // [dim][b][a]
        for (int be = 0; be < K; ++be)
            for (int al = 0; al < K; ++al) {
                double v = e[(be % p) * p + (al % p)];
                if (dim == 2) v *= e[p * p + (be / p) * p + (al / p)];
                Ed[((size_t)c * K + be) * K + al] = v;
            }
    }
}

void rc_orthogonalize(const RcTree& t, const double* U, const std::vector<double>& Ed, RcOrth& o) {
    const int K = t.K;
    o.Q.assign((size_t)t.N * K, 0.0);
    o.R.assign((size_t)t.ncl * K * K, 0.0);
    o.Eo.assign((size_t)t.ncl * K * K, 0.0);
    parallel_for(t.ncl - t.first_leaf, [&](int64_t i) {
        const int64_t c = t.first_leaf + i, b = t.beg[c], n = t.end[c] - t.beg[c];
        if (n > 0) qr_thin((int)n, K, U + (size_t)b * K, &o.Q[(size_t)b * K], &o.R[(size_t)c * K * K]);
    });
    std::vector<double> M((size_t)2 * K * K), Qm((size_t)2 * K * K);
    for (int64_t c = t.first_leaf - 1; c >= 0; --c) {
        for (int s = 0; s < 2; ++s) {   // M = [R_c1 E_c1; R_c2 E_c2]
            const int64_t ch = 2 * c + 1 + s;
            gemm(K, K, K, &o.R[(size_t)ch * K * K], false, &Ed[(size_t)ch * K * K], false, &M[(size_t)s * K * K]);
        }
        qr_thin(2 * K, K, M.data(), Qm.data(), &o.R[(size_t)c * K * K]);
        for (int s = 0; s < 2; ++s)
            std::copy(Qm.begin() + (size_t)s * K * K, Qm.begin() + (size_t)(s + 1) * K * K,
                      o.Eo.begin() + (size_t)(2 * c + 1 + s) * K * K);
    }
}

int rc_truncate(const RcTree& t, const RcOrth& o, const std::vector<double>& H, double tol, RcOut& out) {
    const int K = t.K;
    const size_t KK = (size_t)K * K;
    // total weights, top down
    std::vector<double> G((size_t)t.ncl * KK);
    auto weight = [&](int64_t c) {
        std::vector<double> tmp(KK), tmp2(KK);
        gemm(K, K, K, &o.R[c * KK], false, &H[c * KK], false, tmp.data());
        gemm(K, K, K, tmp.data(), false, &o.R[c * KK], true, &G[c * KK]);
        if (c > 0) {
            const int64_t p = (c - 1) / 2;
            gemm(K, K, K, &o.Eo[c * KK], false, &G[p * KK], false, tmp.data());
            gemm(K, K, K, tmp.data(), false, &o.Eo[c * KK], true, tmp2.data());
            for (size_t i = 0; i < KK; ++i) G[c * KK + i] += tmp2[i];
        }
    };
    for (int64_t n = 1; n - 1 < t.ncl; n *= 2)   // level with clusters [n - 1, 2n - 1)
        parallel_for(n, [&](int64_t i) { weight(n - 1 + i); });
    std::vector<double> lamG((size_t)t.ncl * K), VG((size_t)t.ncl * KK);
    parallel_for(t.ncl, [&](int64_t c) { eig_sym(K, &G[c * KK], &lamG[(size_t)c * K], &VG[c * KK]); });
    double Lmax = 0.0;
    for (int64_t c = 0; c < t.ncl; ++c) Lmax = std::max(Lmax, lamG[(size_t)c * K]);
    const double thr = tol * tol * Lmax;
    // bottom up: per cluster the new basis in old orthonormal coordinates is
    // expressed by Pi_t (r_t x K): Q_t ~ U'_t Pi_t; children-relative transfer blocks
    std::vector<std::vector<double>> Pi(t.ncl), Tc(t.ncl);   // Tc: [m_c][r_c] new basis in the c's candidate coords
    std::vector<int> rk(t.ncl, 0);
    std::vector<std::vector<double>> Ftr(t.ncl);   // for parents: the truncated basis in [child1; child2] coordinates
    auto one = [&](int64_t c) {
        std::vector<double> lam(K), V(KK), tmp(KK);
        if (c >= t.first_leaf) {
            std::copy(&lamG[(size_t)c * K], &lamG[(size_t)c * K] + K, lam.begin());
            std::copy(&VG[c * KK], &VG[c * KK] + KK, V.begin());
            int r = 0;
            while (r < K && lam[r] > thr) ++r;
            r = std::max(r, 1);
            rk[c] = r;
            Tc[c].assign((size_t)K * r, 0.0);   // T_t = V[:, :r]
            for (int i = 0; i < K; ++i)
                for (int j = 0; j < r; ++j) Tc[c][(size_t)i * r + j] = V[(size_t)i * K + j];
            Pi[c].assign((size_t)r * K, 0.0);   // Pi = T^T
            for (int i = 0; i < r; ++i)
                for (int j = 0; j < K; ++j) Pi[c][(size_t)i * K + j] = V[(size_t)j * K + i];
        } else {
            const int64_t c1 = 2 * c + 1, c2 = 2 * c + 2;
            const int r1 = rk[c1], r2 = rk[c2], m = r1 + r2;
            // F = [Pi_c1 Eo_c1; Pi_c2 Eo_c2]  (m x K)
            std::vector<double> Fm((size_t)m * K);
            gemm(r1, K, K, Pi[c1].data(), false, &o.Eo[c1 * KK], false, Fm.data());
            gemm(r2, K, K, Pi[c2].data(), false, &o.Eo[c2 * KK], false, Fm.data() + (size_t)r1 * K);
            // F = Qf Rf (Qf m x K, Rf K x K); the weight in Qf coordinates is Rf G Rf^T
            std::vector<double> Qf((size_t)m * K), Rf(KK), Gh(KK);
            qr_thin(m, K, Fm.data(), Qf.data(), Rf.data());
            gemm(K, K, K, Rf.data(), false, &G[c * KK], false, tmp.data());
            gemm(K, K, K, tmp.data(), false, Rf.data(), true, Gh.data());
            eig_sym(K, Gh.data(), lam.data(), V.data());
            int r = 0;
            while (r < std::min(K, m) && lam[r] > thr) ++r;
            r = std::max(r, 1);
            rk[c] = r;
            // new basis of c in child coordinates: Qf V_r (m x r)
            Ftr[c].assign((size_t)m * r, 0.0);
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < r; ++j) {
                    double s = 0.0;
                    for (int l = 0; l < K; ++l) s += Qf[(size_t)i * K + l] * V[(size_t)l * K + j];
                    Ftr[c][(size_t)i * r + j] = s;
                }
            // Pi_c = V_r^T Rf  (r x K)
            Pi[c].assign((size_t)r * K, 0.0);
            for (int i = 0; i < r; ++i)
                for (int j = 0; j < K; ++j) {
                    double s = 0.0;
                    for (int l = 0; l < K; ++l) s += V[(size_t)l * K + i] * Rf[(size_t)l * K + j];
                    Pi[c][(size_t)i * K + j] = s;
                }
        }
    };
    // leaves, then one level at a time upwards (clusters of a level are independent)
    parallel_for(t.ncl - t.first_leaf, [&](int64_t i) { one(t.first_leaf + i); });
    for (int64_t lev0 = (t.first_leaf + 1) / 2 - 1, n = (t.first_leaf + 1) / 2; n >= 1; n /= 2, lev0 = n - 1)
        parallel_for(n, [&](int64_t i) { one(lev0 + i); });
    int rmax = 1;
    for (int64_t c = 0; c < t.ncl; ++c) rmax = std::max(rmax, rk[c]);
    const int r = rmax;
    out.r = r;
    out.ranks.assign(rk.begin(), rk.end());
    // leaf bases U' = Q_t T_t, padded to r columns
    out.U.assign((size_t)t.N * r, 0.0);
    for (int64_t c = t.first_leaf; c < t.ncl; ++c) {
        const int64_t b = t.beg[c], n = t.end[c] - t.beg[c];
        const int rc = rk[c];
        for (int64_t i = 0; i < n; ++i)
            for (int j = 0; j < rc; ++j) {
                double s = 0.0;
                for (int l = 0; l < K; ++l) s += o.Q[(size_t)(b + i) * K + l] * Tc[c][(size_t)l * rc + j];
                out.U[(size_t)(b + i) * r + j] = s;
            }
    }
    // transfers E'_child [r][r] (child index, parent index): the child's block of Ftr[parent]
    out.E.assign((size_t)t.ncl * r * r, 0.0);
    for (int64_t c = 0; c < t.first_leaf; ++c) {
        const int64_t c1 = 2 * c + 1, c2 = 2 * c + 2;
        const int r1 = rk[c1], rp = rk[c];
        for (int s = 0; s < 2; ++s) {
            const int64_t ch = s ? c2 : c1;
            const int rc = rk[ch], off = s ? r1 : 0;
            for (int i = 0; i < rc; ++i)
                for (int j = 0; j < rp; ++j) out.E[((size_t)ch * r + i) * r + j] = Ftr[c][(size_t)(off + i) * rp + j];
        }
    }
    // coupling projections P_t = Pi_t R_t  [r][K]
    out.P.assign((size_t)t.ncl * r * K, 0.0);
    for (int64_t c = 0; c < t.ncl; ++c) {
        const int rc = rk[c];
        for (int i = 0; i < rc; ++i)
            for (int j = 0; j < K; ++j) {
                double s = 0.0;
                for (int l = 0; l < K; ++l) s += Pi[c][(size_t)i * K + l] * o.R[c * KK + (size_t)l * K + j];
                out.P[((size_t)c * r + i) * K + j] = s;
            }
    }
    return r;
}

}  // namespace fpde
