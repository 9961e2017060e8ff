// Algebraic recompression of the far field's nested bases (host math and device steps).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace fpde {

struct RcTree {
    int64_t N, ncl, first_leaf;   // dofs, clusters (heap order), first leaf cluster
    int K;                        // Chebyshev rank p^dim (<= 32)
    const int64_t* beg;           // [ncl] tree-order row ranges
    const int64_t* end;
};

struct RcOrth {
    std::vector<double> Q;    // [N][K] orthonormal leaf factors (tree order)
    std::vector<double> R;    // [ncl][K][K] U_t = Q_t R_t (nested)
    std::vector<double> Eo;   // [ncl][K][K] orthonormal transfers (child index, parent index)
};

struct RcOut {
    int r = 0;                 // uniform (padded) rank
    std::vector<int> ranks;    // [ncl] rank of each cluster before padding
    std::vector<double> U;     // [N][r] new leaf bases (tree order)
    std::vector<double> E;     // [ncl][r][r] new transfers (child index, parent index)
    std::vector<double> P;     // [ncl][r][K] coupling projections
};

// Dense K x K transfers Ed[c][beta][alpha] from the per-dimension factors Esep[c][dim][b][a].
void rc_dense_transfers(const RcTree& t, int dim, int p, const double* Esep, std::vector<double>& Ed);
// Orthogonalise the nested bases: leaf QR, then QR of the stacked parent transfers.
void rc_orthogonalize(const RcTree& t, const double* U, const std::vector<double>& Ed, RcOrth& o);
// Truncate with relative tolerance tol given H[c] = sum_f sum_{(c,s) far} S C_s S^T; returns r.
int rc_truncate(const RcTree& t, const RcOrth& o, const std::vector<double>& H, double tol, RcOut& out);

// Device steps (fpde_recompress.hip).  St[f][e][beta][alpha] = S_e[alpha][beta] (rank K),
// far list CSR by target (far_ptr, far_src).
// H[t] = sum_f sum_{e in far(t)} S_e C_src(e) S_e^T, C = R^T R per cluster ([ncl][K][K] each)
hipError_t launch_rc_weights(int64_t ncl, int K, int F, int64_t nfar, const int64_t* far_ptr, const int64_t* far_src,
                             const double* St, const double* C, double* H, hipStream_t st);
// Sr[f][e][beta][alpha] = (P_t S_e P_s^T)[alpha][beta], rank r, P [ncl][r][K]; pair e is
// (far_tgt[e], far_src[e])
hipError_t launch_rc_project(int64_t ncl, int K, int r, int F, int64_t nfar, const int64_t* far_tgt,
                             const int64_t* far_src, const double* St, const double* P, double* Sr, hipStream_t st);

}  // namespace fpde
