// C ABI of libfpde: validation, planning, device orchestration of the build
// (Alg. 1 of the paper) and of the operator apply / CG solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <numeric>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fpde.h"
#include "fpde_internal.h"
#include "fpde_plan.h"
#include "fpde_recompress.h"
#include "fpde_threads.h"

namespace fpde {
hipError_t launch_basis_n(const H2Tree& t, int64_t N, const int64_t* perm, const int64_t* nc_ptr,
                          const int64_t* nc_cell, const int8_t* nc_slot, int nqe, const double* qx,
                          const double* qw, const double* lam, int64_t nq_all, double* U,
                          hipStream_t st);
}

using namespace fpde;

namespace {

thread_local std::string g_err;

struct Fail {
    fpde_status st;
    std::string msg;
};

[[noreturn]] void fail(fpde_status st, const std::string& m) { throw Fail{st, m}; }

void hipck(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(FPDE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// device arena: every allocation of an operator is recorded and freed together
struct Arena {
    std::vector<void*> ptrs;
    int64_t bytes = 0;
    uint64_t limit = 0;
    template <class T>
    T* alloc(int64_t n) {
        if (n <= 0) n = 1;
        size_t b = sizeof(T) * (size_t)n;
        if (limit && (uint64_t)(bytes + b) > limit)
            fail(FPDE_ENOMEM, "device memory above max_device_bytes");
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) fail(FPDE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        ptrs.push_back(p);
        bytes += b;
        return (T*)p;
    }
    template <class T>
    T* upload(const std::vector<T>& v, hipStream_t st) {
        T* p = alloc<T>((int64_t)v.size());
        if (!v.empty()) hipck(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st), "upload");
        return p;
    }
    void release(void* p) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it != ptrs.end()) {
            (void)hipFree(p);   // a failure here surfaces at the next checked call
            ptrs.erase(it);
        }
    }
    ~Arena() {
        for (void* p : ptrs) (void)hipFree(p);
    }
};

struct TreeDev {
    int64_t* beg = nullptr;
    int64_t* end = nullptr;
    double* axes = nullptr;
    double* E = nullptr;
    double* node_s = nullptr;
    double* node_k = nullptr;
    int64_t* far_ptr = nullptr;
    int64_t* far_src = nullptr;
    int64_t* perm = nullptr;
};

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct fpde_op {
    HostMesh mesh;
    fpde_opts opts{};
    int F = 1;
    bool plan_only = false;
    std::vector<double> s, kappa;   // [F][M]
    ElementRule er;
    QuadPoints Q;
    NodeCells ncs;
    std::vector<Pair> pairs;        // enumeration order (cell, neighbour)
    std::vector<int64_t> pair_order;// device order (sorted by kind)
    // K tree
    Tree kt;
    std::vector<std::pair<int64_t, int64_t>> kfar, knear;
    std::vector<int64_t> pos_of_dof;
    // density tree
    Tree rt;
    std::vector<std::pair<int64_t, int64_t>> rfar, rnear;
    // CSR in tree order
    std::vector<int64_t> csr_ptr;
    std::vector<int32_t> csr_col;
    // device
    Arena arena;
    hipStream_t stream = nullptr;
    double* d_X = nullptr;
    int32_t* d_C = nullptr;
    uint8_t* d_cint = nullptr;
    double* d_qw = nullptr;
    double* d_lam = nullptr;
    int64_t* d_nc_ptr = nullptr;
    int64_t* d_nc_cell = nullptr;
    int8_t* d_nc_slot = nullptr;
    double* d_B = nullptr;
    double* d_M = nullptr;
    double* d_BM = nullptr;
    double* d_rho = nullptr;       // [F][nq] density at interior points (kept for export)
    int64_t* d_csr_ptr = nullptr;
    int32_t* d_csr_col = nullptr;
    TreeDev kdev;
    int64_t* d_leaf_beg = nullptr;
    int64_t* d_near_ptr = nullptr;
    int64_t* d_near_src = nullptr;
    double* d_near = nullptr;       // near leaf blocks [F][pairs][cap][cap] (build only; repacked as panels)
    double* d_U = nullptr;
    double* d_St = nullptr;         // [F][nfar][k][k] coupling matrices (transposed)
    int64_t cap = 0;
    int ls2 = 0;                    // subtree-root level of the multi-RHS far chain
    int32_t* d_csr_col_dof = nullptr;   // CSR columns as dof indices
    // near leaf blocks packed per target leaf: panel[f][poff[li] + row*pstride[li] + col], columns dof-indexed
    double* d_panel = nullptr;
    int64_t *d_poff = nullptr, *d_pstride = nullptr, *d_pcols_ptr = nullptr;
    int32_t* d_pcols = nullptr;
    int64_t panel_max_stride = 0, panel_total = 0;
    // by leaf slot for the one-vector near rows: panel columns and the ELL form of B + M
    int32_t* d_pcols_pad = nullptr;        // [nleaf][panel_max_stride], -1 padding
    int32_t* d_ell_col = nullptr;          // [nleaf * cap][ell_w] dof columns (see PanelPlan::ell_col)
    double* d_ell_val = nullptr;           // [F][nleaf * cap][ell_w] values of B + M
    int ell_w = 0;
    unsigned int* d_tickets = nullptr;     // [F][ncl] ticket counters of the one-vector upsweep (self-resetting)
    double* d_zh = nullptr;                // [F][ncl][k] coupling sums of the one-vector apply
    // far list of the one-vector apply, sources moved down to the upsweep's subtree levels
    int64_t nfar1 = 0;
    int64_t *d_far1_ptr = nullptr, *d_far1_src = nullptr;
    double* d_St1 = nullptr;               // [F][nfar1][k][k], transposed like d_St
    double* d_zp = nullptr;                // [F][nchunks][k] partial coupling sums
    double* d_Upad = nullptr;              // [nleaf * cap][k] bases by leaf slot
    int64_t* d_perm_pad = nullptr;         // [nleaf * cap] output index by leaf slot, -1 padding
    UpPlan up[2]{};                        // one-launch upsweep plan per precision (0 FP64, 1 FP32)
    FarPlan far_plan{};                    // far targets of the one-vector output kernel
    struct {                               // FP32 operator data of a mixed-precision operator
        float *U = nullptr, *E = nullptr, *St = nullptr, *St1 = nullptr, *panel = nullptr, *Upad = nullptr;
        float* panel_bm = nullptr;   // panels with B + M added (several right-hand sides)
        float *xh = nullptr, *zh = nullptr, *zp = nullptr;   // workspace, one right-hand side
        float *xhR = nullptr, *yhR = nullptr;  // workspace [F][ncl][K][R]
    } f32;
    bool mixed = false;                    // built with FPDE_PREC_MIXED
    struct {                               // recompressed far field (opts.recompress_tol > 0)
        bool on = false;
        int r = 0;                         // uniform rank
        double *U = nullptr, *Upad = nullptr, *E = nullptr, *St = nullptr;   // [N][r], [nleaf cap][r],
        float *U32 = nullptr, *Upad32 = nullptr, *E32 = nullptr, *St32 = nullptr;   // [ncl][r][r], [F][nfar][r][r]
    } rc;
    // apply workspace
    int64_t ws_R = 0;
    double* d_xt = nullptr;
    double* d_xh = nullptr;
    double* d_yh = nullptr;
    // solve workspace ([F][N][R] vectors, per-block partial sums, per-system scalars)
    int64_t sw_R = 0;
    double *d_r = nullptr, *d_p = nullptr, *d_Ap = nullptr, *d_d = nullptr, *d_rout = nullptr;
    double *d_part1 = nullptr, *d_part2 = nullptr, *d_part3 = nullptr, *d_bb = nullptr, *d_rro = nullptr;
    double* d_part_far = nullptr;   // [F][output-kernel blocks] p . Ap partials of fused CG iterations (R = 1)
    CgScalars cg{};
    int* h_nact = nullptr;                    // pinned host copy of the active-system count
    double* d_dinv = nullptr;                 // [F][N] 1 / diag(A_h) (FPDE_FLAG_JACOBI), dof order
    double *d_hist_a = nullptr, *d_hist_b = nullptr;   // Lanczos coefficients of a CG pass [kHist][S]
    fpde_stats_t stats{};
    // profiling: events recorded per apply (gather begin, gather end, far end, out end)
    bool profiling = false;
    std::vector<std::array<hipEvent_t, 5>> prof_ev;
    hipStream_t stream2 = nullptr;            // side stream of the multi-vector far chain (fork/join)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    double* d_tmp = nullptr;                  // [F][nfar][k][R] per-pair coupling products
    // ---- adjoint (fpde_apply_adjoint): build data kept on the device
    struct {
        bool ok = false;
        std::string why;                      // reason when the adjoint is unavailable
        double *s = nullptr, *k = nullptr;    // nodal fields [F][M]
        double *qx = nullptr, *qs = nullptr, *qk = nullptr;   // quadrature points, s and sqrt(kappa) there
        uint8_t* qint = nullptr;
        int32_t* pairs = nullptr;             // singular pair rows (device order)
        double *g = nullptr, *w = nullptr;    // Gauss rule of the singular rules
        int64_t *slot_ptr = nullptr, *slot_idx = nullptr;   // node -> pair * 12 + slot
        TreeDev rdev;                         // density tree
        int64_t *rnear_ptr = nullptr, *rnear_src = nullptr;
        int64_t n_icells = 0;
        int64_t *icells = nullptr, *cell_leaf_ptr = nullptr, *patch_ptr = nullptr, *patch_cell = nullptr;
        int32_t *cell_leaf = nullptr, *leaf_of_node = nullptr;
        int64_t *kst_ptr = nullptr, *kst_idx = nullptr, *rst_ptr = nullptr, *rst_idx = nullptr;
        double *kst_w = nullptr, *rst_w = nullptr;   // Chebyshev-node stencils: node -> (cluster K + alpha)
        // workspace
        int64_t ws_R = 0;
        double *out12 = nullptr, *Ds = nullptr, *Dk = nullptr, *c = nullptr, *xw = nullptr, *xu = nullptr;
        double *chat = nullptr, *mom = nullptr, *Gs = nullptr, *Gk = nullptr, *rGs = nullptr, *rGk = nullptr;
    } adj;
};

// ------------------------------------------------------------------ helpers

namespace {

void validate(const fpde_mesh* m, int F, const double* s, const double* kap, const fpde_opts& o) {
    if (!m) fail(FPDE_EINVAL, "mesh is NULL");
    if (m->dim != 1 && m->dim != 2) fail(FPDE_EINVAL, "dim must be 1 or 2");
    if (m->n_nodes <= 0 || m->n_cells <= 0) fail(FPDE_EINVAL, "empty mesh");
    if (m->n_dofs <= 0 || m->n_dofs >= m->n_nodes) fail(FPDE_EINVAL, "need 0 < n_dofs < n_nodes");
    if (!m->coords || !m->cells || !m->cell_interior) fail(FPDE_EINVAL, "NULL mesh array");
    if (F < 1) fail(FPDE_EINVAL, "n_fields must be >= 1");
    if (!s || !kap) fail(FPDE_EINVAL, "NULL s or kappa");
    if (!(o.s_bar < 1.0) || !(o.s_bar >= 0.0)) fail(FPDE_EDOMAIN, "s_bar must lie in [0,1)");
    if (o.cheb_p < 1 || o.cheb_p > kMaxP) fail(FPDE_EINVAL, "cheb_p must be in [1,8]");
    if (o.nq_sing < 1 || o.nq_sing > kMaxNq || o.nq_reg < 1 || o.nq_reg > kMaxNq)
        fail(FPDE_EINVAL, "nq_sing/nq_reg must be in [1,8]");
    if (o.leaf_size < 1 || o.leaf_size > 256 || o.leaf_size_rho < 1 || o.leaf_size_rho > 64)
        fail(FPDE_EINVAL, "leaf_size in [1,256], leaf_size_rho in [1,64]");
    if (!(o.eta > 0.0)) fail(FPDE_EINVAL, "eta must be > 0");
    if (!(o.recompress_tol >= 0.0 && o.recompress_tol < 1.0)) fail(FPDE_EINVAL, "recompress_tol must be in [0,1)");
    if (o.recompress_tol > 0.0) {
        int kk = 1;
        for (int i = 0; i < m->dim; ++i) kk *= o.cheb_p;
        if (kk > 32) fail(FPDE_EINVAL, "recompression needs a Chebyshev rank p^dim <= 32");
    }
    if (!(o.a_scale > 0.0)) fail(FPDE_EDOMAIN, "a_scale must be > 0");
    if (m->exterior_radius < 0.0) fail(FPDE_EINVAL, "exterior_radius < 0");
    if (m->exterior_radius > 0.0 && (o.n_theta < 1 || !(o.kappa_exterior > 0.0) ||
                                     !(o.s_exterior >= 0.0 && o.s_exterior < 1.0)))
        fail(FPDE_EDOMAIN, "exterior parameters out of range");
    const int64_t M = m->n_nodes;
    for (int64_t i = 0; i < (int64_t)F * M; ++i) {
        if (!(s[i] >= 0.0 && s[i] <= o.s_bar)) fail(FPDE_EDOMAIN, "s outside [0, s_bar]");
        if (!(kap[i] > 0.0)) fail(FPDE_EDOMAIN, "kappa must be > 0");
    }
    const int k = m->dim + 1;
    bool has_ext = false;
    std::vector<uint8_t> on_int(M, 0), on_ext(M, 0);
    for (int64_t c = 0; c < m->n_cells; ++c) {
        for (int a = 0; a < k; ++a) {
            int32_t v = m->cells[a * m->n_cells + c];
            if (v < 0 || v >= M) fail(FPDE_EINVAL, "cell vertex out of range");
            (m->cell_interior[c] ? on_int : on_ext)[v] = 1;
            for (int b = 0; b < a; ++b)
                if (m->cells[b * m->n_cells + c] == v) fail(FPDE_EINVAL, "degenerate cell (repeated vertex)");
        }
        if (!m->cell_interior[c]) has_ext = true;
    }
    for (int64_t v = 0; v < m->n_dofs; ++v)
        if (on_ext[v]) fail(FPDE_EINVAL, "an interior node belongs to an exterior cell");
    if (!has_ext && !(m->exterior_radius > 0.0))
        fail(FPDE_EINVAL, "the exterior region is empty (|Omega_e| = 0) and exterior_radius = 0");
}

H2Tree make_h2(const Tree& t, const TreeDev& d, int p) {
    H2Tree h{};
    h.dim = t.dim;
    h.p = p;
    h.k = t.dim == 2 ? p * p : p;
    h.L = t.L;
    h.ncl = t.ncl;
    h.nleaf = t.nleaf();
    h.first_leaf = t.first_leaf();
    h.beg = d.beg;
    h.end = d.end;
    h.axes = d.axes;
    h.E = d.E;
    h.node_s = d.node_s;
    h.node_k = d.node_k;
    h.far_ptr = d.far_ptr;
    h.far_src = d.far_src;
    return h;
}

// Chebyshev axes of every cluster and the P1 stencil of each of its nodes: up to 3
// (mesh node, P1 weight) of the cell holding it, or (nearest node, 1) outside the
// mesh; node -1 pads.  The values of s and sqrt(kappa) there come from the stencils
// on the device (launch_node_fields).
void cluster_nodes(const fpde_op& op, const Tree& t, const Locator& loc, std::vector<double>& axes,
                   std::vector<int64_t>& st_node, std::vector<double>& st_w) {
    const int d = t.dim, p = op.opts.cheb_p, k = d == 2 ? p * p : p;
    axes.assign(t.ncl * d * p, 0.0);
    st_node.assign(t.ncl * k * 3, -1);
    st_w.assign(t.ncl * k * 3, 0.0);
    parallel_for(t.ncl, [&](int64_t c) {
        double* ax = &axes[c * d * p];
        cheb_axes(d, &t.lo[c * d], &t.hi[c * d], p, ax);
        for (int al = 0; al < k; ++al) {
            double x[2] = {ax[al % p], d == 2 ? ax[p + al / p] : 0.0};
            double lam[3];
            int64_t node = -1;
            const int64_t cell = loc.locate(x, lam, &node);
            const int64_t o = (c * k + al) * 3;
            if (cell < 0) {
                st_node[o] = node;
                st_w[o] = 1.0;
            } else {
                for (int a = 0; a <= d; ++a) {
                    st_node[o + a] = op.mesh.v(a, cell);
                    st_w[o + a] = lam[a];
                }
            }
        }
    });
}

// node -> list of (index, weight), entries sorted by (node, index), no (node, index)
// repeated (the nodes of one stencil are distinct): a counting sort on the node, on host
// threads with atomic counters for long lists, then each node's entries by index
void node_csr(int64_t M, const std::vector<int64_t>& st_node, const std::vector<double>& st_w, int per,
              std::vector<int64_t>& ptr, std::vector<int64_t>& idx, std::vector<double>& wts) {
    const int64_t n = (int64_t)st_node.size();
    ptr.assign(M + 1, 0);
    if (n < (int64_t(1) << 20)) {   // entries come in increasing index: a stable pass suffices
        for (int64_t v : st_node)
            if (v >= 0) ptr[v + 1]++;
        for (int64_t i = 0; i < M; ++i) ptr[i + 1] += ptr[i];
        idx.resize(ptr[M]);
        wts.resize(ptr[M]);
        std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t v = st_node[i];
            if (v < 0) continue;
            idx[fill[v]] = i / per;
            wts[fill[v]++] = st_w[i];
        }
        return;
    }
    constexpr int64_t kChunk = int64_t(1) << 16;
    const int64_t nch = (n + kChunk - 1) / kChunk;
    parallel_for(nch, [&](int64_t ch) {
        for (int64_t i = ch * kChunk; i < std::min(n, (ch + 1) * kChunk); ++i)
            if (st_node[i] >= 0) __atomic_fetch_add(&ptr[st_node[i] + 1], int64_t(1), __ATOMIC_RELAXED);
    }, 2);
    for (int64_t i = 0; i < M; ++i) ptr[i + 1] += ptr[i];
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    std::vector<std::pair<int64_t, double>> e(ptr[M]);
    parallel_for(nch, [&](int64_t ch) {
        for (int64_t i = ch * kChunk; i < std::min(n, (ch + 1) * kChunk); ++i) {
            const int64_t v = st_node[i];
            if (v >= 0) e[__atomic_fetch_add(&fill[v], int64_t(1), __ATOMIC_RELAXED)] = {i / per, st_w[i]};
        }
    }, 2);
    idx.resize(ptr[M]);
    wts.resize(ptr[M]);
    constexpr int64_t kNodes = 4096;
    parallel_for((M + kNodes - 1) / kNodes, [&](int64_t blk) {
        for (int64_t v = blk * kNodes; v < std::min(M, (blk + 1) * kNodes); ++v) {
            std::sort(e.begin() + ptr[v], e.begin() + ptr[v + 1],
                      [](const std::pair<int64_t, double>& a, const std::pair<int64_t, double>& b) { return a.first < b.first; });
            for (int64_t q = ptr[v]; q < ptr[v + 1]; ++q) {
                idx[q] = e[q].first;
                wts[q] = e[q].second;
            }
        }
    }, 2);
}

bool symmetric_pairs(std::vector<std::pair<int64_t, int64_t>> v) {
    std::vector<std::pair<int64_t, int64_t>> w;
    for (auto& p : v) w.push_back({p.second, p.first});
    std::sort(v.begin(), v.end());
    std::sort(w.begin(), w.end());
    return v == w;
}

void far_csr(const Tree& t, const std::vector<std::pair<int64_t, int64_t>>& far,
             std::vector<int64_t>& ptr, std::vector<int64_t>& src) {
    ptr.assign(t.ncl + 1, 0);
    for (auto& pr : far) ptr[pr.first + 1]++;
    for (int64_t c = 0; c < t.ncl; ++c) ptr[c + 1] += ptr[c];
    src.resize(far.size());
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (auto& pr : far) src[fill[pr.first]++] = pr.second;
}

// ------------------------------------------------------------------ planning

void plan(fpde_op& op) {
    auto t0 = std::chrono::steady_clock::now();
    const HostMesh& m = op.mesh;
    const int d = m.dim;
    op.er = element_rule(d, op.opts.nq_reg);
    op.Q = quad_points(m, op.er);
    op.ncs = node_cells(m);
    op.pairs = touching_pairs(m, op.ncs);
    // device order of pairs: by kind (uniform waves), pair order kept within a kind
    {
        int64_t start[4] = {0, 0, 0, 0};
        for (const Pair& p : op.pairs) ++start[p.kind + 1];
        for (int k = 0; k < 3; ++k) start[k + 1] += start[k];
        op.pair_order.resize(op.pairs.size());
        for (int64_t i = 0; i < (int64_t)op.pairs.size(); ++i) op.pair_order[start[op.pairs[i].kind]++] = i;
    }
    // K tree over the dofs, extended boxes (supports of the members' basis functions)
    op.kt = kd_tree(d, m.X.data(), m.M, m.N, op.opts.leaf_size);
    Tree& kt = op.kt;
    kt.lo.assign(kt.ncl * d, 1e300);
    kt.hi.assign(kt.ncl * d, -1e300);
    for (int64_t c = kt.first_leaf(); c < kt.ncl; ++c)
        for (int64_t j = kt.beg[c]; j < kt.end[c]; ++j) {
            int64_t v = kt.perm[j];
            for (int64_t e = op.ncs.ptr[v]; e < op.ncs.ptr[v + 1]; ++e) {
                int64_t cell = op.ncs.cell[e];
                for (int a = 0; a <= d; ++a)
                    for (int kk = 0; kk < d; ++kk) {
                        double x = m.x(kk, m.v(a, cell));
                        kt.lo[c * d + kk] = std::min(kt.lo[c * d + kk], x);
                        kt.hi[c * d + kk] = std::max(kt.hi[c * d + kk], x);
                    }
            }
        }
    for (int64_t c = kt.first_leaf() - 1; c >= 0; --c)
        for (int kk = 0; kk < d; ++kk) {
            kt.lo[c * d + kk] = std::min(kt.lo[(2 * c + 1) * d + kk], kt.lo[(2 * c + 2) * d + kk]);
            kt.hi[c * d + kk] = std::max(kt.hi[(2 * c + 1) * d + kk], kt.hi[(2 * c + 2) * d + kk]);
        }
    partition(kt, op.opts.eta, nullptr, nullptr, op.kfar, op.knear);
    op.pos_of_dof.assign(m.N, -1);
    for (int64_t j = 0; j < m.N; ++j) op.pos_of_dof[kt.perm[j]] = j;
    // density tree over all quadrature points; prune targets without interior points
    op.rt = kd_tree(d, op.Q.x.data(), op.Q.nq, op.Q.nq, op.opts.leaf_size_rho);
    point_boxes(op.rt, op.Q.x.data(), op.Q.nq);
    std::vector<uint8_t> skip(op.rt.ncl, 1);
    for (int64_t c = 0; c < op.rt.ncl; ++c)
        for (int64_t j = op.rt.beg[c]; j < op.rt.end[c]; ++j)
            if (op.Q.q_int[op.rt.perm[j]]) {
                skip[c] = 0;
                break;
            }
    // far only beyond the diameters of the cells holding either cluster's points, so no
    // far pair lies in touching cells (gamma_T = gamma there)
    {
        const std::vector<double> hcell = cell_diameters(m);
        std::vector<double> hq(op.Q.nq);
        for (int64_t q = 0; q < op.Q.nq; ++q) hq[q] = hcell[q / op.Q.nqe];
        const std::vector<double> hc = cluster_h(op.rt, hq.data());
        partition(op.rt, op.opts.eta, &hc, &skip, op.rfar, op.rnear);
    }
    // CSR pattern of B (and M) in tree order: the (row, column) entries of every pair,
    // bucketed by row, then each row's columns sorted and made unique
    {
        // counts and fill by chunks of pairs on host threads, each (pair, row) taking its
        // run of slots with one atomic add; the order inside a row depends on the
        // schedule until the rows are sorted below
        constexpr int64_t kPairs = int64_t(1) << 14;
        const int64_t npair = (int64_t)op.pairs.size(), npch = (npair + kPairs - 1) / kPairs;
        std::vector<int64_t> cnt(m.N + 1, 0);
        parallel_for(npch, [&](int64_t ch) {
            int32_t dofs[5];
            for (int64_t e = ch * kPairs; e < std::min(npair, (ch + 1) * kPairs); ++e) {
                const int nd = pair_dofs(m, op.pairs[e], dofs);
                int64_t ni = 0;
                for (int b = 0; b < nd; ++b) ni += dofs[b] < m.N;
                for (int a = 0; a < nd; ++a)
                    if (dofs[a] < m.N) __atomic_fetch_add(&cnt[op.pos_of_dof[dofs[a]] + 1], ni, __ATOMIC_RELAXED);
            }
        }, 2);
        for (int64_t i = 0; i < m.N; ++i) cnt[i + 1] += cnt[i];
        std::vector<int32_t> col(cnt[m.N]);
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        parallel_for(npch, [&](int64_t ch) {
            int32_t dofs[5];
            for (int64_t e = ch * kPairs; e < std::min(npair, (ch + 1) * kPairs); ++e) {
                const int nd = pair_dofs(m, op.pairs[e], dofs);
                int64_t ni = 0;
                for (int b = 0; b < nd; ++b) ni += dofs[b] < m.N;
                for (int a = 0; a < nd; ++a) {
                    if (dofs[a] >= m.N) continue;
                    int64_t at = __atomic_fetch_add(&fill[op.pos_of_dof[dofs[a]]], ni, __ATOMIC_RELAXED);
                    for (int b = 0; b < nd; ++b)
                        if (dofs[b] < m.N) col[at++] = (int32_t)op.pos_of_dof[dofs[b]];
                }
            }
        }, 2);
        // rows sorted and made unique in place on host threads, then packed in row order
        constexpr int64_t kRows = 1024;
        const int64_t nblk = (m.N + kRows - 1) / kRows;
        std::vector<int64_t> ulen(m.N);
        parallel_for(nblk, [&](int64_t blk) {
            for (int64_t i = blk * kRows; i < std::min(m.N, (blk + 1) * kRows); ++i) {
                auto b = col.begin() + cnt[i], e = col.begin() + cnt[i + 1];
                std::sort(b, e);
                ulen[i] = std::unique(b, e) - b;
            }
        });
        op.csr_ptr.assign(m.N + 1, 0);
        for (int64_t i = 0; i < m.N; ++i) op.csr_ptr[i + 1] = op.csr_ptr[i] + ulen[i];
        op.csr_col.resize(op.csr_ptr[m.N]);
        parallel_for(nblk, [&](int64_t blk) {
            for (int64_t i = blk * kRows; i < std::min(m.N, (blk + 1) * kRows); ++i)
                std::copy(col.begin() + cnt[i], col.begin() + cnt[i] + ulen[i], op.csr_col.begin() + op.csr_ptr[i]);
        });
    }
    op.stats.t_plan_ms = ms_since(t0);
}

int64_t csr_slot(const fpde_op& op, int64_t row, int64_t col) {
    auto b = op.csr_col.begin() + op.csr_ptr[row], e = op.csr_col.begin() + op.csr_ptr[row + 1];
    auto it = std::lower_bound(b, e, (int32_t)col);
    if (it == e || *it != col) fail(FPDE_EINVAL, "internal: CSR slot missing");
    return it - op.csr_col.begin();
}

// contributions (slot, source index) sorted by slot -> ptr/idx
void contrib_csr(int64_t nslots, std::vector<std::pair<int64_t, int64_t>>& c, std::vector<int64_t>& ptr,
                 std::vector<int64_t>& idx) {
    sort_pairs(c, nslots);
    ptr.assign(nslots + 1, 0);
    idx.resize(c.size());
    for (size_t e = 0; e < c.size(); ++e) {
        ptr[c[e].first + 1]++;
        idx[e] = c[e].second;
    }
    for (int64_t i = 0; i < nslots; ++i) ptr[i + 1] += ptr[i];
}

// ------------------------------------------------------------------ device build

// HIP events around a build phase on the build stream (released by the destructor, also
// when the phase throws)
struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    explicit Timer(hipStream_t s) : st(s) {
        hipck(hipEventCreate(&a), "timer event");
        hipck(hipEventCreate(&b), "timer event");
        hipck(hipEventRecord(a, st), "timer record");
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    Timer(const Timer&) = delete;
    Timer& operator=(const Timer&) = delete;
    double stop() {
        hipck(hipEventRecord(b, st), "timer record");
        hipck(hipEventSynchronize(b), "timer sync");
        float ms = 0;
        hipck(hipEventElapsedTime(&ms, a, b), "timer elapsed");
        return ms;
    }
};

// Algebraic recompression of the far field (closing remark of Sec. 5.3): host QR and
// eigen-decompositions of the cluster weights, device weights and coupling projections.
void recompress(fpde_op& op, hipStream_t st) {
    auto t0 = std::chrono::steady_clock::now();
    const HostMesh& m = op.mesh;
    const int d = m.dim, p = op.opts.cheb_p, K = d == 2 ? p * p : p, F = op.F;
    const Tree& kt = op.kt;
    const int64_t N = m.N, ncl = kt.ncl, nfar = (int64_t)op.kfar.size(), nleaf = kt.nleaf();
    Arena& A = op.arena;
    std::vector<double> U((size_t)N * K), Es((size_t)ncl * d * p * p);
    hipck(hipMemcpyAsync(U.data(), op.d_U, U.size() * sizeof(double), hipMemcpyDeviceToHost, st), "U");
    hipck(hipMemcpyAsync(Es.data(), op.kdev.E, Es.size() * sizeof(double), hipMemcpyDeviceToHost, st), "E");
    hipck(hipStreamSynchronize(st), "rc download");
    const RcTree t{N, ncl, kt.first_leaf(), K, kt.beg.data(), kt.end.data()};
    std::vector<double> Ed;
    rc_dense_transfers(t, d, p, Es.data(), Ed);
    RcOrth o;
    rc_orthogonalize(t, U.data(), Ed, o);
    // C_s = R_s^T R_s per cluster; H_t on the device
    const size_t KK = (size_t)K * K;
    std::vector<double> C((size_t)ncl * KK, 0.0), H((size_t)ncl * KK);
    for (int64_t c = 0; c < ncl; ++c)
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j) {
                double v = 0.0;
                for (int l = 0; l < K; ++l) v += o.R[c * KK + (size_t)l * K + i] * o.R[c * KK + (size_t)l * K + j];
                C[c * KK + (size_t)i * K + j] = v;
            }
    double* d_Cw = A.upload(C, st);
    double* d_H = A.alloc<double>((int64_t)ncl * KK);
    hipck(launch_rc_weights(ncl, K, F, nfar, op.kdev.far_ptr, op.kdev.far_src, op.d_St, d_Cw, d_H, st), "rc weights");
    hipck(hipMemcpyAsync(H.data(), d_H, H.size() * sizeof(double), hipMemcpyDeviceToHost, st), "H");
    hipck(hipStreamSynchronize(st), "rc weights sync");
    RcOut out;
    const int r = rc_truncate(t, o, H, op.opts.recompress_tol, out);
    // new bases, transfers and coupling matrices
    op.rc.U = A.upload(out.U, st);
    op.rc.E = A.upload(out.E, st);
    double* d_P = A.upload(out.P, st);
    std::vector<int64_t> ftgt;
    ftgt.reserve(nfar);
    for (auto& pr : op.kfar) ftgt.push_back(pr.first);
    int64_t* d_ftgt = A.upload(ftgt, st);
    op.rc.St = A.alloc<double>((int64_t)F * nfar * r * r);
    hipck(launch_rc_project(ncl, K, r, F, nfar, d_ftgt, op.kdev.far_src, op.d_St, d_P, op.rc.St, st), "rc project");
    op.rc.Upad = A.alloc<double>(nleaf * op.cap * r);
    hipck(launch_pad_rows(nleaf, op.cap, r, op.d_leaf_beg, op.rc.U, op.kdev.perm, op.rc.Upad, op.d_perm_pad, st),
          "rc leaf slots");
    if (op.mixed) {
        op.rc.U32 = A.alloc<float>(N * r);
        op.rc.E32 = A.alloc<float>(ncl * r * r);
        op.rc.St32 = A.alloc<float>((int64_t)F * nfar * r * r);
        op.rc.Upad32 = A.alloc<float>(nleaf * op.cap * r);
        hipck(launch_to_float(N * r, op.rc.U, op.rc.U32, st), "to float");
        hipck(launch_to_float(ncl * r * r, op.rc.E, op.rc.E32, st), "to float");
        hipck(launch_to_float((int64_t)F * nfar * r * r, op.rc.St, op.rc.St32, st), "to float");
        hipck(launch_to_float(nleaf * op.cap * r, op.rc.Upad, op.rc.Upad32, st), "to float");
    }
    hipck(hipStreamSynchronize(st), "rc sync");   // host vectors of the uploads end with this scope
    A.release(d_Cw);
    A.release(d_H);
    A.release(d_P);
    A.release(d_ftgt);
    op.rc.on = true;
    op.rc.r = r;
    int rmin = K;
    double rsum = 0.0;
    for (int v : out.ranks) {
        rmin = std::min(rmin, v);
        rsum += v;
    }
    op.stats.k_rank_rc = r;
    op.stats.k_rank_rc_min = rmin;
    op.stats.k_rank_rc_mean = rsum / std::max<size_t>(1, out.ranks.size());
    op.stats.t_recompress_ms = ms_since(t0);
}

// s and sqrt(kappa) of every field at the nn cluster nodes, [F][nn], from the stencils
void node_fields(Arena& A, int64_t nn, int F, int64_t M, const std::vector<int64_t>& stn,
                 const std::vector<double>& stw, const double* d_s, const double* d_k, TreeDev& td, hipStream_t st) {
    int64_t* d_stn = A.upload(stn, st);
    double* d_stw = A.upload(stw, st);
    td.node_s = A.alloc<double>((int64_t)F * nn);
    td.node_k = A.alloc<double>((int64_t)F * nn);
    hipck(launch_node_fields(nn, F, M, d_stn, d_stw, d_s, d_k, td.node_s, td.node_k, st), "node fields");
    hipck(hipStreamSynchronize(st), "node fields sync");
    A.release(d_stn);
    A.release(d_stw);
}

void build_device(fpde_op& op) {
    const HostMesh& m = op.mesh;
    const int d = m.dim, F = op.F, p = op.opts.cheb_p, k = d == 2 ? p * p : p;
    Arena& A = op.arena;
    A.limit = op.opts.max_device_bytes;
    hipStream_t st = op.stream;
    const int64_t nq = op.Q.nq;
    const int nqe = op.Q.nqe;
    auto t_all = std::chrono::steady_clock::now();

    // ---- uploads
    op.d_X = A.upload(m.X, st);
    op.d_C = A.upload(m.C, st);
    op.d_cint = A.upload(m.interior, st);
    double* d_s = A.upload(op.s, st);
    double* d_k = A.upload(op.kappa, st);
    op.adj.s = d_s;
    op.adj.k = d_k;
    double* d_qx = A.upload(op.Q.x, st);
    op.d_qw = A.upload(op.Q.w, st);
    uint8_t* d_qint = A.upload(op.Q.q_int, st);
    op.d_lam = A.upload(op.er.lam, st);
    op.d_nc_ptr = A.upload(op.ncs.ptr, st);
    op.d_nc_cell = A.upload(op.ncs.cell, st);
    op.d_nc_slot = A.upload(op.ncs.slot, st);
    double* d_qs = A.alloc<double>((int64_t)F * nq);
    double* d_qk = A.alloc<double>((int64_t)F * nq);
    hipck(launch_quad_fields(d, m.nc, nqe, op.d_C, op.d_lam, F, m.M, d_s, d_k, d_qs, d_qk, st), "quad_fields");
    const int64_t nnz = (int64_t)op.csr_col.size();
    op.d_csr_ptr = A.upload(op.csr_ptr, st);
    op.d_csr_col = A.upload(op.csr_col, st);

    // ---- singular near field B (Sec. 4)
    {
        Timer tm(st);
        const int64_t np = (int64_t)op.pairs.size();
        std::vector<int32_t> prow(np * 8, 0);
        // every pair's (CSR slot of B, local entry) contributions, at offsets counted first
        std::vector<int64_t> coff(np + 1, 0);
        std::vector<std::pair<int64_t, int64_t>> contrib;
        constexpr int64_t kBlk = 4096;
        const int64_t nblk = (np + kBlk - 1) / kBlk;
        for (int pass = 0; pass < 2; ++pass) {
            parallel_for(nblk, [&](int64_t blk) {
                int32_t dofs[5];
                for (int64_t gp = blk * kBlk; gp < std::min(np, (blk + 1) * kBlk); ++gp) {
                    const Pair& pr = op.pairs[op.pair_order[gp]];
                    const int nd = pair_dofs(m, pr, dofs);
                    if (pass == 0) {
                        prow[gp * 8] = pr.kind;
                        for (int a = 0; a < 6; ++a) prow[gp * 8 + 1 + a] = pr.v[a];
                        if (d == 1) {   // 1D rows: cell0 (v0, v1), cell1 (v3, v4) -> layout slots 1,2 and 4,5
                            prow[gp * 8 + 1] = pr.v[0];
                            prow[gp * 8 + 2] = pr.v[1];
                            prow[gp * 8 + 4] = pr.v[3];
                            prow[gp * 8 + 5] = pr.v[4];
                        }
                        int ni = 0;
                        for (int a = 0; a < nd; ++a) ni += dofs[a] < m.N;
                        coff[gp + 1] = (int64_t)ni * ni;
                        continue;
                    }
                    int64_t o = coff[gp];
                    for (int a = 0; a < nd; ++a) {
                        if (dofs[a] >= m.N) continue;
                        for (int b = 0; b < nd; ++b) {
                            if (dofs[b] >= m.N) continue;
                            int lo = std::min(a, b), hi = std::max(a, b);
                            contrib[o++] = {csr_slot(op, op.pos_of_dof[dofs[a]], op.pos_of_dof[dofs[b]]),
                                            gp * 25 + lo * 5 + hi};
                        }
                    }
                }
            });
            if (pass == 0) {
                for (int64_t gp = 0; gp < np; ++gp) coff[gp + 1] += coff[gp];
                contrib.resize(coff[np]);
            }
        }
        std::vector<double> g(op.opts.nq_sing), w(op.opts.nq_sing);
        gauss_legendre01(op.opts.nq_sing, g.data(), w.data());
        double* d_g = A.upload(g, st);
        double* d_w = A.upload(w, st);
        int32_t* d_pairs = A.upload(prow, st);
        double* d_loc = A.alloc<double>((int64_t)F * np * 25);
        hipck(hipMemsetAsync(d_loc, 0, sizeof(double) * F * np * 25, st), "memset");
        hipck(launch_singular(d, np, d_pairs, op.d_X, m.M, F, d_s, d_k, op.opts.a_scale, op.opts.s_bar,
                              op.opts.nq_sing, d_g, d_w, d_loc, st), "singular");
        std::vector<int64_t> cptr, cidx;
        contrib_csr(nnz, contrib, cptr, cidx);
        int64_t* d_cptr = A.upload(cptr, st);
        int64_t* d_cidx = A.upload(cidx, st);
        op.d_B = A.alloc<double>((int64_t)F * nnz);
        hipck(launch_segsum(nnz, d_cptr, d_cidx, nullptr, F, d_loc, np * 25, op.d_B, st), "segsum B");
        hipck(hipStreamSynchronize(st), "singular sync");
        A.release(d_loc); A.release(d_cptr); A.release(d_cidx);
        // adjoint: node -> (pair, slot) over the 6 cell-vertex slots of every pair
        {
            std::vector<int64_t> sn(np * 6);
            std::vector<double> sw(np * 6, 1.0);
            for (int64_t gp = 0; gp < np; ++gp)
                for (int a = 0; a < 6; ++a) {
                    const bool used = d == 2 || (a % 3) < 2;   // 1D rows use slots 0,1 and 3,4
                    sn[gp * 6 + a] = used ? prow[gp * 8 + 1 + a] : -1;
                }
            std::vector<int64_t> sp, si;
            std::vector<double> swt;
            node_csr(m.M, sn, sw, 1, sp, si, swt);
            for (auto& x : si) x = (x / 6) * 12 + (x % 6);   // entry -> pair * 12 + slot
            op.adj.slot_ptr = A.upload(sp, st);
            op.adj.slot_idx = A.upload(si, st);
            op.adj.pairs = d_pairs;
            op.adj.g = d_g;
            op.adj.w = d_w;
        }
        op.stats.t_singular_ms = tm.stop();
    }

    // point location in the mesh, for the Chebyshev nodes of both trees
    Locator loc;
    loc.build(m);

    // ---- density rho at every interior quadrature point (Sec. 6.2) and M (Sec. 6.1)
    {
        Timer tm(st);
        const Tree& rt = op.rt;
        std::vector<double> axes, stw;
        std::vector<int64_t> stn;
        cluster_nodes(op, rt, loc, axes, stn, stw);
        {
            std::vector<int64_t> sp, si;
            std::vector<double> swt;
            node_csr(m.M, stn, stw, 3, sp, si, swt);
            op.adj.rst_ptr = A.upload(sp, st);
            op.adj.rst_idx = A.upload(si, st);
            op.adj.rst_w = A.upload(swt, st);
        }
        std::vector<int64_t> fptr, fsrc, nptr, nsrc;
        far_csr(rt, op.rfar, fptr, fsrc);
        // near by leaf index
        nptr.assign(rt.nleaf() + 1, 0);
        for (auto& pr : op.rnear) nptr[pr.first - rt.first_leaf() + 1]++;
        for (int64_t i = 0; i < rt.nleaf(); ++i) nptr[i + 1] += nptr[i];
        nsrc.resize(op.rnear.size());
        for (size_t e = 0; e < op.rnear.size(); ++e) nsrc[e] = op.rnear[e].second;
        TreeDev td;
        td.beg = A.upload(rt.beg, st);
        td.end = A.upload(rt.end, st);
        td.perm = A.upload(rt.perm, st);
        td.axes = A.upload(axes, st);
        node_fields(A, rt.ncl * k, F, m.M, stn, stw, d_s, d_k, td, st);
        td.far_ptr = A.upload(fptr, st);
        td.far_src = A.upload(fsrc, st);
        td.E = A.alloc<double>(rt.ncl * d * p * p);
        int64_t* d_nptr = A.upload(nptr, st);
        int64_t* d_nsrc = A.upload(nsrc, st);
        H2Tree h = make_h2(rt, td, p);
        hipck(launch_transfer(h, td.E, st), "transfer rho");
        double* xh = A.alloc<double>((int64_t)F * rt.ncl * k);
        double* yh = A.alloc<double>((int64_t)F * rt.ncl * k);
        op.d_rho = A.alloc<double>((int64_t)F * nq);
        hipck(hipMemsetAsync(op.d_rho, 0, sizeof(double) * F * nq, st), "memset rho");
        hipck(launch_rho_moments(h, td.perm, d_qx, op.d_qw, nq, F, xh, st), "rho moments");
        for (int lev = rt.L - 1; lev >= 0; --lev) hipck(launch_up_level(h, lev, F, 1, xh, st), "rho up");
        hipck(launch_coupling(h, F, 1, 1.0, op.opts.a_scale, xh, yh, st), "rho coupling");
        for (int lev = 0; lev < rt.L; ++lev) hipck(launch_down_level(h, lev, F, 1, yh, st), "rho down");
        hipck(launch_rho_eval(h, td.perm, d_qx, d_qint, nq, F, yh, op.d_rho, st), "rho eval");
        hipck(launch_rho_near(h, td.perm, d_nptr, d_nsrc, d_qx, op.d_qw, d_qs, d_qk, d_qint, nqe, op.d_C, m.nc,
                              nq, F, op.opts.a_scale, op.d_rho, st), "rho near");
        if (m.R > 0.0)
            hipck(launch_rho_exterior(d, nq, d_qx, d_qs, d_qk, d_qint, F, m.R, op.opts.s_exterior,
                                      std::sqrt(op.opts.kappa_exterior), op.opts.a_scale, op.opts.n_theta,
                                      op.d_rho, st), "rho exterior");
        hipck(hipStreamSynchronize(st), "rho sync");
        A.release(xh);
        A.release(yh);
        A.release(d_nptr);
        A.release(d_nsrc);
        // the density tree stays for the adjoint, with the pair lists closed under
        // transposition: the partition leaves out targets without interior points,
        // the adjoint's target-major sums need those pairs too
        op.adj.rdev = td;
        {
            auto closure = [&rt](std::vector<std::pair<int64_t, int64_t>> v) {
                const size_t n = v.size();
                for (size_t i = 0; i < n; ++i) v.push_back({v[i].second, v[i].first});
                sort_pairs(v, rt.ncl);
                v.erase(std::unique(v.begin(), v.end()), v.end());
                return v;
            };
            const auto afar = closure(op.rfar), anear = closure(op.rnear);
            std::vector<int64_t> ap, as, bp(rt.nleaf() + 1, 0), bs;
            far_csr(rt, afar, ap, as);
            for (auto& pr : anear) bp[pr.first - rt.first_leaf() + 1]++;
            for (int64_t i = 0; i < rt.nleaf(); ++i) bp[i + 1] += bp[i];
            for (auto& pr : anear) bs.push_back(pr.second);
            op.adj.rdev.far_ptr = A.upload(ap, st);
            op.adj.rdev.far_src = A.upload(as, st);
            op.adj.rnear_ptr = A.upload(bp, st);
            op.adj.rnear_src = A.upload(bs, st);
            A.release(td.far_ptr);
            A.release(td.far_src);
        }
        op.stats.t_rho_ms = tm.stop();

        Timer tm2(st);
        std::vector<int64_t> icells;
        for (int64_t c = 0; c < m.nc; ++c)
            if (m.interior[c]) icells.push_back(c);
        std::vector<std::pair<int64_t, int64_t>> contrib;
        for (size_t ci = 0; ci < icells.size(); ++ci) {
            int64_t c = icells[ci];
            for (int a = 0; a <= d; ++a) {
                int32_t va = m.v(a, c);
                if (va >= m.N) continue;
                for (int b = 0; b <= d; ++b) {
                    int32_t vb = m.v(b, c);
                    if (vb >= m.N) continue;
                    int lo = std::min(a, b), hi = std::max(a, b);
                    contrib.push_back({csr_slot(op, op.pos_of_dof[va], op.pos_of_dof[vb]), (int64_t)ci * 9 + lo * 3 + hi});
                }
            }
        }
        int64_t* d_ic = A.upload(icells, st);
        double* d_ml = A.alloc<double>((int64_t)F * icells.size() * 9);
        hipck(launch_mass_local(d, (int64_t)icells.size(), d_ic, nqe, op.d_lam, op.d_qw, op.d_rho, nq, F, d_ml, st),
              "mass local");
        std::vector<int64_t> cptr, cidx;
        contrib_csr(nnz, contrib, cptr, cidx);
        int64_t* d_cptr = A.upload(cptr, st);
        int64_t* d_cidx = A.upload(cidx, st);
        op.d_M = A.alloc<double>((int64_t)F * nnz);
        hipck(launch_segsum(nnz, d_cptr, d_cidx, nullptr, F, d_ml, (int64_t)icells.size() * 9, op.d_M, st),
              "segsum M");
        op.d_BM = A.alloc<double>((int64_t)F * nnz);
        hipck(launch_axpby((int64_t)F * nnz, 1.0, op.d_B, 1.0, op.d_M, op.d_BM, st), "B+M");
        hipck(hipStreamSynchronize(st), "mass sync");
        A.release(d_ic); A.release(d_ml); A.release(d_cptr); A.release(d_cidx);
        op.stats.t_mass_ms = tm2.stop();
    }

    // ---- K~: bases, transfers, near leaf blocks (Sec. 5)
    {
        Timer tm(st);
        const Tree& kt = op.kt;
        std::vector<double> axes, stw;
        std::vector<int64_t> stn;
        cluster_nodes(op, kt, loc, axes, stn, stw);
        {
            std::vector<int64_t> sp, si;
            std::vector<double> swt;
            node_csr(m.M, stn, stw, 3, sp, si, swt);
            op.adj.kst_ptr = A.upload(sp, st);
            op.adj.kst_idx = A.upload(si, st);
            op.adj.kst_w = A.upload(swt, st);
        }
        std::vector<int64_t> fptr, fsrc;
        far_csr(kt, op.kfar, fptr, fsrc);
        TreeDev& td = op.kdev;
        td.beg = A.upload(kt.beg, st);
        td.end = A.upload(kt.end, st);
        td.perm = A.upload(kt.perm, st);
        td.axes = A.upload(axes, st);
        node_fields(A, kt.ncl * k, F, m.M, stn, stw, d_s, d_k, td, st);
        td.far_ptr = A.upload(fptr, st);
        td.far_src = A.upload(fsrc, st);
        td.E = A.alloc<double>(kt.ncl * d * p * p);
        H2Tree h = make_h2(kt, td, p);
        hipck(launch_transfer(h, td.E, st), "transfer K");
        op.d_U = A.alloc<double>(m.N * k);
        hipck(launch_basis_n(h, m.N, td.perm, op.d_nc_ptr, op.d_nc_cell, op.d_nc_slot, nqe, d_qx, op.d_qw,
                             op.d_lam, nq, op.d_U, st), "basis");
        {
            std::vector<int64_t> ftgt;
            for (auto& pr : op.kfar) ftgt.push_back(pr.first);
            int64_t* d_ftgt = A.upload(ftgt, st);
            op.d_St = A.alloc<double>((int64_t)F * op.kfar.size() * k * k);
            hipck(launch_coupling_store(h, (int64_t)op.kfar.size(), d_ftgt, F, -2.0, op.opts.a_scale, op.d_St, st),
                  "coupling store");
            hipck(hipStreamSynchronize(st), "coupling sync");
            A.release(d_ftgt);
        }
        hipck(hipStreamSynchronize(st), "basis sync");
        op.stats.t_bases_ms = tm.stop();

        Timer tm2(st);
        // leaf patches and per-row cell lists
        const int64_t nleaf = kt.nleaf();
        std::vector<int64_t> leaf_beg(nleaf + 1);
        op.cap = 0;
        for (int64_t li = 0; li < nleaf; ++li) {
            leaf_beg[li] = kt.beg[kt.first_leaf() + li];
            op.cap = std::max(op.cap, kt.end[kt.first_leaf() + li] - kt.beg[kt.first_leaf() + li]);
        }
        leaf_beg[nleaf] = m.N;
        std::vector<int64_t> patch_ptr(nleaf + 1, 0), patch_cell, row_ptr(m.N + 1, 0);
        std::vector<int32_t> row_lcell;
        std::vector<int8_t> row_slot;
        int64_t max_patch = 0;
        for (int64_t li = 0; li < nleaf; ++li) {
            std::vector<int64_t> cl;
            for (int64_t j = leaf_beg[li]; j < leaf_beg[li + 1]; ++j) {
                int64_t v = kt.perm[j];
                for (int64_t e = op.ncs.ptr[v]; e < op.ncs.ptr[v + 1]; ++e) cl.push_back(op.ncs.cell[e]);
            }
            std::sort(cl.begin(), cl.end());
            cl.erase(std::unique(cl.begin(), cl.end()), cl.end());
            max_patch = std::max<int64_t>(max_patch, cl.size());
            for (int64_t j = leaf_beg[li]; j < leaf_beg[li + 1]; ++j) {
                int64_t v = kt.perm[j];
                for (int64_t e = op.ncs.ptr[v]; e < op.ncs.ptr[v + 1]; ++e) {
                    int64_t lc = std::lower_bound(cl.begin(), cl.end(), op.ncs.cell[e]) - cl.begin();
                    row_lcell.push_back((int32_t)lc);
                    row_slot.push_back(op.ncs.slot[e]);
                }
                row_ptr[j + 1] = (int64_t)row_lcell.size();
            }
            patch_cell.insert(patch_cell.end(), cl.begin(), cl.end());
            patch_ptr[li + 1] = (int64_t)patch_cell.size();
        }
        std::vector<int64_t> tgt, src, near_ptr(nleaf + 1, 0), near_src_leaf;
        for (auto& pr : op.knear) {
            tgt.push_back(pr.first);
            src.push_back(pr.second);
            near_ptr[pr.first - kt.first_leaf() + 1]++;
            near_src_leaf.push_back(pr.second - kt.first_leaf());
        }
        for (int64_t i = 0; i < nleaf; ++i) near_ptr[i + 1] += near_ptr[i];
        NearPlan np{};
        np.npairs = (int64_t)op.knear.size();
        np.cap = op.cap;
        np.tgt = A.upload(tgt, st);
        np.src = A.upload(src, st);
        np.patch_ptr = A.upload(patch_ptr, st);
        np.patch_cell = A.upload(patch_cell, st);
        np.row_ptr = A.upload(row_ptr, st);
        np.row_lcell = A.upload(row_lcell, st);
        np.row_slot = A.upload(row_slot, st);
        np.nc_ptr = op.d_nc_ptr;
        np.nc_cell = op.d_nc_cell;
        np.nc_slot = op.d_nc_slot;
        std::vector<int64_t> own, mirror;
        if (symmetric_pairs(op.knear)) {
            std::vector<std::pair<std::pair<int64_t, int64_t>, int64_t>> key(op.knear.size());
            for (size_t e = 0; e < op.knear.size(); ++e) key[e] = {op.knear[e], (int64_t)e};
            std::sort(key.begin(), key.end());
            for (size_t e = 0; e < op.knear.size(); ++e) {
                const auto& pr = op.knear[e];
                if (pr.first > pr.second) continue;
                auto it = std::lower_bound(key.begin(), key.end(),
                                           std::make_pair(std::make_pair(pr.second, pr.first), (int64_t)-1));
                own.push_back((int64_t)e);
                mirror.push_back(it->second);
            }
        } else {
            for (size_t e = 0; e < op.knear.size(); ++e) {
                own.push_back((int64_t)e);
                mirror.push_back((int64_t)e);
            }
        }
        np.nown = (int64_t)own.size();
        np.own = A.upload(own, st);
        np.mirror = A.upload(mirror, st);
        op.d_near = A.alloc<double>((int64_t)F * np.npairs * op.cap * op.cap);
        hipck(launch_near_blocks_lds(h, np, max_patch, td.perm, op.d_C, nqe, m.nc, d_qx, op.d_qw, d_qs, d_qk,
                                     op.d_lam, nq, F, op.opts.a_scale, op.d_near, st), "near blocks");
        hipck(hipStreamSynchronize(st), "near sync");
        op.d_leaf_beg = A.upload(leaf_beg, st);
        op.d_near_ptr = A.upload(near_ptr, st);
        op.d_near_src = A.upload(near_src_leaf, st);
        std::vector<int64_t> pcols_ptr(nleaf + 1, 0), poff(nleaf + 1, 0), pstride(nleaf);
        std::vector<int32_t> pcols;
        {   // panels: columns of each leaf = concatenated source leaves of its near pairs
            std::vector<int64_t> pcol_off(np.npairs);
            for (int64_t li = 0; li < nleaf; ++li) {
                int64_t ncol = 0;
                for (int64_t e = near_ptr[li]; e < near_ptr[li + 1]; ++e) {
                    const int64_t ls_ = near_src_leaf[e];
                    pcol_off[e] = ncol;
                    for (int64_t j = leaf_beg[ls_]; j < leaf_beg[ls_ + 1]; ++j) pcols.push_back((int32_t)kt.perm[j]);
                    ncol += leaf_beg[ls_ + 1] - leaf_beg[ls_];
                }
                pcols_ptr[li + 1] = (int64_t)pcols.size();
                pstride[li] = (ncol + 3) / 4 * 4;
                poff[li + 1] = poff[li] + op.cap * pstride[li];
                op.panel_max_stride = std::max(op.panel_max_stride, pstride[li]);
            }
            op.panel_total = poff[nleaf];
            int64_t* d_pcol_off = A.upload(pcol_off, st);
            op.d_poff = A.upload(poff, st);
            op.d_pstride = A.upload(pstride, st);
            op.d_pcols_ptr = A.upload(pcols_ptr, st);
            op.d_pcols = A.upload(pcols, st);
            {
                std::vector<int32_t> pad((size_t)nleaf * op.panel_max_stride, -1);
                for (int64_t li = 0; li < nleaf; ++li)
                    std::copy(pcols.begin() + pcols_ptr[li], pcols.begin() + pcols_ptr[li + 1],
                              pad.begin() + li * op.panel_max_stride);
                op.d_pcols_pad = A.upload(pad, st);
            }
            op.d_panel = A.alloc<double>((int64_t)F * op.panel_total);
            hipck(launch_pack_panels(nleaf, op.cap, np.npairs, op.d_near_ptr, op.d_near_src, op.d_leaf_beg, d_pcol_off,
                                     op.d_poff, op.d_pstride, op.d_pcols_ptr, op.d_near, F, op.d_panel, st), "pack");
            hipck(hipStreamSynchronize(st), "pack sync");
            A.release(d_pcol_off);
            A.release(op.d_near);   // every apply reads the panels
            op.d_near = nullptr;
        }
        for (void* q : {(void*)np.tgt, (void*)np.src, (void*)np.row_ptr, (void*)np.row_lcell, (void*)np.row_slot,
                        (void*)np.own, (void*)np.mirror})
            A.release(q);
        {   // adjoint of the near blocks: patches, leaf of every dof, leaves whose patch holds a cell
            op.adj.patch_ptr = (int64_t*)np.patch_ptr;
            op.adj.patch_cell = (int64_t*)np.patch_cell;
            std::vector<int32_t> lon(m.M, -1);
            for (int64_t li = 0; li < nleaf; ++li)
                for (int64_t j = leaf_beg[li]; j < leaf_beg[li + 1]; ++j) lon[kt.perm[j]] = (int32_t)li;
            std::vector<int64_t> icells, slot_of_cell(m.nc, -1);
            for (int64_t c = 0; c < m.nc; ++c)
                if (m.interior[c]) {
                    slot_of_cell[c] = (int64_t)icells.size();
                    icells.push_back(c);
                }
            std::vector<std::pair<int64_t, int32_t>> cl;
            for (int64_t li = 0; li < nleaf; ++li)
                for (int64_t e = patch_ptr[li]; e < patch_ptr[li + 1]; ++e)
                    if (slot_of_cell[patch_cell[e]] >= 0) cl.push_back({slot_of_cell[patch_cell[e]], (int32_t)li});
            std::sort(cl.begin(), cl.end());
            std::vector<int64_t> clp(icells.size() + 1, 0);
            std::vector<int32_t> cll(cl.size());
            for (size_t i = 0; i < cl.size(); ++i) {
                clp[cl[i].first + 1]++;
                cll[i] = cl[i].second;
            }
            for (size_t i = 0; i < icells.size(); ++i) clp[i + 1] += clp[i];
            op.adj.n_icells = (int64_t)icells.size();
            op.adj.icells = A.upload(icells, st);
            op.adj.cell_leaf_ptr = A.upload(clp, st);
            op.adj.cell_leaf = A.upload(cll, st);
            op.adj.leaf_of_node = A.upload(lon, st);
            op.adj.ok = true;
            if (!symmetric_pairs(op.knear) || !symmetric_pairs(op.kfar)) {
                op.adj.ok = false;
                op.adj.why = "the near/far partitions are not symmetric";
            } else if (nqe > 16) {
                op.adj.ok = false;
                op.adj.why = "more than 16 quadrature points per cell (nq_reg)";
            } else if (k > 64) {
                op.adj.ok = false;
                op.adj.why = "more than 64 Chebyshev nodes per cluster";
            }
        }
        op.stats.t_near_blocks_ms = tm2.stop();
        std::vector<int32_t> cdof(op.csr_col.size());
        for (size_t e = 0; e < cdof.size(); ++e) cdof[e] = (int32_t)kt.perm[op.csr_col[e]];
        op.d_csr_col_dof = A.upload(cdof, st);
        {   // ELL form of B + M by leaf slot, entries in CSR order (rows are never empty: the diagonal
            // is always stored); kept only while the padding costs
            // at most half again the CSR's entries
            int64_t w = 0;
            for (int64_t i = 0; i < m.N; ++i) w = std::max(w, op.csr_ptr[i + 1] - op.csr_ptr[i]);
            w = (w + 3) / 4 * 4;
            const int64_t nslot = nleaf * op.cap;
            bool empty_row = false;
            for (int64_t i = 0; i < m.N; ++i) empty_row = empty_row || op.csr_ptr[i + 1] == op.csr_ptr[i];
            if (w > 0 && !empty_row && nslot * w <= nnz + nnz / 2 + 4 * nslot) {
                std::vector<int32_t> ecol((size_t)(nslot * w), -1);
                std::vector<int64_t> esrc((size_t)(nslot * w), -1);
                for (int64_t li = 0; li < nleaf; ++li)
                    for (int64_t row = leaf_beg[li]; row < leaf_beg[li + 1]; ++row) {
                        const int64_t o = (li * op.cap + row - leaf_beg[li]) * w;
                        for (int64_t e = op.csr_ptr[row]; e < op.csr_ptr[row + 1]; ++e) {
                            ecol[o + e - op.csr_ptr[row]] = cdof[e];
                            esrc[o + e - op.csr_ptr[row]] = e;
                        }
                        // padding: the row's first column with the value 0 (a kernel may read
                        // every entry of a row without a test)
                        for (int64_t e = op.csr_ptr[row + 1] - op.csr_ptr[row]; e < w; ++e)
                            ecol[o + e] = cdof[op.csr_ptr[row]];
                    }
                op.ell_w = (int)w;
                op.d_ell_col = A.upload(ecol, st);
                int64_t* d_esrc = A.upload(esrc, st);
                op.d_ell_val = A.alloc<double>((int64_t)F * nslot * w);
                hipck(launch_ell_values(nslot * w, F, nnz, d_esrc, op.d_BM, op.d_ell_val, st), "ELL values");
                hipck(hipStreamSynchronize(st), "ELL sync");
                A.release(d_esrc);
            }
        }
        // mixed precision: the panel offset of every entry of B + M (touching pairs are near
        // pairs, so each lies in its row's panel); the several-rhs FP32 panels hold B + M too
        std::vector<int64_t> bm_off;
        if (op.mixed) {
            bm_off.assign(nnz, -1);
            std::vector<int64_t> colmap(m.N, -1);
            for (int64_t li = 0; li < nleaf; ++li) {
                for (int64_t c = pcols_ptr[li]; c < pcols_ptr[li + 1]; ++c) colmap[pcols[c]] = c - pcols_ptr[li];
                for (int64_t t = leaf_beg[li]; t < leaf_beg[li + 1]; ++t)
                    for (int64_t e = op.csr_ptr[t]; e < op.csr_ptr[t + 1]; ++e) {
                        const int64_t cp = colmap[kt.perm[op.csr_col[e]]];
                        if (cp < 0) fail(FPDE_EINVAL, "an entry of B + M outside its row's near panel");
                        bm_off[e] = poff[li] + (t - leaf_beg[li]) * pstride[li] + cp;
                    }
                for (int64_t c = pcols_ptr[li]; c < pcols_ptr[li + 1]; ++c) colmap[pcols[c]] = -1;
            }
        }
        if (op.opts.flags & FPDE_FLAG_JACOBI) {
            // 1 / diag(A_h): the diagonal entry of B + M plus the leaf self-block entry of the
            // near panel (far blocks never hold a diagonal entry)
            std::vector<int64_t> bm_idx(m.N, -1), p_idx(m.N, -1);
            for (int64_t li = 0; li < nleaf; ++li)
                for (int64_t t = leaf_beg[li]; t < leaf_beg[li + 1]; ++t) {
                    const int64_t dof = kt.perm[t];
                    for (int64_t e = op.csr_ptr[t]; e < op.csr_ptr[t + 1]; ++e)
                        if (op.csr_col[e] == t) bm_idx[dof] = e;
                    for (int64_t c = pcols_ptr[li]; c < pcols_ptr[li + 1]; ++c)
                        if (pcols[c] == dof) p_idx[dof] = poff[li] + (t - leaf_beg[li]) * pstride[li] + (c - pcols_ptr[li]);
                }
            for (int64_t i = 0; i < m.N; ++i)
                if (bm_idx[i] < 0 || p_idx[i] < 0) fail(FPDE_EINVAL, "Jacobi: no diagonal entry for a dof");
            int64_t* d_bi = A.upload(bm_idx, st);
            int64_t* d_pi = A.upload(p_idx, st);
            op.d_dinv = A.alloc<double>((int64_t)F * m.N);
            hipck(launch_jacobi_diag(m.N, F, nnz, d_bi, op.d_BM, op.panel_total, d_pi, op.d_panel, op.d_dinv, st),
                  "Jacobi diagonal");
            hipck(hipStreamSynchronize(st), "Jacobi sync");   // bm_idx, p_idx end here
            A.release(d_bi);
            A.release(d_pi);
        }
        // launch plans: the one-launch upsweep of the single-vector apply (per
        // precision) and the subtree-root level of the multi-RHS far chain.
        // FPDE_MAX_SUBTREE_DEPTH caps the subtree depths (exercises the deep
        // ticket chains and top sweeps on small trees).
        int max_depth = kt.L;
        if (const char* env = std::getenv("FPDE_MAX_SUBTREE_DEPTH"))
            max_depth = std::max(0, std::min(max_depth, std::atoi(env)));
        // heap id c sits on level floor(log2(c + 1))
        auto level_of = [](int64_t c) {
            int lev = 0;
            while ((int64_t(2) << lev) - 1 <= c) ++lev;
            return lev;
        };
        int lmin = kt.L;   // shallowest far source
        for (auto& pr : op.kfar) lmin = std::min(lmin, level_of(pr.second));
        {   // far targets in heap order; per leaf, the targets on its root path
            std::vector<char> is_tgt(kt.ncl, 0);
            for (auto& pr : op.kfar) is_tgt[pr.first] = 1;
            std::vector<int64_t> tg;
            int ltop = kt.L;
            for (int64_t c = 0; c < kt.ncl; ++c)
                if (is_tgt[c]) {
                    tg.push_back(c);
                    ltop = std::min(ltop, level_of(c));
                }
            op.far_plan.ntgt = (int64_t)tg.size();
            op.far_plan.ltop = ltop;
            op.far_plan.tgt = tg.empty() ? nullptr : A.upload(tg, st);
            hipck(hipStreamSynchronize(st), "far plan upload");   // tg ends here
            // z^ of the one-vector apply: only targets are ever written, the rest stays zero
            op.d_zh = A.alloc<double>((int64_t)F * kt.ncl * k);
            hipck(hipMemsetAsync(op.d_zh, 0, sizeof(double) * F * kt.ncl * k, st), "zh");
        }
        {   // far list of the one-vector apply: its upsweep computes whole subtrees of
            // depth d0 per block, down from level lr = L - d0, without any exchange
            // between blocks.  A far source above lr moves down at most kMoveDown
            // levels to its descendants (coupling matrices S M_r^T, built on the
            // device); the ticket chain of the upsweep covers what is left above.
            constexpr int kMoveDown = 3;
            const int d0 = std::min(plan_up_tree(h, op.cap, lmin, 0).d0, max_depth);
            const int lr = kt.L - d0;
            const int64_t nfar = (int64_t)op.kfar.size();
            std::vector<int64_t> orig1, src1, fptr1(kt.ncl + 1, 0);
            std::vector<int32_t> dep1;
            int lstar = lr;   // the upsweep chain reaches this level
            for (int64_t e = 0; e < nfar; ++e) {
                const int64_t s = op.kfar[e].second;
                const int ls = level_of(s);
                const int lt = ls >= lr ? ls : std::min(lr, ls + kMoveDown);
                const int dd = lt - ls;
                lstar = std::min(lstar, lt);
                const int64_t first = ((s + 1) << dd) - 1;
                for (int64_t q = 0; q < (int64_t(1) << dd); ++q) {
                    orig1.push_back(e);
                    src1.push_back(first + q);
                    dep1.push_back(dd);
                }
                fptr1[op.kfar[e].first + 1] += int64_t(1) << dd;
            }
            for (int64_t c = 0; c < kt.ncl; ++c) fptr1[c + 1] += fptr1[c];
            op.nfar1 = (int64_t)src1.size();
            {   // coupling chunks: at most one pair per slot of a 512-thread block
                const int64_t cs = 512 / (k <= 32 ? 32 : 64);   // at most kChunkWords - 4
                std::vector<int64_t> ck;
                for (int64_t c = 0; c < kt.ncl; ++c) {
                    const int64_t p0 = fptr1[c], p1 = fptr1[c + 1];
                    if (p1 == p0) continue;
                    const int64_t nch = (p1 - p0 + cs - 1) / cs;
                    for (int64_t j = 0; j < nch; ++j) {
                        const int64_t e0 = p0 + j * cs, e1 = std::min(p1, p0 + (j + 1) * cs);
                        ck.insert(ck.end(), {c, e0, e1, (j << 32) | nch});
                        for (int64_t q = 0; q < kChunkWords - 4; ++q) ck.push_back(e0 + q < e1 ? src1[e0 + q] : 0);
                    }
                }
                op.far_plan.nchunks = (int64_t)ck.size() / kChunkWords;
                op.far_plan.chunks = A.upload(ck, st);
                op.far_plan.ctk = A.alloc<unsigned int>((int64_t)F * kt.ncl);
                hipck(hipMemsetAsync(op.far_plan.ctk, 0, sizeof(unsigned int) * F * kt.ncl, st), "coupling tickets");
                op.d_zp = A.alloc<double>((int64_t)F * std::max<int64_t>(1, op.far_plan.nchunks) * k);
                hipck(hipStreamSynchronize(st), "chunk upload");   // ck ends here
            }
            op.d_far1_ptr = A.upload(fptr1, st);
            op.d_far1_src = A.upload(src1, st);
            int64_t* d_orig = A.upload(orig1, st);
            int32_t* d_dep = A.upload(dep1, st);
            op.d_St1 = A.alloc<double>((int64_t)F * op.nfar1 * k * k);
            hipck(launch_expand_coupling(h, op.nfar1, d_orig, op.d_far1_src, d_dep, F, nfar, op.d_St, op.d_St1, st),
                  "moved-down coupling");
            hipck(hipStreamSynchronize(st), "moved-down coupling sync");
            A.release(d_orig);
            A.release(d_dep);
            for (int pr = 0; pr < 2; ++pr) {
                UpPlan u = plan_up_tree(h, op.cap, lstar, pr);
                u.d0 = d0;
                u.ds = std::max(1, std::min(u.ds, max_depth));
                op.up[pr] = u;
            }
        }
        op.ls2 = kt.L;
        while (op.ls2 > 0 && !multi_fits(h, op.ls2, 1)) --op.ls2;
        // bases and output indices by leaf slot for the one-vector output kernel
        op.d_Upad = A.alloc<double>(kt.nleaf() * op.cap * k);
        op.far_plan.perm_pad = op.d_perm_pad = A.alloc<int64_t>(kt.nleaf() * op.cap);
        hipck(launch_pad_rows(kt.nleaf(), op.cap, k, op.d_leaf_beg, op.d_U, op.kdev.perm, op.d_Upad, op.d_perm_pad, st),
              "leaf slots");
        op.d_tickets = A.alloc<unsigned int>((int64_t)F * kt.ncl);
        hipck(hipMemsetAsync(op.d_tickets, 0, sizeof(unsigned int) * F * kt.ncl, st), "tickets");
        if (op.mixed) {   // FP32 copies of the bases, transfers, coupling matrices and panels
            const int64_t nU = m.N * k, nE = kt.ncl * (int64_t)d * p * p, nS = (int64_t)F * op.kfar.size() * k * k;
            op.f32.U = A.alloc<float>(nU);
            op.f32.E = A.alloc<float>(nE);
            op.f32.St = A.alloc<float>(nS);
            op.f32.St1 = A.alloc<float>((int64_t)F * op.nfar1 * k * k);
            op.f32.Upad = A.alloc<float>(kt.nleaf() * op.cap * k);
            hipck(launch_to_float(kt.nleaf() * op.cap * k, op.d_Upad, op.f32.Upad, st), "to float");
            op.f32.panel = A.alloc<float>((int64_t)F * op.panel_total);
            hipck(launch_to_float(nU, op.d_U, op.f32.U, st), "to float");
            hipck(launch_to_float(nE, op.kdev.E, op.f32.E, st), "to float");
            if (nS > 0) hipck(launch_to_float(nS, op.d_St, op.f32.St, st), "to float");
            if (op.nfar1 > 0)
                hipck(launch_to_float((int64_t)F * op.nfar1 * k * k, op.d_St1, op.f32.St1, st), "to float");
            hipck(launch_to_float((int64_t)F * op.panel_total, op.d_panel, op.f32.panel, st), "to float");
            // K_near + B + M in FP32 for the several-rhs apply (the epilogue's FP64 gathers go away)
            op.f32.panel_bm = A.alloc<float>((int64_t)F * op.panel_total);
            hipck(launch_to_float((int64_t)F * op.panel_total, op.d_panel, op.f32.panel_bm, st), "to float");
            int64_t* d_off = A.upload(bm_off, st);
            hipck(launch_panel_add_csr(nnz, F, op.panel_total, d_off, op.d_BM, op.d_panel, op.f32.panel_bm, st),
                  "panel B + M");
            hipck(hipStreamSynchronize(st), "panel B + M sync");   // bm_off ends with this scope
            A.release(d_off);
        }
        hipck(hipStreamSynchronize(st), "tickets sync");
        if (op.opts.recompress_tol > 0.0 && !op.kfar.empty()) recompress(op, st);
    }
    // keep only what apply / load / export need
    // quadrature points and fields stay for the adjoint
    op.adj.qx = d_qx;
    op.adj.qs = d_qs;
    op.adj.qk = d_qk;
    op.adj.qint = d_qint;
    op.stats.t_total_ms = ms_since(t_all) + op.stats.t_plan_ms;
}

void fill_stats(fpde_op& op) {
    fpde_stats_t& S = op.stats;
    S.n_dofs = op.mesh.N;
    S.n_nodes = op.mesh.M;
    S.n_cells = op.mesh.nc;
    S.n_fields = op.F;
    S.n_pairs_identical = S.n_pairs_edge = S.n_pairs_vertex = 0;
    for (auto& p : op.pairs) (p.kind == 0 ? S.n_pairs_identical : p.kind == 1 ? S.n_pairs_edge : S.n_pairs_vertex)++;
    S.csr_nnz = (int64_t)op.csr_col.size();
    S.k_clusters = op.kt.ncl;
    S.k_levels = op.kt.L + 1;
    S.k_leaves = op.kt.nleaf();
    S.k_far = (int64_t)op.kfar.size();
    S.k_near = (int64_t)op.knear.size();
    S.k_rank = op.mesh.dim == 2 ? op.opts.cheb_p * op.opts.cheb_p : op.opts.cheb_p;
    int64_t cap = 0;
    for (int64_t c = op.kt.first_leaf(); c < op.kt.ncl; ++c) cap = std::max(cap, op.kt.end[c] - op.kt.beg[c]);
    S.k_leaf_cap = cap;
    S.rho_points = op.Q.nq;
    S.rho_clusters = op.rt.ncl;
    S.rho_levels = op.rt.L + 1;
    S.rho_far = (int64_t)op.rfar.size();
    S.rho_near = (int64_t)op.rnear.size();
    S.device_bytes = op.arena.bytes;
    S.apply_bytes_near = (int64_t)op.knear.size() * cap * cap * 8;
    S.apply_bytes_csr = S.csr_nnz * (8 + 4) + (op.mesh.N + 1) * 8;
    S.apply_bytes_bases = op.mesh.N * S.k_rank * 8;
}

void ensure_ws(fpde_op& op, int64_t R) {
    if (op.ws_R >= R) return;
    const int d = op.mesh.dim, p = op.opts.cheb_p, k = d == 2 ? p * p : p;
    if (op.d_xt) {
        op.arena.release(op.d_xt); op.arena.release(op.d_xh); op.arena.release(op.d_yh); op.arena.release(op.d_tmp);
    }
    op.d_tmp = op.arena.alloc<double>((int64_t)op.F * std::max<size_t>(1, op.kfar.size()) * k * R);
    op.d_xt = op.arena.alloc<double>((int64_t)op.F * (op.mesh.N + op.cap) * R);
    op.d_xh = op.arena.alloc<double>((int64_t)op.F * op.kt.ncl * k * R);
    op.d_yh = op.arena.alloc<double>((int64_t)op.F * op.kt.ncl * k * R);
    if (op.mixed) {   // FP32 workspace
        if (!op.f32.xh) {
            op.f32.xh = op.arena.alloc<float>((int64_t)op.F * op.kt.ncl * k);
            op.f32.zh = op.arena.alloc<float>((int64_t)op.F * op.kt.ncl * k);
            op.f32.zp = op.arena.alloc<float>((int64_t)op.F * std::max<int64_t>(1, op.far_plan.nchunks) * k);
            hipck(hipMemset(op.f32.zh, 0, sizeof(float) * op.F * op.kt.ncl * k), "zh");
        }
        if (op.f32.xhR) {
            op.arena.release(op.f32.xhR);
            op.arena.release(op.f32.yhR);
        }
        op.f32.xhR = op.arena.alloc<float>((int64_t)op.F * op.kt.ncl * k * R);
        op.f32.yhR = op.arena.alloc<float>((int64_t)op.F * op.kt.ncl * k * R);
    }
    op.ws_R = R;
}

ApplyPlan make_apply_plan(const fpde_op& op, const H2Tree& h) {
    const Tree& kt = op.kt;
    ApplyPlan a{};
    a.N = op.mesh.N;
    a.nleaf = kt.nleaf();
    a.first_leaf = kt.first_leaf();
    a.cap = op.cap;
    a.perm = op.kdev.perm;
    a.leaf_beg = op.d_leaf_beg;
    a.csr_ptr = op.d_csr_ptr;
    a.csr_col = op.d_csr_col;
    a.csr_val = op.d_BM;
    a.nnz = (int64_t)op.csr_col.size();
    a.near_ptr = op.d_near_ptr;
    a.near_src = op.d_near_src;
    a.near_blk = op.d_near;
    a.npairs = (int64_t)op.knear.size();
    a.U = op.d_U;
    a.k = h.k;
    return a;
}

// The one-vector kernels run this apply (the operator's precision pr: 0 FP64, 1 FP32 data)
bool single_path(const fpde_op& op, int pr, int64_t R) {
    const size_t esz = pr ? sizeof(float) : sizeof(double);
    return R == 1 && !op.rc.on && op.up[pr].ok && op.panel_max_stride * (int64_t)esz <= 64 * 1024;
}

// Enqueue one apply on s0 (far chain forked to s1 through fk/jn when s1 != s0).
// ev: optional 5 profiling events (requires s1 == s0).  cg: a CG iteration fused into
// the one-vector output kernel (callers check cg_fusable first).  Capturable.
hipError_t enqueue_apply(fpde_op& op, int parts, int dtype, const void* x, void* y, int64_t R, hipStream_t s0,
                         hipStream_t s1, hipEvent_t fk, hipEvent_t jn, hipEvent_t* ev, const CgFuse* cg = nullptr) {
    const int F = op.F, p = op.opts.cheb_p;
    const H2Tree h = make_h2(op.kt, op.kdev, p);
    const ApplyPlan a = make_apply_plan(op, h);
    const double* cv = nullptr;
    if ((parts & FPDE_PART_B) && (parts & FPDE_PART_M)) cv = op.d_BM;
    else if (parts & FPDE_PART_B) cv = op.d_B;
    else if (parts & FPDE_PART_M) cv = op.d_M;
    const int64_t nfar = (int64_t)op.kfar.size();
    const bool f32 = op.mixed && !(parts & FPDE_PART_FP64);
    const int pr = f32 ? 1 : 0;
    PanelPlan pp{op.d_poff, op.d_pstride, op.d_pcols, op.d_pcols_ptr, op.panel_max_stride, op.d_csr_col_dof};
    pp.pcols_pad = op.d_pcols_pad;
    pp.perm_pad = op.d_perm_pad;
    if (cv == op.d_BM) {
        pp.ell_col = op.d_ell_col;
        pp.ell_val = op.d_ell_val;
        pp.ell_w = op.ell_w;
    }
    if (single_path(op, pr, R)) {
        FarPlan fp = op.far_plan;
        if (cg) fp.cg = *cg;
        H2Tree h1 = h;   // the far list with sources moved down
        h1.far_ptr = op.d_far1_ptr;
        h1.far_src = op.d_far1_src;
        if (f32) {
            OpData<float> od{op.f32.U, op.f32.E, op.f32.St1, op.f32.panel, op.f32.xh, op.f32.zh, op.f32.zp,
                             op.f32.Upad};
            return launch_apply_single(a, h1, pp, op.up[1], fp, parts, F, cv, od, dtype, x, y, op.d_tickets,
                                       s0, ev);
        }
        OpData<double> od{op.d_U, op.kdev.E, op.d_St1, op.d_panel, op.d_xh, op.d_zh, op.d_zp, op.d_Upad};
        return launch_apply_single(a, h1, pp, op.up[0], fp, parts, F, cv, od, dtype, x, y, op.d_tickets, s0,
                                   ev);
    }
    // several right-hand sides: near panels as MFMA GEMMs and the far field as
    // batched products in the operator's precision (FP32 data for a mixed operator)
    // FP32 data, several right-hand sides, B + M and the near panels together: the panels
    // that hold B + M, no row gathers
    // (the several-rhs batched kernels only; the K > 32 fallbacks below read the plain panels)
    const float* panel32 = op.f32.panel;
    const double* cvb = cv;
    PanelPlan ppb = pp;
    const int bmk = FPDE_PART_B | FPDE_PART_M | FPDE_PART_KNEAR;
    if (f32 && op.f32.panel_bm && (parts & bmk) == bmk) {
        panel32 = op.f32.panel_bm;
        cvb = nullptr;
        ppb.ell_col = nullptr;
        ppb.ell_val = nullptr;
    }
    if (op.rc.on) {   // recompressed far field: rank r, dense transfers
        H2Tree hr = h;
        hr.k = op.rc.r;
        if (f32) {
            OpData<float> od{op.rc.U32, nullptr, op.rc.St32, panel32, nullptr, nullptr, nullptr, op.rc.Upad32,
                             op.rc.E32};
            return launch_apply_batched(a, hr, ppb, parts, F, (int)R, cvb, od, op.f32.xhR, op.f32.yhR, dtype, x, y, s0,
                                        ev);
        }
        OpData<double> od{op.rc.U, nullptr, op.rc.St, op.d_panel, nullptr, nullptr, nullptr, op.rc.Upad, op.rc.E};
        return launch_apply_batched(a, hr, ppb, parts, F, (int)R, cvb, od, op.d_xh, op.d_yh, dtype, x, y, s0, ev);
    }
    if (batched_fits(h, op.cap, pr)) {
        if (f32) {
            OpData<float> od{op.f32.U,  op.f32.E, op.f32.St, panel32, nullptr,
                             nullptr,   nullptr,  op.f32.Upad};
            return launch_apply_batched(a, h, ppb, parts, F, (int)R, cvb, od, op.f32.xhR, op.f32.yhR, dtype, x, y, s0,
                                        ev);
        }
        OpData<double> od{op.d_U, op.kdev.E, op.d_St, op.d_panel, nullptr, nullptr, nullptr, op.d_Upad};
        return launch_apply_batched(a, h, ppb, parts, F, (int)R, cvb, od, op.d_xh, op.d_yh, dtype, x, y, s0, ev);
    }
    // otherwise (K > 32): FP64 far field with LDS-resident subtrees, or per-level sweeps
    const void* panel = f32 ? (const void*)op.f32.panel : (const void*)op.d_panel;
    if (multi_fits(h, op.ls2, (int)R))
        return launch_apply_multi(a, h, op.ls2, pp, panel, f32 ? 1 : 0, parts, F, (int)R, cv, op.d_St, nfar, dtype, x,
                                  op.d_xh, op.d_tmp, y, s0, s1, fk, jn, ev);
    return launch_apply_wide(a, h, pp, panel, f32 ? 1 : 0, parts, F, (int)R, cv, op.d_St, dtype, x, op.d_xt, op.d_xh,
                             op.d_yh, y, s0, s1, fk, jn, ev);
}

// The one-vector apply with its workspace carved from the library's static device
// scratch instead of the operator's allocations: no hipMalloc, hipFree or allocating
// library call.  Layout (each part 256-byte aligned): x^ [F][ncl][k], then z^ [F][ncl][k],
// the upsweep tickets and the coupling tickets [F][ncl] (cleared together, since the
// kernels need them zero and the scratch keeps the last call's contents), then the
// coupling partial sums [F][nchunks][k].
void apply_noalloc_impl(fpde_op& op, int dtype, const void* x, void* y, int64_t R, hipStream_t st) {
    if (op.plan_only) fail(FPDE_ESTATE, "operator was built with FPDE_FLAG_PLAN_ONLY");
    if (dtype != FPDE_F64 && dtype != FPDE_F32) fail(FPDE_EINVAL, "dtype must be FPDE_F64 or FPDE_F32");
    if (!x || !y) fail(FPDE_EINVAL, "bad vectors");
    if (R != 1) fail(FPDE_EINVAL, "the allocation-free apply takes one right-hand side per field (nrhs = 1)");
    const int pr = op.mixed ? 1 : 0;
    if (!single_path(op, pr, 1) || op.far_plan.ntgt <= 0)
        fail(FPDE_EINVAL, "the allocation-free apply needs the one-vector path (an operator with far blocks and "
                          "panel rows within 64 KiB)");
    const int F = op.F, p = op.opts.cheb_p, k = op.mesh.dim == 2 ? p * p : p;
    const size_t esz = pr ? sizeof(float) : sizeof(double);
    const int64_t ncl = op.kt.ncl, nch = std::max<int64_t>(1, op.far_plan.nchunks);
    auto up256 = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t b_coef = up256((size_t)F * ncl * k * esz), b_tk = up256((size_t)F * ncl * sizeof(unsigned int));
    const size_t o_xh = 0, o_zh = b_coef, o_tk = o_zh + b_coef, o_ctk = o_tk + b_tk, o_zp = o_ctk + b_tk;
    const size_t need = o_zp + up256((size_t)F * nch * k * esz);
    if (need > kScratchBytes)
        fail(FPDE_EINVAL, "the allocation-free apply needs " + std::to_string(need) + " bytes of workspace; the static "
                          "scratch holds " + std::to_string(kScratchBytes));
    void* base = nullptr;
    hipck(scratch_address(&base), "scratch address");
    unsigned char* sb = (unsigned char*)base;
    hipck(launch_zero_words((int64_t)((o_zp - o_zh) / 4), (uint32_t*)(sb + o_zh), st), "clear scratch");
    const H2Tree h = make_h2(op.kt, op.kdev, p);
    const ApplyPlan a = make_apply_plan(op, h);
    PanelPlan pp{op.d_poff, op.d_pstride, op.d_pcols, op.d_pcols_ptr, op.panel_max_stride, op.d_csr_col_dof};
    pp.pcols_pad = op.d_pcols_pad;
    pp.perm_pad = op.d_perm_pad;
    pp.ell_col = op.d_ell_col;
    pp.ell_val = op.d_ell_val;
    pp.ell_w = op.ell_w;
    FarPlan fp = op.far_plan;
    fp.ctk = (unsigned int*)(sb + o_ctk);
    H2Tree h1 = h;   // the far list with sources moved down
    h1.far_ptr = op.d_far1_ptr;
    h1.far_src = op.d_far1_src;
    unsigned int* tk = (unsigned int*)(sb + o_tk);
    if (pr) {
        OpData<float> od{op.f32.U, op.f32.E, op.f32.St1, op.f32.panel, (float*)(sb + o_xh), (float*)(sb + o_zh),
                         (float*)(sb + o_zp), op.f32.Upad};
        hipck(launch_apply_single(a, h1, pp, op.up[1], fp, FPDE_PART_ALL, F, op.d_BM, od, dtype, x, y, tk, st,
                                  nullptr), "apply");
    } else {
        OpData<double> od{op.d_U, op.kdev.E, op.d_St1, op.d_panel, (double*)(sb + o_xh), (double*)(sb + o_zh),
                          (double*)(sb + o_zp), op.d_Upad};
        hipck(launch_apply_single(a, h1, pp, op.up[0], fp, FPDE_PART_ALL, F, op.d_BM, od, dtype, x, y, tk, st,
                                  nullptr), "apply");
    }
}

void apply_impl(fpde_op& op, int parts, int dtype, const void* x, void* y, int64_t R, hipStream_t st) {
    if (op.plan_only) fail(FPDE_ESTATE, "operator was built with FPDE_FLAG_PLAN_ONLY");
    if (dtype != FPDE_F64 && dtype != FPDE_F32) fail(FPDE_EINVAL, "dtype must be FPDE_F64 or FPDE_F32");
    if (R < 1 || !x || !y) fail(FPDE_EINVAL, "bad vectors");
    ensure_ws(op, R);
    if (op.profiling) {   // the same kernels, serialised on st, with events between the phases
        std::array<hipEvent_t, 5> ev{};
        for (auto& e : ev) hipck(hipEventCreate(&e), "event");
        hipck(enqueue_apply(op, parts, dtype, x, y, R, st, st, nullptr, nullptr, ev.data()), "apply");
        op.prof_ev.push_back(ev);
        return;
    }
    // launched directly: on this runtime a graph launch costs more host time
    // than the apply's three kernel launches and leaves gaps between them
    hipck(enqueue_apply(op, parts, dtype, x, y, R, st, op.stream2, op.ev_fork, op.ev_join, nullptr), "apply launch");
}

// ------------------------------------------------------------------ adjoint

void ensure_adj_ws(fpde_op& op, int64_t R) {
    auto& J = op.adj;
    if (J.ws_R >= R) return;
    Arena& A = op.arena;
    for (void* q : {(void*)J.out12, (void*)J.Ds, (void*)J.Dk, (void*)J.c, (void*)J.xw, (void*)J.xu, (void*)J.chat,
                    (void*)J.mom, (void*)J.Gs, (void*)J.Gk, (void*)J.rGs, (void*)J.rGk})
        if (q) A.release(q);
    const int64_t F = op.F, k = op.kt.ncl > 0 ? (op.mesh.dim == 2 ? op.opts.cheb_p * op.opts.cheb_p : op.opts.cheb_p) : 1;
    const int64_t nq = op.Q.nq, np = (int64_t)op.pairs.size();
    J.out12 = A.alloc<double>(F * np * 12);
    J.Ds = A.alloc<double>(F * nq);
    J.Dk = A.alloc<double>(F * nq);
    J.c = A.alloc<double>(F * nq);
    J.xw = A.alloc<double>(F * op.kt.ncl * k * R);
    J.xu = A.alloc<double>(F * op.kt.ncl * k * R);
    J.Gs = A.alloc<double>(F * op.kt.ncl * k);
    J.Gk = A.alloc<double>(F * op.kt.ncl * k);
    J.chat = A.alloc<double>(F * op.rt.ncl * k);
    J.mom = A.alloc<double>(F * op.rt.ncl * k);
    J.rGs = A.alloc<double>(F * op.rt.ncl * k);
    J.rGk = A.alloc<double>(F * op.rt.ncl * k);
    J.ws_R = R;
}

// gs, gk [F][M] = alpha d/ds_j, alpha d/dkappa_j of sum_r w_r^T A_h u_r
void adjoint_impl(fpde_op& op, double alpha, const double* w, const double* u, int64_t R, double* gs, double* gk,
                  hipStream_t st) {
    if (op.plan_only) fail(FPDE_ESTATE, "operator was built with FPDE_FLAG_PLAN_ONLY");
    if (!op.adj.ok) fail(FPDE_ESTATE, "adjoint unavailable: " + op.adj.why);
    if (!w || !u || !gs || !gk || R < 1) fail(FPDE_EINVAL, "bad vectors");
    if (!std::isfinite(alpha)) fail(FPDE_EINVAL, "alpha must be finite");
    ensure_ws(op, R);
    ensure_adj_ws(op, R);
    auto& J = op.adj;
    const HostMesh& m = op.mesh;
    const int d = m.dim, F = op.F, p = op.opts.cheb_p, k = d == 2 ? p * p : p;
    const int64_t M = m.M, N = m.N, nq = op.Q.nq, np = (int64_t)op.pairs.size();
    const int nqe = op.Q.nqe;
    const double as = op.opts.a_scale;
    hipck(launch_fill((int64_t)F * M, 0.0, gs, st), "fill");
    hipck(launch_fill((int64_t)F * M, 0.0, gk, st), "fill");
    // singular pairs (B)
    hipck(launch_adj_singular(d, np, J.pairs, op.d_X, M, F, J.s, J.k, as, op.opts.s_bar, op.opts.nq_sing, J.g, J.w, w,
                              u, N, (int)R, J.out12, st), "adjoint singular");
    hipck(launch_adj_gather(M, J.slot_ptr, J.slot_idx, nullptr, J.out12, np * 12, F, gs, M, st), "gather");
    hipck(launch_adj_gather(M, J.slot_ptr, J.slot_idx, nullptr, J.out12 + 6, np * 12, F, gk, M, st), "gather");
    // point densities: near blocks of K~, density near sums and exterior
    hipck(launch_fill((int64_t)F * nq, 0.0, J.Ds, st), "fill");
    hipck(launch_fill((int64_t)F * nq, 0.0, J.Dk, st), "fill");
    AdjKnear P{};
    P.dim = d;
    P.nqe = nqe;
    P.R = (int)R;
    P.nc = m.nc;
    P.nq = nq;
    P.N = N;
    P.cells = op.d_C;
    P.qx = J.qx;
    P.qw = op.d_qw;
    P.qs = J.qs;
    P.qk = J.qk;
    P.lam = op.d_lam;
    P.icells = J.icells;
    P.cell_leaf_ptr = J.cell_leaf_ptr;
    P.cell_leaf = J.cell_leaf;
    P.near_ptr = op.d_near_ptr;
    P.near_src = op.d_near_src;
    P.patch_ptr = J.patch_ptr;
    P.patch_cell = J.patch_cell;
    P.leaf_of_node = J.leaf_of_node;
    P.w = w;
    P.u = u;
    P.a_scale = as;
    for (int r = 0; r < (int)R; ++r) {
        P.r = r;
        hipck(launch_adj_knear(P, J.n_icells, F, J.Ds, J.Dk, st), "adjoint near blocks");
    }
    hipck(launch_adj_c(d, m.nc, nqe, op.d_C, op.d_cint, op.d_lam, op.d_qw, w, u, N, (int)R, F, J.c, st), "adjoint c");
    const H2Tree hr = make_h2(op.rt, J.rdev, p);
    hipck(launch_adj_rho_near(hr, J.rdev.perm, J.rnear_ptr, J.rnear_src, J.qx, op.d_qw, J.qs, J.qk, J.c, nqe, op.d_C,
                              m.nc, nq, F, as, J.Ds, J.Dk, st), "adjoint density near");
    if (m.R > 0.0)
        hipck(launch_adj_rho_ext(d, nq, J.qx, J.qs, J.qk, J.qint, J.c, F, m.R, op.opts.s_exterior,
                                 std::sqrt(op.opts.kappa_exterior), as, op.opts.n_theta, J.Ds, J.Dk, st),
              "adjoint exterior");
    hipck(launch_adj_points(M, op.d_nc_ptr, op.d_nc_cell, op.d_nc_slot, nqe, op.d_lam, J.Ds, J.Dk, nq, F, gs, gk, st),
          "adjoint points");
    // far blocks of K~: nested coefficients of w and u
    const H2Tree hk = make_h2(op.kt, op.kdev, p);
    const ApplyPlan a = make_apply_plan(op, hk);
    for (int pass = 0; pass < 2; ++pass) {
        double* xh = pass == 0 ? J.xw : J.xu;
        hipck(launch_gather(a, F, (int)R, FPDE_F64, pass == 0 ? w : u, op.d_xt, st), "gather");
        hipck(launch_leaf_up(a, hk, F, (int)R, op.d_xt, xh, st), "leaf up");
        for (int lev = op.kt.L - 1; lev >= 0; --lev) hipck(launch_up_level(hk, lev, F, (int)R, xh, st), "up");
    }
    const int64_t kf = op.kt.ncl * k;
    hipck(launch_adj_far(hk, -2.0, as, J.xw, kf * R, J.xu, kf * R, (int)R, F, J.Gs, J.Gk, st), "adjoint far K");
    hipck(launch_adj_gather(M, J.kst_ptr, J.kst_idx, J.kst_w, J.Gs, kf, F, gs, M, st), "gather");
    hipck(launch_adj_gather(M, J.kst_ptr, J.kst_idx, J.kst_w, J.Gk, kf, F, gk, M, st), "gather");
    // far blocks of the density: upsweep of c against the moments of the weights
    const int64_t rf = op.rt.ncl * k;
    for (int f = 0; f < F; ++f)
        hipck(launch_rho_moments(hr, J.rdev.perm, J.qx, J.c + (int64_t)f * nq, nq, 1, J.chat + f * rf, st), "moments");
    hipck(launch_rho_moments(hr, J.rdev.perm, J.qx, op.d_qw, nq, F, J.mom, st), "moments");
    for (int lev = op.rt.L - 1; lev >= 0; --lev) {
        hipck(launch_up_level(hr, lev, F, 1, J.chat, st), "up");
        hipck(launch_up_level(hr, lev, F, 1, J.mom, st), "up");
    }
    hipck(launch_adj_far(hr, 1.0, as, J.chat, rf, J.mom, rf, 1, F, J.rGs, J.rGk, st), "adjoint far density");
    hipck(launch_adj_gather(M, J.rst_ptr, J.rst_idx, J.rst_w, J.rGs, rf, F, gs, M, st), "gather");
    hipck(launch_adj_gather(M, J.rst_ptr, J.rst_idx, J.rst_w, J.rGk, rf, F, gk, M, st), "gather");
    if (alpha != 1.0) {
        hipck(launch_scale((int64_t)F * M, alpha, gs, st), "scale");
        hipck(launch_scale((int64_t)F * M, alpha, gk, st), "scale");
    }
}

// ------------------------------------------------------------------ CG solve and iterative refinement

// CG iterations whose Lanczos coefficients are kept for the condition estimate
constexpr int kHist = 2048;

// Number of eigenvalues below x of the symmetric tridiagonal matrix (diagonal d, off-diagonal
// e, e[k] couples k and k + 1): the sign changes of the Sturm sequence (LDL^T pivots).
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
    int cnt = 0;
    double q = 1.0;
    for (size_t k = 0; k < d.size(); ++k) {
        const double off = k > 0 ? e[k - 1] * e[k - 1] : 0.0;
        q = d[k] - x - (k > 0 ? off / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Extreme eigenvalues of the Lanczos matrix of m CG steps, T_kk = 1/alpha_k + beta_{k-1}/alpha_{k-1},
// T_{k,k+1} = sqrt(beta_k)/alpha_k, by bisection on the Sturm count in the Gershgorin interval:
// estimates of the extreme eigenvalues of the (preconditioned) operator CG ran on.
std::pair<double, double> lanczos_extremes(const double* al, const double* be, int m) {
    std::vector<double> d(m), e(m > 0 ? m - 1 : 0);
    for (int k = 0; k < m; ++k) d[k] = 1.0 / al[k] + (k > 0 ? be[k - 1] / al[k - 1] : 0.0);
    for (int k = 0; k + 1 < m; ++k) e[k] = std::sqrt(be[k]) / al[k];
    double lo = INFINITY, hi = -INFINITY;
    for (int k = 0; k < m; ++k) {
        const double rad = (k > 0 ? std::fabs(e[k - 1]) : 0.0) + (k + 1 < m ? std::fabs(e[k]) : 0.0);
        lo = std::min(lo, d[k] - rad);
        hi = std::max(hi, d[k] + rad);
    }
    auto kth = [&](int idx) {   // the idx-th smallest eigenvalue (0-based)
        double a = lo, b = hi;
        for (int it = 0; it < 200 && b - a > 1e-14 * std::max(std::fabs(a), std::fabs(b)); ++it) {
            const double c = 0.5 * (a + b);
            if (sturm_count(d, e, c) > idx) b = c;
            else a = c;
        }
        return 0.5 * (a + b);
    };
    return {kth(0), kth(m - 1)};
}

void ensure_solve_ws(fpde_op& op, int64_t R) {
    if (op.sw_R >= R) return;
    Arena& A = op.arena;
    for (void* q : {(void*)op.d_r, (void*)op.d_p, (void*)op.d_Ap, (void*)op.d_d, (void*)op.d_rout,
                    (void*)op.d_part1, (void*)op.d_part2, (void*)op.d_part3, (void*)op.d_bb, (void*)op.d_rro,
                    (void*)op.d_part_far,
                    (void*)op.cg.rr, (void*)op.cg.rr_next, (void*)op.cg.alpha, (void*)op.cg.beta, (void*)op.cg.tol2,
                    (void*)op.cg.active, (void*)op.cg.active_next, (void*)op.cg.iters, (void*)op.cg.flags,
                    (void*)op.cg.n_active, (void*)op.d_hist_a, (void*)op.d_hist_b})
        if (q) A.release(q);
    const int64_t n = (int64_t)op.F * op.mesh.N * R, S = (int64_t)op.F * R;
    const int64_t nb = cg_row_blocks(op.mesh.N, (int)R, op.F);
    op.d_r = A.alloc<double>(n);
    op.d_p = A.alloc<double>(n);
    op.d_Ap = A.alloc<double>(n);
    op.d_d = A.alloc<double>(n);
    op.d_rout = A.alloc<double>(n);
    op.d_part1 = A.alloc<double>(op.F * nb * R);
    op.d_part2 = A.alloc<double>(op.F * nb * R);
    op.d_part3 = A.alloc<double>(op.F * nb * R);
    op.d_hist_a = A.alloc<double>((int64_t)kHist * S);
    op.d_hist_b = A.alloc<double>((int64_t)kHist * S);
    op.d_part_far = R == 1 ? A.alloc<double>(op.F * op.kt.nleaf() * ((op.cap + 63) / 64)) : nullptr;
    op.d_bb = A.alloc<double>(S);
    op.d_rro = A.alloc<double>(S);
    op.cg.rr = A.alloc<double>(S);
    op.cg.rr_next = A.alloc<double>(S);
    op.cg.active_next = A.alloc<int>(S);
    op.cg.alpha = A.alloc<double>(S);
    op.cg.beta = A.alloc<double>(S);
    op.cg.tol2 = A.alloc<double>(S);
    op.cg.active = A.alloc<int>(S);
    op.cg.iters = A.alloc<int>(S);
    op.cg.flags = A.alloc<int>(S);
    op.cg.n_active = A.alloc<int>(1);
    if (!op.h_nact) hipck(hipHostMalloc((void**)&op.h_nact, sizeof(int), hipHostMallocDefault), "pinned");
    op.sw_R = R;
}

// One CG iteration on the system A d = rout (apply of precision `mixed`):
// Ap = A p; p.Ap; alpha, d += alpha p, r -= alpha Ap, r.r; beta, p = r + beta p.
// One right-hand side per field on the one-vector kernels with a far field: the output
// kernel computes p . Ap and commits the previous iteration's state (no CG_DOT pass)
bool cg_fusable(const fpde_op& op, bool mixed, int64_t R) {
    return single_path(op, mixed ? 1 : 0, R) && op.far_plan.ntgt > 0 && op.d_part_far;
}

// The inner CG of a mixed-precision solve keeps its vectors (r, p, Ap, d) in FP32, half
// the bytes of every pass and of the apply's x and y; it only has to reduce its residual
// by sqrt(rtol) >= 1e-7 (mixed_inner_tol), and the refinement's FP64 residual corrects
// the rest.  The one-vector path with the fused dot product keeps FP64 vectors.
bool cg_vec32(const fpde_op& op, bool mixed, int64_t R) { return mixed && !cg_fusable(op, mixed, R); }

hipError_t enqueue_cg_iteration(fpde_op& op, bool mixed, int64_t R, hipStream_t s0, hipStream_t s1) {
    const CgDims dm{op.mesh.N, (int)R, op.F, cg_row_blocks(op.mesh.N, (int)R, op.F)};
    double* pc3 = op.d_dinv ? op.d_part3 : nullptr;   // r . r partials of the preconditioned iteration
    const int parts = mixed ? FPDE_PART_ALL : (FPDE_PART_ALL | FPDE_PART_FP64);
    hipError_t e;
    if (cg_fusable(op, mixed, R)) {
        const CgFuse cf{op.d_p, op.d_part_far, op.cg.rr, op.cg.rr_next, op.cg.active, op.cg.active_next,
                        op.cg.n_active};
        if ((e = enqueue_apply(op, parts, FPDE_F64, op.d_p, op.d_Ap, R, s0, s1, op.ev_fork, op.ev_join, nullptr,
                               &cf)) != hipSuccess)
            return e;
        const int64_t nb_far = op.kt.nleaf() * ((op.cap + 63) / 64);   // blocks of the output kernel per field
        if ((e = launch_cg_rowblock(CG_UPDATE_UR, dm, op.d_p, op.d_Ap, op.d_d, op.d_r, nullptr, op.d_part2, pc3,
                                    op.d_part_far, op.cg, s0, nb_far, op.d_dinv)) != hipSuccess)
            return e;
        return launch_cg_rowblock(CG_UPDATE_P, dm, op.d_r, nullptr, nullptr, nullptr, op.d_p, nullptr, nullptr,
                                  op.d_part2, op.cg, s0, -1, op.d_dinv, pc3);
    }
    const bool v32 = cg_vec32(op, mixed, R);
    e = enqueue_apply(op, parts, v32 ? FPDE_F32 : FPDE_F64, op.d_p, op.d_Ap, R, s0, s1, op.ev_fork, op.ev_join,
                      nullptr);
    if (e != hipSuccess) return e;
    if ((e = launch_cg_rowblock(CG_DOT, dm, op.d_p, op.d_Ap, nullptr, nullptr, nullptr, op.d_part1, nullptr, nullptr,
                                op.cg, s0, -1, nullptr, nullptr, v32)) != hipSuccess)
        return e;
    if ((e = launch_cg_rowblock(CG_UPDATE_UR, dm, op.d_p, op.d_Ap, op.d_d, op.d_r, nullptr, op.d_part2, pc3,
                                op.d_part1, op.cg, s0, -1, op.d_dinv, nullptr, v32)) != hipSuccess)
        return e;
    return launch_cg_rowblock(CG_UPDATE_P, dm, op.d_r, nullptr, nullptr, nullptr, op.d_p, nullptr, nullptr, op.d_part2,
                              op.cg, s0, -1, op.d_dinv, pc3, v32);
}

// CG on A d = rout from d = 0 until |r_s| <= max(tau_in |rout_s|, rtol_abs_s) for every
// system s (rtol_abs_s = rtol |b_s|, |b_s|^2 in d_bb).  Returns the largest
// per-system iteration count; *breakdown is set if a system lost positivity.
int cg_run(fpde_op& op, bool mixed, int64_t R, double tau_in, double rtol, int maxit, hipStream_t st,
           bool* breakdown, double* cond) {
    const CgDims dm{op.mesh.N, (int)R, op.F, cg_row_blocks(op.mesh.N, (int)R, op.F)};
    const int64_t S = (int64_t)op.F * R;
    op.cg.hist_a = cond ? op.d_hist_a : nullptr;   // the Lanczos coefficients, when an estimate is asked
    op.cg.hist_b = cond ? op.d_hist_b : nullptr;
    op.cg.hist_cap = cond ? kHist : 0;
    hipck(launch_cg_rowblock(CG_COPY_RP, dm, nullptr, op.d_rout, op.d_d, op.d_r, op.d_p, op.d_part1,
                             op.d_dinv ? op.d_part3 : nullptr, nullptr, op.cg, st, -1, op.d_dinv, nullptr,
                             cg_vec32(op, mixed, R)),
          "cg start");
    hipck(launch_cg_start(dm, op.d_part1, op.d_bb, tau_in, rtol, op.cg, st, op.d_dinv ? op.d_part3 : nullptr),
          "cg start");
    hipck(hipMemcpyAsync(op.h_nact, op.cg.n_active, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
    hipck(hipStreamSynchronize(st), "sync");
    *breakdown = false;
    if (*op.h_nact == 0) {
        op.cg.hist_a = op.cg.hist_b = nullptr;
        op.cg.hist_cap = 0;
        return 0;
    }
    int it = 0, chunk = 4;
    while (it < maxit) {
        const int n = std::min(chunk, maxit - it);
        for (int j = 0; j < n; ++j) hipck(enqueue_cg_iteration(op, mixed, R, st, op.stream2), "cg iteration");
        it += n;
        hipck(hipMemcpyAsync(op.h_nact, op.cg.n_active, sizeof(int), hipMemcpyDeviceToHost, st), "copy");
        hipck(hipStreamSynchronize(st), "sync");
        if (*op.h_nact == 0) break;
        chunk = std::min(chunk * 2, 32);
    }
    std::vector<int> iters(S), flags(S);
    hipck(hipMemcpy(iters.data(), op.cg.iters, sizeof(int) * S, hipMemcpyDeviceToHost), "copy");
    hipck(hipMemcpy(flags.data(), op.cg.flags, sizeof(int) * S, hipMemcpyDeviceToHost), "copy");
    for (int f : flags) if (f) *breakdown = true;
    const int itmax = *std::max_element(iters.begin(), iters.end());
    if (cond && itmax > 1) {   // the largest estimate over the systems
        const int m = std::min(itmax, kHist);
        std::vector<double> ha((size_t)m * S), hb((size_t)m * S), a(m), b(m);
        hipck(hipMemcpy(ha.data(), op.d_hist_a, sizeof(double) * m * S, hipMemcpyDeviceToHost), "copy");
        hipck(hipMemcpy(hb.data(), op.d_hist_b, sizeof(double) * m * S, hipMemcpyDeviceToHost), "copy");
        for (int64_t sy = 0; sy < S; ++sy) {
            const int ms = std::min(iters[sy], kHist);
            if (ms < 2) continue;
            for (int k = 0; k < ms; ++k) {
                a[k] = ha[(size_t)k * S + sy];
                b[k] = hb[(size_t)k * S + sy];
            }
            const auto ex = lanczos_extremes(a.data(), b.data(), ms);
            if (ex.first > 0.0) *cond = std::max(*cond, ex.second / ex.first);
        }
    }
    op.cg.hist_a = op.cg.hist_b = nullptr;
    op.cg.hist_cap = 0;
    return itmax;
}

// rout = b - A_fp64 u, per-system |rout|^2 (d_rro) and |b|^2 (d_bb); returns max_s |rout_s| / |b_s|
double outer_residual(fpde_op& op, const double* b, double* u, int64_t R, hipStream_t st) {
    const CgDims dm{op.mesh.N, (int)R, op.F, cg_row_blocks(op.mesh.N, (int)R, op.F)};
    const int64_t S = (int64_t)op.F * R;
    apply_impl(op, FPDE_PART_ALL | FPDE_PART_FP64, FPDE_F64, u, op.d_Ap, R, st);
    hipck(launch_cg_rowblock(CG_RESID, dm, op.d_Ap, b, nullptr, op.d_rout, nullptr, op.d_part1, op.d_part2, nullptr,
                             op.cg, st), "residual");
    hipck(launch_cg_sum2(dm, op.d_part1, op.d_part2, op.d_rro, op.d_bb, st), "residual norms");
    std::vector<double> rr(S), bb(S);
    hipck(hipMemcpyAsync(rr.data(), op.d_rro, sizeof(double) * S, hipMemcpyDeviceToHost, st), "copy");
    hipck(hipMemcpyAsync(bb.data(), op.d_bb, sizeof(double) * S, hipMemcpyDeviceToHost, st), "copy");
    hipck(hipStreamSynchronize(st), "sync");
    double worst = 0.0;
    for (int64_t s = 0; s < S; ++s) {
        const double rel = bb[s] > 0.0 ? std::sqrt(rr[s] / bb[s]) : (rr[s] > 0.0 ? INFINITY : 0.0);
        if (!(rel <= worst)) worst = rel;   // NaN propagates
    }
    return worst;
}

// Inner relative tolerance of the mixed-precision CG inside the refinement loop:
// sqrt(rtol), so that two passes reach rtol when the mixed operator is accurate
// enough (a pass whose reduction falls short is followed by another one).
double mixed_inner_tol(double rtol) { return std::min(1e-2, std::max(1e-7, std::sqrt(rtol))); }
constexpr int kMaxRefinements = 60;

void solve_impl(fpde_op& op, const double* b, double* u, int64_t R, double rtol, int maxit, fpde_solve_info* info,
                hipStream_t st) {
    if (op.plan_only) fail(FPDE_ESTATE, "operator was built with FPDE_FLAG_PLAN_ONLY");
    if (!b || !u || R < 1) fail(FPDE_EINVAL, "bad vectors");
    if (!(rtol > 0.0) || maxit < 1) fail(FPDE_EINVAL, "need rtol > 0 and maxit >= 1");
    ensure_ws(op, R);
    ensure_solve_ws(op, R);
    const int64_t n = (int64_t)op.F * op.mesh.N * R;
    int total = 0, outer = 0;
    bool breakdown = false;
    double worst = outer_residual(op, b, u, R, st), best = worst;
    int stalls = 0;
    double cond = 0.0;
    while (worst > rtol && total < maxit && outer < kMaxRefinements) {
        const double tau = op.mixed ? mixed_inner_tol(rtol) : 0.0;
        bool bd = false;
        total += cg_run(op, op.mixed, R, tau, 0.5 * rtol, maxit - total, st, &bd, outer == 0 ? &cond : nullptr);
        breakdown = breakdown || bd;
        hipck(launch_vec_add(n, op.d_d, u, st, cg_vec32(op, op.mixed, R)), "update");
        worst = outer_residual(op, b, u, R, st);
        ++outer;
        if (worst < 0.5 * best) {
            best = worst;
            stalls = 0;
        } else if (++stalls >= 3) {
            break;
        }
    }
    if (info) {
        info->iterations = total;
        info->rel_residual = worst;
        info->converged = worst <= rtol ? 1 : 0;
        info->refinements = outer;
        info->cond_estimate = cond;
    }
    if (!(worst <= rtol))
        fail(FPDE_ENOCONV, breakdown ? "fpde_solve: CG breakdown (operator not positive definite in working precision)"
                                     : "fpde_solve: not converged within maxit / refinement limit");
}

}  // namespace

// ------------------------------------------------------------------ C ABI

namespace {
fpde_status guarded(const std::function<void()>& fn) {
    try {
        fn();
        g_err.clear();
        return FPDE_OK;
    } catch (const Fail& f) {
        g_err = f.msg;
        return f.st;
    } catch (const std::bad_alloc&) {
        g_err = "host out of memory";
        return FPDE_ENOMEM;
    } catch (const std::exception& e) {
        g_err = e.what();
        return FPDE_EINVAL;
    }
}
}  // namespace

extern "C" {

fpde_status fpde_opts_default(fpde_opts* o) {
    if (!o) return FPDE_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->precision = FPDE_PREC_FP64;
    o->leaf_size = 64;
    o->leaf_size_rho = 64;
    o->cheb_p = 5;
    o->eta = 1.0;
    o->nq_sing = 3;
    o->nq_reg = 3;
    o->s_bar = 0.9;
    o->s_exterior = 0.0;
    o->kappa_exterior = 1.0;
    o->n_theta = 128;
    o->a_scale = 1.0;
    return FPDE_OK;
}

fpde_status fpde_gauss_legendre(int32_t n, double* x, double* w) {
    return guarded([&] {
        if (n < 1 || n > 64 || !x || !w) fail(FPDE_EINVAL, "n in [1,64] and non-NULL arrays required");
        gauss_legendre01(n, x, w);
    });
}

fpde_status fpde_build(const fpde_mesh* mesh, int32_t n_fields, const double* s, const double* kappa,
                       const fpde_opts* opts, fpde_op** out) {
    return guarded([&] {
        if (!out) fail(FPDE_EINVAL, "out is NULL");
        *out = nullptr;
        fpde_opts o;
        if (opts) o = *opts;
        else fpde_opts_default(&o);
        validate(mesh, n_fields, s, kappa, o);
        std::unique_ptr<fpde_op> op(new fpde_op());
        op->opts = o;
        op->F = n_fields;
        op->plan_only = (o.flags & FPDE_FLAG_PLAN_ONLY) != 0;
        op->mixed = o.precision == FPDE_PREC_MIXED;
        HostMesh& m = op->mesh;
        m.dim = mesh->dim;
        m.M = mesh->n_nodes;
        m.N = mesh->n_dofs;
        m.nc = mesh->n_cells;
        m.R = mesh->exterior_radius;
        m.X.assign(mesh->coords, mesh->coords + (int64_t)m.dim * m.M);
        m.C.assign(mesh->cells, mesh->cells + (int64_t)(m.dim + 1) * m.nc);
        m.interior.assign(mesh->cell_interior, mesh->cell_interior + m.nc);
        op->s.assign(s, s + (int64_t)n_fields * m.M);
        op->kappa.assign(kappa, kappa + (int64_t)n_fields * m.M);
        plan(*op);
        if (!op->plan_only) {
            int ndev = 0;
            if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) fail(FPDE_EDEVICE, "no HIP device");
            hipck(hipStreamCreateWithFlags(&op->stream, hipStreamNonBlocking), "stream");
            hipck(hipStreamCreateWithFlags(&op->stream2, hipStreamNonBlocking), "stream");
            hipck(hipEventCreateWithFlags(&op->ev_fork, hipEventDisableTiming), "event");
            hipck(hipEventCreateWithFlags(&op->ev_join, hipEventDisableTiming), "event");
            build_device(*op);
            // set-up of the allocation-free apply: this device's scratch address, once per device
            void* scratch = nullptr;
            hipck(scratch_address(&scratch), "scratch address");
        }
        fill_stats(*op);
        *out = op.release();
    });
}

fpde_status fpde_apply_noalloc(fpde_op* op, int32_t dtype, const void* x, void* y, int64_t nrhs, void* hip_stream) {
    return guarded([&] {
        if (!op) fail(FPDE_EINVAL, "op is NULL");
        apply_noalloc_impl(*op, dtype, x, y, nrhs, (hipStream_t)hip_stream);
    });
}

fpde_status fpde_apply_parts(fpde_op* op, int32_t parts, int32_t dtype, const void* x, void* y, int64_t nrhs,
                             void* hip_stream) {
    return guarded([&] {
        if (!op) fail(FPDE_EINVAL, "op is NULL");
        apply_impl(*op, parts, dtype, x, y, nrhs, (hipStream_t)hip_stream);
    });
}

fpde_status fpde_apply(fpde_op* op, int32_t dtype, const void* x, void* y, int64_t nrhs, void* hip_stream) {
    return fpde_apply_parts(op, FPDE_PART_ALL, dtype, x, y, nrhs, hip_stream);
}

fpde_status fpde_load_vector(fpde_op* op, const double* f_nodal, double* F, void* hip_stream) {
    return guarded([&] {
        if (!op || !f_nodal || !F) fail(FPDE_EINVAL, "NULL argument");
        if (op->plan_only) fail(FPDE_ESTATE, "plan-only operator");
        hipck(launch_load_nv(op->mesh.N, op->mesh.dim + 1, op->d_nc_ptr, op->d_nc_cell, op->d_nc_slot, op->d_C,
                             op->mesh.nc, op->Q.nqe, op->d_lam, op->d_qw, op->d_cint, f_nodal, F,
                             (hipStream_t)hip_stream), "load");
    });
}

fpde_status fpde_solve(fpde_op* op, const double* Fv, double* u, int64_t nrhs, double rtol, int32_t maxit,
                       fpde_solve_info* info, void* hip_stream) {
    return guarded([&] {
        if (!op) fail(FPDE_EINVAL, "op is NULL");
        solve_impl(*op, Fv, u, nrhs, rtol, maxit, info, (hipStream_t)hip_stream);
    });
}

fpde_status fpde_apply_adjoint(fpde_op* op, double alpha, const double* w, const double* u, int64_t nrhs,
                               double* grad_s, double* grad_kappa, void* hip_stream) {
    return guarded([&] {
        if (!op) fail(FPDE_EINVAL, "op is NULL");
        adjoint_impl(*op, alpha, w, u, nrhs, grad_s, grad_kappa, (hipStream_t)hip_stream);
    });
}

fpde_status fpde_profile(fpde_op* op, int32_t enable, fpde_profile_t* out) {
    return guarded([&] {
        if (!op) fail(FPDE_EINVAL, "op is NULL");
        fpde_profile_t acc{};
        for (auto& ev : op->prof_ev) {
            hipck(hipEventSynchronize(ev[4]), "event sync");
            // ev0 start, ev1 end of the far work before the near-field kernel, ev2/ev3 start/stop of that kernel, ev4 end
            float b = 0, c = 0, d = 0, e = 0;
            hipck(hipEventElapsedTime(&b, ev[0], ev[1]), "event time");
            hipck(hipEventElapsedTime(&c, ev[2], ev[3]), "event time");
            hipck(hipEventElapsedTime(&d, ev[3], ev[4]), "event time");
            hipck(hipEventElapsedTime(&e, ev[0], ev[4]), "event time");
            acc.ms_far += b;
            acc.ms_out += c;
            acc.ms_far_out += d;
            acc.ms_total += e;
            acc.n_applies++;
            for (auto& e : ev) (void)hipEventDestroy(e);
        }
        op->prof_ev.clear();
        op->profiling = enable != 0;
        if (out) *out = acc;
    });
}

fpde_status fpde_stats(const fpde_op* op, fpde_stats_t* s) {
    if (!op || !s) return FPDE_EINVAL;
    *s = op->stats;
    s->device_bytes = op->arena.bytes;
    return FPDE_OK;
}

fpde_status fpde_export(const fpde_op* op, int32_t what, int32_t field, void* dst, int64_t* count) {
    return guarded([&] {
        if (!op || !count) fail(FPDE_EINVAL, "NULL argument");
        if (field < 0 || field >= op->F) fail(FPDE_EINVAL, "field out of range");
        const int64_t N = op->mesh.N;
        std::vector<int64_t> iv;
        std::vector<double> dv;
        bool is_int = true;
        auto dof_csr = [&](const double* dvals, std::vector<int64_t>* ptr, std::vector<int64_t>* cols,
                           std::vector<double>* vals) {
            // rows/cols back to dof order
            std::vector<double> hv;
            const int64_t nnz = (int64_t)op->csr_col.size();
            if (dvals) {
                hv.resize(nnz);
                hipck(hipMemcpy(hv.data(), dvals + (int64_t)field * nnz, sizeof(double) * nnz, hipMemcpyDeviceToHost),
                      "export copy");
            }
            std::vector<std::tuple<int64_t, int64_t, double>> e;
            e.reserve(nnz);
            for (int64_t r = 0; r < N; ++r)
                for (int64_t q = op->csr_ptr[r]; q < op->csr_ptr[r + 1]; ++q)
                    e.emplace_back(op->kt.perm[r], op->kt.perm[op->csr_col[q]], dvals ? hv[q] : 0.0);
            std::sort(e.begin(), e.end());
            if (ptr) {
                ptr->assign(N + 1, 0);
                for (auto& t : e) (*ptr)[std::get<0>(t) + 1]++;
                for (int64_t i = 0; i < N; ++i) (*ptr)[i + 1] += (*ptr)[i];
            }
            if (cols) for (auto& t : e) cols->push_back(std::get<1>(t));
            if (vals) for (auto& t : e) vals->push_back(std::get<2>(t));
        };
        switch (what) {
            case FPDE_EXPORT_CSR_ROWPTR: dof_csr(nullptr, &iv, nullptr, nullptr); break;
            case FPDE_EXPORT_CSR_COLS: dof_csr(nullptr, nullptr, &iv, nullptr); break;
            case FPDE_EXPORT_CSR_B:
            case FPDE_EXPORT_CSR_M:
                if (op->plan_only) fail(FPDE_ESTATE, "plan-only operator");
                is_int = false;
                dof_csr(what == FPDE_EXPORT_CSR_B ? op->d_B : op->d_M, nullptr, nullptr, &dv);
                break;
            case FPDE_EXPORT_K_PERM: iv = op->kt.perm; break;
            case FPDE_EXPORT_K_LEAFPTR:
                for (int64_t c = op->kt.first_leaf(); c < op->kt.ncl; ++c) iv.push_back(op->kt.beg[c]);
                iv.push_back(N);
                break;
            case FPDE_EXPORT_K_FAR: for (auto& p : op->kfar) { iv.push_back(p.first); iv.push_back(p.second); } break;
            case FPDE_EXPORT_K_NEAR: for (auto& p : op->knear) { iv.push_back(p.first); iv.push_back(p.second); } break;
            case FPDE_EXPORT_RHO_PERM: iv = op->rt.perm; break;
            case FPDE_EXPORT_RHO_FAR: for (auto& p : op->rfar) { iv.push_back(p.first); iv.push_back(p.second); } break;
            case FPDE_EXPORT_RHO_NEAR: for (auto& p : op->rnear) { iv.push_back(p.first); iv.push_back(p.second); } break;
            case FPDE_EXPORT_RHO:
                if (op->plan_only) fail(FPDE_ESTATE, "plan-only operator");
                is_int = false;
                dv.resize(op->Q.nq);
                hipck(hipMemcpy(dv.data(), op->d_rho + (int64_t)field * op->Q.nq, sizeof(double) * op->Q.nq,
                                hipMemcpyDeviceToHost), "export rho");
                break;
            case FPDE_EXPORT_PAIRS:
                for (auto& p : op->pairs) {
                    iv.push_back(p.kind); iv.push_back(p.c0); iv.push_back(p.c1);
                    for (int a = 0; a < 3; ++a) iv.push_back(p.v[a]);
                    iv.push_back(p.v[4]); iv.push_back(p.v[5]);
                }
                break;
            case FPDE_EXPORT_K_BOXES:
            case FPDE_EXPORT_RHO_BOXES: {
                is_int = false;
                const Tree& t = what == FPDE_EXPORT_K_BOXES ? op->kt : op->rt;
                for (int64_t c = 0; c < t.ncl; ++c) {
                    for (int k = 0; k < t.dim; ++k) dv.push_back(t.lo[c * t.dim + k]);
                    for (int k = 0; k < t.dim; ++k) dv.push_back(t.hi[c * t.dim + k]);
                }
                break;
            }
            default: fail(FPDE_EINVAL, "unknown export");
        }
        const int64_t n = is_int ? (int64_t)iv.size() : (int64_t)dv.size();
        if (dst) {
            if (*count < n) fail(FPDE_EINVAL, "destination too small");
            if (is_int) std::memcpy(dst, iv.data(), sizeof(int64_t) * n);
            else std::memcpy(dst, dv.data(), sizeof(double) * n);
        }
        *count = n;
    });
}

// Releases everything; the HIP results are not reported (there is no status to return)
void fpde_destroy(fpde_op* op) {
    if (!op) return;
    if (op->h_nact) (void)hipHostFree(op->h_nact);
    for (auto& ev : op->prof_ev)
        for (auto& e : ev) (void)hipEventDestroy(e);
    if (op->stream) {
        (void)hipStreamSynchronize(op->stream);
        (void)hipStreamDestroy(op->stream);
    }
    if (op->stream2) {
        (void)hipStreamSynchronize(op->stream2);
        (void)hipStreamDestroy(op->stream2);
    }
    if (op->ev_fork) (void)hipEventDestroy(op->ev_fork);
    if (op->ev_join) (void)hipEventDestroy(op->ev_join);
    delete op;
}

const char* fpde_last_error(void) { return g_err.c_str(); }

}  // extern "C"
