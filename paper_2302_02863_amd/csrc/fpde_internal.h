// Internal declarations shared by the host planner (fpde_host.cpp) and the
// HIP kernels (fpde_kernels.hip).  Plain pointers only; all device arrays are
// structure-of-arrays in HBM.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace fpde {

constexpr int kMaxP = 8;        // Chebyshev points per dimension supported by the kernels
constexpr int kMaxNq = 8;       // Gauss points per direction supported by the kernels
constexpr int kMaxDeg = 16;     // max cells around a node handled by the near-block kernel

// ---------------------------------------------------------------- build kernels

// Local matrices of touching pairs (Sec. 4).  pairs: [np][8] int32 rows
// (kind, cell0 v0 v1 v2, cell1 v0 v1 v2, pad) with canonical vertices; kind 0
// identical, 1 edge, 2 vertex (1D: two vertices per cell).  out: [F][np][25],
// entry a*5+b (a <= b) over the local dof list of the case, already multiplied
// by the pair weight (2 for distinct cells, 1 for identical).
hipError_t launch_singular(int dim, int64_t np, const int32_t* pairs, const double* coords,
                           int64_t n_nodes, int F, const double* s, const double* kappa,
                           double a_scale, double s_bar, int nq, const double* g01,
                           const double* w01, double* out, hipStream_t st);

// out[f*nslots + i] = sum_{k in [ptr[i],ptr[i+1])} w[k] * src[f*src_stride + idx[k]]
hipError_t launch_segsum(int64_t nslots, const int64_t* ptr, const int64_t* idx, const double* w,
                         int F, const double* src, int64_t src_stride, double* out,
                         hipStream_t st);

// s, sqrt(kappa) at the quadrature points: qs[f][q], qk[f][q]
// ns[f][i], nk[f][i] = s_f and sqrt(kappa_f) at node i (< nn) from its stencil of 3
// (mesh node, P1 weight) entries, node -1 padding
hipError_t launch_node_fields(int64_t nn, int F, int64_t M, const int64_t* st_node, const double* st_w,
                              const double* s, const double* kappa, double* ns, double* nk, hipStream_t st);
hipError_t launch_quad_fields(int dim, int64_t nc, int nqe, const int32_t* cells,
                              const double* lam /*[dim+1][nqe]*/, int F, int64_t n_nodes,
                              const double* s, const double* kappa, double* qs, double* qk,
                              hipStream_t st);

// Generic H2 description (one tree).  Clusters in heap order, leaves contiguous.
struct H2Tree {
    int dim, p, k, L;
    int64_t ncl, nleaf, first_leaf;
    const int64_t* beg;        // [ncl] tree-order ranges
    const int64_t* end;
    const double* axes;        // [ncl][dim][p] Chebyshev points per axis
    const double* E;           // [ncl][dim][p][p] child->parent 1D transfers, [b][a]
    const double* node_s;      // [F][ncl][k]
    const double* node_k;      // [F][ncl][k]  sqrt(kappa)
    const int64_t* far_ptr;    // [ncl+1] by target cluster
    const int64_t* far_src;    // [nfar]
};

// Chebyshev transfer matrices E (Sec. 5.3 nested bases).
hipError_t launch_transfer(const H2Tree& t, double* E, hipStream_t st);
// xh[f][parent][alpha][r] = sum_children E^T xh[child]   (one level)
hipError_t launch_up_level(const H2Tree& t, int level, int F, int R, double* xh, hipStream_t st);
// yh[f][child][beta][r] += E yh[parent]                 (one level)
hipError_t launch_down_level(const H2Tree& t, int level, int F, int R, double* yh, hipStream_t st);
// yh[f][s][alpha][r] = fac * sum_far sum_beta gamma(xi_alpha, xi'_beta) xh[f][s'][beta][r]
hipError_t launch_coupling(const H2Tree& t, int F, int R, double fac, double a_scale,
                           const double* xh, double* yh, hipStream_t st);

// Density tree leaf operations (Sec. 6.2): moments m[f][leaf][beta] = sum l_beta(q) w(q)
hipError_t launch_rho_moments(const H2Tree& t, const int64_t* perm, const double* qx,
                              const double* qw, int64_t nq_all, int F, double* xh, hipStream_t st);
// rho[f][q] += sum_alpha l_alpha(q) yh[f][leaf][alpha] for interior q
hipError_t launch_rho_eval(const H2Tree& t, const int64_t* perm, const double* qx,
                           const uint8_t* q_int, int64_t nq_all, int F, const double* yh,
                           double* rho, hipStream_t st);
// near sums with the mesh-dependent kernel gamma_T (eq. e:g-t)
hipError_t launch_rho_near(const H2Tree& t, const int64_t* perm, const int64_t* near_ptr,
                           const int64_t* near_src, const double* qx, const double* qw,
                           const double* qs, const double* qk, const uint8_t* q_int, int nqe,
                           const int32_t* cells, int64_t nc, int64_t nq_all, int F, double a_scale,
                           double* rho, hipStream_t st);
// exterior density beyond |x| = R (eq. e:rho), added at interior points
hipError_t launch_rho_exterior(int dim, int64_t nq_all, const double* qx, const double* qs,
                               const double* qk, const uint8_t* q_int, int F, double R,
                               double s_out, double k_out_sqrt, double a_scale, int n_theta,
                               double* rho, hipStream_t st);
// mass local matrices of interior cells: out[f][ci][6] (a<=b over 3 vertices, 2 in 1D -> 3)
hipError_t launch_mass_local(int dim, int64_t n_int_cells, const int64_t* int_cells, int nqe,
                             const double* lam, const double* qw, const double* rho, int64_t nq_all,
                             int F, double* out, hipStream_t st);

// Leaf bases U[t][alpha] = sum_{tau in S_i} sum_q w psi_i(q) l_alpha(q) (eq. eq:triple_product)
hipError_t launch_basis_n(const H2Tree& t, int64_t N, const int64_t* perm, const int64_t* nc_ptr,
                          const int64_t* nc_cell, const int8_t* nc_slot, int nqe, const double* qx,
                          const double* qw, const double* lam, int64_t nq_all, double* U,
                          hipStream_t st);

// Near leaf blocks of K~ (eq. e:k-near): nb[f][pair][cap][cap]
struct NearPlan {
    int64_t npairs, cap;
    const int64_t* tgt;        // [npairs] target leaf (heap id)
    const int64_t* src;        // [npairs] source leaf
    const int64_t* patch_ptr;  // [nleaf+1] cells of the patch of each leaf (sorted)
    const int64_t* patch_cell; // [...]
    const int64_t* row_ptr;    // [N+1] per tree position: entries into row_lcell/row_slot
    const int32_t* row_lcell;  // local patch index of each cell around the row node
    const int8_t* row_slot;    // vertex slot of the row node in that cell
    const int64_t* nc_ptr;     // node -> cells (global)
    const int64_t* nc_cell;
    const int8_t* nc_slot;
    // the blocks computed: every pair, or, when the pair list is closed under
    // transposition, the pairs (t, s) with t <= s, each also stored transposed as
    // the block of (s, t) (the kernel of K is symmetric in x and y)
    int64_t nown;
    const int64_t* own;        // [nown] pair index
    const int64_t* mirror;     // [nown] index of the pair (s, t), or the pair itself
};
hipError_t launch_near_blocks_lds(const H2Tree& t, const NearPlan& np, int64_t max_patch,
                                  const int64_t* perm, const int32_t* cells, int nqe, int64_t nc,
                                  const double* qx, const double* qw, const double* qs,
                                  const double* qk, const double* lam, int64_t nq_all, int F,
                                  double a_scale, double* nb, hipStream_t st);

// Load vector F_i = sum_q w psi_i(q) f(q) for dofs i (node -> cell lists)
hipError_t launch_load_nv(int64_t N, int nv, const int64_t* nc_ptr, const int64_t* nc_cell,
                          const int8_t* nc_slot, const int32_t* cells, int64_t nc, int nqe,
                          const double* lam, const double* qw, const uint8_t* cell_int,
                          const double* f_nodal, double* F, hipStream_t st);

hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z,
                        hipStream_t st);
hipError_t launch_fill(int64_t n, double v, double* x, hipStream_t st);
hipError_t launch_scale(int64_t n, double alpha, double* x, hipStream_t st);

// ---------------------------------------------------------------- apply kernels

struct ApplyPlan {
    int64_t N, nleaf, first_leaf, cap;
    const int64_t* perm;          // tree position -> dof
    const int64_t* leaf_beg;      // [nleaf+1]
    const int64_t* csr_ptr;       // [N+1] tree-ordered rows
    const int32_t* csr_col;       // tree positions
    const double* csr_val;        // [F][nnz]  B + M
    int64_t nnz;
    const int64_t* near_ptr;      // [nleaf+1] pairs of each target leaf
    const int64_t* near_src;      // [npairs] source leaf index (0-based leaf index)
    const double* near_blk;       // [F][npairs][cap][cap]
    int64_t npairs;
    const double* U;              // [N][k]
    int k;
};

// x_tree[f][t][r] = x[f][perm[t]][r]  (dtype 0 double, 1 float)
hipError_t launch_gather(const ApplyPlan& a, int F, int R, int dtype, const void* x, double* xt,
                         hipStream_t st);
// xh[f][leaf][alpha][r] = sum_{t in leaf} U[t][alpha] xt[f][t][r]
hipError_t launch_leaf_up(const ApplyPlan& a, const H2Tree& t, int F, int R, const double* xt,
                          double* xh, hipStream_t st);
// y[f][perm[t]][r] (=, or += with accumulate) (B+M) xt + K_near xt + U yh   (parts select terms)
hipError_t launch_leaf_out(const ApplyPlan& a, const H2Tree& t, int parts, int F, int R,
                           const double* csr_val_override, const double* xt, const double* yh,
                           int dtype, void* y, hipStream_t st, int accumulate = 0);

hipError_t launch_coupling_store(const H2Tree& t, int64_t nfar, const int64_t* far_tgt, int F, double fac,
                                 double a_scale, double* St, hipStream_t st);
// St1[f][j] = S_orig[j] M_r^T for the far list with sources moved down to src1[j]
// (depth[j] levels below the original source; St layout [f][pair][beta][alpha])
hipError_t launch_expand_coupling(const H2Tree& t, int64_t n1, const int64_t* orig, const int64_t* src1,
                                  const int32_t* depth, int F, int64_t nfar, const double* St, double* St1,
                                  hipStream_t st);
// yh[f][c] = sum_{e in far(c)} S_e xh[f][src(e)]  (per-level fallback)
hipError_t launch_coupling_apply(const H2Tree& t, int F, int R, const double* St, const double* xh, double* yh,
                                 hipStream_t st);
hipError_t launch_to_float(int64_t n, const double* src, float* dst, hipStream_t st);

// ---------------------------------------------------------------- apply, several right-hand sides (fpde_multi.hip)

// LDS needed by the multi-RHS far chain with subtree roots at level ls
bool multi_fits(const H2Tree& t, int ls, int R);
// main stream: CSR + near blocks in place; side stream: upsweep, top levels,
// coupling products; join; per-leaf downsweep fused with the output (FP64).
// ev (optional, 5 events, side == st): start, far chain end, near kernel
// start/stop, end.
struct PanelPlan;
hipError_t launch_apply_multi(const ApplyPlan& a, const H2Tree& t, int ls, const PanelPlan& pp, const void* panel,
                              int panel_f32, int parts, int F, int R, const double* csr_val, const double* St,
                              int64_t nfar, int dtype, const void* x, double* xh, double* tmp, void* y,
                              hipStream_t st, hipStream_t side, hipEvent_t fork, hipEvent_t join, hipEvent_t* ev);
hipError_t launch_apply_wide(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, const void* panel, int panel_f32,
                             int parts, int F, int R, const double* csr_val, const double* St, int dtype,
                             const void* x, double* xt, double* xh, double* yh, void* y, hipStream_t st,
                             hipStream_t side, hipEvent_t fork, hipEvent_t join, hipEvent_t* ev);

// ---------------------------------------------------------------- apply, one right-hand side (fpde_apply.hip)

// Near leaf blocks packed per target leaf into row-major panels
// panel[f][poff[li] + row * pstride[li] + col]; columns are dof indices.
struct PanelPlan {
    const int64_t* poff;        // [nleaf+1]
    const int64_t* pstride;     // [nleaf] row stride (multiple of 4)
    const int32_t* pcols;       // [pcols_ptr[nleaf]] dof of each panel column
    const int64_t* pcols_ptr;   // [nleaf+1]
    int64_t max_stride;
    const int32_t* csr_col_dof; // CSR columns of B + M as dof indices
    // by leaf slot (leaf li, row it -> slot li * cap + it), read by the one-vector apply:
    const int32_t* pcols_pad = nullptr;  // [nleaf][max_stride] panel column dofs, -1 past the leaf's columns
    const int64_t* perm_pad = nullptr;   // [nleaf * cap] output index, -1 for slots past the leaf's rows
    const int32_t* ell_col = nullptr;    // [nleaf * cap][ell_w] dof columns of B + M in CSR order; a row's
                                         // padding repeats its first column (value 0), slots past the leaf's
                                         // rows hold -1
    const double* ell_val = nullptr;     // [F][nleaf * cap][ell_w] values of B + M; null: use the CSR
    int ell_w = 0;
};
// Operator data of one precision used by the single-vector apply
template <typename T>
struct OpData {
    const T* U;       // [N][K] leaf bases (tree order)
    const T* E;       // [ncl][D][P][P] transfers
    const T* St;      // [F][nfar][K][K] coupling matrices, transposed
    const T* panel;   // [F][panel_total]
    T* xh;            // [F][ncl][K] workspace: upsweep coefficients x^
    T* zh;            // [F][ncl][K] coupling sums z^ per target cluster, zero for the others
    T* zp;            // [F][nchunks][K] partial sums of targets split in several coupling chunks
    const T* Upad;    // [nleaf * cap][K] bases by leaf slot (rows of leaf li at li * cap, zero padded)
    const T* Ed = nullptr;   // [ncl][K][K] dense transfers (child index, parent index) of
                             // recompressed bases; nullptr: the Kronecker transfers E
};
// One-launch upsweep: leaf-stage subtree depth d0, upper-stage depth ds
struct UpPlan {
    int d0, ds;
    int lmin;          // shallowest level whose coefficients a far pair reads; the upsweep stops there
    size_t path_lds;   // LDS of the output kernel's root-path walk (bytes, whole depth)
    bool ok;
};
// A CG iteration fused into the one-vector output kernel (one right-hand side per
// field): the kernel adds p . y of its rows to part[f][block], and block 0 of
// field f commits the previous iteration's |r|^2 and activity of system f (block
// 0 of field 0 also clears the active-system count), which the first CG pass
// after a plain apply does otherwise (see fpde_solve.hip).  p null: not fused.
struct CgFuse {
    const double* p = nullptr;   // [F][N] search direction
    double* part = nullptr;      // [F][blocks of the output kernel]
    double *rr = nullptr, *rr_next = nullptr;
    int *active = nullptr, *active_next = nullptr, *n_active = nullptr;
};
// Far targets of the single-vector output kernel
constexpr int kChunkWords = 4 + 16;
struct FarPlan {
    const int64_t* tgt;    // [ntgt] clusters with incoming far pairs, in heap order
    int64_t ntgt;
    int ltop;              // level of the shallowest target
    // coupling work: chunks of at most one pair per slot of a coupling block,
    // kChunkWords words each: target, first pair, end pair, (chunk of the target << 32 |
    // chunks of the target), then the source cluster of each pair of the chunk
    const int64_t* chunks;
    int64_t nchunks;
    unsigned int* ctk;     // [F][ncl] zero-initialised tickets of targets split in several chunks
    const int64_t* perm_pad;   // [nleaf * cap] output index by leaf slot, -1 for padding
    CgFuse cg{};               // set for the applies of fused CG iterations
};
UpPlan plan_up_tree(const H2Tree& t, int64_t cap, int lmin, int prec /*0 double, 1 float*/);
hipError_t launch_pack_panels(int64_t nleaf, int64_t cap, int64_t npairs, const int64_t* near_ptr,
                              const int64_t* near_src, const int64_t* leaf_beg, const int64_t* pcol_off,
                              const int64_t* poff, const int64_t* pstride, const int64_t* pcols_ptr, const double* nb,
                              int F, double* panel, hipStream_t st);
// The far field's leaf output U_leaf Y^_leaf added by the several-right-hand-side near
// kernel (yh null: none); K <= 32
template <typename T>
struct MmFar {
    const T* yh = nullptr;     // [F][ncl][K][R] downsweep coefficients
    const T* Upad = nullptr;   // [nleaf * cap][K] bases by leaf slot
    int64_t ncl = 0, first_leaf = 0;
    int K = 0;
};
// several right-hand sides: Y = Panel X (MFMA) + (B+M) X [+ U Y^] per (leaf, 64 rows, 64 rhs, field);
// x, y [F][N][R]
hipError_t launch_near_mm(const ApplyPlan& a, const PanelPlan& pp, const double* panel, int use_near,
                          const double* csr_val, int F, int R, int dtype, const void* x, void* y, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1, const MmFar<double>& fo = {});
hipError_t launch_near_mm(const ApplyPlan& a, const PanelPlan& pp, const float* panel, int use_near,
                          const double* csr_val, int F, int R, int dtype, const void* x, void* y, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1, const MmFar<float>& fo = {});
// tickets: [F][ncl] zero-initialised counters of the upsweep (left at zero by every launch).
// ev (optional, 5 events): start, start, near/upsweep kernel start/stop, end.
hipError_t launch_apply_single(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, const UpPlan& up,
                               const FarPlan& fp, int parts, int F, const double* csr_val, const OpData<double>& od,
                               int dtype, const void* x, void* y, unsigned int* tickets, hipStream_t st,
                               hipEvent_t* ev);
hipError_t launch_apply_single(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, const UpPlan& up,
                               const FarPlan& fp, int parts, int F, const double* csr_val, const OpData<float>& od,
                               int dtype, const void* x, void* y, unsigned int* tickets, hipStream_t st,
                               hipEvent_t* ev);

// leaf-slot copies of the bases and the output indices (fpde_far1.hip)
// p32[f][off[e]] = p64[f][off[e]] + val[f][e] (B + M added into the FP32 near panels)
hipError_t launch_panel_add_csr(int64_t nnz, int F, int64_t total, const int64_t* off, const double* val,
                                const double* p64, float* p32, hipStream_t st);
hipError_t launch_ell_values(int64_t n, int F, int64_t nnz, const int64_t* src, const double* val, double* out,
                             hipStream_t st);
hipError_t launch_pad_rows(int64_t nleaf, int64_t cap, int k, const int64_t* leaf_beg, const double* U,
                           const int64_t* perm, double* Upad, int64_t* perm_pad, hipStream_t st);
// far field of the one-vector apply after its upsweep (fpde_far1.hip): coupling
// sums z^ per far target (od.St, od.xh -> od.zh), then the downsweep walk and
// U y^ added to y
hipError_t launch_couple_single(const H2Tree& t, const FarPlan& fp, int F, const OpData<double>& od, hipStream_t st);
hipError_t launch_couple_single(const H2Tree& t, const FarPlan& fp, int F, const OpData<float>& od, hipStream_t st);
hipError_t launch_out_single(const ApplyPlan& a, const H2Tree& t, const FarPlan& fp, int F, const OpData<double>& od,
                             int dtype, void* y, hipStream_t st);
hipError_t launch_out_single(const ApplyPlan& a, const H2Tree& t, const FarPlan& fp, int F, const OpData<float>& od,
                             int dtype, void* y, hipStream_t st);

// ---------------------------------------------------------------- apply, many right-hand sides (fpde_batched.hip)

// K <= 32 and the leaf stages fit LDS (prec 0 double, 1 float)
bool batched_fits(const H2Tree& t, int64_t cap, int prec);
// far field in the operator precision (leaf upsweep, level transfers, MFMA coupling per
// target cluster, downsweep), then the near panels (MFMA) + B + M + U Y^ per leaf, all on
// st.  xh, yh: [F][ncl][K][R] workspaces of that precision; od.Upad required.
hipError_t launch_apply_batched(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, int parts, int F, int R,
                                const double* csr_val, const OpData<double>& od, double* xh, double* yh, int dtype,
                                const void* x, void* y, hipStream_t st, hipEvent_t* ev);
hipError_t launch_apply_batched(const ApplyPlan& a, const H2Tree& t, const PanelPlan& pp, int parts, int F, int R,
                                const double* csr_val, const OpData<float>& od, float* xh, float* yh, int dtype,
                                const void* x, void* y, hipStream_t st, hipEvent_t* ev);

// ---------------------------------------------------------------- adjoint (fpde_adjoint.hip, singular pairs in
// fpde_kernels.hip): d/ds_j and d/dkappa_j of sum_r w_r^T A_h u_r

// per pair and field: out[f][pair][12] (d/ds at the 6 cell-vertex slots, then d/dkappa)
hipError_t launch_adj_singular(int dim, int64_t np, const int32_t* pairs, const double* coords, int64_t n_nodes,
                               int F, const double* s, const double* kappa, double a_scale, double s_bar, int nq,
                               const double* g01, const double* w01, const double* w, const double* u, int64_t N,
                               int R, double* out, hipStream_t st);
struct AdjKnear {
    int dim, nqe, R, r;                      // r: the right-hand side of this launch
    int64_t nc, nq, N;
    const int32_t* cells;
    const double *qx, *qw, *qs, *qk, *lam;   // qk: sqrt(kappa) at the points
    const int64_t* icells;                   // interior cells
    const int64_t* cell_leaf_ptr;            // per interior-cell index: leaves whose patch holds it
    const int32_t* cell_leaf;
    const int64_t *near_ptr, *near_src;      // by target leaf index -> source leaf index
    const int64_t *patch_ptr, *patch_cell;   // by leaf index
    const int32_t* leaf_of_node;             // [M] leaf index of a dof, -1 for other nodes
    const double *w, *u;                     // [F][N][R]
    double a_scale;
};
// point densities Ds, Dk [F][nq] (accumulated)
hipError_t launch_adj_knear(const AdjKnear& P, int64_t n_icells, int F, double* Ds, double* Dk, hipStream_t st);
hipError_t launch_adj_c(int dim, int64_t nc, int nqe, const int32_t* cells, const uint8_t* cell_int,
                        const double* lam, const double* qw, const double* w, const double* u, int64_t N, int R,
                        int F, double* c, hipStream_t st);
hipError_t launch_adj_rho_near(const H2Tree& t, const int64_t* perm, const int64_t* near_ptr, const int64_t* near_src,
                               const double* qx, const double* qw, const double* qs, const double* qk,
                               const double* cq, int nqe, const int32_t* cells, int64_t nc, int64_t nq, int F,
                               double a_scale, double* Ds, double* Dk, hipStream_t st);
hipError_t launch_adj_rho_ext(int dim, int64_t nq, const double* qx, const double* qs, const double* qk,
                              const uint8_t* q_int, const double* cq, int F, double R, double s_out,
                              double k_out_sqrt, double a_scale, int n_theta, double* Ds, double* Dk,
                              hipStream_t st);
// gs, gk [F][M] += sum over the points of the cells of each node of lambda * D
hipError_t launch_adj_points(int64_t M, const int64_t* nc_ptr, const int64_t* nc_cell, const int8_t* nc_slot, int nqe,
                             const double* lam, const double* Ds, const double* Dk, int64_t nq, int F, double* gs,
                             double* gk, hipStream_t st);
// per Chebyshev node of every cluster: Gs, Gk [F][ncl][K]
hipError_t launch_adj_far(const H2Tree& t, double fac, double a_scale, const double* a, int64_t af, const double* b,
                          int64_t bf, int R, int F, double* Gs, double* Gk, hipStream_t st);
// out[f][i] += sum_e wts[e] src[f][idx[e]]   (wts NULL: 1)
hipError_t launch_adj_gather(int64_t n, const int64_t* ptr, const int64_t* idx, const double* wts, const double* src,
                             int64_t src_f, int F, double* out, int64_t out_f, hipStream_t st);

// ---------------------------------------------------------------- CG solve (fpde_solve.hip)

struct CgDims {
    int64_t N;      // rows per system
    int R, F;       // right-hand sides, fields: S = F * R systems
    int64_t nb;     // row blocks of the reductions (cg_row_blocks)
};
struct CgScalars {  // device arrays of S entries (n_active: one int)
    // rr: r . z of the committed iteration (z = D^-1 r with the Jacobi preconditioner, else r)
    double *rr, *rr_next, *alpha, *beta, *tol2;
    int *active, *active_next, *iters, *flags, *n_active;
    // Lanczos coefficients of the run: hist_a[k * S + s] = alpha_k, hist_b[k * S + s] = beta_k
    // for k < hist_cap (null: not recorded)
    double *hist_a = nullptr, *hist_b = nullptr;
    int hist_cap = 0;
};
enum { CG_DOT = 0, CG_UPDATE_UR = 1, CG_RESID = 2, CG_COPY_RP = 3, CG_UPDATE_P = 4 };
int64_t cg_row_blocks(int64_t N, int R, int F);
// One row-block pass (see fpde_solve.hip): CG_DOT part1 = a.b; CG_UPDATE_UR u += alpha a,
// r -= alpha b, part1 = r.r; CG_UPDATE_P p = a + beta p; CG_RESID r = b - a, part1 = r.r,
// part2 = b.b; CG_COPY_RP r = p = b, u = 0, part1 = b.b.  part_in: the partials the
// coefficient of CG_UPDATE_UR / CG_UPDATE_P is summed from.
// nb_in: partials per system in part_in (default: the pass's own block count)
// dinv [F][N] (null: no preconditioner): the Jacobi preconditioner z = D^-1 r.  With it
// CG_UPDATE_UR also stores r . r in part2 and CG_UPDATE_P stops on the r . r partials part_in2;
// CG_COPY_RP stores b . z in part1 and b . b in part2.
// v32: the CG vectors (a, b, u, r, p; not CG_COPY_RP's b) are FP32, the inner CG of a
// mixed-precision solve; CG_RESID always works on FP64 vectors.
hipError_t launch_cg_rowblock(int op, const CgDims& d, const void* a, const void* b, void* u, void* r, void* p,
                              double* part1, double* part2, const double* part_in, const CgScalars& c, hipStream_t st,
                              int64_t nb_in = -1, const double* dinv = nullptr, const double* part_in2 = nullptr,
                              bool v32 = false);
// part: b . z partials (rr of the first iteration); part_rr: b . b partials for the stopping
// threshold (null: part)
hipError_t launch_cg_start(const CgDims& d, const double* part, const double* bb0, double tau_in, double rtol,
                           const CgScalars& c, hipStream_t st, const double* part_rr = nullptr);
// dinv[f][i] = 1 / (diagonal of A_h) from the B + M diagonal entries and the panel entries of
// the leaf self-blocks: diag[f][i] = bm[f * nnz + bm_idx[i]] + panel[f * ptot + p_idx[i]]
hipError_t launch_jacobi_diag(int64_t N, int F, int64_t nnz, const int64_t* bm_idx, const double* bm, int64_t ptot,
                              const int64_t* p_idx, const double* panel, double* dinv, hipStream_t st);
hipError_t launch_cg_sum2(const CgDims& d, const double* part1, const double* part2, double* o1, double* o2,
                          hipStream_t st);
// u += d (d FP64, or FP32 with v32)
hipError_t launch_vec_add(int64_t n, const void* d, double* u, hipStream_t st, bool v32 = false);

// ---------------------------------------------------------------- static scratch (fpde_noalloc.hip)

// Size of the file-scope device scratch of the allocation-free apply: every GPU the
// library runs on holds one copy until the process ends.
constexpr size_t kScratchBytes = size_t(8) << 20;
// Device address of the current device's copy (hipGetSymbolAddress on the first call per device).
hipError_t scratch_address(void** out);
// p[0, n) = 0 for n 32-bit words
hipError_t launch_zero_words(int64_t n, uint32_t* p, hipStream_t st);

}  // namespace fpde
