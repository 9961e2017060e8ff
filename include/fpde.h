/*
 * fpde.h -- C ABI of libfpde: the decomposed stiffness operator of the
 * variable-order fractional diffusion problem on P1 simplicial meshes,
 * built and applied on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. 2 of Lei, Turkiyyah, Knio, "Finite element discretizations
 * for variable-order fractional diffusion problems"): find U in the P1 space
 * with U = 0 on the exterior region such that
 *     A(U,V) = int_{Omega_i} f V   for all V,
 *     A(U,V) = int int (U(x)-U(y)) (V(x)-V(y)) gamma(x,y) dy dx,
 *     gamma(x,y) = a(x,y) / |x-y|^{d+s(x)+s(y)},  a = a_scale sqrt(kappa(x) kappa(y)),
 * with 0 <= s <= s_bar < 1 and kappa > 0 (eq. i:s).
 *
 * The stiffness matrix is applied as A = B + K~ + M (Sec. 3, eq. e:decomp):
 *   B   singular near field of touching element pairs (Sec. 4), sparse;
 *   K~  H2 matrix of the smooth interaction of interior elements (Sec. 5):
 *       dense near leaf blocks + Chebyshev far blocks with nested bases;
 *   M   weighted mass matrix whose density rho is computed by a
 *       point-collocation H2 matrix-vector product (Sec. 6.2), plus the
 *       analytic density of an exterior beyond |x| = R (eq. e:rho).
 * B and M share one CSR pattern; the CSR, near blocks and H2 data live in
 * device memory owned by the operator.
 *
 * Conventions
 *   - Every function returns fpde_status (0 = FPDE_OK) and never throws.
 *     On error fpde_last_error() returns a thread-local message.
 *   - Host arrays passed to fpde_build are borrowed for the call only.
 *   - Device vectors are caller-owned, contiguous, layout [F][N][R]: field
 *     (order/diffusivity set) slowest, right-hand side fastest.  N is the
 *     number of interior nodes (dofs); the first N mesh nodes are the dofs.
 *   - hip_stream is a hipStream_t (NULL = default stream).  Work is enqueued
 *     on it; fpde_apply is asynchronous, fpde_solve synchronises.
 *   - One operator is not safe for concurrent calls on two streams.
 */
#ifndef FPDE_H
#define FPDE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FPDE_OK = 0,
    FPDE_EINVAL = -1,   /* malformed argument, mesh or option                    */
    FPDE_EDOMAIN = -2,  /* s outside [0, s_bar], s_bar >= 1, kappa <= 0          */
    FPDE_ENOMEM = -3,   /* device allocation failed or above max_device_bytes    */
    FPDE_EDEVICE = -4,  /* HIP runtime error                                     */
    FPDE_ENOCONV = -5,  /* solver reached maxit                                   */
    FPDE_ESTATE = -6    /* call not valid for this operator (e.g. plan-only)     */
} fpde_status;

/* Operator precision.  FPDE_PREC_MIXED keeps FP32 copies of the near panels, bases,
 * transfers and coupling matrices next to the FP64 data and applies with them
 * (products accumulated in FP32, added in FP64): with one right-hand side the rows of
 * B + M stay FP64; with several, B + M is added into the FP32 near panels and the
 * whole near field runs as one FP32 MFMA product (about 5e-7 relative to the FP64
 * apply on the square 256 workload). */
enum { FPDE_PREC_FP64 = 0, FPDE_PREC_MIXED = 1 };
enum { FPDE_F64 = 0, FPDE_F32 = 1 };

/* flags */
#define FPDE_FLAG_PLAN_ONLY 0x1ull   /* host planning only: no device work (for inspection) */
#define FPDE_FLAG_JACOBI    0x2ull   /* fpde_solve preconditions CG with the diagonal of A_h */

/* Simplicial mesh of Omega = closure(Omega_i) U Omega_e (Sec. 2.3).  Nodes
 * [0, n_dofs) are the nodes strictly inside Omega_i.  SoA layouts:
 * coords[k*n_nodes + v] is coordinate k of node v; cells[a*n_cells + c] is
 * vertex a of cell c.  cell_interior[c] = 1 iff cell c lies in Omega_i (the
 * mesh matches the interface).  exterior_radius R > 0 declares that the
 * exterior continues beyond the ball |x| = R (its density is analytic,
 * eq. e:rho); R = 0 means Omega_e is exactly the meshed exterior cells. */
typedef struct {
    int32_t dim;                 /* 1 or 2                                     */
    int64_t n_nodes;             /* M                                          */
    int64_t n_dofs;              /* N                                          */
    const double *coords;        /* [dim][n_nodes]                             */
    int64_t n_cells;
    const int32_t *cells;        /* [dim+1][n_cells]                           */
    const uint8_t *cell_interior;/* [n_cells]                                  */
    double exterior_radius;
} fpde_mesh;

/* Discretisation options.  fpde_opts_default() fills the values in brackets. */
typedef struct {
    int32_t precision;      /* FPDE_PREC_FP64 | FPDE_PREC_MIXED [FP64]                               */
    int32_t leaf_size;      /* max dofs per leaf of the KD tree of K~ (Sec. 5.1) [64]                 */
    int32_t leaf_size_rho;  /* max quadrature points per leaf of the density tree (Sec. 6.2) [64]     */
    int32_t cheb_p;         /* Chebyshev points per dimension; rank p^dim (eq. eq:interpolant) [5]    */
    double  eta;            /* centre-form admissibility eta*|C-C'| >= (D+D')/2 (Sec. 7) [1.0]         */
    int32_t nq_sing;        /* Gauss points per direction of the singular rules (Sec. 4) [3]          */
    int32_t nq_reg;         /* Gauss points per direction of the per-element rule (Sec. 5.2, 6.1) [3] */
    double  s_bar;          /* substitution bound of the singular rules, s <= s_bar < 1 [0.9]         */
    double  s_exterior;     /* order beyond the ball |x| = R (only if R > 0) [0]                       */
    double  kappa_exterior; /* diffusivity beyond the ball |x| = R [1]                                  */
    int32_t n_theta;        /* periodic trapezoid points of the exterior density (2D) [128]           */
    double  a_scale;        /* a(x,y) = a_scale sqrt(kappa(x) kappa(y)) [1]                            */
    uint64_t flags;         /* FPDE_FLAG_* [0]                                                         */
    uint64_t max_device_bytes; /* 0 = unlimited [0]                                                    */
    double  recompress_tol; /* > 0: algebraic recompression of the far field's nested bases (closing
                               remark of Sec. 5.3) at this relative tolerance: the Chebyshev bases are
                               orthogonalised, and each cluster keeps the directions of its total far
                               weight whose eigenvalues exceed tol^2 times the largest one in the tree,
                               padded to one rank r <= p^dim.  Needs p^dim <= 32.  Applies (any nrhs)
                               and solves then run the several-right-hand-side kernels with rank r;
                               fpde_apply_noalloc rejects such an operator, and fpde_apply_adjoint
                               differentiates the operator without recompression.  [0 = off]      */
} fpde_opts;

typedef struct {
    int64_t n_dofs, n_nodes, n_cells, n_fields;
    int64_t n_pairs_identical, n_pairs_edge, n_pairs_vertex;
    int64_t csr_nnz;
    int64_t k_clusters, k_levels, k_leaves, k_far, k_near, k_rank, k_leaf_cap;
    int64_t rho_points, rho_clusters, rho_levels, rho_far, rho_near;
    int64_t device_bytes;
    /* build phase times in milliseconds (device time measured with events) */
    double t_plan_ms, t_singular_ms, t_near_blocks_ms, t_bases_ms, t_rho_ms, t_mass_ms, t_total_ms;
    /* bytes streamed by one apply with one right-hand side (dominant arrays) */
    int64_t apply_bytes_near, apply_bytes_csr, apply_bytes_bases;
    /* algebraic recompression (recompress_tol > 0): uniform rank r (0 if off), the smallest
       and mean cluster rank before padding, and its build time */
    int64_t k_rank_rc, k_rank_rc_min;
    double k_rank_rc_mean, t_recompress_ms;
} fpde_stats_t;

typedef struct {
    int32_t iterations;      /* CG iterations (worst system, summed over passes) */
    double  rel_residual;    /* max over systems of ||F - A u|| / ||F|| at exit   */
    int32_t converged;
    int32_t refinements;     /* iterative-refinement passes                       */
    double  cond_estimate;   /* largest over systems of lambda_max / lambda_min of the
                                Lanczos matrix of the first CG pass (its first 2048
                                steps): a lower bound on the condition number of A_h,
                                or of D^-1 A_h with FPDE_FLAG_JACOBI; 0 if fewer than 2 steps */
} fpde_solve_info;

typedef struct fpde_op fpde_op;

/* Default options (see fpde_opts). */
fpde_status fpde_opts_default(fpde_opts *opts);

/* Gauss-Legendre rule on [0,1] used by every tensor rule of the library:
 * nodes01[i] = (t_i+1)/2, weights01[i] = w_i/2 with t_i, w_i the n-point
 * Legendre nodes/weights correctly rounded to double.  Host arrays of size n. */
fpde_status fpde_gauss_legendre(int32_t n, double *nodes01, double *weights01);

/* Build the operator (Alg. 1 of the paper: K~ by H2, rho at every quadrature
 * point, then B and M element by element).
 *   mesh      host mesh (borrowed)
 *   n_fields  F >= 1 independent (s, kappa) pairs sharing the mesh
 *   s, kappa  host [F][n_nodes] nodal P1 values
 *   opts      host options (NULL = defaults)
 *   out       receives the operator; free with fpde_destroy
 * Errors: FPDE_EINVAL (mesh/options), FPDE_EDOMAIN (s, kappa, s_bar),
 * FPDE_ENOMEM, FPDE_EDEVICE.  Validation happens before any device work. */
fpde_status fpde_build(const fpde_mesh *mesh, int32_t n_fields, const double *s,
                       const double *kappa, const fpde_opts *opts, fpde_op **out);

/* Parts of the operator for fpde_apply_parts. */
#define FPDE_PART_B      0x1
#define FPDE_PART_M      0x2
#define FPDE_PART_KNEAR  0x4
#define FPDE_PART_KFAR   0x8
#define FPDE_PART_ALL    0xF
/* With FPDE_PREC_MIXED: apply with the FP64 operator data instead of the
 * mixed-precision copies (ignored by an FP64 operator). */
#define FPDE_PART_FP64   0x10

/* y = A x for F fields and nrhs right-hand sides (Sec. 3: y = (B+M)x + K~x).
 *   dtype     FPDE_F64: x, y are double; FPDE_F32: float
 *   x, y      device [F][N][nrhs], must not alias
 * Asynchronous on hip_stream: kernel launches on that stream (on the
 * fallback paths for K > 32 or wide nrhs the far field runs on the operator's
 * side stream, forked from and joined back to hip_stream with events).  Calls on one operator
 * must not run concurrently from several host threads.
 * Errors: FPDE_EINVAL, FPDE_ESTATE, FPDE_EDEVICE. */
fpde_status fpde_apply(fpde_op *op, int32_t dtype, const void *x, void *y, int64_t nrhs,
                       void *hip_stream);

/* As fpde_apply restricted to a subset of FPDE_PART_* (for inspection), or
 * with FPDE_PART_ALL | FPDE_PART_FP64 for the FP64 apply of a mixed operator. */
fpde_status fpde_apply_parts(fpde_op *op, int32_t parts, int32_t dtype, const void *x, void *y,
                             int64_t nrhs, void *hip_stream);

/* fpde_apply without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same y = A x with one right-hand side per field (nrhs must
 * be 1) on the one-vector path (an operator with far blocks and panel rows
 * within 64 KiB), with the apply's workspace (cluster coefficients, coupling partial
 * sums and tickets, about (2 k + 2) F n_clusters + F k n_chunks words) taken
 * from a static device scratch of 8 MiB that the library holds on every GPU
 * it runs on until the process ends, instead of the operator's workspace.
 * Calls no hipMalloc, hipFree or allocating library routine.  Every call on
 * one GPU shares that GPU's scratch (cleared at the start of each call by a
 * fill kernel), so calls that overlap on one GPU, from any operators, race.
 *   dtype, x, y, hip_stream as fpde_apply; asynchronous on hip_stream.
 * Errors: FPDE_EINVAL (nrhs != 1, dtype, NULL vectors, an operator without the
 * one-vector path, or a workspace above the scratch size, reported with the
 * bytes needed), FPDE_ESTATE (plan-only), FPDE_EDEVICE. */
fpde_status fpde_apply_noalloc(fpde_op *op, int32_t dtype, const void *x, void *y, int64_t nrhs,
                               void *hip_stream);

/* Load vector of the weak form's right-hand side, F_i = int_{Omega_i} f psi_i
 * (Sec. 2.3: A(U, V) = int_{Omega_i} f V for the P1 test functions psi_i),
 * by the per-element rule of Sec. 5.2 with f P1-interpolated from its nodal
 * values.  f_nodal: device [n_nodes] double (read); F: device [N] double
 * (overwritten), caller-owned.  Asynchronous on hip_stream.
 * Errors: FPDE_EINVAL (NULL pointers), FPDE_ESTATE (plan-only), FPDE_EDEVICE. */
fpde_status fpde_load_vector(fpde_op *op, const double *f_nodal, double *F, void *hip_stream);

/* Solve A u = F by conjugate gradients (the paper solves with CG, Sec. 7) for
 * every field and right-hand side, each system independently.
 *   F, u      device [F][N][nrhs] double, must not alias; u holds the initial
 *             guess on entry and the solution on exit
 *   rtol      stop when ||F_s - A u_s||_2 <= rtol ||F_s||_2 for every system s,
 *             the residual computed with the FP64 apply
 *   maxit     bound on the total number of CG iterations
 * The solve is an iterative-refinement loop on the FP64 residual: each pass
 * runs unpreconditioned CG on A d = r from d = 0 and adds d to u.  An FP64
 * operator's CG runs to 0.5 rtol in one pass (a second pass only corrects
 * drift of the recursive residual); with FPDE_FLAG_JACOBI each pass is CG
 * preconditioned by the diagonal D of A_h (stopping still on ||r||); an FPDE_PREC_MIXED operator's CG uses the
 * mixed-precision apply and stops each pass at a relative reduction of
 * sqrt(rtol), clamped to [1e-7, 1e-2], and keeps its CG vectors in FP32 (dot
 * products in FP64) unless each field has one right-hand side on the fused
 * one-vector path.  CG iterations are launched back to
 * back on hip_stream; the host polls convergence every few iterations.  Synchronises hip_stream.  info (host, may be NULL): total
 * CG iterations of the worst system summed over passes, final worst relative
 * residual, converged flag, number of refinement passes.
 * Errors: FPDE_EINVAL, FPDE_ESTATE (plan-only), FPDE_ENOCONV (maxit reached,
 * stagnation or breakdown; u and info hold the last iterate), FPDE_EDEVICE. */
fpde_status fpde_solve(fpde_op *op, const double *F, double *u, int64_t nrhs, double rtol,
                       int32_t maxit, fpde_solve_info *info, void *hip_stream);

/* alpha times the gradient of J = sum_r w_r^T A_h(s, kappa) u_r with respect to the nodal
 * order s_j and diffusivity kappa_j of every mesh node and field: the
 * derivative of the discrete bilinear form of Sec. 2-3 (A_h as built, Thm. 6.2)
 * for fixed s_bar.  Every dependence goes through the kernel
 * a_scale sqrt(kappa(x) kappa(y)) |x-y|^{-(d+s(x)+s(y))} at the quadrature and
 * Chebyshev points of the singular rules (Sec. 4), the near and far blocks of
 * K~ (Sec. 5) and the density of M~ (Sec. 6.2, eq. e:rho); the P1 weights of
 * s and kappa at those points carry it to the nodes.  For u the solution of
 * A_h u = F and w the solution of A_h w = g, alpha = -1 gives dJ(u)/ds, the
 * gradient of an objective through the solve (A_h du = -(dA_h) u at fixed F).
 *   alpha       finite scale of both outputs (1 for the plain derivative)
 *   w, u        device [F][N][nrhs] double (dof vectors), must not alias the outputs
 *   grad_s,
 *   grad_kappa  device [F][n_nodes] double, overwritten (summed over nrhs)
 * Asynchronous on hip_stream.  Costs about one build of B, the near blocks and
 * the density (no operator data is re-stored).
 * Errors: FPDE_EINVAL, FPDE_ESTATE (plan-only operator, or partitions that are
 * not symmetric / nq_reg too large, reported by fpde_last_error), FPDE_EDEVICE. */
fpde_status fpde_apply_adjoint(fpde_op *op, double alpha, const double *w, const double *u, int64_t nrhs,
                               double *grad_s, double *grad_kappa, void *hip_stream);

/* Device-time profile of fpde_apply.  While profiling is on, each apply runs
 * the same kernels as without profiling, serialised on the apply's stream,
 * with HIP events: out = start-to-stop timestamps of the near-field kernel
 * (the dominant kernel, launched with hipExtLaunchKernelGGL events: CSR +
 * near leaf blocks, and for one right-hand side the far-field upsweep in the
 * same launch), far = far-field work enqueued before it (the H2 upsweep and
 * coupling of several right-hand sides; 0 for one), far_out = from the end
 * of the near-field kernel to the end of the apply (coupling, downsweep and
 * U yh added to y), total = whole apply.  ms_gather is 0 (the vectors are
 * read in place).  fpde_profile(op, 1, NULL) resets and
 * starts recording; fpde_profile(op, 0, out) stops, waits for the recorded
 * events and returns the sums. */
typedef struct {
    int64_t n_applies;
    double ms_gather, ms_far, ms_out, ms_far_out, ms_total;
} fpde_profile_t;
fpde_status fpde_profile(fpde_op *op, int32_t enable, fpde_profile_t *out);

/* Counts, memory and build-phase timings. */
fpde_status fpde_stats(const fpde_op *op, fpde_stats_t *stats);

/* Copy internal data to host memory for inspection and testing.
 * what: one of FPDE_EXPORT_*; field selects the (s, kappa) set where relevant.
 * dst NULL: only *count is set (number of elements).  Elements are int64 for
 * index data and double for values. */
enum {
    FPDE_EXPORT_CSR_ROWPTR = 1, /* int64 [N+1], rows in dof order                        */
    FPDE_EXPORT_CSR_COLS = 2,   /* int64 [nnz], dof indices                              */
    FPDE_EXPORT_CSR_B = 3,      /* double [nnz], values of B                             */
    FPDE_EXPORT_CSR_M = 4,      /* double [nnz], values of M                             */
    FPDE_EXPORT_K_PERM = 5,     /* int64 [N], dof at each position of the K tree order   */
    FPDE_EXPORT_K_LEAFPTR = 6,  /* int64 [leaves+1], tree-order ranges of the leaves     */
    FPDE_EXPORT_K_FAR = 7,      /* int64 [2*n_far], (target, source) heap cluster ids    */
    FPDE_EXPORT_K_NEAR = 8,     /* int64 [2*n_near], (target, source) heap cluster ids   */
    FPDE_EXPORT_RHO_PERM = 9,   /* int64 [n_q], quadrature point at each tree position   */
    FPDE_EXPORT_RHO_FAR = 10,   /* int64 [2*n_far]                                       */
    FPDE_EXPORT_RHO_NEAR = 11,  /* int64 [2*n_near]                                      */
    FPDE_EXPORT_RHO = 12,       /* double [n_q], density at interior points (0 elsewhere),
                                   point index = cell*nq_per_cell + local point          */
    FPDE_EXPORT_PAIRS = 13,     /* int64 [n_pairs*8]: kind(0 I,1 E,2 V), cell0, cell1,
                                   canonical vertices of cell0 (3), of cell1 tail (2)    */
    FPDE_EXPORT_K_BOXES = 14,   /* double [clusters*2*dim]: lo[dim], hi[dim] (extended)  */
    FPDE_EXPORT_RHO_BOXES = 15  /* double [clusters*2*dim]                               */
};
fpde_status fpde_export(const fpde_op *op, int32_t what, int32_t field, void *dst, int64_t *count);

/* Free the operator and all its device memory (NULL is allowed). */
void fpde_destroy(fpde_op *op);

/* Thread-local message of the last error ("" if none). */
const char *fpde_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FPDE_H */
