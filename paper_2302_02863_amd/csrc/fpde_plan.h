// Host-side planning structures (no device code).  Everything here is
// integer/geometric bookkeeping: touching pairs, cluster trees, block
// partitions, point location.  Floating-point steps that decide structure
// (tree splits, admissibility, quadrature point coordinates) use a fixed
// operation order and are compiled without contraction so the structure is
// reproducible bit for bit.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fpde {

struct HostMesh {
    int dim = 0;
    int64_t M = 0, N = 0, nc = 0;
    std::vector<double> X;          // [dim][M]
    std::vector<int32_t> C;         // [dim+1][nc]
    std::vector<uint8_t> interior;  // [nc]
    double R = 0.0;
    double x(int k, int64_t v) const { return X[k * M + v]; }
    int32_t v(int a, int64_t c) const { return C[a * nc + c]; }
};

// 1D Gauss-Legendre on [0,1] (correctly rounded Legendre nodes/weights, then (t+1)/2, w/2)
void gauss_legendre01(int n, double* x, double* w);

// Per-element rule on the reference simplex (Sec. 5.2 collapsed coordinates)
struct ElementRule {
    int nqe = 0;
    std::vector<double> xh;   // [dim][nqe]
    std::vector<double> wh;   // [nqe]
    std::vector<double> lam;  // [dim+1][nqe] reference shape values
};
ElementRule element_rule(int dim, int n);

struct QuadPoints {
    int64_t nq = 0;
    int nqe = 0;
    std::vector<double> x;    // [dim][nq]
    std::vector<double> w;    // [nq]
    std::vector<uint8_t> q_int;  // [nq] point lies in an interior cell
};
QuadPoints quad_points(const HostMesh& m, const ElementRule& r);

// node -> cells, sorted by cell id, with the node's vertex slot
struct NodeCells {
    std::vector<int64_t> ptr, cell;
    std::vector<int8_t> slot;
};
NodeCells node_cells(const HostMesh& m);

// Touching pairs in canonical orientation (kind 0 identical, 1 edge, 2 vertex)
struct Pair {
    int32_t kind, c0, c1;
    int32_t v[6];   // canonical vertices: cell0 (3), cell1 (3); 1D: (2),(2)
};
std::vector<Pair> touching_pairs(const HostMesh& m, const NodeCells& nc);
// the pairs whose first cell lies in [cbeg, cend), appended to out in cell order
void touching_pairs_range(const HostMesh& m, const NodeCells& nc, int64_t cbeg, int64_t cend, std::vector<Pair>& out);
// local dof list of a pair (global node ids), returns count
int pair_dofs(const HostMesh& m, const Pair& p, int32_t* out);

struct Tree {
    int dim = 0, L = 0;
    int64_t n = 0, ncl = 0;
    std::vector<int64_t> perm, beg, end;
    std::vector<double> lo, hi;   // [ncl][dim] boxes used for admissibility / interpolation
    int64_t first_leaf() const { return (int64_t(1) << L) - 1; }
    int64_t nleaf() const { return int64_t(1) << L; }
};
// KD tree over points pts[k*stride + i] (i < n), global ids = i
Tree kd_tree(int dim, const double* pts, int64_t stride, int64_t n, int leaf);
void point_boxes(Tree& t, const double* pts, int64_t stride);

bool admissible(int dim, const double* lo_a, const double* hi_a, const double* lo_b,
                const double* hi_b, double eta, double min_dist);

// sorts (a, b) pairs with 0 <= a < ncl by a, then b (a counting sort on a, then
// each bucket by b; the result does not depend on the host threads' schedule)
void sort_pairs(std::vector<std::pair<int64_t, int64_t>>& v, int64_t ncl);

// dual-tree partition; a pair is far only if admissible and its boxes are more than
// hc[a] + hc[b] apart (hc == nullptr: more than 0); skip_target[c] != 0 prunes targets
void partition(const Tree& t, double eta, const std::vector<double>* hc,
               const std::vector<uint8_t>* skip_target,
               std::vector<std::pair<int64_t, int64_t>>& far,
               std::vector<std::pair<int64_t, int64_t>>& near);

// Chebyshev axes of a box: out[k*p + a]
void cheb_axes(int dim, const double* lo, const double* hi, int p, double* out);

// Point location: the cell holding a point and its barycentrics (nearest node outside the mesh)
struct Locator {
    const HostMesh* m = nullptr;
    double lo[2], inv[2];
    int64_t nb[2];
    std::vector<int64_t> cptr, cells;   // bucket -> cells
    std::vector<int64_t> nptr, nodes;   // bucket -> nodes
    void build(const HostMesh& mesh);
    // returns cell >= 0 and barycentrics, or -1 and nearest node in *node
    int64_t locate(const double* p, double* lam, int64_t* node) const;
};

// largest edge length of every cell
std::vector<double> cell_diameters(const HostMesh& m);
// per cluster: the largest h_point[i] over its member points i
std::vector<double> cluster_h(const Tree& t, const double* h_point);

}  // namespace fpde
