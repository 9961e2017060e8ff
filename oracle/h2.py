"""H2-consistent operator, evaluated entrywise (oracle; test infrastructure).

Cluster tree (Sec. 5.1): KD tree by repeated median splits along the largest
extent of the cluster's point bounding box.  Readings of details the paper
leaves open (shared with the library):
  * uniform depth L = smallest L with ceil(n / 2^L) <= leaf size;
  * split axis = largest extent, ties -> lowest axis; points are ordered by
    (coordinate, global id); the left child takes the first floor(n/2);
  * the dual traversal starts at (root, root) and refines both clusters.

Admissibility, centre form used in the paper's experiments (Sec. 7):
  eta * |C - C'| >= (D + D') / 2  (C centre, D diagonal of the box), plus
  * for K~: boxes extended to the supports of the cluster's basis functions
    (omega^e, Sec. 5.1) and dist(omega^e, omega^e') > 0, so no far block
    contains a touching element pair;
  * for the density: plain point boxes and dist > h_sigma + h_sigma', h_sigma
    the largest diameter of the cells that hold the cluster's points, so no far
    block pairs points of touching cells and gamma_T = gamma on it (the
    assumption stated with eq. i:addmi-q; two points of touching cells are at
    most diam + diam' apart).  On a quasi-uniform mesh this is the bound
    2 h_max; on a graded exterior it stays local.

Far blocks (eq. eq:interpolant, eq:triple_product): tensor Lagrange
interpolation at p first-kind Chebyshev points per dimension on the box,
  K~_ij = -2 sum_{alpha,beta} U_s[i,alpha] gamma(xi_alpha, xi'_beta) U_s'[j,beta],
  U_s[i,alpha] = sum_{tau in S_i} sum_{q in tau} w psi_i(q) l_alpha(q)
(basis integrals with the same per-element rule as the near field).  Bases are
computed directly for every cluster (no nested transfer), so the library's
nested bases are checked against them.  s and kappa at Chebyshev nodes: P1
interpolation (nearest node outside the mesh).  Near leaf blocks: the exact
entries of K (eq. e:k-near).

Density (Sec. 6.2, eq. eq:matvec): one point tree over all of Q; for a target
q in Q^int,
  rho~(q) = sum_near sum_{q'} gamma_T(q,q') w'
          + sum_far sum_{alpha,beta} l_alpha(q) gamma(xi_alpha, xi'_beta) m_beta,
  m_beta = sum_{q' in source} l'_beta(q') w'.

Pinned by tests/test_oracle_h2.py: the interpolation error of K~ and rho~
against the exact split decays with p, the partition covers every index pair
exactly once, far blocks contain no touching cell pairs.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .fields import field_at_points, gamma
from .assembly import _qdata, touching_cells, _gamma_block, _shape_matrix, mass_from_rho, rho_exterior_at
from .singular import assemble_B


# ----------------------------------------------------------------------------
# tree, boxes, partition
# ----------------------------------------------------------------------------

class ClusterTree:
    """Complete binary KD tree in heap order (root 0, children 2c+1, 2c+2)."""

    def __init__(self, pts: np.ndarray, ids: np.ndarray, leaf: int):
        n = pts.shape[1]
        L = 0
        while -(-n // (1 << L)) > leaf:
            L += 1
        self.L = L
        self.n_clusters = (1 << (L + 1)) - 1
        self.members = [None] * self.n_clusters
        self.members[0] = np.arange(n)
        for c in range((1 << L) - 1):
            idx = self.members[c]
            p = pts[:, idx]
            ext = p.max(axis=1) - p.min(axis=1)
            axis = int(np.argmax(ext))           # first maximum = lowest axis on ties
            order = np.lexsort((ids[idx], p[axis]))
            half = idx.size // 2
            self.members[2 * c + 1] = idx[order[:half]]
            self.members[2 * c + 2] = idx[order[half:]]

    def level(self, c):
        return int(math.floor(math.log2(c + 1)))

    def is_leaf(self, c):
        return c >= (1 << self.L) - 1

    def leaves(self):
        return range((1 << self.L) - 1, self.n_clusters)


def box_of(pts):
    return pts.min(axis=1), pts.max(axis=1)


def _admissible(lo_a, hi_a, lo_b, hi_b, eta, min_dist):
    d = lo_a.size
    s2 = 0.0
    for k in range(d):
        dc = 0.5 * (lo_a[k] + hi_a[k]) - 0.5 * (lo_b[k] + hi_b[k])
        s2 = s2 + dc * dc
    dcent = math.sqrt(s2)
    Da = 0.0
    Db = 0.0
    g2 = 0.0
    for k in range(d):
        wa = hi_a[k] - lo_a[k]
        wb = hi_b[k] - lo_b[k]
        Da = Da + wa * wa
        Db = Db + wb * wb
        gap = max(0.0, lo_b[k] - hi_a[k], lo_a[k] - hi_b[k])
        g2 = g2 + gap * gap
    Da = math.sqrt(Da)
    Db = math.sqrt(Db)
    return (eta * dcent >= 0.5 * (Da + Db)) and (math.sqrt(g2) > min_dist)


def cell_diameters(mesh):
    """Largest edge length of every cell."""
    X = mesh.coords[:, mesh.cells]                 # (dim, dim+1, nc)
    k = mesh.dim + 1
    h = np.zeros(mesh.cells.shape[1])
    for a in range(k):
        for b in range(a + 1, k):
            h = np.maximum(h, np.sqrt(((X[:, a] - X[:, b]) ** 2).sum(axis=0)))
    return h


def cluster_h(tree, h_point):
    """Per cluster: the largest of h_point over its members (h_point: the diameter of
    each point's cell)."""
    out = np.zeros(tree.n_clusters)
    for c in range(tree.n_clusters - 1, -1, -1):
        if tree.is_leaf(c):
            out[c] = h_point[tree.members[c]].max() if tree.members[c].size else 0.0
        else:
            out[c] = max(out[2 * c + 1], out[2 * c + 2])
    return out


def partition(tree, lo, hi, eta, hc=None):
    """Dual traversal from (root, root); ``hc``: per-cluster separation, a pair is far
    only if its boxes are more than hc[a] + hc[b] apart (None: more than 0)."""
    far, near = [], []
    stack = [(0, 0)]
    while stack:
        a, b = stack.pop()
        min_dist = 0.0 if hc is None else hc[a] + hc[b]
        if _admissible(lo[a], hi[a], lo[b], hi[b], eta, min_dist):
            far.append((a, b))
        elif tree.is_leaf(a):
            near.append((a, b))
        else:
            for ca in (2 * a + 1, 2 * a + 2):
                for cb in (2 * b + 1, 2 * b + 2):
                    stack.append((ca, cb))
    return far, near


# ----------------------------------------------------------------------------
# Chebyshev interpolation
# ----------------------------------------------------------------------------

def cheb_nodes(lo, hi, p):
    """Tensor first-kind Chebyshev nodes on a box; (dim, p^dim), dim 0 fastest."""
    d = lo.size
    D = math.sqrt(sum((hi[k] - lo[k]) ** 2 for k in range(d)))
    t = np.cos((2.0 * np.arange(p) + 1.0) * np.pi / (2.0 * p))
    axes = []
    for k in range(d):
        w = max(hi[k] - lo[k], 1e-12 * D)
        axes.append(0.5 * (lo[k] + hi[k]) + 0.5 * w * t)
    if d == 1:
        return axes[0][None, :], axes
    g0, g1 = np.meshgrid(axes[0], axes[1], indexing="xy")   # g0[a1, a0]
    return np.stack([g0.ravel(), g1.ravel()]), axes


def lagrange(axes, x):
    """Tensor Lagrange basis at points x (dim, n) -> (p^dim, n), dim 0 fastest."""
    vals = []
    for k, t in enumerate(axes):
        p = t.size
        Lk = np.ones((p, x.shape[1]))
        for a in range(p):
            for b in range(p):
                if b != a:
                    Lk[a] *= (x[k] - t[b]) / (t[a] - t[b])
        vals.append(Lk)
    if len(axes) == 1:
        return vals[0]
    p0 = axes[0].size
    p1 = axes[1].size
    return (vals[1][:, None, :] * vals[0][None, :, :]).reshape(p0 * p1, x.shape[1])


# ----------------------------------------------------------------------------
# K~ (Sec. 5)
# ----------------------------------------------------------------------------

def node_tree(mesh, opts):
    N = mesh.n_dofs
    pts = mesh.coords[:, :N]
    tree = ClusterTree(pts, np.arange(N), opts["leaf_size"])
    # extended boxes: all vertices of the cells in the supports of the members
    node_cells = [[] for _ in range(mesh.n_nodes)]
    for c in range(mesh.n_cells):
        for v in mesh.cells[:, c]:
            node_cells[int(v)].append(c)
    lo = np.zeros((tree.n_clusters, mesh.dim))
    hi = np.zeros((tree.n_clusters, mesh.dim))
    for c in range(tree.n_clusters):
        cl = sorted({cc for i in tree.members[c] for cc in node_cells[int(i)]})
        verts = np.unique(mesh.cells[:, cl])
        lo[c], hi[c] = box_of(mesh.coords[:, verts])
    return tree, lo, hi, node_cells


def basis_direct(mesh, Q, node_cells, members, axes):
    """U[i, alpha] for the given member dofs, computed directly (eq. eq:triple_product)."""
    nqe = Q["nqe"]
    k = int(np.prod([a.size for a in axes]))
    U = np.zeros((members.size, k))
    for r, i in enumerate(members):
        for c in node_cells[int(i)]:
            slot = int(np.flatnonzero(mesh.cells[:, c] == i)[0])
            pts = np.arange(c * nqe, (c + 1) * nqe)
            lval = lagrange(axes, Q["x"][:, pts])                  # (k, nqe)
            U[r] += lval @ (Q["w"][pts] * Q["lam"][slot, pts])
    return U


def _node_fields(mesh, s, kappa, nodes):
    return field_at_points(mesh, s, nodes), field_at_points(mesh, kappa, nodes)


def assemble_K_h2(mesh, s, kappa, opts, K_exact=None, return_parts=False):
    s = s.reshape(-1)
    kappa = kappa.reshape(-1)
    N = mesh.n_dofs
    p = opts["cheb_p"]
    tree, lo, hi, node_cells = node_tree(mesh, opts)
    far, near = partition(tree, lo, hi, opts["eta"])
    Q = _qdata(mesh, s, kappa, opts["nq_reg"])
    if K_exact is None:
        from .assembly import assemble_split
        K_exact = assemble_split(mesh, s, kappa, opts)["K"]
    K = np.zeros((N, N), dtype=np.result_type(s, kappa, np.float64))
    for a, b in near:
        ra, rb = tree.members[a], tree.members[b]
        K[np.ix_(ra, rb)] = K_exact[np.ix_(ra, rb)]
    cache = {}

    def cl(c):
        if c not in cache:
            nodes, axes = cheb_nodes(lo[c], hi[c], p)
            sn, kn = _node_fields(mesh, s, kappa, nodes)
            U = basis_direct(mesh, Q, node_cells, tree.members[c], axes)
            cache[c] = (nodes, sn, kn, U)
        return cache[c]

    for a, b in far:
        na, sa, ka, Ua = cl(a)
        nb, sb_, kb, Ub = cl(b)
        S = -2.0 * gamma(mesh.dim, opts["a_scale"], na[:, :, None], nb[:, None, :],
                         sa[:, None], sb_[None, :], ka[:, None], kb[None, :])
        K[np.ix_(tree.members[a], tree.members[b])] = Ua @ S @ Ub.T
    if return_parts:
        return K, {"tree": tree, "lo": lo, "hi": hi, "far": far, "near": near, "cache": cache}
    return K


# ----------------------------------------------------------------------------
# rho~ (Sec. 6.2)
# ----------------------------------------------------------------------------

def rho_h2(mesh, s, kappa, opts, Q=None, return_parts=False):
    s = s.reshape(-1)
    kappa = kappa.reshape(-1)
    if Q is None:
        Q = _qdata(mesh, s, kappa, opts["nq_reg"])
    p = opts["cheb_p"]
    nq = Q["w"].size
    tree = ClusterTree(Q["x"], np.arange(nq), opts["leaf_size_rho"])
    lo = np.zeros((tree.n_clusters, mesh.dim))
    hi = np.zeros((tree.n_clusters, mesh.dim))
    for c in range(tree.n_clusters):
        lo[c], hi[c] = box_of(Q["x"][:, tree.members[c]])
    hc = cluster_h(tree, cell_diameters(mesh)[Q["cell"]])
    far, near = partition(tree, lo, hi, opts["eta"], hc)
    T = touching_cells(mesh)
    is_int = mesh.cell_interior[Q["cell"]] > 0
    rho = np.zeros(nq, dtype=np.result_type(s, kappa, np.float64))
    for a, b in near:
        ta = tree.members[a][is_int[tree.members[a]]]
        if ta.size == 0:
            continue
        G = _gamma_block(mesh, opts, Q, ta, tree.members[b], T)
        rho[ta] += G @ Q["w"][tree.members[b]]
    cache = {}

    def cl(c):
        if c not in cache:
            nodes, axes = cheb_nodes(lo[c], hi[c], p)
            sn, kn = _node_fields(mesh, s, kappa, nodes)
            Lm = lagrange(axes, Q["x"][:, tree.members[c]])        # (k, |c|)
            cache[c] = (nodes, sn, kn, Lm)
        return cache[c]

    for a, b in far:
        ta_mask = is_int[tree.members[a]]
        if not ta_mask.any():
            continue
        na, sa, ka, La = cl(a)
        nb, sb_, kb, Lb = cl(b)
        S = gamma(mesh.dim, opts["a_scale"], na[:, :, None], nb[:, None, :],
                  sa[:, None], sb_[None, :], ka[:, None], kb[None, :])
        mb = Lb @ Q["w"][tree.members[b]]
        rho[tree.members[a]] += La.T @ (S @ mb)
    qi = np.flatnonzero(is_int)
    if return_parts:
        return rho[qi], {"tree": tree, "lo": lo, "hi": hi, "far": far, "near": near, "Q": Q, "qi": qi}
    return rho[qi]


def assemble_h2(mesh, s, kappa, opts, split=None):
    """The approximate operator A_h = Q_B + K~ + Q_M^{n,p} of Thm. 6.2 (dense)."""
    from .assembly import assemble_split
    s = s.reshape(-1)
    kappa = kappa.reshape(-1)
    if split is None:
        split = assemble_split(mesh, s, kappa, opts)
    Q = split["Q"]
    qi = split["qi"]
    Kt = assemble_K_h2(mesh, s, kappa, opts, K_exact=split["K"])
    rt = rho_h2(mesh, s, kappa, opts, Q=Q) + rho_exterior_at(mesh, s, kappa, opts, Q, qi)
    Mt = mass_from_rho(mesh, Q, qi, rt, mesh.n_dofs)
    return {"B": split["B"], "K": Kt, "M": Mt, "rho": rt, "split": split}
