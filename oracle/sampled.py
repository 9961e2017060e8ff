"""Individual rows of A_h x at full size (oracle; test infrastructure).

The dense oracle cannot hold the large workloads (16129 dofs -> 2 GB dense,
1.18M quadrature points).  This module computes single rows of
A_h x = (B + K~ + M~) x from the same definitions as ``oracle.singular``,
``oracle.assembly`` and ``oracle.h2``:

* B row i: every touching pair with a cell in the support of psi_i,
  evaluated by the singular rules in canonical orientation (weight 2 / 1).
* K~ row i: the block row of i in the dual-tree partition of the KD tree of
  the dofs (Sec. 5): near leaf blocks by the separated-pair product rule with
  the mesh-dependent kernel, far blocks by Chebyshev interpolation with bases
  computed directly for each cluster (no nested transfers).
* M~ row i: 2 sum_q w psi_i(q) rho~(q) sum_j psi_j(q) x_j over the quadrature
  points q of the cells around i, with rho~ at those points from the
  point-collocation partition of Sec. 6.2 restricted to the clusters that
  contain them (identical to the full partition on those targets), plus the
  exterior density beyond R.

Point location for s and kappa at Chebyshev nodes uses a bucket grid of cell
centroids (every cell that contains a point has its centroid within h_max of
it), choosing the lowest-id containing cell as ``oracle.fields.locate`` does.
"""
from __future__ import annotations

import math

import numpy as np

from .assembly import _qdata, rho_exterior_at
from .fields import gamma
from .h2 import ClusterTree, box_of, cheb_nodes, cluster_h, cell_diameters, lagrange, _admissible
from .singular import canonical_pair, pair_local_dofs, pair_matrix


class _Locator:
    def __init__(self, mesh):
        self.m = mesh
        X = mesh.coords[:, mesh.cells]                    # (d, d+1, nc)
        self.cent = X.mean(axis=1)                        # (d, nc)
        self.h = mesh.h_max()
        self.lo = mesh.coords.min(axis=1) - self.h
        self.nb = np.maximum(1, np.ceil((mesh.coords.max(axis=1) + self.h - self.lo) / self.h)).astype(int)
        b = np.floor((self.cent - self.lo[:, None]) / self.h).astype(int)
        key = b[0] if mesh.dim == 1 else b[0] + self.nb[0] * b[1]
        order = np.argsort(key, kind="stable")
        self.key_sorted = key[order]
        self.cell_sorted = order

    def _candidates(self, p):
        b = np.floor((p - self.lo) / self.h).astype(int)
        keys = []
        if self.m.dim == 1:
            keys = [b[0] + o for o in (-1, 0, 1)]
        else:
            for o1 in (-1, 0, 1):
                for o0 in (-1, 0, 1):
                    keys.append((b[0] + o0) + self.nb[0] * (b[1] + o1))
        out = []
        for k in keys:
            lo = np.searchsorted(self.key_sorted, k, side="left")
            hi = np.searchsorted(self.key_sorted, k, side="right")
            out.append(self.cell_sorted[lo:hi])
        c = np.concatenate(out)
        return np.sort(c)

    def value(self, field, p, tol=1e-12):
        m = self.m
        c = self._candidates(p)
        if c.size:
            X = m.coords[:, m.cells[:, c]]                 # (d, d+1, ncand)
            if m.dim == 1:
                t = (p[0] - X[0, 0]) / (X[0, 1] - X[0, 0])
                L = np.stack([1.0 - t, t])
            else:
                P0 = X[:, 0]
                e1 = X[:, 1] - P0
                e2 = X[:, 2] - P0
                den = e1[0] * e2[1] - e1[1] * e2[0]
                dx = p[:, None] - P0
                b1 = (dx[0] * e2[1] - dx[1] * e2[0]) / den
                b2 = (e1[0] * dx[1] - e1[1] * dx[0]) / den
                L = np.stack([1.0 - b1 - b2, b1, b2])
            hit = np.flatnonzero((L >= -tol).all(axis=0))
            if hit.size:                                   # candidates are sorted: lowest cell id
                j = hit[0]
                v = field[m.cells[0, c[j]]] * L[0, j]
                for a in range(1, m.dim + 1):
                    v = v + field[m.cells[a, c[j]]] * L[a, j]
                return v
        d2 = ((m.coords - p[:, None]) ** 2).sum(axis=0)
        return field[int(np.argmin(d2))]


class SampledOracle:
    def __init__(self, mesh, s, kappa, opts):
        self.m = mesh
        self.s = np.asarray(s, dtype=np.float64).reshape(-1)
        self.k = np.asarray(kappa, dtype=np.float64).reshape(-1)
        self.o = opts
        m = mesh
        N = m.n_dofs
        self.Q = _qdata(m, self.s, self.k, opts["nq_reg"])
        self.nqe = self.Q["nqe"]
        # node -> cells
        flat = m.cells.ravel()
        cell_of = np.tile(np.arange(m.n_cells), m.dim + 1)
        order = np.argsort(flat, kind="stable")
        self.nc_ptr = np.searchsorted(flat[order], np.arange(m.n_nodes + 1))
        self.nc_cell = cell_of[order]
        self.loc = _Locator(m)
        # K tree with boxes extended to the supports of the members
        self.kt = ClusterTree(m.coords[:, :N], np.arange(N), opts["leaf_size"])
        kt = self.kt
        d = m.dim
        self.klo = np.zeros((kt.n_clusters, d))
        self.khi = np.zeros((kt.n_clusters, d))
        for c in range(kt.n_clusters - 1, -1, -1):
            if kt.is_leaf(c):
                cl = np.unique(np.concatenate([self._cells_of(i) for i in kt.members[c]]))
                verts = np.unique(m.cells[:, cl])
                self.klo[c], self.khi[c] = box_of(m.coords[:, verts])
            else:
                self.klo[c] = np.minimum(self.klo[2 * c + 1], self.klo[2 * c + 2])
                self.khi[c] = np.maximum(self.khi[2 * c + 1], self.khi[2 * c + 2])
        self.leaf_of_dof = np.empty(N, dtype=np.int64)
        for c in kt.leaves():
            self.leaf_of_dof[kt.members[c]] = c
        # density tree over all quadrature points (point boxes)
        self.rt = ClusterTree(self.Q["x"], np.arange(self.Q["w"].size), opts["leaf_size_rho"])
        rt = self.rt
        self.rlo = np.zeros((rt.n_clusters, d))
        self.rhi = np.zeros((rt.n_clusters, d))
        for c in range(rt.n_clusters - 1, -1, -1):
            if rt.is_leaf(c):
                self.rlo[c], self.rhi[c] = box_of(self.Q["x"][:, rt.members[c]])
            else:
                self.rlo[c] = np.minimum(self.rlo[2 * c + 1], self.rlo[2 * c + 2])
                self.rhi[c] = np.maximum(self.rhi[2 * c + 1], self.rhi[2 * c + 2])
        self.leaf_of_q = np.empty(self.Q["w"].size, dtype=np.int64)
        for c in rt.leaves():
            self.leaf_of_q[rt.members[c]] = c
        self.rh = cluster_h(rt, cell_diameters(m)[self.Q["cell"]])
        self._xhat = {}
        self._xhat_of = None      # the vector the cached coefficients belong to
        self._mom = {}
        self._nodes = {}

    # ------------------------------------------------------------------ helpers
    def _cells_of(self, v):
        return self.nc_cell[self.nc_ptr[v]:self.nc_ptr[v + 1]]

    def _cells_touching(self, c):
        vs = self.m.cells[:, c]
        return np.unique(np.concatenate([self._cells_of(v) for v in vs]))

    def _touch(self, ca, cb):
        """Boolean (len(ca), len(cb)): cells share a vertex."""
        A = self.m.cells[:, ca]
        B = self.m.cells[:, cb]
        t = np.zeros((ca.size, cb.size), dtype=bool)
        for a in range(A.shape[0]):
            for b in range(B.shape[0]):
                t |= A[a][:, None] == B[b][None, :]
        return t

    def _cluster_nodes(self, key, lo, hi):
        if key not in self._nodes:
            p = self.o["cheb_p"]
            nodes, axes = cheb_nodes(lo, hi, p)
            sn = np.array([self.loc.value(self.s, nodes[:, a]) for a in range(nodes.shape[1])])
            kn = np.array([self.loc.value(self.k, nodes[:, a]) for a in range(nodes.shape[1])])
            self._nodes[key] = (nodes, axes, sn, kn)
        return self._nodes[key]

    def _dof_points(self, i):
        """Quadrature points of the cells around dof i with w * psi_i(q)."""
        cells = self._cells_of(i)
        pts, wpsi = [], []
        for c in cells:
            slot = int(np.flatnonzero(self.m.cells[:, c] == i)[0])
            q = np.arange(c * self.nqe, (c + 1) * self.nqe)
            pts.append(q)
            wpsi.append(self.Q["w"][q] * self.Q["lam"][slot, q])
        return np.concatenate(pts), np.concatenate(wpsi)

    def _basis_row(self, i, axes):
        q, wpsi = self._dof_points(i)
        return lagrange(axes, self.Q["x"][:, q]) @ wpsi

    def _xhat_cluster(self, c, x):
        """U_c^T x_c with the basis of cluster c computed directly (cached for the current x)."""
        if self._xhat_of is None or self._xhat_of.shape != x.shape or not np.array_equal(self._xhat_of, x):
            self._xhat = {}
            self._xhat_of = np.array(x, copy=True)
        if c not in self._xhat:
            nodes, axes, sn, kn = self._cluster_nodes(("k", c), self.klo[c], self.khi[c])
            acc = np.zeros(nodes.shape[1])
            for i in self.kt.members[c]:
                if x[i] != 0.0:
                    acc += self._basis_row(int(i), axes) * x[i]
            self._xhat[c] = acc
        return self._xhat[c]

    # ------------------------------------------------------------------ rows
    def row_B(self, i, x):
        m = self.m
        N = m.n_dofs
        pairs = set()
        for c in self._cells_of(i):
            for c2 in self._cells_touching(c):
                a, b = (int(c), int(c2)) if c <= c2 else (int(c2), int(c))
                pairs.add((a, b))
        tot = 0.0
        for a, b in sorted(pairs):
            kind, v0, v1 = canonical_pair(m, a, b)
            loc = pair_local_dofs(m, kind, v0, v1)
            if i not in loc:
                continue
            L = pair_matrix(m, self.s, self.k, self.o, kind, v0, v1)
            wgt = 1.0 if kind == "I" else 2.0
            ai = loc.index(i)
            for bb, gb in enumerate(loc):
                if gb < N:
                    tot += wgt * L[ai, bb] * x[gb]
        return tot

    def _k_near_entry_row(self, i, leaf_src, x):
        """sum_{j in leaf} K_exact[i, j] x_j (separated pairs, gamma_T)."""
        m = self.m
        qi, wpsi_i = self._dof_points(i)
        ci = qi // self.nqe
        tot = 0.0
        for j in self.kt.members[leaf_src]:
            if x[j] == 0.0:
                continue
            qj, wpsi_j = self._dof_points(int(j))
            cj = qj // self.nqe
            G = gamma(m.dim, self.o["a_scale"], self.Q["x"][:, qi, None], self.Q["x"][:, None, qj],
                      self.Q["s"][qi, None], self.Q["s"][None, qj], self.Q["k"][qi, None], self.Q["k"][None, qj])
            G[self._touch(ci, cj)] = 0.0
            tot += -2.0 * (wpsi_i @ G @ wpsi_j) * x[j]
        return tot

    def row_K(self, i, x):
        kt = self.kt
        leaf = int(self.leaf_of_dof[i])
        path = []
        c = leaf
        while True:
            path.append(c)
            if c == 0:
                break
            c = (c - 1) // 2
        on_path = set(path)
        tot = 0.0
        stack = [(0, 0)]
        eta = self.o["eta"]
        while stack:
            a, b = stack.pop()
            if _admissible(self.klo[a], self.khi[a], self.klo[b], self.khi[b], eta, 0.0):
                na, axa, sa, ka = self._cluster_nodes(("k", a), self.klo[a], self.khi[a])
                nb, axb, sb, kb = self._cluster_nodes(("k", b), self.klo[b], self.khi[b])
                S = -2.0 * gamma(self.m.dim, self.o["a_scale"], na[:, :, None], nb[:, None, :], sa[:, None],
                                 sb[None, :], ka[:, None], kb[None, :])
                tot += self._basis_row(i, axa) @ (S @ self._xhat_cluster(b, x))
            elif kt.is_leaf(a):
                tot += self._k_near_entry_row(i, b, x)
            else:
                for ca in (2 * a + 1, 2 * a + 2):
                    if ca in on_path:
                        for cb in (2 * b + 1, 2 * b + 2):
                            stack.append((ca, cb))
        return tot

    def _moments(self, c):
        if c not in self._mom:
            nodes, axes, sn, kn = self._cluster_nodes(("r", c), self.rlo[c], self.rhi[c])
            mem = self.rt.members[c]
            self._mom[c] = lagrange(axes, self.Q["x"][:, mem]) @ self.Q["w"][mem]
        return self._mom[c]

    def rho_at(self, q):
        """rho~ at one interior quadrature point (Sec. 6.2)."""
        rt = self.rt
        leaf = int(self.leaf_of_q[q])
        path = set()
        c = leaf
        while True:
            path.add(c)
            if c == 0:
                break
            c = (c - 1) // 2
        m = self.m
        cq = np.array([q // self.nqe])
        tot = 0.0
        stack = [(0, 0)]
        eta = self.o["eta"]
        while stack:
            a, b = stack.pop()
            if _admissible(self.rlo[a], self.rhi[a], self.rlo[b], self.rhi[b], eta,
                           self.rh[a] + self.rh[b]):
                na, axa, sa, ka = self._cluster_nodes(("r", a), self.rlo[a], self.rhi[a])
                nb, axb, sb, kb = self._cluster_nodes(("r", b), self.rlo[b], self.rhi[b])
                S = gamma(m.dim, self.o["a_scale"], na[:, :, None], nb[:, None, :], sa[:, None], sb[None, :],
                          ka[:, None], kb[None, :])
                la = lagrange(axa, self.Q["x"][:, [q]])[:, 0]
                tot += la @ (S @ self._moments(b))
            elif rt.is_leaf(a):
                src = rt.members[b]
                G = gamma(m.dim, self.o["a_scale"], self.Q["x"][:, [q]], self.Q["x"][:, src], self.Q["s"][q],
                          self.Q["s"][src], self.Q["k"][q], self.Q["k"][src])
                G[self._touch(cq, src // self.nqe)[0]] = 0.0
                tot += G @ self.Q["w"][src]
            else:
                for ca in (2 * a + 1, 2 * a + 2):
                    if ca in path:
                        for cb in (2 * b + 1, 2 * b + 2):
                            stack.append((ca, cb))
        return float(tot)

    def row_M(self, i, x):
        m = self.m
        N = m.n_dofs
        tot = 0.0
        for c in self._cells_of(i):
            if not m.cell_interior[c]:
                continue
            slot = int(np.flatnonzero(m.cells[:, c] == i)[0])
            q = np.arange(c * self.nqe, (c + 1) * self.nqe)
            rho = np.array([self.rho_at(int(qq)) for qq in q])
            rho = rho + rho_exterior_at(m, self.s, self.k, self.o, self.Q, q)
            vx = np.zeros(q.size)
            for a in range(m.dim + 1):
                v = m.cells[a, c]
                if v < N:
                    vx += self.Q["lam"][a, q] * x[v]
            tot += 2.0 * np.sum(self.Q["w"][q] * self.Q["lam"][slot, q] * rho * vx)
        return tot

    def row_apply(self, rows, x):
        """(A_h x)_i for the given dof rows; returns dict of arrays (B, K, M, total)."""
        x = np.asarray(x, dtype=np.float64)
        out = {"B": [], "K": [], "M": []}
        for i in rows:
            out["B"].append(self.row_B(int(i), x))
            out["K"].append(self.row_K(int(i), x))
            out["M"].append(self.row_M(int(i), x))
        out = {k: np.array(v) for k, v in out.items()}
        out["total"] = out["B"] + out["K"] + out["M"]
        return out
