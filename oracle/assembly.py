"""Dense assembly of the stiffness matrix (oracle; test infrastructure).

* ``assemble_exact``: the Galerkin matrix by its definition, eq. e:l-stiff
  summed over every ordered element pair with an interior cell: touching
  pairs by the singular rules (``oracle.singular``), separated pairs by the
  product of the per-element rule applied to the full integrand
  (u(x)-u(y))(v(x)-v(y)) gamma(x,y).
* ``assemble_split``: the three-way split of Sec. 3, A = B + K + M with
    K_ij = -2 sum_{q,q' in Q^int, cells not touching} psi_i(q) w gamma(q,q') w' psi_j(q')  (eq. e:k)
    M_ij = 2 sum_{tau int} sum_{q in tau} w psi_i psi_j (q) rho(q)                        (eq. e:m)
    rho(q) = sum_{q' in Q, cells not touching} gamma(q,q') w'                              (eq. e:tgt-sum)
  plus, when the exterior continues beyond R, rho_B (eq. e:rho) in M.
  With the same points, B + K + M equals ``assemble_exact`` to rounding.
* ``load_vector``: F_i = sum_{tau int} sum_q w psi_i(q) f(q).

Pinned by tests/test_oracle_assembly.py: symmetry, positive definiteness, zero
row sums over all nodes, the split identity, scale invariance, and the
closed-form solutions in 1D and on the disk.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fields import quad_points, p1_at, gamma
from .singular import assemble_B
from .exterior import rho_ball_exterior


def touching_cells(mesh):
    """Sparse boolean (nc, nc): cells sharing at least one vertex (incl. self)."""
    nc = mesh.n_cells
    C = sp.csr_matrix((np.ones(mesh.cells.size), (np.repeat(np.arange(nc), mesh.dim + 1),
                                                   mesh.cells.T.ravel())), shape=(nc, mesh.n_nodes))
    T = (C @ C.T).tocsr()
    T.data[:] = 1.0
    return T


def _qdata(mesh, s, kappa, nq):
    Q = quad_points(mesh, nq)
    Q["s"] = p1_at(mesh, s, Q["cell"], Q["lam"])
    Q["k"] = p1_at(mesh, kappa, Q["cell"], Q["lam"])
    return Q


def _gamma_block(mesh, opts, Q, ia, ib, T):
    """gamma_T between point sets ia (rows) and ib (cols); zero on touching cells."""
    G = gamma(mesh.dim, opts["a_scale"], Q["x"][:, ia, None], Q["x"][:, None, ib],
              Q["s"][ia, None], Q["s"][None, ib], Q["k"][ia, None], Q["k"][None, ib])
    touch = T[Q["cell"][ia]][:, Q["cell"][ib]].toarray() > 0
    G[touch] = 0.0
    return G


def rho_direct(mesh, s, kappa, opts, Q=None, targets=None):
    """rho(q) = sum_{q'} gamma_T(q,q') w' for target points (default: all of Q^int)."""
    if Q is None:
        Q = _qdata(mesh, s, kappa, opts["nq_reg"])
    T = touching_cells(mesh)
    if targets is None:
        targets = np.flatnonzero(mesh.cell_interior[Q["cell"]] > 0)
    allp = np.arange(Q["w"].size)
    out = np.zeros(targets.size, dtype=np.result_type(Q["s"], Q["k"], np.float64))
    ch = max(1, 2_000_000 // allp.size)
    for s0 in range(0, targets.size, ch):
        ia = targets[s0:s0 + ch]
        G = _gamma_block(mesh, opts, Q, ia, allp, T)
        out[s0:s0 + ch] = G @ Q["w"]
    return out


def rho_exterior_at(mesh, s, kappa, opts, Q, targets):
    if mesh.exterior_radius <= 0.0:
        return np.zeros(targets.size)
    return rho_ball_exterior(mesh.dim, Q["x"][:, targets], Q["s"][targets], Q["k"][targets],
                             mesh.exterior_radius, opts["s_exterior"], opts.get("kappa_exterior", 1.0),
                             opts["a_scale"], opts["n_theta"])


def _shape_matrix(mesh, Q, pts, ncol):
    """P[i, l] = psi_i(q_l) for dof rows i (sparse), points pts."""
    rows, cols, vals = [], [], []
    for a in range(mesh.dim + 1):
        v = mesh.cells[a, Q["cell"][pts]]
        keep = v < ncol
        rows.append(v[keep])
        cols.append(np.flatnonzero(keep))
        vals.append(Q["lam"][a, pts][keep])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(ncol, pts.size))


def mass_from_rho(mesh, Q, pts, rho, N):
    """M_ij = 2 sum_q w psi_i psi_j rho(q) over the given interior points."""
    P = _shape_matrix(mesh, Q, pts, N)
    return 2.0 * (P @ sp.diags(Q["w"][pts] * rho) @ P.T).toarray()


def assemble_split(mesh, s, kappa, opts):
    """Return dict(B, K, M, rho, Q) of the exact (non-H2) split."""
    s = s.reshape(-1)
    kappa = kappa.reshape(-1)
    N = mesh.n_dofs
    B = assemble_B(mesh, s, kappa, opts)
    Q = _qdata(mesh, s, kappa, opts["nq_reg"])
    T = touching_cells(mesh)
    qi = np.flatnonzero(mesh.cell_interior[Q["cell"]] > 0)
    rho = rho_direct(mesh, s, kappa, opts, Q, qi) + rho_exterior_at(mesh, s, kappa, opts, Q, qi)
    M = mass_from_rho(mesh, Q, qi, rho, N)
    P = _shape_matrix(mesh, Q, qi, N)
    K = np.zeros((N, N), dtype=np.result_type(s, kappa, np.float64))
    ch = max(1, 4_000_000 // qi.size)
    for s0 in range(0, qi.size, ch):
        ia = qi[s0:s0 + ch]
        G = _gamma_block(mesh, opts, Q, ia, qi, T)
        K += -2.0 * (P[:, s0:s0 + ch] @ ((Q["w"][ia][:, None] * G * Q["w"][qi][None, :]) @ P.T.toarray()))
    return {"B": B, "K": K, "M": M, "rho": rho, "Q": Q, "qi": qi}


def assemble_exact(mesh, s, kappa, opts, all_columns=True):
    """Galerkin matrix by definition over interior rows (columns: all nodes)."""
    s = s.reshape(-1)
    kappa = kappa.reshape(-1)
    N = mesh.n_dofs
    ncol = mesh.n_nodes if all_columns else N
    A = assemble_B(mesh, s, kappa, opts, all_columns=True)
    Q = _qdata(mesh, s, kappa, opts["nq_reg"])
    T = touching_cells(mesh).tolil()
    nqe = Q["nqe"]
    nc = mesh.n_cells
    interior = mesh.cell_interior.astype(bool)
    k = mesh.dim + 1
    for c in np.flatnonzero(interior):
        ia = np.arange(c * nqe, (c + 1) * nqe)
        others = np.array([c2 for c2 in range(nc) if c2 not in set(T.rows[c])])
        if others.size == 0:
            continue
        ib = (others[:, None] * nqe + np.arange(nqe)[None, :]).ravel()
        G = gamma(mesh.dim, opts["a_scale"], Q["x"][:, ia, None], Q["x"][:, None, ib],
                  Q["s"][ia, None], Q["s"][None, ib], Q["k"][ia, None], Q["k"][None, ib])
        G = G * Q["w"][ia, None] * Q["w"][None, ib]
        G = G.reshape(nqe, others.size, nqe)                       # (q, tau', q')
        # Phi over the 2k local vertices: (psi(x) - psi(y))
        lx = Q["lam"][:, ia]                                        # (k, q)
        ly = Q["lam"][:, ib].reshape(k, others.size, nqe)           # (k, tau', q')
        phi = np.concatenate([np.broadcast_to(lx[:, :, None, None], (k, nqe, others.size, nqe)),
                              -np.broadcast_to(ly[:, None, :, :], (k, nqe, others.size, nqe))])
        loc = np.einsum("aqtr,qtr,bqtr->tab", phi, G, phi)         # (tau', 2k, 2k)
        wgt = np.where(interior[others], 1.0, 2.0)                  # ext partner: both orders
        loc *= wgt[:, None, None]
        vid = np.concatenate([np.broadcast_to(mesh.cells[:, c][:, None], (k, others.size)),
                              mesh.cells[:, others]])                # (2k, tau')
        for a in range(2 * k):
            ra = vid[a]
            keep = ra < N
            for b in range(2 * k):
                cb = vid[b]
                kk = keep & (cb < ncol)
                np.add.at(A, (ra[kk], cb[kk]), loc[kk, a, b])
    if mesh.exterior_radius > 0.0:
        qi = np.flatnonzero(mesh.cell_interior[Q["cell"]] > 0)
        rb = rho_exterior_at(mesh, s, kappa, opts, Q, qi)
        Mo = mass_from_rho(mesh, Q, qi, rb, N)
        A[:, :N] += Mo
    return A if all_columns else A[:, :N]


def load_vector(mesh, f_nodal, opts):
    """F_i = sum_{tau int} sum_q w psi_i(q) f(q), f P1-interpolated."""
    Q = quad_points(mesh, opts["nq_reg"])
    qi = np.flatnonzero(mesh.cell_interior[Q["cell"]] > 0)
    fq = p1_at(mesh, f_nodal, Q["cell"][qi], Q["lam"][:, qi])
    P = _shape_matrix(mesh, Q, qi, mesh.n_dofs)
    return P @ (Q["w"][qi] * fq)
