"""Touching element pairs: the singular near-field B (oracle; test infrastructure).

2D (Sec. 4 of the paper).  Reference triangle (0,0),(1,0),(1,1); chi(x^) = v0 + J x^,
J = [v1-v0 | v2-v1].  Each touching pair is evaluated once, in canonical
orientation, and enters B with weight 2 (vertex, edge) or 1 (identical): this
counts both ordered pairs (tau,tau') and (tau',tau), including an interior cell
next to an exterior one (the reading that makes B the sum of A_{tau,tau'} over
every ordered touching pair with an interior cell).

* vertex  (eq. e:int-v-2): 2 regions T_V^(1,2), xi = zeta^{1/(4-2 s_bar)},
          Jacobian factor eta2, local dofs {P, tau.v1, tau.v2, tau'.v1, tau'.v2}.
* edge    (eq. e:int-e): 5 regions T_E^(k), Jacobians eta1^2 (k=1), eta1^2 eta2,
          local dofs {v0, v1, tau.v2, tau'.v2}.
* identical (eq. e:int-i-2): 3 regions (+3 mirrored), xi = zeta^{1/(4-2 s_bar)},
          eta2 = t^{1/(2-2 s_bar)}.  Two misprints of the printed maps are
          corrected so that the regions tile the reference pair and agree with
          the printed rescaled differences: the second component of T_I^(2)
          carries a factor eta1, and d_I^(3) = J(-eta3, 1-eta3).

Canonical orientation (both the oracle and the library use it):
  identical: vertices in ascending global id;
  edge:      tau = lower cell id; shared edge (e0<e1) is (v0,v1) in both cells;
  vertex:    tau = lower cell id; shared node is v0, the other two ascending.

1D (the paper gives only 2D rules; derived here by the same technique):
* identical tau=[v0,v1]: x^-y^ = t, y^ = (1-t) u, t = zeta^{1/(2-2 s_bar)}:
  A_ab = sig_a sig_b 2/(2-2 s_bar) sum w w a |J|^{1-s(x)-s(y)} zeta^{(2s_bar-s-s)/(2-2s_bar)} (1-t),
  sig = (-1, +1).
* vertex  tau=[P,A], tau'=[P,B]: x = P + (A-P) al, y = P + (B-P) be, regions
  (al,be) = xi (1,eta) and xi (eta,1), xi = zeta^{1/(3-2 s_bar)}:
  A = h1 h2/(3-2 s_bar) sum_regions sum w w a zeta^{(2s_bar-s-s)/(3-2s_bar)} Phi_a Phi_b / D^{1+s+s},
  Phi over {P, A, B} = (be-al, al, -be) / xi, D = h1 al + h2 be (rescaled).

Pinned by tests/test_oracle_singular.py: region maps tile the reference pair
(polynomial moments, Jacobians by sympy), rescaled differences agree with the
maps, convergence to an independent polar/ray brute force, 1D closed forms.
"""
from __future__ import annotations

import numpy as np

from .rules import gauss01


# ----------------------------------------------------------------------------
# pair enumeration
# ----------------------------------------------------------------------------

def canonical_pair(mesh, c, c2):
    """Kind and canonical vertex tuples of two touching cells (c < c2, or c == c2)."""
    vc = [int(v) for v in mesh.cells[:, c]]
    if c == c2:
        return ("I", tuple(sorted(vc)), tuple(sorted(vc)))
    v2 = [int(v) for v in mesh.cells[:, c2]]
    shared = sorted(set(vc) & set(v2))
    if len(shared) == mesh.dim + 1:
        raise ValueError("duplicate cell")
    if mesh.dim == 2 and len(shared) == 2:
        e0, e1 = shared
        t0 = [v for v in vc if v not in shared][0]
        t1 = [v for v in v2 if v not in shared][0]
        return ("E", (e0, e1, t0), (e0, e1, t1))
    if len(shared) == 1:
        P = shared[0]
        o0 = sorted(v for v in vc if v != P)
        o1 = sorted(v for v in v2 if v != P)
        return ("V", (P, *o0), (P, *o1))
    raise ValueError("unexpected sharing")


def touching_pairs(mesh):
    """All touching pairs with at least one interior cell, canonical orientation.

    Returns a list of tuples (kind, c0, c1, verts0, verts1) with kind in
    {"I", "E", "V"}; verts are the canonical vertex tuples of the two cells.
    """
    cells = mesh.cells.T
    nc = cells.shape[0]
    node_cells = {}
    for c in range(nc):
        for v in cells[c]:
            node_cells.setdefault(int(v), []).append(c)
    out = []
    interior = mesh.cell_interior.astype(bool)
    for c in range(nc):
        vc = [int(v) for v in cells[c]]
        if interior[c]:
            kind, a, b = canonical_pair(mesh, c, c)
            out.append((kind, c, c, a, b))
        nbrs = sorted({c2 for v in vc for c2 in node_cells[v] if c2 > c})
        for c2 in nbrs:
            if not (interior[c] or interior[c2]):
                continue
            kind, a, b = canonical_pair(mesh, c, c2)
            out.append((kind, c, c2, a, b))
    return out


def pair_local_dofs(mesh, kind, v0, v1):
    """Local dof list of a canonical pair (order of the local matrices)."""
    if kind == "I":
        return list(v0)
    if kind == "E":
        return [v0[0], v0[1], v0[2], v1[2]]
    return list(v0) + list(v1[1:]) if mesh.dim == 2 else [v0[0], v0[1], v1[1]]


# ----------------------------------------------------------------------------
# 2D rules
# ----------------------------------------------------------------------------

def _tensor4(n):
    g, w = gauss01(n)
    Z, E1, E2, E3 = np.meshgrid(g, g, g, g, indexing="ij")
    W = np.einsum("a,b,c,d->abcd", w, w, w, w)
    return Z.ravel(), E1.ravel(), E2.ravel(), E3.ravel(), W.ravel()


def _jac(X):
    """J = [v1-v0 | v2-v1] for a (2,3) vertex array."""
    return np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 1]], axis=1)


def _lam(xh):
    return np.stack([1.0 - xh[0], xh[0] - xh[1], xh[1]])


def _vertex_regions(xi, e1, e2, e3):
    """Regions of e:map-v: (x^, y^, Phi, (a,b) with d = J_tau a - J_tau' b, extra factor)."""
    one = np.ones_like(e1)
    r1 = (np.stack([xi, xi * e1]), np.stack([xi * e2, xi * e2 * e3]),
          np.stack([e2 - 1, 1 - e1, e1, e2 * e3 - e2, -e2 * e3]),
          (np.stack([one, e1]), np.stack([e2, e2 * e3])), e2)
    r2 = (np.stack([xi * e2, xi * e2 * e3]), np.stack([xi, xi * e1]),
          np.stack([1 - e2, e2 - e2 * e3, e2 * e3, e1 - 1, -e1]),
          (np.stack([e2, e2 * e3]), np.stack([one, e1])), e2)
    return [r1, r2]


def _edge_regions(xi, e1, e2, e3):
    """Regions of the edge case (Sec. 4.2) with their Psi, d and Jacobian factors."""
    one = np.ones_like(e1)
    regs = []
    # k = 1
    a = np.stack([one, e1 * e3]); b = np.stack([1 - e1 * e2, e1 * (1 - e2)])
    psi = np.stack([-e1 * e2, e1 * (1 - e3), e1 * e3, -e1 * (1 - e2)])
    regs.append((xi * a, xi * b, psi, (a, b), e1 ** 2))
    # k = 2
    a = np.stack([one, e1]); b = np.stack([1 - e1 * e2 * e3, e1 * e2 * (1 - e3)])
    psi = np.stack([-e1 * e2 * e3, -e1 * (1 - e2), e1, -e1 * e2 * (1 - e3)])
    regs.append((xi * a, xi * b, psi, (a, b), e1 ** 2 * e2))
    # k = 3
    a = np.stack([1 - e1 * e2, e1 * (1 - e2)]); b = np.stack([one, e1 * e2 * e3])
    psi = np.stack([e1 * e2, -e1 * (1 - e2 * e3), e1 * (1 - e2), -e1 * e2 * e3])
    regs.append((xi * a, xi * b, psi, (a, b), e1 ** 2 * e2))
    # k = 4
    a = np.stack([1 - e1 * e2 * e3, e1 * e2 * (1 - e3)]); b = np.stack([one, e1])
    psi = np.stack([e1 * e2 * e3, e1 * (1 - e2), e1 * e2 * (1 - e3), -e1])
    regs.append((xi * a, xi * b, psi, (a, b), e1 ** 2 * e2))
    # k = 5
    a = np.stack([1 - e1 * e2 * e3, e1 * (1 - e2 * e3)]); b = np.stack([one, e1 * e2])
    psi = np.stack([e1 * e2 * e3, -e1 * (1 - e2), e1 * (1 - e2 * e3), -e1 * e2])
    regs.append((xi * a, xi * b, psi, (a, b), e1 ** 2 * e2))
    return regs


def _identical_regions(xi, e1, e2, e3):
    """Regions k=1..3 of the identical case with corrected T_I^(2) and d_I^(3).

    Returns (x^, y^, Psi, dhat) where x^ - y^ = xi*eta1*eta2*dhat.
    """
    regs = []
    regs.append((np.stack([xi, xi * (1 - e1 + e1 * e2)]), np.stack([xi * (1 - e1 * e2 * e3), xi * (1 - e1)]),
                 np.stack([-e3, e3 - 1, np.ones_like(e3)]), np.stack([e3, np.ones_like(e3)])))
    regs.append((np.stack([xi, xi * e1 * (1 - e2 + e2 * e3)]), np.stack([xi * (1 - e1 * e2), xi * e1 * (1 - e2)]),
                 np.stack([-np.ones_like(e3), 1 - e3, e3]), np.stack([np.ones_like(e3), e3])))
    regs.append((np.stack([xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3)]), np.stack([xi, xi * e1 * (1 - e2)]),
                 np.stack([e3, -np.ones_like(e3), 1 - e3]), np.stack([-e3, 1 - e3])))
    return regs


def local_matrix_2d(kind, X0, X1, s0, s1, k0, k1, a_scale, s_bar, n):
    """Local matrix of one touching pair (without the pair weight).

    X0, X1: (2,3) canonical vertex coordinates of tau, tau'; s*, k*: nodal
    order/diffusivity at those vertices.  Returns the matrix over the local dof
    list of the case.
    """
    Z, E1, E2, E3, W = _tensor4(n)
    J0 = _jac(X0)
    J1 = _jac(X1)
    det0 = abs(np.linalg.det(J0))
    det1 = abs(np.linalg.det(J1))
    sb = s_bar
    if kind in ("V", "E"):
        xi = Z ** (1.0 / (4.0 - 2.0 * sb))
        regs = _vertex_regions(xi, E1, E2, E3) if kind == "V" else _edge_regions(xi, E1, E2, E3)
        nd = 5 if kind == "V" else 4
        A = np.zeros((nd, nd), dtype=np.result_type(s0, s1, k0, k1, np.float64))
        for xh, yh, phi, (a, b), fac in regs:
            lx = _lam(xh)
            ly = _lam(yh)
            sx = (s0[:, None] * lx).sum(0)
            sy = (s1[:, None] * ly).sum(0)
            ka = np.sqrt((k0[:, None] * lx).sum(0) * (k1[:, None] * ly).sum(0))
            d = J0 @ a - J1 @ b
            r = np.sqrt((d ** 2).sum(0))
            f = W * a_scale * ka * Z ** ((2 * sb - sx - sy) / (4 - 2 * sb)) * fac / r ** (2 + sx + sy)
            A += (phi * f) @ phi.T
        return A * det0 * det1 / (4.0 - 2.0 * sb)
    if kind == "I":
        xi = Z ** (1.0 / (4.0 - 2.0 * sb))
        e2 = E2 ** (1.0 / (2.0 - 2.0 * sb))          # eta2 = t^{1/(2-2 s_bar)}
        A = np.zeros((3, 3), dtype=np.result_type(s0, k0, np.float64))
        for xh, yh, psi, dh in _identical_regions(xi, E1, e2, E3):
            lx = _lam(xh)
            ly = _lam(yh)
            sx = (s0[:, None] * lx).sum(0)
            sy = (s0[:, None] * ly).sum(0)
            ka = np.sqrt((k0[:, None] * lx).sum(0) * (k0[:, None] * ly).sum(0))
            d = J0 @ dh
            r = np.sqrt((d ** 2).sum(0))
            f = (W * a_scale * ka * Z ** ((2 * sb - sx - sy) / (4 - 2 * sb)) * E1 ** (2 - sx - sy)
                 * E2 ** ((2 * sb - sx - sy) / (2 - 2 * sb)) / r ** (2 + sx + sy))
            A += (psi * f) @ psi.T
        return A * det0 * det0 / ((2.0 - sb) * (2.0 - 2.0 * sb))
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# 1D rules
# ----------------------------------------------------------------------------

def local_matrix_1d(kind, x0, x1, s0, s1, k0, k1, a_scale, s_bar, n):
    """1D local matrices.  kind "I": tau = [x0[0], x0[1]] (dofs v0, v1).
    kind "V": tau = (P, A), tau' = (P, B) given as x0 = (xP, xA), x1 = (xP, xB),
    dofs {P, A, B}."""
    g, w = gauss01(n)
    Z, U = np.meshgrid(g, g, indexing="ij")
    W = np.outer(w, w)
    Z, U, W = Z.ravel(), U.ravel(), W.ravel()
    sb = s_bar
    if kind == "I":
        J = x0[1] - x0[0]
        t = Z ** (1.0 / (2.0 - 2.0 * sb))
        yh = (1.0 - t) * U
        xh = yh + t
        sx = (1 - xh) * s0[0] + xh * s0[1]
        sy = (1 - yh) * s0[0] + yh * s0[1]
        ka = np.sqrt(((1 - xh) * k0[0] + xh * k0[1]) * ((1 - yh) * k0[0] + yh * k0[1]))
        val = (2.0 / (2.0 - 2.0 * sb) * W * a_scale * ka * abs(J) ** (1 - sx - sy)
               * Z ** ((2 * sb - sx - sy) / (2 - 2 * sb)) * (1 - t)).sum()
        sig = np.array([-1.0, 1.0])
        return np.outer(sig, sig) * val
    if kind == "V":
        h1 = abs(x0[1] - x0[0])
        h2 = abs(x1[1] - x1[0])
        xi = Z ** (1.0 / (3.0 - 2.0 * sb))
        A = np.zeros((3, 3), dtype=np.result_type(s0, s1, k0, k1, np.float64))
        for al_t, be_t in ((np.ones_like(U), U), (U, np.ones_like(U))):
            al = xi * al_t
            be = xi * be_t
            sx = (1 - al) * s0[0] + al * s0[1]
            sy = (1 - be) * s1[0] + be * s1[1]
            ka = np.sqrt(((1 - al) * k0[0] + al * k0[1]) * ((1 - be) * k1[0] + be * k1[1]))
            phi = np.stack([be_t - al_t, al_t, -be_t])
            D = h1 * al_t + h2 * be_t
            f = W * a_scale * ka * Z ** ((2 * sb - sx - sy) / (3 - 2 * sb)) / D ** (1 + sx + sy)
            A += (phi * f) @ phi.T
        return A * h1 * h2 / (3.0 - 2.0 * sb)
    raise ValueError(kind)


def pair_matrix(mesh, s, kappa, opts, kind, v0, v1):
    """Local matrix of a canonical pair (without the pair weight)."""
    i0 = np.array(v0)
    i1 = np.array(v1)
    if mesh.dim == 2:
        return local_matrix_2d(kind, mesh.coords[:, i0], mesh.coords[:, i1], s[i0], s[i1], kappa[i0], kappa[i1],
                               opts["a_scale"], opts["s_bar"], opts["nq_sing"])
    return local_matrix_1d(kind, mesh.coords[0, i0], mesh.coords[0, i1], s[i0], s[i1], kappa[i0], kappa[i1],
                           opts["a_scale"], opts["s_bar"], opts["nq_sing"])


# ----------------------------------------------------------------------------
# assembly of B
# ----------------------------------------------------------------------------

def assemble_B(mesh, s, kappa, opts, all_columns=False, rows=None):
    """Dense B over interior rows.  Columns: dofs (default) or all mesh nodes.

    ``rows``: optional subset of dof rows to assemble (pairs not touching a
    requested row are skipped); returns a full-width array regardless.
    """
    N = mesh.n_dofs
    ncol = mesh.n_nodes if all_columns else N
    B = np.zeros((N, ncol), dtype=np.result_type(s, kappa, np.float64))
    want = None if rows is None else set(int(r) for r in rows)
    a_scale = opts["a_scale"]
    sb = opts["s_bar"]
    n = opts["nq_sing"]
    for kind, c0, c1, v0, v1 in touching_pairs(mesh):
        loc = pair_local_dofs(mesh, kind, v0, v1)
        if want is not None and not (want & set(loc)):
            continue
        i0 = np.array(v0)
        i1 = np.array(v1)
        if mesh.dim == 2:
            L = local_matrix_2d(kind, mesh.coords[:, i0], mesh.coords[:, i1], s[i0], s[i1],
                                kappa[i0], kappa[i1], a_scale, sb, n)
        else:
            L = local_matrix_1d(kind, mesh.coords[0, i0], mesh.coords[0, i1], s[i0], s[i1],
                                kappa[i0], kappa[i1], a_scale, sb, n)
        wgt = 1.0 if kind == "I" else 2.0
        for a, ga in enumerate(loc):
            if ga >= N:
                continue
            for b, gb in enumerate(loc):
                if gb < ncol:
                    B[ga, gb] += wgt * L[a, b]
    return B
