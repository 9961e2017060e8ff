"""Geometry, P1 fields and the kernel (oracle; test infrastructure).

Kernel (Sec. 2): gamma(x,y) = a(x,y) / |x-y|^{d+s(x)+s(y)} with
a(x,y) = a_scale * sqrt(kappa(x) kappa(y)).  ``a_scale`` is 1 for the
paper's variable-order tests; the constant-order closed-form tests use the
fractional-Laplacian normalisation C_{d,s}/2.

s and kappa are P1 nodal fields.  At a point inside a cell they are the P1
interpolant; at a point outside the mesh (only Chebyshev nodes can be there)
the value of the nearest mesh node is used (lowest node id on ties).
"""
from __future__ import annotations

import numpy as np

from .rules import element_rule, barycentric_ref


def cell_geometry(mesh):
    """v0 (dim, nc), J (dim, dim, nc) with J=[v1-v0 | v2-v1], |det J| (nc,)."""
    X = mesh.coords[:, mesh.cells]            # (dim, dim+1, nc)
    v0 = X[:, 0]
    if mesh.dim == 1:
        J = (X[:, 1] - X[:, 0])[:, None, :]
        det = np.abs(J[0, 0])
    else:
        J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 1]], axis=1)  # J[:, col, c]
        det = np.abs(J[0, 0] * J[1, 1] - J[0, 1] * J[1, 0])
    return v0, J, det


def quad_points(mesh, nq: int):
    """All element quadrature points Q (Sec. 6.1).

    Returns dict with
      x   (dim, nc*nqe) physical points, cell-major (point c*nqe + l)
      w   (nc*nqe,)     weights |J| * w_l
      lam (dim+1, nc*nqe) shape values of the cell's vertices at the point
      cell (nc*nqe,)    owning cell
    """
    xh, wh = element_rule(mesh.dim, nq)
    nqe = wh.size
    v0, J, det = cell_geometry(mesh)
    # x = v0 + J xh, evaluated as (v0 + J[:,0] xh0) + J[:,1] xh1
    x = v0[:, :, None] + J[:, 0, :, None] * xh[0][None, None, :]
    if mesh.dim == 2:
        x = x + J[:, 1, :, None] * xh[1][None, None, :]
    nc = mesh.n_cells
    lam = barycentric_ref(mesh.dim, xh)      # (dim+1, nqe)
    return {
        "x": x.reshape(mesh.dim, nc * nqe),
        "w": (det[:, None] * wh[None, :]).reshape(-1),
        "lam": np.broadcast_to(lam[:, None, :], (mesh.dim + 1, nc, nqe)).reshape(mesh.dim + 1, -1).copy(),
        "cell": np.repeat(np.arange(nc), nqe),
        "nqe": nqe,
    }


def p1_at(mesh, field: np.ndarray, cells: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """P1 value of a nodal field at points given by (cell, barycentric weights)."""
    return (field[mesh.cells[:, cells]] * lam).sum(axis=0)


def gamma(d: int, a_scale: float, x, y, sx, sy, kx, ky):
    """gamma(x,y) for arrays of point pairs (broadcasting)."""
    r = np.sqrt(((x - y) ** 2).sum(axis=0))
    return a_scale * np.sqrt(kx * ky) * r ** (-(d + sx + sy))


def locate(mesh, pts: np.ndarray, tol: float = 1e-12):
    """Point location by brute force.

    Returns (cell, lam) per point; cell = -1 when the point lies in no cell, in
    which case ``lam`` holds the nearest node id in row 0 (as float).
    The first (lowest id) containing cell is used.
    """
    d = mesh.dim
    npts = pts.shape[1]
    cell = np.full(npts, -1, dtype=np.int64)
    lam = np.zeros((d + 1, npts))
    v0, J, det = cell_geometry(mesh)
    X = mesh.coords[:, mesh.cells]
    chunk = 256
    for s0 in range(0, npts, chunk):
        p = pts[:, s0:s0 + chunk]                            # (d, P)
        if d == 1:
            a, b = X[0, 0][:, None], X[0, 1][:, None]        # (nc,1)
            t = (p[0][None, :] - a) / (b - a)                # (nc, P)
            L = np.stack([1.0 - t, t])                       # (2, nc, P)
        else:
            # barycentric w.r.t. the physical vertices (P0,P1,P2)
            P0, P1, P2 = X[:, 0], X[:, 1], X[:, 2]
            e1 = P1 - P0
            e2 = P2 - P0
            den = e1[0] * e2[1] - e1[1] * e2[0]              # (nc,)
            dx = p[:, None, :] - P0[:, :, None]              # (2, nc, P)
            b1 = (dx[0] * e2[1][:, None] - dx[1] * e2[0][:, None]) / den[:, None]
            b2 = (e1[0][:, None] * dx[1] - e1[1][:, None] * dx[0]) / den[:, None]
            L = np.stack([1.0 - b1 - b2, b1, b2])
        inside = (L >= -tol).all(axis=0)                     # (nc, P)
        has = inside.any(axis=0)
        first = np.argmax(inside, axis=0)
        idx = np.arange(p.shape[1])
        cell[s0:s0 + chunk] = np.where(has, first, -1)
        lam[:, s0:s0 + chunk] = L[:, first, idx]
    out = np.flatnonzero(cell < 0)
    for k in out:
        dist2 = ((mesh.coords - pts[:, k:k + 1]) ** 2).sum(axis=0)
        lam[:, k] = 0.0
        lam[0, k] = float(np.argmin(dist2))
    return cell, lam


def field_at_points(mesh, field: np.ndarray, pts: np.ndarray):
    """P1 interpolation of a nodal field at arbitrary points (nearest node outside)."""
    cell, lam = locate(mesh, pts)
    out = np.empty(pts.shape[1], dtype=np.result_type(field, np.float64))
    ok = cell >= 0
    out[ok] = (field[mesh.cells[:, cell[ok]]] * lam[:, ok]).sum(axis=0)
    out[~ok] = field[lam[0, ~ok].astype(np.int64)]
    return out
