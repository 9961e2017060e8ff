"""Solves of the Galerkin system A_h u = F (oracle; test infrastructure).

* ``solve_dense``: the discrete solution of Sec. 2 by a dense Cholesky
  factorisation of the symmetric positive definite A_h (the paper solves the
  same system with conjugate gradients, Sec. 7; the solution is the same).
* ``conjugate_gradient``: textbook unpreconditioned CG (Hestenes-Stiefel) on
  a dense matrix, used to compare iteration counts and stopping behaviour
  (relative residual ||F - A u|| / ||F||).
* ``l2_norm``: ||U_h||_{L2} over the interior cells of a P1 function (exact:
  the per-cell rule integrates the square of a linear function exactly).
* ``l2_error``: ||u - U_h||_{L2} / ||u||_{L2} over the interior cells (the
  norm of Sec. 7), for a P1 solution U_h (zero on the non-dof nodes) against a
  function u given pointwise, by a 7-point-per-direction rule on each cell
  (collapsed coordinates on triangles).

Pinned by tests/test_oracle_solve.py: CG and Cholesky agree, the residual of
both vanishes to rounding, and the closed-form solutions of the fractional
Laplacian are reproduced (tests/test_oracle_assembly.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .rules import barycentric_ref, gauss01


def solve_dense(A: np.ndarray, F: np.ndarray) -> np.ndarray:
    """u = A^{-1} F for SPD A (F may hold several right-hand sides as columns)."""
    c = scipy.linalg.cho_factor(np.asarray(A, dtype=np.float64), lower=True)
    return scipy.linalg.cho_solve(c, np.asarray(F, dtype=np.float64))


def conjugate_gradient(A: np.ndarray, F: np.ndarray, rtol: float = 1e-10, maxit: int = 10000,
                       u0: np.ndarray | None = None):
    """Unpreconditioned CG for one right-hand side.  Returns (u, iterations, rel_residual)."""
    F = np.asarray(F, dtype=np.float64)
    u = np.zeros_like(F) if u0 is None else np.array(u0, dtype=np.float64)
    r = F - A @ u
    p = r.copy()
    rr = float(r @ r)
    fn = float(np.sqrt(F @ F))
    if fn == 0.0:
        return u, 0, 0.0
    it = 0
    while np.sqrt(rr) > rtol * fn and it < maxit:
        Ap = A @ p
        alpha = rr / float(p @ Ap)
        u += alpha * p
        r -= alpha * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return u, it, float(np.sqrt(rr)) / fn


def l2_error(mesh, u_dofs: np.ndarray, u_exact, n: int = 7) -> float:
    """Relative L2 error over the interior cells of the P1 function with dof values u_dofs.

    ``u_exact(x)`` takes points (dim, nq) and returns values (nq,).
    """
    g, w = gauss01(n)
    if mesh.dim == 1:
        xh, wt = g[None, :], w
    else:
        Z, E = np.meshgrid(g, g, indexing="ij")
        xh = np.stack([Z.ravel(), (Z * E).ravel()])
        wt = (np.outer(w, w) * Z).ravel()
    lam = barycentric_ref(mesh.dim, xh)                     # (dim+1, nq)
    full = np.zeros(mesh.n_nodes)
    full[:mesh.n_dofs] = u_dofs
    err2 = nrm2 = 0.0
    for c in np.flatnonzero(mesh.cell_interior):
        v = mesh.cells[:, c]
        X = mesh.coords[:, v]
        if mesh.dim == 1:
            J = X[:, 1:] - X[:, :1]
        else:
            J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 1]], axis=1)
        det = abs(np.linalg.det(J))
        x = X[:, :1] + J @ xh
        uh = full[v] @ lam
        ue = u_exact(x)
        err2 += det * float((wt * (uh - ue) ** 2).sum())
        nrm2 += det * float((wt * ue ** 2).sum())
    return float(np.sqrt(err2 / nrm2))


def l2_norm(mesh, u_dofs: np.ndarray) -> float:
    """||U_h||_{L2} over the interior cells for the P1 function with dof values u_dofs."""
    full = np.zeros(mesh.n_nodes)
    full[:mesh.n_dofs] = u_dofs
    X = mesh.coords[:, mesh.cells]                     # (dim, dim+1, nc)
    if mesh.dim == 1:
        vol = np.abs(X[0, 1] - X[0, 0])
    else:
        vol = 0.5 * np.abs((X[0, 1] - X[0, 0]) * (X[1, 2] - X[1, 0]) - (X[1, 1] - X[1, 0]) * (X[0, 2] - X[0, 0]))
    U = full[mesh.cells]                               # (dim+1, nc)
    # integral of a linear function squared over a simplex: vol * (sum u_a^2 + (sum u_a)^2) / ((d+1)(d+2))
    d = mesh.dim
    q = vol * ((U ** 2).sum(axis=0) + U.sum(axis=0) ** 2) / ((d + 1) * (d + 2))
    return float(np.sqrt((q * mesh.cell_interior).sum()))
