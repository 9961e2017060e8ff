"""Derivatives of w^T A_h(s, kappa) u with respect to the nodal order and
diffusivity (oracle; test infrastructure).

A_h = B + K~ + M~ is the operator of Thm. 6.2 as ``oracle.h2.assemble_h2``
builds it.  For a fixed substitution parameter s_bar it is an analytic
function of the nodal values s_j and kappa_j: every s- and kappa-dependence
enters through P1 interpolation, powers |x-y|^{-(d+s(x)+s(y))} (after the
substitutions of Sec. 4 these are the same powers, rewritten), square roots
sqrt(kappa(x) kappa(y)) and the exterior density of eq. e:rho.  The trees,
partitions and quadrature points depend on the mesh only.  The complex-step
derivative

    d/dt w^T A_h(s + t ds, kappa + t dk) u |_{t=0}
        = Im(w^T A_h(s + i h ds, kappa + i h dk) u) / h,    h = 1e-30,

is therefore exact to rounding (no difference of nearby values is taken).

* ``bilinear``     w^T A_h u (summed over right-hand-side columns).
* ``directional``  the complex-step directional derivative above.
* ``gradient``     the full gradient over all nodes, one complex assembly per
                   node and field (small meshes only).
* ``objective_directional``  derivative of J(s) = 1/2 ||u(s) - u_obs||^2 with
                   u(s) = A_h(s, kappa)^{-1} F, by the same complex step through a
                   dense LU solve (the complex-symmetric A_h is not Hermitian).

Pinned by tests/test_oracle_adjoint.py: central finite differences of the real
assembly, the exact scaling laws A_h(2T) = 2^{d-2s} A_h(T) (constant s,
bounded exterior) and A_h(lambda kappa) = lambda A_h(kappa) differentiated in
closed form, and the symmetry of the derivative in (w, u).
"""
from __future__ import annotations

import numpy as np

from .h2 import assemble_h2

STEP = 1e-30


def bilinear(mesh, s, kappa, opts, w, u):
    ref = assemble_h2(mesh, np.asarray(s).reshape(-1), np.asarray(kappa).reshape(-1), opts)
    A = ref["B"] + ref["K"] + ref["M"]
    w = np.asarray(w).reshape(mesh.n_dofs, -1)
    u = np.asarray(u).reshape(mesh.n_dofs, -1)
    return np.sum(w * (A @ u))


def directional(mesh, s, kappa, opts, w, u, ds=None, dk=None, h=STEP):
    s = np.asarray(s, dtype=np.float64).reshape(-1)
    kappa = np.asarray(kappa, dtype=np.float64).reshape(-1)
    sc = s + 1j * h * (np.zeros_like(s) if ds is None else np.asarray(ds, dtype=np.float64))
    kc = kappa + 1j * h * (np.zeros_like(kappa) if dk is None else np.asarray(dk, dtype=np.float64))
    return float(np.imag(bilinear(mesh, sc, kc, opts, w, u)) / h)


def objective_directional(mesh, s, kappa, opts, F, u_obs, ds=None, dk=None, h=STEP):
    s = np.asarray(s, dtype=np.float64).reshape(-1)
    kappa = np.asarray(kappa, dtype=np.float64).reshape(-1)
    sc = s + 1j * h * (np.zeros_like(s) if ds is None else np.asarray(ds, dtype=np.float64))
    kc = kappa + 1j * h * (np.zeros_like(kappa) if dk is None else np.asarray(dk, dtype=np.float64))
    ref = assemble_h2(mesh, sc, kc, opts)
    A = ref["B"] + ref["K"] + ref["M"]
    u = np.linalg.solve(A, np.asarray(F, dtype=np.complex128))
    J = 0.5 * np.sum((u - u_obs) ** 2)
    return float(np.imag(J) / h)


def gradient(mesh, s, kappa, opts, w, u):
    """(grad_s, grad_kappa) over all mesh nodes."""
    M = mesh.n_nodes
    gs = np.zeros(M)
    gk = np.zeros(M)
    e = np.zeros(M)
    for j in range(M):
        e[j] = 1.0
        gs[j] = directional(mesh, s, kappa, opts, w, u, ds=e)
        gk[j] = directional(mesh, s, kappa, opts, w, u, dk=e)
        e[j] = 0.0
    return gs, gk
