"""Pins for the oracle's derivatives of w^T A_h u (``oracle.adjoint``).

* complex step against central finite differences of the real assembly;
* scaling in the order: for constant s and a bounded exterior, A_h(2T) =
  2^{d-2s} A_h(T) exactly (rules in reference coordinates, partitions and
  quadrature scale with the mesh), so the derivative along ds = 1 obeys
  D(2T) = 2^{d-2s} (D(T) - 2 ln 2 A_h(T));
* homogeneity in the diffusivity: A_h(lambda kappa) = lambda A_h(kappa), so the
  derivative along dk = kappa equals w^T A_h u;
* symmetry: A_h is symmetric for every (s, kappa), so is its derivative.
"""
import math

import numpy as np
import pytest

from fpde_inputs import configs
from fpde_inputs.meshes import Mesh
from oracle.adjoint import bilinear, directional


def _case(name="square"):
    if name == "square":
        P = configs.square(5, 2, leaf_size=8, leaf_size_rho=16, cheb_p=3)
    elif name == "disk":      # exterior beyond R = 1.1 (analytic density)
        P = configs.disk(6, leaf_size=8, leaf_size_rho=16, cheb_p=3)
    else:                     # 1D rules
        P = configs.interval(n_int=16, n_ext=4, leaf_size=4, leaf_size_rho=8, cheb_p=3)
    rng = np.random.default_rng(3)
    w = rng.standard_normal(P.mesh.n_dofs)
    u = rng.standard_normal(P.mesh.n_dofs)
    return P, w, u


@pytest.mark.parametrize("name", ["square", "disk", "interval"])
def test_complex_step_matches_central_differences(name):
    P, w, u = _case(name)
    rng = np.random.default_rng(4)
    M = P.mesh.n_nodes
    s, k = P.s[0], P.kappa[0]
    ds = rng.uniform(-1, 1, M) * 0.05
    dk = rng.uniform(-1, 1, M) * 0.1
    for dsv, dkv in ((ds, None), (None, dk), (ds, dk)):
        cs = directional(P.mesh, s, k, P.opts, w, u, ds=dsv, dk=dkv)
        eps = 1e-5
        sp = s + (eps * dsv if dsv is not None else 0)
        sm = s - (eps * dsv if dsv is not None else 0)
        kp = k + (eps * dkv if dkv is not None else 0)
        km = k - (eps * dkv if dkv is not None else 0)
        fd = (bilinear(P.mesh, sp, kp, P.opts, w, u) - bilinear(P.mesh, sm, km, P.opts, w, u)) / (2 * eps)
        assert abs(cs - fd) <= 1e-7 * abs(cs), (cs, fd)


def test_order_scaling_law():
    P = configs.square(4, 2, leaf_size=8, leaf_size_rho=16, cheb_p=3)
    m = P.mesh
    s0 = 0.6
    s = np.full(m.n_nodes, s0)
    k = np.ones(m.n_nodes)
    rng = np.random.default_rng(5)
    w = rng.standard_normal(m.n_dofs)
    u = rng.standard_normal(m.n_dofs)
    m2 = Mesh(m.dim, 2.0 * m.coords, m.cells, m.cell_interior, m.n_dofs, 0.0, m.info)
    m1 = Mesh(m.dim, m.coords, m.cells, m.cell_interior, m.n_dofs, 0.0, m.info)
    ones = np.ones(m.n_nodes)
    a1 = bilinear(m1, s, k, P.opts, w, u)
    a2 = bilinear(m2, s, k, P.opts, w, u)
    c = 2.0 ** (2 - 2 * s0)
    assert abs(a2 - c * a1) <= 1e-12 * abs(a2)
    d1 = directional(m1, s, k, P.opts, w, u, ds=ones)
    d2 = directional(m2, s, k, P.opts, w, u, ds=ones)
    assert abs(d2 - c * (d1 - 2.0 * math.log(2.0) * a1)) <= 1e-11 * abs(d2), (d2, d1, a1)


def test_kappa_homogeneity_and_symmetry():
    P, w, u = _case()
    s, k = P.s[0], P.kappa[0]
    a = bilinear(P.mesh, s, k, P.opts, w, u)
    dk = directional(P.mesh, s, k, P.opts, w, u, dk=k)
    assert abs(dk - a) <= 1e-12 * abs(a)
    rng = np.random.default_rng(6)
    ds = rng.uniform(-1, 1, P.mesh.n_nodes)
    d_wu = directional(P.mesh, s, k, P.opts, w, u, ds=ds)
    d_uw = directional(P.mesh, s, k, P.opts, u, w, ds=ds)
    assert abs(d_wu - d_uw) <= 1e-12 * abs(d_wu)


def test_objective_through_the_solve():
    """d/dt J(s + t ds) with J = 1/2 ||A_h^{-1} F - u_obs||^2: complex step through the
    dense solve against central differences."""
    from oracle.adjoint import objective_directional
    from oracle.assembly import load_vector
    from oracle.h2 import assemble_h2
    from oracle.solve import solve_dense
    P = configs.square(4, 2, leaf_size=8, leaf_size_rho=16, cheb_p=3)
    m = P.mesh
    F = load_vector(m, P.f, P.opts)
    u_obs = 0.5 * solve_dense(*(lambda r: (r["B"] + r["K"] + r["M"], F))(assemble_h2(m, P.s[0], P.kappa[0], P.opts)))
    ds = np.random.default_rng(7).uniform(-1, 1, m.n_nodes) * 0.05

    def J(s):
        r = assemble_h2(m, s, P.kappa[0], P.opts)
        u = solve_dense(r["B"] + r["K"] + r["M"], F)
        return 0.5 * np.sum((u - u_obs) ** 2)
    cs = objective_directional(m, P.s[0], P.kappa[0], P.opts, F, u_obs, ds=ds)
    eps = 1e-5
    fd = (J(P.s[0] + eps * ds) - J(P.s[0] - eps * ds)) / (2 * eps)
    assert abs(cs - fd) <= 1e-7 * abs(cs), (cs, fd)
