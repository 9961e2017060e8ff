"""Graded exterior meshes for the density (the remark on quasi-uniform exterior meshes after
Sec. 7.2: grid lines graded away from the interface use the decay of gamma to cut the
quadrature points of Omega_e).

* The band's first layer has the interior spacing, the next ones grow by the ratio q
  until the last line lands on the band's width.
* The interior grid, its jitter and the dofs are those of the uniform mesh; the
  exterior has O(log n) layers.
* The oracle's density at every interior quadrature point changes by less than
  5e-4 relative against the uniform exterior band (n = 16, q = 1.25), far below the
  discretisation error of the problem.
"""
import numpy as np

from fpde_inputs import configs
from fpde_inputs.meshes import graded_band
from oracle.assembly import rho_direct


def test_graded_band_layers():
    h, q = 1.0 / 128, 1.25
    t = graded_band(h, 0.5, q)
    w = np.diff(np.concatenate([[0.0], t]))
    assert abs(w[0] - h) < 1e-15 and abs(t[-1] - 0.5) < 1e-15
    ratios = w[2:] / w[1:-1]
    assert np.allclose(ratios, q, rtol=1e-12)
    assert w[1] >= w[0] and t.size < 20


def test_graded_square_keeps_the_interior_and_cuts_cells():
    U = configs.square(128)
    G = configs.square(128, graded=1.25)
    mu, mg = U.mesh, G.mesh
    assert mg.n_dofs == mu.n_dofs
    assert np.array_equal(mg.coords[:, :mg.n_dofs], mu.coords[:, :mu.n_dofs])
    assert np.allclose(mg.coords.min(axis=1), -0.5) and np.allclose(mg.coords.max(axis=1), 1.5)
    assert (mg.cell_interior > 0).sum() == (mu.cell_interior > 0).sum()
    assert mg.n_cells < 0.4 * mu.n_cells
    # every interior cell lies in the unit square, every exterior cell outside it
    X = mg.coords[:, mg.cells]
    cen = X.mean(axis=1)
    inside = (cen > 0).all(axis=0) & (cen < 1).all(axis=0)
    assert np.array_equal(inside, mg.cell_interior > 0)


def test_graded_density_matches_uniform_band():
    U = configs.square(16)
    G = configs.square(16, graded=1.25)
    ru = rho_direct(U.mesh, U.s[0], U.kappa[0], U.opts)
    rg = rho_direct(G.mesh, G.s[0], G.kappa[0], G.opts)
    d = np.abs(rg - ru) / np.abs(ru)
    assert d.max() < 5e-4, d.max()
