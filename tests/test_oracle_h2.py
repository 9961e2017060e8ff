"""Pins for the oracle's H2-consistent operator (Sec. 5 and 6.2).

* the dual-tree partition covers every index pair exactly once;
* no far block of K~ contains a touching cell pair (extended boxes), and
  gamma_T = gamma on the density's far blocks (distance guard);
* the interpolation error of K~ and rho~ against the exact split decays
  geometrically with the Chebyshev order p (Prop. 5.1, 6.1);
* the direct density sum converges to the closed form in 1D (constant order).
"""
import math

import numpy as np
import pytest

from fpde_inputs import configs
from oracle.assembly import assemble_split, touching_cells, rho_direct
from oracle.fields import quad_points
from oracle.h2 import (ClusterTree, assemble_K_h2, cell_diameters, cheb_nodes, cluster_h, lagrange,
                       node_tree, partition, rho_h2)


@pytest.fixture(scope="module")
def prob():
    P = configs.square(12, 6, leaf_size=16, leaf_size_rho=32)
    m = P.mesh
    s = 0.3 + 0.2 * (m.coords[0] + m.coords[1])   # linear: no P1 kinks inside cells of the Chebyshev boxes
    k = np.ones_like(s)
    sp = assemble_split(m, s, k, P.opts)
    return P, s, k, sp


def test_tree_uniform_depth_and_median():
    rng = np.random.default_rng(0)
    pts = rng.uniform(size=(2, 1000))
    t = ClusterTree(pts, np.arange(1000), 64)
    assert t.L == 4                                  # ceil(1000/16) = 63 <= 64
    sizes = [t.members[c].size for c in t.leaves()]
    assert max(sizes) <= 64 and min(sizes) >= 62
    allm = np.sort(np.concatenate([t.members[c] for c in t.leaves()]))
    assert np.array_equal(allm, np.arange(1000))


def test_partition_covers_once(prob):
    P, s, k, sp = prob
    tree, lo, hi, node_cells = node_tree(P.mesh, P.opts)
    far, near = partition(tree, lo, hi, P.opts["eta"])
    N = P.mesh.n_dofs
    cnt = np.zeros((N, N), dtype=int)
    for a, b in far + near:
        cnt[np.ix_(tree.members[a], tree.members[b])] += 1
    assert (cnt == 1).all()
    assert len(far) > 0
    # far blocks contain no touching cell pairs
    T = touching_cells(P.mesh)
    for a, b in far:
        ca = sorted({c for i in tree.members[a] for c in node_cells[int(i)]})
        cb = sorted({c for i in tree.members[b] for c in node_cells[int(i)]})
        assert T[ca][:, cb].nnz == 0


def test_lagrange_reproduces_polynomials():
    lo, hi = np.array([0.1, -0.3]), np.array([0.4, 0.2])
    nodes, axes = cheb_nodes(lo, hi, 4)
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, size=(2, 30))
    f = lambda z: 1 + 2 * z[0] - z[1] + z[0] ** 3 * z[1] ** 2 - 0.5 * z[1] ** 3
    L = lagrange(axes, x)
    assert np.allclose(L.T @ f(nodes), f(x), atol=1e-11)
    assert np.allclose(lagrange(axes, nodes), np.eye(16), atol=1e-13)


def test_h2_error_decays_with_p(prob):
    P, s, k, sp = prob
    ek, er = [], []
    for p in (2, 3, 4, 5, 6):
        o = dict(P.opts, cheb_p=p)
        K = assemble_K_h2(P.mesh, s, k, o, K_exact=sp["K"])
        r = rho_h2(P.mesh, s, k, o, Q=sp["Q"])
        ek.append(np.linalg.norm(K - sp["K"]) / np.linalg.norm(sp["K"]))
        er.append(np.abs(r - sp["rho"]).max() / np.abs(sp["rho"]).max())
    for e in (ek, er):
        assert all(e[i + 1] < 0.6 * e[i] for i in range(len(e) - 1)), e
    assert ek[-1] < 3e-4 and er[-1] < 3e-4


def test_rho_direct_1d_closed_form():
    # constant s on Omega=(-L,L): rho(x) = [(x-a)^{-2s} - (x+L)^{-2s} + (b-x)^{-2s} - (L-x)^{-2s}] / (2s)
    # with S_tau = [a, b]; the per-element Gauss sum converges to it.
    s = 0.4
    errs = []
    for nq in (3, 6, 12):
        P = configs.interval(n_int=16, n_ext=8)
        m = P.mesh
        sv = np.full(m.n_nodes, s)
        o = dict(P.opts, nq_reg=nq)
        rho = rho_direct(m, sv, np.ones_like(sv), o)
        from oracle.fields import quad_points
        Q = quad_points(m, nq)
        qi = np.flatnonzero(m.cell_interior[Q["cell"]] > 0)
        x = Q["x"][0, qi]
        h = m.info["h"]
        L = 2.0
        c = Q["cell"][qi]
        left = m.coords[0, m.cells[:, c]].min(axis=0)
        a = left - h
        b = left + 2 * h
        ref = ((x - a) ** (-2 * s) - (x + L) ** (-2 * s) + (b - x) ** (-2 * s) - (L - x) ** (-2 * s)) / (2 * s)
        errs.append(np.abs(rho - ref).max() / ref.max())
    assert errs[1] < errs[0] and errs[2] < errs[1] and errs[2] < 1e-6, errs


@pytest.mark.parametrize("n,graded", [(8, 0.0), (16, 1.5)])
def test_density_partition_local_guard(n, graded):
    # Sec. 6.2: gamma_T = gamma must hold on every far density block, i.e. no far pair of
    # clusters holds points of touching cells.  The guard dist > h_a + h_b uses the cells of
    # each cluster's own points; on a graded exterior it is much smaller than 2 h_max for the
    # interior clusters, and the partition still covers every point pair once.
    P = configs.square(n, n // 2, graded=graded, leaf_size_rho=32)
    m = P.mesh
    Q = quad_points(m, P.opts["nq_reg"])
    nq = Q["w"].size
    tree = ClusterTree(Q["x"], np.arange(nq), P.opts["leaf_size_rho"])
    lo = np.array([Q["x"][:, tree.members[c]].min(axis=1) for c in range(tree.n_clusters)])
    hi = np.array([Q["x"][:, tree.members[c]].max(axis=1) for c in range(tree.n_clusters)])
    hq = cell_diameters(m)[Q["cell"]]
    hc = cluster_h(tree, hq)
    # the diameters are the longest edges, brute force per cell
    X = m.coords[:, m.cells]
    hb = np.array([max(np.linalg.norm(X[:, a, c] - X[:, b, c]) for a in range(3) for b in range(a + 1, 3))
                   for c in range(m.n_cells)])
    assert np.allclose(cell_diameters(m), hb, rtol=1e-15, atol=0)
    for c in range(tree.n_clusters):
        assert hc[c] == hq[tree.members[c]].max()
    far, near = partition(tree, lo, hi, P.opts["eta"], hc)
    cnt = np.zeros((nq, nq), dtype=np.int8)
    for a, b in far + near:
        cnt[np.ix_(tree.members[a], tree.members[b])] += 1
    assert (cnt == 1).all()
    assert len(far) > 0
    T = touching_cells(m)
    for a, b in far:
        assert T[Q["cell"][tree.members[a]]][:, Q["cell"][tree.members[b]]].nnz == 0
    if graded:
        # interior clusters keep a separation near the interior cells' size
        inner = [c for c in tree.leaves() if (m.cell_interior[Q["cell"][tree.members[c]]] > 0).all()]
        assert inner and max(hc[c] for c in inner) < 0.4 * hb.max()
