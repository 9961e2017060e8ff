"""The square workload reproduces the mesh the paper prints counts for: its finest
variable-order test mesh T_6 (Sec. 7.2), with the interior domain half the width of
the whole domain.  Fixture: tests/golden/paper_mesh_T6.txt."""
import os

import numpy as np

from fpde_inputs import configs

HERE = os.path.dirname(os.path.abspath(__file__))


def _fixture(name):
    vals = {}
    for line in open(os.path.join(HERE, "golden", name)):
        line = line.split("#", 1)[0].split()
        if len(line) == 2:
            vals[line[0]] = float(line[1])
    return vals


def test_square128_matches_the_papers_T6_counts():
    g = _fixture("paper_mesh_T6.txt")
    m = configs.square(128).mesh
    assert m.n_dofs == int(g["interior_dofs"])
    assert m.cells.shape[1] == int(g["cells_total"])
    inner = m.coords[:, :m.n_dofs]
    h = m.info["h"]
    # interior nodes are jittered by at most 0.1 h; the interior domain's edge lies one h beyond them
    w_in = (inner.max(axis=1) - inner.min(axis=1)).max() + 2 * h
    w_all = (m.coords.max(axis=1) - m.coords.min(axis=1)).max()
    assert abs(w_in / w_all - g["interior_to_total_width"]) < 0.25 * h / w_all
    # every interior cell has its three vertices within the interior square
    ci = m.cells[:, m.cell_interior > 0]
    assert np.all(m.coords[:, ci].min(axis=(1, 2)) >= -1e-12)
    assert np.all(m.coords[:, ci].max(axis=(1, 2)) <= 1 + 1e-12)


def test_bump_recipe_is_the_papers_variable_order_test():
    # Sec. 7.2: Omega = (-2,2)^2, Omega_i = (-1,1)^2, T_6 has the printed counts; the order is
    # s* = 0.7 outside the bump's support square of side l = 1 centred at (-0.4, 0.4), and
    # s* + eta e^{-2} at the centre (bump(0) = e^{-1} in each direction), eta = 0.2
    g = _fixture("paper_mesh_T6.txt")
    P = configs.bump(6)
    m = P.mesh
    assert m.n_dofs == int(g["interior_dofs"]) and m.cells.shape[1] == int(g["cells_total"])
    assert np.allclose(m.coords.min(axis=1), -2.0) and np.allclose(m.coords.max(axis=1), 2.0)
    inner = m.coords[:, :m.n_dofs]
    assert inner.min() > -1.0 and inner.max() < 1.0
    x1, x2 = m.coords
    s = P.s[0]
    out = (np.abs(x1 + 0.4) >= 0.5) | (np.abs(x2 - 0.4) >= 0.5)
    inner_sq = (np.abs(x1 + 0.4) < 0.45) & (np.abs(x2 - 0.4) < 0.45)   # exp(-1/(1-r^2)) underflows as |r| -> 1
    assert np.all(s[out] == 0.7) and np.all(s[~out] >= 0.7) and np.all(s[inner_sq] > 0.7)
    c = configs.bump_order(np.array([-0.4]), np.array([0.4]))
    assert abs(c[0] - (0.7 + 0.2 * np.exp(-2.0))) < 1e-15
    # one coordinate direction at a time: bump(x; 1) = exp(-1 / (1 - 4 x^2))
    x = np.array([0.1, 0.3, 0.49])
    ref = 0.7 + 0.2 * np.exp(-1.0) * np.exp(-1.0 / (1.0 - 4.0 * x ** 2))
    assert np.allclose(configs.bump_order(-0.4 + np.zeros(3), 0.4 + x), ref, rtol=1e-14, atol=0)
    assert P.f.min() == P.f.max() == 20.0 and np.all(P.kappa == 1.0)
    # the grids are nested: every node of T_j is a node of T_{j+1}
    a = configs.bump(2).mesh.coords
    b = configs.bump(3).mesh.coords
    key = lambda X: set(map(tuple, np.round(X.T * 1024).astype(np.int64)))  # noqa: E731
    assert key(a) <= key(b)
