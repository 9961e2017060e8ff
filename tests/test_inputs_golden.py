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
