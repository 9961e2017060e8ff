"""CPU tests of the C ABI and the host planner (no GPU needed).

* the library loads and exports every function include/fpde.h declares;
* the library's Gauss-Legendre rule is bit-identical to the oracle's;
* a plan-only build produces the same touching pairs (canonical orientation),
  the same KD trees and boxes (bit for bit) and the same block partitions as
  the oracle;
* input validation returns the documented error codes before any device work.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from fpde_inputs import configs
from oracle.rules import gauss01
from oracle.singular import touching_pairs
from oracle.h2 import ClusterTree, box_of, cell_diameters, cluster_h, node_tree, partition
from oracle.fields import quad_points

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fp():
    import paper_2302_02863_amd as fp
    fp.lib()
    return fp


def test_library_exports_every_declared_symbol(fp):
    hdr = open(os.path.join(ROOT, "include", "fpde.h")).read()
    names = sorted(set(re.findall(r"^\s*(?:fpde_status|void|const char\s*\*)\s*(fpde_\w+)\s*\(", hdr, re.M)))
    assert len(names) >= 10, names
    L = ctypes.CDLL(fp._abi.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_gauss_legendre_bitwise(fp):
    for n in range(1, 17):
        x, w = fp.gauss_legendre(n)
        xo, wo = gauss01(n)
        assert np.array_equal(x, xo), n
        assert np.array_equal(w, wo), n


def _plan(fp, P):
    return fp.Operator(P.mesh, P.s, P.kappa, P.opts, plan_only=True)


CASES = {
    "square_jitter": lambda: configs.square(12, 6, leaf_size=16, leaf_size_rho=32),
    "square_regular": lambda: configs.square(8, 4, jitter=0.0, leaf_size=8, leaf_size_rho=16),
    "interval": lambda: configs.interval(n_int=40, n_ext=10, leaf_size=8, leaf_size_rho=16),
    "disk": lambda: configs.disk(8, s_const=0.6, leaf_size=16, leaf_size_rho=32),
}


@pytest.mark.parametrize("case", list(CASES))
def test_pairs_match_oracle(fp, case):
    P = CASES[case]()
    op = _plan(fp, P)
    got = op.export("PAIRS").reshape(-1, 8)
    ref = touching_pairs(P.mesh)
    assert got.shape[0] == len(ref)
    kinds = {"I": 0, "E": 1, "V": 2}
    d = P.mesh.dim
    for row, (kind, c0, c1, v0, v1) in zip(got, ref):
        assert row[0] == kinds[kind] and row[1] == c0 and row[2] == c1
        assert tuple(row[3:3 + d + 1]) == tuple(v0)
        if d == 2:
            assert tuple(row[6:8]) == tuple(v1[1:])
        else:
            assert row[6] == v1[1]
    st = op.stats()
    assert st["n_pairs_identical"] == int(P.mesh.cell_interior.sum())


def _leaf_sets(perm, leafptr):
    return [tuple(sorted(perm[leafptr[i]:leafptr[i + 1]])) for i in range(len(leafptr) - 1)]


@pytest.mark.parametrize("case", list(CASES))
def test_k_tree_and_partition_match_oracle(fp, case):
    P = CASES[case]()
    op = _plan(fp, P)
    tree, lo, hi, _ = node_tree(P.mesh, P.opts)
    perm = op.export("K_PERM")
    leafptr = op.export("K_LEAFPTR")
    ref_leaves = [tuple(sorted(tree.members[c])) for c in tree.leaves()]
    assert _leaf_sets(perm, leafptr) == ref_leaves
    boxes = op.export("K_BOXES").reshape(tree.n_clusters, 2, P.mesh.dim)
    assert np.array_equal(boxes[:, 0], lo) and np.array_equal(boxes[:, 1], hi)
    far, near = partition(tree, lo, hi, P.opts["eta"])
    gf = {tuple(p) for p in op.export("K_FAR").reshape(-1, 2)}
    gn = {tuple(p) for p in op.export("K_NEAR").reshape(-1, 2)}
    assert gf == set(far) and gn == set(near)


# 73,728 quadrature points: the planner splits the tree levels, the partition's
# subtrees and the sort of its pair lists on host threads (at least 65,536 points, a
# front of 1,024 pairs, 16,384 pairs)
RHO_CASES = dict(CASES, square_threads=lambda: configs.square(32, 16, leaf_size=16, leaf_size_rho=32))


@pytest.mark.parametrize("case", list(RHO_CASES))
def test_rho_tree_and_partition_match_oracle(fp, case):
    P = RHO_CASES[case]()
    op = _plan(fp, P)
    m = P.mesh
    Q = quad_points(m, P.opts["nq_reg"])
    nq = Q["w"].size
    tree = ClusterTree(Q["x"], np.arange(nq), P.opts["leaf_size_rho"])
    perm = op.export("RHO_PERM")
    assert perm.size == nq
    boxes = op.export("RHO_BOXES").reshape(tree.n_clusters, 2, m.dim)
    for c in range(tree.n_clusters):
        blo, bhi = box_of(Q["x"][:, tree.members[c]])
        assert np.array_equal(boxes[c, 0], blo) and np.array_equal(boxes[c, 1], bhi), c
    leaf0 = (1 << tree.L) - 1
    for li, c in enumerate(tree.leaves()):
        pass
    lo = boxes[:, 0]
    hi = boxes[:, 1]
    far, near = partition(tree, lo, hi, P.opts["eta"], cluster_h(tree, cell_diameters(m)[Q["cell"]]))
    is_int = m.cell_interior[Q["cell"]] > 0
    has_int = [bool(is_int[tree.members[c]].any()) for c in range(tree.n_clusters)]
    ef = op.export("RHO_FAR").reshape(-1, 2)
    en = op.export("RHO_NEAR").reshape(-1, 2)
    gf = {tuple(p) for p in ef}
    gn = {tuple(p) for p in en}
    assert gf == {p for p in far if has_int[p[0]]}
    assert gn == {p for p in near if has_int[p[0]]}
    for e in (ef, en):   # ordered by target, then source, without repeats (the device lists' order)
        key = e[:, 0].astype(np.int64) * tree.n_clusters + e[:, 1]
        assert np.all(np.diff(key) > 0)
    # tree membership: leaves hold the same points
    sizes = np.diff([0] + [tree.members[c].size for c in tree.leaves()]).size
    assert sizes == tree.n_clusters - leaf0


def _bad(fp, P, **kw):
    s = kw.pop("s", P.s)
    kappa = kw.pop("kappa", P.kappa)
    mesh = kw.pop("mesh", P.mesh)
    opts = dict(P.opts, **kw)
    with pytest.raises(fp.FpdeError) as e:
        fp.Operator(mesh, s, kappa, opts, plan_only=True)
    return e.value.status


def test_validation_errors(fp):
    from fpde_inputs.meshes import Mesh
    P = configs.square(4, 2)
    assert _bad(fp, P, s=P.s + 0.5) == fp._abi.FPDE_EDOMAIN          # s > s_bar
    assert _bad(fp, P, kappa=-P.kappa) == fp._abi.FPDE_EDOMAIN       # kappa <= 0
    assert _bad(fp, P, s_bar=1.0) == fp._abi.FPDE_EDOMAIN
    m = P.mesh
    bad_int = m.cell_interior.copy()
    bad_int[:] = 0                                                   # interior nodes in exterior cells
    assert _bad(fp, P, mesh=Mesh(2, m.coords, m.cells, bad_int, m.n_dofs)) == fp._abi.FPDE_EINVAL
    all_int = np.ones_like(m.cell_interior)                          # |Omega_e| = 0 and R = 0
    assert _bad(fp, P, mesh=Mesh(2, m.coords, m.cells, all_int, m.n_dofs)) == fp._abi.FPDE_EINVAL
    cells = m.cells.copy()
    cells[0, 0] = m.n_nodes + 5
    assert _bad(fp, P, mesh=Mesh(2, m.coords, cells, m.cell_interior, m.n_dofs)) == fp._abi.FPDE_EINVAL
    assert _bad(fp, P, cheb_p=20) == fp._abi.FPDE_EINVAL
    assert _bad(fp, P, recompress_tol=-1e-3) == fp._abi.FPDE_EINVAL
    assert _bad(fp, P, recompress_tol=1.0) == fp._abi.FPDE_EINVAL
    assert _bad(fp, P, recompress_tol=1e-3, cheb_p=6) == fp._abi.FPDE_EINVAL   # rank 36 > 32


def test_plan_only_rejects_apply(fp):
    import torch
    P = configs.square(4, 2)
    op = _plan(fp, P)
    st = op.stats()
    assert st["n_dofs"] == P.mesh.n_dofs and st["csr_nnz"] > 0
    n = ctypes.c_int64(0)
    r = fp.lib().fpde_apply(op._h, 0, ctypes.c_void_p(1), ctypes.c_void_p(2), 1, None)
    assert r == fp._abi.FPDE_ESTATE
