"""Pins for the oracle's solves (O8): Cholesky and CG agree on the discrete system.

The closed-form solutions of the fractional Laplacian pin the solve end to end
(tests/test_oracle_assembly.py uses ``solve_dense``); here CG is checked
against the factorisation and against the residual it reports.
"""
import numpy as np

from fpde_inputs import configs
from oracle.assembly import assemble_split, load_vector
from oracle.solve import conjugate_gradient, solve_dense


def test_cg_matches_cholesky_and_residual():
    P = configs.interval(n_int=48, n_ext=24)
    sp = assemble_split(P.mesh, P.s[0], P.kappa[0], P.opts)
    A = sp["B"] + sp["K"] + sp["M"]
    F = load_vector(P.mesh, P.f, P.opts)
    u = solve_dense(A, F)
    assert np.linalg.norm(A @ u - F) < 1e-12 * np.linalg.norm(F)
    uc, it, rel = conjugate_gradient(A, F, rtol=1e-12)
    assert rel <= 1e-12 and 0 < it <= 2 * len(F)
    assert np.linalg.norm(A @ uc - F) / np.linalg.norm(F) < 2e-12
    assert np.linalg.norm(uc - u) < 1e-9 * np.linalg.norm(u)


def test_solve_dense_several_rhs():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((30, 30))
    A = X @ X.T + 30 * np.eye(30)
    B = rng.standard_normal((30, 3))
    U = solve_dense(A, B)
    for j in range(3):
        assert np.allclose(U[:, j], np.linalg.solve(A, B[:, j]), rtol=1e-12, atol=1e-14)
