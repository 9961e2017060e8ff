"""The row-sampled oracle equals the dense H2-consistent oracle row by row."""
import numpy as np
import pytest

from fpde_inputs import configs
from oracle.h2 import assemble_h2
from oracle.sampled import SampledOracle


@pytest.mark.parametrize("mk", [
    lambda: configs.square(12, 6, leaf_size=16, leaf_size_rho=32, cheb_p=4),
    lambda: configs.disk(12, s_const=0.6, leaf_size=16, leaf_size_rho=32, cheb_p=4),
    lambda: configs.interval(n_int=64, n_ext=16, leaf_size=8, leaf_size_rho=16, cheb_p=5),
])
def test_rows_match_dense(mk):
    P = mk()
    m = P.mesh
    ref = assemble_h2(m, P.s[0], P.kappa[0], P.opts)
    x = P.x[0, :, 0]
    so = SampledOracle(m, P.s[0], P.kappa[0], P.opts)
    rng = np.random.default_rng(3)
    rows = rng.choice(m.n_dofs, size=6, replace=False)
    out = so.row_apply(rows, x)
    for key in ("B", "K", "M"):
        yr = (ref[key] @ x)[rows]
        scale = np.abs(ref[key] @ x).max()
        assert np.abs(out[key] - yr).max() < 1e-12 * scale, key


def test_rows_for_two_vectors_in_turn():
    """Rows for a second vector must not reuse far-field coefficients of the first."""
    import numpy as np
    from fpde_inputs import configs
    from oracle.h2 import assemble_h2
    from oracle.sampled import SampledOracle
    P = configs.square(10, 5, leaf_size=12, leaf_size_rho=24, cheb_p=3)
    m = P.mesh
    ref = assemble_h2(m, P.s[0], P.kappa[0], P.opts)
    A = ref["B"] + ref["K"] + ref["M"]
    so = SampledOracle(m, P.s[0], P.kappa[0], P.opts)
    rng = np.random.default_rng(2)
    rows = [0, m.n_dofs // 2, m.n_dofs - 1]
    for _ in range(2):
        x = rng.standard_normal(m.n_dofs)
        out = so.row_apply(rows, x)
        yr = A @ x
        assert np.abs(out["total"] - yr[rows]).max() <= 1e-12 * np.abs(yr).max()
