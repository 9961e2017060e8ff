"""Full-size parity: the 128 x 128 square workload (16129 dofs, 131072 cells) in the
launch configuration the benchmark times, checked on sampled rows that the oracle
computes one by one (oracle.sampled), at 1e-10 of the output's max norm."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from fpde_inputs import configs  # noqa: E402
from oracle.sampled import SampledOracle  # noqa: E402

TOL = 1e-10


def test_square128_sampled_rows():
    import paper_2302_02863_amd as fp
    P = configs.square(128)
    m = P.mesh
    print(f"[fullsize] build N={m.n_dofs}", flush=True)
    op = fp.Operator(m, P.s, P.kappa, P.opts)
    x = torch.tensor(P.x, device="cuda")
    y = op.apply(x)
    parts = {k: op.apply(x, parts=v) for k, v in (("B", fp.PART_B), ("M", fp.PART_M),
                                                  ("K", fp.PART_KNEAR | fp.PART_KFAR))}
    torch.cuda.synchronize()
    y = y.cpu().numpy()[0, :, 0]
    parts = {k: v.cpu().numpy()[0, :, 0] for k, v in parts.items()}
    rng = np.random.default_rng(17)
    # random rows plus rows next to the interface (first/last grid lines of the interior)
    rows = list(rng.choice(m.n_dofs, size=4, replace=False))
    xy = m.coords[:, :m.n_dofs]
    h = m.info["h"]
    near_bdry = np.flatnonzero((xy.min(axis=0) < 1.6 * h) | (xy.max(axis=0) > 1 - 1.6 * h))
    rows += list(rng.choice(near_bdry, size=2, replace=False))
    so = SampledOracle(m, P.s[0], P.kappa[0], P.opts)
    out = so.row_apply(rows, P.x[0, :, 0])
    scale = np.abs(y).max()
    for key in ("B", "M", "K"):
        err = np.abs(parts[key][rows] - out[key]).max() / scale
        print(f"[fullsize] {key}: max err / |y|_inf = {err:.2e}", flush=True)
        assert err < TOL, key
    err = np.abs(y[rows] - out["total"]).max() / scale
    print(f"[fullsize] total: {err:.2e}", flush=True)
    assert err < TOL
