"""GPU parity of the HIP path against the oracle (FP64 mode, tolerance 1e-10).

Every comparison goes through the C ABI (libfpde.so): exported CSR values of B
and M, the density at interior quadrature points, each part of the apply, the
full apply, several right-hand sides and fields, float32 vectors, and
run-to-run bitwise reproducibility.  Sizes span several leaves/tiles and
ragged leaves; the oracle finishes each case in seconds.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from fpde_inputs import configs  # noqa: E402
from oracle.h2 import assemble_h2, assemble_K_h2  # noqa: E402
from oracle.assembly import assemble_split  # noqa: E402

TOL = 1e-10

CASES = {
    "square": lambda: configs.square(12, 6, leaf_size=16, leaf_size_rho=32, cheb_p=4),
    "square_regular": lambda: configs.square(10, 5, jitter=0.0, leaf_size=12, leaf_size_rho=24, cheb_p=3),
    "interval": lambda: configs.interval(n_int=64, n_ext=16, leaf_size=8, leaf_size_rho=16, cheb_p=5),
    "disk": lambda: configs.disk(8, s_const=0.6, leaf_size=16, leaf_size_rho=32, cheb_p=4),
    "disk_far": lambda: configs.disk(16, s_const=0.6, leaf_size=16, leaf_size_rho=32, cheb_p=4),
}

_cache = {}


def _case(name):
    if name not in _cache:
        import paper_2302_02863_amd as fp
        P = CASES[name]()
        print(f"[parity] building case {name}: N={P.mesh.n_dofs} cells={P.mesh.n_cells}", flush=True)
        split = assemble_split(P.mesh, P.s[0], P.kappa[0], P.opts)
        ref = assemble_h2(P.mesh, P.s[0], P.kappa[0], P.opts, split=split)
        op = fp.Operator(P.mesh, P.s, P.kappa, P.opts)
        _cache[name] = (P, ref, op)
    return _cache[name]


def _dense_csr(op, which):
    ptr = op.export("CSR_ROWPTR")
    cols = op.export("CSR_COLS")
    vals = op.export(which)
    N = op.n_dofs
    A = np.zeros((N, N))
    for i in range(N):
        A[i, cols[ptr[i]:ptr[i + 1]]] = vals[ptr[i]:ptr[i + 1]]
    return A


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("name", list(CASES))
def test_B_and_M_values(name):
    P, ref, op = _case(name)
    assert _rel(_dense_csr(op, "CSR_B"), ref["B"]) < TOL
    assert _rel(_dense_csr(op, "CSR_M"), ref["M"]) < TOL


@pytest.mark.parametrize("name", list(CASES))
def test_density(name):
    P, ref, op = _case(name)
    rho = op.export("RHO")
    qi = ref["split"]["qi"]
    assert _rel(rho[qi], ref["rho"]) < TOL
    # zero at exterior points
    mask = np.ones(rho.size, bool)
    mask[qi] = False
    assert np.all(rho[mask] == 0.0)


def _apply(op, x, parts):
    xt = torch.tensor(x, device="cuda")
    y = op.apply(xt, parts=parts)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_apply_parts_and_full(name):
    import paper_2302_02863_amd as fp
    P, ref, op = _case(name)
    x = P.x
    xv = x[0, :, 0]
    K, parts = assemble_K_h2(P.mesh, P.s[0], P.kappa[0], P.opts, K_exact=ref["split"]["K"], return_parts=True)
    tree = parts["tree"]
    Knear = np.zeros_like(K)
    for a, b in parts["near"]:
        ix = np.ix_(tree.members[a], tree.members[b])
        Knear[ix] = K[ix]
    Kfar = K - Knear
    for mask, Aref in ((fp.PART_B, ref["B"]), (fp.PART_M, ref["M"]), (fp.PART_KNEAR, Knear),
                       (fp.PART_KFAR, Kfar)):
        y = _apply(op, x, mask)[0, :, 0]
        yr = Aref @ xv
        if not np.any(Aref):          # e.g. no far blocks on a tiny mesh: the part must be exactly zero
            assert np.all(y == 0.0), mask
            continue
        assert np.linalg.norm(y - yr) / np.linalg.norm(yr) < TOL, mask
    A = ref["B"] + ref["K"] + ref["M"]
    y = _apply(op, x, fp.PART_ALL)[0, :, 0]
    yr = A @ xv
    err = np.linalg.norm(y - yr) / np.linalg.norm(yr)
    print(f"[parity] {name}: full apply rel err {err:.2e}")
    assert err < TOL


def test_apply_parts_several_rhs():
    """The several-right-hand-side kernels on part subsets: B + M together read the
    ELL rows by leaf slot, B or M alone the CSR; the near panels alone and with both."""
    import paper_2302_02863_amd as fp
    P, ref, op = _case("square")
    K, parts = assemble_K_h2(P.mesh, P.s[0], P.kappa[0], P.opts, K_exact=ref["split"]["K"], return_parts=True)
    tree = parts["tree"]
    Knear = np.zeros_like(K)
    for a, b in parts["near"]:
        ix = np.ix_(tree.members[a], tree.members[b])
        Knear[ix] = K[ix]
    rng = np.random.default_rng(21)
    x = rng.standard_normal((1, op.n_dofs, 8))
    for mask, Aref in ((fp.PART_B, ref["B"]), (fp.PART_M, ref["M"]), (fp.PART_B | fp.PART_M, ref["B"] + ref["M"]),
                       (fp.PART_KNEAR, Knear), (fp.PART_B | fp.PART_M | fp.PART_KNEAR, ref["B"] + ref["M"] + Knear)):
        y = _apply(op, x, mask)[0]
        yr = Aref @ x[0]
        err = np.linalg.norm(y - yr, axis=0) / np.linalg.norm(yr, axis=0)
        assert err.max() < TOL, (mask, err.max())


def test_many_rhs_fields_and_float32():
    import paper_2302_02863_amd as fp
    P = configs.square(8, 4, leaf_size=12, leaf_size_rho=24, cheb_p=3)
    m = P.mesh
    s2 = np.stack([P.s[0], np.clip(0.2 + 0.5 * m.coords[0] ** 2 * 0.3 + 0.1 * m.coords[1], 0.05, 0.85)])
    k2 = np.stack([P.kappa[0], np.ones(m.n_nodes) * 1.5])
    op = fp.Operator(m, s2, k2, P.opts)
    rng = np.random.default_rng(5)
    R = 5
    x = rng.standard_normal((2, m.n_dofs, R))
    y = _apply(op, x, fp.PART_ALL)
    for f in range(2):
        ref = assemble_h2(m, s2[f], k2[f], P.opts)
        A = ref["B"] + ref["K"] + ref["M"]
        yr = A @ x[f]
        assert np.linalg.norm(y[f] - yr) / np.linalg.norm(yr) < TOL, f
    # float32 vectors: the apply computes in FP64 and rounds the result once
    x32 = x.astype(np.float32)
    y32 = op.apply(torch.tensor(x32, device="cuda"))
    torch.cuda.synchronize()
    y64 = _apply(op, x32.astype(np.float64), fp.PART_ALL)
    assert np.abs(y32.cpu().numpy() - y64).max() <= 1e-6 * np.abs(y64).max()


def test_wide_rhs_fallback_and_profiled_path():
    """Many right-hand sides take the per-level sweep path; a profiled apply (events between
    the launches) must equal the plain apply bit for bit, and both the oracle."""
    import paper_2302_02863_amd as fp
    P, ref, op = _case("square")
    A = ref["B"] + ref["K"] + ref["M"]
    rng = np.random.default_rng(9)
    for R in (40, 3):
        x = rng.standard_normal((1, op.n_dofs, R))
        y = _apply(op, x, fp.PART_ALL)[0]
        yr = A @ x[0]
        assert np.linalg.norm(y - yr) / np.linalg.norm(yr) < TOL, R
    y_plain = _apply(op, P.x, fp.PART_ALL)
    op.profile(True)
    y_prof = _apply(op, P.x, fp.PART_ALL)
    pr = op.profile(False)
    assert pr["n_applies"] == 1 and pr["ms_out"] > 0
    assert np.array_equal(y_plain, y_prof)


MIXED_TOL = 1e-6   # per matvec, relative 2-norm against the FP64 oracle


@pytest.mark.parametrize("name", list(CASES))
def test_mixed_precision_apply(name):
    """FP32 near panels, bases, transfers and coupling (FP64 CSR of B + M): the
    matvec stays within 1e-6 of the FP64 oracle; FPDE_PART_FP64 on the same
    operator reproduces the FP64 operator bit for bit."""
    import paper_2302_02863_amd as fp
    P, ref, op64 = _case(name)
    o = dict(P.opts)
    o["precision"] = "mixed"
    op = fp.Operator(P.mesh, P.s, P.kappa, o)
    A = ref["B"] + ref["K"] + ref["M"]
    rng = np.random.default_rng(21)
    for x in (P.x[0, :, 0], rng.standard_normal(op.n_dofs), np.sin(np.pi * P.mesh.coords[0, :op.n_dofs])):
        y = _apply(op, x.reshape(1, -1, 1), fp.PART_ALL)[0, :, 0]
        yr = A @ x
        err = np.linalg.norm(y - yr) / np.linalg.norm(yr)
        assert err < MIXED_TOL, err
    print(f"[parity] {name}: mixed apply rel err {err:.2e}")
    y64 = _apply(op, P.x, fp.PART_ALL | fp.PART_FP64)
    assert np.array_equal(y64, _apply(op64, P.x, fp.PART_ALL))
    # plain and profiled mixed applies agree bit for bit
    yg = _apply(op, P.x, fp.PART_ALL)
    op.profile(True)
    yp = _apply(op, P.x, fp.PART_ALL)
    op.profile(False)
    assert np.array_equal(yg, yp)
    op.close()


def test_top_level_sweeps(monkeypatch):
    """Cap the subtree depths so the upsweep takes a ticket at every level (and the
    multi-RHS path runs its top sweeps); results must not change."""
    import paper_2302_02863_amd as fp
    P = configs.square(16, 8, leaf_size=8, leaf_size_rho=32, cheb_p=3)
    ref = assemble_h2(P.mesh, P.s[0], P.kappa[0], P.opts)
    A = ref["B"] + ref["K"] + ref["M"]
    for depth in ("0", "1", "2"):
        monkeypatch.setenv("FPDE_MAX_SUBTREE_DEPTH", depth)
        for prec in ("fp64", "mixed"):
            o = dict(P.opts)
            o["precision"] = prec
            op = fp.Operator(P.mesh, P.s, P.kappa, o)
            for _ in range(3):   # tickets reset themselves between launches
                y = _apply(op, P.x, fp.PART_ALL)[0, :, 0]
                yr = A @ P.x[0, :, 0]
                tol = TOL if prec == "fp64" else MIXED_TOL
                assert np.linalg.norm(y - yr) / np.linalg.norm(yr) < tol, (depth, prec)
            op.close()


def test_bitwise_reproducible():
    import paper_2302_02863_amd as fp
    P, ref, op = _case("square")
    y1 = _apply(op, P.x, fp.PART_ALL)
    y2 = _apply(op, P.x, fp.PART_ALL)
    assert np.array_equal(y1, y2)
    op2 = fp.Operator(P.mesh, P.s, P.kappa, P.opts)
    y3 = _apply(op2, P.x, fp.PART_ALL)
    assert np.array_equal(y1, y3)


def test_load_vector():
    from oracle.assembly import load_vector
    P, ref, op = _case("disk")
    f = np.cos(P.mesh.coords[0]) + P.mesh.coords[1] ** 2
    F = op.load_vector(torch.tensor(f, device="cuda"))
    torch.cuda.synchronize()
    Fr = load_vector(P.mesh, f, P.opts)
    assert _rel(F.cpu().numpy(), Fr) < 1e-13


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_fields_and_rhs(precision):
    """Several order fields x 64 right-hand sides (the batched workload's shape at a
    small mesh): near panels as MFMA GEMMs, FP64 (1e-10) and FP32 operator data (1e-6)."""
    import paper_2302_02863_amd as fp
    P = configs.batched(16, n_fields=3, nrhs=64, leaf_size=16, leaf_size_rho=32, cheb_p=4)
    m = P.mesh
    o = dict(P.opts)
    o["precision"] = precision
    op = fp.Operator(m, P.s, P.kappa, o)
    tol = TOL if precision == "fp64" else MIXED_TOL
    for dt in (torch.float64, torch.float32):
        x = torch.tensor(P.x, device="cuda", dtype=dt)
        y = op.apply(x).double().cpu().numpy()
        for f in range(P.s.shape[0]):
            ref = assemble_h2(m, P.s[f], P.kappa[f], P.opts)
            A = ref["B"] + ref["K"] + ref["M"]
            yr = A @ x[f].double().cpu().numpy()
            err = np.linalg.norm(y[f] - yr, axis=0) / np.linalg.norm(yr, axis=0)
            lim = tol if dt == torch.float64 else max(tol, 1e-6)
            assert err.max() < lim, (precision, dt, f, err.max())
    op.close()
