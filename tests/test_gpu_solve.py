"""GPU solve (CG with iterative refinement on the FP64 residual) against the oracle.

The oracle's dense H2-consistent matrix A_h = B + K~ + M~ and load vector are
solved by Cholesky (``oracle.solve.solve_dense``); the library's solve must
reach the same discrete solution to 1e-8 relative for every field and
right-hand side, in FP64 and in mixed precision.  The constant-order interval
case also lands on the closed-form solution within the discretisation error.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from fpde_inputs import configs  # noqa: E402
from oracle.assembly import assemble_split, load_vector  # noqa: E402
from oracle.h2 import assemble_h2  # noqa: E402
from oracle.solve import solve_dense  # noqa: E402

SOL_TOL = 1e-8

CASES = {
    "interval": lambda **kw: configs.interval(n_int=64, n_ext=16, leaf_size=8, leaf_size_rho=16, cheb_p=5, **kw),
    "interval_const": lambda **kw: configs.interval_const(n_int=64, leaf_size=8, leaf_size_rho=16, cheb_p=5, **kw),
    "square": lambda **kw: configs.square(12, 6, leaf_size=16, leaf_size_rho=32, cheb_p=4, **kw),
}

_cache = {}


def _oracle(name):
    if name not in _cache:
        P = CASES[name]()
        print(f"[solve] oracle for {name}: N={P.mesh.n_dofs}", flush=True)
        split = assemble_split(P.mesh, P.s[0], P.kappa[0], P.opts)
        ref = assemble_h2(P.mesh, P.s[0], P.kappa[0], P.opts, split=split)
        A = ref["B"] + ref["K"] + ref["M"]
        F = load_vector(P.mesh, P.f, P.opts)
        _cache[name] = (P, A, F)
    return _cache[name]


def _op(P, **opts):
    import paper_2302_02863_amd as fp
    o = dict(P.opts)
    o.update(opts)
    return fp.Operator(P.mesh, P.s, P.kappa, o)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_load_vector(name, precision):
    P, A, F = _oracle(name)
    u_ref = solve_dense(A, F)
    op = _op(P, precision=precision)
    Fd = torch.tensor(F, device="cuda").reshape(1, -1, 1)
    print(f"[solve] {name} {precision}", flush=True)
    u, info = op.solve(Fd, rtol=1e-12, maxit=5000)
    torch.cuda.synchronize()
    assert info["converged"] and info["rel_residual"] <= 1e-12, info
    assert _rel(u[0, :, 0].cpu().numpy(), u_ref) < SOL_TOL, info
    if precision == "mixed":
        assert info["refinements"] >= 2, info


def test_solve_closed_form_interval():
    # s = 0.5 on (-1,1), a = C_{1,s}/2: the discrete solution approaches sqrt(1 - x^2)
    P, A, F = _oracle("interval_const")
    op = _op(P)
    u, info = op.solve(torch.tensor(F, device="cuda").reshape(1, -1, 1), rtol=1e-12)
    m = P.mesh
    ue = configs.closed_form_u(1, 0.5, m.coords[0, :m.n_dofs] ** 2)
    uh = u[0, :, 0].cpu().numpy()
    err = np.sqrt(((uh - ue) ** 2).mean()) / np.sqrt((ue ** 2).mean())
    assert err < 0.012, err


def test_solve_many_rhs_and_fields():
    P = configs.square(12, 6, leaf_size=16, leaf_size_rho=32, cheb_p=4)
    m = P.mesh
    rng = np.random.default_rng(5)
    s2 = np.stack([P.s[0], np.clip(P.s[0] * 0.8 + 0.05, 0.05, 0.85)])
    k2 = np.stack([P.kappa[0], np.ones_like(P.kappa[0])])
    refs = []
    for f in range(2):
        split = assemble_split(m, s2[f], k2[f], P.opts)
        ref = assemble_h2(m, s2[f], k2[f], P.opts, split=split)
        refs.append(ref["B"] + ref["K"] + ref["M"])
    R = 3
    b = rng.standard_normal((2, m.n_dofs, R))
    import paper_2302_02863_amd as fp
    for precision in ("fp64", "mixed"):
        o = dict(P.opts)
        o["precision"] = precision
        op = fp.Operator(m, s2, k2, o)
        print(f"[solve] two fields x {R} rhs, {precision}", flush=True)
        u, info = op.solve(torch.tensor(b, device="cuda"), rtol=1e-12, maxit=5000)
        assert info["converged"], info
        uh = u.cpu().numpy()
        for f in range(2):
            ur = solve_dense(refs[f], b[f])
            for r in range(R):
                assert _rel(uh[f, :, r], ur[:, r]) < SOL_TOL, (precision, f, r)


def test_solve_initial_guess_and_noconv():
    P, A, F = _oracle("square")
    op = _op(P)
    Fd = torch.tensor(F, device="cuda").reshape(1, -1, 1)
    u0 = torch.tensor(solve_dense(A, F), device="cuda").reshape(1, -1, 1).contiguous()
    u, info = op.solve(Fd, u=u0.clone(), rtol=1e-8)
    assert info["converged"] and info["iterations"] == 0 and info["refinements"] == 0, info
    # too few iterations: FPDE_ENOCONV, the iterate and the residual are still reported
    u, info = op.solve(Fd, rtol=1e-14, maxit=3, raise_on_noconv=False)
    assert not info["converged"] and 0 < info["iterations"] <= 3 and 0 < info["rel_residual"] < 1, info
    import paper_2302_02863_amd as fp
    with pytest.raises(fp.FpdeError, match="FPDE_ENOCONV"):
        op.solve(Fd, rtol=1e-14, maxit=3)


def test_solve_reproducible():
    P, A, F = _oracle("square")
    op = _op(P, precision="mixed")
    Fd = torch.tensor(F, device="cuda").reshape(1, -1, 1)
    u1, i1 = op.solve(Fd, rtol=1e-11)
    u2, i2 = op.solve(Fd, rtol=1e-11)
    assert i1 == i2
    assert torch.equal(u1, u2)
