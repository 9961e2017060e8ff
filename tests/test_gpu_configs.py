"""GPU parity on configurations the other parity files do not reach.

* Chebyshev rank K = p^2 above 32 (p = 6 and p = 8, the largest the library
  accepts): one right-hand side takes the one-vector path's 64-lane pair slots
  and its non-register upsweep branch, a few right-hand sides the LDS-resident
  subtree sweeps, many the per-level sweeps.  FP64 within 1e-10 of the
  H2-consistent oracle (eq. eq:interpolant with p points per dimension),
  mixed precision within 1e-6.
* The 1D workload at its full size (512 interior elements, 511 dofs): the
  variable-order apply against the dense oracle, FP64 and mixed CG with
  refinement against the oracle's Cholesky solution, and the constant-order
  s = 1/2 run against the closed form sqrt(1 - x^2) (Sec. 7.1), with the
  same L2 error as the oracle's own solution.
* The ends of the admissible orders: s = 0, s just below s_bar, and a jump
  from 0 to 0.85, applied and solved against the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from fpde_inputs import configs  # noqa: E402
from oracle.assembly import assemble_split, load_vector  # noqa: E402
from oracle.h2 import assemble_h2, assemble_K_h2  # noqa: E402
from oracle.solve import l2_error, solve_dense  # noqa: E402

TOL = 1e-10
MIXED_TOL = 1e-6
SOL_TOL = 1e-8

_cache = {}


def _oracle(key, make):
    if key not in _cache:
        P = make()
        print(f"[configs] oracle for {key}: N={P.mesh.n_dofs}", flush=True)
        split = assemble_split(P.mesh, P.s[0], P.kappa[0], P.opts)
        ref = assemble_h2(P.mesh, P.s[0], P.kappa[0], P.opts, split=split)
        _cache[key] = (P, ref)
    return _cache[key]


def _op(P, **kw):
    import paper_2302_02863_amd as fp
    o = dict(P.opts)
    o.update(kw)
    return fp.Operator(P.mesh, P.s, P.kappa, o)


def _apply(op, x, parts=None):
    import paper_2302_02863_amd as fp
    y = op.apply(torch.tensor(x, device="cuda"), parts=fp.PART_ALL if parts is None else parts)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("p", [6, 8])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_chebyshev_rank_above_32(p, precision):
    import paper_2302_02863_amd as fp
    P, ref = _oracle(f"square16_p{p}",
                     lambda: configs.square(16, 8, leaf_size=16, leaf_size_rho=32, cheb_p=p))
    A = ref["B"] + ref["K"] + ref["M"]
    op = _op(P, precision=precision)
    st = op.stats()
    assert st["k_rank"] == p * p > 32 and st["k_far"] > 0
    tol = TOL if precision == "fp64" else MIXED_TOL
    rng = np.random.default_rng(30 + p)
    for R in (1, 4, 40):
        x = rng.standard_normal((1, op.n_dofs, R))
        y = _apply(op, x)[0]
        yr = A @ x[0]
        err = (np.linalg.norm(y - yr, axis=0) / np.linalg.norm(yr, axis=0)).max()
        print(f"[configs] p={p} {precision} R={R}: max rel err {err:.2e}", flush=True)
        assert err < tol, (R, err)
    if precision == "fp64":
        # the far blocks alone, one vector (the path with 64-lane pair slots)
        K, parts = assemble_K_h2(P.mesh, P.s[0], P.kappa[0], P.opts, K_exact=ref["split"]["K"], return_parts=True)
        tree = parts["tree"]
        Kfar = K.copy()
        for a, b in parts["near"]:
            Kfar[np.ix_(tree.members[a], tree.members[b])] = 0.0
        x = rng.standard_normal((1, op.n_dofs, 1))
        y = _apply(op, x, fp.PART_KFAR)[0, :, 0]
        yr = Kfar @ x[0, :, 0]
        assert np.linalg.norm(y - yr) / np.linalg.norm(yr) < TOL
    op.close()


def test_interval512_apply_and_solve():
    """The 1D workload at full size: s = 0.5 + 0.3 sin(pi x), 512 interior elements."""
    P, ref = _oracle("interval512", lambda: configs.interval(n_int=512))
    assert P.mesh.n_dofs == 511
    A = ref["B"] + ref["K"] + ref["M"]
    op = _op(P)
    y = _apply(op, P.x)[0, :, 0]
    yr = A @ P.x[0, :, 0]
    err = np.linalg.norm(y - yr) / np.linalg.norm(yr)
    print(f"[configs] interval512 apply rel err {err:.2e}", flush=True)
    assert err < TOL
    F = load_vector(P.mesh, P.f, P.opts)
    u_ref = solve_dense(A, F)
    for precision in ("fp64", "mixed"):
        opp = op if precision == "fp64" else _op(P, precision="mixed")
        u, info = opp.solve(torch.tensor(F, device="cuda").reshape(1, -1, 1), rtol=1e-12, maxit=20000)
        torch.cuda.synchronize()
        e = np.linalg.norm(u.cpu().numpy()[0, :, 0] - u_ref) / np.linalg.norm(u_ref)
        print(f"[configs] interval512 {precision} solve: {info}, rel err {e:.2e}", flush=True)
        assert e < SOL_TOL, (precision, e)
        if opp is not op:
            opp.close()
    op.close()


def test_interval512_closed_form():
    """Constant order s = 1/2 with the fractional-Laplacian normalisation and the
    exterior beyond R handled analytically: the library's solution has the oracle's
    L2 error against sqrt(1 - x^2) (the two solutions agree to 1e-8)."""
    P, ref = _oracle("interval_const512", lambda: configs.interval_const(n_int=512))
    A = ref["B"] + ref["K"] + ref["M"]
    F = load_vector(P.mesh, P.f, P.opts)
    u_ref = solve_dense(A, F)
    op = _op(P)
    u, info = op.solve(torch.tensor(F, device="cuda").reshape(1, -1, 1), rtol=1e-12, maxit=20000)
    torch.cuda.synchronize()
    u = u.cpu().numpy()[0, :, 0]
    exact = lambda x: configs.closed_form_u(1, 0.5, x[0] ** 2)  # noqa: E731
    e_gpu = l2_error(P.mesh, u, exact)
    e_ref = l2_error(P.mesh, u_ref, exact)
    print(f"[configs] interval_const512: L2 error {e_gpu:.4e} (oracle {e_ref:.4e})", flush=True)
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) < SOL_TOL
    assert abs(e_gpu - e_ref) < 1e-6 * e_ref + 1e-12
    assert e_gpu < 2.5e-3
    op.close()


def _with_order(P, s):
    from dataclasses import replace
    return replace(P, s=np.asarray(s, dtype=np.float64)[None, :])


@pytest.mark.parametrize("order", ["zero", "near_s_bar", "jump"])
def test_extreme_orders(order):
    """The ends of the admissible orders: s = 0 everywhere (kernel |x - y|^-d), s just
    below s_bar = 0.9, and a jump from 0 to 0.85 across x1 = 0.5: FP64 apply within
    1e-10 of the oracle, mixed within 1e-6, Jacobi PCG within 1e-8 of its Cholesky
    solution."""
    base = configs.square(12, 6, leaf_size=16, leaf_size_rho=32, cheb_p=4)
    x1 = base.mesh.coords[0]
    s = {"zero": np.zeros_like(x1), "near_s_bar": np.full_like(x1, 0.899),
         "jump": np.where(x1 < 0.5, 0.0, 0.85)}[order]
    P, ref = _oracle(f"order_{order}", lambda: _with_order(base, s))
    A = ref["B"] + ref["K"] + ref["M"]
    x = np.random.default_rng(51).standard_normal((1, P.mesh.n_dofs, 3))
    for precision, tol in (("fp64", TOL), ("mixed", MIXED_TOL)):
        op = _op(P, precision=precision, jacobi=True)
        y = _apply(op, x)[0]
        yr = A @ x[0]
        err = (np.linalg.norm(y - yr, axis=0) / np.linalg.norm(yr, axis=0)).max()
        F = op.load_vector(torch.tensor(P.f, device="cuda")).reshape(1, -1, 1)
        u, info = op.solve(F, rtol=1e-12, maxit=20000)
        u = u.cpu().numpy()[0, :, 0]
        op.close()
        uref = solve_dense(A, load_vector(P.mesh, P.f, P.opts))
        eu = np.linalg.norm(u - uref) / np.linalg.norm(uref)
        print(f"[configs] s {order} {precision}: apply {err:.2e}, solve {eu:.2e} ({info['iterations']} it)", flush=True)
        assert err < tol and eu < SOL_TOL, (precision, err, eu)
