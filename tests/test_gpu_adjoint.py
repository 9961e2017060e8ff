"""GPU adjoint (fpde_apply_adjoint) against the oracle's complex-step derivatives.

The library returns the full gradient of J = w^T A_h(s, kappa) u over all mesh
nodes; the oracle differentiates its dense H2-consistent assembly by complex
step (exact to rounding, pinned in tests/test_oracle_adjoint.py).  Directional
derivatives along random directions are compared on cases that span several
leaves, far blocks, an analytic exterior and the 1D rules; on a tiny mesh the
whole gradient is compared node by node.  Tolerance 1e-10, relative to the
absolute sum sum_j |g_j d_j| of the terms of the directional derivative.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from fpde_inputs import configs  # noqa: E402
from oracle.adjoint import directional  # noqa: E402

TOL = 1e-10

CASES = {
    "square": lambda: configs.square(12, 6, leaf_size=16, leaf_size_rho=32, cheb_p=4),
    "interval": lambda: configs.interval(n_int=64, n_ext=16, leaf_size=8, leaf_size_rho=16, cheb_p=5),
    "disk": lambda: configs.disk(8, leaf_size=16, leaf_size_rho=32, cheb_p=4),
}


def _grad(P, w, u):
    import paper_2302_02863_amd as fp
    op = fp.Operator(P.mesh, P.s, P.kappa, P.opts)
    gs, gk = op.apply_adjoint(torch.tensor(w, device="cuda"), torch.tensor(u, device="cuda"))
    torch.cuda.synchronize()
    return gs.cpu().numpy()[0], gk.cpu().numpy()[0], op


@pytest.mark.parametrize("name", list(CASES))
def test_directional_derivatives(name):
    P = CASES[name]()
    m = P.mesh
    rng = np.random.default_rng(12)
    w = rng.standard_normal((1, m.n_dofs, 1))
    u = rng.standard_normal((1, m.n_dofs, 1))
    print(f"[adjoint] {name}: N={m.n_dofs} M={m.n_nodes}", flush=True)
    gs, gk, op = _grad(P, w, u)
    for trial in range(3):
        ds = rng.uniform(-1, 1, m.n_nodes)
        dk = rng.uniform(-1, 1, m.n_nodes)
        for dsv, dkv in ((ds, None), (None, dk)):
            ref = directional(m, P.s[0], P.kappa[0], P.opts, w[0, :, 0], u[0, :, 0], ds=dsv, dk=dkv)
            g, d = (gs, dsv) if dsv is not None else (gk, dkv)
            got = float(g @ d)
            scale = float(np.abs(g * d).sum())
            print(f"[adjoint] {name} trial {trial} {'s' if dsv is not None else 'kappa'}: "
                  f"{got:.15e} vs {ref:.15e}", flush=True)
            assert abs(got - ref) <= TOL * scale, (got, ref, scale)
    op.close()


def test_gradient_node_by_node_and_several_rhs():
    """Single entries of the gradient (interior, boundary and exterior nodes) with two
    right-hand sides, each against the oracle's derivative along that node alone."""
    P = configs.square(4, 2, leaf_size=6, leaf_size_rho=12, cheb_p=3)
    m = P.mesh
    rng = np.random.default_rng(13)
    R = 2
    w = rng.standard_normal((1, m.n_dofs, R))
    u = rng.standard_normal((1, m.n_dofs, R))
    gs, gk, op = _grad(P, w, u)
    nodes = np.concatenate([rng.choice(m.n_dofs, 5, replace=False),
                            rng.choice(np.arange(m.n_dofs, m.n_nodes), 5, replace=False)])
    scale_s, scale_k = np.abs(gs).max(), np.abs(gk).max()
    for j in nodes:
        e = np.zeros(m.n_nodes)
        e[j] = 1.0
        rs = directional(m, P.s[0], P.kappa[0], P.opts, w[0], u[0], ds=e)
        rk = directional(m, P.s[0], P.kappa[0], P.opts, w[0], u[0], dk=e)
        print(f"[adjoint] node {j}: ds {gs[j]:.15e} vs {rs:.15e}; dkappa {gk[j]:.15e} vs {rk:.15e}", flush=True)
        assert abs(gs[j] - rs) <= TOL * scale_s, (j, gs[j], rs)
        assert abs(gk[j] - rk) <= TOL * scale_k, (j, gk[j], rk)
    # bitwise reproducible
    gs2, gk2 = op.apply_adjoint(torch.tensor(w, device="cuda"), torch.tensor(u, device="cuda"))
    torch.cuda.synchronize()
    assert np.array_equal(gs2.cpu().numpy()[0], gs) and np.array_equal(gk2.cpu().numpy()[0], gk)
    op.close()


def test_autograd_solve_gradient():
    """J(s, kappa) = 1/2 ||u - u_obs||^2 with u = A_h^{-1} F through FracSolve: the
    autograd gradient (adjoint CG + fpde_apply_adjoint) against the oracle's complex
    step through a dense solve, along random directions."""
    from paper_2302_02863_amd.autograd import frac_solve
    from oracle.adjoint import objective_directional
    from oracle.assembly import load_vector
    P = configs.square(8, 4, leaf_size=12, leaf_size_rho=24, cheb_p=3)
    m = P.mesh
    F = load_vector(m, P.f, P.opts)
    rng = np.random.default_rng(17)
    u_obs = 0.3 * rng.standard_normal(m.n_dofs)
    s = torch.tensor(P.s, requires_grad=True)
    k = torch.tensor(P.kappa, requires_grad=True)
    Fd = torch.tensor(F, device="cuda").reshape(1, -1, 1)
    u = frac_solve(s, k, Fd, m, P.opts, 1e-13)
    J = 0.5 * ((u[0, :, 0] - torch.tensor(u_obs, device="cuda")) ** 2).sum()
    J.backward()
    gs = s.grad.numpy()[0]
    gk = k.grad.numpy()[0]
    for trial in range(2):
        d = rng.uniform(-1, 1, m.n_nodes)
        for which, g in (("s", gs), ("kappa", gk)):
            kw = {"ds": d} if which == "s" else {"dk": d}
            ref = objective_directional(m, P.s[0], P.kappa[0], P.opts, F, u_obs, **kw)
            got = float(g @ d)
            print(f"[autograd] {which} trial {trial}: {got:.15e} vs {ref:.15e}", flush=True)
            assert abs(got - ref) <= 1e-8 * float(np.abs(g * d).sum()), (which, got, ref)


def test_full_gradient_two_fields_against_golden():
    """Every entry of the gradient over all 113 nodes of a disk with an analytic exterior,
    K~ far blocks and density far blocks, for two (s, kappa) fields and two right-hand sides,
    against the oracle's complex-step gradient stored by tests/golden/make_adjoint_disk8.py.
    alpha = -1 returns the exact negation."""
    import os
    import paper_2302_02863_amd as fp
    P = configs.adjoint_disk(8)
    m = P.mesh
    ref = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "adjoint_disk8_F2.txt"))
    rs = np.zeros((2, m.n_nodes))
    rk = np.zeros((2, m.n_nodes))
    rs[ref[:, 0].astype(int), ref[:, 1].astype(int)] = ref[:, 2]
    rk[ref[:, 0].astype(int), ref[:, 1].astype(int)] = ref[:, 3]
    assert ref.shape[0] == 2 * m.n_nodes
    op = fp.Operator(m, P.s, P.kappa, P.opts)
    st = op.stats()
    print(f"[adjoint] disk8 F=2: N={m.n_dofs} M={m.n_nodes} k_far={st['k_far']} rho_far={st['rho_far']}",
          flush=True)
    assert st["k_far"] > 0 and st["rho_far"] > 0
    w = torch.tensor(P.extra["w"], device="cuda")
    u = torch.tensor(P.x, device="cuda")
    gs, gk = op.apply_adjoint(w, u)
    ns, nk = op.apply_adjoint(w, u, alpha=-1.0)
    torch.cuda.synchronize()
    gs, gk, ns, nk = (t.cpu().numpy() for t in (gs, gk, ns, nk))
    assert np.array_equal(ns, -gs) and np.array_equal(nk, -gk)
    for f in range(2):
        es = np.abs(gs[f] - rs[f]).max() / np.abs(rs[f]).max()
        ek = np.abs(gk[f] - rk[f]).max() / np.abs(rk[f]).max()
        print(f"[adjoint] field {f}: max node error / max |g|: s {es:.2e}, kappa {ek:.2e}", flush=True)
        assert es <= TOL and ek <= TOL, (f, es, ek)
    op.close()


def test_fracsolve_shapes_and_repeated_backward():
    """FracSolve returns u in F's shape (here [F, N]) and keeps its operator alive for a
    second backward through a retained graph, which gives the same gradient bit for bit."""
    from paper_2302_02863_amd.autograd import frac_solve
    from oracle.assembly import load_vector
    P = configs.square(6, 3, leaf_size=8, leaf_size_rho=16, cheb_p=3)
    m = P.mesh
    F = torch.tensor(load_vector(m, P.f, P.opts), device="cuda").reshape(1, -1)
    s = torch.tensor(P.s, requires_grad=True)
    k = torch.tensor(P.kappa, requires_grad=True)
    Fr = F.clone().requires_grad_(True)
    u = frac_solve(s, k, Fr, m, P.opts, 1e-13)
    assert u.shape == Fr.shape
    J = (u ** 2).sum()
    J.backward(retain_graph=True)
    g1 = (s.grad.clone(), k.grad.clone(), Fr.grad.clone())
    assert g1[2].shape == Fr.shape
    s.grad = k.grad = Fr.grad = None
    J.backward()
    torch.cuda.synchronize()
    for a, b in zip(g1, (s.grad, k.grad, Fr.grad)):
        assert torch.equal(a, b)
