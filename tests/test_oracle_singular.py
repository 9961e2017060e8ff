"""Pins for the oracle's singular near-field rules (Sec. 4, and the 1D analogue).

* The region maps of the vertex, edge and identical cases tile the reference
  pair exactly once (polynomial moments) and their Jacobians are the factors
  the rules use (complex-step derivatives of the maps).
* The rescaled shape-function differences and distances agree with the maps.
* The rules converge to an independent brute force (polar/ray integration
  with closed-form radial integrals, constant order).
* 1D rules against closed forms and mpmath.
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import singular as S
from oracle.rules import gauss01


def _grid4(n):
    g, w = gauss01(n)
    Z, E1, E2, E3 = np.meshgrid(g, g, g, g, indexing="ij")
    W = np.einsum("a,b,c,d->abcd", w, w, w, w)
    return Z.ravel(), E1.ravel(), E2.ravel(), E3.ravel(), W.ravel()


def _regions(kind, xi, e1, e2, e3):
    if kind == "V":
        return [(r[0], r[1]) for r in S._vertex_regions(xi, e1, e2, e3)]
    if kind == "E":
        return [(r[0], r[1]) for r in S._edge_regions(xi, e1, e2, e3)]
    return [(r[0], r[1]) for r in S._identical_regions(xi, e1, e2, e3)]


def _factors(kind, xi, e1, e2, e3):
    """Jacobian the oracle's rule uses for each region (before the zeta/t substitutions)."""
    if kind == "V":
        return [xi ** 3 * r[4] for r in S._vertex_regions(xi, e1, e2, e3)]
    if kind == "E":
        return [xi ** 3 * r[4] for r in S._edge_regions(xi, e1, e2, e3)]
    return [xi ** 3 * e1 ** 2 * e2 for _ in range(3)]


@pytest.mark.parametrize("kind", ["V", "E", "I"])
def test_region_jacobians_complex_step(kind):
    rng = np.random.default_rng(7)
    v = rng.uniform(0.05, 0.95, size=(4, 25))
    h = 1e-30
    base = _regions(kind, *v)
    facs = _factors(kind, *v)
    for k in range(len(base)):
        Jm = np.zeros((25, 4, 4))
        for var in range(4):
            vv = v.astype(complex)
            vv[var] += 1j * h
            xh, yh = _regions(kind, *vv)[k]
            out = np.concatenate([xh, yh])          # (4, 25)
            Jm[:, :, var] = (out.imag / h).T
        det = np.abs(np.linalg.det(Jm))
        assert np.allclose(det, facs[k], rtol=1e-12, atol=0), (kind, k)


def _tri_moment(a, b):
    return 1.0 / ((b + 1) * (a + b + 2))


@pytest.mark.parametrize("kind", ["V", "E", "I"])
def test_regions_tile_reference_pair(kind):
    Z, E1, E2, E3, W = _grid4(8)
    regs = _regions(kind, Z, E1, E2, E3)
    facs = _factors(kind, Z, E1, E2, E3)
    for (a, b, c, d) in [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1),
                         (2, 1, 0, 1), (1, 1, 1, 1), (0, 2, 2, 0), (3, 0, 0, 2)]:
        tot = 0.0
        for (xh, yh), f in zip(regs, facs):
            g = xh[0] ** a * xh[1] ** b * yh[0] ** c * yh[1] ** d
            if kind == "I":   # regions 4..6 are the mirror images (x^ <-> y^)
                g = g + yh[0] ** a * yh[1] ** b * xh[0] ** c * xh[1] ** d
            tot += (W * f * g).sum()
        exact = _tri_moment(a, b) * _tri_moment(c, d)
        assert abs(tot - exact) < 1e-13 * max(1.0, exact), (kind, (a, b, c, d), tot, exact)


def _lam(xh):
    return np.stack([1.0 - xh[0], xh[0] - xh[1], xh[1]])


def test_rescaled_differences_match_maps():
    rng = np.random.default_rng(3)
    xi, e1, e2, e3 = rng.uniform(0.05, 0.95, size=(4, 40))
    # two triangles sharing v0 (vertex case) / v0,v1 (edge case)
    P = np.array([0.1, 0.2])
    XV0 = np.stack([P, [0.4, 0.25], [0.35, 0.5]], axis=1)
    XV1 = np.stack([P, [-0.2, 0.1], [-0.1, -0.2]], axis=1)
    for xh, yh, phi, (a, b), _ in S._vertex_regions(xi, e1, e2, e3):
        lx, ly = _lam(xh), _lam(yh)
        diff = np.stack([lx[0] - ly[0], lx[1], lx[2], -ly[1], -ly[2]])
        assert np.allclose(diff, xi * phi, atol=1e-15)
        J0, J1 = S._jac(XV0), S._jac(XV1)
        x = XV0[:, :1] + J0 @ xh
        y = XV1[:, :1] + J1 @ yh
        assert np.allclose(x - y, xi * (J0 @ a - J1 @ b), atol=1e-15)
    XE0 = np.stack([[0.0, 0.0], [0.3, 0.05], [0.1, 0.3]], axis=1)
    XE1 = np.stack([[0.0, 0.0], [0.3, 0.05], [0.25, -0.2]], axis=1)
    J0, J1 = S._jac(XE0), S._jac(XE1)
    for xh, yh, psi, (a, b), _ in S._edge_regions(xi, e1, e2, e3):
        lx, ly = _lam(xh), _lam(yh)
        diff = np.stack([lx[0] - ly[0], lx[1] - ly[1], lx[2], -ly[2]])
        assert np.allclose(diff, xi * psi, atol=1e-15)
        x = XE0[:, :1] + J0 @ xh
        y = XE1[:, :1] + J1 @ yh
        assert np.allclose(x - y, xi * (J0 @ a - J1 @ b), atol=1e-15)
    for xh, yh, psi, dh in S._identical_regions(xi, e1, e2, e3):
        scale = xi * e1 * e2
        assert np.allclose(_lam(xh) - _lam(yh), scale * psi, atol=1e-15)
        assert np.allclose(xh - yh, scale * dh, atol=1e-15)


# ----------------------------------------------------------------------------
# independent brute force: polar integration around x, closed-form radial part
# ----------------------------------------------------------------------------

def _affine_shape(X):
    """Coefficients (grad, const) of the 3 P1 shape functions of triangle X (2,3)."""
    M = np.vstack([X, np.ones(3)])            # [x; y; 1] columns per vertex
    C = np.linalg.inv(M)                      # rows: lambda_a = C[a] @ [x, y, 1]
    return C[:, :2], C[:, 2]


def _ray_interval(X, x, e):
    """[r0, r1] of the ray x + r e (e: (2,T)) inside triangle X; empty -> r0 >= r1."""
    G, c = _affine_shape(X)
    lo = np.zeros(e.shape[1])
    hi = np.full(e.shape[1], np.inf)
    for a in range(3):
        val = G[a] @ x + c[a]                 # lambda_a(x)
        slope = G[a] @ e                      # d lambda_a / dr
        with np.errstate(divide="ignore", invalid="ignore"):
            r = -val / slope
        pos = slope > 0
        neg = slope < 0
        lo = np.where(pos, np.maximum(lo, r), lo)
        hi = np.where(neg, np.minimum(hi, r), hi)
        zero = slope == 0
        hi = np.where(zero & (val < 0), -1.0, hi)
    return lo, hi


def brute_pair(kind, X0, X1, s, n_out=28, n_th=20):
    """Local matrix of a touching pair, constant order s, a = 1 (same dof order as the oracle)."""
    k0 = 3
    if kind == "I":
        verts = [0, 1, 2]
        dof_in0 = [0, 1, 2]; dof_in1 = [0, 1, 2]
    elif kind == "E":
        dof_in0 = [0, 1, 2, -1]; dof_in1 = [0, 1, -1, 2]
    else:
        dof_in0 = [0, 1, 2, -1, -1]; dof_in1 = [0, -1, -1, 1, 2]
    nd = len(dof_in0)
    G0, c0 = _affine_shape(X0)
    G1, c1 = _affine_shape(X1)
    gu, gw = gauss01(n_out)
    q1, q2 = (3.0, 1.0) if kind == "V" else ((1.0, 3.0) if kind == "E" else (1.0, 1.0))
    U, V = np.meshgrid(gu, gu, indexing="ij")
    Wt = np.outer(gw, gw)
    xi = U ** q1
    eta = V ** q2
    wt = Wt * q1 * U ** (q1 - 1) * q2 * V ** (q2 - 1) * xi
    xh = np.stack([xi.ravel(), (xi * eta).ravel()])
    wt = wt.ravel()
    J0 = S._jac(X0)
    det0 = abs(np.linalg.det(J0))
    xs = X0[:, :1] + J0 @ xh
    tg, tw = gauss01(n_th)
    A = np.zeros((nd, nd))
    for p in range(xs.shape[1]):
        x = xs[:, p]
        ang = np.sort(np.mod(np.arctan2(X1[1] - x[1], X1[0] - x[0]), 2 * np.pi))
        brk = np.concatenate([ang, [ang[0] + 2 * np.pi]])
        th = (brk[:-1, None] + (brk[1:] - brk[:-1])[:, None] * tg[None, :]).ravel()
        thw = ((brk[1:] - brk[:-1])[:, None] * tw[None, :]).ravel()
        e = np.stack([np.cos(th), np.sin(th)])
        r0, r1 = _ray_interval(X1, x, e)
        ok = r1 > r0
        r0 = np.where(ok, r0, 1.0)
        r1 = np.where(ok, r1, 1.0)

        def F(pw):
            return (r1 ** (pw + 1) - r0 ** (pw + 1)) / (pw + 1)
        cvec = np.zeros((nd, th.size))
        gvec = np.zeros((nd, th.size))
        for a in range(nd):
            psx = (G0[dof_in0[a]] @ x + c0[dof_in0[a]]) if dof_in0[a] >= 0 else 0.0
            if dof_in1[a] >= 0:
                ext = G1[dof_in1[a]] @ x + c1[dof_in1[a]]
                gvec[a] = G1[dof_in1[a]] @ e
            else:
                ext = 0.0
            cvec[a] = psx - ext
        f1, f2, f3 = F(-1 - 2 * s), F(-2 * s), F(1 - 2 * s)
        if kind == "I":
            f1 = np.zeros_like(f1); f2 = np.zeros_like(f2)
            f3 = r1 ** (2 - 2 * s) / (2 - 2 * s)
        for a in range(nd):
            for b in range(nd):
                val = cvec[a] * cvec[b] * f1 - (cvec[a] * gvec[b] + cvec[b] * gvec[a]) * f2 + gvec[a] * gvec[b] * f3
                A[a, b] += wt[p] * det0 * (thw * np.where(ok, val, 0.0)).sum()
    return A


_GEOM = {
    "I": (np.array([[0.0, 0.31, 0.27], [0.0, 0.04, 0.29]]), None),
    "E": (np.array([[0.0, 0.3, 0.12], [0.0, 0.05, 0.31]]), np.array([[0.0, 0.3, 0.22], [0.0, 0.05, -0.24]])),
    "V": (np.array([[0.0, 0.3, 0.21], [0.0, 0.02, 0.27]]), np.array([[0.0, -0.25, -0.05], [0.0, 0.08, -0.3]])),
}


@pytest.mark.parametrize("kind", ["I", "E", "V"])
@pytest.mark.parametrize("s", [0.3, 0.7])
def test_rule_converges_to_brute_force(kind, s):
    X0, X1 = _GEOM[kind]
    if X1 is None:
        X1 = X0
    ref = brute_pair(kind, X0, X1, s)
    one = np.ones(3)
    nrm = np.abs(ref).max()

    def err(sb, n):
        A = S.local_matrix_2d(kind, X0, X1, s * one, s * one, one, one, 1.0, sb, n)
        return np.abs(A - ref).max() / nrm, A
    # with s_bar = s the zeta and t factors are constant: fast convergence
    e20, A20 = err(s, 20)
    assert e20 < 1e-4, e20
    # with s_bar = 0.9 the rule converges algebraically in n (non-analytic powers)
    errs = [err(0.9, n)[0] for n in (3, 6, 12, 20)]
    assert all(errs[k + 1] < errs[k] for k in range(3)), errs
    assert errs[-1] < 2e-4 and errs[0] < 5e-2, errs
    # row sums of every local matrix vanish (partition of unity of the pair's shape functions)
    assert np.abs(A20.sum(axis=1)).max() < 1e-12 * nrm


def test_brute_force_is_converged():
    X0, X1 = _GEOM["E"]
    a = brute_pair("E", X0, X1, 0.6, n_out=20, n_th=16)
    b = brute_pair("E", X0, X1, 0.6, n_out=32, n_th=24)
    assert np.abs(a - b).max() / np.abs(b).max() < 5e-5


# ----------------------------------------------------------------------------
# 1D
# ----------------------------------------------------------------------------

def test_1d_identical_closed_form():
    # int_0^h int_0^h |x-y|^{1-2s} = 2 h^{3-2s} / ((2-2s)(3-2s)); entries sig_a sig_b h^{-2} times that
    h = 0.37
    for s, sb, n, tol in [(0.5, 0.5, 3, 1e-14), (0.75, 0.75, 2, 1e-13), (0.6, 0.9, 24, 1e-6)]:
        one = np.ones(2)
        A = S.local_matrix_1d("I", np.array([0.2, 0.2 + h]), None, s * one, None, one, None, 1.0, sb, n)
        exact = 2 * h ** (1 - 2 * s) / ((2 - 2 * s) * (3 - 2 * s))
        assert abs(A[1, 1] - exact) < tol * exact, (s, sb, A[1, 1], exact)
        assert abs(A[0, 1] + exact) < tol * exact


def test_1d_vertex_mpmath():
    h1, h2, s = 0.3, 0.45, 0.65
    one = np.ones(2)
    A = S.local_matrix_1d("V", np.array([0.0, -h1]), np.array([0.0, h2]), s * one, s * one, one, one, 1.0, s, 16)
    A9 = S.local_matrix_1d("V", np.array([0.0, -h1]), np.array([0.0, h2]), s * one, s * one, one, one, 1.0, 0.9, 16)
    mpmath.mp.dps = 20

    def ent(a, b):
        def f(al, be):
            phi = [be - al, al, -be]
            return phi[a] * phi[b] * (h1 * al + h2 * be) ** (-1 - 2 * s)
        return float(h1 * h2 * mpmath.quad(f, [0, 1], [0, 1]))
    for a, b in [(0, 0), (1, 1), (2, 2), (1, 2), (0, 1)]:
        ref = ent(a, b)
        assert abs(A[a, b] - ref) < 1e-12 * abs(ref), (a, b, A[a, b], ref)
        assert abs(A9[a, b] - ref) < 2e-4 * abs(ref), (a, b, A9[a, b], ref)
