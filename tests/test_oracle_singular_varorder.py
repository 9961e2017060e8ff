"""Pins for the variable-order arithmetic of the oracle's singular rules (Sec. 4).

The rules of eqs. e:int-v-2, e:int-e and e:int-i-2 evaluate the order s and the
diffusivity kappa at both integration points of every quadrature node: s(x)
from tau's nodal values at x, s(y) from tau''s nodal values at y.  Constant
fields cannot tell the two apart, so these pins use affine fields
s(x) = s_c + g_s . x and kappa(x) = k_c + g_k . x, which P1 reproduces exactly.

* 2D: each touching-pair kind against an independent brute force in polar
  coordinates around x: the outer integral over tau by a graded collapsed
  Gauss rule, the angle split at the directions of tau''s vertices, and the
  radial integral along each ray by composite Gauss panels in u = ln r (the
  integrand r^{-s(x)-s(y(r))} is smooth in u), with the part below
  r1 e^{-36} integrated in closed form at frozen order.  The fields are
  evaluated from their global affine form, not from nodal values.
* 1D: the identical and vertex rules against mpmath tanh-sinh quadrature of
  the raw double integral.
* Sensitivity: a planted slip in the oracle's inputs (s(y) or kappa(y) taken
  from tau's nodal values) misses these references by several percent, far
  outside the tolerance, and so does freezing the order at the centroid.
"""
import mpmath
import numpy as np
import pytest

from oracle import singular as S
from oracle.rules import gauss01

S_FIELD = (0.45, np.array([0.6, -0.4]))     # s(x) = 0.45 + 0.6 x1 - 0.4 x2: [0.27, 0.68] on the pairs
K_FIELD = (1.2, np.array([-0.9, 0.7]))      # kappa(x) = 1.2 - 0.9 x1 + 0.7 x2 > 0 on the pairs

_GEOM = {
    "I": (np.array([[0.0, 0.31, 0.27], [0.0, 0.04, 0.29]]), None),
    "E": (np.array([[0.0, 0.3, 0.12], [0.0, 0.05, 0.31]]), np.array([[0.0, 0.3, 0.22], [0.0, 0.05, -0.24]])),
    "V": (np.array([[0.0, 0.3, 0.21], [0.0, 0.02, 0.27]]), np.array([[0.0, -0.25, -0.05], [0.0, 0.08, -0.3]])),
}


def _affine_shape(X):
    """Gradients and constants of the three P1 shape functions of triangle X (2,3)."""
    C = np.linalg.inv(np.vstack([X, np.ones(3)]))
    return C[:, :2], C[:, 2]


def _ray_interval(X, x, e):
    """[r0, r1] of the rays x + r e (e: (2,T)) inside triangle X; empty when r0 >= r1."""
    G, c = _affine_shape(X)
    lo = np.zeros(e.shape[1])
    hi = np.full(e.shape[1], np.inf)
    for a in range(3):
        val = G[a] @ x + c[a]
        slope = G[a] @ e
        with np.errstate(divide="ignore", invalid="ignore"):
            r = -val / slope
        lo = np.where(slope > 0, np.maximum(lo, r), lo)
        hi = np.where(slope < 0, np.minimum(hi, r), hi)
        hi = np.where((slope == 0) & (val < 0), -1.0, hi)
    return lo, hi


def brute_pair_varorder(kind, X0, X1, sfield, kfield, n_out=28, n_th=20, depth=36.0, npan=8):
    """Local matrix of a touching pair with affine order and diffusivity, a = sqrt(k k).

    Same dof order as the oracle's rule: I {v0,v1,v2}; E {v0,v1,tau.v2,tau'.v2};
    V {P, tau.v1, tau.v2, tau'.v1, tau'.v2}.
    """
    if kind == "I":
        d0, d1 = [0, 1, 2], [0, 1, 2]
    elif kind == "E":
        d0, d1 = [0, 1, 2, -1], [0, 1, -1, 2]
    else:
        d0, d1 = [0, 1, 2, -1, -1], [0, -1, -1, 1, 2]
    nd = len(d0)
    G0, c0 = _affine_shape(X0)
    G1, c1 = _affine_shape(X1)
    # outer rule over tau: (xi, xi eta) collapsed, graded towards the shared vertex (V) or edge (E)
    gu, gw = gauss01(n_out)
    q1, q2 = (3.0, 1.0) if kind == "V" else ((1.0, 3.0) if kind == "E" else (1.0, 1.0))
    U, V = np.meshgrid(gu, gu, indexing="ij")
    xi, eta = U ** q1, V ** q2
    wt = (np.outer(gw, gw) * q1 * U ** (q1 - 1) * q2 * V ** (q2 - 1) * xi).ravel()
    J0 = np.stack([X0[:, 1] - X0[:, 0], X0[:, 2] - X0[:, 1]], axis=1)
    det0 = abs(np.linalg.det(J0))
    xs = X0[:, :1] + J0 @ np.stack([xi.ravel(), (xi * eta).ravel()])
    tg, tw = gauss01(n_th)
    pg, pw = gauss01(npan)
    sc, sgr = sfield
    kc, kgr = kfield
    A = np.zeros((nd, nd))
    for p in range(xs.shape[1]):
        x = xs[:, p]
        sx = sc + sgr @ x
        kx = kc + kgr @ x
        ang = np.sort(np.mod(np.arctan2(X1[1] - x[1], X1[0] - x[0]), 2 * np.pi))
        brk = np.concatenate([ang, [ang[0] + 2 * np.pi]])
        th = (brk[:-1, None] + (brk[1:] - brk[:-1])[:, None] * tg[None, :]).ravel()
        thw = ((brk[1:] - brk[:-1])[:, None] * tw[None, :]).ravel()
        e = np.stack([np.cos(th), np.sin(th)])
        r0, r1 = _ray_interval(X1, x, e)
        ok = r1 > r0
        r0 = np.where(ok, r0, 0.5)
        r1 = np.where(ok, r1, 1.0)
        # psi_a(x) - psi_a(x + r e) = cv_a - r gv_a (tau' shape functions extended affinely)
        cv = np.zeros((nd, th.size))
        gv = np.zeros((nd, th.size))
        for a in range(nd):
            inside = (G0[d0[a]] @ x + c0[d0[a]]) if d0[a] >= 0 else 0.0
            ext = 0.0
            if d1[a] >= 0:
                ext = G1[d1[a]] @ x + c1[d1[a]]
                gv[a] = G1[d1[a]] @ e
            cv[a] = inside - ext
        # radial integral in u = ln r: integrand (cv - r gv)(cv - r gv) a r^{-s(x)-s(y)} du
        u_eps = np.log(r1) - depth
        ulo = np.maximum(np.log(np.maximum(r0, 1e-300)), u_eps)
        uhi = np.log(r1)
        npn = np.maximum(1, np.ceil(uhi - ulo).astype(int))
        k = np.arange(npn.max())
        hw = (uhi - ulo) / npn
        uu = ulo[:, None, None] + hw[:, None, None] * (k[None, :, None] + pg[None, None, :])
        ww = hw[:, None, None] * pw[None, None, :] * (k[None, :, None] < npn[:, None, None])
        uu = np.minimum(uu, uhi[:, None, None]).reshape(th.size, -1)
        ww = ww.reshape(th.size, -1)
        r = np.exp(uu)
        y = x[:, None, None] + r[None] * e[:, :, None]
        sy = sc + np.einsum("i,irq->rq", sgr, y)
        ky = kc + np.einsum("i,irq->rq", kgr, y)
        base = ww * np.sqrt(kx * ky) * r ** (-sx - sy)
        cr = cv[:, :, None] - r[None] * gv[:, :, None]
        M = np.einsum("arq,brq,rq->abr", cr, cr, base)
        # r in [r0, eps], eps = r1 e^{-depth}: order frozen at s(y) = s(x), closed form
        eps = np.exp(u_eps)
        tail_on = r0 < eps
        lo = np.where(tail_on, r0, eps)
        sig = 2.0 * sx

        def F(pwr):
            with np.errstate(divide="ignore", invalid="ignore"):
                v = (eps ** (pwr + 1) - lo ** (pwr + 1)) / (pwr + 1)
            return np.where(lo > 0, v, 0.0) if pwr + 1 < 0 else v
        f1, f2, f3 = F(-1 - sig), F(-sig), F(1 - sig)
        tail = kx * (cv[:, None] * cv[None, :] * f1 - (cv[:, None] * gv[None, :] + gv[:, None] * cv[None, :]) * f2
                     + gv[:, None] * gv[None, :] * f3)
        M = M + np.where(tail_on, tail, 0.0)
        A += wt[p] * det0 * (thw * np.where(ok, M, 0.0)).sum(axis=-1)
    return A


def _nodal(field, X):
    return field[0] + field[1] @ X


@pytest.fixture(scope="module")
def brute_2d():
    out = {}
    for kind, (X0, X1) in _GEOM.items():
        X1 = X0 if X1 is None else X1
        out[kind] = brute_pair_varorder(kind, X0, X1, S_FIELD, K_FIELD)
    return out


def test_brute_force_varorder_is_converged():
    X0, X1 = _GEOM["E"]
    a = brute_pair_varorder("E", X0, X1, S_FIELD, K_FIELD, n_out=20, n_th=14, depth=30.0, npan=6)
    b = brute_pair_varorder("E", X0, X1, S_FIELD, K_FIELD, n_out=34, n_th=26, depth=40.0, npan=10)
    assert np.abs(a - b).max() / np.abs(b).max() < 5e-5


def test_brute_force_reduces_to_constant_order_closed_radial():
    # with g = 0 the radial integral has a closed form; the log-panel rule must reproduce it
    X0, X1 = _GEOM["V"]
    s = 0.55
    A = brute_pair_varorder("V", X0, X1, (s, np.zeros(2)), (1.0, np.zeros(2)), n_out=12, n_th=10)
    one = np.ones(3)
    R = S.local_matrix_2d("V", X0, X1, s * one, s * one, one, one, 1.0, s, 24)
    assert np.abs(A - R).max() / np.abs(R).max() < 3e-4


@pytest.mark.parametrize("kind", ["I", "E", "V"])
def test_varorder_rule_converges_to_brute_force(kind, brute_2d):
    X0, X1 = _GEOM[kind]
    X1 = X0 if X1 is None else X1
    ref = brute_2d[kind]
    nrm = np.abs(ref).max()
    s0, s1 = _nodal(S_FIELD, X0), _nodal(S_FIELD, X1)
    k0, k1 = _nodal(K_FIELD, X0), _nodal(K_FIELD, X1)

    def err(n, s1_=s1, k1_=k1, s0_=s0):
        A = S.local_matrix_2d(kind, X0, X1, s0_, s1_, k0, k1_, 1.0, 0.9, n)
        return np.abs(A - ref).max() / nrm
    errs = [err(n) for n in (6, 12, 20, 28)]
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 5e-5, errs
    # the pin sees the order's variation: frozen at the centroid value it misses by percents
    sc = np.full(3, S_FIELD[0] + S_FIELD[1] @ X0.mean(axis=1))
    assert err(20, s1_=sc, s0_=sc) > 1e-2
    if kind != "I":
        # planted slips: s(y) or kappa(y) from tau's nodal values instead of tau''s
        assert err(20, s1_=s0) > 5e-2
        assert err(20, k1_=k0) > 5e-2


# ----------------------------------------------------------------------------
# 1D: mpmath tanh-sinh on the raw double integrals
# ----------------------------------------------------------------------------

def _s1(x):
    return 0.55 + 0.35 * x


def _k1(x):
    return 1.1 - 0.6 * x


def test_1d_identical_varorder_mpmath():
    x0, h = 0.1, 0.4
    mpmath.mp.dps = 15

    def f(x, t):   # y = x - t < x; the integrand is symmetric in (x, y)
        y = x - t
        return 2 * t ** (1 - _s1(x) - _s1(y)) * mpmath.sqrt(_k1(x) * _k1(y)) / h ** 2
    ref = float(mpmath.quad(lambda x: mpmath.quad(lambda t: f(x, t), [0, x - x0]), [x0, x0 + h]))
    xs = np.array([x0, x0 + h])
    errs = []
    for n in (4, 8, 16, 32):
        A = S.local_matrix_1d("I", xs, None, _s1(xs), None, _k1(xs), None, 1.0, 0.9, n)
        assert abs(A[0, 1] + A[1, 1]) < 1e-14 * A[1, 1]
        errs.append(abs(A[1, 1] - ref) / ref)
    assert errs[-1] < 1e-9 and errs[1] < errs[0], errs
    # frozen order misses by percents
    sc = np.full(2, _s1(x0 + 0.5 * h))
    Af = S.local_matrix_1d("I", xs, None, sc, None, _k1(xs), None, 1.0, 0.9, 16)
    assert abs(Af[1, 1] - ref) / ref > 1e-2


def test_1d_vertex_varorder_mpmath():
    P, h1, h2 = 0.05, 0.3, 0.45
    mpmath.mp.dps = 15

    def ent(a, b):
        def f(al, be):
            x, y = P - h1 * al, P + h2 * be
            phi = [be - al, al, -be]
            return phi[a] * phi[b] * mpmath.sqrt(_k1(x) * _k1(y)) * (h1 * al + h2 * be) ** (-1 - _s1(x) - _s1(y))
        return float(h1 * h2 * mpmath.quad(f, [0, 1], [0, 1]))
    idx = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 1)]
    ref = {ab: ent(*ab) for ab in idx}
    nrm = max(abs(v) for v in ref.values())
    xa, xb = np.array([P, P - h1]), np.array([P, P + h2])

    def err(n, sb=_s1(xb), kb=_k1(xb)):
        A = S.local_matrix_1d("V", xa, xb, _s1(xa), sb, _k1(xa), kb, 1.0, 0.9, n)
        return max(abs(A[a, b] - ref[(a, b)]) for a, b in idx) / nrm
    errs = [err(n) for n in (4, 8, 16, 32)]
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 1e-5, errs
    # planted slips: s(y) or kappa(y) from tau's nodal values
    assert err(16, sb=_s1(xa)) > 5e-2
    assert err(16, kb=_k1(xa)) > 5e-2
