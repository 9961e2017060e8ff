"""Workload recipes: meshes, nodal order/diffusivity fields, options and vectors.

Each recipe returns a :class:`Problem`.  All randomness comes from
``numpy.random.default_rng(seed)`` with the seeds listed in the recipe, so the
oracle and the GPU path see bit-identical inputs.

Named workloads (sizes follow the configurations the library is measured on):

* ``interval``  1D, interior (-1,1), Omega=(-2,2), s=0.5+0.3 sin(pi x), kappa=1.
* ``interval_const``  1D, s=0.5, fractional-Laplacian normalisation, exterior
  beyond R=1+26h handled analytically (closed-form solution sqrt(1-x^2)).
* ``square``  2D, interior (0,1)^2 with n x n squares split in two, Omega =
  (-0.5,1.5)^2, interior nodes jittered by U(-0.1h,0.1h) (seed 0),
  s=0.3+0.2(x1+x2), kappa=1+0.5 cos(2 pi x1) cos(2 pi x2), x ~ N(0,1) (seed 1).
* ``disk``  unit disk (elliptical map of an n x n grid) with a meshed annulus
  to R=1.1 and the exterior beyond R handled analytically.
* ``batched``  2D square without jitter, kappa=1, F order fields
  s_k = 0.5+0.3 sin(k pi x1) cos(pi x2), R right-hand sides ~ N(0,1) (seed 3).
* ``bump``  the variable-order test of the paper's Sec. 7.2: Omega = (-2,2)^2,
  interior (-1,1)^2 on the uniform grid T_j (2^{j+1} squares a side inside,
  split along one diagonal), s = s* + eta bump(x1 - c1; l) bump(x2 - c2; l)
  with bump(x; l) = exp(-1/(1-r^2)), r = 2x/l, for |r| < 1 (else 0), s* = 0.7,
  eta = 0.2, l = 1, c = (-0.4, 0.4), a = 1, f = 20.
* ``adjoint_disk``  small disk with an analytic exterior and two fields (the
  disk's order with kappa = 1, and a perturbed order with kappa = 1 + 0.3 x1),
  two right-hand sides u ~ N(0,1) (seed 14) and weights w ~ N(0,1) (seed 15).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .meshes import Mesh, interval_mesh, square_mesh, square_mesh_graded, disk_mesh


DEFAULT_OPTS = dict(
    precision="fp64",   # "fp64" or "mixed"
    leaf_size=64,
    leaf_size_rho=64,
    cheb_p=5,
    eta=1.0,
    nq_sing=3,
    nq_reg=3,
    s_bar=0.9,
    s_exterior=0.0,
    n_theta=128,
    a_scale=1.0,
)


@dataclass
class Problem:
    name: str
    mesh: Mesh
    s: np.ndarray        # (F, M) nodal order field(s)
    kappa: np.ndarray    # (F, M) nodal diffusivity field(s), kappa > 0
    opts: dict
    f: np.ndarray        # (M,) nodal source term (interior load)
    x: np.ndarray        # (F, N, R) test vectors for the operator apply
    extra: dict = field(default_factory=dict)


def frac_laplacian_half_constant(d: int, s: float) -> float:
    """C_{d,s}/2, the constant that turns the bilinear form into ((-Delta)^s u, v)."""
    c = s * 2.0 ** (2 * s) * math.gamma((d + 2 * s) / 2) / (math.pi ** (d / 2) * math.gamma(1 - s))
    return 0.5 * c


def closed_form_u(d: int, s: float, r2: np.ndarray) -> np.ndarray:
    """Solution of (-Delta)^s u = 1 in the unit ball, u = 0 outside."""
    c = 2.0 ** (-2 * s) * math.gamma(d / 2) / (math.gamma(d / 2 + s) * math.gamma(1 + s))
    return c * np.clip(1.0 - r2, 0.0, None) ** s


def _opts(**kw):
    o = dict(DEFAULT_OPTS)
    o.update(kw)
    return o


def interval(n_int: int = 512, n_ext: int | None = None, nrhs: int = 1, seed: int = 1, **kw) -> Problem:
    if n_ext is None:
        n_ext = n_int // 2
    m = interval_mesh(n_int, n_ext)
    x = m.coords[0]
    s = (0.5 + 0.3 * np.sin(np.pi * x))[None, :]
    kappa = np.ones_like(s)
    rng = np.random.default_rng(seed)
    vec = rng.standard_normal((1, m.n_dofs, nrhs))
    return Problem("interval", m, s, kappa, _opts(leaf_size=kw.pop("leaf_size", 32), **kw),
                   np.ones(m.n_nodes), vec)


def interval_const(n_int: int = 512, n_ext: int | None = None, s: float = 0.5, **kw) -> Problem:
    h = 2.0 / n_int
    if n_ext is None:
        n_ext = max(2, int(round(26 * n_int / 512)))
    R = 1.0 + n_ext * h
    m = interval_mesh(n_int, n_ext, exterior_radius=R)
    sv = np.full((1, m.n_nodes), s)
    kappa = np.ones_like(sv)
    rng = np.random.default_rng(1)
    vec = rng.standard_normal((1, m.n_dofs, 1))
    kw.setdefault("s_bar", max(s, 0.5))
    kw.setdefault("leaf_size", 32)
    o = _opts(a_scale=frac_laplacian_half_constant(1, s), s_exterior=s, **kw)
    return Problem("interval_const", m, sv, kappa, o, np.ones(m.n_nodes), vec, {"s": s})


def square(n: int = 128, pad: int | None = None, jitter: float = 0.1, nrhs: int = 1, graded: float = 0.0,
           **kw) -> Problem:
    """``graded`` > 1: the exterior band (-0.5, 1.5)^2 \\ [0,1]^2 graded geometrically with that ratio
    (same interior grid, jitter, fields and vectors)."""
    if pad is None:
        pad = n // 2
    if graded > 1.0:
        m = square_mesh_graded(n, 0.5, graded, jitter=jitter, seed=0)
    else:
        m = square_mesh(n, pad, jitter=jitter, seed=0)
    x1, x2 = m.coords
    # range [0.1, 0.9] on (-0.5, 1.5)^2; the clip only removes rounding of the grid coordinates
    s = np.clip(0.3 + 0.2 * (x1 + x2), 0.1, 0.9)[None, :]
    kappa = (1.0 + 0.5 * np.cos(2 * np.pi * x1) * np.cos(2 * np.pi * x2))[None, :]
    rng = np.random.default_rng(1)
    vec = rng.standard_normal((1, m.n_dofs, nrhs))
    return Problem("square", m, s, kappa, _opts(**kw), np.ones(m.n_nodes), vec)


def disk(n: int = 512, layers: int | None = None, s_const: float | None = None, **kw) -> Problem:
    """Unit disk plus annulus to R=1.1; exterior beyond R is analytic.

    ``s_const`` given: constant order with the fractional-Laplacian normalisation
    (closed-form test).  Otherwise s = 0.5 + 0.25 tanh((|x|-0.5)/0.05), a = 1.
    """
    R = 1.1
    if layers is None:
        layers = max(1, int(round(0.1 / (2.0 / n))))
    m = disk_mesh(n, layers, R, exterior_radius=R)
    r = np.sqrt((m.coords ** 2).sum(axis=0))
    if s_const is not None:
        s = np.full((1, m.n_nodes), s_const)
        kw.setdefault("s_bar", max(0.9, s_const))
        o = _opts(a_scale=frac_laplacian_half_constant(2, s_const), s_exterior=s_const, **kw)
    else:
        s = (0.5 + 0.25 * np.tanh((r - 0.5) / 0.05))[None, :]
        o = _opts(s_exterior=0.75, **kw)
    kappa = np.ones_like(s)
    rng = np.random.default_rng(2)
    vec = rng.standard_normal((1, m.n_dofs, 1))
    return Problem("disk", m, s, kappa, o, np.ones(m.n_nodes), vec, {"s_const": s_const})


def batched(n: int = 256, pad: int | None = None, n_fields: int = 16, nrhs: int = 64, **kw) -> Problem:
    if pad is None:
        pad = n // 2
    m = square_mesh(n, pad, jitter=0.0)
    x1, x2 = m.coords
    ks = np.arange(1, n_fields + 1)[:, None]
    s = 0.5 + 0.3 * np.sin(ks * np.pi * x1[None, :]) * np.cos(np.pi * x2[None, :])
    kappa = np.ones_like(s)
    rng = np.random.default_rng(3)
    vec = rng.standard_normal((n_fields, m.n_dofs, nrhs)).astype(np.float32).astype(np.float64)
    return Problem("batched", m, s, kappa, _opts(**kw), np.ones(m.n_nodes), vec)


def adjoint_disk(n: int = 8, **kw) -> Problem:
    """Two (s, kappa) fields on disk(n); x holds u [2, N, 2], extra["w"] the weights w."""
    kw.setdefault("leaf_size", 6)
    kw.setdefault("leaf_size_rho", 12)
    kw.setdefault("cheb_p", 3)
    P = disk(n, **kw)
    x1, x2 = P.mesh.coords
    s = np.stack([P.s[0], P.s[0] + 0.05 * np.sin(2 * np.pi * x1) * np.cos(np.pi * x2)])
    kappa = np.stack([np.ones_like(x1), 1.0 + 0.3 * x1])
    u = np.random.default_rng(14).standard_normal((2, P.mesh.n_dofs, 2))
    w = np.random.default_rng(15).standard_normal((2, P.mesh.n_dofs, 2))
    return Problem("adjoint_disk", P.mesh, s, kappa, P.opts, P.f, u, {"w": w})


def bump_order(x1, x2, s_star=0.7, eta=0.2, ell=1.0, center=(-0.4, 0.4)):
    """s* + eta bump(x1 - c1; l) bump(x2 - c2; l), bump(x; l) = exp(-1/(1-r^2)), r = 2x/l."""
    def bump(x):
        r = 2.0 * x / ell
        out = np.zeros_like(r)
        m = np.abs(r) < 1.0
        out[m] = np.exp(-1.0 / (1.0 - r[m] ** 2))
        return out
    return s_star + eta * bump(x1 - center[0]) * bump(x2 - center[1])


def bump(j: int = 6, eta: float = 0.2, s_star: float = 0.7, f: float = 20.0, **kw) -> Problem:
    """The paper's variable-order bump problem on the uniform grid T_j of (-2,2)^2."""
    n = 2 ** (j + 1)
    m = square_mesh(n, n // 2, jitter=0.0, lo=-1.0, hi=1.0)
    x1, x2 = m.coords
    s = bump_order(x1, x2, s_star=s_star, eta=eta)[None, :]
    kappa = np.ones_like(s)
    rng = np.random.default_rng(16)
    vec = rng.standard_normal((1, m.n_dofs, 1))
    return Problem("bump", m, s, kappa, _opts(**kw), np.full(m.n_nodes, f), vec,
                   {"j": j, "eta": eta, "s_star": s_star})
