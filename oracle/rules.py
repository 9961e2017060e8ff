"""Quadrature rules (oracle; test infrastructure).

* ``gauss01(n)``: n-point Gauss-Legendre rule on [0,1] (the tensor rules of
  Sec. 4 and Sec. 5.2 are products of it).
* ``element_rule(dim, n)``: the per-element rule used for separated element
  pairs (Sec. 5.2, collapsed coordinates x^=(xi, xi*eta1) on the reference
  triangle with vertices (0,0),(1,0),(1,1)) and for the weighted mass matrix
  (Sec. 6.1, "the same scheme but only for x").  In 1D it is plain Gauss on [0,1].

Pinned by tests/test_oracle_rules.py: exact polynomial moments of the
reference simplex.
"""
from __future__ import annotations

import functools

import mpmath
import numpy as np


@functools.lru_cache(maxsize=None)
def _legendre_rule(n: int):
    """Nodes/weights of n-point Gauss-Legendre on [-1,1], correctly rounded to double.

    Roots of P_n by Newton's method in 50-digit arithmetic; w = 2/((1-t^2) P_n'(t)^2).
    """
    with mpmath.workdps(50):
        ts, ws = [], []
        for i in range(1, n + 1):
            t = mpmath.cos(mpmath.pi * (i - mpmath.mpf(1) / 4) / (n + mpmath.mpf(1) / 2))
            for _ in range(100):
                p0, p1 = mpmath.mpf(1), t
                for k in range(2, n + 1):
                    p0, p1 = p1, ((2 * k - 1) * t * p1 - (k - 1) * p0) / k
                dp = n * (t * p1 - p0) / (t * t - 1) if n > 1 else mpmath.mpf(1)
                dt = p1 / dp
                t -= dt
                if abs(dt) < mpmath.mpf(10) ** -45:
                    break
            p0, p1 = mpmath.mpf(1), t
            for k in range(2, n + 1):
                p0, p1 = p1, ((2 * k - 1) * t * p1 - (k - 1) * p0) / k
            dp = n * (t * p1 - p0) / (t * t - 1) if n > 1 else mpmath.mpf(1)
            ts.append(float(t))
            ws.append(float(2 / ((1 - t * t) * dp * dp)))
    order = np.argsort(ts)
    return np.array(ts)[order], np.array(ws)[order]


def gauss01(n: int):
    """n-point Gauss-Legendre on [0,1]: xi = (t+1)/2, w = w_t/2 (t, w_t correctly rounded)."""
    t, w = _legendre_rule(n)
    return 0.5 * (t + 1.0), 0.5 * w


def element_rule(dim: int, n: int):
    """Reference points (dim, nq) and weights (nq,) on the reference simplex."""
    g, w = gauss01(n)
    if dim == 1:
        return g[None, :].copy(), w.copy()
    if dim == 2:
        xi = np.repeat(g, n)
        eta = np.tile(g, n)
        wt = np.repeat(w, n) * np.tile(w, n) * xi
        return np.stack([xi, xi * eta]), wt
    raise ValueError("dim must be 1 or 2")


def barycentric_ref(dim: int, xh: np.ndarray) -> np.ndarray:
    """Shape functions of the reference simplex at reference points.

    2D reference triangle (0,0),(1,0),(1,1): l0 = 1-x1, l1 = x1-x2, l2 = x2.
    1D reference interval [0,1]: l0 = 1-x, l1 = x.
    Returns (dim+1, ...) array.
    """
    if dim == 1:
        return np.stack([1.0 - xh[0], xh[0]])
    return np.stack([1.0 - xh[0], xh[0] - xh[1], xh[1]])
