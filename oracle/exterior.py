"""Density of the exterior beyond the auxiliary ball (oracle; test infrastructure).

For an exterior that continues beyond |y| = R (Sec. 7.1.1, eq. e:rho):
  rho_B(x) = int_{|y|>R} gamma(x,y) dy.
With s(y) = s_out and kappa(y) = kappa_out beyond R, and sig = s(x) + s_out,
integrating the radial variable exactly gives
  2D: rho_B(x) = a(x) / sig * int_0^{2 pi} t(theta,x)^{-sig} d theta,
      t = sqrt(mu^2 + R^2 - |x|^2) - mu,  mu = x1 cos(theta) + x2 sin(theta);
  1D: rho_B(x) = a(x) / sig * ((R - x)^{-sig} + (R + x)^{-sig}),
where a(x) = a_scale * sqrt(kappa(x) kappa_out).  For sig = 2s this is the
paper's formula.  The theta integral uses the periodic trapezoid rule with
n_theta points (the integrand is smooth and periodic; the paper's 9-point
Gauss rule is too coarse near |x| -> 1 for R = 1.1).

Pinned by tests/test_oracle_exterior.py: closed form at x = 0 and a
brute-force 2D integral at an off-centre point.
"""
from __future__ import annotations

import numpy as np


def rho_ball_exterior(dim, x, s_x, kappa_x, R, s_out, kappa_out, a_scale, n_theta):
    sig = s_x + s_out
    a = a_scale * np.sqrt(kappa_x * kappa_out)
    if dim == 1:
        return a / sig * ((R - x[0]) ** (-sig) + (R + x[0]) ** (-sig))
    th = 2.0 * np.pi * np.arange(n_theta) / n_theta
    mu = x[0][:, None] * np.cos(th)[None, :] + x[1][:, None] * np.sin(th)[None, :]
    r2 = (x ** 2).sum(axis=0)[:, None]
    t = np.sqrt(mu * mu + R * R - r2) - mu
    integral = (t ** (-sig[:, None])).sum(axis=1) * (2.0 * np.pi / n_theta)
    return a / sig * integral
