"""Pins for the analytic exterior density beyond the auxiliary ball (eq. e:rho)."""
import math

import numpy as np
from scipy import integrate

from oracle.exterior import rho_ball_exterior


def test_rho_ball_centre_closed_form():
    R, s, so = 1.1, 0.7, 0.7
    v = rho_ball_exterior(2, np.zeros((2, 1)), np.array([s]), np.array([1.0]), R, so, 1.0, 1.0, 128)
    assert abs(v[0] - 2 * math.pi * R ** (-(s + so)) / (s + so)) < 1e-13 * v[0]


def test_rho_ball_offcentre_bruteforce():
    R, sx, so = 1.1, 0.4, 0.75
    x = np.array([0.55, -0.6])
    v = rho_ball_exterior(2, x[:, None], np.array([sx]), np.array([2.0]), R, so, 0.5, 1.3, 128)[0]
    # brute force in polar coordinates about the origin: |y| = r > R
    def inner(th):
        def f(r):
            y = r * np.array([math.cos(th), math.sin(th)])
            return r * np.linalg.norm(x - y) ** (-(2 + sx + so))
        return integrate.quad(f, R, np.inf, epsabs=0, epsrel=1e-12, limit=200)[0]
    ref = 1.3 * math.sqrt(2.0 * 0.5) * integrate.quad(inner, 0, 2 * math.pi, epsabs=0, epsrel=1e-11, limit=200)[0]
    assert abs(v - ref) < 1e-9 * ref


def test_rho_ball_1d():
    R, sx, so = 1.2, 0.3, 0.6
    x = 0.35
    v = rho_ball_exterior(1, np.array([[x]]), np.array([sx]), np.array([1.0]), R, so, 1.0, 1.0, 0)[0]
    f = lambda y: abs(x - y) ** (-(1 + sx + so))
    ref = integrate.quad(f, R, np.inf, epsrel=1e-13)[0] + integrate.quad(f, -np.inf, -R, epsrel=1e-13)[0]
    assert abs(v - ref) < 1e-10 * ref
