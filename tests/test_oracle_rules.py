"""Pins for the oracle's quadrature rules: exact moments of the reference simplex."""
import numpy as np
import pytest

from oracle.rules import gauss01, element_rule, barycentric_ref


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_gauss01_exact_degree(n):
    x, w = gauss01(n)
    for k in range(2 * n):
        assert abs((w * x ** k).sum() - 1.0 / (k + 1)) < 1e-14
    # not exact one degree beyond
    assert abs((w * x ** (2 * n)).sum() - 1.0 / (2 * n + 1)) > 1e-12


@pytest.mark.parametrize("n", [2, 3, 4])
def test_element_rule_triangle_moments(n):
    # reference triangle (0,0),(1,0),(1,1): 0 <= x2 <= x1 <= 1
    # int x1^a x2^b = 1 / ((b+1)(a+b+2))
    xh, w = element_rule(2, n)
    for a in range(0, 2 * n - 1):
        for b in range(0, 2 * n - 1 - a):
            exact = 1.0 / ((b + 1) * (a + b + 2))
            assert abs((w * xh[0] ** a * xh[1] ** b).sum() - exact) < 1e-14, (a, b)
    assert abs(w.sum() - 0.5) < 1e-15


def test_barycentric_partition_of_unity_and_vertices():
    xh = np.array([[0.0, 1.0, 1.0, 0.3], [0.0, 0.0, 1.0, 0.1]])
    lam = barycentric_ref(2, xh)
    assert np.allclose(lam.sum(axis=0), 1.0)
    assert np.allclose(lam[:, :3], np.eye(3))
    lam1 = barycentric_ref(1, np.array([[0.0, 1.0]]))
    assert np.allclose(lam1, np.eye(2))
