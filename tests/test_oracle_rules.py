"""Pins of the oracle's 1D rules and Lagrange operators against closed forms and exactness."""
import math

import numpy as np
import pytest

from oracle import rules


def _moment(k):
    return 2.0 / (k + 1) if k % 2 == 0 else 0.0


def test_gauss_lobatto_closed_forms():
    x, w = rules.gauss_lobatto(3)
    np.testing.assert_allclose(x, [-1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 3, 4 / 3, 1 / 3], rtol=1e-14)
    x, w = rules.gauss_lobatto(4)
    r = 1 / math.sqrt(5)
    np.testing.assert_allclose(x, [-1, -r, r, 1], atol=1e-15)
    np.testing.assert_allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6], rtol=1e-14)


def test_gauss_radau_closed_forms():
    x, w = rules.gauss_radau_left(2)
    np.testing.assert_allclose(x, [-1, 1 / 3], atol=1e-15)
    np.testing.assert_allclose(w, [0.5, 1.5], rtol=1e-14)
    x, w = rules.gauss_radau_left(3)
    s6 = math.sqrt(6)
    np.testing.assert_allclose(x, [-1, (1 - s6) / 5, (1 + s6) / 5], atol=1e-15)
    np.testing.assert_allclose(w, [2 / 9, (16 + s6) / 18, (16 - s6) / 18], rtol=1e-14)


@pytest.mark.parametrize("n", range(2, 9))
def test_exactness_degrees(n):
    for name, deg in (("GL", 2 * n - 3), ("LGR", 2 * n - 2), ("LG", 2 * n - 1)):
        x, w = rules.RULES[name](n)
        assert abs(w.sum() - 2.0) < 1e-14
        for k in range(deg + 1):
            assert abs(np.dot(w, x ** k) - _moment(k)) < 1e-13, (name, n, k)
        # first degree that is not integrated exactly (an even power for the symmetric rules)
        k = deg + 1
        if name == "LGR" or k % 2 == 0:
            assert abs(np.dot(w, x ** k) - _moment(k)) > 1e-8, (name, n, k)


@pytest.mark.parametrize("rule", ["GL", "LGR", "LG"])
@pytest.mark.parametrize("n", [2, 4, 7])
def test_lagrange_operators_exact_on_polynomials(rule, n):
    x, _ = rules.RULES[rule](n)
    D = rules.derivative_matrix(x)
    t = np.linspace(-1, 1, 11)
    L = rules.lagrange_eval(x, t)
    for k in range(n):
        np.testing.assert_allclose(L @ x ** k, t ** k, atol=1e-13)
        np.testing.assert_allclose(D @ x ** k, k * x ** (k - 1) if k else 0 * x, atol=1e-12)
