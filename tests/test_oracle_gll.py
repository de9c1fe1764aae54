"""Pins for the oracle's GLL nodes, weights and derivative matrix.

Each check is fixed by mathematics, not by re-running the oracle's formula:
closed-form nodes/weights (golden fixture), symmetry, quadrature exactness,
exact differentiation of monomials, and an independent library root finder.
"""

import json
import math
import os

import numpy as np
import pytest

from oracle import gll

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gll_closed_forms.json")
ORDERS = list(range(1, 16))


def _eval(expr):
    return float(eval(expr, {"__builtins__": {}}, {"sqrt": math.sqrt}))


def test_closed_form_nodes_and_weights():
    with open(GOLDEN) as fh:
        data = json.load(fh)["orders"]
    for key, ref in data.items():
        n = int(key)
        xi = gll.gll_nodes(n)
        w = gll.gll_weights(n)
        np.testing.assert_allclose(xi, [_eval(s) for s in ref["nodes"]],
                                   rtol=0, atol=2e-16)
        np.testing.assert_allclose(w, [_eval(s) for s in ref["weights"]],
                                   rtol=0, atol=4e-16)


@pytest.mark.parametrize("n", ORDERS)
def test_nodes_symmetric_sorted_and_match_library_roots(n):
    xi = gll.gll_nodes(n)
    assert xi[0] == -1.0 and xi[-1] == 1.0
    assert np.all(np.diff(xi) > 0)
    np.testing.assert_array_equal(xi, -xi[::-1])
    if n % 2 == 0:
        assert xi[n // 2] == 0.0
    if n > 1:
        roots = np.sort(np.polynomial.legendre.Legendre.basis(n).deriv().roots().real)
        np.testing.assert_allclose(xi[1:-1], roots, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", ORDERS)
def test_quadrature_exact_to_degree_2n_minus_1(n):
    xi, w = gll.gll_nodes(n), gll.gll_weights(n)
    assert abs(w.sum() - 2.0) < 1e-14
    for p in range(0, 2 * n):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.dot(w, xi ** p) - exact) < 1e-13, p
    # degree 2n is NOT integrated exactly by n+1 Lobatto points
    assert abs(np.dot(w, xi ** (2 * n)) - 2.0 / (2 * n + 1)) > 1e-11


@pytest.mark.parametrize("n", ORDERS)
def test_derivative_matrix_is_exact_on_monomials(n):
    xi = gll.gll_nodes(n)
    d = gll.diff_matrix(n)
    scale = n * n
    for p in range(0, n + 1):
        exact = p * xi ** (p - 1) if p > 0 else np.zeros_like(xi)
        np.testing.assert_allclose(d @ xi ** p, exact, rtol=0,
                                   atol=1e-14 * scale * max(1, p))
    # a degree n+1 monomial is not in the space: derivative is not exact
    assert np.max(np.abs(d @ xi ** (n + 1) - (n + 1) * xi ** n)) > 1e-3


@pytest.mark.parametrize("n", ORDERS)
def test_derivative_matrix_structure(n):
    d = gll.diff_matrix(n)
    # constants differentiate to zero (negative-sum diagonal)
    assert np.max(np.abs(d.sum(axis=1))) < 1e-13 * n * n
    # centro-antisymmetry D[n-i, n-j] = -D[i, j]
    np.testing.assert_allclose(d[::-1, ::-1], -d, rtol=0, atol=1e-13 * n * n)
    # closed-form corner entries D00 = -n(n+1)/4, Dnn = +n(n+1)/4
    assert abs(d[0, 0] + n * (n + 1) / 4.0) < 1e-12 * n * n
    assert abs(d[n, n] - n * (n + 1) / 4.0) < 1e-12 * n * n
    # interior diagonal is zero (up to rounding)
    if n > 1:
        assert np.max(np.abs(np.diag(d)[1:-1])) < 1e-12 * n * n


def test_order_one_matrix():
    np.testing.assert_array_equal(gll.diff_matrix(1),
                                  [[-0.5, 0.5], [-0.5, 0.5]])
