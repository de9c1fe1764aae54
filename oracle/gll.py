"""GLL nodes, quadrature weights and the collocation derivative matrix (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Context: the paper (section 1) names the spectral element method as the
discretisation of the solver whose snapshots are analysed; the fields are
stored at the Gauss-Lobatto-Legendre (GLL) points of order-N elements.  The
definitions below are the textbook ones (Deville, Fischer & Mund 2002, ch. 2):

* nodes: xi_0 = -1, xi_N = +1 and the N-1 roots of P_N' in between;
* weights: w_j = 2 / (N (N+1) P_N(xi_j)^2);
* derivative matrix D_ij = l_j'(xi_i), the derivative of the j-th Lagrange
  cardinal polynomial at node i.  Off the diagonal
  D_ij = P_N(xi_i) / (P_N(xi_j) (xi_i - xi_j)); the diagonal is set to minus
  the off-diagonal row sum, so that D applied to a constant is zero up to
  rounding (the derivative of a constant is exactly zero).
"""

import math

import numpy as np


def legendre_with_derivs(n, x):
    """Return (P_n(x), P_n'(x), P_n''(x)) by the three-term recurrence.

    Bonnet's recurrence  (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}  with
    P_0 = 1, P_1 = x; the derivative from
    (1 - x^2) P_n' = n (P_{n-1} - x P_n), and the second derivative from
    Legendre's equation (1 - x^2) P'' - 2 x P' + n (n+1) P = 0.  ``x`` must be
    strictly inside (-1, 1) for the derivative formulas.
    """
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if n == 0:
        return p_prev, np.zeros_like(x), np.zeros_like(x)
    p = x.copy()
    for k in range(1, n):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    one_m_x2 = 1.0 - x * x
    dp = n * (p_prev - x * p) / one_m_x2
    d2p = (2.0 * x * dp - n * (n + 1) * p) / one_m_x2
    return p, dp, d2p


def legendre_value(n, x):
    """P_n(x) by Bonnet's recurrence (valid on the closed interval)."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if n == 0:
        return p_prev
    p = x.copy()
    for k in range(1, n):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    return p


def gll_nodes(n):
    """GLL nodes xi_0 < ... < xi_n on [-1, 1] for polynomial order n >= 1.

    Interior nodes are the roots of P_n', found by Newton's method on P_n'
    (using P_n'' from Legendre's equation) started from the Chebyshev-Gauss-
    Lobatto points -cos(pi j / n).  The result is symmetrised
    (xi_{n-j} = -xi_j, and the middle node is 0 for even n).
    """
    if n < 1:
        raise ValueError("order must be >= 1")
    xi = -np.cos(np.pi * np.arange(n + 1) / n)
    interior = xi[1:-1].copy()
    for _ in range(100):
        if interior.size == 0:
            break
        _, dp, d2p = legendre_with_derivs(n, interior)
        step = dp / d2p
        interior = interior - step
        if np.max(np.abs(step)) < 1e-17:
            break
    # one more Newton step at convergence to settle the last ulp
    if interior.size:
        _, dp, d2p = legendre_with_derivs(n, interior)
        interior = interior - dp / d2p
    xi = np.concatenate(([-1.0], interior, [1.0]))
    xi = 0.5 * (xi - xi[::-1])
    if n % 2 == 0:
        xi[n // 2] = 0.0
    return xi


def gll_weights(n, xi=None):
    """GLL quadrature weights w_j = 2 / (n (n+1) P_n(xi_j)^2)."""
    if xi is None:
        xi = gll_nodes(n)
    p = legendre_value(n, xi)
    return 2.0 / (n * (n + 1) * p * p)


def diff_matrix(n, xi=None):
    """Collocation derivative matrix D (shape (n+1, n+1)), D_ij = l_j'(xi_i).

    (Df)_i is the derivative at node i of the degree-n interpolant of the
    nodal values f_j.  Off-diagonal entries from the closed form in the
    module docstring; diagonal = minus the row sum of the off-diagonal part.
    """
    if xi is None:
        xi = gll_nodes(n)
    p = legendre_value(n, xi)
    m = n + 1
    d = np.zeros((m, m), dtype=np.float64)
    for i in range(m):
        for j in range(m):
            if i != j:
                d[i, j] = p[i] / (p[j] * (xi[i] - xi[j]))
    for i in range(m):
        d[i, i] = -math.fsum(d[i, j] for j in range(m) if j != i)
    return d
