"""Pins of the L-BFGS oracle: the two-loop recursion equals the dense BFGS
inverse-Hessian update applied to g (the identity the recursion is built
on), reproduces the secant condition H y = s for the newest pair, gives -g
with no pairs, and on a strictly convex quadratic with exact line searches
reaches the minimiser in at most n steps when the memory holds n pairs
(finite termination of BFGS with exact line search)."""
import numpy as np

from oracle import lbfgs as LB


def test_two_loop_equals_dense_bfgs_update():
    rng = np.random.default_rng(0)
    n, m = 12, 5
    A = rng.standard_normal((n, n))
    A = A @ A.T + n * np.eye(n)
    S = [rng.standard_normal(n) for _ in range(m)]
    Y = [A @ s for s in S]                     # curvature y^T s > 0
    g = rng.standard_normal(n)
    H = LB.bfgs_inverse(S, Y, n)
    np.testing.assert_allclose(LB.two_loop(g, S, Y), -H @ g, rtol=1e-12, atol=1e-12)
    # secant condition of the newest pair
    np.testing.assert_allclose(-LB.two_loop(Y[-1], S, Y), S[-1], rtol=1e-10, atol=1e-12)


def test_no_pairs_gives_steepest_descent():
    g = np.arange(5.0)
    np.testing.assert_array_equal(LB.two_loop(g, [], []), -g)


def test_finite_termination_on_a_quadratic():
    rng = np.random.default_rng(1)
    n = 8
    A = rng.standard_normal((n, n))
    A = A @ A.T + np.eye(n)
    b = rng.standard_normal(n)
    x = np.zeros(n)
    S, Y = [], []
    g = A @ x - b
    for k in range(n):
        p = LB.two_loop(g, S, Y)
        t = -(g @ p) / (p @ A @ p)              # exact line search
        xn = x + t * p
        gn = A @ xn - b
        S.append(xn - x)
        Y.append(gn - g)
        x, g = xn, gn
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-10)
