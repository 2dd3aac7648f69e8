"""Pins of the nonlinear-kernel C-SVC oracle (Table 3's problem): the XOR
closed form under the RBF kernel, 3^n enumeration with the explicit Q, and
the linear kernel against the linear C-SVC oracle."""
import numpy as np
import pytest

import synth
from oracle import bruteforce, features, kernel, ssnal


@pytest.mark.parametrize("alpha,C", [(1.0, 100.0), (0.5, 100.0), (1.0, 0.5)])
def test_xor_closed_form(alpha, C):
    """Corners (+-1, +-1) with y = x1 x2.  Each point has two neighbours of the
    other class at squared distance 4 and one point of its own class at 8,
    so with x_i = t for all i (symmetry; y^T x = 0 holds) (Q x)_i =
    t (1 - exp(-2/alpha))^2 =: t kappa and f = 2 kappa t^2 - 4 t, minimised
    at t = min(1/kappa, C)."""
    X = np.array([[1.0, 1.0], [-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])
    y = np.array([1, 1, -1, -1], np.int8)
    K = features.rbf_kernel(X, X, alpha)
    kappa = (1.0 - np.exp(-2.0 / alpha)) ** 2
    t = min(1.0 / kappa, C)
    r = kernel.solve(K, y, C, tol=1e-10)
    assert r.status == "OK"
    np.testing.assert_allclose(r.x, t, rtol=1e-8)
    assert r.obj == pytest.approx(2 * kappa * t * t - 4 * t, rel=1e-10)


@pytest.mark.parametrize("seed", range(4))
def test_rbf_matches_enumeration(seed):
    rng = np.random.default_rng(700 + seed)
    X = rng.standard_normal((7, 2))
    y = np.where(X[:, 0] * X[:, 1] > 0, 1, -1).astype(np.int8)
    if np.all(y == y[0]):
        y[0] = -y[0]
    K = features.rbf_kernel(X, X, 0.8)
    Q = kernel.kernel_q(K, y)
    C = 2.0
    f_star, x_star = bruteforce.general_qp_by_enumeration(
        Q, -np.ones(7), y.astype(np.float64), 0.0, np.zeros(7), np.full(7, C))
    r = kernel.solve(K, y, C, tol=1e-10)
    assert r.status == "OK"
    assert r.obj == pytest.approx(f_star, abs=1e-9 * (1 + abs(f_star)))
    np.testing.assert_allclose(r.x, x_star, atol=1e-6)       # RBF Q is positive definite


def test_linear_kernel_matches_linear_oracle():
    X, y = synth.tiny_problem(30, 4, 9)
    C = 1.0
    r_lin = ssnal.solve(X, y, C, tol=1e-10)
    r_ker = kernel.solve(X @ X.T, y, C, tol=1e-10)
    assert r_ker.status == "OK"
    assert r_ker.obj == pytest.approx(r_lin.obj, abs=1e-8 * (1 + abs(r_lin.obj)))
